// hmc_device.hpp -- per-site arithmetic of the sweeps for gfx950: the
// counter-based generator, the keyed shuffle, the cone proposal of Table A1
// and the energy change of Eq. 2.  Templated on the spin precision R.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hmc_internal.h"

namespace hmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications; the key is bumped by the Weyl constants between
// rounds.  Counter words: (sweep, id, tag, instance).  Placing the per-site
// id in the second word leaves both multiplications of the first round, and
// one of the second, on wave-uniform values.
// ---------------------------------------------------------------------------
struct Rand4 { uint32_t r0, r1, r2, r3; };

// a ^ b ^ c in one gfx950 V_BITOP3 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Rand4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Rand4{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Keyed permutation of [0, n) used to shuffle one colour (Table A2):
// balanced 4-round Feistel network on 2*half bits whose round function is
// the MurmurHash3 32-bit finaliser (public domain), with cycle walking
// until the image falls inside [0, n).  Terminates: the orbit of x < n under
// a permutation of [0, 2^(2 half)) returns to [0, n).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t mix32(uint32_t v)
{
    v ^= v >> 16;
    v *= 0x85EBCA6Bu;
    v ^= v >> 13;
    v *= 0xC2B2AE35u;
    v ^= v >> 16;
    return v;
}

__device__ __forceinline__ uint32_t shuffle_index(uint32_t x, uint32_t n, uint32_t half,
                                                  uint32_t mask, const Rand4 key)
{
    const uint32_t k[4] = {key.r0, key.r1, key.r2, key.r3};
    do {
        uint32_t lo = x & mask, hi = x >> half;
#pragma unroll
        for (int round = 0; round < 4; ++round) {
            const uint32_t nlo = hi ^ (mix32(lo ^ k[round]) & mask);
            hi = lo;
            lo = nlo;
        }
        x = (hi << half) | lo;
    } while (x >= n);
    return x;
}

// Inverse of shuffle_index: the rounds undone in reverse order, walking with
// the inverse bijection until the preimage falls inside [0, n).
__device__ __forceinline__ uint32_t unshuffle_index(uint32_t y, uint32_t n, uint32_t half,
                                                    uint32_t mask, const Rand4 key)
{
    const uint32_t k[4] = {key.r0, key.r1, key.r2, key.r3};
    do {
        uint32_t lo = y & mask, hi = y >> half;
#pragma unroll
        for (int round = 3; round >= 0; --round) {
            const uint32_t plo = hi;
            hi = lo ^ (mix32(plo ^ k[round]) & mask);
            lo = plo;
        }
        y = (hi << half) | lo;
    } while (y >= n);
    return y;
}

// ---------------------------------------------------------------------------
// Precision-specific primitives.  FP32 uses the hardware transcendentals
// (v_sin/v_cos take revolutions, v_exp is 2^x, v_rsq, v_rcp, v_sqrt);
// FP64 uses the accurate library routines.
// ---------------------------------------------------------------------------
template <typename R> struct Prim;

template <> struct Prim<float> {
    // ((r >> 9) + 1/2) 2^-23, in (0, 1): the top 23 bits become the mantissa
    // of a float in [1, 2) (one V_ALIGNBIT shifts them under the exponent
    // 0x7F), from which 1 - 2^-24 is subtracted exactly (both operands within
    // a factor of 2).
    static __device__ __forceinline__ float u01(uint32_t r)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, r, 9u)) - 0x1.fffffep-1f;
    }
    static __device__ __forceinline__ void sincos_turns(float u, float* s, float* c)
    {
        *s = __builtin_amdgcn_sinf(u);
        *c = __builtin_amdgcn_cosf(u);
    }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // exp(-dE/T) as 2^(-dE * log2(e)/T); scale = log2(e)/T.
    static __device__ __forceinline__ float boltzmann(float dE, float scale)
    {
        return __builtin_amdgcn_exp2f(-dE * scale);
    }
    static __host__ __device__ __forceinline__ float scale_for(double T) { return (float)(1.4426950408889634 / T); }
};

template <> struct Prim<double> {
    // (r + 1/2) 2^-32, exact in FP64, in (0, 1).
    static __device__ __forceinline__ double u01(uint32_t r)
    {
        return __builtin_fma((double)r, 0x1p-32, 0x1p-33);
    }
    // sin and cos of 2 pi u (sincospi needs no argument reduction by pi).
    static __device__ __forceinline__ void sincos_turns(double u, double* s, double* c)
    {
        sincospi(2.0 * u, s, c);
    }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    // exp(-dE/T); scale = 1/T.
    static __device__ __forceinline__ double boltzmann(double dE, double scale) { return exp(-dE * scale); }
    static __host__ __device__ __forceinline__ double scale_for(double T) { return 1.0 / T; }
};

template <typename R> struct V3 { R x, y, z; };

template <typename R>
__device__ __forceinline__ R dot(const V3<R>& a, const V3<R>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Sx^2 Sy^2 + Sx^2 Sz^2 + Sy^2 Sz^2 (cubic term of Eq. 2).
template <typename R>
__device__ __forceinline__ R cubic_f(const V3<R>& s)
{
    const R x2 = s.x * s.x, y2 = s.y * s.y, z2 = s.z * s.z;
    return x2 * y2 + x2 * z2 + y2 * z2;
}

// Cone proposal: uniform in solid angle on the cap of half-angle theta about
// s, with c1 = 1 - cos(theta): 1 - cos(alpha) = u0 c1, azimuth 2 pi u1 in the
// orthonormal basis of Duff et al. (JCGT 6(1), 2017); renormalised.
template <typename R>
__device__ __forceinline__ V3<R> cone_move(const V3<R>& s, R u0, R u1, R c1)
{
    using P = Prim<R>;
    const R d = u0 * c1;
    const R cosa = R(1) - d;
    const R sina = P::sqrt_(d * (R(2) - d));
    R sp, cp;
    P::sincos_turns(u1, &sp, &cp);
    const R sign = __builtin_copysign(R(1), s.z);
    const R a = -P::rcp(sign + s.z);
    const R b = s.x * s.y * a;
    const V3<R> b1{R(1) + sign * s.x * s.x * a, sign * b, -sign * s.x};
    const V3<R> b2{b, sign + s.y * s.y * a, -s.y};
    V3<R> v;
    v.x = cosa * s.x + sina * (cp * b1.x + sp * b2.x);
    v.y = cosa * s.y + sina * (cp * b1.y + sp * b2.y);
    v.z = cosa * s.z + sina * (cp * b1.z + sp * b2.z);
    // |v|^2 = 1 + e with e of the order of the rounding error; one Newton step
    // for 1/sqrt(1 + e) is exact to O(e^2)
    const R inv = R(1.5) - R(0.5) * dot(v, v);
    return V3<R>{v.x * inv, v.y * inv, v.z * inv};
}

// Model constants in the spin precision.
template <typename R> struct Model {
    R J, Ku, Kc;
    V3<R> e;   // uniaxial axis (unit)
    V3<R> h;   // field
};

// One-site terms of Eq. 2 kept for the observables: projection on the
// uniaxial axis and the cubic function, of the old and the proposed spin.
template <typename R> struct SiteTerms { R se, te, cs, ct; };

// Energy change of one site (Eq. 2) when s becomes t, with the local field
// hl = J * (sum of the six neighbours) + h.
template <typename R>
__device__ __forceinline__ R delta_e(const Model<R>& m, const V3<R>& s, const V3<R>& t, const V3<R>& hl,
                                     SiteTerms<R>& k)
{
    R dE = -((t.x - s.x) * hl.x + (t.y - s.y) * hl.y + (t.z - s.z) * hl.z);
    k = SiteTerms<R>{R(0), R(0), R(0), R(0)};
    if (m.Ku != R(0)) {
        k.se = dot(s, m.e);
        k.te = dot(t, m.e);
        dE -= m.Ku * (k.te - k.se) * (k.te + k.se);
    }
    if (m.Kc != R(0)) {
        k.cs = cubic_f(s);
        k.ct = cubic_f(t);
        dE += m.Kc * (k.ct - k.cs);
    }
    return dE;
}

template <typename R>
__device__ __forceinline__ R delta_e(const Model<R>& m, const V3<R>& s, const V3<R>& t, const V3<R>& hl)
{
    SiteTerms<R> k;
    return delta_e(m, s, t, hl, k);
}

// Site contributions to the observables, accumulated in FP64.
struct Acc {
    double M[3] = {0.0, 0.0, 0.0};
    double ex = 0.0, eu = 0.0, ec = 0.0, ez = 0.0;
    double tq[3] = {0.0, 0.0, 0.0};
};

// A thread's sums of its sampled site terms over its z chunk of a colour
// pass (z_chunk x sites-per-thread terms), kept in the spin precision and
// converted to FP64 once per chunk; no FP64 register is live in the march.
// The chunk sums carry FP32 rounding of the order of the site terms' own
// (relative 1e-7 times the square root of the number of terms).
template <typename R>
struct Part {
    R M[3] = {R(0), R(0), R(0)};
    R ex = R(0), eu = R(0), ec = R(0), ez = R(0);
    R tq[3] = {R(0), R(0), R(0)};
};

// The accumulator the pass adds site terms to: the partial sums for FP32
// spins, the FP64 Acc itself for FP64 spins.
template <typename R>
__device__ __forceinline__ auto& site_acc(Acc& a, Part<R>& p)
{
    if constexpr (sizeof(R) == 4) return p;
    else return a;
}

// Adds the partial sums into the FP64 accumulator and clears them (nothing
// to do when the pass adds to Acc directly).
template <typename A>
__device__ __forceinline__ void flush_part(Acc& acc, A& p)
{
    if constexpr (!__is_same(A, Acc)) {
        acc.M[0] += (double)p.M[0];
        acc.M[1] += (double)p.M[1];
        acc.M[2] += (double)p.M[2];
        acc.ex += (double)p.ex;
        acc.eu += (double)p.eu;
        acc.ec += (double)p.ec;
        acc.ez += (double)p.ez;
        acc.tq[0] += (double)p.tq[0];
        acc.tq[1] += (double)p.tq[1];
        acc.tq[2] += (double)p.tq[2];
        p = A{};
    }
}

// Adds the one-site terms of s (anisotropy, Zeeman, moment) and, when
// TORQUE, s x (-dE_anis/ds), to the FP64 Acc or to spin-precision partial
// sums (each term is formed in the spin precision either way).
template <typename R, bool TORQUE, typename A>
__device__ __forceinline__ void add_site(A& a, const Model<R>& m, const V3<R>& s)
{
    a.M[0] += s.x;
    a.M[1] += s.y;
    a.M[2] += s.z;
    const R se = dot(s, m.e);
    a.eu += -m.Ku * se * se;
    a.ec += m.Kc * cubic_f(s);
    a.ez += -dot(m.h, s);
    if (TORQUE) {
        const R x2 = s.x * s.x, y2 = s.y * s.y, z2 = s.z * s.z;
        const R gx = R(2) * m.Ku * se * m.e.x - R(2) * m.Kc * s.x * (y2 + z2);
        const R gy = R(2) * m.Ku * se * m.e.y - R(2) * m.Kc * s.y * (x2 + z2);
        const R gz = R(2) * m.Ku * se * m.e.z - R(2) * m.Kc * s.z * (x2 + y2);
        a.tq[0] += s.y * gz - s.z * gy;
        a.tq[1] += s.z * gx - s.x * gz;
        a.tq[2] += s.x * gy - s.y * gx;
    }
}

}  // namespace hmc
