// hmc_kernels.hip -- gfx950 kernels of the parallel Metropolis sweeps
// (Lepadatu et al., arXiv:2103.03517, Sec. 2, Tables A1 and A2).
//
// Spin storage: colour-split structure of arrays.  Site (x, y, z) has colour
// c = (x + y + z) & 1 (red = 0) and colour index k = (x + nx*(y + ny*z)) / 2;
// its components live in s[c][0..2][k].  Within a colour, k = kx + hx*(y +
// ny*z) with hx = nx/2, and the x-partner with the same k is the other colour.
// Every kernel reads one colour as neighbours and writes only the other, so a
// colour pass has no read/write overlap (Sec. 2: the two sets do not
// interact in Eq. 2).
#include <hip/hip_runtime.h>

#include <math.h>

#include "hmc_device.hpp"
#include "hmc_internal.h"

namespace hmc {

template <typename R>
struct KArgs {
    R* s[2][3];
    uint32_t hx, ny, nz, P, Nc;
    Model<R> m;
    uint32_t key0, key1, inst;
    DevState* st;
    const R* c1tab;
    double* part;
    uint32_t* cnt;       // [2][cnt_stride]
    uint32_t cnt_stride;
};

template <typename R>
static KArgs<R> make_args(const DevLattice& d)
{
    KArgs<R> a;
    char* base = static_cast<char*>(d.spins);
    for (int c = 0; c < 2; ++c)
        for (int k = 0; k < 3; ++k) a.s[c][k] = reinterpret_cast<R*>(base + (size_t)(3 * c + k) * d.pitch);
    a.hx = (uint32_t)d.hx;
    a.ny = (uint32_t)d.ny;
    a.nz = (uint32_t)d.nz;
    a.P = (uint32_t)d.P;
    a.Nc = (uint32_t)d.Nc;
    a.m.J = (R)d.J;
    a.m.Ku = (R)d.Ku;
    a.m.Kc = (R)d.Kc;
    a.m.e = V3<R>{(R)d.eu[0], (R)d.eu[1], (R)d.eu[2]};
    a.m.h = V3<R>{(R)d.h[0], (R)d.h[1], (R)d.h[2]};
    a.key0 = d.key0;
    a.key1 = d.key1;
    a.inst = d.instance;
    a.st = d.st;
    a.c1tab = static_cast<const R*>(d.c1tab);
    a.part = d.part;
    a.cnt = d.cnt;
    a.cnt_stride = (uint32_t)d.max_blocks;
    return a;
}

// Work-groups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that XCD x receives one contiguous range of logical
// tiles: neighbouring tiles, whose halos overlap, then share an L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nblk)
{
    const uint32_t per = nblk >> 3, rem = nblk & 7u;
    const uint32_t x = b & 7u, i = b >> 3;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Work-group sum in a fixed order (butterfly within each wave, then waves in
// order), so results do not depend on scheduling.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NV>
__device__ __forceinline__ void block_sum_write(double (&v)[NV], double* scratch, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) scratch[wave * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += scratch[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

__device__ __forceinline__ void block_count_write(uint32_t v, uint32_t* scratch, uint32_t* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += scratch[w];
        *out = s;
    }
}

template <typename R>
__device__ __forceinline__ void write_partials(const Acc& acc, double* part, uint32_t b, double* scratch)
{
    double v[kNumPart] = {acc.M[0], acc.M[1], acc.M[2], acc.ex, acc.eu, acc.ec, acc.ez,
                          acc.tq[0], acc.tq[1], acc.tq[2], 0.0, 0.0};
    block_sum_write<kNumPart>(v, scratch, part + (size_t)b * kNumPart);
}

// ---------------------------------------------------------------------------
// Initial spins: along a direction, or uniform on the sphere from Philox
// tag 4 (z = 2 u0 - 1, azimuth 2 pi u1).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void init_kernel(const KArgs<R> a, int mode, R d0, R d1, R d2)
{
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= a.Nc) return;
    V3<R> s{d0, d1, d2};
    if (mode == 1) {
        const uint32_t r = k / a.hx;
        const uint32_t y = r % a.ny, z = r / a.ny;
        const uint32_t site = 2u * k + ((y + z + (uint32_t)c) & 1u);
        const Rand4 rn = philox(0u, site, 4u, a.inst, a.key0, a.key1);
        const R zc = R(2) * Prim<R>::u01(rn.r0) - R(1);
        const R rho = Prim<R>::sqrt_(R(1) - zc * zc);
        R sp, cp;
        Prim<R>::sincos_turns(Prim<R>::u01(rn.r1), &sp, &cp);
        s = V3<R>{rho * cp, rho * sp, zc};
    }
    a.s[c][0][k] = s.x;
    a.s[c][1][k] = s.y;
    a.s[c][2][k] = s.z;
}

// ---------------------------------------------------------------------------
// Standard colour pass (Table A1, MonteCarlo_Red(Black)ParallelPass).
//
// A work-group owns Q = 256*SPT consecutive in-plane colour indices and
// marches over z_chunk planes.  The other colour's plane z sits in LDS as a
// window [base - hx, base + Q + hx) (the x and y neighbours); its z-1, z and
// z+1 values at the owned columns stay in registers.  Each plane of each
// colour is therefore fetched once per pass (plus a halo of 2*hx entries per
// plane), and the loads for plane z+1/z+2 are issued before plane z is
// computed.  OBS (black pass only) fuses the observables: the black site after
// its update plus its red x-partner (same colour index), and the exchange of
// the black site with its six final red neighbours, so every site and every
// bond is counted once.
// ---------------------------------------------------------------------------
template <typename R, int C, bool OBS, int SPT>
__global__ __launch_bounds__(kThreads) void pass_kernel(const KArgs<R> a, const uint32_t zc,
                                                        const uint32_t nqb, const uint32_t nblk,
                                                        const R scale)
{
    constexpr int O = 1 - C;
    constexpr uint32_t Q = kThreads * SPT;
    extern __shared__ __align__(16) unsigned char smem[];
    R* lds = reinterpret_cast<R*>(smem);

    const uint32_t hx = a.hx, P = a.P, nz = a.nz;
    const uint32_t W = Q + 2u * hx;
    const uint32_t t = threadIdx.x;
    const uint32_t b = xcd_remap(blockIdx.x, nblk);
    const uint32_t qb = b % nqb, zb = b / nqb;
    const uint32_t base = qb * Q;
    const uint32_t z0 = zb * zc;
    const uint32_t zn = min(zc, nz - z0);

    const int theta = a.st->theta;
    const uint32_t sweep = (uint32_t)a.st->sweep;
    const R c1 = a.c1tab[theta];
    const Model<R> m = a.m;

    uint32_t qm[SPT], kx[SPT], yy[SPT];
    bool act[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const uint32_t q = base + t + kThreads * j;
        act[j] = q < P;
        qm[j] = act[j] ? q : q % P;
        kx[j] = qm[j] % hx;
        yy[j] = qm[j] / hx;
    }
    // halo slots of the LDS window: window index and in-plane index
    const uint32_t nh = 2u * hx;
    uint32_t hw[kMaxHalo], hg[kMaxHalo];
#pragma unroll
    for (int i = 0; i < kMaxHalo; ++i) {
        const uint32_t slot = t + kThreads * i;
        hw[i] = slot < hx ? slot : slot + Q;
        hg[i] = (base + hw[i] + P - hx) % P;
    }
    auto plane = [&](int zz) -> uint32_t {
        const int w = zz < 0 ? zz + (int)nz : (zz >= (int)nz ? zz - (int)nz : zz);
        return P * (uint32_t)w;
    };

    R om[SPT][3], o0[SPT][3], op[SPT][3], opp[SPT][3];
    R sc[SPT][3], sn[SPT][3];
    R hp[kMaxHalo][3], hpp[kMaxHalo][3];

    // prologue: planes z0-1, z0, z0+1 of the other colour, window of z0 in LDS
    {
        const uint32_t fm = plane((int)z0 - 1), f0 = plane((int)z0), fp = plane((int)z0 + 1);
#pragma unroll
        for (int j = 0; j < SPT; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                om[j][c] = a.s[O][c][qm[j] + fm];
                o0[j][c] = a.s[O][c][qm[j] + f0];
                op[j][c] = a.s[O][c][qm[j] + fp];
                sc[j][c] = a.s[C][c][qm[j] + f0];
            }
#pragma unroll
        for (int i = 0; i < kMaxHalo; ++i)
            if (t + kThreads * i < nh)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    lds[c * W + hw[i]] = a.s[O][c][hg[i] + f0];
                    hp[i][c] = a.s[O][c][hg[i] + fp];
                }
#pragma unroll
        for (int j = 0; j < SPT; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) lds[c * W + hx + t + kThreads * j] = o0[j][c];
    }
    __syncthreads();

    uint32_t nacc = 0;
    Acc acc;

    for (uint32_t zi = 0; zi < zn; ++zi) {
        const uint32_t z = z0 + zi;
        const bool more = zi + 1 < zn;
        if (more) {
            const uint32_t fpp = plane((int)z + 2), fn = plane((int)z + 1);
#pragma unroll
            for (int j = 0; j < SPT; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    opp[j][c] = a.s[O][c][qm[j] + fpp];
                    sn[j][c] = a.s[C][c][qm[j] + fn];
                }
#pragma unroll
            for (int i = 0; i < kMaxHalo; ++i)
                if (t + kThreads * i < nh)
#pragma unroll
                    for (int c = 0; c < 3; ++c) hpp[i][c] = a.s[O][c][hg[i] + fpp];
        }

        const R* Lw = lds + (zi & 1u) * 3u * W;
        const uint32_t fz = P * z;
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            if (!act[j]) continue;
            const uint32_t w = hx + t + kThreads * j;
            const uint32_t p = (yy[j] + z + (uint32_t)C) & 1u;
            // window index of the x-neighbour that is not the same-k partner
            const uint32_t wd = p ? (kx[j] == hx - 1 ? w + 1 - hx : w + 1)
                                  : (kx[j] == 0 ? w + hx - 1 : w - 1);
            R nb[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R xd = Lw[c * W + wd];
                const R xm = p ? o0[j][c] : xd;
                const R xp = p ? xd : o0[j][c];
                nb[c] = ((((xm + xp) + Lw[c * W + w - hx]) + Lw[c * W + w + hx]) + om[j][c]) + op[j][c];
            }
            const V3<R> hl{m.J * nb[0] + m.h.x, m.J * nb[1] + m.h.y, m.J * nb[2] + m.h.z};
            const V3<R> s{sc[j][0], sc[j][1], sc[j][2]};
            const uint32_t k = qm[j] + fz;
            const Rand4 rn = philox(sweep, 2u * k + p, (uint32_t)C, a.inst, a.key0, a.key1);
            const V3<R> tr = cone_move(s, Prim<R>::u01(rn.r0), Prim<R>::u01(rn.r1), c1);
            const R dE = delta_e(m, s, tr, hl);
            const bool ok = Prim<R>::u01(rn.r2) < Prim<R>::boltzmann(dE, scale);
            const V3<R> f = ok ? tr : s;
            a.s[C][0][k] = f.x;
            a.s[C][1][k] = f.y;
            a.s[C][2][k] = f.z;
            nacc += ok ? 1u : 0u;
            if (OBS) {
                const V3<R> partner{o0[j][0], o0[j][1], o0[j][2]};
                acc.ex += (double)(-m.J * (f.x * nb[0] + f.y * nb[1] + f.z * nb[2]));
                add_site<R, false>(acc, m, f);
                add_site<R, false>(acc, m, partner);
            }
        }

        if (more) {
            R* Ln = lds + ((zi + 1u) & 1u) * 3u * W;
#pragma unroll
            for (int j = 0; j < SPT; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) Ln[c * W + hx + t + kThreads * j] = op[j][c];
#pragma unroll
            for (int i = 0; i < kMaxHalo; ++i)
                if (t + kThreads * i < nh)
#pragma unroll
                    for (int c = 0; c < 3; ++c) Ln[c * W + hw[i]] = hp[i][c];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < SPT; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                om[j][c] = o0[j][c];
                o0[j][c] = op[j][c];
                op[j][c] = opp[j][c];
                sc[j][c] = sn[j][c];
            }
#pragma unroll
        for (int i = 0; i < kMaxHalo; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) hp[i][c] = hpp[i][c];
    }

    // LDS is free after the last barrier of the loop
    double* scratch = reinterpret_cast<double*>(smem);
    block_count_write(nacc, reinterpret_cast<uint32_t*>(scratch + 64), a.cnt + (size_t)C * a.cnt_stride + b);
    if (OBS) write_partials<R>(acc, a.part, b, scratch);
}

// ---------------------------------------------------------------------------
// Neighbour sum of colour index k of colour C (its six neighbours are of the
// other colour), in the order x-, x+, y-, y+, z-, z+; also the other-colour
// x-partner with the same index.  Used by the gather kernels.
// ---------------------------------------------------------------------------
template <typename R, int C>
__device__ __forceinline__ void gather_neighbours(const KArgs<R>& a, uint32_t k, V3<R>& nb, V3<R>& partner,
                                                  uint32_t& site)
{
    constexpr int O = 1 - C;
    const uint32_t hx = a.hx, ny = a.ny, nz = a.nz, P = a.P;
    const uint32_t kx = k % hx, r = k / hx;
    const uint32_t y = r % ny, z = r / ny;
    const uint32_t p = (y + z + (uint32_t)C) & 1u;
    site = 2u * k + p;
    const uint32_t row = k - kx;                      // hx*(y + ny*z)
    const uint32_t d = p ? (kx == hx - 1 ? row : k + 1) : (kx == 0 ? row + hx - 1 : k - 1);
    const uint32_t fz = P * z;
    const uint32_t ym = kx + hx * (y == 0 ? ny - 1 : y - 1) + fz;
    const uint32_t yp = kx + hx * (y == ny - 1 ? 0 : y + 1) + fz;
    const uint32_t inpl = kx + hx * y;
    const uint32_t zm = inpl + P * (z == 0 ? nz - 1 : z - 1);
    const uint32_t zp = inpl + P * (z == nz - 1 ? 0 : z + 1);
    R v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R* o = a.s[O][c];
        const R same = o[k], xd = o[d];
        const R xm = p ? same : xd;
        const R xp = p ? xd : same;
        v[c] = ((((xm + xp) + o[ym]) + o[yp]) + o[zm]) + o[zp];
        (&partner.x)[c] = same;
    }
    nb = V3<R>{v[0], v[1], v[2]};
}

// ---------------------------------------------------------------------------
// Constrained pair pass (Table A2, ConstrainedMonteCarlo_ParallelPass), one
// thread per pair of colour C.  The shuffled order pi of the colour indices
// is a keyed bijection evaluated inline (nothing is stored); pair k is
// (pi(2k), pi(2k+1)).  M_L is the moment along eC at the start of the sweep
// (one value for both colours, as in the paper).  OBS (black pass) fuses the
// observables over the two black sites and their red x-partners; because pi
// is a bijection every site is covered once.
// ---------------------------------------------------------------------------
template <typename R, int C, bool OBS>
__global__ __launch_bounds__(kThreads) void pair_kernel(const KArgs<R> a, const V3<R> ec, const uint32_t half,
                                                        const uint32_t mask, const uint32_t npairs, const R scale)
{
    __shared__ double scratch[kNumPart * (kThreads / 64) + 8];
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const int theta = a.st->theta;
    const uint32_t sweep = (uint32_t)a.st->sweep;
    const R c1 = a.c1tab[theta];
    const Model<R> m = a.m;
    const double* M = a.st->M;
    const double ML = M[0] * (double)ec.x + M[1] * (double)ec.y + M[2] * (double)ec.z;
    const R invML = (R)(1.0 / fabs(ML));
    const Rand4 key = philox(sweep, 0u, 5u + (uint32_t)C, a.inst, a.key0, a.key1);

    uint32_t nacc = 0;
    Acc acc;
    if (k < npairs) {
        const uint32_t ia = shuffle_index(2u * k, a.Nc, half, mask, key);
        const uint32_t ja = shuffle_index(2u * k + 1u, a.Nc, half, mask, key);
        V3<R> nbi, nbj, pti, ptj;
        uint32_t site_i, site_j;
        gather_neighbours<R, C>(a, ia, nbi, pti, site_i);
        gather_neighbours<R, C>(a, ja, nbj, ptj, site_j);
        const V3<R> si{a.s[C][0][ia], a.s[C][1][ia], a.s[C][2][ia]};
        const V3<R> sj{a.s[C][0][ja], a.s[C][1][ja], a.s[C][2][ja]};
        const Rand4 rn = philox(sweep, k, 2u + (uint32_t)C, a.inst, a.key0, a.key1);
        const V3<R> ti = cone_move(si, Prim<R>::u01(rn.r0), Prim<R>::u01(rn.r1), c1);

        // compensation of the transverse change, along/perpendicular to eC
        const R pi_old = dot(si, ec), pi_new = dot(ti, ec), pj_old = dot(sj, ec);
        V3<R> pj;
        pj.x = (sj.x - pj_old * ec.x) + (si.x - pi_old * ec.x) - (ti.x - pi_new * ec.x);
        pj.y = (sj.y - pj_old * ec.y) + (si.y - pi_old * ec.y) - (ti.y - pi_new * ec.y);
        pj.z = (sj.z - pj_old * ec.z) + (si.z - pi_old * ec.z) - (ti.z - pi_new * ec.z);
        const R q = dot(sj, sj) - dot(pj, pj);
        bool ok = q > R(0);
        const R pj_new = (pj_old >= R(0) ? R(1) : R(-1)) * Prim<R>::sqrt_(ok ? q : R(1));
        const V3<R> tj{pj.x + pj_new * ec.x, pj.y + pj_new * ec.y, pj.z + pj_new * ec.z};
        // (M_L'/M_L)^2 with M_L' = |M_L| + change along eC
        const R x = ((pi_new + pj_new) - pi_old - pj_old) * invML;
        ok = ok && (R(1) + x > R(0)) && (ML != 0.0);
        const V3<R> hi{m.J * nbi.x + m.h.x, m.J * nbi.y + m.h.y, m.J * nbi.z + m.h.z};
        const V3<R> hj{m.J * nbj.x + m.h.x, m.J * nbj.y + m.h.y, m.J * nbj.z + m.h.z};
        const R dE = delta_e(m, si, ti, hi) + delta_e(m, sj, tj, hj);
        const R ratio = (R(1) + x) * (R(1) + x) * fabs(pj_old / pj_new);
        ok = ok && (Prim<R>::u01(rn.r2) < ratio * Prim<R>::boltzmann(dE, scale));
        const V3<R> fi = ok ? ti : si;
        const V3<R> fj = ok ? tj : sj;
        if (ok) {
            a.s[C][0][ia] = ti.x; a.s[C][1][ia] = ti.y; a.s[C][2][ia] = ti.z;
            a.s[C][0][ja] = tj.x; a.s[C][1][ja] = tj.y; a.s[C][2][ja] = tj.z;
            nacc = 2;
        }
        if (OBS) {
            acc.ex += (double)(-m.J * dot(fi, nbi)) + (double)(-m.J * dot(fj, nbj));
            add_site<R, true>(acc, m, fi);
            add_site<R, true>(acc, m, fj);
            add_site<R, true>(acc, m, pti);
            add_site<R, true>(acc, m, ptj);
        }
    }
    block_count_write(nacc, reinterpret_cast<uint32_t*>(scratch + kNumPart * (kThreads / 64)),
                      a.cnt + (size_t)C * a.cnt_stride + blockIdx.x);
    if (OBS) write_partials<R>(acc, a.part, blockIdx.x, scratch);
}

// ---------------------------------------------------------------------------
// Measurement of the current spins: one thread per colour index k covers the
// black site k (with its six red neighbours: every bond once) and the red
// site k.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void measure_kernel(const KArgs<R> a)
{
    __shared__ double scratch[kNumPart * (kThreads / 64) + 8];
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    Acc acc;
    if (k < a.Nc) {
        V3<R> nb, red;
        uint32_t site;
        gather_neighbours<R, 1>(a, k, nb, red, site);
        const V3<R> blk{a.s[1][0][k], a.s[1][1][k], a.s[1][2][k]};
        acc.ex += (double)(-a.m.J * dot(blk, nb));
        add_site<R, true>(acc, a.m, blk);
        add_site<R, true>(acc, a.m, red);
    }
    write_partials<R>(acc, a.part, blockIdx.x, scratch);
}

// ---------------------------------------------------------------------------
// Per-sweep finalize (one work-group): fixed-order reduction of the
// work-group partials, the adaptive cone angle of Table A1 (one degree up
// when accepted/N > 1/2, else down, within [1, 180]), the sweep counter,
// and on sampled sweeps the shifted FP64 accumulators of Eq. 6.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void finalize_kernel(DevState* st, const double* part, const uint32_t* cnt,
                                                            uint32_t cnt_stride, uint32_t nred, uint32_t nblack,
                                                            uint32_t npart, int flags, double T, double N)
{
    __shared__ double red_d[kThreads];
    __shared__ unsigned long long red_i[kThreads];
    __shared__ double tot[kNumPart];
    const uint32_t t = threadIdx.x;

    unsigned long long c = 0;
    if (flags & kFinCounts) {
        for (uint32_t i = t; i < nred; i += kThreads) c += cnt[i];
        for (uint32_t i = t; i < nblack; i += kThreads) c += cnt[cnt_stride + i];
    }
    red_i[t] = c;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < (uint32_t)s) red_i[t] += red_i[t + s];
        __syncthreads();
    }
    if (flags & kFinObs) {
        for (int slot = 0; slot < kNumPart; ++slot) {
            double v = 0.0;
            for (uint32_t i = t; i < npart; i += kThreads) v += part[(size_t)i * kNumPart + slot];
            red_d[t] = v;
            __syncthreads();
            for (int s = kThreads / 2; s > 0; s >>= 1) {
                if (t < (uint32_t)s) red_d[t] += red_d[t + s];
                __syncthreads();
            }
            if (t == 0) tot[slot] = red_d[0];
            __syncthreads();
        }
    }
    if (t != 0) return;

    if (flags & kFinCounts) {
        const long long accepted = (long long)red_i[0];
        st->accepted_last = accepted;
        if (2.0 * (double)accepted > N) {
            if (st->theta < 180) st->theta += 1;
        } else {
            if (st->theta > 1) st->theta -= 1;
        }
        st->sweep += 1;
    }
    if (flags & kFinObs) {
        bool finite = true;
        for (int i = 0; i < 10; ++i) finite = finite && isfinite(tot[i]);
        if (!finite) st->nonfinite = 1;
        st->M[0] = tot[kMx];
        st->M[1] = tot[kMy];
        st->M[2] = tot[kMz];
        st->E_exch = tot[kEexch];
        st->E_uni = tot[kEuni];
        st->E_cub = tot[kEcub];
        st->E_zee = tot[kEzee];
        if (flags & kFinTorque) {
            st->torque[0] = tot[kTx];
            st->torque[1] = tot[kTy];
            st->torque[2] = tot[kTz];
        }
        if (flags & kFinSample) {
            double x[5];
            x[1] = tot[kMx] / N;
            x[2] = tot[kMy] / N;
            x[3] = tot[kMz] / N;
            x[0] = sqrt(x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
            x[4] = (tot[kEexch] + tot[kEuni] + tot[kEcub] + tot[kEzee]) / N;
            if (st->samples == 0)
                for (int i = 0; i < 5; ++i) st->shift[i] = x[i];
            for (int i = 0; i < 5; ++i) {
                const double d = x[i] - st->shift[i];
                st->sum[i] += d;
                st->sum2[i] += d * d;
            }
            st->sum_eanis += (tot[kEuni] + tot[kEcub]) / N;
            if (flags & kFinTorque) {
                for (int i = 0; i < 3; ++i) st->sum_torque[i] += tot[kTx + i] / N;
                st->torque_samples += 1;
            }
            st->samples += 1;
            st->T_sample = T;
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

int64_t max_blocks_for(int32_t nx, int32_t ny, int32_t nz)
{
    const uint64_t P = (uint64_t)(nx / 2) * (uint64_t)ny;
    return (int64_t)cdiv(P, kThreads) * (int64_t)nz;
}

int64_t pass_blocks(const DevLattice& d, int spt, int zc)
{
    return (int64_t)cdiv((uint64_t)d.P, (uint64_t)kThreads * spt) * (int64_t)cdiv((uint64_t)d.nz, (uint64_t)zc);
}

hipError_t launch_init(const DevLattice& d, hipStream_t s)
{
    dim3 grid(cdiv((uint64_t)d.Nc, kThreads), 2);
    if (d.precision == 32) {
        auto a = make_args<float>(d);
        init_kernel<float><<<grid, kThreads, 0, s>>>(a, d.init_mode, (float)d.init_dir[0], (float)d.init_dir[1],
                                                     (float)d.init_dir[2]);
    } else {
        auto a = make_args<double>(d);
        init_kernel<double><<<grid, kThreads, 0, s>>>(a, d.init_mode, d.init_dir[0], d.init_dir[1], d.init_dir[2]);
    }
    return hipGetLastError();
}

template <typename R, int C, bool OBS, int SPT>
static void pass_go(const DevLattice& d, int zc, double T, hipStream_t s)
{
    const auto a = make_args<R>(d);
    const uint32_t nqb = cdiv((uint64_t)d.P, (uint64_t)kThreads * SPT);
    const uint32_t nzb = cdiv((uint64_t)d.nz, (uint64_t)zc);
    const uint32_t nblk = nqb * nzb;
    const size_t lds = 2 * 3 * (size_t)(kThreads * SPT + 2 * d.hx) * sizeof(R);
    pass_kernel<R, C, OBS, SPT><<<nblk, kThreads, lds < 1024 ? 1024 : lds, s>>>(a, (uint32_t)zc, nqb, nblk,
                                                                                 Prim<R>::scale_for(T));
}

template <typename R, int SPT>
static void pass_dispatch_c(const DevLattice& d, int colour, bool obs, int zc, double T, hipStream_t s)
{
    if (colour == 0) pass_go<R, 0, false, SPT>(d, zc, T, s);
    else if (obs) pass_go<R, 1, true, SPT>(d, zc, T, s);
    else pass_go<R, 1, false, SPT>(d, zc, T, s);
}

template <typename R>
static void pass_dispatch(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s)
{
    if (spt == 1) pass_dispatch_c<R, 1>(d, colour, obs, zc, T, s);
    else if (spt == 2) pass_dispatch_c<R, 2>(d, colour, obs, zc, T, s);
    else pass_dispatch_c<R, 4>(d, colour, obs, zc, T, s);
}

hipError_t launch_pass(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s,
                       int64_t* blocks)
{
    if (d.precision == 32) pass_dispatch<float>(d, colour, obs, spt, zc, T, s);
    else pass_dispatch<double>(d, colour, obs, spt, zc, T, s);
    *blocks = pass_blocks(d, spt, zc);
    return hipGetLastError();
}

template <typename R>
static void pair_go(const DevLattice& d, int colour, const double eC[3], double T, hipStream_t s)
{
    const auto a = make_args<R>(d);
    const uint32_t n = (uint32_t)d.Nc;
    uint32_t bits = 2;
    while (bits < 32 && (1ull << bits) < n) bits += 2;
    const uint32_t half = bits / 2;
    const uint32_t mask = half >= 32 ? 0xFFFFFFFFu : ((1u << half) - 1u);
    const uint32_t npairs = n / 2;
    const V3<R> ec{(R)eC[0], (R)eC[1], (R)eC[2]};
    const uint32_t grid = cdiv(npairs, kThreads);
    const R scale = Prim<R>::scale_for(T);
    if (colour == 0) pair_kernel<R, 0, false><<<grid, kThreads, 0, s>>>(a, ec, half, mask, npairs, scale);
    else pair_kernel<R, 1, true><<<grid, kThreads, 0, s>>>(a, ec, half, mask, npairs, scale);
}

hipError_t launch_pair_pass(const DevLattice& d, int colour, const double eC[3], double T, hipStream_t s,
                            int64_t* blocks)
{
    if (d.precision == 32) pair_go<float>(d, colour, eC, T, s);
    else pair_go<double>(d, colour, eC, T, s);
    *blocks = cdiv((uint64_t)(d.Nc / 2), kThreads);
    return hipGetLastError();
}

hipError_t launch_measure(const DevLattice& d, hipStream_t s, int64_t* blocks)
{
    const uint32_t grid = cdiv((uint64_t)d.Nc, kThreads);
    if (d.precision == 32) measure_kernel<float><<<grid, kThreads, 0, s>>>(make_args<float>(d));
    else measure_kernel<double><<<grid, kThreads, 0, s>>>(make_args<double>(d));
    *blocks = grid;
    return hipGetLastError();
}

hipError_t launch_finalize(const DevLattice& d, int64_t red_blocks, int64_t black_blocks, int64_t part_blocks,
                           int flags, double T, hipStream_t s)
{
    finalize_kernel<<<1, kThreads, 0, s>>>(d.st, d.part, d.cnt, (uint32_t)d.max_blocks, (uint32_t)red_blocks,
                                            (uint32_t)black_blocks, (uint32_t)part_blocks, flags, T, (double)d.N);
    return hipGetLastError();
}

}  // namespace hmc
