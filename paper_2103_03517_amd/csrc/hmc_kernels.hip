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
//
// Global memory is accessed through buffer resources: the per-plane offset
// travels in a scalar register, so the per-column offsets are computed once,
// and out-of-range accesses are dropped by the hardware.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "hmc_device.hpp"
#include "hmc_internal.h"

namespace hmc {

constexpr int32_t kBufferConfig = 0x00020000;   // raw buffer, gfx9-family data format

template <typename R>
struct KArgs {
    R* s[2][3];
    uint32_t hx, ny, nz, P, Nc;
    uint32_t arr_bytes;  // bytes of one component array (range of the buffer resources)
    Model<R> m;
    uint32_t key0, key1, inst;
    DevState* st;
    const R* c1tab;
    double* part;
    uint32_t* cnt;       // [2][cnt_stride]
    uint32_t cnt_stride;
    uint32_t apz;        // 1: anti-periodic along z (the z-wrap bond enters with a minus sign)
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
    a.arr_bytes = (uint32_t)((uint64_t)d.Nc * sizeof(R));
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
    a.apz = (uint32_t)d.apz;
    return a;
}

// One lattice of a batch (device table, filled on the host by
// batch_fill_entry): its kernel arguments and its launch shape.
template <typename R>
struct BatchEntry {
    KArgs<R> a;
    uint32_t zc, nqb, nblk, pad;
    double N;
};

// ---------------------------------------------------------------------------
// Buffer-resource access to the six component arrays.
// ---------------------------------------------------------------------------
template <typename R> struct Gm;

template <> struct Gm<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
    }
};

template <> struct Gm<double> {
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, double v)
    {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
    }
};

template <typename R>
__device__ __forceinline__ V3<R> neg(const V3<R>& v)
{
    return V3<R>{-v.x, -v.y, -v.z};
}

template <typename R>
struct Arrays {
    __amdgpu_buffer_rsrc_t r[2][3];
    __device__ __forceinline__ explicit Arrays(const KArgs<R>& a)
    {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                r[c][k] = __builtin_amdgcn_make_buffer_rsrc(a.s[c][k], 0, (int)a.arr_bytes, kBufferConfig);
    }
    // spin of colour c at byte offset voff + soff
    __device__ __forceinline__ V3<R> get(int c, uint32_t voff, uint32_t soff) const
    {
        return V3<R>{Gm<R>::ld(r[c][0], voff, soff), Gm<R>::ld(r[c][1], voff, soff), Gm<R>::ld(r[c][2], voff, soff)};
    }
    __device__ __forceinline__ void put(int c, uint32_t voff, uint32_t soff, const V3<R>& v) const
    {
        Gm<R>::st(r[c][0], voff, soff, v.x);
        Gm<R>::st(r[c][1], voff, soff, v.y);
        Gm<R>::st(r[c][2], voff, soff, v.z);
    }
};

// ---------------------------------------------------------------------------
// LDS plane of the other colour: float4 entries for FP32 (one 16-byte access
// per neighbour), three component planes for FP64.
// ---------------------------------------------------------------------------
template <typename R> struct LdsPlane;

template <> struct LdsPlane<float> {
    static constexpr size_t bytes_per_entry = 16;
    static __device__ __forceinline__ void put(unsigned char* p, uint32_t W, uint32_t e, const V3<float>& v)
    {
        (void)W;
        reinterpret_cast<float4*>(p)[e] = make_float4(v.x, v.y, v.z, 0.0f);
    }
    static __device__ __forceinline__ V3<float> get(const unsigned char* p, uint32_t W, uint32_t e)
    {
        (void)W;
        const float4 q = reinterpret_cast<const float4*>(p)[e];
        return V3<float>{q.x, q.y, q.z};
    }
};

template <> struct LdsPlane<double> {
    static constexpr size_t bytes_per_entry = 24;
    static __device__ __forceinline__ void put(unsigned char* p, uint32_t W, uint32_t e, const V3<double>& v)
    {
        double* d = reinterpret_cast<double*>(p);
        d[e] = v.x;
        d[W + e] = v.y;
        d[2 * W + e] = v.z;
    }
    static __device__ __forceinline__ V3<double> get(const unsigned char* p, uint32_t W, uint32_t e)
    {
        const double* d = reinterpret_cast<const double*>(p);
        return V3<double>{d[e], d[W + e], d[2 * W + e]};
    }
};

size_t pass_lds_bytes(int precision, int hx, int spt)
{
    const size_t W = (size_t)kThreads * spt + 2 * (size_t)hx;
    const size_t e = precision == 32 ? LdsPlane<float>::bytes_per_entry : LdsPlane<double>::bytes_per_entry;
    const size_t b = 2 * W * e;
    return b < 1024 ? 1024 : b;
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

// ---------------------------------------------------------------------------
// Fixed-order reductions.  Within a wave a butterfly, across the four waves
// of a work-group in wave order, across work-groups by the finalize kernel,
// each thread taking work-groups t, t+256, ... in order.  The results
// therefore do not depend on scheduling.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sums NV values over the work-group; the totals land in scratch[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) scratch[NV + wave * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += scratch[NV + w * NV + threadIdx.x];
        scratch[threadIdx.x] = s;
    }
    __syncthreads();
}

// The end of a producing launch: work-group b writes its acceptance count
// and (OBS) its partial sums.  They are reduced by finalize_kernel, launched
// next on the same stream (the kernel boundary makes them visible).
template <typename R, bool OBS>
__device__ __forceinline__ void block_end(const KArgs<R>& a, int colour, uint32_t b, uint32_t nacc, const Acc& acc,
                                          double* scratch)
{
    if (OBS) {
        double v[kNumPart] = {acc.M[0], acc.M[1], acc.M[2], acc.ex, acc.eu, acc.ec, acc.ez,
                              acc.tq[0], acc.tq[1], acc.tq[2], (double)nacc, 0.0};
        block_sum<kNumPart>(v, scratch);
        if (threadIdx.x < kNumPart) a.part[(size_t)b * kNumPart + threadIdx.x] = scratch[threadIdx.x];
        if (threadIdx.x == 0) a.cnt[(size_t)colour * a.cnt_stride + b] = (uint32_t)scratch[10];
    } else {
        uint32_t c = wave_sum(nacc);
        __syncthreads();
        uint32_t* s32 = reinterpret_cast<uint32_t*>(scratch);
        if ((threadIdx.x & 63) == 0) s32[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < kThreads / 64; ++w) tot += s32[w];
            a.cnt[(size_t)colour * a.cnt_stride + b] = tot;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-sweep finalize (one work-group): the fixed-order reduction of the
// work-group results of the colour-1 (and, for the counts, colour-0) launch,
// then Table A1's cone-angle rule (one degree up when accepted/N > 1/2, else
// down, within [1, 180]), the sweep counter and on sampled sweeps the
// shifted FP64 accumulators of Eq. 6.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void finalize_body(DevState* st, const double* part, const uint32_t* cnt,
                                              uint32_t cnt_stride, uint32_t nred, uint32_t nblack, uint32_t npart,
                                              int fin, double T, double N, double* scratch)
{
    const uint32_t t = threadIdx.x;
    double v[kNumPart + 1];
#pragma unroll
    for (int i = 0; i <= kNumPart; ++i) v[i] = 0.0;
    if (fin & kFinCounts) {
        unsigned long long c = 0;
        for (uint32_t i = t; i < nred; i += kThreads) c += cnt[i];
        for (uint32_t i = t; i < nblack; i += kThreads) c += cnt[cnt_stride + i];
        v[kNumPart] = (double)c;
    }
    if (fin & kFinObs) {
        // each thread takes whole 96-byte records: six independent 16-byte loads
        for (uint32_t i = t; i < npart; i += kThreads) {
            const double2* p = reinterpret_cast<const double2*>(part + (size_t)i * kNumPart);
#pragma unroll
            for (int k = 0; k < kNumPart / 2; ++k) {
                const double2 q = p[k];
                v[2 * k] += q.x;
                v[2 * k + 1] += q.y;
            }
        }
    }
    block_sum<kNumPart + 1>(v, scratch);
    if (t != 0) return;
    const double* tot = scratch;
    if (fin & kFinCounts) {
        const long long accepted = (long long)tot[kNumPart];
        st->accepted_last = accepted;
        if (2.0 * (double)accepted > N) {
            if (st->theta < 180) st->theta += 1;
        } else {
            if (st->theta > 1) st->theta -= 1;
        }
        st->sweep += 1;
    }
    if (fin & kFinObs) {
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
        if (fin & kFinTorque) {
            st->torque[0] = tot[kTx];
            st->torque[1] = tot[kTy];
            st->torque[2] = tot[kTz];
        }
        if (fin & kFinSample) {
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
            if (fin & kFinTorque) {
                for (int i = 0; i < 3; ++i) st->sum_torque[i] += tot[kTx + i] / N;
                st->torque_samples += 1;
            }
            st->samples += 1;
            st->T_sample = T;
        }
    }
}

__global__ __launch_bounds__(kThreads) void finalize_kernel(DevState* st, const double* part, const uint32_t* cnt,
                                                            uint32_t cnt_stride, uint32_t nred, uint32_t nblack,
                                                            uint32_t npart, int fin, double T, double N)
{
    __shared__ double scratch[5 * (kNumPart + 1)];
    finalize_body(st, part, cnt, cnt_stride, nred, nblack, npart, fin, T, N, scratch);
}

// Finalize of a batch: work-group i folds the results of lattice i with its
// own flags fin[i] (a lattice that does not sample ignores the partials of a
// black pass that computed them for others).
template <typename R>
__global__ __launch_bounds__(kThreads) void finalize_batch_kernel(const BatchEntry<R>* __restrict__ tab,
                                                                  const double* __restrict__ T,
                                                                  const int32_t* __restrict__ fin)
{
    __shared__ double scratch[5 * (kNumPart + 1)];
    const BatchEntry<R>& E = tab[blockIdx.x];
    const int f = fin[blockIdx.x];
    finalize_body(E.a.st, E.a.part, E.a.cnt, E.a.cnt_stride, E.nblk, E.nblk, (f & kFinObs) ? E.nblk : 0u, f,
                  T[blockIdx.x], E.N, scratch);
}

// Clears the accumulators of every lattice of a batch (work-group i, lattice
// i); spins, cone angle, counters and the last measurement are kept.
template <typename R>
__global__ __launch_bounds__(64) void reset_batch_kernel(const BatchEntry<R>* __restrict__ tab)
{
    if (threadIdx.x != 0) return;
    DevState* st = tab[blockIdx.x].a.st;
    st->samples = 0;
    st->torque_samples = 0;
    for (int i = 0; i < 5; ++i) st->shift[i] = st->sum[i] = st->sum2[i] = 0.0;
    st->sum_eanis = 0.0;
    for (int i = 0; i < 3; ++i) st->sum_torque[i] = 0.0;
    st->T_sample = 0.0;
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
// The Metropolis update of one site (Table A1, Eq. 1, Eq. 2): cone proposal,
// energy change in the local field, acceptance P < exp(-dE/T).  Returns the
// final spin; OBS adds the site and its red x-partner to the observables.
// ---------------------------------------------------------------------------
template <typename R, bool OBS>
__device__ __forceinline__ V3<R> update_site(const Model<R>& m, const V3<R>& s, const V3<R>& nb,
                                             const V3<R>& partner, const Rand4& rn, R c1, R scale,
                                             uint32_t& nacc, Acc& acc)
{
    const V3<R> hl{m.J * nb.x + m.h.x, m.J * nb.y + m.h.y, m.J * nb.z + m.h.z};
    const V3<R> tr = cone_move(s, Prim<R>::u01(rn.r0), Prim<R>::u01(rn.r1), c1);
    SiteTerms<R> k;
    const R dE = delta_e(m, s, tr, hl, k);
    const bool ok = Prim<R>::u01(rn.r2) < Prim<R>::boltzmann(dE, scale);
    const V3<R> f = ok ? tr : s;
    nacc += ok ? 1u : 0u;
    if (OBS) {
        const V3<R> fp{f.x + partner.x, f.y + partner.y, f.z + partner.z};
        acc.M[0] += (double)fp.x;
        acc.M[1] += (double)fp.y;
        acc.M[2] += (double)fp.z;
        acc.ex += (double)(-m.J * dot(f, nb));
        if (m.Ku != R(0)) {
            const R sf = ok ? k.te : k.se, sp = dot(partner, m.e);
            acc.eu += (double)(-m.Ku * (sf * sf + sp * sp));
        }
        if (m.Kc != R(0)) acc.ec += (double)(m.Kc * ((ok ? k.ct : k.cs) + cubic_f(partner)));
        acc.ez += (double)(-dot(m.h, fp));
    }
    return f;
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
// computed.  The march is unrolled by four so that the four register planes
// rotate by renaming.  OBS (black pass only) fuses the observables: the black
// site after its update plus its red x-partner (same colour index), and the
// exchange of the black site with its six final red neighbours, so every
// site and every bond is counted once.
// ---------------------------------------------------------------------------
template <typename R, int SPT, int HALO>
struct PassCtx {
    uint32_t hx, P, nz, W, z0, zn;
    uint32_t voff[SPT];          // byte offset of each owned column in a plane
    uint32_t w[SPT];             // its LDS entry
    uint32_t wd[2][SPT];         // LDS entry of its second x-neighbour, by z parity
    uint32_t par[SPT];           // x parity of the column at z = z0
    bool act[SPT];
    uint32_t hvoff[HALO], hw[HALO];
    bool hact[HALO];
    unsigned char* lds[2];
    R c1, scale;
    uint32_t sweep;
    bool apz;
};

template <typename R, int C, bool OBS, int SPT, int HALO, int K>
__device__ __forceinline__ void pass_step(const KArgs<R>& a, const Arrays<R>& g, const PassCtx<R, SPT, HALO>& x,
                                          uint32_t zi, V3<R> (&om)[SPT], V3<R> (&o0)[SPT], V3<R> (&op)[SPT],
                                          V3<R> (&opp)[SPT], V3<R> (&sc)[SPT], V3<R> (&sn)[SPT],
                                          V3<R> (&hp)[HALO], V3<R> (&hpp)[HALO], uint32_t& nacc, Acc& acc)
{
    constexpr int O = 1 - C;
    constexpr int B = K & 1;
    const uint32_t z = x.z0 + zi;
    const bool more = zi + 1 < x.zn;
    auto plane_off = [&](uint32_t zz) -> uint32_t {
        return x.P * (uint32_t)sizeof(R) * (zz >= x.nz ? zz - x.nz : zz);
    };
    if (more) {
        const uint32_t fpp = plane_off(z + 2), fn = plane_off(z + 1);
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            opp[j] = g.get(O, x.voff[j], fpp);
            sn[j] = g.get(C, x.voff[j], fn);
        }
#pragma unroll
        for (int i = 0; i < HALO; ++i)
            if (x.hact[i]) hpp[i] = g.get(O, x.hvoff[i], fpp);
        // anti-periodic z: plane z + 2 = nz is plane 0 seen across the
        // boundary; it serves only as the z+1 neighbour of plane nz - 1.
        // The uniform branch is taken once per tile at most.
        if (__builtin_expect(x.apz && z + 2u == x.nz, 0)) {
            __asm__ volatile("");
#pragma unroll
            for (int j = 0; j < SPT; ++j) opp[j] = neg(opp[j]);
        }
    }
    const unsigned char* L = x.lds[B];
    const uint32_t fz = plane_off(z);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        if (!x.act[j]) continue;
        const uint32_t p = x.par[j] ^ (uint32_t)B;
        const V3<R> xd = LdsPlane<R>::get(L, x.W, x.wd[B][j]);
        const V3<R> ym = LdsPlane<R>::get(L, x.W, x.w[j] - x.hx);
        const V3<R> yp = LdsPlane<R>::get(L, x.W, x.w[j] + x.hx);
        const V3<R> xm = p ? o0[j] : xd;
        const V3<R> xp = p ? xd : o0[j];
        const V3<R> nb{((((xm.x + xp.x) + ym.x) + yp.x) + om[j].x) + op[j].x,
                       ((((xm.y + xp.y) + ym.y) + yp.y) + om[j].y) + op[j].y,
                       ((((xm.z + xp.z) + ym.z) + yp.z) + om[j].z) + op[j].z};
        const uint32_t k = x.voff[j] / (uint32_t)sizeof(R) + x.P * (z >= x.nz ? z - x.nz : z);
        const Rand4 rn = philox(x.sweep, 2u * k + p, (uint32_t)C, a.inst, a.key0, a.key1);
        const V3<R> f = update_site<R, OBS>(a.m, sc[j], nb, o0[j], rn, x.c1, x.scale, nacc, acc);
        g.put(C, x.voff[j], fz, f);
    }
    if (more) {
        unsigned char* Ln = x.lds[B ^ 1];
#pragma unroll
        for (int j = 0; j < SPT; ++j) LdsPlane<R>::put(Ln, x.W, x.w[j], op[j]);
#pragma unroll
        for (int i = 0; i < HALO; ++i)
            if (x.hact[i]) LdsPlane<R>::put(Ln, x.W, x.hw[i], hp[i]);
    }
    __syncthreads();
}

// One work-group of a colour pass: logical tile b (column block b % nqb,
// z-slab b / nqb) of the lattice described by a.
template <typename R, int C, bool OBS, int SPT, int HALO>
__device__ __forceinline__ void pass_tile(const KArgs<R>& a, const uint32_t zc, const uint32_t nqb, const uint32_t b,
                                          const R scale, unsigned char* smem)
{
    constexpr int O = 1 - C;
    constexpr uint32_t Q = kThreads * SPT;

    const Arrays<R> g(a);
    PassCtx<R, SPT, HALO> x;
    x.hx = a.hx;
    x.P = a.P;
    x.nz = a.nz;
    x.W = Q + 2u * a.hx;
    const uint32_t t = threadIdx.x;
    const uint32_t qb = b % nqb, zb = b / nqb;
    const uint32_t base = qb * Q;
    x.z0 = zb * zc;
    x.zn = min(zc, a.nz - x.z0);
    x.lds[0] = smem;
    x.lds[1] = smem + (size_t)x.W * LdsPlane<R>::bytes_per_entry;
    x.c1 = a.c1tab[a.st->theta];
    x.sweep = (uint32_t)a.st->sweep;
    x.scale = scale;
    x.apz = a.apz != 0;

#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const uint32_t q = base + t + kThreads * j;
        x.act[j] = q < a.P;
        const uint32_t qm = x.act[j] ? q : q % a.P;
        const uint32_t kx = qm % a.hx, yy = qm / a.hx;
        x.voff[j] = qm * (uint32_t)sizeof(R);
        x.w[j] = a.hx + t + kThreads * j;
        x.par[j] = (yy + x.z0 + (uint32_t)C) & 1u;
        // window entry of the x-neighbour that is not the same-index partner:
        // x+1 (wrapping inside the row) when the site's x is odd, else x-1
#pragma unroll
        for (int bpar = 0; bpar < 2; ++bpar) {
            const uint32_t p = x.par[j] ^ (uint32_t)bpar;
            const uint32_t w = x.w[j];
            x.wd[bpar][j] = p ? (kx == a.hx - 1 ? w + 1 - a.hx : w + 1) : (kx == 0 ? w + a.hx - 1 : w - 1);
        }
    }
    const uint32_t nh = 2u * a.hx;
#pragma unroll
    for (int i = 0; i < HALO; ++i) {
        const uint32_t slot = t + kThreads * i;
        x.hact[i] = slot < nh;
        x.hw[i] = slot < a.hx ? slot : slot + Q;
        x.hvoff[i] = ((base + x.hw[i] + a.P - a.hx) % a.P) * (uint32_t)sizeof(R);
    }

    V3<R> rA[SPT], rB[SPT], rC[SPT], rD[SPT], s0[SPT], s1[SPT], h0[HALO], h1[HALO];
    {
        auto plane_off = [&](int zz) -> uint32_t {
            const int w = zz < 0 ? zz + (int)a.nz : (zz >= (int)a.nz ? zz - (int)a.nz : zz);
            return a.P * (uint32_t)sizeof(R) * (uint32_t)w;
        };
        const uint32_t fm = plane_off((int)x.z0 - 1), f0 = plane_off((int)x.z0), fp = plane_off((int)x.z0 + 1);
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            rA[j] = g.get(O, x.voff[j], fm);
            rB[j] = g.get(O, x.voff[j], f0);
            rC[j] = g.get(O, x.voff[j], fp);
            s0[j] = g.get(C, x.voff[j], f0);
        }
#pragma unroll
        for (int i = 0; i < HALO; ++i)
            if (x.hact[i]) {
                LdsPlane<R>::put(x.lds[0], x.W, x.hw[i], g.get(O, x.hvoff[i], f0));
                h0[i] = g.get(O, x.hvoff[i], fp);
            }
#pragma unroll
        for (int j = 0; j < SPT; ++j) LdsPlane<R>::put(x.lds[0], x.W, x.w[j], rB[j]);
        // anti-periodic z: the z-1 plane of z0 = 0 and the z+1 plane of
        // z0 = nz - 1 lie across the boundary (both used only as z neighbours)
        if (x.apz && x.z0 == 0) {
#pragma unroll
            for (int j = 0; j < SPT; ++j) rA[j] = neg(rA[j]);
        }
        if (x.apz && x.z0 + 1u == a.nz) {
#pragma unroll
            for (int j = 0; j < SPT; ++j) rC[j] = neg(rC[j]);
        }
    }
    __syncthreads();

    uint32_t nacc = 0;
    Acc acc;
    uint32_t zi = 0;
    for (; zi + 4 <= x.zn; zi += 4) {
        pass_step<R, C, OBS, SPT, HALO, 0>(a, g, x, zi + 0, rA, rB, rC, rD, s0, s1, h0, h1, nacc, acc);
        pass_step<R, C, OBS, SPT, HALO, 1>(a, g, x, zi + 1, rB, rC, rD, rA, s1, s0, h1, h0, nacc, acc);
        pass_step<R, C, OBS, SPT, HALO, 2>(a, g, x, zi + 2, rC, rD, rA, rB, s0, s1, h0, h1, nacc, acc);
        pass_step<R, C, OBS, SPT, HALO, 3>(a, g, x, zi + 3, rD, rA, rB, rC, s1, s0, h1, h0, nacc, acc);
    }
    if (zi < x.zn) pass_step<R, C, OBS, SPT, HALO, 0>(a, g, x, zi + 0, rA, rB, rC, rD, s0, s1, h0, h1, nacc, acc);
    if (zi + 1 < x.zn) pass_step<R, C, OBS, SPT, HALO, 1>(a, g, x, zi + 1, rB, rC, rD, rA, s1, s0, h1, h0, nacc, acc);
    if (zi + 2 < x.zn) pass_step<R, C, OBS, SPT, HALO, 2>(a, g, x, zi + 2, rC, rD, rA, rB, s0, s1, h0, h1, nacc, acc);

    // LDS is free after the last barrier of the march
    block_end<R, OBS>(a, C, b, nacc, acc, reinterpret_cast<double*>(smem));
}

template <typename R, int C, bool OBS, int SPT, int HALO>
__global__ __launch_bounds__(kThreads) void pass_kernel(const KArgs<R> a, const uint32_t zc, const uint32_t nqb,
                                                        const uint32_t nblk, const R scale)
{
    extern __shared__ __align__(16) unsigned char smem[];
    pass_tile<R, C, OBS, SPT, HALO>(a, zc, nqb, xcd_remap(blockIdx.x, nblk), scale, smem);
}

// The same colour pass over a batch of lattices in one launch.  Lattice i of
// the launch owns the logical work-groups [start[i], start[i+1]); ent[i] is
// its entry in the batch table and scale[ent[i]] its -1/T.  Each tile runs
// exactly as in the single-lattice launch, so every lattice evolves bit for
// bit as it would alone.
template <typename R, int C, bool OBS, int SPT, int HALO>
__global__ __launch_bounds__(kThreads) void pass_batch_kernel(const BatchEntry<R>* __restrict__ tab,
                                                              const uint32_t* __restrict__ start,
                                                              const uint32_t* __restrict__ ent, const uint32_t n,
                                                              const uint32_t nblk, const R* __restrict__ scale)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t gb = xcd_remap(blockIdx.x, nblk);
    uint32_t lo = 0, hi = n;   // start[lo] <= gb < start[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= gb) lo = mid;
        else hi = mid;
    }
    const uint32_t e = ent[lo];
    const BatchEntry<R>& E = tab[e];
    pass_tile<R, C, OBS, SPT, HALO>(E.a, E.zc, E.nqb, gb - start[lo], scale[e], smem);
}

// ---------------------------------------------------------------------------
// Neighbour sum of colour index k of colour C (its six neighbours are of the
// other colour), in the order x-, x+, y-, y+, z-, z+; also the other-colour
// x-partner with the same index.  Used by the gather kernels.
// ---------------------------------------------------------------------------
template <typename R, int C>
__device__ __forceinline__ void gather_neighbours(const KArgs<R>& a, const Arrays<R>& g, uint32_t k, V3<R>& nb,
                                                  V3<R>& partner, uint32_t& site)
{
    constexpr int O = 1 - C;
    constexpr uint32_t rs = sizeof(R);
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
    const V3<R> same = g.get(O, k * rs, 0), xd = g.get(O, d * rs, 0);
    const V3<R> vym = g.get(O, ym * rs, 0), vyp = g.get(O, yp * rs, 0);
    V3<R> vzm = g.get(O, zm * rs, 0), vzp = g.get(O, zp * rs, 0);
    if (a.apz) {
        if (z == 0) vzm = neg(vzm);
        if (z == nz - 1) vzp = neg(vzp);
    }
    const V3<R> xm = p ? same : xd;
    const V3<R> xp = p ? xd : same;
    nb = V3<R>{((((xm.x + xp.x) + vym.x) + vyp.x) + vzm.x) + vzp.x,
               ((((xm.y + xp.y) + vym.y) + vyp.y) + vzm.y) + vzp.y,
               ((((xm.z + xp.z) + vym.z) + vyp.z) + vzm.z) + vzp.z};
    partner = same;
}

// ---------------------------------------------------------------------------
// Constrained sweep (Table A2).  A constrained call works on an AoS copy of
// the spins (one 16-byte FP32 / 32-byte FP64 entry per site, both colours),
// made on entry and copied back on exit, so that a random gather is one
// cache line instead of three.  Before each colour pass the neighbour sums of
// that colour are precomputed (the other colour does not change during the
// pass, so they are exact); the pair pass then needs, for each spin of a
// pair, its own entry and its neighbour sum: two lines for the random
// partner instead of twenty-one.
// ---------------------------------------------------------------------------
template <typename R> struct Vec4T;
template <> struct Vec4T<float> { using type = float4; };
template <> struct Vec4T<double> { using type = double4; };
template <typename R> using Vec4 = typename Vec4T<R>::type;

template <typename R>
__device__ __forceinline__ V3<R> ld4(const Vec4<R>* p, uint32_t i)
{
    const Vec4<R> q = p[i];
    return V3<R>{q.x, q.y, q.z};
}

template <typename R>
__device__ __forceinline__ void st4(Vec4<R>* p, uint32_t i, const V3<R>& v)
{
    Vec4<R> q;
    q.x = v.x;
    q.y = v.y;
    q.z = v.z;
    q.w = R(0);
    p[i] = q;
}

// SoA -> AoS (to_aos) or AoS -> SoA, both colours; aos[c * Nc + k].
template <typename R, bool TO_AOS>
__global__ __launch_bounds__(kThreads) void aos_copy_kernel(const KArgs<R> a, Vec4<R>* aos)
{
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= a.Nc) return;
    const size_t i = (size_t)c * a.Nc + k;
    if (TO_AOS) {
        st4<R>(aos + (size_t)c * a.Nc, k, V3<R>{a.s[c][0][k], a.s[c][1][k], a.s[c][2][k]});
    } else {
        const Vec4<R> q = aos[i];
        a.s[c][0][k] = q.x;
        a.s[c][1][k] = q.y;
        a.s[c][2][k] = q.z;
    }
}

// Colour indices of the six neighbours (other colour) of colour index k of
// colour C, in the order x-, x+, y-, y+, z-, z+.
template <int C>
__device__ __forceinline__ void neighbour_indices(uint32_t k, uint32_t hx, uint32_t ny, uint32_t nz, uint32_t P,
                                                  uint32_t (&nb)[6], bool& zm_wraps, bool& zp_wraps)
{
    const uint32_t kx = k % hx, r = k / hx;
    const uint32_t y = r % ny, z = r / ny;
    const uint32_t p = (y + z + (uint32_t)C) & 1u;
    const uint32_t row = k - kx;
    const uint32_t d = p ? (kx == hx - 1 ? row : k + 1) : (kx == 0 ? row + hx - 1 : k - 1);
    const uint32_t fz = P * z, inpl = kx + hx * y;
    nb[0] = p ? k : d;
    nb[1] = p ? d : k;
    nb[2] = kx + hx * (y == 0 ? ny - 1 : y - 1) + fz;
    nb[3] = kx + hx * (y == ny - 1 ? 0 : y + 1) + fz;
    nb[4] = inpl + P * (z == 0 ? nz - 1 : z - 1);
    nb[5] = inpl + P * (z == nz - 1 ? 0 : z + 1);
    zm_wraps = z == 0;
    zp_wraps = z == nz - 1;
}

// Neighbour sums of colour C (from the AoS copy of the other colour).  With
// OBS (C = 1, after the red pass) it also adds the one-site terms of every
// red site (the same-index partner of black site k) to the observables.
template <typename R, int C, bool OBS>
__global__ __launch_bounds__(kThreads) void nbsum_kernel(const KArgs<R> a, const Vec4<R>* aos, Vec4<R>* nbs)
{
    __shared__ double scratch[5 * kNumPart];
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const Vec4<R>* other = aos + (size_t)(1 - C) * a.Nc;
    Acc acc;
    if (k < a.Nc) {
        uint32_t id[6];
        bool wm, wp;
        neighbour_indices<C>(k, a.hx, a.ny, a.nz, a.P, id, wm, wp);
        V3<R> v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = ld4<R>(other, id[i]);
        if (a.apz) {
            if (wm) v[4] = neg(v[4]);
            if (wp) v[5] = neg(v[5]);
        }
        const V3<R> nb{((((v[0].x + v[1].x) + v[2].x) + v[3].x) + v[4].x) + v[5].x,
                       ((((v[0].y + v[1].y) + v[2].y) + v[3].y) + v[4].y) + v[5].y,
                       ((((v[0].z + v[1].z) + v[2].z) + v[3].z) + v[4].z) + v[5].z};
        st4<R>(nbs, k, nb);
        if (OBS) add_site<R, true>(acc, a.m, ld4<R>(other, k));
    }
    if (OBS) {
        double vv[kNumPart] = {acc.M[0], acc.M[1], acc.M[2], acc.ex, acc.eu, acc.ec, acc.ez,
                               acc.tq[0], acc.tq[1], acc.tq[2], 0.0, 0.0};
        block_sum<kNumPart>(vv, scratch);
        if (threadIdx.x < kNumPart) a.part[(size_t)blockIdx.x * kNumPart + threadIdx.x] = scratch[threadIdx.x];
    }
}

// Pair pass of colour C.  The shuffled order pi of the colour indices is a
// keyed bijection evaluated inline (nothing is stored); pair k is
// (pi(2k), pi(2k+1)).  One thread per colour index a: the thread whose a is
// the first spin of its pair (pi^-1(a) even) runs the pair move, so the
// first spin is read coalesced and only the partner is a random gather.  M_L
// is the moment along eC at the start of the sweep (one value for both
// colours, as in the paper).  OBS (black pass) adds the two black sites and
// their exchange with their final red neighbours; since pi is a bijection
// every black site is covered once.  Results go to row part_base + block.
template <typename R, int C, bool OBS>
__global__ __launch_bounds__(kThreads) void pair_kernel(const KArgs<R> a, Vec4<R>* aos, const Vec4<R>* nbs,
                                                        const V3<R> ec, const uint32_t half, const uint32_t mask,
                                                        const R scale, const uint32_t part_base)
{
    __shared__ double scratch[5 * kNumPart];
    Vec4<R>* own = aos + (size_t)C * a.Nc;
    const uint32_t ia = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t sweep = (uint32_t)a.st->sweep;
    const R c1 = a.c1tab[a.st->theta];
    const Model<R> m = a.m;
    const double* M = a.st->M;
    const double ML = M[0] * (double)ec.x + M[1] * (double)ec.y + M[2] * (double)ec.z;
    const R invML = (R)(1.0 / fabs(ML));
    const Rand4 key = philox(sweep, 0u, 5u + (uint32_t)C, a.inst, a.key0, a.key1);

    uint32_t nacc = 0;
    Acc acc;
    const uint32_t pos = ia < a.Nc ? unshuffle_index(ia, a.Nc, half, mask, key) : 1u;
    if ((pos & 1u) == 0u) {
        const uint32_t k = pos >> 1;
        const uint32_t ja = shuffle_index(pos + 1u, a.Nc, half, mask, key);
        const V3<R> si = ld4<R>(own, ia), nbi = ld4<R>(nbs, ia);
        const V3<R> sj = ld4<R>(own, ja), nbj = ld4<R>(nbs, ja);
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
        const R xr = ((pi_new + pj_new) - pi_old - pj_old) * invML;
        ok = ok && (R(1) + xr > R(0)) && (ML != 0.0);
        const V3<R> hi{m.J * nbi.x + m.h.x, m.J * nbi.y + m.h.y, m.J * nbi.z + m.h.z};
        const V3<R> hj{m.J * nbj.x + m.h.x, m.J * nbj.y + m.h.y, m.J * nbj.z + m.h.z};
        const R dE = delta_e(m, si, ti, hi) + delta_e(m, sj, tj, hj);
        const R ratio = (R(1) + xr) * (R(1) + xr) * fabs(pj_old / pj_new);
        ok = ok && (Prim<R>::u01(rn.r2) < ratio * Prim<R>::boltzmann(dE, scale));
        const V3<R> fi = ok ? ti : si;
        const V3<R> fj = ok ? tj : sj;
        if (ok) {
            st4<R>(own, ia, ti);
            st4<R>(own, ja, tj);
            nacc = 2;
        }
        if (OBS) {
            acc.ex += (double)(-m.J * dot(fi, nbi)) + (double)(-m.J * dot(fj, nbj));
            add_site<R, true>(acc, m, fi);
            add_site<R, true>(acc, m, fj);
        }
    }
    KArgs<R> ra = a;
    ra.part = a.part + (size_t)part_base * kNumPart;
    block_end<R, OBS>(ra, C, blockIdx.x, nacc, acc, scratch);
}

// ---------------------------------------------------------------------------
// Measurement of the current spins: one thread per colour index k covers the
// black site k (with its six red neighbours: every bond once) and the red
// site k; the last work-group stores M, the energies and the torque.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void measure_kernel(const KArgs<R> a)
{
    __shared__ double scratch[8 * kNumPart];
    const Arrays<R> g(a);
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    Acc acc;
    if (k < a.Nc) {
        V3<R> nb, red;
        uint32_t site;
        gather_neighbours<R, 1>(a, g, k, nb, red, site);
        const V3<R> blk = g.get(1, k * (uint32_t)sizeof(R), 0);
        acc.ex += (double)(-a.m.J * dot(blk, nb));
        add_site<R, true>(acc, a.m, blk);
        add_site<R, true>(acc, a.m, red);
    }
    block_end<R, true>(a, 1, blockIdx.x, 0u, acc, scratch);
}

// Mean spin of every z plane (both colours), for wall profiles: work-group z
// sums the 2P spins of plane z in a fixed order and writes the mean to
// out[3z .. 3z+2].
template <typename R>
__global__ __launch_bounds__(kThreads) void plane_mean_kernel(const KArgs<R> a, double* out)
{
    __shared__ double scratch[5 * 3];
    const Arrays<R> g(a);
    const uint32_t z = blockIdx.x;
    const uint32_t off = a.P * (uint32_t)sizeof(R) * z;
    double v[3] = {0.0, 0.0, 0.0};
    for (uint32_t q = threadIdx.x; q < a.P; q += kThreads) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const V3<R> s = g.get(c, q * (uint32_t)sizeof(R), off);
            v[0] += (double)s.x;
            v[1] += (double)s.y;
            v[2] += (double)s.z;
        }
    }
    block_sum<3>(v, scratch);
    if (threadIdx.x < 3) out[3 * (size_t)z + threadIdx.x] = scratch[threadIdx.x] / (2.0 * (double)a.P);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

int64_t max_blocks_for(int32_t nx, int32_t ny, int32_t nz)
{
    const uint64_t P = (uint64_t)(nx / 2) * (uint64_t)ny;
    const uint64_t Nc = P * (uint64_t)nz;
    const int64_t pass = (int64_t)cdiv(P, kThreads) * (int64_t)nz;
    const int64_t gather = 2 * (int64_t)cdiv(Nc, kThreads);   // neighbour-sum + pair partials
    return pass > gather ? pass : gather;
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

template <typename R, int C, bool OBS, int SPT, int HALO>
static void pass_go(const KArgs<R>& a, const DevLattice& d, int zc, double T, hipStream_t s)
{
    const uint32_t nqb = cdiv((uint64_t)d.P, (uint64_t)kThreads * SPT);
    const uint32_t nzb = cdiv((uint64_t)d.nz, (uint64_t)zc);
    const uint32_t nblk = nqb * nzb;
    pass_kernel<R, C, OBS, SPT, HALO><<<nblk, kThreads, pass_lds_bytes(d.precision, d.hx, SPT), s>>>(
        a, (uint32_t)zc, nqb, nblk, Prim<R>::scale_for(T));
}

template <typename R, int SPT, int HALO>
static void pass_dispatch_c(const KArgs<R>& a, const DevLattice& d, int colour, bool obs, int zc, double T,
                            hipStream_t s)
{
    if (colour == 0) pass_go<R, 0, false, SPT, HALO>(a, d, zc, T, s);
    else if (obs) pass_go<R, 1, true, SPT, HALO>(a, d, zc, T, s);
    else pass_go<R, 1, false, SPT, HALO>(a, d, zc, T, s);
}

static int halo_slots(int hx)
{
    const int halo = (2 * hx + kThreads - 1) / kThreads;
    return halo <= 1 ? 1 : (halo == 2 ? 2 : 4);
}

template <typename R, int SPT>
static void pass_dispatch_h(const KArgs<R>& a, const DevLattice& d, int colour, bool obs, int zc, double T,
                            hipStream_t s)
{
    const int halo = halo_slots(d.hx);
    if (halo == 1) pass_dispatch_c<R, SPT, 1>(a, d, colour, obs, zc, T, s);
    else if (halo == 2) pass_dispatch_c<R, SPT, 2>(a, d, colour, obs, zc, T, s);
    else pass_dispatch_c<R, SPT, 4>(a, d, colour, obs, zc, T, s);
}

template <typename R>
static void pass_dispatch(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s)
{
    const auto a = make_args<R>(d);
    if (spt == 1) pass_dispatch_h<R, 1>(a, d, colour, obs, zc, T, s);
    else if (spt == 2) pass_dispatch_h<R, 2>(a, d, colour, obs, zc, T, s);
    else pass_dispatch_h<R, 4>(a, d, colour, obs, zc, T, s);
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
static void constrained_go(const DevLattice& d, int step, const double eC[3], double T, hipStream_t s,
                           int64_t* blocks)
{
    const auto a = make_args<R>(d);
    Vec4<R>* aos = static_cast<Vec4<R>*>(d.aos);
    Vec4<R>* nbs = static_cast<Vec4<R>*>(d.nbs);
    const uint32_t n = (uint32_t)d.Nc;
    const uint32_t grid = cdiv(n, kThreads);
    *blocks = grid;
    if (step == kAosIn) {
        aos_copy_kernel<R, true><<<dim3(grid, 2), kThreads, 0, s>>>(a, aos);
        return;
    }
    if (step == kAosOut) {
        aos_copy_kernel<R, false><<<dim3(grid, 2), kThreads, 0, s>>>(a, aos);
        return;
    }
    if (step == kNbRed) {
        nbsum_kernel<R, 0, false><<<grid, kThreads, 0, s>>>(a, aos, nbs);
        return;
    }
    if (step == kNbBlack) {
        nbsum_kernel<R, 1, true><<<grid, kThreads, 0, s>>>(a, aos, nbs);
        return;
    }
    uint32_t bits = 2;
    while (bits < 32 && (1ull << bits) < n) bits += 2;
    const uint32_t half = bits / 2;
    const uint32_t mask = half >= 32 ? 0xFFFFFFFFu : ((1u << half) - 1u);
    const V3<R> ec{(R)eC[0], (R)eC[1], (R)eC[2]};
    const R scale = Prim<R>::scale_for(T);
    if (step == kPairRed) pair_kernel<R, 0, false><<<grid, kThreads, 0, s>>>(a, aos, nbs, ec, half, mask, scale, 0u);
    else pair_kernel<R, 1, true><<<grid, kThreads, 0, s>>>(a, aos, nbs, ec, half, mask, scale, grid);
}

hipError_t launch_constrained(const DevLattice& d, int step, const double eC[3], double T, hipStream_t s,
                              int64_t* blocks)
{
    if (d.precision == 32) constrained_go<float>(d, step, eC, T, s, blocks);
    else constrained_go<double>(d, step, eC, T, s, blocks);
    return hipGetLastError();
}

hipError_t launch_plane_means(const DevLattice& d, double* out, hipStream_t s)
{
    if (d.precision == 32) plane_mean_kernel<float><<<d.nz, kThreads, 0, s>>>(make_args<float>(d), out);
    else plane_mean_kernel<double><<<d.nz, kThreads, 0, s>>>(make_args<double>(d), out);
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
                           int fin, double T, hipStream_t s)
{
    finalize_kernel<<<1, kThreads, 0, s>>>(d.st, d.part, d.cnt, (uint32_t)d.max_blocks, (uint32_t)red_blocks,
                                            (uint32_t)black_blocks, (uint32_t)part_blocks, fin, T, (double)d.N);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
size_t batch_entry_bytes(int precision)
{
    return precision == 32 ? sizeof(BatchEntry<float>) : sizeof(BatchEntry<double>);
}

int batch_group(const DevLattice& d, int spt) { return (spt == 1 ? 0 : spt == 2 ? 1 : 2) * 3 +
                                                      (halo_slots(d.hx) == 1 ? 0 : halo_slots(d.hx) == 2 ? 1 : 2); }

void batch_store_scale(int precision, double T, void* dst, size_t i)
{
    if (precision == 32) static_cast<float*>(dst)[i] = Prim<float>::scale_for(T);
    else static_cast<double*>(dst)[i] = Prim<double>::scale_for(T);
}

template <typename R>
static void fill_entry(void* dst, const DevLattice& d, int spt, int zc)
{
    BatchEntry<R> E;
    memset(&E, 0, sizeof(E));
    E.a = make_args<R>(d);
    E.zc = (uint32_t)zc;
    E.nqb = cdiv((uint64_t)d.P, (uint64_t)kThreads * spt);
    E.nblk = (uint32_t)pass_blocks(d, spt, zc);
    E.N = (double)d.N;
    memcpy(dst, &E, sizeof(E));
}

void batch_fill_entry(void* dst, const DevLattice& d, int spt, int zc)
{
    if (d.precision == 32) fill_entry<float>(dst, d, spt, zc);
    else fill_entry<double>(dst, d, spt, zc);
}

template <typename R, int SPT, int HALO>
static void pass_batch_go(const BatchLaunch& b, int colour, bool obs, hipStream_t s)
{
    const auto* tab = static_cast<const BatchEntry<R>*>(b.tab);
    const auto* sc = static_cast<const R*>(b.scale);
    if (colour == 0)
        pass_batch_kernel<R, 0, false, SPT, HALO><<<b.nblk, kThreads, b.lds, s>>>(tab, b.start, b.ent, b.n, b.nblk, sc);
    else if (obs)
        pass_batch_kernel<R, 1, true, SPT, HALO><<<b.nblk, kThreads, b.lds, s>>>(tab, b.start, b.ent, b.n, b.nblk, sc);
    else
        pass_batch_kernel<R, 1, false, SPT, HALO><<<b.nblk, kThreads, b.lds, s>>>(tab, b.start, b.ent, b.n, b.nblk, sc);
}

template <typename R>
static void pass_batch_dispatch(const BatchLaunch& b, int colour, bool obs, hipStream_t s)
{
    switch (b.group) {
    case 0: pass_batch_go<R, 1, 1>(b, colour, obs, s); break;
    case 1: pass_batch_go<R, 1, 2>(b, colour, obs, s); break;
    case 2: pass_batch_go<R, 1, 4>(b, colour, obs, s); break;
    case 3: pass_batch_go<R, 2, 1>(b, colour, obs, s); break;
    case 4: pass_batch_go<R, 2, 2>(b, colour, obs, s); break;
    case 5: pass_batch_go<R, 2, 4>(b, colour, obs, s); break;
    case 6: pass_batch_go<R, 4, 1>(b, colour, obs, s); break;
    case 7: pass_batch_go<R, 4, 2>(b, colour, obs, s); break;
    default: pass_batch_go<R, 4, 4>(b, colour, obs, s); break;
    }
}

hipError_t launch_pass_batch(int precision, const BatchLaunch& b, int colour, bool obs, hipStream_t s)
{
    if (precision == 32) pass_batch_dispatch<float>(b, colour, obs, s);
    else pass_batch_dispatch<double>(b, colour, obs, s);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(int precision, const void* tab, uint32_t count, const double* T,
                                 const int32_t* fin, hipStream_t s)
{
    if (precision == 32)
        finalize_batch_kernel<float><<<count, kThreads, 0, s>>>(static_cast<const BatchEntry<float>*>(tab), T, fin);
    else
        finalize_batch_kernel<double><<<count, kThreads, 0, s>>>(static_cast<const BatchEntry<double>*>(tab), T,
                                                                 fin);
    return hipGetLastError();
}

hipError_t launch_reset_batch(int precision, const void* tab, uint32_t count, hipStream_t s)
{
    if (precision == 32) reset_batch_kernel<float><<<count, 64, 0, s>>>(static_cast<const BatchEntry<float>*>(tab));
    else reset_batch_kernel<double><<<count, 64, 0, s>>>(static_cast<const BatchEntry<double>*>(tab));
    return hipGetLastError();
}

}  // namespace hmc
