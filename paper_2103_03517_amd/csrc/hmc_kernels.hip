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
#include "hmc_pass.hpp"

namespace hmc {

size_t pass_lds_bytes(int precision, int hx, int spt)
{
    const size_t W = (size_t)kThreads * spt + 2 * (size_t)hx;
    const size_t e = precision == 32 ? LdsPlane<float>::bytes_per_entry : LdsPlane<double>::bytes_per_entry;
    const size_t b = 2 * W * e;
    return b < 1024 ? 1024 : b;
}

__global__ __launch_bounds__(kThreads) void finalize_kernel(DevState* st, const double* part, const uint32_t* cnt,
                                                            uint32_t cnt_stride, uint32_t nred, uint32_t nblack,
                                                            uint32_t npart, int fin, double T, double N)
{
    __shared__ double scratch[5 * (kNumPart + 1)];
    finalize_body(st, part, cnt, cnt_stride, nred, nblack, npart, fin, T, N, scratch);
}

// ---------------------------------------------------------------------------
// Initial spins: along a direction, or uniform on the sphere from Philox
// tag 4 (z = 2 u0 - 1, azimuth 2 pi u1).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void init_kernel(const KArgs<R> a, int mode, R d0, R d1, R d2,
                                                       double width)
{
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= a.Nc) return;
    V3<R> s{d0, d1, d2};
    if (mode == 2) {
        // one wall across z: the T = 0 profile (sech u, 0, -tanh u)
        const uint32_t z = k / a.P;
        const double u = M_PI * ((double)z - (0.5 * (double)a.nz - 0.5)) / width;
        s = V3<R>{(R)(1.0 / cosh(u)), R(0), (R)(-tanh(u))};
    }
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
    if (a.zbound) {
        if (z == 0) vzm = across_z(vzm, a.zbound);
        if (z == nz - 1) vzp = across_z(vzp, a.zbound);
    }
    V3<R> xm = p ? same : xd;
    V3<R> xp = p ? xd : same;
    V3<R> v2 = vym, v3 = vyp;
    if (a.mask[C]) {
        const uint32_t mb = a.mask[C][k];
        const V3<R> zero{R(0), R(0), R(0)};
        if (!(mb & 1u)) xm = zero;
        if (!(mb & 2u)) xp = zero;
        if (!(mb & 4u)) v2 = zero;
        if (!(mb & 8u)) v3 = zero;
        if (!(mb & 16u)) vzm = zero;
        if (!(mb & 32u)) vzp = zero;
    }
    nb = V3<R>{((((xm.x + xp.x) + v2.x) + v3.x) + vzm.x) + vzp.x,
               ((((xm.y + xp.y) + v2.y) + v3.y) + vzm.y) + vzp.y,
               ((((xm.z + xp.z) + v2.z) + v3.z) + vzm.z) + vzp.z};
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

// Neighbour sums of colour C (from the AoS copy of the other colour).
template <typename R, int C>
__global__ __launch_bounds__(kThreads) void nbsum_kernel(const KArgs<R> a, const Vec4<R>* aos, Vec4<R>* nbs)
{
    const Vec4<R>* other = aos + (size_t)(1 - C) * a.Nc;
    for (uint32_t k = blockIdx.x * kThreads + threadIdx.x; k < a.Nc; k += gridDim.x * kThreads) {
        uint32_t id[6];
        bool wm, wp;
        neighbour_indices<C>(k, a.hx, a.ny, a.nz, a.P, id, wm, wp);
        V3<R> v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = ld4<R>(other, id[i]);
        if (a.zbound) {
            if (wm) v[4] = across_z(v[4], a.zbound);
            if (wp) v[5] = across_z(v[5], a.zbound);
        }
        if (a.mask[C]) {
            const uint32_t mb = a.mask[C][k];
#pragma unroll
            for (int i = 0; i < 6; ++i)
                if (!((mb >> i) & 1u)) v[i] = V3<R>{R(0), R(0), R(0)};
        }
        const V3<R> nb{((((v[0].x + v[1].x) + v[2].x) + v[3].x) + v[4].x) + v[5].x,
                       ((((v[0].y + v[1].y) + v[2].y) + v[3].y) + v[4].y) + v[5].y,
                       ((((v[0].z + v[1].z) + v[2].z) + v[3].z) + v[4].z) + v[5].z};
        st4<R>(nbs, k, nb);
    }
}

// Pair pass of colour C.  The shuffled order pi of the colour indices is a
// keyed bijection evaluated inline (nothing is stored); pair k is
// (pi(2k), pi(2k+1)).  One thread per colour index a: the thread whose a is
// the first spin of its pair (pi^-1(a) even) runs the pair move, so the
// first spin is read coalesced and only the partner is a random gather.  M_L
// is the moment along eC at the start of the sweep (one value for both
// colours, as in the paper).  OBS adds the one-site terms (moment,
// anisotropy, Zeeman, torque) of both final spins of every pair, and in the
// black pass also their exchange with their final red neighbours; since pi
// is a bijection every site is covered once, and every bond once through its
// black end.  Results go to row part_base + block (red pass: rows 0 .., black
// pass: rows grid ..).
template <typename R, int C, bool OBS>
__global__ __launch_bounds__(kThreads) void pair_kernel(const KArgs<R> a, Vec4<R>* aos, const Vec4<R>* nbs,
                                                        const V3<R> ec, const uint32_t half, const uint32_t mask,
                                                        const R scale, const uint32_t part_base)
{
    __shared__ double scratch[5 * kNumPart];
    Vec4<R>* own = aos + (size_t)C * a.Nc;
    const uint32_t sweep = (uint32_t)a.st->sweep;
    const R c1 = a.c1tab[a.st->theta];
    const Model<R> m = a.m;
    const double* M = a.st->M;
    const double ML = M[0] * (double)ec.x + M[1] * (double)ec.y + M[2] * (double)ec.z;
    const R invML = (R)(1.0 / fabs(ML));
    const Rand4 key = philox(sweep, 0u, 5u + (uint32_t)C, a.inst, a.key0, a.key1);

    uint32_t nacc = 0;
    Acc acc;
    for (uint32_t ia = blockIdx.x * kThreads + threadIdx.x; ia < a.Nc; ia += gridDim.x * kThreads) {
        const uint32_t pos = unshuffle_index(ia, a.Nc, half, mask, key);
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
                nacc += 2;
            }
            if (OBS) {
                if (C == 1) acc.ex += (double)(-m.J * dot(fi, nbi)) + (double)(-m.J * dot(fj, nbj));
                add_site<R, true>(acc, m, fi);
                add_site<R, true>(acc, m, fj);
            }
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
                                                     (float)d.init_dir[2], d.init_width);
    } else {
        auto a = make_args<double>(d);
        init_kernel<double><<<grid, kThreads, 0, s>>>(a, d.init_mode, d.init_dir[0], d.init_dir[1], d.init_dir[2],
                                                      d.init_width);
    }
    return hipGetLastError();
}

hipError_t launch_pass(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s,
                       int64_t* blocks)
{
    *blocks = pass_blocks(d, spt, zc);
    if (d.mask) return launch_pass_masked(d, colour, obs, spt, zc, T, s);
    if (pass_deep(d)) return launch_pass_deep(d, colour, obs, spt, zc, T, s);
    return PassLaunch<false, false>::run(d, colour, obs, spt, zc, T, s);
}

template <typename R>
static void constrained_go(const DevLattice& d, int step, const double eC[3], double T, hipStream_t s,
                           int64_t* blocks)
{
    const auto a = make_args<R>(d);
    Vec4<R>* aos = static_cast<Vec4<R>*>(d.aos);
    Vec4<R>* nbs = static_cast<Vec4<R>*>(d.nbs);
    const uint32_t n = (uint32_t)d.Nc;
    const uint32_t full = cdiv(n, kThreads);
    const uint32_t grid = full < (uint32_t)kGatherBlocks ? full : (uint32_t)kGatherBlocks;
    *blocks = grid;
    if (step == kAosIn) {
        aos_copy_kernel<R, true><<<dim3(full, 2), kThreads, 0, s>>>(a, aos);
        return;
    }
    if (step == kAosOut) {
        aos_copy_kernel<R, false><<<dim3(full, 2), kThreads, 0, s>>>(a, aos);
        return;
    }
    if (step == kNbRed) {
        nbsum_kernel<R, 0><<<full, kThreads, 0, s>>>(a, aos, nbs);
        return;
    }
    if (step == kNbBlack) {
        nbsum_kernel<R, 1><<<full, kThreads, 0, s>>>(a, aos, nbs);
        return;
    }
    uint32_t bits = 2;
    while (bits < 32 && (1ull << bits) < n) bits += 2;
    const uint32_t half = bits / 2;
    const uint32_t mask = half >= 32 ? 0xFFFFFFFFu : ((1u << half) - 1u);
    const V3<R> ec{(R)eC[0], (R)eC[1], (R)eC[2]};
    const R scale = Prim<R>::scale_for(T);
    if (step == kPairRed) pair_kernel<R, 0, true><<<grid, kThreads, 0, s>>>(a, aos, nbs, ec, half, mask, scale, 0u);
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

}  // namespace hmc
