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

// The per-sweep finalize, one work-group of 1024 threads: all of them sum
// the counts, the first 256 fold the records (or the group sums left by
// fold_groups_kernel in l2).  A lone work-group has no occupancy to gain, so
// the register budget of four waves per SIMD goes to loads in flight.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
void finalize_kernel(DevState* st, const double* part, uint32_t stride, const uint32_t* cnt, uint32_t nred,
                     uint32_t nblack, uint32_t npart, const double* l2, int fin, double T, double N)
{
    __shared__ double scratch[kFinScratch];
    __shared__ DevState sst;
    finalize_body<1024>(st, part, stride, cnt, nred, nblack, npart, l2, fin, T, N, scratch, &sst);
}

// Work-group g: the sum S_g of record group g (the order of finalize_body),
// its first nrows components stored at l2[g * kNumPart ..].
__global__ __launch_bounds__(kGroupThreads) void fold_groups_kernel(const double* part, uint32_t stride,
                                                                    uint32_t npart, uint32_t nrows, double* l2)
{
    __shared__ double scratch[5 * kNumPart];
    if (nrows == (uint32_t)kTorqueRows)
        group_sums<kGroupThreads, kTorqueRows>(part, stride, npart, blockIdx.x, blockIdx.x + 1u, scratch,
                                               scratch + 4 * kNumPart);
    else
        group_sums<kGroupThreads, kObsRows>(part, stride, npart, blockIdx.x, blockIdx.x + 1u, scratch,
                                            scratch + 4 * kNumPart);
    if (threadIdx.x < nrows) l2[(size_t)blockIdx.x * kNumPart + threadIdx.x] = scratch[4 * kNumPart + threadIdx.x];
}

// ---------------------------------------------------------------------------
// Set-up of a lattice's workspace: the chain state (zeroed, cone angle
// theta0) and the cone table 1 - cos(theta), both precisions, from values
// passed by argument (so nothing is copied from host memory).
// ---------------------------------------------------------------------------
struct C1Table {
    double d[181];
    float f[181];
};

__global__ __launch_bounds__(kThreads) void setup_kernel(DevState* st, int theta0, const C1Table tab, double* c1d,
                                                         float* c1f)
{
    const uint32_t t = threadIdx.x;
    if (t < 181) {
        c1d[t] = tab.d[t];
        c1f[t] = tab.f[t];
    }
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    for (uint32_t i = t; i < sizeof(DevState) / 4; i += kThreads) w[i] = 0u;
    __syncthreads();
    if (t == 0) st->theta = theta0;
}

hipError_t launch_setup(const DevLattice& d, const double* c1d_host, int theta0, void* c1_dev, hipStream_t s)
{
    C1Table tab;
    for (int i = 0; i < 181; ++i) {
        tab.d[i] = c1d_host[i];
        tab.f[i] = (float)c1d_host[i];
    }
    double* c1d = static_cast<double*>(c1_dev);
    float* c1f = reinterpret_cast<float*>(c1d + 181);
    setup_kernel<<<1, kThreads, 0, s>>>(d.st, theta0, tab, c1d, c1f);
    return hipGetLastError();
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
// the spins (one 4-vector per site, both colours), made on entry and copied
// back on exit.  Before each colour's pair pass a stencil kernel writes, for
// every site of that colour in site order, a record of its spin and the sum
// of its six neighbours (32 bytes FP32, 64 FP64; the other colour does not
// change during the pass, so the sums are exact).  A pair then needs its two
// records -- the first read in site order, the partner's at a random
// address, the pairing being a random permutation: one cache line per pair
// instead of seven sites -- and writes its new spins into the AoS copy.
// ---------------------------------------------------------------------------
template <typename R> struct Vec4T;
template <> struct Vec4T<float> { using type = float4; };
template <> struct Vec4T<double> { using type = double4; };
template <typename R> using Vec4 = typename Vec4T<R>::type;

template <typename R>
struct Rec {
    Vec4<R> s;    // spin (w unused)
    Vec4<R> nb;   // sum of the six neighbours (other colour)
};

template <typename R>
__device__ __forceinline__ V3<R> v3(const Vec4<R>& q)
{
    return V3<R>{q.x, q.y, q.z};
}

template <typename R>
__device__ __forceinline__ Vec4<R> v4(const V3<R>& v)
{
    Vec4<R> q;
    q.x = v.x;
    q.y = v.y;
    q.z = v.z;
    q.w = R(0);
    return q;
}

#ifndef HMC_PAIR_BLOCKS
#define HMC_PAIR_BLOCKS 512      // most work-groups of the pair pass
#endif
#ifndef HMC_PAIR_TILE_BLOCKS
#define HMC_PAIR_TILE_BLOCKS 2   // blocks of 256 colour indices per pair-pass tile
#endif
constexpr uint32_t kPairTile = HMC_PAIR_TILE_BLOCKS * kThreads;

// the smallest power of two >= n
constexpr uint32_t ring_size(uint32_t n)
{
    uint32_t r = 1;
    while (r < n) r *= 2;
    return r;
}

#ifndef HMC_NB_BLOCKS
#define HMC_NB_BLOCKS 2048       // most work-groups of the record stencil
#endif

// SoA -> AoS (to_aos) or AoS -> SoA, both colours; aos[c * Nc + k].
template <typename R, bool TO_AOS>
__global__ __launch_bounds__(kThreads) void aos_copy_kernel(const KArgs<R> a, Vec4<R>* aos)
{
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= a.Nc) return;
    Vec4<R>* q = aos + (size_t)c * a.Nc + k;
    if (TO_AOS) {
        *q = v4<R>(V3<R>{a.s[c][0][k], a.s[c][1][k], a.s[c][2][k]});
    } else {
        const Vec4<R> v = *q;
        a.s[c][0][k] = v.x;
        a.s[c][1][k] = v.y;
        a.s[c][2][k] = v.z;
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

// Records of colour C over work-groups b, b + count, ... of the launch:
// site k's spin and the sum of its neighbours (the other colour's AoS spins).
template <typename R, int C>
__device__ __forceinline__ void records_range(const KArgs<R>& a, const Vec4<R>* aos, Rec<R>* rec, uint32_t b,
                                              uint32_t count)
{
    const Vec4<R>* other = aos + (size_t)(1 - C) * a.Nc;
    const Vec4<R>* own = aos + (size_t)C * a.Nc;
    for (uint32_t k = b * kThreads + threadIdx.x; k < a.Nc; k += count * kThreads) {
        uint32_t id[6];
        bool wm, wp;
        neighbour_indices<C>(k, a.hx, a.ny, a.nz, a.P, id, wm, wp);
        V3<R> v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = v3<R>(other[id[i]]);
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
        Rec<R> r;
        r.s = own[k];
        r.nb = v4<R>(nb);
        rec[k] = r;
    }
}

template <typename R, int C>
__global__ __launch_bounds__(kThreads) void records_kernel(const KArgs<R> a, const Vec4<R>* aos, Rec<R>* rec)
{
    records_range<R, C>(a, aos, rec, blockIdx.x, gridDim.x);
}

// The end of one constrained sweep and the start of the next in one launch:
// work-group 0 runs the per-sweep finalize (the records of the two pair
// passes, nrec rows each), the others write the colour-0 records of the next
// sweep, which need only the spins.  The finalize and the records touch
// disjoint memory, so the finalize runs in the shadow of the stencil.
template <typename R>
__global__ __launch_bounds__(kThreads) void finalize_records_kernel(const KArgs<R> a, const Vec4<R>* aos, Rec<R>* rec,
                                                                    uint32_t nrec, int fin, double T, double N)
{
    // the pair passes write at most 2 x HMC_PAIR_BLOCKS records: one group
    static_assert(2 * HMC_PAIR_BLOCKS <= kGroupRecords, "the fused finalize folds one group of records");
    __shared__ double scratch[kFinScratch];
    __shared__ DevState sst;
    if (blockIdx.x == 0) {
        finalize_body<kThreads>(a.st, a.part, a.cnt_stride, a.cnt, nrec, nrec, 2 * nrec, nullptr, fin, T, N, scratch,
                                &sst);
        return;
    }
    records_range<R, 0>(a, aos, rec, blockIdx.x - 1, gridDim.x - 1);
}

// Feistel domain of the shuffle of N_c indices: 2*half bits, the smallest
// even width covering N_c.
struct Shuffle {
    uint32_t half, mask;
};

static inline Shuffle shuffle_for(uint32_t n)
{
    uint32_t bits = 2;
    while (bits < 32 && (1ull << bits) < n) bits += 2;
    Shuffle f;
    f.half = bits / 2;
    f.mask = f.half >= 32 ? 0xFFFFFFFFu : ((1u << f.half) - 1u);
    return f;
}

// Per-sweep constants of a pair pass.
template <typename R>
struct PairCtx {
    Model<R> m;
    V3<R> ec;
    R c1, scale, invML;
    double ML;
    uint32_t sweep, inst, key0, key1;
};

// The pair move of Table A2 on pair k = (i, j) of colour C, with the records
// ri, rj of its two spins: cone move of S_i, compensation of the transverse
// change by S_j (perpendicular to eC; the parallel part from the length),
// M_L ratio and Jacobian, Metropolis test with exp(-(dE_i + dE_j)/T); on
// acceptance both new spins go to the AoS copy.  OBS adds the one-site terms
// of both final spins (and in the black pass their exchange with their final
// red neighbours).
template <typename R, int C, bool OBS, typename A>
__device__ __forceinline__ void pair_move(const PairCtx<R>& x, Vec4<R>* own, uint32_t k, uint32_t ia, uint32_t ja,
                                          const Rec<R>& ri, const Rec<R>& rj, uint32_t& nacc, A& acc)
{
    const Model<R>& m = x.m;
    const V3<R>& ec = x.ec;
    const V3<R> si = v3<R>(ri.s), nbi = v3<R>(ri.nb);
    const V3<R> sj = v3<R>(rj.s), nbj = v3<R>(rj.nb);
    const Rand4 rn = philox(x.sweep, k, 2u + (uint32_t)C, x.inst, x.key0, x.key1);
    const V3<R> ti = cone_move(si, Prim<R>::u01(rn.r0), Prim<R>::u01(rn.r1), x.c1);

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
    const R xr = ((pi_new + pj_new) - pi_old - pj_old) * x.invML;
    ok = ok && (R(1) + xr > R(0)) && (x.ML != 0.0);
    const V3<R> hi{m.J * nbi.x + m.h.x, m.J * nbi.y + m.h.y, m.J * nbi.z + m.h.z};
    const V3<R> hj{m.J * nbj.x + m.h.x, m.J * nbj.y + m.h.y, m.J * nbj.z + m.h.z};
    const R dE = delta_e(m, si, ti, hi) + delta_e(m, sj, tj, hj);
    const R ratio = (R(1) + xr) * (R(1) + xr) * fabs(pj_old / pj_new);
    ok = ok && (Prim<R>::u01(rn.r2) < ratio * Prim<R>::boltzmann(dE, x.scale));
    const V3<R> fi = ok ? ti : si;
    const V3<R> fj = ok ? tj : sj;
    if (ok) {
        own[ia] = v4<R>(ti);
        own[ja] = v4<R>(tj);
        nacc += 2;
    }
    if (OBS) {
        if (C == 1) acc.ex += (-m.J * dot(fi, nbi)) + (-m.J * dot(fj, nbj));
        add_site<R, true>(acc, m, fi);
        add_site<R, true>(acc, m, fj);
    }
}

// Pair pass of colour C.  The shuffled order pi of the colour indices is a
// keyed bijection evaluated inline (nothing is stored); pair k is
// (pi(2k), pi(2k+1)) (N_c is even: nx and ny are).  A work-group scans tiles
// of kPairTile consecutive colour indices a (blocks of 256); a is the first
// spin of pair pi^-1(a)/2 when pi^-1(a) is even, and such pairs are queued in
// LDS in scan order (blocks in order, wave ballots, waves in order), so the
// queue never depends on scheduling; a tile takes one ballot round, two
// barriers, for all of its blocks.
// The queue is a ring in LDS drained in rounds of 256 pairs, one per thread,
// and what is left of it stays for the next tile: every lane runs a pair
// move, and the first record of each pair is read near site order (only the
// partner's is a random gather).  M_L is the moment along eC at the
// start of the sweep (one value for both colours, as in the paper).  OBS adds
// the one-site terms of both final spins of every pair; since pi is a
// bijection every site is covered once, and in the black pass every bond once
// through its black end.  Results go to row part_base + block (red pass: rows
// 0 .., black pass: rows grid ..).
template <typename R, int C, bool OBS>
__global__ __launch_bounds__(kThreads) void pair_kernel(const KArgs<R> a, Vec4<R>* aos, const Rec<R>* rec,
                                                        const V3<R> ec, const Shuffle f, const R scale,
                                                        const uint32_t part_base)
{
    constexpr uint32_t kU = kPairTile / kThreads;            // indices per thread and tile
    constexpr uint32_t kTrip = kPairTile;                    // indices scanned per tile
    constexpr uint32_t kRing = ring_size(kThreads - 1 + kTrip);  // queue ring: 255 left + kTrip new
    static_assert((kRing & (kRing - 1)) == 0 && kRing >= kThreads - 1 + kTrip, "queue ring too small");
    constexpr int kWaves = kThreads / 64;
    __shared__ double scratch[5 * kNumPart];
    __shared__ uint32_t qa[kRing], qj[kRing], qk[kRing];
    __shared__ uint32_t wcnt[kU][kWaves];
    Vec4<R>* own = aos + (size_t)C * a.Nc;
    PairCtx<R> x;
    x.m = a.m;
    x.ec = ec;
    x.sweep = (uint32_t)a.st->sweep;
    x.c1 = a.c1tab[a.st->theta];
    x.scale = scale;
    const double* M = a.st->M;
    x.ML = M[0] * (double)ec.x + M[1] * (double)ec.y + M[2] * (double)ec.z;
    x.invML = (R)(1.0 / fabs(x.ML));
    x.inst = a.inst;
    x.key0 = a.key0;
    x.key1 = a.key1;
    const Rand4 key = philox(x.sweep, 0u, 5u + (uint32_t)C, a.inst, a.key0, a.key1);

    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const uint32_t tiles = (a.Nc + kTrip - 1u) / kTrip;
    uint32_t nacc = 0;
    Acc acc;
    Part<R> part;                                            // FP32 spins: the thread's sums, then FP64
    auto& pa = site_acc<R>(acc, part);
    // pairs queued and pairs taken so far, the same in every thread; the
    // queue holds entries head .. tail - 1 at their positions modulo kRing
    uint32_t head = 0, tail = 0;
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        uint32_t ia[kU], ja[kU], k[kU];
        bool first[kU];
        uint64_t ball[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            ia[u] = tile * kTrip + u * kThreads + t;
            first[u] = false;
            ja[u] = 0;
            k[u] = 0;
            if (ia[u] < a.Nc) {
                const uint32_t pos = unshuffle_index(ia[u], a.Nc, f.half, f.mask, key);
                first[u] = (pos & 1u) == 0u;
                if (first[u]) {
                    ja[u] = shuffle_index(pos + 1u, a.Nc, f.half, f.mask, key);
                    k[u] = pos >> 1;
                }
            }
            ball[u] = __ballot(first[u]);
            if (lane == 0) wcnt[u][wave] = (uint32_t)__popcll(ball[u]);
        }
        // every wave has left the previous tile's queue reads: the slots past
        // tail are free
        __syncthreads();
        // appended in scan order: index block u = 0 (waves in order), then u = 1
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            uint32_t off = tail, total = tail;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                off += (uint32_t)w < wave ? wcnt[u][w] : 0u;
                total += wcnt[u][w];
            }
            if (first[u]) {
                const uint32_t e = (off + (uint32_t)__popcll(ball[u] & below)) & (kRing - 1u);
                qa[e] = ia[u];
                qj[e] = ja[u];
                qk[e] = k[u];
            }
            tail = total;
        }
        __syncthreads();
        for (; tail - head >= kThreads; head += kThreads) {
            const uint32_t e = (head + t) & (kRing - 1u);
            const uint32_t i = qa[e], j = qj[e];
            pair_move<R, C, OBS>(x, own, qk[e], i, j, rec[i], rec[j], nacc, pa);
        }
    }
    if (t < tail - head) {
        const uint32_t e = (head + t) & (kRing - 1u);
        const uint32_t i = qa[e], j = qj[e];
        pair_move<R, C, OBS>(x, own, qk[e], i, j, rec[i], rec[j], nacc, pa);
    }
    if constexpr (OBS) flush_part(acc, pa);
    KArgs<R> ra = a;
    ra.part = a.part + part_base;
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

// Colour-split bond masks from masks in site order: site i = 2k + p of row
// (y, z) has colour c = (x + y + z) & 1 and colour index k.
__global__ __launch_bounds__(kThreads) void split_masks_kernel(const uint8_t* src, uint8_t* dst, uint32_t Nc,
                                                               uint32_t hx, uint32_t ny)
{
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= Nc) return;
    const uint32_t r = k / hx;
    const uint32_t y = r % ny, z = r / ny;
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) dst[(size_t)c * Nc + k] = src[2 * (size_t)k + ((y + z + c) & 1u)];
}

hipError_t launch_split_masks(const DevLattice& d, const uint8_t* src, hipStream_t s)
{
    split_masks_kernel<<<cdiv((uint64_t)d.Nc, kThreads), kThreads, 0, s>>>(src, d.mask, (uint32_t)d.Nc,
                                                                             (uint32_t)d.hx, (uint32_t)d.ny);
    return hipGetLastError();
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
    Rec<R>* rec = reinterpret_cast<Rec<R>*>(aos + 2 * (size_t)d.Nc);
    const uint32_t n = (uint32_t)d.Nc;
    const uint32_t full = cdiv(n, kThreads);
    const uint32_t tiles = cdiv(n, kPairTile);
    const uint32_t pgrid = tiles < (uint32_t)HMC_PAIR_BLOCKS ? tiles : (uint32_t)HMC_PAIR_BLOCKS;
    const uint32_t ngrid = full < (uint32_t)HMC_NB_BLOCKS ? full : (uint32_t)HMC_NB_BLOCKS;
    *blocks = pgrid;
    if (step == kAosIn) {
        aos_copy_kernel<R, true><<<dim3(full, 2), kThreads, 0, s>>>(a, aos);
    } else if (step == kAosOut) {
        aos_copy_kernel<R, false><<<dim3(full, 2), kThreads, 0, s>>>(a, aos);
    } else if (step == kNbRed) {
        records_kernel<R, 0><<<ngrid, kThreads, 0, s>>>(a, aos, rec);
    } else if (step == kNbBlack) {
        records_kernel<R, 1><<<ngrid, kThreads, 0, s>>>(a, aos, rec);
    } else {
        const V3<R> ec{(R)eC[0], (R)eC[1], (R)eC[2]};
        const R scale = Prim<R>::scale_for(T);
        const Shuffle f = shuffle_for(n);
        if (step == kPairRed) pair_kernel<R, 0, true><<<pgrid, kThreads, 0, s>>>(a, aos, rec, ec, f, scale, 0u);
        else pair_kernel<R, 1, true><<<pgrid, kThreads, 0, s>>>(a, aos, rec, ec, f, scale, pgrid);
    }
}

hipError_t launch_constrained(const DevLattice& d, int step, const double eC[3], double T, hipStream_t s,
                              int64_t* blocks)
{
    if (d.precision == 32) constrained_go<float>(d, step, eC, T, s, blocks);
    else constrained_go<double>(d, step, eC, T, s, blocks);
    return hipGetLastError();
}

template <typename R>
static void finalize_records_go(const DevLattice& d, int64_t rec_blocks, int fin, double T, hipStream_t s)
{
    Vec4<R>* aos = static_cast<Vec4<R>*>(d.aos);
    const uint32_t full = cdiv((uint64_t)d.Nc, kThreads);
    const uint32_t ngrid = 1u + (full < (uint32_t)HMC_NB_BLOCKS ? full : (uint32_t)HMC_NB_BLOCKS);
    finalize_records_kernel<R><<<ngrid, kThreads, 0, s>>>(make_args<R>(d), aos,
                                                          reinterpret_cast<Rec<R>*>(aos + 2 * (size_t)d.Nc),
                                                          (uint32_t)rec_blocks, fin, T, (double)d.N);
}

hipError_t launch_finalize_nbsum(const DevLattice& d, int64_t rec_blocks, int fin, double T, hipStream_t s)
{
    if (d.precision == 32) finalize_records_go<float>(d, rec_blocks, fin, T, s);
    else finalize_records_go<double>(d, rec_blocks, fin, T, s);
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
    const uint32_t stride = (uint32_t)d.max_blocks;
    const uint32_t G = (uint32_t)cdiv((uint64_t)part_blocks, (uint64_t)kGroupRecords);
    const double* l2 = nullptr;
    if ((fin & kFinObs) && G > kFinGroupsInKernel) {
        // the group sums, in parallel, into the space after the partial rows
        double* g2 = d.part + (size_t)kNumPart * stride;
        const uint32_t nrows = (fin & kFinTorque) ? (uint32_t)kTorqueRows : (uint32_t)kObsRows;
        fold_groups_kernel<<<G, kGroupThreads, 0, s>>>(d.part, stride, (uint32_t)part_blocks, nrows, g2);
        l2 = g2;
    }
    finalize_kernel<<<1, 1024, 0, s>>>(d.st, d.part, stride, d.cnt, (uint32_t)red_blocks, (uint32_t)black_blocks,
                                       (uint32_t)part_blocks, l2, fin, T, (double)d.N);
    return hipGetLastError();
}

}  // namespace hmc
