// hmc_pass.hpp -- device code shared by the kernel translation units:
// kernel arguments, buffer-resource access, LDS planes, fixed-order
// reductions, the per-sweep finalize and the tile of the standard colour
// pass (hmc_kernels.hip launches it for one lattice, hmc_batch_kernels.hip
// for a batch).
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
#pragma once

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
    uint32_t cnt_stride; // row stride of cnt and of part ([kNumPart][cnt_stride] doubles)
    uint32_t zbound;     // z boundary: 0 periodic, 1 anti-periodic, 2 open
    const uint8_t* mask[2];  // per colour, Nc bytes of active-bond bits (x-, x+, y-, y+, z-, z+), or null
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
    a.zbound = (uint32_t)d.zbound;
    a.mask[0] = d.mask;
    a.mask[1] = d.mask ? d.mask + d.Nc : nullptr;
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

// A neighbour seen across the z boundary: its sign flipped (anti-periodic,
// zbound 1) or no bond at all (open, zbound 2).
template <typename R>
__device__ __forceinline__ V3<R> across_z(const V3<R>& v, uint32_t zbound)
{
    return zbound == 1 ? neg(v) : V3<R>{R(0), R(0), R(0)};
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

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Halo slots per thread of the standard pass (a template argument).
static inline int halo_slots(int hx)
{
    const int halo = (2 * hx + kThreads - 1) / kThreads;
    return halo <= 1 ? 1 : (halo == 2 ? 2 : 4);
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
// Fixed-order reductions.  Within a wave a DPP tree, across the four waves
// of a work-group in wave order, across work-groups by the finalize kernel in
// the order set out at finalize_body.  The results therefore do not depend
// on scheduling.
// ---------------------------------------------------------------------------
// Cross-lane moves for the wave sum: DPP row operations (gfx9 encodings),
// which run on the vector ALU instead of the LDS crossbar.
constexpr int kDppQuadSwap1 = 0xB1;        // quad_perm [1,0,3,2]: lane i takes lane i ^ 1
constexpr int kDppQuadSwap2 = 0x4E;        // quad_perm [2,3,0,1]: lane i takes lane i ^ 2
constexpr int kDppRowHalfMirror = 0x141;   // lane i takes lane 7 - i within its 8-lane half-row
constexpr int kDppRowMirror = 0x140;       // lane i takes lane 15 - i within its 16-lane row

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint64_t lo = dpp_u32<CTRL>((uint32_t)u), hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
        return __builtin_bit_cast(T, lo | (hi << 32));
    }
}

template <typename T>
__device__ __forceinline__ T read_lane(T v, int lane)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, v), lane));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
        const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
        return __builtin_bit_cast(T, lo | (hi << 32));
    }
}

// Sum over the 64 lanes of a wave (all lanes active), the same on every
// lane: pairs, quads, half-rows and rows by DPP moves (at each step the two
// lanes of a pair add the same two values, so they hold the same sum), then
// the four row sums as (row0 + row1) + (row2 + row3).
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v += dpp_move<kDppQuadSwap1>(v);
    v += dpp_move<kDppQuadSwap2>(v);
    v += dpp_move<kDppRowHalfMirror>(v);
    v += dpp_move<kDppRowMirror>(v);
    const T r0 = read_lane(v, 0), r1 = read_lane(v, 16), r2 = read_lane(v, 32), r3 = read_lane(v, 48);
    return (r0 + r1) + (r2 + r3);
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
// and (OBS) its partial sums, component e at part[e * cnt_stride + b] (one
// row per component, so the finalize reads each row coalesced): the moment
// and the energies, and with TQ the torque.  They are reduced by
// finalize_kernel, launched next on the same stream (the kernel boundary
// makes them visible).  scratch: at least 5 * kTorqueRows + 2 doubles.
template <typename R, bool OBS, bool TQ = true>
__device__ __forceinline__ void block_end(const KArgs<R>& a, int colour, uint32_t b, uint32_t nacc, const Acc& acc,
                                          double* scratch)
{
    if (OBS) {
        constexpr int NV = TQ ? kTorqueRows : kObsRows;
        double v[NV];
        v[kMx] = acc.M[0];
        v[kMy] = acc.M[1];
        v[kMz] = acc.M[2];
        v[kEexch] = acc.ex;
        v[kEuni] = acc.eu;
        v[kEcub] = acc.ec;
        v[kEzee] = acc.ez;
        if constexpr (TQ) {
            v[kTx] = acc.tq[0];
            v[kTy] = acc.tq[1];
            v[kTz] = acc.tq[2];
        }
        // the count as an integer, its wave sums published by block_sum's barriers
        uint32_t* s32 = reinterpret_cast<uint32_t*>(scratch + 5 * NV);
        const uint32_t c = wave_sum(nacc);
        if ((threadIdx.x & 63) == 0) s32[threadIdx.x >> 6] = c;
        block_sum<NV>(v, scratch);
        if (threadIdx.x < (uint32_t)NV) a.part[(size_t)threadIdx.x * a.cnt_stride + b] = scratch[threadIdx.x];
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < kThreads / 64; ++w) tot += s32[w];
            a.cnt[(size_t)colour * a.cnt_stride + b] = tot;
        }
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
// Per-sweep finalize: the fixed-order reduction of the work-group results of
// the colour-1 (and, for the counts, colour-0) launch, then Table A1's
// cone-angle rule (one degree up when accepted/N > 1/2, else down, within
// [1, 180]), the sweep counter and on sampled sweeps the shifted FP64
// accumulators of Eq. 6.
//
// The records are folded in one order, whichever kernel folds them.  They
// form groups of 1024 (group g: records 1024g .. 1024g + 1023).  In a group,
// thread t of 256 adds records 1024g + t, + 256, + 512 and + 768 in turn
// (from 0.0); wave_sum adds the threads of each wave and the four wave sums
// are added in wave order (from 0.0), giving the group sum S_g.  The total is
// ((0.0 + S_0) + S_1) + ... .  A group is one round of loads (4 per folded row
// and thread: the 7 rows of M and the energies, 10 with the torque).
// With more than one group the single-lattice path forms the group sums in
// parallel (fold_groups_kernel, one work-group per group) and the finalize
// adds them; the batch and constrained finalizes form them one after the
// other (a 1024-thread work-group would form four per round).
// The counts are integers, summed in any order.
// ---------------------------------------------------------------------------
constexpr int kGroupRecords = 1024;
constexpr int kGroupThreads = 256;
// doubles of shared memory finalize_body needs: the wave sums [16][kNumPart],
// the group sums of a round [4][kNumPart], the totals [kNumPart + 1] and the
// per-wave counts [16]
constexpr int kFinScratch = 16 * kNumPart + 4 * kNumPart + kNumPart + 1 + 16;
// group sums the single-lattice finalize forms itself; above this,
// fold_groups_kernel forms them in parallel first.  One work-group reading
// several groups is bound by what one CU can fetch (measured on MI355X: 24
// us for the 7 groups of a 384^3 pass with 8-plane chunks, against 13 us
// with the parallel fold), so the finalize takes one group at most.
constexpr uint32_t kFinGroupsInKernel = 1;

// The group sums S_g of groups g0, g0 + 1, ... (those below G), one group
// per 256 threads of the work-group, into sg[j * kNumPart ..] for group
// g0 + j (shared memory; wsum holds [NT / 64][kNumPart]).  Every thread of
// the work-group calls it (it holds barriers).
template <int NT, int NR>
__device__ __forceinline__ void group_sums(const double* part, uint32_t stride, uint32_t npart, uint32_t g0,
                                           uint32_t G, double* wsum, double* sg)
{
    constexpr int PG = NT / kGroupThreads;
    const uint32_t t = threadIdx.x, tl = t % (uint32_t)kGroupThreads;
    const uint32_t g = g0 + t / (uint32_t)kGroupThreads;
    if (g < G) {                       // uniform over each 256 threads (whole waves)
        const uint32_t r0 = g * (uint32_t)kGroupRecords + tl;
        double q[4][NR];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t r = r0 + (uint32_t)(u * kGroupThreads);
            const double* p = part + (r < npart ? r : 0u);     // record 0 always exists
#pragma unroll
            for (int e = 0; e < NR; ++e) q[u][e] = p[(size_t)e * stride];
        }
        // a record past the end adds +0.0, which changes no sum (no partial
        // sum here is ever -0.0), so the loads need no branch
        double v[NR];
#pragma unroll
        for (int e = 0; e < NR; ++e) v[e] = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool in = r0 + (uint32_t)(u * kGroupThreads) < npart;
#pragma unroll
            for (int e = 0; e < NR; ++e) v[e] += in ? q[u][e] : 0.0;
        }
        // all wave sums first, then one branch for the stores
#pragma unroll
        for (int e = 0; e < NR; ++e) v[e] = wave_sum(v[e]);
        if ((t & 63u) == 0) {
#pragma unroll
            for (int e = 0; e < NR; ++e) wsum[(t >> 6) * kNumPart + e] = v[e];
        }
    }
    __syncthreads();
    if (t < (uint32_t)(PG * NR)) {
        const uint32_t j = t / (uint32_t)NR, e = t % (uint32_t)NR;
        if (g0 + j < G) {
            double x = 0.0;
            for (int w = 0; w < kGroupThreads / 64; ++w)
                x += wsum[((int)j * (kGroupThreads / 64) + w) * kNumPart + (int)e];
            sg[j * kNumPart + e] = x;
        }
    }
    __syncthreads();
}

// The finalize of one lattice by one work-group of NT threads (256 or 1024).
// stride: row stride of part and cnt; l2: the group sums computed by
// fold_groups_kernel ([G][kNumPart]), or null when this work-group computes
// them.  sst: shared memory for a copy of the chain state, read at the start
// so that the state update at the end does not wait for global memory.
template <int NT>
__device__ __forceinline__ void finalize_body(DevState* st, const double* part, uint32_t stride, const uint32_t* cnt,
                                              uint32_t nred, uint32_t nblack, uint32_t npart, const double* l2,
                                              int fin, double T, double N, double* scratch, DevState* sst)
{
    static_assert(NT >= kGroupThreads && NT % 64 == 0 && NT <= 1024, "work-group size");
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    double* wsum = scratch;                                                   // [16][kNumPart]
    double* sg = scratch + 16 * kNumPart;                                     // [4][kNumPart]
    double* tot = sg + 4 * kNumPart;                                          // [kNumPart + 1]
    unsigned long long* wc = reinterpret_cast<unsigned long long*>(tot + kNumPart + 1);   // [NT / 64]
    // the last wave takes no part in the record fold: one of its threads
    // copies the chain state while the others fold
    if (t == (uint32_t)NT - 1) *sst = *st;
    if (fin & kFinCounts) {
        // integer sums: any order gives the same total; eight loads in flight
        constexpr int UC = 8;
        const uint32_t nc = nred + nblack;
        unsigned long long c = 0;
        for (uint32_t i = t; i < nc; i += UC * NT) {
            uint32_t w[UC];
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const uint32_t j = i + (uint32_t)u * NT;
                const uint32_t jj = j < nc ? j : i;                    // always in range
                const uint32_t x = jj < nred ? cnt[jj] : cnt[stride + (jj - nred)];
                w[u] = j < nc ? x : 0u;
            }
#pragma unroll
            for (int u = 0; u < UC; ++u) c += w[u];
        }
        c = wave_sum(c);
        if (lane == 0) wc[wave] = c;
    }
    if (fin & kFinObs) {
        const uint32_t G = (npart + (uint32_t)kGroupRecords - 1u) / (uint32_t)kGroupRecords;
        const bool torque = (fin & kFinTorque) != 0;
        const uint32_t nrows = torque ? (uint32_t)kTorqueRows : (uint32_t)kObsRows;
        if (l2 != nullptr) {
            if (t < (uint32_t)kNumPart) {
                double x = 0.0;
                if (t < nrows)
                    for (uint32_t g = 0; g < G; ++g) x += l2[(size_t)g * kNumPart + t];
                tot[t] = x;
            }
        } else {
            // rounds of NT / 256 groups formed side by side, added in order
            constexpr uint32_t PG = NT / kGroupThreads;
            double run = 0.0;          // threads 0..nrows-1: the running total
            for (uint32_t g0 = 0; g0 < G; g0 += PG) {
                if (torque) group_sums<NT, kTorqueRows>(part, stride, npart, g0, G, wsum, sg);
                else group_sums<NT, kObsRows>(part, stride, npart, g0, G, wsum, sg);
                if (t < nrows)
                    for (uint32_t j = 0; j < PG && g0 + j < G; ++j) run += sg[j * kNumPart + t];
            }
            if (t < (uint32_t)kNumPart) tot[t] = run;
        }
    }
    __syncthreads();
    if ((fin & kFinCounts) && t == (uint32_t)kNumPart) {
        unsigned long long c = 0;
        for (int w = 0; w < NT / 64; ++w) c += wc[w];
        tot[kNumPart] = (double)c;
    }
    __syncthreads();
    if (t != 0) return;
    const DevState& cur = *sst;
    if (fin & kFinCounts) {
        const long long accepted = (long long)tot[kNumPart];
        st->accepted_last = accepted;
        int32_t th = cur.theta;
        if (2.0 * (double)accepted > N) {
            if (th < 180) th += 1;
        } else {
            if (th > 1) th -= 1;
        }
        st->theta = th;
        st->sweep = cur.sweep + 1;
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
            const bool first = cur.samples == 0;
            for (int i = 0; i < 5; ++i) {
                const double sh = first ? x[i] : cur.shift[i];
                if (first) st->shift[i] = x[i];
                const double d = x[i] - sh;
                st->sum[i] = cur.sum[i] + d;
                st->sum2[i] = cur.sum2[i] + d * d;
            }
            st->sum_eanis = cur.sum_eanis + (tot[kEuni] + tot[kEcub]) / N;
            if (fin & kFinTorque) {
                for (int i = 0; i < 3; ++i) st->sum_torque[i] = cur.sum_torque[i] + tot[kTx + i] / N;
                st->torque_samples = cur.torque_samples + 1;
            }
            st->samples = cur.samples + 1;
            st->T_sample = T;
        }
    }
}

// ---------------------------------------------------------------------------
// The Metropolis update of one site (Table A1, Eq. 1, Eq. 2): cone proposal,
// energy change in the local field, acceptance P < exp(-dE/T).  Returns the
// final spin; OBS adds the site and its red x-partner to the observables.
// ---------------------------------------------------------------------------
template <typename R, bool OBS, typename A>
__device__ __forceinline__ V3<R> update_site(const Model<R>& m, const V3<R>& s, const V3<R>& nb,
                                             const V3<R>& partner, const Rand4& rn, R c1, R scale,
                                             uint32_t& nacc, A& acc)
{
    const V3<R> hl{m.J * nb.x + m.h.x, m.J * nb.y + m.h.y, m.J * nb.z + m.h.z};
    const V3<R> tr = cone_move(s, Prim<R>::u01(rn.r0), Prim<R>::u01(rn.r1), c1);
    SiteTerms<R> k;
    const R dE = delta_e(m, s, tr, hl, k);
    const bool ok = Prim<R>::u01(rn.r2) < Prim<R>::boltzmann(dE, scale);
    const V3<R> f = ok ? tr : s;
    nacc += ok ? 1u : 0u;
    if (OBS) {
        // acc is the FP64 Acc (FP64 spins) or the spin-precision partial sums
        const V3<R> fp{f.x + partner.x, f.y + partner.y, f.z + partner.z};
        acc.M[0] += fp.x;
        acc.M[1] += fp.y;
        acc.M[2] += fp.z;
        acc.ex += -m.J * dot(f, nb);
        if (m.Ku != R(0)) {
            const R sf = ok ? k.te : k.se, sp = dot(partner, m.e);
            acc.eu += -m.Ku * (sf * sf + sp * sp);
        }
        if (m.Kc != R(0)) acc.ec += m.Kc * ((ok ? k.ct : k.cs) + cubic_f(partner));
        if (m.h.x != R(0) || m.h.y != R(0) || m.h.z != R(0)) acc.ez += -dot(m.h, fp);
    }
    return f;
}

// ---------------------------------------------------------------------------
// Standard colour pass (Table A1, MonteCarlo_Red(Black)ParallelPass).
//
// A work-group owns Q = 256*SPT consecutive in-plane colour indices and
// marches over z_chunk planes.  The other colour's plane z sits in LDS as a
// window [base - hx, base + Q + hx) (the x and y neighbours), so each plane
// of each colour is fetched once per pass (plus a halo of 2*hx entries per
// plane).  Two marches share this layout and differ in how far ahead the
// loads run:
//
// * depth one (march1): step z issues the other colour's plane z+2 and the
//   own colour's plane z+1; the other colour's z-1, z, z+1 and z+2 values at
//   the owned columns stay in registers, rotating by renaming over a march
//   unrolled by four.  Best while the spins stay in the 256 MB last-level
//   cache, whose latency one plane of look-ahead covers.
// * depth two (march2): step z issues the other colour's plane z+3 and the
//   own colour's plane z+2, so two planes of loads are in flight while one
//   is computed; the same-index partner comes from the window and becomes
//   the z-1 value of the next step, and three register planes rotate over a
//   march unrolled by three.  Best for lattices that stream from HBM.
//
// OBS (black pass only) fuses the observables: the black site after its
// update plus its red x-partner (same colour index), and the exchange of the
// black site with its six final red neighbours, so every site and every bond
// is counted once.  With FP32 spins a thread sums these terms in FP32 over
// its z chunk (z_chunk x SPT sites) and converts the sums to FP64 once;
// everything above the thread is FP64.
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
    uint32_t zbound;
};

// Depth-one march: one step, plane z = z0 + zi; the register planes om, o0,
// op, opp hold the other colour's z-1, z, z+1 and z+2 (in flight), sc and
// sn the own colour's z and z+1 (in flight), hp and hpp the halo's z+1 and
// z+2 (in flight).
template <typename R, int C, bool OBS, int SPT, int HALO, int K, bool MASK, typename A>
__device__ __forceinline__ void step1(const KArgs<R>& a, const Arrays<R>& g, const PassCtx<R, SPT, HALO>& x,
                                          uint32_t zi, V3<R> (&om)[SPT], V3<R> (&o0)[SPT], V3<R> (&op)[SPT],
                                          V3<R> (&opp)[SPT], V3<R> (&sc)[SPT], V3<R> (&sn)[SPT],
                                          V3<R> (&hp)[HALO], V3<R> (&hpp)[HALO], uint32_t& nacc, A& acc)
{
    constexpr int O = 1 - C;
    constexpr int B = K & 1;
    const uint32_t z = x.z0 + zi;
    const bool more = zi + 1 < x.zn;
    auto plane_off = [&](uint32_t zz) -> uint32_t {
        return x.P * (uint32_t)sizeof(R) * (zz >= x.nz ? zz - x.nz : zz);
    };
    if (more) {
        // the look-ahead loads leave at a raised wave priority: the march is
        // bound by their latency, and the SIMD then issues them before other
        // waves' arithmetic (measured on MI355X: 256^3 FP32 pass 53.7 -> 53.0
        // us)
        __builtin_amdgcn_s_setprio(2);
        const uint32_t fpp = plane_off(z + 2), fn = plane_off(z + 1);
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            opp[j] = g.get(O, x.voff[j], fpp);
            sn[j] = g.get(C, x.voff[j], fn);
        }
#pragma unroll
        for (int i = 0; i < HALO; ++i)
            if (x.hact[i]) hpp[i] = g.get(O, x.hvoff[i], fpp);
        __builtin_amdgcn_s_setprio(0);
        // anti-periodic or open z: plane z + 2 = nz is plane 0 seen across
        // the boundary; it serves only as the z+1 neighbour of plane nz - 1.
        // The uniform branch is taken once per tile at most.
        if (__builtin_expect(x.zbound != 0 && z + 2u == x.nz, 0)) {
            __asm__ volatile("");
#pragma unroll
            for (int j = 0; j < SPT; ++j) opp[j] = across_z(opp[j], x.zbound);
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
        const uint32_t k = x.voff[j] / (uint32_t)sizeof(R) + x.P * (z >= x.nz ? z - x.nz : z);
        V3<R> nb;
        if (MASK) {
            // bonds cut by the site's mask (intergrain bonds) weigh zero
            const uint32_t mb = a.mask[C][k];
            const R w0 = (mb & 1u) ? R(1) : R(0), w1 = (mb & 2u) ? R(1) : R(0);
            const R w2 = (mb & 4u) ? R(1) : R(0), w3 = (mb & 8u) ? R(1) : R(0);
            const R w4 = (mb & 16u) ? R(1) : R(0), w5 = (mb & 32u) ? R(1) : R(0);
            nb = V3<R>{((((w0 * xm.x + w1 * xp.x) + w2 * ym.x) + w3 * yp.x) + w4 * om[j].x) + w5 * op[j].x,
                       ((((w0 * xm.y + w1 * xp.y) + w2 * ym.y) + w3 * yp.y) + w4 * om[j].y) + w5 * op[j].y,
                       ((((w0 * xm.z + w1 * xp.z) + w2 * ym.z) + w3 * yp.z) + w4 * om[j].z) + w5 * op[j].z};
        } else {
            nb = V3<R>{((((xm.x + xp.x) + ym.x) + yp.x) + om[j].x) + op[j].x,
                       ((((xm.y + xp.y) + ym.y) + yp.y) + om[j].y) + op[j].y,
                       ((((xm.z + xp.z) + ym.z) + yp.z) + om[j].z) + op[j].z};
        }
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

template <typename R, int C, bool OBS, int SPT, int HALO, bool MASK>
__device__ __forceinline__ void march1(const KArgs<R>& a, const Arrays<R>& g, const PassCtx<R, SPT, HALO>& x,
                                       uint32_t& nacc, Acc& acc)
{
    constexpr int O = 1 - C;
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
        // anti-periodic or open z: the z-1 plane of z0 = 0 and the z+1 plane
        // of z0 = nz - 1 lie across the boundary (both used only as z
        // neighbours)
        if (x.zbound != 0 && x.z0 == 0) {
#pragma unroll
            for (int j = 0; j < SPT; ++j) rA[j] = across_z(rA[j], x.zbound);
        }
        if (x.zbound != 0 && x.z0 + 1u == a.nz) {
#pragma unroll
            for (int j = 0; j < SPT; ++j) rC[j] = across_z(rC[j], x.zbound);
        }
    }
    __syncthreads();

    Part<R> part;
    auto& pa = site_acc<R>(acc, part);
    uint32_t zi = 0;
    for (; zi + 4 <= x.zn; zi += 4) {
        step1<R, C, OBS, SPT, HALO, 0, MASK>(a, g, x, zi + 0, rA, rB, rC, rD, s0, s1, h0, h1, nacc, pa);
        step1<R, C, OBS, SPT, HALO, 1, MASK>(a, g, x, zi + 1, rB, rC, rD, rA, s1, s0, h1, h0, nacc, pa);
        step1<R, C, OBS, SPT, HALO, 2, MASK>(a, g, x, zi + 2, rC, rD, rA, rB, s0, s1, h0, h1, nacc, pa);
        step1<R, C, OBS, SPT, HALO, 3, MASK>(a, g, x, zi + 3, rD, rA, rB, rC, s1, s0, h1, h0, nacc, pa);
    }
    if (zi < x.zn) step1<R, C, OBS, SPT, HALO, 0, MASK>(a, g, x, zi + 0, rA, rB, rC, rD, s0, s1, h0, h1, nacc, pa);
    if (zi + 1 < x.zn) step1<R, C, OBS, SPT, HALO, 1, MASK>(a, g, x, zi + 1, rB, rC, rD, rA, s1, s0, h1, h0, nacc, pa);
    if (zi + 2 < x.zn) step1<R, C, OBS, SPT, HALO, 2, MASK>(a, g, x, zi + 2, rC, rD, rA, rB, s0, s1, h0, h1, nacc, pa);
    if constexpr (OBS) flush_part(acc, pa);

}

// Depth-two march: one step, plane z = z0 + zi.  op: the other colour's plane
// z+1 (landed); on: the slot that receives plane z+3.  sc, sn: the own
// colour's plane z (landed) and the slot for plane z+2; hp, hn: the halo
// likewise; mc, mn: the masks likewise.  om holds plane z-1 on entry and
// plane z on exit.
//
// Every step issues its loads unconditionally, so that the number of
// memory operations between a load and its use is the same on every path
// (the compiler's wait counts are then those of the steady state); the
// planes are clamped to the last one the tile needs, so the loads of the
// last steps re-read planes just fetched.
template <typename R, int C, bool OBS, int SPT, int HALO, bool MASK, typename A>
__device__ __forceinline__ void step2(const KArgs<R>& a, const Arrays<R>& g, const PassCtx<R, SPT, HALO>& x,
                                          uint32_t zi, V3<R> (&om)[SPT], V3<R> (&op)[SPT], V3<R> (&on)[SPT],
                                          V3<R> (&sc)[SPT], V3<R> (&sn)[SPT], V3<R> (&hp)[HALO],
                                          V3<R> (&hn)[HALO], uint32_t (&mc)[SPT], uint32_t (&mn)[SPT],
                                          uint32_t& nacc, A& acc)
{
    constexpr int O = 1 - C;
    const uint32_t z = x.z0 + zi;
    const uint32_t B = zi & 1u;
    const uint32_t zend = x.z0 + x.zn;      // <= nz
    auto plane_off = [&](uint32_t zz) -> uint32_t {
        return x.P * (uint32_t)sizeof(R) * (zz >= x.nz ? zz - x.nz : zz);
    };
    // loads two planes ahead: the other colour's plane z+3 (the z+1
    // neighbour of plane z+2) and the own colour's plane z+2
    // (at the normal wave priority: raising it around these loads, as the
    // depth-one step does, measured 0.5-1.3 % slower at 384^3 and 464^3)
    const uint32_t z3 = min(z + 3u, zend), z2 = min(z + 2u, zend - 1u);
    const uint32_t f3 = plane_off(z3), f2 = plane_off(z2);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        on[j] = g.get(O, x.voff[j], f3);
        sn[j] = g.get(C, x.voff[j], f2);
        if (MASK) mn[j] = a.mask[C][x.voff[j] / (uint32_t)sizeof(R) + x.P * z2];
    }
#pragma unroll
    for (int i = 0; i < HALO; ++i) hn[i] = g.get(O, x.hvoff[i], f3);
    // anti-periodic or open z: plane nz is plane 0 seen across the boundary
    // (only ever the z+1 neighbour of plane nz - 1); a uniform branch taken
    // in the top tile only
    if (__builtin_expect(x.zbound != 0 && z3 == x.nz, 0)) {
        __asm__ volatile("");
#pragma unroll
        for (int j = 0; j < SPT; ++j) on[j] = across_z(on[j], x.zbound);
    }
    // plane z+1 (issued two steps ago) into the other LDS buffer; its
    // readers of the step before have passed the barrier
    {
        unsigned char* Ln = B ? x.lds[0] : x.lds[1];   // a select keeps the LDS addressing
#pragma unroll
        for (int j = 0; j < SPT; ++j) LdsPlane<R>::put(Ln, x.W, x.w[j], op[j]);
#pragma unroll
        for (int i = 0; i < HALO; ++i)
            if (x.hact[i]) LdsPlane<R>::put(Ln, x.W, x.hw[i], hp[i]);
    }
    const unsigned char* L = B ? x.lds[1] : x.lds[0];
    const uint32_t fz = plane_off(z);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        if (!x.act[j]) continue;
        const uint32_t p = x.par[j] ^ B;
        const V3<R> xd = LdsPlane<R>::get(L, x.W, B ? x.wd[1][j] : x.wd[0][j]);
        const V3<R> ym = LdsPlane<R>::get(L, x.W, x.w[j] - x.hx);
        const V3<R> yp = LdsPlane<R>::get(L, x.W, x.w[j] + x.hx);
        const V3<R> o0 = LdsPlane<R>::get(L, x.W, x.w[j]);
        const V3<R> xm = p ? o0 : xd;
        const V3<R> xp = p ? xd : o0;
        const uint32_t k = x.voff[j] / (uint32_t)sizeof(R) + x.P * z;
        V3<R> nb;
        if (MASK) {
            // bonds cut by the site's mask (intergrain bonds) weigh zero
            const uint32_t mb = mc[j];
            const R w0 = (mb & 1u) ? R(1) : R(0), w1 = (mb & 2u) ? R(1) : R(0);
            const R w2 = (mb & 4u) ? R(1) : R(0), w3 = (mb & 8u) ? R(1) : R(0);
            const R w4 = (mb & 16u) ? R(1) : R(0), w5 = (mb & 32u) ? R(1) : R(0);
            nb = V3<R>{((((w0 * xm.x + w1 * xp.x) + w2 * ym.x) + w3 * yp.x) + w4 * om[j].x) + w5 * op[j].x,
                       ((((w0 * xm.y + w1 * xp.y) + w2 * ym.y) + w3 * yp.y) + w4 * om[j].y) + w5 * op[j].y,
                       ((((w0 * xm.z + w1 * xp.z) + w2 * ym.z) + w3 * yp.z) + w4 * om[j].z) + w5 * op[j].z};
        } else {
            nb = V3<R>{((((xm.x + xp.x) + ym.x) + yp.x) + om[j].x) + op[j].x,
                       ((((xm.y + xp.y) + ym.y) + yp.y) + om[j].y) + op[j].y,
                       ((((xm.z + xp.z) + ym.z) + yp.z) + om[j].z) + op[j].z};
        }
        const Rand4 rn = philox(x.sweep, 2u * k + p, (uint32_t)C, a.inst, a.key0, a.key1);
        const V3<R> f = update_site<R, OBS>(a.m, sc[j], nb, o0, rn, x.c1, x.scale, nacc, acc);
        g.put(C, x.voff[j], fz, f);
        om[j] = o0;
    }
    __syncthreads();
}

template <typename R, int C, bool OBS, int SPT, int HALO, bool MASK>
__device__ __forceinline__ void march2(const KArgs<R>& a, const Arrays<R>& g, const PassCtx<R, SPT, HALO>& x,
                                       uint32_t& nacc, Acc& acc)
{
    constexpr int O = 1 - C;
    // register planes: the other colour's z-1 (om) and three rotating slots
    // (planes z+1, z+2, z+3 at step z), the own colour's and the halo's
    // three rotating slots, and the masks'
    V3<R> om[SPT], oA[SPT], oB[SPT], oC[SPT], sA[SPT], sB[SPT], sC[SPT], hA[HALO], hB[HALO], hC[HALO];
    uint32_t mA[SPT], mB[SPT], mC[SPT];
    {
        auto plane_off = [&](int zz) -> uint32_t {
            const int w = zz < 0 ? zz + (int)a.nz : (zz >= (int)a.nz ? zz - (int)a.nz : zz);
            return a.P * (uint32_t)sizeof(R) * (uint32_t)w;
        };
        // planes z0-1 .. z0+2 of the other colour, z0 and z0+1 of the own
        // colour (clamped to the tile's last needed plane, as in the steps)
        const uint32_t zend = x.z0 + x.zn;
        const uint32_t pB = min(x.z0 + 2u, zend), sBz = min(x.z0 + 1u, zend - 1u);
        const uint32_t fm = plane_off((int)x.z0 - 1), f0 = plane_off((int)x.z0), f1 = plane_off((int)x.z0 + 1),
                       f2 = plane_off((int)pB), fs1 = plane_off((int)sBz);
        // plane z0 (written to LDS below) is loaded last: waiting for it
        // waits for every other prologue load, so no prologue load is still
        // in flight when the march starts and the waits inside the march are
        // set by the march alone
        V3<R> o0[SPT], h0[HALO];
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            om[j] = g.get(O, x.voff[j], fm);
            oA[j] = g.get(O, x.voff[j], f1);
            oB[j] = g.get(O, x.voff[j], f2);
            sA[j] = g.get(C, x.voff[j], f0);
            sB[j] = g.get(C, x.voff[j], fs1);
            if (MASK) {
                mA[j] = a.mask[C][x.voff[j] / (uint32_t)sizeof(R) + a.P * x.z0];
                mB[j] = a.mask[C][x.voff[j] / (uint32_t)sizeof(R) + a.P * sBz];
            }
        }
#pragma unroll
        for (int i = 0; i < HALO; ++i) {
            hA[i] = g.get(O, x.hvoff[i], f1);
            hB[i] = g.get(O, x.hvoff[i], f2);
        }
#pragma unroll
        for (int j = 0; j < SPT; ++j) o0[j] = g.get(O, x.voff[j], f0);
#pragma unroll
        for (int i = 0; i < HALO; ++i) h0[i] = g.get(O, x.hvoff[i], f0);
#pragma unroll
        for (int i = 0; i < HALO; ++i)
            if (x.hact[i]) LdsPlane<R>::put(x.lds[0], x.W, x.hw[i], h0[i]);
#pragma unroll
        for (int j = 0; j < SPT; ++j) LdsPlane<R>::put(x.lds[0], x.W, x.w[j], o0[j]);
        // anti-periodic or open z: plane -1 (the z-1 neighbour of plane 0)
        // and plane nz (the z+1 neighbour of plane nz - 1) lie across the
        // boundary
        if (x.zbound != 0) {
#pragma unroll
            for (int j = 0; j < SPT; ++j) {
                if (x.z0 == 0) om[j] = across_z(om[j], x.zbound);
                if (x.z0 + 1u == a.nz) oA[j] = across_z(oA[j], x.zbound);
                if (pB == a.nz) oB[j] = across_z(oB[j], x.zbound);
            }
        }
    }
    __syncthreads();

    Part<R> part;
    auto& pa = site_acc<R>(acc, part);
    uint32_t zi = 0;
    for (; zi + 3 <= x.zn; zi += 3) {
        step2<R, C, OBS, SPT, HALO, MASK>(a, g, x, zi + 0, om, oA, oC, sA, sC, hA, hC, mA, mC, nacc, pa);
        step2<R, C, OBS, SPT, HALO, MASK>(a, g, x, zi + 1, om, oB, oA, sB, sA, hB, hA, mB, mA, nacc, pa);
        step2<R, C, OBS, SPT, HALO, MASK>(a, g, x, zi + 2, om, oC, oB, sC, sB, hC, hB, mC, mB, nacc, pa);
    }
    if (zi < x.zn) step2<R, C, OBS, SPT, HALO, MASK>(a, g, x, zi + 0, om, oA, oC, sA, sC, hA, hC, mA, mC, nacc, pa);
    if (zi + 1 < x.zn) step2<R, C, OBS, SPT, HALO, MASK>(a, g, x, zi + 1, om, oB, oA, sB, sA, hB, hA, mB, mA, nacc, pa);
    if constexpr (OBS) flush_part(acc, pa);

}

// One work-group of a colour pass: logical tile b (column block b % nqb,
// z-slab b / nqb) of the lattice described by a, with the march of depth
// two when DEEP.
template <typename R, int C, bool OBS, int SPT, int HALO, bool MASK, bool DEEP>
__device__ __forceinline__ void pass_tile(const KArgs<R>& a, const uint32_t zc, const uint32_t nqb, const uint32_t b,
                                          const R scale, unsigned char* smem)
{
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
    x.zbound = a.zbound;

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

    uint32_t nacc = 0;
    Acc acc;
    if constexpr (DEEP) march2<R, C, OBS, SPT, HALO, MASK>(a, g, x, nacc, acc);
    else march1<R, C, OBS, SPT, HALO, MASK>(a, g, x, nacc, acc);
    // LDS is free after the last barrier of the march
    block_end<R, OBS, false>(a, C, b, nacc, acc, reinterpret_cast<double*>(smem));
}

// The depth-two FP32 variants with up to two sites per thread are held to
// 128 registers (four waves per SIMD), which they reach without spilling.
template <typename R, int SPT, int HALO, bool DEEP>
constexpr int pass_waves_per_eu()
{
    return DEEP && sizeof(R) == 4 && (SPT == 1 || (SPT == 2 && HALO <= 2)) ? 4 : 1;
}

template <typename R, int C, bool OBS, int SPT, int HALO, bool MASK, bool DEEP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(pass_waves_per_eu<R, SPT, HALO, DEEP>())))
void pass_kernel(const KArgs<R> a, const uint32_t zc, const uint32_t nqb, const uint32_t nblk, const R scale)
{
    extern __shared__ __align__(16) unsigned char smem[];
    pass_tile<R, C, OBS, SPT, HALO, MASK, DEEP>(a, zc, nqb, xcd_remap(blockIdx.x, nblk), scale, smem);
}


// Launch of one colour pass of one lattice; the kernel variant follows the
// launch shape (sites per thread), the halo width and the colour.  Each
// translation unit instantiates one family: the plain depth-one march in
// hmc_kernels.hip, the masked one in hmc_masked_kernels.hip, the depth-two
// march in hmc_deep_kernels.hip (so they compile in parallel).
template <bool MASK, bool DEEP>
struct PassLaunch {
    template <typename R, int C, bool OBS, int SPT, int HALO>
    static void go(const KArgs<R>& a, const DevLattice& d, int zc, double T, hipStream_t s)
    {
        const uint32_t nqb = cdiv((uint64_t)d.P, (uint64_t)kThreads * SPT);
        const uint32_t nzb = cdiv((uint64_t)d.nz, (uint64_t)zc);
        const uint32_t nblk = nqb * nzb;
        pass_kernel<R, C, OBS, SPT, HALO, MASK, DEEP><<<nblk, kThreads, pass_lds_bytes(d.precision, d.hx, SPT), s>>>(
            a, (uint32_t)zc, nqb, nblk, Prim<R>::scale_for(T));
    }

    template <typename R, int SPT, int HALO>
    static void by_colour(const KArgs<R>& a, const DevLattice& d, int colour, bool obs, int zc, double T,
                          hipStream_t s)
    {
        if (colour == 0) go<R, 0, false, SPT, HALO>(a, d, zc, T, s);
        else if (obs) go<R, 1, true, SPT, HALO>(a, d, zc, T, s);
        else go<R, 1, false, SPT, HALO>(a, d, zc, T, s);
    }

    template <typename R, int SPT>
    static void by_halo(const KArgs<R>& a, const DevLattice& d, int colour, bool obs, int zc, double T,
                        hipStream_t s)
    {
        const int halo = halo_slots(d.hx);
        if (halo == 1) by_colour<R, SPT, 1>(a, d, colour, obs, zc, T, s);
        else if (halo == 2) by_colour<R, SPT, 2>(a, d, colour, obs, zc, T, s);
        else by_colour<R, SPT, 4>(a, d, colour, obs, zc, T, s);
    }

    template <typename R>
    static void by_shape(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s)
    {
        const auto a = make_args<R>(d);
        if (spt == 1) by_halo<R, 1>(a, d, colour, obs, zc, T, s);
        else if (spt == 2) by_halo<R, 2>(a, d, colour, obs, zc, T, s);
        else by_halo<R, 4>(a, d, colour, obs, zc, T, s);
    }

    static hipError_t run(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s)
    {
        if (d.precision == 32) by_shape<float>(d, colour, obs, spt, zc, T, s);
        else by_shape<double>(d, colour, obs, spt, zc, T, s);
        return hipGetLastError();
    }
};

// The colour pass of a lattice with bond masks (hmc_masked_kernels.hip).
hipError_t launch_pass_masked(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s);
// The colour pass with the depth-two march (hmc_deep_kernels.hip).
hipError_t launch_pass_deep(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s);

}  // namespace hmc
