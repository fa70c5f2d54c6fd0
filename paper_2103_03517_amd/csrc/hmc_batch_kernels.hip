// hmc_batch_kernels.hip -- the kernels of batches (hmc_batch_* in hmc.h):
// one colour-pass launch over the lattices of a kernel-variant group, the
// per-lattice finalize and accumulator reset, and their launchers.
#include "hmc_pass.hpp"

namespace hmc {

// Finalize of a batch: work-group i folds the results of lattice i with its
// own flags fin[i] (a lattice that does not sample ignores the partials of a
// black pass that computed them for others).
// (256 threads: the record fold of finalize_body needs no more, and the
// lattices of a batch are small enough that the counts take a round or two)
template <typename R>
__global__ __launch_bounds__(kThreads) void finalize_batch_kernel(const BatchEntry<R>* __restrict__ tab,
                                                                  const double* __restrict__ T,
                                                                  const int32_t* __restrict__ fin)
{
    __shared__ double scratch[kFinScratch];
    __shared__ DevState sst;
    const BatchEntry<R>& E = tab[blockIdx.x];
    const int f = fin[blockIdx.x];
    finalize_body<kThreads>(E.a.st, E.a.part, E.a.cnt_stride, E.a.cnt, E.nblk, E.nblk,
                            (f & kFinObs) ? E.nblk : 0u, nullptr, f, T[blockIdx.x], E.N, scratch, &sst);
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
    pass_tile<R, C, OBS, SPT, HALO, false, false>(E.a, E.zc, E.nqb, gb - start[lo], scale[e], smem);
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
