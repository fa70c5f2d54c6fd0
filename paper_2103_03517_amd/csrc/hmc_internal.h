// hmc_internal.h -- layout of the device workspace and the launchers that the
// C interface (hmc_api.cpp) calls in the kernel translation unit
// (hmc_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hmc {

constexpr int kThreads = 256;        // work-group size of every kernel
constexpr int kMaxHalo = 4;          // halo slots per thread: nx <= 1024
constexpr int kNumPart = 12;         // doubles per work-group partial
constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 64 * 1024;  // dynamic LDS budget of one work-group
constexpr uint64_t kDeepMarchBytes = 256ull << 20;  // spins above which the pass looks two planes ahead

// Per-work-group partial sums written by the passes and reduced in a fixed
// order by the finalize kernel.
enum PartSlot {
    kMx = 0, kMy, kMz,          // sum of S
    kEexch, kEuni, kEcub, kEzee, // energy terms, each bond once
    kTx, kTy, kTz,              // anisotropy torque
};
// Rows a launch writes and the finalize folds: the moment and the energies,
// plus the torque where it is measured (constrained sweeps and measurements).
// The acceptance counts go to their own integer rows; the part rows past
// these hold nothing.
constexpr int kObsRows = 7;
constexpr int kTorqueRows = 10;

// What the finalize kernel folds into the chain state.
enum FinFlags {
    kFinCounts = 1,      // acceptance counts: adapt theta, advance the sweep counter
    kFinObs = 2,         // M and the energies
    kFinTorque = 4,      // also the torque
    kFinSample = 8,      // add the reduced values to the accumulators
};

// Device-resident chain state (one per lattice, inside the workspace).
struct DevState {
    int32_t theta;            // cone angle, degrees
    int32_t nonfinite;        // sticky: a reduction met a non-finite value
    int64_t sweep;            // global sweep counter
    int64_t accepted_last;
    int64_t samples;
    int64_t torque_samples;
    double M[3];
    double E_exch, E_uni, E_cub, E_zee;
    double torque[3];
    double shift[5];          // first sample of (m_l, m_x, m_y, m_z, E/N)
    double sum[5];            // sum of (x - shift)
    double sum2[5];           // sum of (x - shift)^2
    double sum_eanis;         // sum of (E_uni + E_cub)/N
    double sum_torque[3];     // sum of torque/N over constrained samples
    double T_sample;
};

// Everything a kernel launcher needs about one lattice.
struct DevLattice {
    int32_t precision;        // 32 or 64
    int32_t nx, ny, nz;
    int32_t hx;               // nx / 2
    int32_t P;                // hx * ny: sites of one colour per plane
    int64_t N;                // nx * ny * nz
    int64_t Nc;               // N / 2: sites per colour
    size_t pitch;             // bytes between the component arrays
    void* spins;              // [colour][component][Nc] of float or double
    DevState* st;
    const void* c1tab;        // 181 reals: 1 - cos(theta) for theta in degrees
    void* aos;                // constrained sweeps: [colour][Nc] 4-vectors of the spins, then [Nc]
                              // records (spin, neighbour sum) of the colour being paired
    double* part;             // [kNumPart][max_blocks]: work-group partials, one row per component
    uint32_t* cnt;            // [2][max_blocks]
    int64_t max_blocks;
    double J, Ku, eu[3], Kc, h[3];
    uint32_t key0, key1, instance;
    int32_t init_mode;        // 0 aligned, 1 uniform random, 2 wall across z
    double init_dir[3];
    double init_width;        // wall width of init_mode 2
    int32_t zbound;           // z boundary: 0 periodic, 1 anti-periodic, 2 open
    uint8_t* mask;            // [colour][Nc] active-bond bits, or null (every bond)
    int32_t prefetch;         // look-ahead of the standard pass: 0 automatic, 1 or 2 planes
};

// The march depth of a lattice: as set, or automatically two for spins
// larger than the last-level cache; always one with bond masks.
inline bool pass_deep(const DevLattice& d)
{
    if (d.mask || d.prefetch == 1) return false;
    return d.prefetch == 2 || (uint64_t)d.N * 3ull * (uint64_t)(d.precision / 8) > kDeepMarchBytes;
}

// Launchers (hmc_kernels.hip).  Each returns the HIP status of the launch;
// *blocks receives the number of work-groups that wrote results.
hipError_t launch_init(const DevLattice& d, hipStream_t s);
// Zeroes the chain state (cone angle theta0) and writes the cone table, 181
// doubles at c1_dev followed by the same 181 values as floats.
hipError_t launch_setup(const DevLattice& d, const double* c1d_host, int theta0, void* c1_dev, hipStream_t s);
// Splits N bytes of bond masks in site order at src (device) into the
// colour-split mask array of the lattice.
hipError_t launch_split_masks(const DevLattice& d, const uint8_t* src, hipStream_t s);
hipError_t launch_pass(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s,
                       int64_t* blocks);
// Steps of a constrained call: copy the spins into the AoS working copy, the
// neighbour sums of colour 0 or 1, the pair pass of colour 0 or 1, copy back.
enum ConstrainedStep { kAosIn = 0, kNbRed, kPairRed, kNbBlack, kPairBlack, kAosOut };
hipError_t launch_constrained(const DevLattice& d, int step, const double eC[3], double T, hipStream_t s,
                              int64_t* blocks);
// The finalize of a constrained sweep (pair records of rec_blocks rows per
// colour, flags fin) together with the colour-0 records of the next sweep.
hipError_t launch_finalize_nbsum(const DevLattice& d, int64_t rec_blocks, int fin, double T, hipStream_t s);
hipError_t launch_measure(const DevLattice& d, hipStream_t s, int64_t* blocks);
// Mean spin of each z plane into out[3*nz] (device memory).
hipError_t launch_plane_means(const DevLattice& d, double* out, hipStream_t s);
// Reduces the counts of the colour-0 (red_blocks) and colour-1 (black_blocks)
// launches and the partials of part_blocks work-groups into the state.
hipError_t launch_finalize(const DevLattice& d, int64_t red_blocks, int64_t black_blocks, int64_t part_blocks,
                           int fin, double T, hipStream_t s);
// Number of work-groups of the standard pass for a launch shape.
int64_t pass_blocks(const DevLattice& d, int spt, int zc);
// Dynamic LDS bytes of the standard pass for a launch shape.
size_t pass_lds_bytes(int precision, int hx, int spt);
// Largest partial count any launch can need.
int64_t max_blocks_for(int32_t nx, int32_t ny, int32_t nz);
// Groups of 1024 records the finalize folds for n work-group records; the
// workspace holds this many group sums after the partial rows.
inline int64_t fold_groups_for(int64_t n) { return (n + 1023) / 1024; }

// Batches.  The table of a batch holds one entry per lattice (kernel
// arguments and launch shape), built on the host by batch_fill_entry.  The
// lattices of one colour-pass launch share a kernel variant: batch_group
// names it (sites per thread and halo slots, 9 classes).
size_t batch_entry_bytes(int precision);
void batch_fill_entry(void* dst, const DevLattice& d, int spt, int zc);
int batch_group(const DevLattice& d, int spt);
// Stores the Boltzmann scale the kernels use for temperature T (float or
// double by precision) at element i of dst (host memory).
void batch_store_scale(int precision, double T, void* dst, size_t i);
constexpr int kBatchGroups = 9;

// One colour-pass launch over the lattices of a group.
struct BatchLaunch {
    int group;                 // kernel variant
    const void* tab;           // device: the batch table
    const uint32_t* start;     // device: n + 1 work-group offsets
    const uint32_t* ent;       // device: n table indices
    uint32_t n;                // lattices in this launch
    uint32_t nblk;             // start[n]
    size_t lds;                // dynamic LDS bytes (largest of the group)
    const void* scale;         // device: per-table-entry scale, float or double
};
hipError_t launch_pass_batch(int precision, const BatchLaunch& b, int colour, bool obs, hipStream_t s);
// Work-group i reduces lattice i's results with flags fin[i] (FinFlags);
// T[i] is its temperature.
hipError_t launch_finalize_batch(int precision, const void* tab, uint32_t count, const double* T,
                                 const int32_t* fin, hipStream_t s);
// Work-group i clears lattice i's accumulators.
hipError_t launch_reset_batch(int precision, const void* tab, uint32_t count, hipStream_t s);

}  // namespace hmc
