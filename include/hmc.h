/*
 * hmc.h -- C interface of the MI355X (gfx950) library for the parallel
 * adaptive Metropolis sweeps of a classical Heisenberg spin lattice
 * (Lepadatu et al., arXiv:2103.03517).
 *
 * The library updates a simple-cubic, periodic (optionally anti-periodic
 * along z) lattice of unit spins
 * with the spin Hamiltonian of Eq. 2 (nearest-neighbour exchange J,
 * uniaxial anisotropy Ku along eu, cubic anisotropy Kc with the Cartesian
 * axes as easy axes for Kc > 0, Zeeman field h), in reduced units: J is
 * the energy unit, k_B = 1 and the moment mu0*mu_S is folded into h.
 *
 * Ownership and threading:
 *   - the caller owns one device workspace of hmc_workspace_bytes() bytes
 *     (for example a torch uint8 tensor) that must outlive the handle;
 *     the library keeps the spins, the cone angle, the sweep counter and
 *     the accumulators there and never allocates device memory itself;
 *   - the library allocates only the small host-side handle, released by
 *     hmc_destroy();
 *   - all work is enqueued on the HIP stream given at hmc_init_lattice();
 *     hmc_sweep() and hmc_constrained_sweep() return without waiting;
 *     hmc_observables(), hmc_copy_spins(), hmc_get_state(),
 *     hmc_set_state() and hmc_read_timing() synchronise that stream;
 *   - one handle must not be used from two threads at once; different
 *     handles are independent.
 *
 * Every function returns an hmc_status (0 on success, negative on error)
 * unless stated otherwise; nothing aborts or throws.  After an error,
 * hmc_last_error() gives a message for the handle involved.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 * (seed low word, seed high word) and counter (sweep, id, tag, instance);
 * tag 0/1 = standard update of a red/black site (id = site id
 * x + nx*(y + ny*z)), 2/3 = constrained pair move of colour 0/1 (id = pair
 * index), 4 = random initial spin (sweep word 0), 5/6 = Feistel keys of
 * the colour-0/1 shuffle (id 0).  Results therefore do not depend on the
 * launch configuration.
 */
#ifndef HMC_H
#define HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMC_OK = 0,
    HMC_EINVAL = -1,    /* a null pointer, a non-finite or out-of-range value */
    HMC_EDIM = -2,      /* lattice dimensions not even, below 2, or too large */
    HMC_ENOMEM = -3,    /* workspace too small or misaligned */
    HMC_EHIP = -4,      /* a HIP runtime call failed */
    HMC_ESTATE = -5,    /* state buffer of the wrong size, for another lattice, or corrupt */
    HMC_ENUMERIC = -6   /* a non-finite value appeared in the reductions */
} hmc_status;

typedef struct hmc_lattice hmc_lattice;

/* Lattice and model parameters (Eq. 2, Sec. 3 of the paper). */
typedef struct {
    int32_t  nx, ny, nz;    /* each even and >= 2 (the red/black colouring of a
                               periodic axis needs an even length, Sec. 2),
                               except nz >= 1 of any parity with an open z
                               boundary; nx <= 1024; nx*ny*nz < 2^32 and
                               nx*ny*nz*precision/16 < 2^32 bytes */
    int32_t  precision;     /* 32: FP32 spins and energy changes, FP64 sums;
                               64: FP64 throughout */
    double   J;             /* exchange (energy unit) */
    double   Ku;            /* uniaxial anisotropy constant */
    double   eu[3];         /* uniaxial easy axis, normalised inside; non-zero */
    double   Kc;            /* cubic anisotropy constant */
    double   h[3];          /* Zeeman field mu0*mu_S*H_a in energy units */
    uint64_t seed;          /* Philox key */
    uint32_t instance;      /* fourth Philox counter word */
    int32_t  init;          /* 0: every spin along init_dir; 1: uniform on the sphere;
                               2: one domain wall across z (for boundary_z = 1): the
                               T = 0 profile S = (sech u, 0, -tanh u), u = pi (z - z0) /
                               init_width, centred between planes nz/2 - 1 and nz/2 */
    double   init_dir[3];   /* non-zero when init == 0 */
    int32_t  theta0_deg;    /* initial cone angle, 1..180 degrees */
    int32_t  boundary_z;    /* 0: periodic along z; 1: anti-periodic along z (the
                               bond between planes nz-1 and 0 couples S_i to -S_j),
                               which holds one domain wall across z (the domain-wall
                               method of Sec. 3); 2: open along z (no bond between
                               planes nz-1 and 0: a film, Sec. 4); x and y stay
                               periodic */
    int32_t  bond_masks;    /* 1: keep a per-site mask of active bonds (set with
                               hmc_set_bond_masks; every bond active until then),
                               1 byte per spin more in the workspace; 0: none */
    double   init_width;    /* wall width of init = 2 (sites, > 0) */
} hmc_params;

/* Observables.  The instantaneous values describe the spins at the time of
 * the call; the averages cover the sampled sweeps since the last
 * hmc_reset_stats().  Index alpha of the 4-arrays: 0 = l (|m|), 1 = x,
 * 2 = y, 3 = z, with m = M/N the spatially averaged moment (Eq. 6). */
typedef struct {
    int64_t n;              /* number of spins N */
    int64_t sweeps_done;    /* global sweep counter */
    int64_t samples;        /* sampled sweeps since the last reset */
    int64_t torque_samples; /* of which constrained sweeps */
    int64_t accepted_last;  /* accepted updates of the last sweep (a pair counts 2) */
    int32_t theta_deg;      /* current cone angle */
    int32_t precision;
    double  M[3];           /* sum_i S_i */
    double  m;              /* |M| / N */
    double  E;              /* total energy, every bond counted once */
    double  E_exch, E_uni, E_cub, E_zee;
    double  torque[3];      /* sum_i S_i x (-dE_anis/dS_i) */
    double  mean_m[4];      /* <m_alpha> */
    double  var_m[4];       /* <m_alpha^2> - <m_alpha>^2 */
    double  mean_E;         /* <E>/N */
    double  var_E;          /* variance of E/N */
    double  mean_Eanis;     /* <E_uni + E_cub>/N */
    double  mean_torque[3]; /* <torque>/N over the constrained samples */
    double  chi[4];         /* N var(m_alpha) / T, Eq. 6 with mu_S = k_B = 1 */
    double  T_sample;       /* temperature of the last sampled sweep */
} hmc_obs;

/* Per-kernel timing collected with HIP events on the handle's stream while
 * timing is enabled.  Kinds: 0 = standard colour pass, 1 = constrained pair
 * pass, 2 = reductions (the per-sweep finalize: cone angle, counters,
 * accumulators, with the parallel fold of the work-group records that comes
 * before it on large lattices; and the measurement of the current spins),
 * 3 = the rest:
 * initialisation, the copies in and out of a constrained call, and its
 * neighbour-sum stencils (between sweeps launched together with the
 * finalize). */
typedef struct {
    int64_t count[4];
    double  total_ms[4];
} hmc_timing;

/* Size in bytes of the device workspace for these parameters, 0 if the
 * parameters are invalid: 44 bytes per spin at FP32 (88 at FP64) -- the
 * spins (12), and the working copies of constrained sweeps: the spins as
 * 4-vectors (16) and, for the colour being paired, a record of each site's
 * spin and neighbour sum (16 per spin) -- plus a few MB of reduction
 * partials. */
size_t hmc_workspace_bytes(const hmc_params* p);

/* Validates p, lays the lattice out in dev_ws (device memory, 256-byte
 * aligned, at least hmc_workspace_bytes(p) bytes, owned by the caller)
 * and enqueues the initial state (init == 0: along init_dir; init == 1:
 * uniform on the sphere from Philox tag 4) on hip_stream (a hipStream_t,
 * NULL for the default stream), without waiting for it (nothing is copied
 * from host memory).  On success *out receives the handle.
 * Errors: HMC_EINVAL, HMC_EDIM, HMC_ENOMEM, HMC_EHIP. */
int hmc_init_lattice(const hmc_params* p, void* dev_ws, size_t ws_bytes,
                     void* hip_stream, hmc_lattice** out);

/* Enqueues n_sweeps (>= 0) iterations of the parallel Metropolis algorithm
 * of Table A1 at temperature T (> 0, finite): a red pass, a black pass
 * (each site: cone move uniform in solid angle within the current cone
 * angle, accepted when P < exp(-dE/T), Eq. 1, with dE from Eq. 2), then
 * the cone angle moves one degree toward an acceptance rate of 1/2.  If
 * sample != 0 every sweep adds m_alpha, E, E_anis to the accumulators
 * (Eq. 6).  Errors: HMC_EINVAL, HMC_EHIP. */
int hmc_sweep(hmc_lattice* L, double T, int32_t n_sweeps, int32_t sample);

/* Enqueues n_sweeps iterations of the parallel constrained algorithm of
 * Table A2 with constraint direction eC (non-zero, normalised inside).  The
 * call works on a site-contiguous copy of the spins in the workspace (made
 * at the start of the call, copied back at its end):
 * M_L = sum_i S_i . eC taken once at the start of each sweep, each colour
 * shuffled by a keyed permutation, consecutive shuffled spins paired, the
 * second spin of a pair compensating the first one's transverse change,
 * and the pair accepted when P < (M_L'/M_L)^2 |S_j.eC / S_j'.eC|
 * exp(-dE/T).  A pair with no real compensating spin, or whose new M_L
 * would not be positive, is rejected.  Sampled sweeps also accumulate the
 * anisotropy torque.  Errors: HMC_EINVAL, HMC_EHIP. */
int hmc_constrained_sweep(hmc_lattice* L, double T, const double eC[3],
                          int32_t n_sweeps, int32_t sample);

/* Measures the current spins and copies counters and accumulators into
 * *out (synchronises).  Returns HMC_ENUMERIC (with *out filled) if a
 * non-finite value was met in any reduction since the lattice was set. */
int hmc_observables(hmc_lattice* L, hmc_obs* out);

/* Clears the accumulators (not the spins, cone angle or sweep counter). */
int hmc_reset_stats(hmc_lattice* L);

/* Bond masks of a lattice created with bond_masks = 1: host_mask holds one
 * byte per site in site order (i = x + nx*(y + ny*z)); bit k set means the
 * bond to neighbour k is active, in the order x-, x+, y-, y+, z-, z+ (bits
 * 6-7 must be clear).  A cut bond carries no exchange: the intergrain bonds
 * of a granular film (Sec. 4).  Each bond must be cut or kept at both ends
 * (checked; bonds across an open z boundary are not checked, they do not
 * exist).  The masks are configuration, not chain state: state images do
 * not carry them.  Synchronises.  Errors: HMC_EINVAL (no masks, asymmetric
 * or out-of-range bits), HMC_ENOMEM, HMC_EHIP. */
int hmc_set_bond_masks(hmc_lattice* L, const uint8_t* host_mask);

/* As hmc_set_bond_masks, without waiting: the masks are copied from
 * host_mask on the lattice's stream, so host_mask must stay valid and
 * unchanged until the stream has passed the call (pinned host memory keeps
 * the copy asynchronous).  check != 0 runs the symmetry check first (on the
 * host, before anything is enqueued); check == 0 skips it, for masks already
 * checked (the same masks given to another lattice of the same shape).
 * Errors: HMC_EINVAL, HMC_EHIP. */
int hmc_set_bond_masks_async(hmc_lattice* L, const uint8_t* host_mask, int32_t check);

/* Mean spin of every z plane (a slice of nx*ny sites, both colours) of the
 * current spins: host_out receives 3*nz doubles, plane z at 3z .. 3z+2.  The
 * magnetisation profile across a wall held by the anti-periodic boundary
 * (Sec. 3, Eq. 5).  Synchronises.  Errors: HMC_EINVAL, HMC_EHIP. */
int hmc_plane_means(hmc_lattice* L, double* host_out);

/* Copies the spins between the device and host_xyz, an array of 3*N
 * doubles in AoS order S[3*i + a] with site id i = x + nx*(y + ny*z).
 * to_host != 0: device -> host; else host -> device, each vector divided by
 * its length (zero or non-finite vectors are stored as given; FP32 lattices
 * round to nearest).  Synchronises. */
int hmc_copy_spins(hmc_lattice* L, double* host_xyz, int32_t to_host);

/* Checkpoint: hmc_state_bytes() gives the size of a state image (spins,
 * cone angle, sweep counter, accumulators and the parameters it belongs
 * to); get/set copy it to/from host memory.  Because the random numbers
 * are counter-based, a restored lattice continues bit for bit.
 * hmc_set_state returns HMC_ESTATE for an image of another lattice, and for
 * one whose chain state is out of range (a cone angle outside [1, 180],
 * negative counters, more torque samples than samples, an acceptance count
 * above N); the lattice is then left as it was. */
size_t hmc_state_bytes(const hmc_lattice* L);
int hmc_get_state(hmc_lattice* L, void* host_buf, size_t bytes);
int hmc_set_state(hmc_lattice* L, const void* host_buf, size_t bytes);

/* Launch shape of the standard pass: each work-group of 256 threads
 * covers 256*sites_per_thread in-plane sites of one colour and marches
 * over z_chunk planes.  sites_per_thread in {1, 2, 4}; z_chunk in
 * [1, 1024].  The spins produced do not depend on the shape (random
 * numbers are keyed by site); reduction orders, and so the last bits of
 * the observables, do.  Default: 2 sites per thread (1 where the LDS
 * window of 512 sites would not fit) and z_chunk 16; lattices whose spins
 * exceed 256 MiB (the march that loads two planes ahead) take 8 at FP32
 * and 32 at FP64.
 * Errors: HMC_EINVAL. */
int hmc_set_launch(hmc_lattice* L, int32_t sites_per_thread, int32_t z_chunk);
int hmc_get_launch(const hmc_lattice* L, int32_t* sites_per_thread, int32_t* z_chunk);

/* Look-ahead of the standard pass's march over z: depth 1 issues the loads
 * of the planes one step ahead of their use, depth 2 two steps ahead (more
 * loads in flight, for lattices that stream from HBM); 0 (the default)
 * takes 2 when the spins exceed 256 MiB (the last-level cache) and 1
 * otherwise.  Lattices with bond masks always use depth 1, and so does a
 * batch sweep (its chunks are sized to the cache).  The spins do not
 * depend on the depth.  hmc_get_prefetch gives the depth hmc_sweep uses.
 * Errors: HMC_EINVAL (depth outside 0..2, or 2 with bond masks). */
int hmc_set_prefetch(hmc_lattice* L, int32_t depth);
int hmc_get_prefetch(const hmc_lattice* L, int32_t* depth);

/* Per-kernel timing (see hmc_timing).  Enabling resets the totals;
 * hmc_read_timing synchronises and returns the totals so far. */
int hmc_set_timing(hmc_lattice* L, int32_t enable);
int hmc_read_timing(hmc_lattice* L, hmc_timing* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * measurement that hmc_observables makes of a lattice's current spins (M,
 * m = |M|/N, the energy terms of Eq. 2 with every bond once, the anisotropy
 * torque), on spins held by the caller and without a lattice handle or a
 * workspace.  The reduction scratch (per-work-group partials and the reduced
 * values) lives in a static device array of the library: 6.51 MiB per GPU,
 * held from the first call on that GPU until the process ends.
 *   p:         the lattice's parameters (validated as by hmc_init_lattice;
 *              bond_masks must be 0);
 *   dev_spins: device memory (256-byte aligned, at least spins_bytes bytes,
 *              owned by the caller, only read) holding the spins in the
 *              layout of a lattice workspace: six component arrays (colour 0
 *              x, y, z, then colour 1 x, y, z) of N/2 reals each, one every
 *              pitch = N/2 * precision/8 bytes rounded up to a multiple of
 *              256 -- the first 6*pitch bytes of a workspace laid out by
 *              hmc_init_lattice for p;
 *   out:       receives n, precision, M, m, E and its terms and torque; the
 *              counters and averages are 0 (there is no chain).
 * Work goes to hip_stream on the current device (which must be the stream's),
 * and the call synchronises it.  N above 2^25 spins: HMC_EDIM.  Calls on one
 * GPU share its scratch array: calls that overlap on one GPU (from two host
 * threads, or on two streams) race and must be serialised by the caller.
 * Errors: HMC_EINVAL, HMC_EDIM, HMC_ENOMEM (spins_bytes below 6*pitch, or
 * misaligned), HMC_EHIP, HMC_ENUMERIC (out filled). */
int hmc_measure_static(const hmc_params* p, const void* dev_spins, size_t spins_bytes, void* hip_stream,
                       hmc_obs* out);

/* Asynchronous reads, for loops that keep the device busy while the host
 * admits and retires work (continuous batching).  A snapshot is the chain
 * state of a lattice -- counters and the accumulators of Eq. 6 -- as the
 * stream reaches the call: hmc_snapshot_enqueue enqueues, for lattice i of
 * lattices[0 .. count-1] (all on one stream), a copy of its state into
 * host_dst + i * hmc_snapshot_bytes() and returns at once.  host_dst should
 * be pinned host memory (hipHostMalloc, or a pinned torch tensor) so that the
 * copies do not block; it is valid once the stream has passed the call (an
 * event recorded after it has completed).  hmc_snapshot_observables fills
 * *out from one such record of a lattice of n spins and the given precision,
 * as hmc_observables would from the accumulators (the instantaneous fields
 * are those of the last sampled or constrained sweep, not a fresh
 * measurement); it returns HMC_ENUMERIC, with *out filled, if the record
 * carries the non-finite flag.  Errors: HMC_EINVAL, HMC_EHIP. */
size_t hmc_snapshot_bytes(void);
int hmc_snapshot_enqueue(hmc_lattice* const* lattices, int32_t count, void* host_dst);
int hmc_snapshot_observables(const void* record, int64_t n, int32_t precision, hmc_obs* out);

/* As hmc_plane_means, into 3*nz doubles of device memory at dev_out (owned
 * by the caller), enqueued on the lattice's stream without waiting. */
int hmc_plane_means_async(hmc_lattice* L, double* dev_out);

/* Releases the handle.  Work already enqueued for the lattice is not
 * waited for (launches copy their arguments); the workspace must stay valid
 * until that work has run. */
void hmc_destroy(hmc_lattice* L);
const char* hmc_strerror(int status);
const char* hmc_last_error(const hmc_lattice* L);

/* ------------------------------------------------------------------------
 * Batches: many independent lattices (the separate runs at many
 * temperatures and sizes that Sec. 3 sweeps over, e.g. for m(T)) advanced
 * together.  A batch sweep issues one launch per colour pass for every
 * group of lattices that share a kernel variant (sites per thread and
 * halo width: at most 9 groups, usually one or two), and one finalize
 * launch in which work-group i folds lattice i's counts and sums.  Each
 * lattice keeps its own spins, cone angle, sweep counter and
 * accumulators, and each of its tiles runs exactly as in hmc_sweep, so
 * with the same launch shape a lattice in a batch ends bit for bit where
 * it would alone (random numbers are keyed by the lattice's own seed and
 * instance, not by its place in the batch).
 *
 * Ownership: the caller owns the lattices, which must outlive the batch,
 * and a device workspace of hmc_batch_workspace_bytes(count) bytes
 * (256-byte aligned) that holds the batch table and the per-lattice
 * temperatures.  The library allocates the host handle, a small pinned
 * staging buffer for the table uploads and, for graph replays, one
 * capture stream; hmc_batch_destroy releases them.  All work goes to the
 * stream of the lattices, which must be the same for all of them.
 * ------------------------------------------------------------------------ */
typedef struct hmc_batch hmc_batch;

/* Device workspace for a batch of count (1 .. 65536) lattices; 0 if count
 * is out of range.  About 0.4 KB per lattice. */
size_t hmc_batch_workspace_bytes(int32_t count);

/* Builds a batch over lattices[0 .. count-1] (distinct handles, one
 * precision, one stream).  The launch shape of each lattice is the one set
 * by hmc_set_launch (a later change is picked up by the next batch call).
 * Lattices with bond masks are not accepted (they are swept alone).
 * Errors: HMC_EINVAL (null, duplicate, mixed precision or stream, bond
 * masks), HMC_ENOMEM (workspace too small or misaligned), HMC_EHIP. */
int hmc_batch_create(hmc_lattice* const* lattices, int32_t count, void* dev_ws, size_t ws_bytes,
                     hmc_batch** out);

/* Replaces the lattices of a batch with lattices[0 .. count-1] (same rules
 * as hmc_batch_create), reusing its workspace, staging buffer and stream:
 * count may be at most the capacity of the workspace given at creation
 * (the largest n with hmc_batch_workspace_bytes(n) <= ws_bytes).  The new
 * table is uploaded on the stream; graphs are captured again when next
 * needed.  Errors: HMC_EINVAL, HMC_ENOMEM (above the capacity), HMC_EHIP. */
int hmc_batch_set_lattices(hmc_batch* B, hmc_lattice* const* lattices, int32_t count);

/* Enqueues n_sweeps standard sweeps (Table A1) of every lattice of the
 * batch, lattice i at temperature T[i] (count values, each > 0 and
 * finite); sample as in hmc_sweep.  Observables are read per lattice with
 * hmc_observables.  Errors: HMC_EINVAL, HMC_EHIP. */
int hmc_batch_sweep(hmc_batch* B, const double* T, int32_t n_sweeps, int32_t sample);

/* As hmc_batch_sweep, with a sample flag per lattice (sample[i] != 0:
 * lattice i accumulates), so that lattices in different phases of their
 * runs (equilibration, sampling) advance together.  The black pass computes
 * the fused sums whenever any lattice samples.  Errors: HMC_EINVAL,
 * HMC_EHIP. */
int hmc_batch_sweep_each(hmc_batch* B, const double* T, const int32_t* sample, int32_t n_sweeps);

/* Observables of every lattice: out[i] receives what hmc_observables
 * gives for lattice i (the current spins are measured).  Synchronises the
 * stream once.  Returns the first error of any lattice (HMC_ENUMERIC with
 * all of out filled). */
int hmc_batch_observables(hmc_batch* B, hmc_obs* out);

/* Clears the accumulators of every lattice, as hmc_reset_stats does, with
 * one kernel on the stream and without synchronising. */
int hmc_batch_reset_stats(hmc_batch* B);

/* Autotuner.  Every configuration is timed as a sweep call runs it (chunk
 * after chunk, max(trial_sweeps, 20) sweeps each, at temperatures T).  It
 * picks the chunk size among 0 (one chunk), 96, 128, 160, 192, 224 and
 * 256 MiB; then, for each distinct lattice size in turn (largest total
 * first), the fastest admissible launch shape (sites_per_thread 1, 2, 4
 * within the LDS budget; z_chunk 2 .. 64, powers of two up to nz) with the
 * other sizes held; then the chunk size again.  trial_sweeps: 1 .. 1000.
 * The shapes are set on the lattices (hmc_get_launch reads them), the
 * chunk size on the batch (hmc_batch_get_chunk_bytes).  Every lattice's state is saved before and
 * restored after (host copies), so tuning leaves the chains where they
 * were.  Synchronises.  Errors: HMC_EINVAL, HMC_EHIP, HMC_ENOMEM (host). */
int hmc_batch_tune(hmc_batch* B, const double* T, int32_t trial_sweeps);

/* Chunking: a batch sweep call splits the lattices (in order) into
 * ceil(total / bytes) chunks of about equal bytes of spins and finishes all
 * its sweeps on one chunk before the next, so that a chunk stays in the
 * 256 MB Infinity Cache while it is swept.  Each lattice still runs red
 * pass, black pass and finalize for every sweep in order, so its results do
 * not depend on the chunking.  bytes = 0 (the default): one chunk.
 * hmc_batch_tune chooses it.  Errors: HMC_EINVAL (negative), HMC_EHIP. */
int hmc_batch_set_chunk_bytes(hmc_batch* B, int64_t bytes);
int hmc_batch_get_chunk_bytes(const hmc_batch* B, int64_t* bytes);

/* Graph replay: with sweeps_per_graph > 0, runs of that many sweeps are
 * captured once (per chunk and sample flag) as a HIP graph on a private stream and
 * replayed on the lattices' stream, which removes the per-launch host
 * cost; sweeps_per_graph = 0 (the default) launches eagerly.  Replays do
 * exactly the work of the eager launches.  Timing (below) uses eager
 * launches.  Errors: HMC_EINVAL (negative or above 4096). */
int hmc_batch_set_graph(hmc_batch* B, int32_t sweeps_per_graph);

/* Per-launch timing of batch sweeps, kinds as in hmc_timing (0: colour
 * passes, 2: finalize). */
int hmc_batch_set_timing(hmc_batch* B, int32_t enable);
int hmc_batch_read_timing(hmc_batch* B, hmc_timing* out);

/* Waits for the stream and releases the handle (not the lattices). */
void hmc_batch_destroy(hmc_batch* B);
const char* hmc_batch_last_error(const hmc_batch* B);

#ifdef __cplusplus
}
#endif
#endif
