// hmc_api.cpp -- the C interface declared in include/hmc.h: parameter
// validation, workspace layout, the per-sweep launch sequence, host<->device
// copies, checkpoints and event timing.  All arithmetic of the method runs in
// the kernels of hmc_kernels.hip.
#include "hmc.h"

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "hmc_handle.h"
#include "hmc_internal.h"

using hmc::DevLattice;
using hmc::DevState;
using hmc::Layout;

// ---------------------------------------------------------------------------
// Launch-event timer
// ---------------------------------------------------------------------------
namespace hmc {

hipError_t Timer::flush(hipStream_t s)
{
    if (used == 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < used; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
        if (e != hipSuccess) return e;
        tot.count[kind[i]] += 1;
        tot.total_ms[kind[i]] += ms;
    }
    used = 0;
    return hipSuccess;
}

hipError_t Timer::enable(hipStream_t s, bool enable_)
{
    if (on) {
        hipError_t e = flush(s);
        if (e != hipSuccess) return e;
    }
    on = enable_;
    tot = hmc_timing{};
    while (on && ev.size() < 2 * kMaxEvents) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
    }
    kind.resize(kMaxEvents);
    return hipSuccess;
}

hipError_t Timer::begin(hipStream_t s)
{
    if (used == kMaxEvents) {
        hipError_t e = flush(s);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(ev[2 * used], s);
}

hipError_t Timer::end(hipStream_t s, int k)
{
    hipError_t e = hipEventRecord(ev[2 * used + 1], s);
    if (e != hipSuccess) return e;
    kind[used] = k;
    used += 1;
    return hipSuccess;
}

void Timer::destroy()
{
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    used = 0;
    on = false;
}

}  // namespace hmc

namespace {

constexpr uint32_t kStateMagic = 0x484D4331u;  // "HMC1"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool finite3(const double v[3]) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }
bool nonzero3(const double v[3]) { return v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0; }

int validate(const hmc_params* p, char* msg, size_t n)
{
    if (!p) { snprintf(msg, n, "null parameter block"); return HMC_EINVAL; }
    const int32_t d[3] = {p->nx, p->ny, p->nz};
    // x and y are periodic and must be even for the red/black colouring; z
    // too unless it is open, where any nz >= 1 is allowed
    const bool open_z = p->boundary_z == 2;
    for (int i = 0; i < 3; ++i) {
        const bool free_axis = i == 2 && open_z;
        if (free_axis ? d[i] < 1 : (d[i] < 2 || (d[i] & 1))) {
            snprintf(msg, n, "lattice dimensions must be even and >= 2 (nz >= 1 with an open z boundary; "
                             "got %d x %d x %d)", p->nx, p->ny, p->nz);
            return HMC_EDIM;
        }
    }
    if (p->nx > 1024) { snprintf(msg, n, "nx must be <= 1024 (got %d)", p->nx); return HMC_EDIM; }
    const uint64_t N = (uint64_t)p->nx * (uint64_t)p->ny * (uint64_t)p->nz;
    if (N >= (1ull << 32)) { snprintf(msg, n, "nx*ny*nz must be < 2^32"); return HMC_EDIM; }
    if (p->precision != 32 && p->precision != 64) {
        snprintf(msg, n, "precision must be 32 or 64 (got %d)", p->precision);
        return HMC_EINVAL;
    }
    // each component array is addressed by 32-bit byte offsets
    if (N / 2 * (uint64_t)(p->precision / 8) > 0xFFFFFFFFull) {
        snprintf(msg, n, "lattice too large: one component array must stay below 4 GiB");
        return HMC_EDIM;
    }
    if (!isfinite(p->J) || !isfinite(p->Ku) || !isfinite(p->Kc) || !finite3(p->eu) || !finite3(p->h)) {
        snprintf(msg, n, "model constants must be finite");
        return HMC_EINVAL;
    }
    if (!nonzero3(p->eu)) { snprintf(msg, n, "uniaxial axis eu must be non-zero"); return HMC_EINVAL; }
    if (p->init < 0 || p->init > 2) { snprintf(msg, n, "init must be 0, 1 or 2"); return HMC_EINVAL; }
    if (p->init == 2 && !(p->init_width > 0.0 && isfinite(p->init_width))) {
        snprintf(msg, n, "init = 2 needs a positive, finite init_width");
        return HMC_EINVAL;
    }
    if (p->init == 0 && (!finite3(p->init_dir) || !nonzero3(p->init_dir))) {
        snprintf(msg, n, "init_dir must be finite and non-zero");
        return HMC_EINVAL;
    }
    if (p->theta0_deg < 1 || p->theta0_deg > 180) {
        snprintf(msg, n, "theta0_deg must be in [1, 180] (got %d)", p->theta0_deg);
        return HMC_EINVAL;
    }
    if (p->boundary_z < 0 || p->boundary_z > 2) {
        snprintf(msg, n, "boundary_z must be 0 (periodic), 1 (anti-periodic) or 2 (open)");
        return HMC_EINVAL;
    }
    if (p->bond_masks != 0 && p->bond_masks != 1) {
        snprintf(msg, n, "bond_masks must be 0 or 1");
        return HMC_EINVAL;
    }
    return HMC_OK;
}

Layout layout_for(const hmc_params* p)
{
    Layout L{};
    const uint64_t Nc = (uint64_t)p->nx * p->ny * p->nz / 2;
    const size_t rs = p->precision / 8;
    L.pitch = align_up(Nc * rs, hmc::kAlign);
    size_t off = 6 * L.pitch;
    // constrained sweeps: an AoS copy of both colours (4 reals per site),
    // then the records (spin, neighbour sum: 8 reals) of one colour
    L.off_aos = off;
    off += align_up(2 * Nc * 4 * rs + Nc * 8 * rs, hmc::kAlign);
    L.off_state = off;
    off += align_up(sizeof(DevState), hmc::kAlign);
    L.off_c1 = off;
    off += align_up(181 * sizeof(double) + 181 * sizeof(float), hmc::kAlign);
    L.max_blocks = hmc::max_blocks_for(p->nx, p->ny, p->nz);
    L.off_part = off;
    // kNumPart rows of max_blocks partials, then the group sums of the fold
    off += align_up(((size_t)L.max_blocks + (size_t)hmc::fold_groups_for(L.max_blocks)) * hmc::kNumPart *
                        sizeof(double), hmc::kAlign);
    L.off_cnt = off;
    off += align_up((size_t)L.max_blocks * 2 * sizeof(uint32_t), hmc::kAlign);
    L.off_mask = off;
    if (p->bond_masks) off += align_up(2 * Nc, hmc::kAlign);
    L.total = off;
    return L;
}

}  // namespace

namespace hmc {

int check_params(const hmc_params* p, char* msg, size_t n) { return validate(p, msg, n); }

size_t spin_pitch(const hmc_params* p) { return layout_for(p).pitch; }

}  // namespace hmc

namespace {

struct StateHeader {
    uint32_t magic, precision;
    int32_t nx, ny, nz, boundary_z;
    uint64_t seed;
    uint32_t instance, bond_masks;
    double J, Ku, eu[3], Kc, h[3];
};

}  // namespace

namespace {

int fail(hmc_lattice* L, int status, const char* what, hipError_t e = hipSuccess)
{
    if (L) {
        if (e != hipSuccess) snprintf(L->err, sizeof(L->err), "%s: %s", what, hipGetErrorString(e));
        else snprintf(L->err, sizeof(L->err), "%s", what);
    }
    return status;
}

// Runs one launch, bracketed by events on the lattice's stream when timing.
template <class F>
int launch(hmc_lattice* L, int kind, const char* what, F f)
{
    if (L->timer.on) {
        hipError_t r = L->timer.begin(L->stream);
        if (r != hipSuccess) return fail(L, HMC_EHIP, "timing event", r);
    }
    hipError_t e = f();
    if (e != hipSuccess) return fail(L, HMC_EHIP, what, e);
    if (L->timer.on) {
        hipError_t r = L->timer.end(L->stream, kind);
        if (r != hipSuccess) return fail(L, HMC_EHIP, "timing event", r);
    }
    return HMC_OK;
}

int measure(hmc_lattice* L)
{
    int64_t nb = 0;
    int st = launch(L, 2, "measure kernel", [&] { return hmc::launch_measure(L->d, L->stream, &nb); });
    if (st == HMC_OK)
        st = launch(L, 2, "finalize kernel", [&] {
            return hmc::launch_finalize(L->d, 0, 0, nb, hmc::kFinObs | hmc::kFinTorque, 0.0, L->stream);
        });
    if (st == HMC_OK) L->m_valid = true;
    return st;
}

}  // namespace

extern "C" {

size_t hmc_workspace_bytes(const hmc_params* p)
{
    char msg[128];
    if (validate(p, msg, sizeof(msg)) != HMC_OK) return 0;
    return layout_for(p).total;
}

int hmc_init_lattice(const hmc_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, hmc_lattice** out)
{
    if (!out) return HMC_EINVAL;
    *out = nullptr;
    char msg[256];
    int st = validate(p, msg, sizeof(msg));
    if (st != HMC_OK) return st;
    const Layout lay = layout_for(p);
    if (!dev_ws || ws_bytes < lay.total || ((uintptr_t)dev_ws % hmc::kAlign) != 0) return HMC_ENOMEM;

    hmc_lattice* L = new (std::nothrow) hmc_lattice();
    if (!L) return HMC_ENOMEM;
    L->p = *p;
    L->stream = static_cast<hipStream_t>(hip_stream);
    L->lay = lay;
    const double eun = sqrt(p->eu[0] * p->eu[0] + p->eu[1] * p->eu[1] + p->eu[2] * p->eu[2]);
    for (int a = 0; a < 3; ++a) L->p.eu[a] = p->eu[a] / eun;
    if (p->init == 0) {
        const double dn = sqrt(p->init_dir[0] * p->init_dir[0] + p->init_dir[1] * p->init_dir[1] +
                               p->init_dir[2] * p->init_dir[2]);
        for (int a = 0; a < 3; ++a) L->p.init_dir[a] = p->init_dir[a] / dn;
    }

    DevLattice& d = L->d;
    char* base = static_cast<char*>(dev_ws);
    d.precision = p->precision;
    d.nx = p->nx;
    d.ny = p->ny;
    d.nz = p->nz;
    d.hx = p->nx / 2;
    d.P = d.hx * p->ny;
    d.N = (int64_t)p->nx * p->ny * p->nz;
    d.Nc = d.N / 2;
    d.pitch = lay.pitch;
    d.spins = base;
    d.aos = base + lay.off_aos;
    d.st = reinterpret_cast<DevState*>(base + lay.off_state);
    d.c1tab = p->precision == 64 ? static_cast<const void*>(base + lay.off_c1)
                                 : static_cast<const void*>(base + lay.off_c1 + 181 * sizeof(double));
    d.part = reinterpret_cast<double*>(base + lay.off_part);
    d.cnt = reinterpret_cast<uint32_t*>(base + lay.off_cnt);
    d.max_blocks = lay.max_blocks;
    d.J = p->J;
    d.Ku = p->Ku;
    d.Kc = p->Kc;
    for (int a = 0; a < 3; ++a) {
        d.eu[a] = L->p.eu[a];
        d.h[a] = p->h[a];
        d.init_dir[a] = L->p.init_dir[a];
    }
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.instance = p->instance;
    d.init_mode = p->init;
    d.init_width = p->init_width;
    d.zbound = p->boundary_z;
    d.mask = p->bond_masks ? reinterpret_cast<uint8_t*>(base + lay.off_mask) : nullptr;
    d.prefetch = 0;

    // 1 - cos(theta) = 2 sin^2(theta/2) for theta = 0..180 degrees
    for (int th = 0; th <= 180; ++th) {
        const double s = sin((double)th * M_PI / 360.0);
        L->c1d[th] = 2.0 * s * s;
        L->c1f[th] = (float)L->c1d[th];
    }
    // default launch shape: 512 in-plane sites per work-group, narrowed to
    // 256 sites when the LDS window would exceed its budget; 16 planes while
    // the spins fit the last-level cache.  Spins that stream from HBM (the
    // depth-two march) take 8 planes at FP32: shorter slabs give more
    // work-groups to spread over the chip (measured on MI355X at 384^3 and
    // 464^3 FP32: 2.9 % and 1.9 % faster passes), and the finalize folds the
    // extra records in parallel.  At FP64 they take 32: fewer slab ends to
    // re-read (measured on MI355X: 256^3 63.9-64.3 against 62.8-63.0 G
    // updates/s with 16 planes and 60.4 with 8; 384^3 61.0-61.4 against
    // 60.3-60.7).
    if (hmc::pass_lds_bytes(p->precision, d.hx, L->spt) > hmc::kMaxLds) L->spt = 1;
    if (hmc::pass_deep(d)) L->zc = p->precision == 32 ? 8 : 32;
    memset(&L->init_state, 0, sizeof(L->init_state));
    L->init_state.theta = p->theta0_deg;

    // nothing is copied from host memory and nothing waits: the chain state
    // and the cone table are written by a kernel from its arguments
    hipError_t e = hmc::launch_setup(L->d, L->c1d, p->theta0_deg, base + lay.off_c1, L->stream);
    // every bond active until hmc_set_bond_masks says otherwise
    if (e == hipSuccess && d.mask) e = hipMemsetAsync(d.mask, 0x3F, 2 * (size_t)d.Nc, L->stream);
    if (e != hipSuccess) { delete L; return HMC_EHIP; }
    st = launch(L, 3, "init kernel", [&] { return hmc::launch_init(L->d, L->stream); });
    if (st == HMC_OK) st = measure(L);
    if (st != HMC_OK) { delete L; return st; }
    *out = L;
    return HMC_OK;
}

int hmc_sweep(hmc_lattice* L, double T, int32_t n_sweeps, int32_t sample)
{
    if (!L) return HMC_EINVAL;
    if (!(T > 0.0) || !isfinite(T)) return fail(L, HMC_EINVAL, "temperature must be positive and finite");
    if (n_sweeps < 0) return fail(L, HMC_EINVAL, "n_sweeps must be >= 0");
    const bool obs = sample != 0;
    for (int32_t it = 0; it < n_sweeps; ++it) {
        int64_t nr = 0, nb = 0;
        int st = launch(L, 0, "red pass", [&] {
            return hmc::launch_pass(L->d, 0, false, L->spt, L->zc, T, L->stream, &nr);
        });
        if (st == HMC_OK)
            st = launch(L, 0, "black pass", [&] {
                return hmc::launch_pass(L->d, 1, obs, L->spt, L->zc, T, L->stream, &nb);
            });
        if (st == HMC_OK)
            st = launch(L, 2, "finalize kernel", [&] {
                const int fin = hmc::kFinCounts | (obs ? (hmc::kFinObs | hmc::kFinSample) : 0);
                return hmc::launch_finalize(L->d, nr, nb, obs ? nb : 0, fin, T, L->stream);
            });
        if (st != HMC_OK) return st;
        L->m_valid = obs;
    }
    return HMC_OK;
}

int hmc_constrained_sweep(hmc_lattice* L, double T, const double eC[3], int32_t n_sweeps, int32_t sample)
{
    if (!L) return HMC_EINVAL;
    if (!(T > 0.0) || !isfinite(T)) return fail(L, HMC_EINVAL, "temperature must be positive and finite");
    if (!eC || !finite3(eC) || !nonzero3(eC)) return fail(L, HMC_EINVAL, "eC must be finite and non-zero");
    if (n_sweeps < 0) return fail(L, HMC_EINVAL, "n_sweeps must be >= 0");
    const double n = sqrt(eC[0] * eC[0] + eC[1] * eC[1] + eC[2] * eC[2]);
    const double e[3] = {eC[0] / n, eC[1] / n, eC[2] / n};
    if (n_sweeps == 0) return HMC_OK;
    if (!L->m_valid) {
        int st = measure(L);
        if (st != HMC_OK) return st;
    }
    using hmc::launch_constrained;
    int64_t nb = 0;
    auto step = [&](int kind, int which, const char* what) {
        return launch(L, kind, what, [&] { return launch_constrained(L->d, which, e, T, L->stream, &nb); });
    };
    int st = step(3, hmc::kAosIn, "copy to the AoS working copy");
    if (st == HMC_OK) st = step(3, hmc::kNbRed, "red neighbour sums");
    const int fin = hmc::kFinCounts | hmc::kFinObs | hmc::kFinTorque | (sample ? hmc::kFinSample : 0);
    for (int32_t it = 0; it < n_sweeps && st == HMC_OK; ++it) {
        st = step(1, hmc::kPairRed, "red pair pass");
        if (st == HMC_OK) st = step(3, hmc::kNbBlack, "black neighbour sums");
        if (st == HMC_OK) st = step(1, hmc::kPairBlack, "black pair pass");
        // the finalize; before another sweep, in one launch with that
        // sweep's red neighbour sums
        if (st == HMC_OK && it + 1 < n_sweeps)
            st = launch(L, 3, "finalize and red neighbour sums", [&] {
                return hmc::launch_finalize_nbsum(L->d, nb, fin, T, L->stream);
            });
        else if (st == HMC_OK)
            st = launch(L, 2, "finalize kernel", [&] {
                return hmc::launch_finalize(L->d, nb, nb, 2 * nb, fin, T, L->stream);
            });
    }
    if (st == HMC_OK) st = step(3, hmc::kAosOut, "copy back from the AoS working copy");
    if (st == HMC_OK) L->m_valid = true;
    return st;
}

}  // extern "C"

namespace hmc {

int enqueue_observables(hmc_lattice* L, DevState* host_dst)
{
    int st = measure(L);
    if (st != HMC_OK) return st;
    hipError_t e = hipMemcpyAsync(host_dst, L->d.st, sizeof(DevState), hipMemcpyDeviceToHost, L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "reading the device state", e);
    return HMC_OK;
}

int finish_observables(hmc_lattice* L, const DevState& s, hmc_obs* out)
{
    memset(out, 0, sizeof(*out));
    const double N = (double)L->d.N;
    out->n = L->d.N;
    out->sweeps_done = s.sweep;
    out->samples = s.samples;
    out->torque_samples = s.torque_samples;
    out->accepted_last = s.accepted_last;
    out->theta_deg = s.theta;
    out->precision = L->d.precision;
    for (int a = 0; a < 3; ++a) {
        out->M[a] = s.M[a];
        out->torque[a] = s.torque[a];
    }
    out->m = sqrt(s.M[0] * s.M[0] + s.M[1] * s.M[1] + s.M[2] * s.M[2]) / N;
    out->E_exch = s.E_exch;
    out->E_uni = s.E_uni;
    out->E_cub = s.E_cub;
    out->E_zee = s.E_zee;
    out->E = s.E_exch + s.E_uni + s.E_cub + s.E_zee;
    out->T_sample = s.T_sample;
    if (s.samples > 0) {
        const double ns = (double)s.samples;
        for (int i = 0; i < 4; ++i) {
            const double mu = s.sum[i] / ns;
            out->mean_m[i] = s.shift[i] + mu;
            out->var_m[i] = s.sum2[i] / ns - mu * mu;
            out->chi[i] = s.T_sample > 0.0 ? N * out->var_m[i] / s.T_sample : 0.0;
        }
        const double mu = s.sum[4] / ns;
        out->mean_E = s.shift[4] + mu;
        out->var_E = s.sum2[4] / ns - mu * mu;
        out->mean_Eanis = s.sum_eanis / ns;
    }
    if (s.torque_samples > 0)
        for (int a = 0; a < 3; ++a) out->mean_torque[a] = s.sum_torque[a] / (double)s.torque_samples;
    if (s.nonfinite) return fail(L, HMC_ENUMERIC, "a non-finite value appeared in the reductions");
    return HMC_OK;
}

}  // namespace hmc

extern "C" {

int hmc_observables(hmc_lattice* L, hmc_obs* out)
{
    if (!L || !out) return HMC_EINVAL;
    DevState s;
    int st = hmc::enqueue_observables(L, &s);
    if (st != HMC_OK) return st;
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "reading the device state", e);
    return hmc::finish_observables(L, s, out);
}

int hmc_reset_stats(hmc_lattice* L)
{
    if (!L) return HMC_EINVAL;
    DevState s;
    hipError_t e = hipMemcpyAsync(&s, L->d.st, sizeof(s), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "reading the device state", e);
    s.samples = 0;
    s.torque_samples = 0;
    for (int i = 0; i < 5; ++i) s.shift[i] = s.sum[i] = s.sum2[i] = 0.0;
    s.sum_eanis = 0.0;
    for (int a = 0; a < 3; ++a) s.sum_torque[a] = 0.0;
    s.T_sample = 0.0;
    L->init_state = s;
    e = hipMemcpyAsync(L->d.st, &L->init_state, sizeof(s), hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "writing the device state", e);
    return HMC_OK;
}

}  // extern "C"

namespace {

// A bond must be active or cut at both of its ends (bit k of a site and the
// opposite bit of its neighbour k); bonds across an open z boundary do not
// exist and are not checked.  Row by row, without divisions.
int check_bond_masks(hmc_lattice* L, const uint8_t* host_mask)
{
    const DevLattice& d = L->d;
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz, plane = nx * ny;
    for (int64_t z = 0; z < nz; ++z) {
        const bool zcut = d.zbound == 2 && z == nz - 1;
        const int64_t zn = z + 1 == nz ? 0 : z + 1;
        for (int64_t y = 0; y < ny; ++y) {
            const int64_t yn = y + 1 == ny ? 0 : y + 1;
            const uint8_t* row = host_mask + nx * (y + ny * z);
            const uint8_t* rowy = host_mask + nx * (yn + ny * z);
            const uint8_t* rowz = host_mask + nx * y + plane * zn;
            for (int64_t x = 0; x < nx; ++x) {
                const uint8_t m = row[x];
                const uint8_t mx = row[x + 1 == nx ? 0 : x + 1];
                if ((m & 0xC0u) || ((m >> 1) & 1u) != (mx & 1u) || ((m >> 3) & 1u) != ((rowy[x] >> 2) & 1u) ||
                    (!zcut && ((m >> 5) & 1u) != ((rowz[x] >> 4) & 1u))) {
                    char msg[160];
                    if (m & 0xC0u) snprintf(msg, sizeof(msg), "bond masks use bits 0..5 only");
                    else
                        snprintf(msg, sizeof(msg), "bond masks are not symmetric at site (%lld, %lld, %lld)",
                                 (long long)x, (long long)y, (long long)z);
                    return fail(L, HMC_EINVAL, msg);
                }
            }
        }
    }
    return HMC_OK;
}

// Copies the site-ordered masks into the workspace's constrained working
// area (free between constrained calls; 16 bytes per site or more) and
// splits them by colour on the device.
int upload_bond_masks(hmc_lattice* L, const uint8_t* host_mask)
{
    uint8_t* tmp = static_cast<uint8_t*>(L->d.aos);
    hipError_t e = hipMemcpyAsync(tmp, host_mask, (size_t)L->d.N, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hmc::launch_split_masks(L->d, tmp, L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "copying the bond masks", e);
    L->m_valid = false;
    return HMC_OK;
}

}  // namespace

extern "C" {

int hmc_set_bond_masks(hmc_lattice* L, const uint8_t* host_mask)
{
    if (!L || !host_mask) return HMC_EINVAL;
    if (!L->d.mask) return fail(L, HMC_EINVAL, "the lattice was created without bond masks");
    int st = check_bond_masks(L, host_mask);
    if (st == HMC_OK) st = upload_bond_masks(L, host_mask);
    if (st != HMC_OK) return st;
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "copying the bond masks", e);
    return HMC_OK;
}

int hmc_set_bond_masks_async(hmc_lattice* L, const uint8_t* host_mask, int32_t check)
{
    if (!L || !host_mask) return HMC_EINVAL;
    if (!L->d.mask) return fail(L, HMC_EINVAL, "the lattice was created without bond masks");
    if (check) {
        int st = check_bond_masks(L, host_mask);
        if (st != HMC_OK) return st;
    }
    return upload_bond_masks(L, host_mask);
}

int hmc_plane_means(hmc_lattice* L, double* host_out)
{
    if (!L || !host_out) return HMC_EINVAL;
    // the reduction partials are free between sweeps; nz <= max_blocks
    int st = launch(L, 2, "plane-mean kernel", [&] { return hmc::launch_plane_means(L->d, L->d.part, L->stream); });
    if (st != HMC_OK) return st;
    hipError_t e = hipMemcpyAsync(host_out, L->d.part, 3 * sizeof(double) * (size_t)L->d.nz, hipMemcpyDeviceToHost,
                                  L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "reading the plane means", e);
    return HMC_OK;
}

int hmc_copy_spins(hmc_lattice* L, double* host_xyz, int32_t to_host)
{
    if (!L || !host_xyz) return HMC_EINVAL;
    const DevLattice& d = L->d;
    const size_t rs = d.precision / 8;
    const size_t bytes = (size_t)d.Nc * rs;
    std::vector<char> buf;
    try {
        buf.resize(6 * bytes);
    } catch (...) {
        return fail(L, HMC_ENOMEM, "host staging buffer");
    }
    char* base = static_cast<char*>(d.spins);
    auto get = [&](int c, int a, int64_t k) -> double {
        const char* p = buf.data() + (size_t)(3 * c + a) * bytes;
        return d.precision == 64 ? reinterpret_cast<const double*>(p)[k] : (double)reinterpret_cast<const float*>(p)[k];
    };
    auto put = [&](int c, int a, int64_t k, double v) {
        char* p = buf.data() + (size_t)(3 * c + a) * bytes;
        if (d.precision == 64) reinterpret_cast<double*>(p)[k] = v;
        else reinterpret_cast<float*>(p)[k] = (float)v;
    };
    hipError_t e = hipSuccess;
    if (to_host) {
        for (int i = 0; i < 6 && e == hipSuccess; ++i)
            e = hipMemcpyAsync(buf.data() + i * bytes, base + i * d.pitch, bytes, hipMemcpyDeviceToHost, L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
        if (e != hipSuccess) return fail(L, HMC_EHIP, "copying spins to the host", e);
    }
    // site id i = 2k + p, colour c = (x + y + z) & 1
    for (int64_t k = 0; k < d.Nc; ++k) {
        const int64_t r = k / d.hx;
        const int64_t y = r % d.ny, z = r / d.ny;
        for (int c = 0; c < 2; ++c) {
            const int64_t i = 2 * k + ((y + z + c) & 1);
            if (to_host) {
                for (int a = 0; a < 3; ++a) host_xyz[3 * i + a] = get(c, a, k);
            } else {
                // directions are normalised on the way in; zero or non-finite
                // vectors are stored as given
                const double* v = host_xyz + 3 * i;
                const double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                const double inv = (n2 > 0.0 && isfinite(n2)) ? 1.0 / sqrt(n2) : 1.0;
                for (int a = 0; a < 3; ++a) put(c, a, k, v[a] * inv);
            }
        }
    }
    if (!to_host) {
        for (int i = 0; i < 6 && e == hipSuccess; ++i)
            e = hipMemcpyAsync(base + i * d.pitch, buf.data() + i * bytes, bytes, hipMemcpyHostToDevice, L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
        if (e != hipSuccess) return fail(L, HMC_EHIP, "copying spins to the device", e);
        L->m_valid = false;
    }
    return HMC_OK;
}

size_t hmc_state_bytes(const hmc_lattice* L)
{
    if (!L) return 0;
    return sizeof(StateHeader) + sizeof(DevState) + 6 * (size_t)L->d.Nc * (L->d.precision / 8);
}

static void fill_header(const hmc_lattice* L, StateHeader* h)
{
    memset(h, 0, sizeof(*h));
    h->magic = kStateMagic;
    h->precision = (uint32_t)L->p.precision;
    h->nx = L->p.nx;
    h->ny = L->p.ny;
    h->nz = L->p.nz;
    h->boundary_z = L->p.boundary_z;
    h->seed = L->p.seed;
    h->bond_masks = (uint32_t)L->p.bond_masks;
    h->instance = L->p.instance;
    h->J = L->p.J;
    h->Ku = L->p.Ku;
    h->Kc = L->p.Kc;
    for (int a = 0; a < 3; ++a) {
        h->eu[a] = L->p.eu[a];
        h->h[a] = L->p.h[a];
    }
}

int hmc_get_state(hmc_lattice* L, void* host_buf, size_t bytes)
{
    if (!L || !host_buf) return HMC_EINVAL;
    if (bytes < hmc_state_bytes(L)) return fail(L, HMC_ESTATE, "state buffer too small");
    char* out = static_cast<char*>(host_buf);
    StateHeader h;
    fill_header(L, &h);
    memcpy(out, &h, sizeof(h));
    const size_t bytes_c = (size_t)L->d.Nc * (L->d.precision / 8);
    char* base = static_cast<char*>(L->d.spins);
    hipError_t e = hipMemcpyAsync(out + sizeof(h), L->d.st, sizeof(DevState), hipMemcpyDeviceToHost, L->stream);
    for (int i = 0; i < 6 && e == hipSuccess; ++i)
        e = hipMemcpyAsync(out + sizeof(h) + sizeof(DevState) + i * bytes_c, base + i * L->d.pitch, bytes_c,
                           hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "reading the state", e);
    return HMC_OK;
}

int hmc_set_state(hmc_lattice* L, const void* host_buf, size_t bytes)
{
    if (!L || !host_buf) return HMC_EINVAL;
    if (bytes < hmc_state_bytes(L)) return fail(L, HMC_ESTATE, "state buffer too small");
    const char* in = static_cast<const char*>(host_buf);
    StateHeader h, mine;
    memcpy(&h, in, sizeof(h));
    fill_header(L, &mine);
    if (memcmp(&h, &mine, sizeof(h)) != 0) return fail(L, HMC_ESTATE, "state image belongs to another lattice");
    const size_t bytes_c = (size_t)L->d.Nc * (L->d.precision / 8);
    char* base = static_cast<char*>(L->d.spins);
    // the kernels index the cone-angle table with theta: an image whose chain
    // state is out of range is refused before anything reaches the device
    DevState img;
    memcpy(&img, in + sizeof(h), sizeof(DevState));
    if (img.theta < 1 || img.theta > 180 || img.sweep < 0 || img.samples < 0 || img.torque_samples < 0 ||
        img.torque_samples > img.samples || img.accepted_last < 0 || img.accepted_last > L->d.N ||
        (img.nonfinite != 0 && img.nonfinite != 1))
        return fail(L, HMC_ESTATE, "state image holds an out-of-range cone angle or counter");
    L->init_state = img;
    hipError_t e = hipMemcpyAsync(L->d.st, &L->init_state, sizeof(DevState), hipMemcpyHostToDevice, L->stream);
    for (int i = 0; i < 6 && e == hipSuccess; ++i)
        e = hipMemcpyAsync(base + i * L->d.pitch, in + sizeof(h) + sizeof(DevState) + i * bytes_c, bytes_c,
                           hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "writing the state", e);
    L->m_valid = false;
    return HMC_OK;
}

int hmc_set_launch(hmc_lattice* L, int32_t sites_per_thread, int32_t z_chunk)
{
    if (!L) return HMC_EINVAL;
    if (sites_per_thread != 1 && sites_per_thread != 2 && sites_per_thread != 4)
        return fail(L, HMC_EINVAL, "sites_per_thread must be 1, 2 or 4");
    if (z_chunk < 1 || z_chunk > 1024) return fail(L, HMC_EINVAL, "z_chunk must be in [1, 1024]");
    if (hmc::pass_lds_bytes(L->d.precision, L->d.hx, sites_per_thread) > hmc::kMaxLds)
        return fail(L, HMC_EINVAL, "launch shape needs more than 64 KiB of LDS");
    L->spt = sites_per_thread;
    L->zc = z_chunk;
    return HMC_OK;
}

int hmc_get_launch(const hmc_lattice* L, int32_t* sites_per_thread, int32_t* z_chunk)
{
    if (!L || !sites_per_thread || !z_chunk) return HMC_EINVAL;
    *sites_per_thread = L->spt;
    *z_chunk = L->zc;
    return HMC_OK;
}

int hmc_set_prefetch(hmc_lattice* L, int32_t depth)
{
    if (!L) return HMC_EINVAL;
    if (depth < 0 || depth > 2) return fail(L, HMC_EINVAL, "prefetch depth must be 0, 1 or 2");
    if (depth == 2 && L->d.mask) return fail(L, HMC_EINVAL, "lattices with bond masks look one plane ahead");
    L->d.prefetch = depth;
    return HMC_OK;
}

int hmc_get_prefetch(const hmc_lattice* L, int32_t* depth)
{
    if (!L || !depth) return HMC_EINVAL;
    *depth = hmc::pass_deep(L->d) ? 2 : 1;
    return HMC_OK;
}

int hmc_set_timing(hmc_lattice* L, int32_t enable)
{
    if (!L) return HMC_EINVAL;
    hipError_t e = L->timer.enable(L->stream, enable != 0);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "switching timing", e);
    return HMC_OK;
}

int hmc_read_timing(hmc_lattice* L, hmc_timing* out)
{
    if (!L || !out) return HMC_EINVAL;
    hipError_t e = L->timer.flush(L->stream);
    if (e != hipSuccess) return fail(L, HMC_EHIP, "reading the timing events", e);
    *out = L->timer.tot;
    return HMC_OK;
}

void hmc_destroy(hmc_lattice* L)
{
    if (!L) return;
    // launches copy their arguments, so work still queued on the stream does
    // not use the handle; only the timing events go with it
    L->timer.destroy();
    delete L;
}

size_t hmc_snapshot_bytes(void) { return sizeof(DevState); }

int hmc_snapshot_enqueue(hmc_lattice* const* lattices, int32_t count, void* host_dst)
{
    if (!lattices || !host_dst || count < 0) return HMC_EINVAL;
    for (int32_t i = 0; i < count; ++i)
        if (!lattices[i] || lattices[i]->stream != lattices[0]->stream) return HMC_EINVAL;
    char* out = static_cast<char*>(host_dst);
    for (int32_t i = 0; i < count; ++i) {
        hmc_lattice* L = lattices[i];
        hipError_t e = hipMemcpyAsync(out + (size_t)i * sizeof(DevState), L->d.st, sizeof(DevState),
                                      hipMemcpyDeviceToHost, L->stream);
        if (e != hipSuccess) return fail(L, HMC_EHIP, "enqueueing a state snapshot", e);
    }
    return HMC_OK;
}

int hmc_snapshot_observables(const void* record, int64_t n, int32_t precision, hmc_obs* out)
{
    if (!record || !out || n <= 0 || (precision != 32 && precision != 64)) return HMC_EINVAL;
    DevState s;
    memcpy(&s, record, sizeof(s));
    hmc_lattice shim;
    shim.d.N = n;
    shim.d.precision = precision;
    return hmc::finish_observables(&shim, s, out);
}

int hmc_plane_means_async(hmc_lattice* L, double* dev_out)
{
    if (!L || !dev_out) return HMC_EINVAL;
    return launch(L, 2, "plane-mean kernel", [&] { return hmc::launch_plane_means(L->d, dev_out, L->stream); });
}

const char* hmc_strerror(int status)
{
    switch (status) {
    case HMC_OK: return "success";
    case HMC_EINVAL: return "invalid argument";
    case HMC_EDIM: return "invalid lattice dimensions";
    case HMC_ENOMEM: return "workspace too small or misaligned";
    case HMC_EHIP: return "HIP runtime error";
    case HMC_ESTATE: return "state image does not match the lattice";
    case HMC_ENUMERIC: return "non-finite value in the reductions";
    default: return "unknown status";
    }
}

const char* hmc_last_error(const hmc_lattice* L)
{
    return L ? L->err : "no lattice";
}

}  // extern "C"
