// hmc_batch.cpp -- batches of independent lattices (hmc_batch_* in hmc.h):
// the table that maps the work-groups of one colour-pass launch onto the
// lattices, temperature uploads, graph capture and replay, and the launch
// shape autotuner.  All arithmetic of the method runs in the kernels of
// hmc_kernels.hip; this file only arranges launches.
#include "hmc.h"

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <array>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "hmc_handle.h"
#include "hmc_internal.h"

namespace {

constexpr int32_t kMaxBatch = 65536;
constexpr int32_t kMaxGraphSweeps = 4096;
// Chunk sizes the autotuner tries (bytes of spins; 0 = one chunk).  A
// chunk is swept through all the sweeps of a call before the next one, so
// that it stays in the 256 MB Infinity Cache; too small a chunk leaves the
// device short of work-groups.
constexpr size_t kChunkCandidates[] = {0, 96u << 20, 128u << 20, 160u << 20, 192u << 20, 224u << 20, 256u << 20};
// sweeps per chunk when a chunk size is timed: the first sweep of a chunk
// reads it from HBM, the following ones from the cache, as in a long call
constexpr int32_t kChunkTrialSweeps = 20;
constexpr size_t kAlign = hmc::kAlign;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Regions of the batch workspace: the table and the group index arrays
// (uploaded when the launch shapes change), then the per-call arrays of
// temperatures, Boltzmann scales and finalize flags (uploaded when they
// change).
struct BatchLayout {
    size_t off_tab, off_idx, off_T, off_scale, off_fin, total;
    size_t entry;   // table stride, bytes
};

BatchLayout batch_layout(int32_t count, int precision)
{
    BatchLayout b{};
    b.entry = hmc::batch_entry_bytes(precision);
    const size_t entry_max = std::max(hmc::batch_entry_bytes(32), hmc::batch_entry_bytes(64));
    b.off_tab = 0;
    size_t off = align_up((size_t)count * entry_max, kAlign);
    b.off_idx = off;
    off += align_up((size_t)hmc::kBatchGroups * (2 * (size_t)count + 1) * sizeof(uint32_t), kAlign);
    b.off_T = off;
    off += align_up((size_t)count * sizeof(double), kAlign);
    b.off_scale = off;
    off += align_up((size_t)count * sizeof(double), kAlign);
    b.off_fin = off;
    off += align_up((size_t)count * sizeof(int32_t), kAlign);
    b.total = off;
    return b;
}

}  // namespace

struct hmc_batch {
    std::vector<hmc_lattice*> lat;
    int32_t capacity = 0;      // most lattices the workspace and staging hold
    int precision = 32;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    BatchLayout lay{};
    // launch shapes the table was built with
    std::vector<std::pair<int, int>> shape;
    // chunks: consecutive table entries [first, first + count) and the
    // colour-pass launches (one per kernel variant) that cover them
    struct Chunk {
        uint32_t first = 0, count = 0;
        std::vector<hmc::BatchLaunch> launches;
    };
    std::vector<Chunk> chunks;
    size_t chunk_bytes = 0;
    // pinned staging of the uploads: a ring of kRing buffers, each reused
    // once the copy last made from it has run, so that the host can prepare
    // uploads while earlier work is still queued; staging and upload_done
    // name the buffer in use and its event
    static constexpr int kRing = 4;
    char* ring[kRing] = {};
    hipEvent_t ring_ev[kRing] = {};
    int ring_cur = 0;
    char* staging = nullptr;
    hipEvent_t upload_done = nullptr;
    bool table_valid = false;
    bool call_valid = false;
    std::vector<double> T_last;
    std::vector<int32_t> fin_last;
    bool any_sample = false;
    // graph replay
    int32_t graph_sweeps = 0;
    hipStream_t cap = nullptr;
    std::vector<std::array<hipGraphExec_t, 2>> exec;   // per chunk, per sample flag
    hmc::Timer timer;
    char err[256] = {0};
};

namespace {

int bfail(hmc_batch* B, int status, const char* what, hipError_t e = hipSuccess)
{
    if (B) {
        if (e != hipSuccess) snprintf(B->err, sizeof(B->err), "%s: %s", what, hipGetErrorString(e));
        else snprintf(B->err, sizeof(B->err), "%s", what);
    }
    return status;
}

void drop_graphs(hmc_batch* B)
{
    bool any = false;
    for (auto& pair : B->exec)
        for (auto g : pair) any = any || g != nullptr;
    // a replay may still be running on the stream
    if (any) (void)hipStreamSynchronize(B->stream);
    for (auto& pair : B->exec)
        for (auto& g : pair)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    B->exec.assign(B->chunks.size(), {nullptr, nullptr});
}

// Moves to the next staging buffer of the ring and waits until the upload
// last made from it has run.
hipError_t staging_wait(hmc_batch* B)
{
    B->ring_cur = (B->ring_cur + 1) % hmc_batch::kRing;
    B->staging = B->ring[B->ring_cur];
    B->upload_done = B->ring_ev[B->ring_cur];
    return hipEventSynchronize(B->upload_done);
}

hipError_t upload(hmc_batch* B, size_t off, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(B->ws + off, B->staging + off, bytes, hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess) e = hipEventRecord(B->upload_done, B->stream);
    return e;
}

// Rebuilds and uploads the table if any lattice's launch shape changed.
int refresh_table(hmc_batch* B)
{
    const size_t n = B->lat.size();
    bool same = B->table_valid;
    for (size_t i = 0; i < n && same; ++i)
        same = B->shape[i] == std::make_pair(B->lat[i]->spt, B->lat[i]->zc);
    if (same) return HMC_OK;

    hipError_t e = staging_wait(B);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "waiting for the staging buffer", e);
    char* tab = B->staging + B->lay.off_tab;
    uint32_t* idx = reinterpret_cast<uint32_t*>(B->staging + B->lay.off_idx);
    for (size_t i = 0; i < n; ++i) {
        hmc_lattice* L = B->lat[i];
        B->shape[i] = {L->spt, L->zc};
        hmc::batch_fill_entry(tab + i * B->lay.entry, L->d, L->spt, L->zc);
    }
    // chunks of consecutive lattices: k = ceil(total / chunk_bytes) chunks
    // of about equal bytes of spins (lattice i goes to the chunk that holds
    // the middle of its bytes), so no chunk is left with a small remainder
    B->chunks.clear();
    const size_t rs = (size_t)B->precision / 8;
    double total = 0.0;
    for (size_t i = 0; i < n; ++i) total += (double)B->lat[i]->d.N * 3.0 * (double)rs;
    const size_t k = B->chunk_bytes > 0 ? std::max<size_t>(1, (size_t)std::ceil(total / (double)B->chunk_bytes)) : 1;
    const double target = total / (double)k;
    double before = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double b = (double)B->lat[i]->d.N * 3.0 * (double)rs;
        const size_t c = std::min(k - 1, (size_t)((before + 0.5 * b) / target));
        if (B->chunks.empty() || c != B->chunks.size() - 1) {
            hmc_batch::Chunk ch;
            ch.first = (uint32_t)i;
            B->chunks.push_back(std::move(ch));
        }
        B->chunks.back().count += 1;
        before += b;
    }
    // one launch per kernel variant present in a chunk; the work-group
    // offsets and table indices of all launches are packed in the index
    // region (2 m + 1 words for a launch over m lattices, 3 n words at most)
    const uint32_t* dev_idx = reinterpret_cast<const uint32_t*>(B->ws + B->lay.off_idx);
    size_t cursor = 0;
    for (auto& c : B->chunks) {
        std::vector<std::vector<uint32_t>> members(hmc::kBatchGroups);
        for (uint32_t i = c.first; i < c.first + c.count; ++i)
            members[hmc::batch_group(B->lat[i]->d, B->lat[i]->spt)].push_back(i);
        for (int g = 0; g < hmc::kBatchGroups; ++g) {
            const auto& m = members[g];
            if (m.empty()) continue;
            uint32_t* start = idx + cursor;
            uint32_t* ent = start + m.size() + 1;
            hmc::BatchLaunch bl{};
            bl.group = g;
            bl.tab = B->ws + B->lay.off_tab;
            bl.start = dev_idx + cursor;
            bl.ent = bl.start + m.size() + 1;
            bl.n = (uint32_t)m.size();
            cursor += 2 * m.size() + 1;
            uint64_t acc = 0;
            size_t lds = 0;
            for (size_t j = 0; j < m.size(); ++j) {
                const hmc_lattice* L = B->lat[m[j]];
                start[j] = (uint32_t)acc;
                ent[j] = m[j];
                acc += (uint64_t)hmc::pass_blocks(L->d, L->spt, L->zc);
                lds = std::max(lds, hmc::pass_lds_bytes(B->precision, L->d.hx, L->spt));
            }
            if (acc > 0x7FFFFFFFull)
                return bfail(B, HMC_EINVAL, "batch needs more than 2^31 work-groups per launch");
            start[m.size()] = (uint32_t)acc;
            bl.nblk = (uint32_t)acc;
            bl.lds = lds;
            bl.scale = B->ws + B->lay.off_scale;
            c.launches.push_back(bl);
        }
    }
    e = upload(B, 0, B->lay.off_T);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "uploading the batch table", e);
    drop_graphs(B);
    B->table_valid = true;
    return HMC_OK;
}

// Temperatures and sample flags of this call (sample == nullptr: none
// sampled; one_flag >= 0: that flag for every lattice).
int set_call(hmc_batch* B, const double* T, const int32_t* sample, int one_flag)
{
    const size_t n = B->lat.size();
    for (size_t i = 0; i < n; ++i)
        if (!(T[i] > 0.0) || !isfinite(T[i])) return bfail(B, HMC_EINVAL, "temperatures must be positive and finite");
    std::vector<int32_t> fin(n);
    bool any = false;
    for (size_t i = 0; i < n; ++i) {
        const bool smp = one_flag >= 0 ? one_flag != 0 : (sample && sample[i] != 0);
        fin[i] = hmc::kFinCounts | (smp ? (hmc::kFinObs | hmc::kFinSample) : 0);
        any = any || smp;
    }
    B->any_sample = any;
    if (B->call_valid && std::equal(T, T + n, B->T_last.begin()) && fin == B->fin_last) return HMC_OK;
    hipError_t e = staging_wait(B);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "waiting for the staging buffer", e);
    double* Ts = reinterpret_cast<double*>(B->staging + B->lay.off_T);
    char* sc = B->staging + B->lay.off_scale;
    int32_t* fs = reinterpret_cast<int32_t*>(B->staging + B->lay.off_fin);
    for (size_t i = 0; i < n; ++i) {
        Ts[i] = T[i];
        hmc::batch_store_scale(B->precision, T[i], sc, i);
        fs[i] = fin[i];
    }
    e = upload(B, B->lay.off_T, B->lay.total - B->lay.off_T);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "uploading the temperatures", e);
    B->T_last.assign(T, T + n);
    B->fin_last = fin;
    B->call_valid = true;
    return HMC_OK;
}

// Enqueues one sweep of the lattices of chunk c on stream s.
template <class Pre, class Post>
hipError_t enqueue_sweep(hmc_batch* B, size_t c, bool obs, hipStream_t s, Pre pre, Post post)
{
    const auto& ch = B->chunks[c];
    hipError_t e = hipSuccess;
    for (int colour = 0; colour < 2 && e == hipSuccess; ++colour)
        for (const auto& bl : ch.launches) {
            if ((e = pre()) != hipSuccess) return e;
            if ((e = hmc::launch_pass_batch(B->precision, bl, colour, obs, s)) != hipSuccess) return e;
            if ((e = post(0)) != hipSuccess) return e;
        }
    if ((e = pre()) != hipSuccess) return e;
    e = hmc::launch_finalize_batch(B->precision, B->ws + B->lay.off_tab + (size_t)ch.first * B->lay.entry, ch.count,
                                   reinterpret_cast<const double*>(B->ws + B->lay.off_T) + ch.first,
                                   reinterpret_cast<const int32_t*>(B->ws + B->lay.off_fin) + ch.first, s);
    if (e != hipSuccess) return e;
    return post(2);
}

hipError_t eager_sweep(hmc_batch* B, size_t c, bool obs)
{
    if (!B->timer.on)
        return enqueue_sweep(B, c, obs, B->stream, [] { return hipSuccess; }, [](int) { return hipSuccess; });
    return enqueue_sweep(
        B, c, obs, B->stream, [B] { return B->timer.begin(B->stream); },
        [B](int k) { return B->timer.end(B->stream, k); });
}

// One sweep of every lattice (chunk after chunk).
hipError_t eager_sweep_all(hmc_batch* B, bool obs)
{
    hipError_t e = hipSuccess;
    for (size_t c = 0; c < B->chunks.size() && e == hipSuccess; ++c) e = eager_sweep(B, c, obs);
    return e;
}

hipError_t build_graph(hmc_batch* B, size_t c, bool obs)
{
    if (!B->cap) {
        hipError_t e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t ee = hipSuccess;
    for (int32_t i = 0; i < B->graph_sweeps && ee == hipSuccess; ++i)
        ee = enqueue_sweep(B, c, obs, B->cap, [] { return hipSuccess; }, [](int) { return hipSuccess; });
    e = hipStreamEndCapture(B->cap, &g);
    if (ee != hipSuccess) e = ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&B->exec[c][obs ? 1 : 0], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

void destroy_batch(hmc_batch* B)
{
    if (!B) return;
    (void)hipStreamSynchronize(B->stream);
    drop_graphs(B);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    for (int r = 0; r < hmc_batch::kRing; ++r) {
        if (B->ring_ev[r]) (void)hipEventDestroy(B->ring_ev[r]);
        if (B->ring[r]) (void)hipHostFree(B->ring[r]);
    }
    B->timer.destroy();
    delete B;
}

// The checks shared by hmc_batch_create and hmc_batch_set_lattices.
int check_lattices(hmc_lattice* const* lattices, int32_t count)
{
    if (!lattices || count < 1 || count > kMaxBatch) return HMC_EINVAL;
    // lattices with bond masks run the masked pass, which batches do not have
    for (int32_t i = 0; i < count; ++i)
        if (!lattices[i] || lattices[i]->d.mask) return HMC_EINVAL;
    std::vector<hmc_lattice*> sorted(lattices, lattices + count);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return HMC_EINVAL;
    for (int32_t i = 1; i < count; ++i)
        if (lattices[i]->d.precision != lattices[0]->d.precision || lattices[i]->stream != lattices[0]->stream)
            return HMC_EINVAL;
    return HMC_OK;
}

}  // namespace

extern "C" {

size_t hmc_batch_workspace_bytes(int32_t count)
{
    if (count < 1 || count > kMaxBatch) return 0;
    return batch_layout(count, 64).total;
}

int hmc_batch_create(hmc_lattice* const* lattices, int32_t count, void* dev_ws, size_t ws_bytes, hmc_batch** out)
{
    if (!out) return HMC_EINVAL;
    *out = nullptr;
    int st = check_lattices(lattices, count);
    if (st != HMC_OK) return st;
    const BatchLayout lay = batch_layout(count, lattices[0]->d.precision);
    if (!dev_ws || ws_bytes < hmc_batch_workspace_bytes(count) || ((uintptr_t)dev_ws % kAlign) != 0)
        return HMC_ENOMEM;
    // capacity: the most lattices this workspace holds (sizes grow with the count)
    int32_t lo = count, hi = kMaxBatch;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (hmc_batch_workspace_bytes(mid) <= ws_bytes) lo = mid;
        else hi = mid - 1;
    }
    const int32_t capacity = lo;
    const size_t staging_bytes = batch_layout(capacity, 64).total;

    hmc_batch* B = new (std::nothrow) hmc_batch();
    if (!B) return HMC_ENOMEM;
    B->lat.assign(lattices, lattices + count);
    B->capacity = capacity;
    B->precision = lattices[0]->d.precision;
    B->stream = lattices[0]->stream;
    B->ws = static_cast<char*>(dev_ws);
    B->lay = lay;
    B->shape.assign(count, {0, 0});
    hipError_t e = hipSuccess;
    for (int r = 0; r < hmc_batch::kRing && e == hipSuccess; ++r) {
        e = hipHostMalloc(reinterpret_cast<void**>(&B->ring[r]), staging_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ring_ev[r], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(B->ring_ev[r], B->stream);
        if (e == hipSuccess) memset(B->ring[r], 0, staging_bytes);
    }
    if (e != hipSuccess) {
        destroy_batch(B);
        return HMC_EHIP;
    }
    B->staging = B->ring[0];
    B->upload_done = B->ring_ev[0];
    st = refresh_table(B);
    if (st == HMC_OK) {
        e = hipStreamSynchronize(B->stream);
        if (e != hipSuccess) st = HMC_EHIP;
    }
    if (st != HMC_OK) {
        destroy_batch(B);
        return st;
    }
    *out = B;
    return HMC_OK;
}

}  // extern "C"

namespace {

int batch_sweep(hmc_batch* B, const double* T, const int32_t* sample, int one_flag, int32_t n_sweeps)
{
    if (!B) return HMC_EINVAL;
    if (!T) return bfail(B, HMC_EINVAL, "null temperature array");
    if (n_sweeps < 0) return bfail(B, HMC_EINVAL, "n_sweeps must be >= 0");
    int st = set_call(B, T, sample, one_flag);
    if (st == HMC_OK) st = refresh_table(B);
    if (st != HMC_OK) return st;
    // the black pass computes the fused sums if any lattice samples; the
    // finalize flags decide per lattice whether they are used
    const bool obs = B->any_sample;
    // all the sweeps of one chunk before the next: the chunk stays in the
    // Infinity Cache; each lattice still runs red, black, finalize per sweep
    for (size_t c = 0; c < B->chunks.size(); ++c) {
        int32_t done = 0;
        if (B->graph_sweeps > 0 && !B->timer.on) {
            hipGraphExec_t& g = B->exec[c][obs ? 1 : 0];
            while (n_sweeps - done >= B->graph_sweeps) {
                if (!g) {
                    hipError_t e = build_graph(B, c, obs);
                    if (e != hipSuccess) return bfail(B, HMC_EHIP, "capturing the sweep graph", e);
                }
                hipError_t e = hipGraphLaunch(g, B->stream);
                if (e != hipSuccess) return bfail(B, HMC_EHIP, "replaying the sweep graph", e);
                done += B->graph_sweeps;
            }
        }
        for (; done < n_sweeps; ++done) {
            hipError_t e = eager_sweep(B, c, obs);
            if (e != hipSuccess) return bfail(B, HMC_EHIP, "batch sweep launch", e);
        }
    }
    if (n_sweeps > 0)
        for (size_t i = 0; i < B->lat.size(); ++i) B->lat[i]->m_valid = (B->fin_last[i] & hmc::kFinSample) != 0;
    return HMC_OK;
}

}  // namespace

extern "C" {

int hmc_batch_sweep(hmc_batch* B, const double* T, int32_t n_sweeps, int32_t sample)
{
    return batch_sweep(B, T, nullptr, sample != 0 ? 1 : 0, n_sweeps);
}

int hmc_batch_sweep_each(hmc_batch* B, const double* T, const int32_t* sample, int32_t n_sweeps)
{
    if (B && !sample) return bfail(B, HMC_EINVAL, "null sample-flag array");
    return batch_sweep(B, T, sample, -1, n_sweeps);
}

int hmc_batch_tune(hmc_batch* B, const double* T, int32_t trial_sweeps)
{
    if (!B) return HMC_EINVAL;
    if (!T) return bfail(B, HMC_EINVAL, "null temperature array");
    if (trial_sweeps < 1 || trial_sweeps > 1000) return bfail(B, HMC_EINVAL, "trial_sweeps must be in [1, 1000]");
    int st = set_call(B, T, nullptr, 0);
    if (st != HMC_OK) return st;
    const size_t n = B->lat.size();

    // save every chain
    std::vector<std::vector<char>> saved(n);
    try {
        for (size_t i = 0; i < n; ++i) saved[i].resize(hmc_state_bytes(B->lat[i]));
    } catch (...) {
        return bfail(B, HMC_ENOMEM, "host memory for the saved states");
    }
    for (size_t i = 0; i < n; ++i)
        if (hmc_get_state(B->lat[i], saved[i].data(), saved[i].size()) != HMC_OK)
            return bfail(B, HMC_EHIP, "saving a lattice state");

    // size classes, largest total first
    std::map<std::tuple<int, int, int>, std::vector<size_t>> cls;
    for (size_t i = 0; i < n; ++i) cls[{B->lat[i]->d.nx, B->lat[i]->d.ny, B->lat[i]->d.nz}].push_back(i);
    std::vector<std::vector<size_t>> order;
    for (auto& kv : cls) order.push_back(kv.second);
    std::stable_sort(order.begin(), order.end(), [&](const auto& a, const auto& b) {
        return (double)a.size() * (double)B->lat[a[0]]->d.N > (double)b.size() * (double)B->lat[b[0]]->d.N;
    });

    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const bool was_timing = B->timer.on;
    B->timer.on = false;
    // everything is timed in the order of a sweep call: chunk after chunk,
    // kChunkTrialSweeps sweeps each (one chunk when chunking is off)
    auto time_chunked = [&](float* ms) -> int {
        int s2 = refresh_table(B);
        if (s2 != HMC_OK) return s2;
        hipError_t r = eager_sweep_all(B, false);
        if (r == hipSuccess) r = hipEventRecord(e0, B->stream);
        for (size_t c = 0; c < B->chunks.size() && r == hipSuccess; ++c)
            for (int32_t k = 0; k < std::max(trial_sweeps, kChunkTrialSweeps) && r == hipSuccess; ++k)
                r = eager_sweep(B, c, false);
        if (r == hipSuccess) r = hipEventRecord(e1, B->stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
        return r == hipSuccess ? HMC_OK : bfail(B, HMC_EHIP, "timing a batch configuration", r);
    };
    st = e == hipSuccess ? HMC_OK : bfail(B, HMC_EHIP, "hipEventCreate", e);
    // the chunk size with the current shapes
    auto tune_chunk = [&]() {
        size_t best_chunk = B->chunk_bytes;
        float best_ms = 0.f;
        bool first = true;
        for (size_t cb : kChunkCandidates) {
            if (st != HMC_OK) break;
            B->chunk_bytes = cb;
            B->table_valid = false;
            float ms = 0.f;
            st = time_chunked(&ms);
            if (st == HMC_OK && (first || ms < best_ms)) {
                best_ms = ms;
                best_chunk = cb;
                first = false;
            }
        }
        B->chunk_bytes = best_chunk;
        B->table_valid = false;
    };
    tune_chunk();
    // the launch shape of each size class under that chunking
    for (const auto& members : order) {
        if (st != HMC_OK) break;
        const hmc_lattice* L0 = B->lat[members[0]];
        std::pair<int, int> best = {L0->spt, L0->zc};
        float best_ms = 0.f;
        st = time_chunked(&best_ms);
        for (int spt : {1, 2, 4}) {
            if (hmc::pass_lds_bytes(B->precision, L0->d.hx, spt) > hmc::kMaxLds) continue;
            for (int zc = 2; zc <= 64 && zc <= L0->d.nz && st == HMC_OK; zc *= 2) {
                if (std::make_pair(spt, zc) == best) continue;
                for (size_t i : members) {
                    B->lat[i]->spt = spt;
                    B->lat[i]->zc = zc;
                }
                float ms = 0.f;
                st = time_chunked(&ms);
                if (st == HMC_OK && ms < best_ms) {
                    best_ms = ms;
                    best = {spt, zc};
                }
            }
        }
        for (size_t i : members) {
            B->lat[i]->spt = best.first;
            B->lat[i]->zc = best.second;
        }
    }
    // and the chunk size again with the final shapes
    tune_chunk();
    B->timer.on = was_timing;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);

    // restore every chain, whatever happened above
    for (size_t i = 0; i < n; ++i)
        if (hmc_set_state(B->lat[i], saved[i].data(), saved[i].size()) != HMC_OK && st == HMC_OK)
            st = bfail(B, HMC_EHIP, "restoring a lattice state");
    if (st == HMC_OK) st = refresh_table(B);
    if (st == HMC_OK) {
        e = hipStreamSynchronize(B->stream);
        if (e != hipSuccess) st = bfail(B, HMC_EHIP, "hipStreamSynchronize", e);
    }
    return st;
}

int hmc_batch_set_lattices(hmc_batch* B, hmc_lattice* const* lattices, int32_t count)
{
    if (!B) return HMC_EINVAL;
    int st = check_lattices(lattices, count);
    if (st != HMC_OK) return bfail(B, st, "invalid lattice list (null, duplicate, masked or mixed)");
    if (lattices[0]->d.precision != B->precision || lattices[0]->stream != B->stream)
        return bfail(B, HMC_EINVAL, "the lattices must keep the batch's precision and stream");
    if (count > B->capacity) return bfail(B, HMC_ENOMEM, "more lattices than the workspace holds");
    hipError_t e = staging_wait(B);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "waiting for the staging buffer", e);
    drop_graphs(B);
    B->lat.assign(lattices, lattices + count);
    B->lay = batch_layout(count, B->precision);
    B->shape.assign(count, {0, 0});
    B->table_valid = false;
    B->call_valid = false;
    B->T_last.clear();
    B->fin_last.clear();
    return refresh_table(B);
}

int hmc_batch_observables(hmc_batch* B, hmc_obs* out)
{
    if (!B) return HMC_EINVAL;
    if (!out) return bfail(B, HMC_EINVAL, "null output array");
    const size_t n = B->lat.size();
    std::vector<hmc::DevState> s;
    try {
        s.resize(n);
    } catch (...) {
        return bfail(B, HMC_ENOMEM, "host memory for the device states");
    }
    for (size_t i = 0; i < n; ++i) {
        int st = hmc::enqueue_observables(B->lat[i], &s[i]);
        if (st != HMC_OK) {
            (void)hipStreamSynchronize(B->stream);
            return bfail(B, st, hmc_last_error(B->lat[i]));
        }
    }
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "reading the device states", e);
    int worst = HMC_OK;
    for (size_t i = 0; i < n; ++i) {
        int st = hmc::finish_observables(B->lat[i], s[i], out + i);
        if (st != HMC_OK && worst == HMC_OK) {
            worst = st;
            bfail(B, st, hmc_last_error(B->lat[i]));
        }
    }
    return worst;
}

int hmc_batch_reset_stats(hmc_batch* B)
{
    if (!B) return HMC_EINVAL;
    hipError_t e = hmc::launch_reset_batch(B->precision, B->ws + B->lay.off_tab, (uint32_t)B->lat.size(), B->stream);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "clearing the accumulators", e);
    return HMC_OK;
}

int hmc_batch_set_chunk_bytes(hmc_batch* B, int64_t bytes)
{
    if (!B) return HMC_EINVAL;
    if (bytes < 0) return bfail(B, HMC_EINVAL, "chunk bytes must be >= 0");
    if ((size_t)bytes != B->chunk_bytes) {
        hipError_t e = staging_wait(B);
        if (e != hipSuccess) return bfail(B, HMC_EHIP, "waiting for the staging buffer", e);
        B->chunk_bytes = (size_t)bytes;
        B->table_valid = false;
        return refresh_table(B);
    }
    return HMC_OK;
}

int hmc_batch_get_chunk_bytes(const hmc_batch* B, int64_t* bytes)
{
    if (!B || !bytes) return HMC_EINVAL;
    *bytes = (int64_t)B->chunk_bytes;
    return HMC_OK;
}

int hmc_batch_set_graph(hmc_batch* B, int32_t sweeps_per_graph)
{
    if (!B) return HMC_EINVAL;
    if (sweeps_per_graph < 0 || sweeps_per_graph > kMaxGraphSweeps)
        return bfail(B, HMC_EINVAL, "sweeps_per_graph must be in [0, 4096]");
    if (sweeps_per_graph != B->graph_sweeps) {
        hipError_t e = hipStreamSynchronize(B->stream);
        if (e != hipSuccess) return bfail(B, HMC_EHIP, "hipStreamSynchronize", e);
        drop_graphs(B);
        B->graph_sweeps = sweeps_per_graph;
    }
    return HMC_OK;
}

int hmc_batch_set_timing(hmc_batch* B, int32_t enable)
{
    if (!B) return HMC_EINVAL;
    hipError_t e = B->timer.enable(B->stream, enable != 0);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "switching timing", e);
    return HMC_OK;
}

int hmc_batch_read_timing(hmc_batch* B, hmc_timing* out)
{
    if (!B || !out) return HMC_EINVAL;
    hipError_t e = B->timer.flush(B->stream);
    if (e != hipSuccess) return bfail(B, HMC_EHIP, "reading the timing events", e);
    *out = B->timer.tot;
    return HMC_OK;
}

void hmc_batch_destroy(hmc_batch* B) { destroy_batch(B); }

const char* hmc_batch_last_error(const hmc_batch* B) { return B ? B->err : "no batch"; }

}  // extern "C"
