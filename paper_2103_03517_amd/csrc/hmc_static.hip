// hmc_static.hip -- hmc_measure_static: the measurement of hmc_observables
// (moment, the energy terms of Eq. 2 with every bond once, the anisotropy
// torque) on spins held by the caller, for callers that cannot allocate
// device memory.  The per-work-group partials, the acceptance-count rows the
// reduction kernels also write, and the reduced values live in `scratch`, a
// static device array of the library (one copy per GPU, held until the
// process ends), instead of a workspace.  The kernels are those of
// hmc_observables (measure, then the fixed-order finalize), launched with the
// same grid, so both entry points give the same bits.
#include "hmc.h"

#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <mutex>

#include "hmc_handle.h"
#include "hmc_internal.h"

namespace {

// Largest lattice: 2^25 spins, so at most 2^24 sites per colour and
// 2^24 / 256 = 65536 work-groups of the measurement, each writing one double
// to each of the kNumPart partial rows and one count per colour row.
constexpr uint64_t kStaticMaxSpins = 1ull << 25;
constexpr size_t kStaticRecords = (kStaticMaxSpins / 2) / hmc::kThreads;
constexpr size_t kStateBytes = (sizeof(hmc::DevState) + 255) / 256 * 256;
constexpr size_t kPartBytes = (kStaticRecords + kStaticRecords / 1024) * hmc::kNumPart * sizeof(double);
constexpr size_t kCntBytes = 2 * kStaticRecords * sizeof(uint32_t);
constexpr size_t kScratchBytes = kStateBytes + kPartBytes + kCntBytes;   // 6822400 B (6.51 MiB)
static_assert(kScratchBytes % 256 == 0, "scratch regions stay 256-byte aligned");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on each GPU (the host-side name is only a
// stand-in), looked up on the first call made with that GPU current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_for_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Zeroes n 32-bit words (the reduced-state record before each call: its
// non-finite flag is sticky).  A kernel rather than a memset node, so that
// the call can sit in a captured graph.
__global__ void clear_words_kernel(uint32_t* p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

extern "C" int hmc_measure_static(const hmc_params* p, const void* dev_spins, size_t spins_bytes,
                                  void* hip_stream, hmc_obs* out)
{
    if (!p || !dev_spins || !out) return HMC_EINVAL;
    char msg[256];
    int st = hmc::check_params(p, msg, sizeof(msg));
    if (st != HMC_OK) return st;
    if (p->bond_masks) return HMC_EINVAL;
    const uint64_t N = (uint64_t)p->nx * (uint64_t)p->ny * (uint64_t)p->nz;
    if (N > kStaticMaxSpins) return HMC_EDIM;
    const size_t pitch = hmc::spin_pitch(p);
    if (spins_bytes < 6 * pitch || ((uintptr_t)dev_spins % hmc::kAlign) != 0) return HMC_ENOMEM;

    void* base = nullptr;
    if (scratch_for_current_device(&base) != hipSuccess) return HMC_EHIP;
    char* sc = static_cast<char*>(base);
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);

    hmc::DevLattice d;
    memset(&d, 0, sizeof(d));
    d.precision = p->precision;
    d.nx = p->nx;
    d.ny = p->ny;
    d.nz = p->nz;
    d.hx = p->nx / 2;
    d.P = d.hx * p->ny;
    d.N = (int64_t)N;
    d.Nc = d.N / 2;
    d.pitch = pitch;
    d.spins = const_cast<void*>(dev_spins);      // read only by the measurement
    d.st = reinterpret_cast<hmc::DevState*>(sc);
    d.part = reinterpret_cast<double*>(sc + kStateBytes);
    d.cnt = reinterpret_cast<uint32_t*>(sc + kStateBytes + kPartBytes);
    d.max_blocks = (int64_t)kStaticRecords;      // row stride of the counts and of the partials
    d.J = p->J;
    d.Ku = p->Ku;
    d.Kc = p->Kc;
    const double eun = sqrt(p->eu[0] * p->eu[0] + p->eu[1] * p->eu[1] + p->eu[2] * p->eu[2]);
    for (int a = 0; a < 3; ++a) {
        d.eu[a] = p->eu[a] / eun;
        d.h[a] = p->h[a];
    }
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.instance = p->instance;
    d.zbound = p->boundary_z;

    const uint32_t words = (uint32_t)(sizeof(hmc::DevState) / 4);
    clear_words_kernel<<<1, 128, 0, s>>>(reinterpret_cast<uint32_t*>(sc), words);
    hipError_t e = hipGetLastError();
    int64_t nb = 0;
    if (e == hipSuccess) e = hmc::launch_measure(d, s, &nb);
    if (e == hipSuccess && (size_t)nb > kStaticRecords) e = hipErrorInvalidValue;   // not reached: N is bounded
    if (e == hipSuccess) e = hmc::launch_finalize(d, 0, 0, nb, hmc::kFinObs | hmc::kFinTorque, 0.0, s);
    hmc::DevState r;
    if (e == hipSuccess) e = hipMemcpyAsync(&r, sc, sizeof(r), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return HMC_EHIP;

    memset(out, 0, sizeof(*out));
    out->n = d.N;
    out->precision = p->precision;
    out->theta_deg = 0;
    for (int a = 0; a < 3; ++a) {
        out->M[a] = r.M[a];
        out->torque[a] = r.torque[a];
    }
    out->m = sqrt(r.M[0] * r.M[0] + r.M[1] * r.M[1] + r.M[2] * r.M[2]) / (double)d.N;
    out->E_exch = r.E_exch;
    out->E_uni = r.E_uni;
    out->E_cub = r.E_cub;
    out->E_zee = r.E_zee;
    out->E = r.E_exch + r.E_uni + r.E_cub + r.E_zee;
    return r.nonfinite ? HMC_ENUMERIC : HMC_OK;
}
