// hmc_handle.h -- host-side handles of the C interface: the lattice handle,
// its workspace layout, and the launch-event timer shared by lattices and
// batches.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "hmc.h"
#include "hmc_internal.h"

namespace hmc {

// Offsets of the regions of a lattice workspace.
struct Layout {
    size_t pitch, off_aos, off_state, off_c1, off_part, off_cnt, off_mask, total;
    int64_t max_blocks;
};

// Per-launch HIP events on one stream, summed by kind (hmc_timing).  The
// events are created when timing is switched on, so that a timed region does
// not pay for their creation.
struct Timer {
    static constexpr size_t kMaxEvents = 16384;   // event pairs before a flush
    bool on = false;
    std::vector<hipEvent_t> ev;                   // start/stop pairs
    std::vector<int> kind;
    size_t used = 0;
    hmc_timing tot{};

    // Waits for the stream and adds the recorded pairs to the totals.
    hipError_t flush(hipStream_t s);
    // Flushes, clears the totals and switches timing on or off.
    hipError_t enable(hipStream_t s, bool enable);
    hipError_t begin(hipStream_t s);
    hipError_t end(hipStream_t s, int k);
    void destroy();
};

// Validation of a parameter block (HMC_OK or the status hmc_init_lattice
// would return, with a message), and the byte pitch of its spin component
// arrays in a workspace (the six arrays lie at 0, pitch, .., 5 pitch).
int check_params(const hmc_params* p, char* msg, size_t n);
size_t spin_pitch(const hmc_params* p);

// Observables in two halves, so that a batch can read many lattices with one
// synchronisation: enqueue the measurement and the copy of the device state
// into host_dst (which must stay valid until the stream is synchronised),
// then fill *out from it.
int enqueue_observables(hmc_lattice* L, DevState* host_dst);
int finish_observables(hmc_lattice* L, const DevState& s, hmc_obs* out);

}  // namespace hmc

struct hmc_lattice {
    hmc::DevLattice d;
    hmc_params p;
    hipStream_t stream;
    hmc::Layout lay;
    int spt = 2, zc = 16;
    bool m_valid = false;
    char err[256] = {0};
    double c1d[181];
    float c1f[181];
    hmc::DevState init_state;
    hmc::Timer timer;
};
