// hmc_deep_kernels.hip -- the standard colour pass with the depth-two march
// (loads two planes ahead of the update), used for lattices whose spins do
// not fit the last-level cache.  Same tile layout and per-site code as the
// depth-one pass; kept in its own translation unit so that the two families
// compile in parallel.
#include "hmc_pass.hpp"

namespace hmc {

hipError_t launch_pass_deep(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s)
{
    return PassLaunch<false, true>::run(d, colour, obs, spt, zc, T, s);
}

}  // namespace hmc
