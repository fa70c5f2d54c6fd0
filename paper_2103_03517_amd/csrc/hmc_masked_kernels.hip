// hmc_masked_kernels.hip -- the standard colour pass of lattices with
// per-site bond masks (granular films, whose bonds between grains carry no
// exchange).  The same tile code as the unmasked pass, with each neighbour
// weighted by its bond bit; kept in its own translation unit so that the
// unmasked kernels and their build are unchanged.
#include "hmc_pass.hpp"

namespace hmc {

hipError_t launch_pass_masked(const DevLattice& d, int colour, bool obs, int spt, int zc, double T, hipStream_t s)
{
    return PassLaunch<true, false>::run(d, colour, obs, spt, zc, T, s);
}

}  // namespace hmc
