// Space-time chains at L = 14 with the streaming register window.
#include "spacetime_win.h"

namespace mcmc {
template hipError_t launch_spacetime_win_L<14>(const SpaceTimeArgs& a, hipStream_t s);
}  // namespace mcmc
