// Explicit instantiations of the chain kernel for L = 21, 22.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<21>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<22>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
