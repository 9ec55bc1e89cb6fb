// Explicit instantiations of the chain kernel for L = 19, 20.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<19>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<20>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
