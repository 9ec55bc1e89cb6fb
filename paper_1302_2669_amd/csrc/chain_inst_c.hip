// Explicit instantiations of the chain kernel for L = 13.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<13>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
