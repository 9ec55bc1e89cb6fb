// Explicit instantiations of the chain kernel for L = 10, 11, 12.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<10>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<11>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<12>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
