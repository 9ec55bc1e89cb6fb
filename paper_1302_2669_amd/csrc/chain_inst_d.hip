// Explicit instantiations of the chain kernel for L = 14, 15, 16.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<14>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<15>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<16>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
