// Explicit instantiations of the chain kernel for L = 17, 18.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<17>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<18>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
