// Explicit instantiations of the chain kernel for L = 2, 3, 4, 5, 6, 7, 8, 9.
#include "chain_kernel.h"

namespace mcmc {
template hipError_t launch_chain_L<2>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<3>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<4>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<5>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<6>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<7>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<8>(const ChainArgs&, hipStream_t, bool, bool);
template hipError_t launch_chain_L<9>(const ChainArgs&, hipStream_t, bool, bool);
}  // namespace mcmc
