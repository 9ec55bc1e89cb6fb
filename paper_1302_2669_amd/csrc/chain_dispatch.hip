// Runtime-L dispatch to the compile-time-L chain kernels.  The kernels are
// instantiated in the chain_inst_*.hip translation units (compiled in
// parallel); this file only selects one.
#include "internal.h"

namespace mcmc {

hipError_t launch_chain(int L, const ChainArgs& a, hipStream_t s, bool trace, bool resume) {
  switch (L) {
#define MCMC_CASE(LL) \
  case LL:            \
    return launch_chain_L<LL>(a, s, trace, resume);
    MCMC_CASE(2) MCMC_CASE(3) MCMC_CASE(4) MCMC_CASE(5) MCMC_CASE(6) MCMC_CASE(7)
    MCMC_CASE(8) MCMC_CASE(9) MCMC_CASE(10) MCMC_CASE(11) MCMC_CASE(12) MCMC_CASE(13)
    MCMC_CASE(14) MCMC_CASE(15) MCMC_CASE(16) MCMC_CASE(17) MCMC_CASE(18) MCMC_CASE(19)
    MCMC_CASE(20) MCMC_CASE(21) MCMC_CASE(22) MCMC_CASE(23) MCMC_CASE(24) MCMC_CASE(25)
#undef MCMC_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace mcmc
