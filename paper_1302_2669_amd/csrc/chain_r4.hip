// Persistent chain kernel for L = 23..25 (two-word rows, 3 waves per SIMD).
// Each kernel's L range is small enough to compile in about two minutes and
// to share one register budget; a batch runs one kernel per range its
// syndromes fall in.
// Philox blocks four at a time: at 3 waves per SIMD the extra independent
// multiplies gain 5-10% here (measured; at L = 19-21 they cost as much).
#define MCMC_PAIRED_PHILOX 4
#include "chain_body.h"

namespace mcmc {

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
chains_r4_kernel(const RunArgs a) {
  chains_persistent<23, 25>(a);
}

template <>
hipError_t launch_chains_range<4>(const RunArgs& a, int waves, int wg, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  const int per_wg = wg / 64;
  const int blocks = (waves + per_wg - 1) / per_wg;
  hipLaunchKernelGGL(chains_r4_kernel, dim3((unsigned)blocks), dim3((unsigned)wg), 0, s, a);
  return hipGetLastError();
}

}  // namespace mcmc
