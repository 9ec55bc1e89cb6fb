// Persistent chain kernel for L = 2..13 (one-word rows, 6 waves per SIMD).
// Each kernel's L range is small enough to compile in about two minutes and
// to share one register budget; a batch runs one kernel per range its
// syndromes fall in.
// At 80 VGPRs, computing Philox blocks in pairs costs more spills than the
// extra independent work gains at 6 waves per SIMD: blocks one at a time.
#define MCMC_PAIRED_PHILOX 0
#include "chain_body.h"

namespace mcmc {

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6)))
chains_r0_kernel(const RunArgs a) {
  chains_persistent<2, 13>(a);
}

template <>
hipError_t launch_chains_range<0>(const RunArgs& a, int waves, int wg, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  const int per_wg = wg / 64;
  const int blocks = (waves + per_wg - 1) / per_wg;
  hipLaunchKernelGGL(chains_r0_kernel, dim3((unsigned)blocks), dim3((unsigned)wg), 0, s, a);
  return hipGetLastError();
}

}  // namespace mcmc
