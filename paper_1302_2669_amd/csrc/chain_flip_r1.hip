// Persistent chain kernel for L = 14..16 under independent bit/phase flips
// (energy = x parts + z parts; one-word rows, 5 waves per SIMD).  Same launch shape and
// Philox grouping as the depolarizing kernel of this range; only the per-qubit
// weight-change terms differ.
#define MCMC_PAIRED_PHILOX 1
#include "chain_body.h"

namespace mcmc {

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
chains_flip_r1_kernel(const RunArgs a) {
  chains_persistent<14, 16, 1>(a);
}

template <>
hipError_t launch_chains_flip_range<1>(const RunArgs& a, int waves, int wg, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  const int per_wg = wg / 64;
  const int blocks = (waves + per_wg - 1) / per_wg;
  hipLaunchKernelGGL(chains_flip_r1_kernel, dim3((unsigned)blocks), dim3((unsigned)wg), 0, s, a);
  return hipGetLastError();
}

}  // namespace mcmc
