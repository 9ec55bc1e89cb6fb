// Gate-network training support on the device (not part of the paper's
// method): initial parameters, the budget labels, class targets relative to
// the start decision, the keyed shuffle of each epoch and the epoch's loss
// sum.  The epoch loop itself (gather, forward,
// backward, Adam) is sequenced by mcmc_cnn_train_epoch in cnn_api.cpp.
//
// Random numbers: Philox4x32-10 with key = seed, domain 3 of the fourth
// counter word with class field 3:
//   initial weight i:   counter (i >> 1, 0, 0, 3<<30 | 3<<28 | 0xFE<<20),
//                       words 2(i&1), 2(i&1)+1 -> (a, b);
//   shuffle round r:    counter (v, r, epoch, 3<<30 | 3<<28 | 0xFD<<20), word 0.
#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace mcmc {

namespace {

constexpr uint32_t CTR3_INIT = (3u << 30) | (3u << 28) | (0xFEu << 20);
constexpr uint32_t CTR3_SHUFFLE = (3u << 30) | (3u << 28) | (0xFDu << 20);

// He-normal weights, zero biases.  Weight i of a block with fan-in f is
// sqrt(-2 ln u1) cos(2 pi u2) sqrt(2 / f) in double, rounded to float, with
// u1 = (a + 1) 2^-32 in (0, 1] and u2 = b 2^-32 in [0, 1) (Box-Muller).
__global__ void __launch_bounds__(256) cnn_init_kernel(int64_t n, CnnOffsets o, int fan1,
                                                       int fan2, int fanh, uint32_t k0,
                                                       uint32_t k1, float* __restrict__ prm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int fan = 0;
  if (i < o.b1) fan = fan1;
  else if (i >= o.W2 && i < o.b2) fan = fan2;
  else if (i >= o.W3 && i < o.b3) fan = fan2;
  else if (i >= o.Wh && i < o.bh) fan = fanh;
  if (fan == 0) { prm[i] = 0.0f; return; }
  const uint4 w = philox4x32_10(make_uint4((uint32_t)(i >> 1), 0u, 0u, CTR3_INIT), k0, k1);
  const uint32_t a = (i & 1) ? w.z : w.x;
  const uint32_t b = (i & 1) ? w.w : w.y;
  const double u1 = ((double)a + 1.0) * 0x1p-32;
  const double u2 = (double)b * 0x1p-32;
  const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
  prm[i] = (float)(z * sqrt(2.0 / (double)fan));
}

// budget = 0 if the no-sweep decision equals the full-budget one, else 1 if
// the short-budget decision does, else 2
__global__ void __launch_bounds__(256) budget_labels_kernel(int64_t n, const uint8_t* __restrict__ d0,
                                                            const uint8_t* __restrict__ d1,
                                                            const uint8_t* __restrict__ d2,
                                                            int32_t* __restrict__ budget) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  budget[i] = d0[i] == d2[i] ? 0 : (d1[i] == d2[i] ? 1 : 2);
}

// Class targets relative to the start decision: out[i][k] = prob[i][k ^ s_i]
// with s_i the low two bits of start[i] (classes are the two logical
// parities, so XOR composes two classes).
__global__ void __launch_bounds__(256) relative_targets_kernel(int64_t n, const uint8_t* __restrict__ start,
                                                               const float* __restrict__ prob,
                                                               float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  const int64_t i = t >> 2;
  const int k = (int)(t & 3);
  out[t] = prob[i * 4 + (k ^ (start[i] & 3))];
}

// Keyed permutation of [0, n): a 4-round balanced Feistel network on b bits
// (b = the smallest even number >= 2 with 2^b >= n), round function the low
// b/2 bits of a Philox word, and cycle walking back into [0, n).
__device__ __forceinline__ uint32_t feistel(uint32_t x, int half, uint32_t epoch, uint32_t k0,
                                            uint32_t k1) {
  const uint32_t mask = (1u << half) - 1u;
  uint32_t l = x >> half, r = x & mask;
  for (uint32_t rnd = 0; rnd < 4; ++rnd) {
    const uint32_t f = philox4x32_10(make_uint4(r, rnd, epoch, CTR3_SHUFFLE), k0, k1).x & mask;
    const uint32_t nl = r, nr = l ^ f;
    l = nl;
    r = nr;
  }
  return (l << half) | r;
}

__global__ void __launch_bounds__(256) permutation_kernel(int64_t n, int half, uint32_t epoch,
                                                          uint32_t k0, uint32_t k1,
                                                          int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t domain = (int64_t)1 << (2 * half);
  uint32_t y = feistel((uint32_t)i, half, epoch, k0, k1);
  for (int64_t g = 0; g < domain && (int64_t)y >= n; ++g) y = feistel(y, half, epoch, k0, k1);
  perm[i] = (int32_t)y;
}

// acc[0] += sum of loss[0..B), added in index order by one thread
__global__ void loss_sum_kernel(int64_t B, const float* __restrict__ loss,
                                double* __restrict__ acc) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int64_t i = 0; i < B; ++i) s += (double)loss[i];
  acc[0] += s;
}

__global__ void zero_f64_kernel(double* p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) p[0] = 0.0;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int permutation_half_bits(int64_t n) {
  int b = 2;
  while (((int64_t)1 << b) < n) b += 2;
  return b / 2;
}

hipError_t cnn_init_params(int L, uint64_t seed, float* prm, hipStream_t s) {
  const CnnOffsets o = cnn_offsets(L);
  hipLaunchKernelGGL(cnn_init_kernel, dim3(blocks(o.total)), dim3(256), 0, s, o.total, o,
                     9 * 3, 9 * 32, 32 * L * L, (uint32_t)(seed & 0xFFFFFFFFull),
                     (uint32_t)(seed >> 32), prm);
  return hipGetLastError();
}

hipError_t gate_budget_labels(int64_t n, const uint8_t* d0, const uint8_t* d1, const uint8_t* d2,
                              int32_t* budget, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(budget_labels_kernel, dim3(blocks(n)), dim3(256), 0, s, n, d0, d1, d2,
                     budget);
  return hipGetLastError();
}

hipError_t gate_relative_targets(int64_t n, const uint8_t* start, const float* prob, float* out,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(relative_targets_kernel, dim3(blocks(4 * n)), dim3(256), 0, s, n, start, prob,
                     out);
  return hipGetLastError();
}

hipError_t cnn_permutation(int64_t n, uint64_t seed, uint32_t epoch, int32_t* perm,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(permutation_kernel, dim3(blocks(n)), dim3(256), 0, s, n,
                     permutation_half_bits(n), epoch, (uint32_t)(seed & 0xFFFFFFFFull),
                     (uint32_t)(seed >> 32), perm);
  return hipGetLastError();
}

hipError_t cnn_loss_sum(int64_t B, const float* loss, double* acc, bool reset, hipStream_t s) {
  if (reset) {
    hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(64), 0, s, acc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, s, B, loss, acc);
  return hipGetLastError();
}

}  // namespace mcmc
