// Device-built plan for a batch of one code size whose syndromes each carry a
// sweep budget (route 0: no counted sweep, 1: short, 2: full), as set by the
// gate.  Three groups in descending cost (full, short, none); the items of a
// group are written in whatever order the atomics give, which changes no
// result: every chain is keyed by its syndrome id, class, temperature and
// replica, and every output goes to the syndrome's own slots.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "internal.h"

namespace mcmc {
namespace {

__device__ __forceinline__ int budget_group(uint8_t route) {
  return route >= 2 ? 0 : (route == 1 ? 1 : 2);
}

// Per wave: one atomic per group for the wave's items of that group, which
// adds their number to cursor[group]; returns this lane's slot (the cursor's
// old value plus its rank among the wave's items of its group).
__device__ __forceinline__ uint32_t wave_claim(uint32_t* cursor, int g, bool active) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t pos = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint64_t m = __ballot(active && g == k);
    if (m == 0) continue;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&cursor[k], (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (active && g == k) pos = base + (uint32_t)__popcll(m & lt);
  }
  return pos;
}

__global__ void __launch_bounds__(256) budget_count_kernel(const BudgetArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  const int g = active ? budget_group(a.route[i]) : 0;
  (void)wave_claim(a.counts, g, active);
}

__global__ void budget_finalize_kernel(const BudgetArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t first = 0, cum = 0;
  for (int g = 0; g < 3; ++g) {
    const uint32_t ng = a.counts[g];
    GroupDesc d{};
    d.L = a.L;
    d.K = a.K;
    d.C = a.C;
    d.burn = a.burn;
    d.sweep_begin = 0;
    d.sweep_end = a.burn + a.sweeps[g];
    d.first_item = (int32_t)first;
    d.n_items = (int32_t)ng;
    d.n_tasks = (int64_t)ng * 4 * a.K * a.C;
    a.groups[g] = d;
    a.counts[4 + g] = first;        // cursor of the group's items
    first += ng;
    cum += (uint32_t)((d.n_tasks + TILE - 1) / TILE);
    a.tile_cum[g] = cum;
  }
}

__global__ void __launch_bounds__(256) budget_scatter_kernel(const BudgetArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  const int g = active ? budget_group(a.route[i]) : 0;
  const uint32_t pos = wave_claim(a.counts + 4, g, active);
  if (!active) return;
  const int L = a.L;
  ItemDesc it{};
  it.orig = i;
  it.syn_off = i * (int64_t)(2 * L * (L - 1));
  it.rows_off = i * (int64_t)words_per_config(L) * 4;
  it.chain_off = i * 4 * (int64_t)a.K * a.C;
  it.corr_off = i * (int64_t)(2 * L * L - 2 * L + 1);
  it.table_off = a.beta ? i * 4 * (int64_t)a.K : a.table0_off;
  it.beta_bar = a.beta ? a.beta[i] : a.beta0;
  it.beta_star = it.beta_bar;
  it.sid = a.ids[i];
  it.group = g;
  it.err_thr = 0;
  a.items[pos] = it;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_budget_plan(const BudgetArgs& a, hipStream_t s) {
  hipError_t e = launch_zero(a.counts, 8, s);
  if (e != hipSuccess) return e;
  if (a.n > 0)
    hipLaunchKernelGGL(budget_count_kernel, dim3(blocks_of(a.n)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(budget_finalize_kernel, dim3(1), dim3(64), 0, s, a);
  if (a.n > 0)
    hipLaunchKernelGGL(budget_scatter_kernel, dim3(blocks_of(a.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mcmc
