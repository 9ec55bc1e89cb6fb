// Random-scan chains (Sec. IV as written): every Metropolis step picks one
// stabilizer uniformly at random among all n_stab, computes its change of
// energy and applies it with the Metropolis probability; n is summed after
// every step.  A sweep is n_stab steps.  This is the paper's own chain, kept
// beside the colour-phased kernels as a statistical cross-check of their scan
// order; it is not the throughput path.
//
// Mapping.  One lane per chain as in the colour-phased kernels, but a random
// site needs its rows by a runtime index, so each lane's packed configuration
// lives in LDS, word-major with the wave's 64 lanes side by side
// (word k of lane l at [k][l]: any rows, no bank conflicts).  A step reads and
// rewrites the words of the site's 3-4 qubits.  Workgroups are one wave; no
// barrier after the set-up.
//
// Randomness: step t of a sweep uses block t >> 1 of Philox4x32-10 at counter
// (t >> 1, sweep, syndrome_id, 2<<30 | cls<<28 | temp<<20 | chain): word
// 2(t&1) picks the site, floor(u n_stab / 2^32), word 2(t&1)+1 decides.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "internal.h"

namespace mcmc {
namespace {

constexpr int RS_LANES = 64;
constexpr uint32_t RS_NONE = 0xFFFFu;

// Per site: its 3-4 qubits as (grid row << 8 | field) 16-bit codes, two per
// word, RS_NONE for a missing neighbour of a boundary stabilizer.
struct SiteQubits {
  uint32_t q01, q23;
};

__device__ __forceinline__ uint32_t qcode(int row, int field) {
  return ((uint32_t)row << 8) | (uint32_t)field;
}

__device__ SiteQubits site_qubits(int L, int s) {
  const int nstar = L * (L - 1);
  uint32_t q[4] = {RS_NONE, RS_NONE, RS_NONE, RS_NONE};
  int k = 0;
  if (s < nstar) {  // star (i, j) at grid (2i+1, 2j)
    const int i = s / L, j = s % L;
    q[k++] = qcode(2 * i, j);
    q[k++] = qcode(2 * i + 2, j);
    if (j > 0) q[k++] = qcode(2 * i + 1, j - 1);
    if (j < L - 1) q[k++] = qcode(2 * i + 1, j);
  } else {          // plaquette (i, j) at grid (2i, 2j+1)
    const int t = s - nstar;
    const int i = t / (L - 1), j = t % (L - 1);
    if (i > 0) q[k++] = qcode(2 * i - 1, j);
    if (i < L - 1) q[k++] = qcode(2 * i + 1, j);
    q[k++] = qcode(2 * i, j);
    q[k++] = qcode(2 * i, j + 1);
  }
  SiteQubits r;
  r.q01 = q[0] | (q[1] << 16);
  r.q23 = q[2] | (q[3] << 16);
  return r;
}

template <int NOISE>
__global__ void __launch_bounds__(RS_LANES) chains_random_kernel(const RunArgs a) {
  extern __shared__ uint32_t rs_lds[];
  const GroupDesc g = a.g0;
  const int L = g.L;
  const int W = words_per_row(L);
  const int R = 2 * L - 1;
  const int RW = R * W;
  const int nstab = 2 * L * (L - 1);
  const int nstar = L * (L - 1);
  const int lane = threadIdx.x;
  SiteQubits* sites = reinterpret_cast<SiteQubits*>(rs_lds);
  uint32_t* st = rs_lds + 2 * nstab;             // [RW][64]
  for (int s = lane; s < nstab; s += RS_LANES) sites[s] = site_qubits(L, s);
  __syncthreads();

  const int64_t t = (int64_t)blockIdx.x * RS_LANES + lane;
  if (t >= g.n_tasks) return;
  const int K = g.K, C = g.C;
  const int64_t per_item = 4 * (int64_t)K * C;
  const int64_t item = t / per_item;
  const int rem = (int)(t - item * per_item);
  const int chain = rem % C;
  const int kt = (rem / C) % K;
  const int cls = rem / (C * K);
  const int64_t out = item * per_item + rem;
  const int64_t rows_off = item * RW * 4;
  const uint32_t sid = a.syndrome_ids ? a.syndrome_ids[item] : (uint32_t)item;

  const uint32_t thr1 = a.table0[kt][0], thr2 = a.table0[kt][1], thr3 = a.table0[kt][2],
                 thr4 = a.table0[kt][3];

  int32_t n;
  int64_t Ssum = 0, Acnt = 0;
  if (a.resume_rows) {
    for (int k = 0; k < RW; ++k)
      st[k * RS_LANES + lane] = a.resume_rows[(int64_t)k * a.total_chains + out];
    n = a.resume_n[out];
    Ssum = a.resume_S[out];
    Acnt = a.resume_A[out];
  } else {
    for (int k = 0; k < RW; ++k) st[k * RS_LANES + lane] = a.init_rows[rows_off + k * 4 + cls];
    n = a.init_n[item * 4 + cls];
  }

  const uint32_t ctr3 = (2u << 30) | ((uint32_t)cls << 28) | ((uint32_t)(kt + 1) << 20) |
                        (uint32_t)chain;
  for (int sweep = g.sweep_begin; sweep < g.sweep_end; ++sweep) {
    const bool counted = sweep >= g.burn;
    uint4 blk = make_uint4(0, 0, 0, 0);
    for (int step = 0; step < nstab; ++step) {
      if ((step & 1) == 0)
        blk = philox4x32_10(make_uint4((uint32_t)(step >> 1), (uint32_t)sweep, sid, ctr3), a.k0,
                            a.k1);
      const uint32_t u_site = (step & 1) ? blk.z : blk.x;
      const uint32_t u_acc = (step & 1) ? blk.w : blk.y;
      const int s = (int)__umulhi(u_site, (uint32_t)nstab);
      const bool star = s < nstar;
      const SiteQubits sq = sites[s];
      const uint32_t qc[4] = {sq.q01 & 0xFFFFu, sq.q01 >> 16, sq.q23 & 0xFFFFu, sq.q23 >> 16};
      int delta = 0;
      for (int k = 0; k < 4; ++k) {
        if (qc[k] == RS_NONE) continue;
        const int row = (int)(qc[k] >> 8), field = (int)(qc[k] & 0xFFu);
        const uint32_t word = st[(row * W + (field >> 4)) * RS_LANES + lane];
        const uint32_t code = (word >> (2 * (field & 15))) & 3u;
        const int x = (int)(code & 1u), z = (int)(code >> 1);
        const int own = star ? x : z, other = star ? z : x;
        delta += NOISE == 1 ? 1 - 2 * own : (1 - other) * (1 - 2 * own);
      }
      const uint32_t thr = delta == 1 ? thr1 : (delta == 2 ? thr2 : (delta == 3 ? thr3 : thr4));
      const bool accept = delta <= 0 || u_acc < thr;
      if (accept) {
        const uint32_t bit = star ? 1u : 2u;
        for (int k = 0; k < 4; ++k) {
          if (qc[k] == RS_NONE) continue;
          const int row = (int)(qc[k] >> 8), field = (int)(qc[k] & 0xFFu);
          st[(row * W + (field >> 4)) * RS_LANES + lane] ^= bit << (2 * (field & 15));
        }
        n += delta;
        ++Acnt;
      }
      if (counted) Ssum += n;
    }
  }

  a.S_out[out] = Ssum;
  a.A_out[out] = Acnt;
  a.n_out[out] = n;
  if (a.state_rows)
    for (int k = 0; k < RW; ++k)
      a.state_rows[(int64_t)k * a.total_chains + out] = st[k * RS_LANES + lane];
  if (a.final_rows && chain == 0 && kt == K - 1)
    for (int k = 0; k < RW; ++k) a.final_rows[rows_off + k * 4 + cls] = st[k * RS_LANES + lane];
}

}  // namespace

size_t random_scan_lds_bytes(int L) {
  const int nstab = 2 * L * (L - 1);
  return (size_t)2 * nstab * sizeof(uint32_t) +
         (size_t)words_per_config(L) * RS_LANES * sizeof(uint32_t);
}

hipError_t launch_chains_random(const RunArgs& a, hipStream_t s) {
  const int64_t T = a.g0.n_tasks;
  if (T == 0) return hipSuccess;
  const int64_t blocks = (T + RS_LANES - 1) / RS_LANES;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  const size_t lds = random_scan_lds_bytes(a.g0.L);
  if (a.noise == MCMC_NOISE_BITPHASE)
    hipLaunchKernelGGL(chains_random_kernel<1>, dim3((unsigned)blocks), dim3(RS_LANES), lds, s, a);
  else
    hipLaunchKernelGGL(chains_random_kernel<0>, dim3((unsigned)blocks), dim3(RS_LANES), lds, s, a);
  return hipGetLastError();
}

}  // namespace mcmc
