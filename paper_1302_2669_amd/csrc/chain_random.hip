// Random-scan chains (Sec. IV as written): every Metropolis step picks one
// stabilizer uniformly at random among all n_stab, computes its change of
// energy and applies it with the Metropolis probability; n is summed after
// every step.  A sweep is n_stab steps.  This is the paper's own chain, kept
// beside the colour-phased kernels as a statistical cross-check of their scan
// order; it is not the throughput path.
//
// Mapping.  One lane per chain as in the colour-phased kernels, but a random
// site needs its rows by a runtime index, so each lane's packed configuration
// lives in LDS, word-major with the workgroup's lanes side by side
// (word k of lane l at [k][l]: any rows, no bank conflicts), plus one spare
// word per lane.  The site table holds each qubit's word index and bit
// offset, so a step issues its four word reads at once (a missing neighbour
// reads the spare word), looks the weight change of each code up in a
// 2-bit-field constant, and applies an accepted move with four LDS XORs
// (two qubits of a site may share a word).  Workgroups are two waves; no
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

// two waves per workgroup share one copy of the site table, so that a CU
// holds more chains' configurations (5 waves per SIMD at L = 13 instead of 4);
// the largest code (L = 25) still fits the default 64 KB of dynamic LDS
constexpr int RS_LANES = 128;
constexpr uint32_t RS_NONE = 0xFFFFu;

// Per site: its 3-4 qubits as 16-bit codes, two per word: the qubit's word
// of the packed configuration (grid row * words per row + field / 16) << 5 |
// its bit offset 2 (field % 16); RS_NONE for a missing neighbour of a
// boundary stabilizer (word indices stay below 2^11, so no code equals it).
struct SiteQubits {
  uint32_t q01, q23;
};

__device__ __forceinline__ uint32_t qcode(int W, int row, int field) {
  return ((uint32_t)(row * W + (field >> 4)) << 5) | (uint32_t)(2 * (field & 15));
}

__device__ SiteQubits site_qubits(int L, int s) {
  const int nstar = L * (L - 1);
  const int W = words_per_row(L);
  uint32_t q[4] = {RS_NONE, RS_NONE, RS_NONE, RS_NONE};
  int k = 0;
  if (s < nstar) {  // star (i, j) at grid (2i+1, 2j)
    const int i = s / L, j = s % L;
    q[k++] = qcode(W, 2 * i, j);
    q[k++] = qcode(W, 2 * i + 2, j);
    if (j > 0) q[k++] = qcode(W, 2 * i + 1, j - 1);
    if (j < L - 1) q[k++] = qcode(W, 2 * i + 1, j);
  } else {          // plaquette (i, j) at grid (2i, 2j+1)
    const int t = s - nstar;
    const int i = t / (L - 1), j = t % (L - 1);
    if (i > 0) q[k++] = qcode(W, 2 * i - 1, j);
    if (i < L - 1) q[k++] = qcode(W, 2 * i + 1, j);
    q[k++] = qcode(W, 2 * i, j);
    q[k++] = qcode(W, 2 * i, j + 1);
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
  uint32_t* st = rs_lds + 2 * nstab;             // [RW][RS_LANES]
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
  // missing neighbours of boundary stabilizers read and "flip" a spare word
  // of the lane (with a zero mask), so that every step issues its four reads
  // and four XORs without branches
  const int sink = RW * RS_LANES + lane;
  for (int sweep = g.sweep_begin; sweep < g.sweep_end; ++sweep) {
    const bool counted = sweep >= g.burn;
    // The draws and the site entry of step t + 1 are taken while step t is
    // processed (the site table is read-only), so that their latency
    // overlaps the current step.
    uint4 blk = philox4x32_10(make_uint4(0u, (uint32_t)sweep, sid, ctr3), a.k0, a.k1);
    int s = (int)__umulhi(blk.x, (uint32_t)nstab);
    uint32_t u_acc = blk.y;
    SiteQubits sq = sites[s];
    for (int step = 0; step < nstab; ++step) {
      int s_next = 0;
      uint32_t acc_next = 0;
      SiteQubits sq_next = sq;
      if (step + 1 < nstab) {
        uint32_t u_site_next;
        if (((step + 1) & 1) == 0) {
          blk = philox4x32_10(make_uint4((uint32_t)((step + 1) >> 1), (uint32_t)sweep, sid, ctr3),
                              a.k0, a.k1);
          u_site_next = blk.x;
          acc_next = blk.y;
        } else {
          u_site_next = blk.z;
          acc_next = blk.w;
        }
        s_next = (int)__umulhi(u_site_next, (uint32_t)nstab);
        sq_next = sites[s_next];
      }
      const bool star = s < nstar;
      const uint32_t qc[4] = {sq.q01 & 0xFFFFu, sq.q01 >> 16, sq.q23 & 0xFFFFu, sq.q23 >> 16};
      int addr[4];
      uint32_t sh[4];
      bool valid[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        valid[k] = qc[k] != RS_NONE;
        addr[k] = valid[k] ? (int)(qc[k] >> 5) * RS_LANES + lane : sink;
        sh[k] = qc[k] & 31u;
      }
      uint32_t word[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) word[k] = st[addr[k]];
      // change of the qubit's weight when the site's Pauli is applied, plus
      // one, in 2-bit fields by its code (x + 2z): depolarizing, the weight
      // (1 - other)(1 - 2 own) of own = the part the site flips (x for a star,
      // z for a plaquette); bit/phase flips, 1 - 2 own
      const uint32_t lut = NOISE == 1 ? (star ? 0x22u : 0x0Au) : (star ? 0x52u : 0x46u);
      int delta = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t code = (word[k] >> sh[k]) & 3u;
        const int term = (int)((lut >> (2u * code)) & 3u) - 1;
        delta += valid[k] ? term : 0;
      }
      // threshold of delta = 1..4 (delta <= 0 is accepted whatever it is)
      const uint32_t t12 = delta == 1 ? thr1 : thr2;
      const uint32_t t34 = delta == 3 ? thr3 : thr4;
      const uint32_t thr = delta <= 2 ? t12 : t34;
      const bool accept = (delta <= 0) | (u_acc < thr);
      if (accept) {
        const uint32_t bit = star ? 1u : 2u;
        // read-modify-writes in LDS order: two qubits of a site may share a word
#pragma unroll
        for (int k = 0; k < 4; ++k) atomicXor(&st[addr[k]], valid[k] ? bit << sh[k] : 0u);
        n += delta;
        ++Acnt;
      }
      if (counted) Ssum += n;
      s = s_next;
      sq = sq_next;
      u_acc = acc_next;
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
         (size_t)(words_per_config(L) + 1) * RS_LANES * sizeof(uint32_t);
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
