// Kernels around the chain kernel: class starts, unpacking, the estimator and
// the error sampler (arXiv:1302.2669, Sec. II-IV).
#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace mcmc {

// ---------------------------------------------------------------------------
// Class starts (Sec. IV: every class needs a starting configuration consistent
// with the syndrome).  E0 explains each lit plaquette (2i, 2j+1) by X on
// (2i, 0), (2i, 2), ..., (2i, 2j) and each lit star (2i+1, 2j) by Z on
// (0, 2j), (2, 2j), ..., (2i, 2j); so on even row 2i the x part of field k is
// the parity of lit plaquettes (i, j >= k) and the z part of field k the
// parity of lit stars (i' >= i, k).  Odd rows stay empty.  E0 lies in class
// (bx, bz) = (parity of all lit plaquettes, parity of all lit stars);
// class c multiplies it by X-bar (X on row 0) if bx != c&1 and by Z-bar
// (Z on column 0) if bz != c>>1.  One thread per (syndrome, class).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) init_kernel(const StartArgs a) {
  const int64_t sc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sc >= a.n * 4) return;
  const int cls = (int)(sc & 3);
  const StartItem si = start_item(a, sc >> 2);
  const int L = si.L;
  const int nstab = 2 * L * (L - 1);
  const int nstar = L * (L - 1);
  const uint8_t* sy = si.sy;
  const int W = words_per_row(L);

  int bx = 0, bz = 0;
  for (int k = 0; k < nstab; ++k) {
    const int lit = sy[k] != 0;
    if (k < nstar) bz ^= lit; else bx ^= lit;
  }
  const int xbar = bx ^ (cls & 1);
  const int zbar = bz ^ (cls >> 1);

  int weight = 0;
  uint32_t colpar = 0;  // bit k: parity of lit stars (i' >= i, k)
  for (int i = L - 1; i >= 0; --i) {
    if (i <= L - 2)
      for (int k = 0; k < L; ++k) colpar ^= (uint32_t)(sy[i * L + k] != 0) << k;
    // x parts of even row 2i: suffix parity of plaquettes (i, j >= k)
    uint32_t xbits = 0, p = 0;
    for (int j = L - 2; j >= 0; --j) {
      p ^= (uint32_t)(sy[nstar + i * (L - 1) + j] != 0);
      xbits |= p << j;
    }
    uint32_t zbits = colpar;
    if (i == 0 && xbar) xbits ^= (1u << L) - 1u;
    if (zbar) zbits ^= 1u;
    weight += si.noise ? __builtin_popcount(xbits) + __builtin_popcount(zbits)
                      : __builtin_popcount(xbits | zbits);
    if (a.bytes) {  // qubit (2i, 2k) is number i*side + k; odd-row qubits are I
      const int side = 2 * L - 1, nq = 2 * L * L - 2 * L + 1;
      uint8_t* out = a.bytes + (si.orig * 4 + cls) * nq;
      for (int k = 0; k < L; ++k)
        out[i * side + k] = (uint8_t)(((xbits >> k) & 1u) | (((zbits >> k) & 1u) << 1));
      if (i >= 1)
        for (int f = 0; f < L - 1; ++f) out[(i - 1) * side + L + f] = 0;
    }
    if (!a.rows) continue;
    for (int w = 0; w < W; ++w) {
      uint32_t word = 0;
      for (int f = 0; f < 16; ++f) {
        const int k = 16 * w + f;
        uint32_t code = 3u;  // padding
        if (k < L) code = ((xbits >> k) & 1u) | (((zbits >> k) & 1u) << 1);
        word |= code << (2 * f);
      }
      a.rows[si.rows_off + ((2 * i) * W + w) * 4 + cls] = word;
    }
    if (i >= 1) {  // odd row 2i-1: empty, padding beyond L-1 fields
      for (int w = 0; w < W; ++w)
        a.rows[si.rows_off + ((2 * i - 1) * W + w) * 4 + cls] = ~field_mask(L - 1, w);
    }
  }
  if (a.weights) a.weights[si.orig * 4 + cls] = weight;
}

hipError_t launch_init(const StartArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t work = a.n * 4;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) zero_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Clears a small device buffer with a kernel (no memset node, so that the
// sequence can be captured into a graph and replayed).
hipError_t launch_zero(uint32_t* p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unpack `count` packed configurations (word-major, element stride `stride`)
// into one byte per qubit (row-major over the grid) and/or their weights.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) unpack_kernel(int L, int noise,
                                                     const uint32_t* __restrict__ rows,
                                                     int64_t count, int64_t stride,
                                                     uint8_t* __restrict__ out,
                                                     int32_t* __restrict__ weights) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int W = words_per_row(L);
  const int nq = 2 * L * L - 2 * L + 1;
  int q = 0, weight = 0;
  for (int r = 0; r < 2 * L - 1; ++r) {
    const int fields = (r & 1) ? L - 1 : L;
    for (int f = 0; f < fields; ++f) {
      const uint32_t word = rows[(int64_t)(r * W + f / 16) * stride + e];
      const uint8_t code = (uint8_t)((word >> (2 * (f % 16))) & 3u);
      weight += noise ? (code & 1) + (code >> 1) : code != 0;
      if (out) out[e * nq + q] = code;
      ++q;
    }
  }
  if (weights) weights[e] = weight;
}

hipError_t launch_unpack(int L, int noise, const uint32_t* rows, int64_t count, int64_t stride,
                         uint8_t* out, int32_t* weights, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, L,
                     noise,
                     rows, count, stride, out, weights);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Estimator and decision (Eq. main, Sec. IV.A), one thread per syndrome, FP64
// in a fixed order with no contraction:
//   mean_{E,k} = (sum_c S) / (C * 4 * sweeps)   (mean final weight if sweeps = 0;
//                n_stab samples per sweep instead of 4 for the random scan)
//   K = 1 : I_E = (beta* / 2)(f0 + mean_{E,1}) + (beta_bar - beta*) mean_{E,1}
//           (trapezoid to the sampled temperature, <n> held above it; the
//           plain trapezoid when beta* = beta_bar)
//   K even: I_E = (h / 3)(f0 + 4 f1 + 2 f2 + ... + f_K), h = beta_bar / K
//   f0 = <n> at beta = 0: 3/4 n_q (depolarizing), n_q (bit/phase flips)
//   log Z_E = n_stab log 2 - I_E,  P_E = softmax(log Z)
// Decision by the integer key sum_{k<K} w_k S_{E,k} + S_{E,K} (all I_E share
// f0 and the denominator), ties to the lowest class.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
__global__ void __launch_bounds__(128) decide_kernel(const DecideArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n) return;
  GroupDesc g;
  int64_t orig, chain_off, rows_off, corr_off;
  double beta_bar, beta_star;
  int noise = 0;
  int64_t per_sweep = 4;
  if (a.items) {
    const ItemDesc it = a.items[s];
    g = a.groups[it.group];
    orig = it.orig;
    chain_off = it.chain_off;
    rows_off = it.rows_off;
    corr_off = it.corr_off;
    beta_bar = it.beta_bar;
    beta_star = it.beta_star;
    noise = it.noise;
  } else {
    g = a.g0;
    orig = s;
    chain_off = s * 4 * (int64_t)g.K * g.C;
    rows_off = s * (int64_t)words_per_config(g.L) * 4;
    corr_off = s * (int64_t)(2 * g.L * g.L - 2 * g.L + 1);
    beta_bar = a.beta_bar;
    beta_star = a.beta_star;
    noise = a.noise;
    if (a.samples_per_sweep > 0) per_sweep = a.samples_per_sweep;
  }
  const int K = g.K, C = g.C, L = g.L;
  const int sweeps = g.sweep_end - g.burn;
  const bool counted = sweeps > 0;
  const double denom = counted ? (double)((int64_t)C * per_sweep * sweeps) : (double)C;
  const double nq = (double)(2 * L * L - 2 * L + 1);
  const double f0 = noise ? nq : 0.75 * nq;
  const double log_z0 = (double)(2 * L * (L - 1)) * a.ln2;
  double logz[4];
  int64_t key[4];
  for (int e = 0; e < 4; ++e) {
    const int64_t base = chain_off + (int64_t)e * K * C;
    double acc = f0;
    int64_t kk = 0;
    double mean_last = 0.0, mean_first = 0.0;
    for (int k = 0; k < K; ++k) {
      int64_t sum = 0;
      for (int c = 0; c < C; ++c)
        sum += counted ? a.S[base + (int64_t)k * C + c] : (int64_t)a.n_final[base + (int64_t)k * C + c];
      const double mean = (double)sum / denom;
      if (k == 0) mean_first = mean;
      if (k + 1 < K) {
        acc = acc + ((k + 1) % 2 == 1 ? 4.0 : 2.0) * mean;
        kk += ((k + 1) % 2 == 1 ? 4 : 2) * sum;
      } else {
        acc = acc + mean;
        kk += sum;
        mean_last = mean;
      }
    }
    double integral;
    if (K == 1) {
      integral = (beta_star / 2.0) * (f0 + mean_first) + (beta_bar - beta_star) * mean_first;
    } else {
      const double h = beta_bar / (double)K;
      integral = (acc * h) / 3.0;
    }
    logz[e] = log_z0 - integral;
    key[e] = kk;
    if (a.mean_n) a.mean_n[orig * 4 + e] = mean_last;
  }
  double m = logz[0];
  for (int e = 1; e < 4; ++e) m = logz[e] > m ? logz[e] : m;
  double ex[4];
  for (int e = 0; e < 4; ++e) ex[e] = exp(logz[e] - m);
  const double tot = ((ex[0] + ex[1]) + ex[2]) + ex[3];
  for (int e = 0; e < 4; ++e) a.class_prob[orig * 4 + e] = ex[e] / tot;
  int best = 0;
  for (int e = 1; e < 4; ++e)
    if (key[e] < key[best]) best = e;
  // a gate's class route: the decision composed with the predicted class
  // (classes are the two logical parities, so composition is XOR)
  if (a.flip) best ^= a.flip[orig] & 3;
  a.chosen[orig] = (uint8_t)best;

  if (a.correction && a.final_rows) {
    const int W = words_per_row(L);
    uint8_t* out = a.correction + corr_off;
    int q = 0;
    for (int r = 0; r < 2 * L - 1; ++r) {
      const int fields = (r & 1) ? L - 1 : L;
      for (int f = 0; f < fields; ++f) {
        const uint32_t word = a.final_rows[rows_off + (r * W + f / 16) * 4 + best];
        out[q++] = (uint8_t)((word >> (2 * (f % 16))) & 3u);
      }
    }
  }
}
#pragma clang fp contract(on)

hipError_t launch_decide(const DecideArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(decide_kernel, dim3((unsigned)((a.n + 127) / 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Depolarizing errors (Eq. pauliChannel with p/3 each), their syndrome and
// class.  One workgroup per sample: the errors are drawn into LDS (one Philox
// block serves two qubits), then every site takes its parity.
// ---------------------------------------------------------------------------
constexpr int SAMPLE_MAX_NQ = 2 * MCMC_L_MAX * MCMC_L_MAX - 2 * MCMC_L_MAX + 1;

__device__ __forceinline__ void sample_one(int L, int noise, uint32_t threshold, uint32_t k0,
                                           uint32_t k1,
                                           uint32_t sid, uint8_t* err, uint8_t* __restrict__ syn,
                                           uint8_t* __restrict__ true_class,
                                           uint8_t* __restrict__ errors) {
  const int side = 2 * L - 1;
  const int nq = 2 * L * L - 2 * L + 1;
  const int nstab = 2 * L * (L - 1);
  const int nstar = L * (L - 1);
  for (int pr = threadIdx.x; pr < (nq + 1) / 2; pr += blockDim.x) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)pr, 0u, sid, 1u << 30), k0, k1);
    for (int h = 0; h < 2; ++h) {
      const int q = 2 * pr + h;
      if (q >= nq) break;
      const uint32_t u0 = h ? w.z : w.x;
      const uint32_t u1 = h ? w.w : w.y;
      if (noise) {  // independent flips: x part from u0, z part from u1
        err[q] = (uint8_t)((u0 < threshold ? 1 : 0) | (u1 < threshold ? 2 : 0));
        continue;
      }
      const uint32_t type = (uint32_t)(((uint64_t)u1 * 3u) >> 32);  // 0 X, 1 Y, 2 Z
      const uint8_t code = (uint8_t)(type == 0 ? 1 : (type == 1 ? 3 : 2));
      err[q] = u0 < threshold ? code : (uint8_t)0;
    }
  }
  __syncthreads();
  auto qidx = [side](int r, int c) { return (r * side + c) >> 1; };
  for (int site = threadIdx.x; site < nstab; site += blockDim.x) {
    int r, c, bit;
    if (site < nstar) {
      r = 2 * (site / L) + 1; c = 2 * (site % L); bit = 2;      // stars see z parts
    } else {
      const int k = site - nstar;
      r = 2 * (k / (L - 1)); c = 2 * (k % (L - 1)) + 1; bit = 1;  // plaquettes see x parts
    }
    int par = 0;
    if (r > 0) par ^= (err[qidx(r - 1, c)] & bit) != 0;
    if (r < side - 1) par ^= (err[qidx(r + 1, c)] & bit) != 0;
    if (c > 0) par ^= (err[qidx(r, c - 1)] & bit) != 0;
    if (c < side - 1) par ^= (err[qidx(r, c + 1)] & bit) != 0;
    syn[site] = (uint8_t)par;
  }
  if (threadIdx.x == 0) {
    int bx = 0, bz = 0;
    for (int r = 0; r < side; r += 2) bx ^= err[qidx(r, 0)] & 1;
    for (int c = 0; c < side; c += 2) bz ^= (err[qidx(0, c)] >> 1) & 1;
    *true_class = (uint8_t)(bx + 2 * bz);
  }
  if (errors)
    for (int q = threadIdx.x; q < nq; q += blockDim.x) errors[q] = err[q];
}

__global__ void __launch_bounds__(256) sample_kernel(int L, int noise, uint32_t threshold,
                                                     uint32_t k0,
                                                     uint32_t k1, const uint32_t* __restrict__ ids,
                                                     uint32_t id_base, int64_t n,
                                                     uint8_t* __restrict__ syn,
                                                     uint8_t* __restrict__ true_class,
                                                     uint8_t* __restrict__ errors) {
  __shared__ uint8_t err[SAMPLE_MAX_NQ + 1];
  const int64_t smp = blockIdx.x;
  if (smp >= n) return;
  const uint32_t sid = ids ? ids[smp] : id_base + (uint32_t)smp;
  const int nq = 2 * L * L - 2 * L + 1;
  const int nstab = 2 * L * (L - 1);
  sample_one(L, noise, threshold, k0, k1, sid, err, syn + smp * nstab, true_class + smp,
             errors ? errors + smp * nq : nullptr);
}

__global__ void __launch_bounds__(256) sample_items_kernel(const ItemDesc* __restrict__ items,
                                                           const GroupDesc* __restrict__ groups,
                                                           int64_t n, uint32_t k0, uint32_t k1,
                                                           uint8_t* __restrict__ syn,
                                                           uint8_t* __restrict__ true_class) {
  __shared__ uint8_t err[SAMPLE_MAX_NQ + 1];
  const int64_t smp = blockIdx.x;
  if (smp >= n) return;
  const ItemDesc it = items[smp];
  sample_one(groups[it.group].L, it.noise, it.err_thr, k0, k1, it.sid, err, syn + it.syn_off,
             true_class + it.orig, nullptr);
}

hipError_t launch_sample_items(const ItemDesc* items, const GroupDesc* groups, int64_t n,
                               uint32_t k0, uint32_t k1, uint8_t* syn, uint8_t* true_class,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(sample_items_kernel, dim3((unsigned)n), dim3(256), 0, s, items, groups, n, k0,
                     k1, syn, true_class);
  return hipGetLastError();
}

hipError_t launch_sample(int L, int noise, uint32_t threshold, uint32_t k0, uint32_t k1,
                         const uint32_t* ids, uint32_t id_base, int64_t n, uint8_t* syn,
                         uint8_t* true_class, uint8_t* errors, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)n), dim3(256), 0, s, L, noise, threshold, k0,
                     k1, ids,
                     id_base, n, syn, true_class, errors);
  return hipGetLastError();
}

}  // namespace mcmc

namespace mcmc {

// ---------------------------------------------------------------------------
// Matching start (Sec. III, Sec. IV): each class's chain starts from a low-
// weight configuration of that class, built per anyon type by a greedy
// matching and a cheapest parity change ("enhanced" matching).
//
// Per type: distances are Manhattan |di| + |dj|; boundary distance j+1 or
// L-1-j (plaquettes, left/right), i+1 or L-1-i (stars, top/bottom), nearer
// side first, ties to left/top.  For d = 1, 2, ...: each free anyon a in
// row-major order takes the first free b > a (row-major) at distance d, else
// its boundary if that is at distance d.  The class parity of the type is
// the number of left/top boundary matches mod 2; the other parity comes from
// the cheapest single change, searched over boundary matches (switch side)
// and then pairs (split into one left/top and one right/bottom match), first
// minimum winning; with no anyon it is the logical string.  Paths: plaquette
// pair: X on (2i1, 2j+2) for j between j1 and j2, then (2i+1, 2j2+1) for
// i1 <= i < i2; star pair: Z on (2i+2, 2j1) for i1 <= i < i2, then
// (2i2+1, 2j+1) for j between j1 and j2.
//
// One thread per syndrome; working bit-rows (one bit per qubit of a grid row)
// live in LDS, [row][thread] so that lanes hit distinct banks.
// ---------------------------------------------------------------------------
constexpr int MATCH_THREADS = 64;
constexpr int MATCH_R = 2 * MCMC_L_MAX - 1;

struct MatchLds {
  uint32_t plane[4][MATCH_R][MATCH_THREADS];  // x base, x flipped, z base, z flipped
  uint32_t freem[MCMC_L_MAX][MATCH_THREADS];
};

__device__ __forceinline__ void toggle_bits(uint32_t (*pl)[MATCH_THREADS], int row, int lo, int hi,
                                            int tid) {
  // toggle fields lo..hi-1 of grid row `row`
  if (hi > lo) pl[row][tid] ^= ((hi >= 32 ? 0u : (1u << hi)) - 1u) ^ ((1u << lo) - 1u);
}

// XOR the boundary string of anyon (i, j) on `side` into plane pl.
__device__ __forceinline__ void paint_boundary(uint32_t (*pl)[MATCH_THREADS], int L, bool star,
                                               int i, int j, int side, int tid) {
  if (!star) {
    if (side == 0) toggle_bits(pl, 2 * i, 0, j + 1, tid);
    else toggle_bits(pl, 2 * i, j + 1, L, tid);
  } else {
    const int r0 = side == 0 ? 0 : i + 1, r1 = side == 0 ? i + 1 : L;
    for (int k = r0; k < r1; ++k) pl[2 * k][tid] ^= 1u << j;
  }
}

__device__ __forceinline__ void paint_pair(uint32_t (*pl)[MATCH_THREADS], bool star, int i1, int j1,
                                           int i2, int j2, int tid) {
  const int jl = j1 < j2 ? j1 : j2, jh = j1 < j2 ? j2 : j1;
  if (!star) {
    toggle_bits(pl, 2 * i1, jl + 1, jh + 1, tid);             // (2i1, 2j+2), jl <= j < jh
    for (int i = i1; i < i2; ++i) pl[2 * i + 1][tid] ^= 1u << j2;  // (2i+1, 2j2+1)
  } else {
    for (int i = i1; i < i2; ++i) pl[2 * i + 2][tid] ^= 1u << j1;  // (2i+2, 2j1)
    toggle_bits(pl, 2 * i2 + 1, jl, jh, tid);                 // (2i2+1, 2j+1), jl <= j < jh
  }
}

__global__ void __launch_bounds__(MATCH_THREADS) init_matching_kernel(const StartArgs a) {
  __shared__ MatchLds sh;
  const int tid = threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * MATCH_THREADS + tid;
  if (s >= a.n) return;
  const StartItem si = start_item(a, s);
  const int L = si.L;
  const int R = 2 * L - 1;
  const int nstar = L * (L - 1);
  const uint8_t* sy = si.sy;
  for (int p = 0; p < 4; ++p)
    for (int r = 0; r < R; ++r) sh.plane[p][r][tid] = 0u;

  int base_par[2];
  for (int t = 0; t < 2; ++t) {  // t = 0: plaquettes (x parts), t = 1: stars (z parts)
    const bool star = t == 1;
    const int nr = star ? L - 1 : L, nc = star ? L : L - 1;
    const int off = star ? 0 : nstar;
    uint32_t (*base)[MATCH_THREADS] = sh.plane[2 * t];
    uint32_t (*flip)[MATCH_THREADS] = sh.plane[2 * t + 1];
    bool any_free = false;
    for (int i = 0; i < nr; ++i) {
      uint32_t m = 0;
      for (int j = 0; j < nc; ++j) m |= (uint32_t)(sy[off + i * nc + j] != 0) << j;
      sh.freem[i][tid] = m;
      any_free |= m != 0;
    }
    auto sd = [&](int i, int j, int side) {
      return star ? (side == 0 ? i + 1 : L - 1 - i) : (side == 0 ? j + 1 : L - 1 - j);
    };
    int left = 0;
    // best parity change: boundary kind (a, side) and pair kind (a, b, option)
    int bb_delta = 1 << 30, bb_i = -1, bb_j = 0, bb_side = 0;
    int bp_delta = 1 << 30, bp_i1 = -1, bp_j1 = 0, bp_i2 = 0, bp_j2 = 0, bp_opt = 0;
    for (int d = 1; any_free; ++d) {
      for (int i = 0; i < nr; ++i) {
        int j = -1;
        while (true) {
          const uint32_t cur = sh.freem[i][tid];
          const uint32_t m = (j + 1 >= 32) ? 0u : (cur & (~0u << (j + 1)));
          if (!m) break;
          j = __builtin_ctz(m);
          // first free partner b > a at distance d
          int bi = -1, bj = -1;
          if (j + d < nc && ((cur >> (j + d)) & 1u)) {
            bi = i; bj = j + d;
          } else {
            for (int di = 1; di <= d && i + di < nr; ++di) {
              const uint32_t rm = sh.freem[i + di][tid];
              const int dj = d - di;
              if (dj > 0) {
                if (j - dj >= 0 && ((rm >> (j - dj)) & 1u)) { bi = i + di; bj = j - dj; break; }
                if (j + dj < nc && ((rm >> (j + dj)) & 1u)) { bi = i + di; bj = j + dj; break; }
              } else if ((rm >> j) & 1u) {
                bi = i + di; bj = j; break;
              }
            }
          }
          if (bi >= 0) {
            sh.freem[i][tid] &= ~(1u << j);
            sh.freem[bi][tid] &= ~(1u << bj);
            paint_pair(base, star, i, j, bi, bj, tid);
            for (int opt = 0; opt < 2; ++opt) {
              const int delta = sd(i, j, opt) + sd(bi, bj, 1 - opt) - d;
              if (delta < bp_delta) {
                bp_delta = delta; bp_i1 = i; bp_j1 = j; bp_i2 = bi; bp_j2 = bj; bp_opt = opt;
              }
            }
          } else {
            const int dn0 = sd(i, j, 0), dn1 = sd(i, j, 1);
            const int side = dn0 <= dn1 ? 0 : 1;
            if ((side == 0 ? dn0 : dn1) == d) {
              sh.freem[i][tid] &= ~(1u << j);
              paint_boundary(base, L, star, i, j, side, tid);
              left += side == 0;
              const int delta = (side == 0 ? dn1 - dn0 : dn0 - dn1);
              if (delta < bb_delta) { bb_delta = delta; bb_i = i; bb_j = j; bb_side = side; }
            }
          }
        }
      }
      any_free = false;
      for (int i = 0; i < nr; ++i) any_free |= sh.freem[i][tid] != 0;
    }
    base_par[t] = left & 1;
    // flipped parity = base xor the cheapest change
    for (int r = 0; r < R; ++r) flip[r][tid] = base[r][tid];
    if (bb_i >= 0 && (bp_i1 < 0 || bb_delta <= bp_delta)) {
      paint_boundary(flip, L, star, bb_i, bb_j, bb_side, tid);
      paint_boundary(flip, L, star, bb_i, bb_j, 1 - bb_side, tid);
    } else if (bp_i1 >= 0) {
      paint_pair(flip, star, bp_i1, bp_j1, bp_i2, bp_j2, tid);
      paint_boundary(flip, L, star, bp_i1, bp_j1, bp_opt, tid);
      paint_boundary(flip, L, star, bp_i2, bp_j2, 1 - bp_opt, tid);
    } else if (!star) {
      toggle_bits(flip, 0, 0, L, tid);                          // X-bar: row 0
    } else {
      for (int k = 0; k < L; ++k) flip[2 * k][tid] ^= 1u;       // Z-bar: column 0
    }
  }

  const int W = words_per_row(L);
  const int nq = 2 * L * L - 2 * L + 1, side_len = 2 * L - 1;
  for (int cls = 0; cls < 4; ++cls) {
    uint32_t (*xp)[MATCH_THREADS] = sh.plane[((cls & 1) == base_par[0]) ? 0 : 1];
    uint32_t (*zp)[MATCH_THREADS] = sh.plane[((cls >> 1) == base_par[1]) ? 2 : 3];
    const int64_t sc = si.orig * 4 + cls;
    int weight = 0;
    for (int r = 0; r < R; ++r) {
      const int fields = (r & 1) ? L - 1 : L;
      const uint32_t xb = xp[r][tid], zb = zp[r][tid];
      const uint32_t valid = fields >= 32 ? ~0u : ((1u << fields) - 1u);
      weight += si.noise ? __builtin_popcount(xb & valid) + __builtin_popcount(zb & valid)
                        : __builtin_popcount((xb | zb) & valid);
      if (a.rows) {
        for (int w = 0; w < W; ++w) {
          uint32_t word = 0;
          for (int f = 0; f < 16; ++f) {
            const int k = 16 * w + f;
            const uint32_t code = k < fields ? (((xb >> k) & 1u) | (((zb >> k) & 1u) << 1)) : 3u;
            word |= code << (2 * f);
          }
          a.rows[si.rows_off + (r * W + w) * 4 + cls] = word;
        }
      }
      if (a.bytes) {
        // first qubit of row r: (r * side_len + (r & 1)) / 2
        uint8_t* out = a.bytes + sc * nq + (r * side_len + (r & 1)) / 2;
        for (int k = 0; k < fields; ++k)
          out[k] = (uint8_t)(((xb >> k) & 1u) | (((zb >> k) & 1u) << 1));
      }
    }
    if (a.weights) a.weights[sc] = weight;
  }
}

hipError_t launch_init_matching(const StartArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(init_matching_kernel,
                     dim3((unsigned)((a.n + MATCH_THREADS - 1) / MATCH_THREADS)),
                     dim3(MATCH_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_mode(uint32_t init, const StartArgs& a, hipStream_t s, bool may_create) {
  if (init == MCMC_INIT_MWPM) return launch_init_mwpm(a, s, may_create);
  if (init == MCMC_INIT_MATCHING) return launch_init_matching(a, s);
  return launch_init(a, s);
}

}  // namespace mcmc
