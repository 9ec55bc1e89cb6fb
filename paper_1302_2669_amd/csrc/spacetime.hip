// Imperfect stabilizer measurements (Sec. VI): Metropolis chains over
// space-time hypotheses with energy n + xi m.
//
// A hypothesis of T measurement rounds holds the depolarizing data error E_t
// of every interval t = 0..T-1 and the wrong outcomes M_t of every round
// t < T-1 (the last round is perfect).  Round t reports
// s_t = syn(E_0 ... E_t) xor M_t.  Moves that keep every s_t and the class of
// the accumulated error:
//   spatial (t, k): stabilizer k applied to E_t;
//   time (t, q, P), t < T-1: Pauli P (X or Z) applied to qubit q in E_t and
//     E_{t+1}, and M_t toggled on the stabilizers that anticommute with P on
//     q (its plaquettes for X, its stars for Z) -- Sec. VI's deformation.
// A sweep takes every spatial move (t, then site order) and then every time
// move (t, q, X before Z).  Move (t, k) uses draw d = t n_stab + k, move
// (t, q, P) d = T n_stab + 2 t (n_q + 1) + 2 q + (P == Z): two draws per
// round are skipped so that every round starts a Philox block.  Draw d is
// word d & 3 at counter (d >> 2, sweep, syndrome_id,
// 3<<30 | cls<<28 | 1<<20 | chain).  n and m are summed after each half of a
// counted sweep.
//
// Mapping.  One lane per chain.  A hypothesis is T (2 n_q)-bit data planes
// (16 qubits per word, qubit order) and T-1 n_stab-bit outcome planes: far
// more state than registers hold, so it lives in a global buffer, word-major
// over all chains (a wave's access to one word is one 256-byte line).  Moves
// run in the exact sequential order above, so the chains are bit-identical to
// a sequential implementation.
//
// For L <= ST_FAST_L_MAX a kernel templated on L keeps the words of the
// current interval (spatial half) or of intervals t, t+1 and round t's
// outcomes (time half) in registers, where every qubit, site and stabilizer
// index is a compile-time constant; the buffer is then read and written once
// per interval.  Larger codes run a templated kernel that keeps only a
// streaming window of those words in registers (spacetime_win.h).  Neither
// holds hypotheses in LDS, so occupancy is set by registers alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spacetime_common.h"

namespace mcmc {
namespace {

constexpr uint32_t ST_NONE = 0xFFFFu;
constexpr int ST_SAMPLE_NQ = 2048;   // accumulated-error bytes of the sampler
constexpr int ST_FAST_L_MAX = SPACETIME_FAST_L_MAX;
static_assert(2 * MCMC_L_MAX * MCMC_L_MAX - 2 * MCMC_L_MAX + 1 <= ST_SAMPLE_NQ,
              "sampler buffer holds every qubit of the largest code");
static_assert(2 * MCMC_L_MAX * MCMC_L_MAX - 2 * MCMC_L_MAX + 1 < (int)ST_NONE,
              "qubit and stabilizer indices fit the 16-bit table entries");

__device__ __forceinline__ uint32_t pack2(uint32_t lo, uint32_t hi) { return lo | (hi << 16); }

// ---- sampler ----------------------------------------------------------------
// Interval t: the depolarizing rule of the single-round sampler with counter
// word 1 = 1 + t; round t < T-1: outcome k wrong iff word k & 3 of Philox at
// (k >> 2, 0x80000000 | t, id, 1<<30) is below floor(p_M 2^32).
__global__ void __launch_bounds__(256) st_sample_kernel(int L, int T, uint32_t thr_d,
                                                        uint32_t thr_m, uint32_t k0, uint32_t k1,
                                                        uint32_t id_base, int64_t n,
                                                        uint8_t* __restrict__ obs,
                                                        uint8_t* __restrict__ true_class) {
  __shared__ uint8_t acc[ST_SAMPLE_NQ];  // accumulated error of the sample
  const int64_t smp = blockIdx.x;
  if (smp >= n) return;
  const uint32_t sid = id_base + (uint32_t)smp;
  const int side = 2 * L - 1;
  const int nq = 2 * L * L - 2 * L + 1;
  const int nstab = 2 * L * (L - 1);
  const int nstar = L * (L - 1);
  for (int q = threadIdx.x; q < nq; q += blockDim.x) acc[q] = 0;
  __syncthreads();
  for (int t = 0; t < T; ++t) {
    for (int pr = threadIdx.x; pr < (nq + 1) / 2; pr += blockDim.x) {
      const uint4 w = philox4x32_10(make_uint4((uint32_t)pr, (uint32_t)(1 + t), sid, 1u << 30),
                                    k0, k1);
      for (int h = 0; h < 2; ++h) {
        const int q = 2 * pr + h;
        if (q >= nq) break;
        const uint32_t u0 = h ? w.z : w.x;
        const uint32_t u1 = h ? w.w : w.y;
        const uint32_t type = (uint32_t)(((uint64_t)u1 * 3u) >> 32);
        const uint8_t code = (uint8_t)(type == 0 ? 1 : (type == 1 ? 3 : 2));
        if (u0 < thr_d) acc[q] ^= code;
      }
    }
    __syncthreads();
    uint8_t* o = obs + (smp * T + t) * nstab;
    for (int k = threadIdx.x; k < nstab; k += blockDim.x) {
      int r, c, bit;
      if (k < nstar) {
        r = 2 * (k / L) + 1; c = 2 * (k % L); bit = 2;
      } else {
        const int kk = k - nstar;
        r = 2 * (kk / (L - 1)); c = 2 * (kk % (L - 1)) + 1; bit = 1;
      }
      int par = 0;
      if (r > 0) par ^= (acc[((r - 1) * side + c) >> 1] & bit) != 0;
      if (r < side - 1) par ^= (acc[((r + 1) * side + c) >> 1] & bit) != 0;
      if (c > 0) par ^= (acc[(r * side + c - 1) >> 1] & bit) != 0;
      if (c < side - 1) par ^= (acc[(r * side + c + 1) >> 1] & bit) != 0;
      if (t < T - 1) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)(k >> 2), 0x80000000u | (uint32_t)t,
                                                 sid, 1u << 30), k0, k1);
        par ^= word_of(w, k & 3) < thr_m;
      }
      o[k] = (uint8_t)par;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int bx = 0, bz = 0;
    for (int r = 0; r < side; r += 2) bx ^= acc[(r * side) >> 1] & 1;
    for (int c = 0; c < side; c += 2) bz ^= (acc[c >> 1] >> 1) & 1;
    true_class[smp] = (uint8_t)(bx + 2 * bz);
  }
}

// ---- class starts: the perfect last round of every history -------------------
__global__ void __launch_bounds__(256) st_last_kernel(int64_t n, int T, int nstab,
                                                      const uint8_t* __restrict__ obs,
                                                      uint8_t* __restrict__ last) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nstab) return;
  const int64_t h = i / nstab;
  last[i] = obs[(h * T + (T - 1)) * nstab + (i - h * nstab)] != 0;
}

// ---- chains, register-resident intervals (small codes) -----------------------
template <int L>
// 8 waves per SIMD (64 registers), the most a SIMD holds: the move sequence is
// latency-bound (Philox chains, table loads), and more resident waves hide
// more of it than the extra spills cost (measured at L = 7: 4.9e11 moves/s
// against 4.3e11 at 4 waves).  The spills are stores in the move sequences
// whose values are read back only after the last sweep.
__global__ void __launch_bounds__(ST_LANES) __attribute__((amdgpu_waves_per_eu(8)))
st_chain_fast_kernel(const SpaceTimeArgs a) {
  using G = StGeo<L>;
  constexpr int NQ = G::NQ, NSTAB = G::NSTAB, NSTAR = G::NSTAR, WQ = G::WQ, WM = G::WM;
  __shared__ uint32_t tthr[32];                     // [25] time-move thresholds
  __shared__ uint32_t sthr[4];                      // spatial thresholds
  const int T = a.T;
  const int lane = threadIdx.x;
  if (lane < 25) tthr[lane] = a.t_thr[lane];
  if (lane < 4) sthr[lane] = a.sp_thr[lane];
  __syncthreads();

  const int64_t task = (int64_t)blockIdx.x * ST_LANES + lane;
  if (task >= a.n_tasks) return;
  // the hypothesis in global memory, word-major over all chains (coalesced):
  // it is read and written once per interval, not per move
  const int64_t stride = a.n_tasks;
  uint32_t* Ew = a.state + task;                        // [T*WQ][stride]
  uint32_t* Mw = Ew + (int64_t)T * WQ * stride;         // [(T-1)*WM][stride]
  const StTask tk = st_task(a, task);
  const uint32_t sid = tk.sid;
  int32_t n = 0, m = 0;
  st_start(a, tk, NQ, NSTAB, WQ, WM, Ew, Mw, stride, n, m);

  const uint32_t ctr3 = (3u << 30) | ((uint32_t)tk.cls << 28) | (1u << 20) | (uint32_t)tk.chain;
  const uint32_t always = a.t_always;
  int64_t Sn = 0, Sm = 0, Acnt = 0;
  for (int sweep = 0; sweep < a.sweep_end; ++sweep) {
    const bool counted = sweep >= a.burn;
    // spatial half: interval t in registers
    for (int t = 0; t < T; ++t) {
      uint32_t e[WQ];
#pragma unroll
      for (int w = 0; w < WQ; ++w) e[w] = Ew[(t * WQ + w) * stride];
      const uint32_t blk0 = (uint32_t)(t * (NSTAB / 4));
      uint4 blk = make_uint4(0, 0, 0, 0);
      // accepted moves of this interval, in a fenced 32-bit counter: left as
      // a 64-bit sum the compiler defers and spills every move's flag
      uint32_t na = 0;
      static_for<NSTAB>([&](auto SS) {
        constexpr int s = decltype(SS)::value;
        constexpr bool star = s < NSTAR;
        if constexpr ((s & 3) == 0) {
          blk = philox4x32_10(
              make_uint4(st_opaque(blk0 + (uint32_t)(s / 4)), (uint32_t)sweep, sid, ctr3), a.k0,
              a.k1);
        }
        const uint32_t u = word_of(blk, s & 3);
        int delta = 0;
        static_for<4>([&](auto KK) {
          constexpr int q = G::site_qubit(s, decltype(KK)::value);
          if constexpr (q >= 0) {
            const uint32_t code = (e[q >> 4] >> (2 * (q & 15))) & 3u;
            const int x = (int)(code & 1u), z = (int)(code >> 1);
            delta += star ? (1 - z) * (1 - 2 * x) : (1 - x) * (1 - 2 * z);
          }
        });
        // threshold by table lookup and both tests evaluated (no select chain,
        // no short circuit): a branch per move would split the unrolled sweep
        // into thousands of exec-masked blocks; (delta - 1) & 3 stays in the
        // table for delta <= 0, where the lookup is not used
        const bool acc = (delta <= 0) | (u < sthr[(delta - 1) & 3]);
        const uint32_t flip = acc ? (star ? 1u : 2u) : 0u;
        static_for<4>([&](auto KK) {
          constexpr int q = G::site_qubit(s, decltype(KK)::value);
          if constexpr (q >= 0) e[q >> 4] ^= flip << (2 * (q & 15));
        });
        n += acc ? delta : 0;
        na += acc ? 1u : 0u;
        st_fence(e);
        asm volatile("" : "+v"(n), "+v"(na));
      });
      Acnt += na;
#pragma unroll
      for (int w = 0; w < WQ; ++w) Ew[(t * WQ + w) * stride] = e[w];
    }
    if (counted) { Sn += n; Sm += m; }
    // time half: intervals t, t+1 and round t's outcomes in registers
    for (int t = 0; t + 1 < T; ++t) {
      uint32_t e0[WQ], e1[WQ], mm[WM];
#pragma unroll
      for (int w = 0; w < WQ; ++w) {
        e0[w] = Ew[(t * WQ + w) * stride];
        e1[w] = Ew[((t + 1) * WQ + w) * stride];
      }
#pragma unroll
      for (int w = 0; w < WM; ++w) mm[w] = Mw[(t * WM + w) * stride];
      const uint32_t blk0 = (uint32_t)((T * NSTAB + 2 * t * (NQ + 1)) / 4);
      uint4 blk = make_uint4(0, 0, 0, 0);
      uint32_t na = 0;   // accepted moves of this round, as above
      static_for<2 * NQ>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        constexpr int q = r >> 1, kind = r & 1;
        constexpr int w = q >> 4, sh = 2 * (q & 15);
        if constexpr ((r & 3) == 0) {
          blk = philox4x32_10(
              make_uint4(st_opaque(blk0 + (uint32_t)(r / 4)), (uint32_t)sweep, sid, ctr3), a.k0,
              a.k1);
        }
        const uint32_t u = word_of(blk, r & 3);
        const uint32_t c0 = (e0[w] >> sh) & 3u, c1 = (e1[w] >> sh) & 3u;
        int dn;
        if constexpr (kind == 0)
          dn = (1 - (int)(c0 >> 1)) * (1 - 2 * (int)(c0 & 1u)) +
               (1 - (int)(c1 >> 1)) * (1 - 2 * (int)(c1 & 1u));
        else
          dn = (1 - (int)(c0 & 1u)) * (1 - 2 * (int)(c0 >> 1)) +
               (1 - (int)(c1 & 1u)) * (1 - 2 * (int)(c1 >> 1));
        constexpr int sa = G::qubit_stab(q, kind, 0), sb = G::qubit_stab(q, kind, 1);
        int dm = 0;
        if constexpr (sa >= 0) dm += 1 - 2 * (int)((mm[sa >> 5] >> (sa & 31)) & 1u);
        if constexpr (sb >= 0) dm += 1 - 2 * (int)((mm[sb >> 5] >> (sb & 31)) & 1u);
        const int ei = (dn + 2) * 5 + (dm + 2);
        const bool acc = (((always >> ei) & 1u) != 0) | (u < tthr[ei]);
        const uint32_t fl = acc ? (uint32_t)(kind == 0 ? 1u : 2u) << sh : 0u;
        e0[w] ^= fl;
        e1[w] ^= fl;
        if constexpr (sa >= 0) mm[sa >> 5] ^= (acc ? 1u : 0u) << (sa & 31);
        if constexpr (sb >= 0) mm[sb >> 5] ^= (acc ? 1u : 0u) << (sb & 31);
        n += acc ? dn : 0;
        m += acc ? dm : 0;
        na += acc ? 1u : 0u;
        st_fence(e0);
        st_fence(e1);
        st_fence(mm);
        asm volatile("" : "+v"(n), "+v"(m), "+v"(na));
      });
      Acnt += na;
#pragma unroll
      for (int w = 0; w < WQ; ++w) {
        Ew[(t * WQ + w) * stride] = e0[w];
        Ew[((t + 1) * WQ + w) * stride] = e1[w];
      }
#pragma unroll
      for (int w = 0; w < WM; ++w) Mw[(t * WM + w) * stride] = mm[w];
    }
    if (counted) { Sn += n; Sm += m; }
  }
  st_finish(a, tk, NQ, WQ, Ew, stride, Sn, Sm, Acnt, n, m);
}

// ---- estimator --------------------------------------------------------------
#pragma clang fp contract(off)
__global__ void __launch_bounds__(128) st_decide_kernel(const SpaceTimeArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int C = a.chains, L = a.L, T = a.T;
  const int sweeps = a.sweep_end - a.burn;
  const bool counted = sweeps > 0;
  const double denom = counted ? (double)((int64_t)C * 2 * sweeps) : (double)C;
  const double nq = (double)(2 * L * L - 2 * L + 1), nstab = (double)(2 * L * (L - 1));
  const double f0 = 0.75 * nq * (double)T + a.xi * (0.5 * nstab * (double)(T - 1));
  double key[4], logz[4];
  for (int e = 0; e < 4; ++e) {
    int64_t sn = 0, sm = 0;
    for (int c = 0; c < C; ++c) {
      const int64_t k = (i * 4 + e) * C + c;
      sn += counted ? a.Sn[k] : (int64_t)a.n_final[k];
      sm += counted ? a.Sm[k] : (int64_t)a.m_final[k];
    }
    key[e] = (double)sn + a.xi * (double)sm;
    logz[e] = -((a.beta_bar / 2.0) * (f0 + key[e] / denom));
    if (a.mean_n) a.mean_n[i * 4 + e] = (double)sn / denom;
    if (a.mean_m) a.mean_m[i * 4 + e] = (double)sm / denom;
  }
  double mx = logz[0];
  for (int e = 1; e < 4; ++e) mx = logz[e] > mx ? logz[e] : mx;
  double ex[4];
  for (int e = 0; e < 4; ++e) ex[e] = exp(logz[e] - mx);
  const double tot = ((ex[0] + ex[1]) + ex[2]) + ex[3];
  for (int e = 0; e < 4; ++e) a.class_prob[i * 4 + e] = ex[e] / tot;
  int best = 0;
  for (int e = 1; e < 4; ++e)
    if (key[e] < key[best]) best = e;
  a.chosen[i] = (uint8_t)best;
  if (a.correction) {
    const int nqi = 2 * L * L - 2 * L + 1;
    const uint8_t* src = a.final_c + (i * 4 + best) * nqi;
    for (int q = 0; q < nqi; ++q) a.correction[i * nqi + q] = src[q];
  }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_spacetime_sample(int L, int T, uint32_t thr_d, uint32_t thr_m, uint32_t k0,
                                   uint32_t k1, uint32_t id_base, int64_t n, uint8_t* obs,
                                   uint8_t* true_class, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(st_sample_kernel, dim3((unsigned)n), dim3(256), 0, s, L, T, thr_d, thr_m, k0,
                     k1, id_base, n, obs, true_class);
  return hipGetLastError();
}

hipError_t launch_spacetime_last(int64_t n, int T, int nstab, const uint8_t* obs, uint8_t* last,
                                 hipStream_t s) {
  const int64_t total = n * nstab;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(st_last_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, n, T, nstab,
                     obs, last);
  return hipGetLastError();
}

namespace {

template <int L>
hipError_t launch_fast(const SpaceTimeArgs& a, hipStream_t s) {
  if (!a.state) return hipErrorInvalidValue;
  hipLaunchKernelGGL(st_chain_fast_kernel<L>, dim3(blocks_for(a.n_tasks, ST_LANES)),
                     dim3(ST_LANES), 0, s, a);
  return hipGetLastError();
}

template <int LL>
hipError_t dispatch_window(const SpaceTimeArgs& a, hipStream_t s) {
  if constexpr (LL > SPACETIME_WIN_L_MAX) {
    return hipErrorInvalidValue;
  } else {
    if (a.L == LL) return launch_spacetime_win_L<LL>(a, s);
    return dispatch_window<LL + 1>(a, s);
  }
}

template <int LL>
hipError_t dispatch_fast(const SpaceTimeArgs& a, hipStream_t s) {
  if constexpr (LL > ST_FAST_L_MAX) {
    return hipErrorInvalidValue;
  } else {
    if (a.L == LL) return launch_fast<LL>(a, s);
    return dispatch_fast<LL + 1>(a, s);
  }
}

}  // namespace

hipError_t launch_spacetime_chains(const SpaceTimeArgs& a, hipStream_t s) {
  if (a.n_tasks == 0) return hipSuccess;
  if (a.L <= ST_FAST_L_MAX) return dispatch_fast<2>(a, s);
  return dispatch_window<SPACETIME_WIN_L_MIN>(a, s);
}

hipError_t launch_spacetime_decide(const SpaceTimeArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(st_decide_kernel, dim3(blocks_for(a.n, 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

}  // namespace mcmc
