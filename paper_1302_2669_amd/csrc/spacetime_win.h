// Space-time chains (Sec. VI) for mid-size codes with a streaming window of
// registers: the moves run in the same sequential order as every other
// space-time kernel (a sweep: every spatial move, interval by interval in
// site order, then every time move, round by round, qubit by qubit, X before
// Z; draws as in spacetime.hip), unrolled with every qubit, site and
// stabilizer index a compile-time constant, as in the register-interval
// kernel for small codes.  What differs is how much of the hypothesis is in
// registers at once: each state word is loaded a few moves before the first
// move that reads it and stored right after the last move that writes it, so
// only the words of a few grid rows are live (the stars of one row touch
// three grid rows; a run of time moves touches one data word of each of the
// two intervals and the outcome words of the neighbouring stabilizers).  The
// interval's data words are streamed twice in the spatial half (once for the
// star moves, once for the plaquette moves, which start again at row 0).
// Each code size is instantiated in a translation unit of its own
// (spacetime_win_<L>.hip), so that the builds run in parallel.
#pragma once

#include "spacetime_common.h"

namespace mcmc {

namespace {

// words are loaded this many moves before their first use
constexpr int ST_PREFETCH = 24;

// Per-move load and store masks of the two halves of a sweep: bit w of word
// w >> 6 for state word w.
template <int L>
struct StWindow {
  using G = StGeo<L>;
  static constexpr int NQ = G::NQ, NSTAB = G::NSTAB, NSTAR = G::NSTAR, WQ = G::WQ, WM = G::WM;
  static_assert(WQ <= 128 && WM <= 128, "word masks are 128 bits");

  struct Spatial {
    uint64_t load[NSTAB][2], store[NSTAB][2];
  };
  static constexpr Spatial spatial() {
    Spatial r{};
    for (int s = 0; s < NSTAB; ++s) r.load[s][0] = r.load[s][1] = r.store[s][0] = r.store[s][1] = 0;
    for (int pass = 0; pass < 2; ++pass) {   // stars, then plaquettes
      const int s0 = pass == 0 ? 0 : NSTAR, s1 = pass == 0 ? NSTAR : NSTAB;
      int first[128] = {}, last[128] = {};
      for (int w = 0; w < WQ; ++w) first[w] = last[w] = -1;
      for (int s = s0; s < s1; ++s)
        for (int k = 0; k < 4; ++k) {
          const int q = G::site_qubit(s, k);
          if (q < 0) continue;
          if (first[q >> 4] < 0) first[q >> 4] = s;
          last[q >> 4] = s;
        }
      for (int w = 0; w < WQ; ++w) {
        if (first[w] < 0) continue;
        const int at = first[w] - ST_PREFETCH < s0 ? s0 : first[w] - ST_PREFETCH;
        r.load[at][w >> 6] |= 1ull << (w & 63);
        r.store[last[w]][w >> 6] |= 1ull << (w & 63);
      }
    }
    return r;
  }

  struct Time {
    uint64_t load_e[2 * NQ][2], store_e[2 * NQ][2], load_m[2 * NQ][2], store_m[2 * NQ][2];
  };
  static constexpr Time time() {
    Time r{};
    for (int i = 0; i < 2 * NQ; ++i)
      for (int h = 0; h < 2; ++h) r.load_e[i][h] = r.store_e[i][h] = r.load_m[i][h] = r.store_m[i][h] = 0;
    // data word w: moves 32 w .. 32 w + 31 (qubits 16 w .. 16 w + 15, X and Z)
    for (int w = 0; w < WQ; ++w) {
      const int first = 32 * w, last = 32 * w + 31 < 2 * NQ - 1 ? 32 * w + 31 : 2 * NQ - 1;
      r.load_e[first - ST_PREFETCH < 0 ? 0 : first - ST_PREFETCH][w >> 6] |= 1ull << (w & 63);
      r.store_e[last][w >> 6] |= 1ull << (w & 63);
    }
    int first[128] = {}, last[128] = {};
    for (int w = 0; w < WM; ++w) first[w] = last[w] = -1;
    for (int i = 0; i < 2 * NQ; ++i)
      for (int k = 0; k < 2; ++k) {
        const int st = G::qubit_stab(i >> 1, i & 1, k);
        if (st < 0) continue;
        if (first[st >> 5] < 0) first[st >> 5] = i;
        last[st >> 5] = i;
      }
    for (int w = 0; w < WM; ++w) {
      if (first[w] < 0) continue;
      r.load_m[first[w] - ST_PREFETCH < 0 ? 0 : first[w] - ST_PREFETCH][w >> 6] |= 1ull << (w & 63);
      r.store_m[last[w]][w >> 6] |= 1ull << (w & 63);
    }
    return r;
  }

  static constexpr Spatial SP = spatial();
  static constexpr Time TM = time();

  // The plans are sound: replaying them, every word a move reads or writes
  // is loaded and not yet stored, every word is loaded and stored once per
  // pass, and none is left loaded at a pass's end.
  static constexpr bool any(const uint64_t (&m)[2]) { return (m[0] | m[1]) != 0; }
  static constexpr bool has(const uint64_t (&m)[2], int w) { return (m[w >> 6] >> (w & 63)) & 1ull; }
  static constexpr bool spatial_sound() {
    for (int pass = 0; pass < 2; ++pass) {
      const int s0 = pass == 0 ? 0 : NSTAR, s1 = pass == 0 ? NSTAR : NSTAB;
      bool live[128] = {};
      int loads[128] = {}, stores[128] = {};
      for (int s = s0; s < s1; ++s) {
        if (any(SP.load[s]))
          for (int w = 0; w < WQ; ++w)
            if (has(SP.load[s], w)) { if (live[w]) return false; live[w] = true; ++loads[w]; }
        for (int k = 0; k < 4; ++k) {
          const int q = G::site_qubit(s, k);
          if (q >= 0 && !live[q >> 4]) return false;
        }
        if (any(SP.store[s]))
          for (int w = 0; w < WQ; ++w)
            if (has(SP.store[s], w)) { if (!live[w]) return false; live[w] = false; ++stores[w]; }
      }
      for (int w = 0; w < WQ; ++w)
        if (live[w] || loads[w] != stores[w] || loads[w] > 1) return false;
    }
    return true;
  }
  static constexpr bool time_sound() {
    bool le[128] = {}, lm[128] = {};
    for (int r = 0; r < 2 * NQ; ++r) {
      if (any(TM.load_e[r]))
        for (int w = 0; w < WQ; ++w)
          if (has(TM.load_e[r], w)) { if (le[w]) return false; le[w] = true; }
      if (any(TM.load_m[r]))
        for (int w = 0; w < WM; ++w)
          if (has(TM.load_m[r], w)) { if (lm[w]) return false; lm[w] = true; }
      if (!le[(r >> 1) >> 4]) return false;
      for (int k = 0; k < 2; ++k) {
        const int st = G::qubit_stab(r >> 1, r & 1, k);
        if (st >= 0 && !lm[st >> 5]) return false;
      }
      if (any(TM.store_e[r]))
        for (int w = 0; w < WQ; ++w)
          if (has(TM.store_e[r], w)) { if (!le[w]) return false; le[w] = false; }
      if (any(TM.store_m[r]))
        for (int w = 0; w < WM; ++w)
          if (has(TM.store_m[r], w)) { if (!lm[w]) return false; lm[w] = false; }
    }
    for (int w = 0; w < 128; ++w)
      if (le[w] || lm[w]) return false;
    return true;
  }
};

// address of word W of a plane: the index passes through a register first,
// so that the compiler computes the address where it is used instead of
// keeping every word's address live across the loops
template <int W>
__device__ __forceinline__ uint32_t* word_at(uint32_t* base, int64_t stride) {
  return base + (int64_t)st_opaque((uint32_t)W) * stride;
}

// static_for over 0..N-1 in chunks of 1024 (a fold expression per chunk:
// the compiler limits how deep one may nest)
template <int N, int B = 0, class F>
__device__ __forceinline__ void static_for_long(F&& f) {
  constexpr int CHUNK = 1024;
  if constexpr (B < N) {
    static_for<(N - B < CHUNK ? N - B : CHUNK)>(
        [&](auto I) { f(std::integral_constant<int, B + decltype(I)::value>{}); });
    static_for_long<N, B + CHUNK>(f);
  }
}

// f(W) for every word W < N whose bit is set in (LO, HI)
template <int N, uint64_t LO, uint64_t HI, class F>
__device__ __forceinline__ void for_bits(F&& f) {
  if constexpr ((LO | HI) != 0) {
    static_for<N>([&](auto W) {
      constexpr int w = decltype(W)::value;
      if constexpr ((((w < 64 ? LO : HI) >> (w & 63)) & 1ull) != 0) f(W);
    });
  }
}

template <int L>
__global__ void __launch_bounds__(ST_LANES) __attribute__((amdgpu_waves_per_eu(8)))
st_chain_win_kernel(const SpaceTimeArgs a) {
  using G = StGeo<L>;
  using P = StWindow<L>;
  static_assert(P::spatial_sound(), "spatial load/store plan");
  static_assert(P::time_sound(), "time load/store plan");
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
    // spatial half
    for (int t = 0; t < T; ++t) {
      uint32_t* E = Ew + (int64_t)t * WQ * stride;
      uint32_t e[WQ];
      const uint32_t blk0 = (uint32_t)(t * (NSTAB / 4));
      uint4 blk = make_uint4(0, 0, 0, 0);
      uint32_t na = 0;   // accepted moves, in a fenced 32-bit counter
      static_for_long<NSTAB>([&](auto SS) {
        constexpr int s = decltype(SS)::value;
        constexpr bool star = s < NSTAR;
        for_bits<WQ, P::SP.load[s][0], P::SP.load[s][1]>([&](auto W) {
          e[decltype(W)::value] = *word_at<decltype(W)::value>(E, stride);
        });
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
        const bool acc = (delta <= 0) | (u < sthr[(delta - 1) & 3]);
        const uint32_t flip = acc ? (star ? 1u : 2u) : 0u;
        static_for<4>([&](auto KK) {
          constexpr int q = G::site_qubit(s, decltype(KK)::value);
          if constexpr (q >= 0) {
            e[q >> 4] ^= flip << (2 * (q & 15));
            st_fence1(e[q >> 4]);
          }
        });
        n += acc ? delta : 0;
        na += acc ? 1u : 0u;
        asm volatile("" : "+v"(n), "+v"(na));
        for_bits<WQ, P::SP.store[s][0], P::SP.store[s][1]>([&](auto W) {
          *word_at<decltype(W)::value>(E, stride) = e[decltype(W)::value];
        });
      });
      Acnt += na;
    }
    if (counted) { Sn += n; Sm += m; }
    // time half: intervals t, t+1 and round t's outcomes
    for (int t = 0; t + 1 < T; ++t) {
      uint32_t* E0 = Ew + (int64_t)t * WQ * stride;
      uint32_t* E1 = E0 + (int64_t)WQ * stride;
      uint32_t* M = Mw + (int64_t)t * WM * stride;
      uint32_t e0[WQ], e1[WQ], mm[WM];
      const uint32_t blk0 = (uint32_t)((T * NSTAB + 2 * t * (NQ + 1)) / 4);
      uint4 blk = make_uint4(0, 0, 0, 0);
      uint32_t na = 0;
      static_for_long<2 * NQ>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        constexpr int q = r >> 1, kind = r & 1;
        constexpr int w = q >> 4, sh = 2 * (q & 15);
        for_bits<WQ, P::TM.load_e[r][0], P::TM.load_e[r][1]>([&](auto W) {
          e0[decltype(W)::value] = *word_at<decltype(W)::value>(E0, stride);
          e1[decltype(W)::value] = *word_at<decltype(W)::value>(E1, stride);
        });
        for_bits<WM, P::TM.load_m[r][0], P::TM.load_m[r][1]>([&](auto W) {
          mm[decltype(W)::value] = *word_at<decltype(W)::value>(M, stride);
        });
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
        st_fence1(e0[w]);
        st_fence1(e1[w]);
        if constexpr (sa >= 0) {
          mm[sa >> 5] ^= (acc ? 1u : 0u) << (sa & 31);
          st_fence1(mm[sa >> 5]);
        }
        if constexpr (sb >= 0) {
          mm[sb >> 5] ^= (acc ? 1u : 0u) << (sb & 31);
          st_fence1(mm[sb >> 5]);
        }
        n += acc ? dn : 0;
        m += acc ? dm : 0;
        na += acc ? 1u : 0u;
        asm volatile("" : "+v"(n), "+v"(m), "+v"(na));
        for_bits<WQ, P::TM.store_e[r][0], P::TM.store_e[r][1]>([&](auto W) {
          *word_at<decltype(W)::value>(E0, stride) = e0[decltype(W)::value];
          *word_at<decltype(W)::value>(E1, stride) = e1[decltype(W)::value];
        });
        for_bits<WM, P::TM.store_m[r][0], P::TM.store_m[r][1]>([&](auto W) {
          *word_at<decltype(W)::value>(M, stride) = mm[decltype(W)::value];
        });
      });
      Acnt += na;
    }
    if (counted) { Sn += n; Sm += m; }
  }
  st_finish(a, tk, NQ, WQ, Ew, stride, Sn, Sm, Acnt, n, m);
}

}  // namespace

template <int L>
hipError_t launch_spacetime_win_L(const SpaceTimeArgs& a, hipStream_t s) {
  if (a.n_tasks == 0) return hipSuccess;
  if (!a.state || a.L != L) return hipErrorInvalidValue;
  hipLaunchKernelGGL(st_chain_win_kernel<L>,
                     dim3((unsigned)((a.n_tasks + ST_LANES - 1) / ST_LANES)), dim3(ST_LANES), 0,
                     s, a);
  return hipGetLastError();
}

}  // namespace mcmc
