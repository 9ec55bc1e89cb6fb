// Pieces shared by the space-time chain kernels (Sec. VI): the lattice as
// compile-time tables, the compiler fences of the unrolled move sequences,
// and the per-chain set-up and outputs.  The hypothesis of a chain lives in
// a global buffer, word-major over all chains: data word w of interval t at
// Ew[(t WQ + w) stride], outcome word w of round t at Mw[(t WM + w) stride].
#pragma once

#include "device_common.h"
#include "internal.h"

namespace mcmc {

constexpr int ST_LANES = 64;

template <int L>
struct StGeo {
  static constexpr int SIDE = 2 * L - 1;
  static constexpr int NQ = 2 * L * L - 2 * L + 1;
  static constexpr int NSTAB = 2 * L * (L - 1);
  static constexpr int NSTAR = L * (L - 1);
  static constexpr int WQ = (NQ + 15) / 16;
  static constexpr int WM = (NSTAB + 31) / 32;
  // qubit k (0..3) of site s in the generic kernel's order, -1 if missing
  static constexpr int site_qubit(int s, int k) {
    int r = 0, c = 0;
    if (s < NSTAR) { r = 2 * (s / L) + 1; c = 2 * (s % L); }
    else { r = 2 * ((s - NSTAR) / (L - 1)); c = 2 * ((s - NSTAR) % (L - 1)) + 1; }
    int q[4] = {-1, -1, -1, -1};
    int n = 0;
    if (r > 0) q[n++] = ((r - 1) * SIDE + c) / 2;
    if (r < SIDE - 1) q[n++] = ((r + 1) * SIDE + c) / 2;
    if (c > 0) q[n++] = (r * SIDE + c - 1) / 2;
    if (c < SIDE - 1) q[n++] = (r * SIDE + c + 1) / 2;
    return q[k];
  }
  // stabilizer k (0..1) anticommuting with X (kind 0: plaquettes) or Z
  // (kind 1: stars) on qubit q, -1 if missing
  static constexpr int qubit_stab(int q, int kind, int k) {
    const int r = (2 * q) / SIDE, c = 2 * q - r * SIDE;
    int pl[2] = {-1, -1}, st[2] = {-1, -1};
    int np = 0, ns = 0;
    const int dr[4] = {-1, 1, 0, 0}, dc[4] = {0, 0, -1, 1};
    for (int d = 0; d < 4; ++d) {
      const int rr = r + dr[d], cc = c + dc[d];
      if (rr < 0 || rr >= SIDE || cc < 0 || cc >= SIDE) continue;
      if (rr & 1) st[ns++] = ((rr - 1) / 2) * L + cc / 2;
      else pl[np++] = NSTAR + (rr / 2) * (L - 1) + (cc - 1) / 2;
    }
    return kind == 0 ? pl[k] : st[k];
  }
};

// After a move its state words pass through an empty asm statement, and each
// Philox block index is made opaque: a flip only touches bits that the
// compiler can prove other moves do not read, so without the fences it
// extracts every move's fields from the words as loaded and keeps them all
// live (hundreds of registers, then scratch).
template <int N>
__device__ __forceinline__ void st_fence(uint32_t (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" : "+v"(x[i]));
}
__device__ __forceinline__ void st_fence1(uint32_t& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ uint32_t st_opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// The chain of task `task`: history item, position rem = cls * C + chain in
// the item's block, and the history's syndrome id.
struct StTask {
  int64_t item;
  int rem, cls, chain;
  uint32_t sid;
};
__device__ __forceinline__ StTask st_task(const SpaceTimeArgs& a, int64_t task) {
  StTask k;
  const int C = a.chains;
  k.item = task / (4 * C);
  k.rem = (int)(task - k.item * 4 * C);
  k.cls = k.rem / C;
  k.chain = k.rem % C;
  k.sid = a.ids ? a.ids[k.item] : (uint32_t)k.item;
  return k;
}

// Class start into the buffer: every flipped outcome before the last round
// blamed on the measurement (M_t = s_t), no data error before the last
// interval, and the class-cls matching start of the last round's syndrome in
// interval T-1.  Sets n and m of the start.
__device__ __forceinline__ void st_start(const SpaceTimeArgs& a, const StTask& k, int nq,
                                         int nstab, int WQ, int WM, uint32_t* Ew, uint32_t* Mw,
                                         int64_t stride, int32_t& n, int32_t& m) {
  const int T = a.T;
  n = 0;
  m = 0;
  for (int w = 0; w < (T - 1) * WQ; ++w) Ew[w * stride] = 0u;
  const uint8_t* b = a.reps + (k.item * 4 + k.cls) * nq;
  for (int w = 0; w < WQ; ++w) {
    uint32_t word = 0;
    for (int f = 0; f < 16; ++f) {
      const int q = 16 * w + f;
      if (q < nq) word |= (uint32_t)(b[q] & 3u) << (2 * f);
    }
    Ew[(int64_t)((T - 1) * WQ + w) * stride] = word;
  }
  n = a.rep_weight[k.item * 4 + k.cls];
  for (int t = 0; t + 1 < T; ++t) {
    const uint8_t* o = a.obs + (k.item * T + t) * nstab;
    for (int w = 0; w < WM; ++w) {
      uint32_t word = 0;
      for (int bit = 0; bit < 32; ++bit) {
        const int s = 32 * w + bit;
        if (s < nstab && o[s] != 0) word |= 1u << bit;
      }
      Mw[(int64_t)(t * WM + w) * stride] = word;
      m += __builtin_popcount(word);
    }
  }
}

// Per-chain outputs; chain 0 of each class also writes the accumulated data
// error of its final hypothesis (the correction candidate).
__device__ __forceinline__ void st_finish(const SpaceTimeArgs& a, const StTask& k, int nq, int WQ,
                                          const uint32_t* Ew, int64_t stride, int64_t Sn,
                                          int64_t Sm, int64_t Acnt, int32_t n, int32_t m) {
  const int64_t out = k.item * 4 * a.chains + k.rem;
  a.Sn[out] = Sn;
  a.Sm[out] = Sm;
  a.A[out] = Acnt;
  a.n_final[out] = n;
  a.m_final[out] = m;
  if (a.final_c && k.chain == 0) {
    uint8_t* o = a.final_c + (k.item * 4 + k.cls) * nq;
    for (int w = 0; w < WQ; ++w) {
      uint32_t word = 0;
      for (int t = 0; t < a.T; ++t) word ^= Ew[(int64_t)(t * WQ + w) * stride];
      for (int f = 0; f < 16; ++f) {
        const int q = 16 * w + f;
        if (q < nq) o[q] = (uint8_t)((word >> (2 * f)) & 3u);
      }
    }
  }
}

// The space-time chains with a streaming window of registers at code size L
// (spacetime_win.h; one translation unit per L in [SPACETIME_WIN_L_MIN,
// SPACETIME_WIN_L_MAX]).
template <int L>
hipError_t launch_spacetime_win_L(const SpaceTimeArgs& a, hipStream_t s);

}  // namespace mcmc
