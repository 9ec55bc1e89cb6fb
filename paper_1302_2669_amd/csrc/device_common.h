// Device-side building blocks shared by the decoder's kernels: packed chain
// layout, Philox4x32-10 and compile-time loops.
//
// Packed layout of one configuration (registers and memory alike)
// ---------------------------------------------------------------
// Grid row r (0 .. 2L-2) holds the qubits (r, c), r+c even, left to right:
// L of them on even rows, L-1 on odd rows.  Each qubit is a 2-bit field
// (bit 0 = x part, bit 1 = z part), 16 fields per 32-bit word, W = ceil(L/16)
// words per row.  Fields past the end of a row hold Y (code 3): a Y qubit
// never changes the weight of a star or plaquette move, so it doubles as the
// "missing neighbour" of a weight-3 boundary stabilizer.
//
// Star (i, j) (grid (2i+1, 2j)) touches field j of even rows 2i and 2i+2 and
// fields j-1, j of odd row 2i+1.  Plaquette (i, j) (grid (2i, 2j+1)) touches
// field j of odd rows 2i-1 and 2i+1 and fields j, j+1 of even row 2i.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace mcmc {

template <int L>
struct Geo {
  static constexpr int R = 2 * L - 1;            // grid rows
  static constexpr int W = (L + 15) / 16;        // 32-bit words per row
  static constexpr int RW = R * W;               // words per configuration
  static constexpr int S = L * (L - 1) / 2;      // sites per colour
  static constexpr int NSTAB = 2 * L * (L - 1);
  static constexpr int NQ = 2 * L * L - 2 * L + 1;
};

// Words per row and per configuration for a runtime L.
__host__ __device__ inline int words_per_row(int L) { return (L + 15) / 16; }
__host__ __device__ inline int words_per_config(int L) { return (2 * L - 1) * words_per_row(L); }

// Valid-field mask (both bits of each field) of word w of a row with `fields` qubits.
__host__ __device__ constexpr uint32_t field_mask(int fields, int w) {
  const int lo = 16 * w;
  const int n = fields - lo;
  return n <= 0 ? 0u : (n >= 16 ? 0xFFFFFFFFu : ((1u << (2 * n)) - 1u));
}

// ---- compile-time loop ---------------------------------------------------
template <int... Is, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) --------------------
constexpr uint32_t PHILOX_M0 = 0xD2511F53u;
constexpr uint32_t PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u;
constexpr uint32_t PHILOX_W1 = 0xBB67AE85u;

__device__ __forceinline__ void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

// a ^ b ^ k in one three-input bit operation (truth table 0x96); k is
// wave-uniform (the Philox round key) and sits in an SGPR.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

__device__ __forceinline__ uint4 philox_round(uint4 c, uint32_t k0, uint32_t k1) {
  uint32_t h0, l0, h1, l1;
  mulhilo(PHILOX_M0, c.x, h0, l0);
  mulhilo(PHILOX_M1, c.z, h1, l1);
  return make_uint4(xor3_key(h1, c.y, k0), l1, xor3_key(h0, c.w, k1), l0);
}

// Rounds first..9 of Philox4x32-10 on counter c; key (k0, k1) is the ORIGINAL
// key (round r uses k + r*W).  The loop body holds two rounds, so the word
// rotation of a round costs no register moves; the loop itself is kept rolled
// because the chain kernel inlines one copy per block of draws.
__device__ __forceinline__ uint4 philox_rounds(uint4 c, uint32_t k0, uint32_t k1, int first) {
  k0 += (uint32_t)first * PHILOX_W0;
  k1 += (uint32_t)first * PHILOX_W1;
  int r = first;
  if ((10 - first) & 1) {
    c = philox_round(c, k0, k1);
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
    ++r;
  }
#pragma unroll 1
  for (; r < 10; r += 2) {
    c = philox_round(c, k0, k1);
    c = philox_round(c, k0 + PHILOX_W0, k1 + PHILOX_W1);
    k0 += 2 * PHILOX_W0;
    k1 += 2 * PHILOX_W1;
  }
  return c;
}

// The same rounds on two counters at once, interleaved: the two products of
// one round of each counter are independent, which doubles the work a wave
// can issue between dependent multiplies.
__device__ __forceinline__ void philox_rounds2(uint4& c, uint4& e, uint32_t k0, uint32_t k1,
                                               int first) {
  k0 += (uint32_t)first * PHILOX_W0;
  k1 += (uint32_t)first * PHILOX_W1;
  int r = first;
  if ((10 - first) & 1) {
    c = philox_round(c, k0, k1);
    e = philox_round(e, k0, k1);
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
    ++r;
  }
#pragma unroll 1
  for (; r < 10; r += 2) {
    c = philox_round(c, k0, k1);
    e = philox_round(e, k0, k1);
    c = philox_round(c, k0 + PHILOX_W0, k1 + PHILOX_W1);
    e = philox_round(e, k0 + PHILOX_W0, k1 + PHILOX_W1);
    k0 += 2 * PHILOX_W0;
    k1 += 2 * PHILOX_W1;
  }
}

// Four counters at once, interleaved like philox_rounds2.
__device__ __forceinline__ void philox_rounds4(uint4 (&c)[4], uint32_t k0, uint32_t k1,
                                               int first) {
  k0 += (uint32_t)first * PHILOX_W0;
  k1 += (uint32_t)first * PHILOX_W1;
  int r = first;
  if ((10 - first) & 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = philox_round(c[i], k0, k1);
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
    ++r;
  }
#pragma unroll 1
  for (; r < 10; r += 2) {
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = philox_round(c[i], k0, k1);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = philox_round(c[i], k0 + PHILOX_W0, k1 + PHILOX_W1);
    k0 += 2 * PHILOX_W0;
    k1 += 2 * PHILOX_W1;
  }
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  return philox_rounds(c, k0, k1, 0);
}

// Chain-move draws: counter (blk, sweep, sid, ctr3).  The parts of the first
// two rounds that do not depend on blk are computed once per lane (sid) and
// once per sweep; blk is a compile-time constant, so its first-round product
// folds away.
struct ChainRng {
  uint32_t k0, k1;
  uint32_t sid_hi, sid_lo;   // M1 * sid
  uint32_t ctr3;
  uint32_t ctr3_sw;          // ctr3, made opaque once per sweep (see begin_sweep)
  uint32_t sw_hi, sw_lo;     // M0 * (sid_hi ^ sweep ^ k0), per sweep

  __device__ __forceinline__ void init(uint32_t key0, uint32_t key1, uint32_t sid, uint32_t c3) {
    k0 = key0;
    k1 = key1;
    ctr3 = c3;
    mulhilo(PHILOX_M1, sid, sid_hi, sid_lo);
  }
  __device__ __forceinline__ void begin_sweep(uint32_t sweep) {
    mulhilo(PHILOX_M0, sid_hi ^ sweep ^ k0, sw_hi, sw_lo);
    // The second-round product of every block depends only on (blk, ctr3);
    // without this the compiler hoists all of them out of the sweep loop and
    // keeps two live registers per block, which costs far more occupancy
    // than the one multiply per block it saves.
    ctr3_sw = ctr3;
    asm volatile("" : "+v"(ctr3_sw));
  }
  template <int BLK>
  __device__ __forceinline__ uint4 block() const {
    constexpr uint64_t pb = (uint64_t)PHILOX_M0 * (uint64_t)(uint32_t)BLK;
    constexpr uint32_t hi0 = (uint32_t)(pb >> 32), lo0 = (uint32_t)pb;
    // after round 0: (sid_hi ^ sweep ^ k0, sid_lo, hi0 ^ ctr3 ^ k1, lo0)
    uint32_t qh, ql;
    mulhilo(PHILOX_M1, hi0 ^ ctr3_sw ^ k1, qh, ql);
    const uint4 c = make_uint4(qh ^ sid_lo ^ (k0 + PHILOX_W0), ql,
                               sw_hi ^ lo0 ^ (k1 + PHILOX_W1), sw_lo);
    return philox_rounds(c, k0, k1, 2);
  }
  // Blocks BLK and BLK + 1 together (identical words to two block() calls).
  template <int BLK>
  __device__ __forceinline__ void block_pair(uint4& b0, uint4& b1) const {
    constexpr uint64_t pa = (uint64_t)PHILOX_M0 * (uint64_t)(uint32_t)BLK;
    constexpr uint64_t pc = (uint64_t)PHILOX_M0 * (uint64_t)(uint32_t)(BLK + 1);
    constexpr uint32_t ha = (uint32_t)(pa >> 32), la = (uint32_t)pa;
    constexpr uint32_t hc = (uint32_t)(pc >> 32), lc = (uint32_t)pc;
    uint32_t qh, ql, rh, rl;
    mulhilo(PHILOX_M1, ha ^ ctr3_sw ^ k1, qh, ql);
    mulhilo(PHILOX_M1, hc ^ ctr3_sw ^ k1, rh, rl);
    b0 = make_uint4(qh ^ sid_lo ^ (k0 + PHILOX_W0), ql, sw_hi ^ la ^ (k1 + PHILOX_W1), sw_lo);
    b1 = make_uint4(rh ^ sid_lo ^ (k0 + PHILOX_W0), rl, sw_hi ^ lc ^ (k1 + PHILOX_W1), sw_lo);
    philox_rounds2(b0, b1, k0, k1, 2);
  }
  // Blocks BLK .. BLK + 3 together.
  template <int BLK>
  __device__ __forceinline__ void block_quad(uint4 (&b)[4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t pa = (uint64_t)PHILOX_M0 * (uint64_t)(uint32_t)(BLK + i);
      const uint32_t ha = (uint32_t)(pa >> 32), la = (uint32_t)pa;
      uint32_t qh, ql;
      mulhilo(PHILOX_M1, ha ^ ctr3_sw ^ k1, qh, ql);
      b[i] = make_uint4(qh ^ sid_lo ^ (k0 + PHILOX_W0), ql, sw_hi ^ la ^ (k1 + PHILOX_W1), sw_lo);
    }
    philox_rounds4(b, k0, k1, 2);
  }
};

__device__ __forceinline__ uint32_t word_of(const uint4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

}  // namespace mcmc
