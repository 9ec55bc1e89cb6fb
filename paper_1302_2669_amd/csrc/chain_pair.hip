// Colour-phased Metropolis chains, two chains per lane, for codes up to L = 8
// (Sec. IV, Sec. IV.A, Sec. V of arXiv:1302.2669): the second chain mapping
// a plan can choose for its small codes (mcmc_tuning.pair_small).
//
// A row of a code with L <= 8 fills at most half a 32-bit word, so one lane
// keeps two chains in the same registers: chain A in fields 0..7 and chain B
// in fields 8..15 of every row word.  The SWAR arithmetic of the one-chain
// kernel (chain_body.h) then evaluates a grid row of same-coloured sites of
// both chains at once: their sites land in nibbles 0..3 (A) and 4..7 (B) of
// the neighbour sums.  The only place where the halves would meet is the
// west neighbour of a star in field 0 or 8, which reads the padding value
// instead; every flip mask stays inside its half because rows end at field
// L - 1 <= 7.  Each chain keeps its own draws (Philox counter of its own
// syndrome, class, temperature and replica, the blocks of both chains
// computed together), its own acceptance thresholds (two LDS columns per
// lane) and its own weight, sums and accept count, so every output is the
// one-chain kernel's bit for bit.
//
// Tasks: a pair tile of a group covers tasks first .. first + 127; lane l
// runs tasks first + l (A) and first + 64 + l (B).  A lane whose B task is
// past the group's end runs B as a copy of A and writes nothing for it.
// Plans only: no trace, no resume, no exported state.
#include "chain_body.h"

namespace mcmc {

namespace {

constexpr uint32_t HALF_LO = 0x0000FFFFu;

// fields 0..n-1 of both halves
__host__ __device__ constexpr uint32_t pair_fields(int n) {
  return field_mask(n, 0) | (field_mask(n, 0) << 16);
}
// nibble-LSB mask of the sites of one row in both halves
__host__ __device__ constexpr uint32_t pair_sites(int par, int limit) {
  return site_nibbles(par, limit, 0) | (site_nibbles(par, limit, 0) << 16);
}

// Blocks BLK of two chains' streams together (both keyed by the same seed).
template <int BLK>
__device__ __forceinline__ void block_two(const ChainRng& A, const ChainRng& B, uint4& a,
                                          uint4& b) {
  constexpr uint64_t pb = (uint64_t)PHILOX_M0 * (uint64_t)(uint32_t)BLK;
  constexpr uint32_t hb = (uint32_t)(pb >> 32), lb = (uint32_t)pb;
  uint32_t qh, ql, rh, rl;
  mulhilo(PHILOX_M1, hb ^ A.ctr3_sw ^ A.k1, qh, ql);
  mulhilo(PHILOX_M1, hb ^ B.ctr3_sw ^ B.k1, rh, rl);
  a = make_uint4(qh ^ A.sid_lo ^ (A.k0 + PHILOX_W0), ql, A.sw_hi ^ lb ^ (A.k1 + PHILOX_W1),
                 A.sw_lo);
  b = make_uint4(rh ^ B.sid_lo ^ (B.k0 + PHILOX_W0), rl, B.sw_hi ^ lb ^ (B.k1 + PHILOX_W1),
                 B.sw_lo);
  philox_rounds2(a, b, A.k0, A.k1, 2);
}

struct PairChain {
  ItemDesc it;
  int64_t out;
  int cls, kt, chain;
};

__device__ __forceinline__ PairChain pair_chain(const RunArgs& a, const GroupDesc& g, int64_t t) {
  PairChain c;
  const int64_t per_item = 4 * (int64_t)g.K * g.C;
  const int64_t item_local = t / per_item;
  const int rem = (int)(t - item_local * per_item);
  c.chain = rem % g.C;
  c.kt = (rem / g.C) % g.K;
  c.cls = rem / (g.C * g.K);
  c.it = a.items[g.first_item + item_local];
  c.out = c.it.chain_off + rem;
  return c;
}

template <int L, int NOISE>
__device__ __forceinline__ void run_pair(const RunArgs& a, const GroupDesc& g, int64_t tA,
                                         bool has_b, uint32_t (*lds_tbl)[512], const int col) {
  using G = Geo<L>;
  constexpr int R = G::R, S = G::S;
  static_assert(L <= PAIR_L_MAX && PAIR_L_MAX <= 8, "two chains per word need rows of at most 8 fields");
  const PairChain A = pair_chain(a, g, tA);
  const PairChain B = has_b ? pair_chain(a, g, tA + 64) : A;

#pragma unroll
  for (int e = 0; e < 9; ++e) {
    uint32_t va = 0xFFFFFFFFu, vb = 0xFFFFFFFFu;
    if (e > 4) {
      va = a.tables[A.it.table_off + A.kt * 4 + (e - 5)];
      vb = a.tables[B.it.table_off + B.kt * 4 + (e - 5)];
    }
    lds_tbl[e][col] = va;
    lds_tbl[e][256 + col] = vb;
  }

  uint32_t st[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    st[r] = (a.init_rows[A.it.rows_off + r * 4 + A.cls] & HALF_LO) |
            (a.init_rows[B.it.rows_off + r * 4 + B.cls] << 16);
  int32_t nA = a.init_n[A.it.orig * 4 + A.cls];
  int32_t nB = a.init_n[B.it.orig * 4 + B.cls];
  int64_t SA = 0, SB = 0, AA = 0, AB = 0;

  ChainRng rA, rB;
  rA.init(a.k0, a.k1, A.it.sid, ((uint32_t)A.cls << 28) | ((uint32_t)(A.kt + 1) << 20) |
                                    (uint32_t)A.chain);
  rB.init(a.k0, a.k1, B.it.sid, ((uint32_t)B.cls << 28) | ((uint32_t)(B.kt + 1) << 20) |
                                    (uint32_t)B.chain);

  for (int sweep = g.sweep_begin; sweep < g.sweep_end; ++sweep) {
    rA.begin_sweep((uint32_t)sweep);
    rB.begin_sweep((uint32_t)sweep);
    uint4 bA = make_uint4(0, 0, 0, 0), bB = make_uint4(0, 0, 0, 0);
    int32_t dA = 0, dB = 0;   // weight changes of the current phase
    int32_t cA = 0, cB = 0;   // accepted moves of the sweep

    // as in the one-chain kernel: no computation of a later row is hoisted
    // above the end of the current one
    auto fence = [&]() {
#pragma unroll
      for (int r = 0; r < R; ++r) asm volatile("" : "+v"(st[r]));
      asm volatile("" : "+v"(dA), "+v"(dB), "+v"(cA), "+v"(cB));
    };
    auto end_phase = [&]() {
      nA += dA;
      nB += dB;
      dA = dB = 0;
      if (sweep >= g.burn) {
        SA += nA;
        SB += nB;
      }
    };

    // Accept decisions of one row of both chains (nibble m of `sum`: site m
    // of A, nibble 4 + m: site m of B); leaves the nibble-LSB accept mask.
    auto decide_row = [&](auto PAR, auto NSITE, auto D0, auto LIMIT, uint32_t sum) -> uint32_t {
      constexpr int par = decltype(PAR)::value, nsite = decltype(NSITE)::value;
      constexpr int d0 = decltype(D0)::value, limit = decltype(LIMIT)::value;
      uint32_t ra = 0, rb = 0;
      static_for<nsite>([&](auto MM) {
        constexpr int m = decltype(MM)::value;
        constexpr int d = d0 + m;
        if constexpr ((d & 3) == 0) block_two<d / 4>(rA, rB, bA, bB);
        const uint32_t ta = lds_tbl[(sum >> (4 * m)) & 15u][col];
        const uint32_t tb = lds_tbl[(sum >> (16 + 4 * m)) & 15u][256 + col];
        ra = push_accept(ra, word_of(bA, d & 3), ta);
        rb = push_accept(rb, word_of(bB, d & 3), tb);
      });
      // bit m: site m of A, bit 4 + m: site m of B
      const uint32_t bits = (__builtin_bitreverse32(ra) >> (32 - nsite)) |
                            ((__builtin_bitreverse32(rb) >> (32 - nsite)) << 4);
      constexpr uint32_t sites = pair_sites(par, limit);
      const uint32_t low = ~(sum + 0x33333333u) >> 3;   // nibble LSB: t <= 4
      const uint32_t acc = (spread_nibbles(bits & 0xFFu) | low) & sites;
      const uint32_t nm = (acc << 4) - acc;
      const uint32_t kept = sum & nm;
      const int32_t ka = (int32_t)__builtin_popcount(acc & HALF_LO);
      const int32_t kb = (int32_t)__builtin_popcount(acc >> 16);
      dA += (int32_t)nibble_sum(kept & HALF_LO, 0u) - 4 * ka;
      dB += (int32_t)nibble_sum(kept >> 16, 0u) - 4 * kb;
      cA += ka;
      cB += kb;
      return acc;
    };

    // ---------------- stars: colours 0 and 1 ----------------
    static_for<2>([&](auto PH) {
      constexpr int phi = decltype(PH)::value;
      static_for<L - 1>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int par = (i + phi) & 1;
        constexpr int nsite = (L - par + 1) / 2;
        constexpr int rank0 = star_row_rank<L>(i, phi);
        uint32_t cO = c_star_of<NOISE>(st[2 * i + 1]);
        if constexpr (NOISE == 1) cO |= 0x55555555u & ~pair_fields(L - 1);   // pad: c = 1
        const uint32_t cN = c_star_of<NOISE>(st[2 * i]);
        const uint32_t cS = c_star_of<NOISE>(st[2 * i + 2]);
        // west neighbours; fields 0 and 8 read the padding value 1
        const uint32_t cWest = ((cO << 2) & ~0x00030003u) | 0x00010001u;
        constexpr uint32_t M = 0x33333333u;
        const uint32_t sum = ((cN >> (2 * par)) & M) + ((cS >> (2 * par)) & M) +
                             ((cO >> (2 * par)) & M) + ((cWest >> (2 * par)) & M);
        const uint32_t acc = decide_row(std::integral_constant<int, par>{},
                                        std::integral_constant<int, nsite>{},
                                        std::integral_constant<int, phi * S + rank0>{},
                                        std::integral_constant<int, L>{}, sum);
        const uint32_t ax = acc << (2 * par);
        st[2 * i] ^= ax;
        st[2 * i + 2] ^= ax;
        st[2 * i + 1] ^= (ax | (ax >> 2)) & pair_fields(L - 1) & 0x55555555u;
        fence();
      });
      end_phase();
    });

    // ---------------- plaquettes: colours 2 and 3 ----------------
    static_for<2>([&](auto PH) {
      constexpr int phi = 2 + decltype(PH)::value;
      static_for<L>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int par = (i + phi - 2) & 1;
        constexpr int nsite = (L - par) / 2;
        constexpr int rank0 = plaq_row_rank<L>(i, phi - 2);
        if constexpr (nsite > 0) {
          const uint32_t cE = c_plaq_of<NOISE>(st[2 * i]);
          uint32_t cN = 0x55555555u, cS = 0x55555555u;
          if constexpr (i > 0) cN = c_plaq_of<NOISE>(st[2 * i - 1]);
          if constexpr (i < L - 1) cS = c_plaq_of<NOISE>(st[2 * i + 1]);
          const uint32_t cEast = cE >> 2;   // a site's east field stays in its half
          constexpr uint32_t M = 0x33333333u;
          const uint32_t sum = ((cN >> (2 * par)) & M) + ((cS >> (2 * par)) & M) +
                               ((cE >> (2 * par)) & M) + ((cEast >> (2 * par)) & M);
          const uint32_t acc = decide_row(std::integral_constant<int, par>{},
                                          std::integral_constant<int, nsite>{},
                                          std::integral_constant<int, phi * S + rank0>{},
                                          std::integral_constant<int, L - 1>{}, sum);
          const uint32_t az = acc << (2 * par + 1);
          if constexpr (i > 0) st[2 * i - 1] ^= az;
          if constexpr (i < L - 1) st[2 * i + 1] ^= az;
          st[2 * i] ^= az | (az << 2);
          fence();
        }
      });
      end_phase();
    });
    AA += cA;
    AB += cB;
  }

  a.S_out[A.out] = SA;
  a.A_out[A.out] = AA;
  a.n_out[A.out] = nA;
  if (has_b) {
    a.S_out[B.out] = SB;
    a.A_out[B.out] = AB;
    a.n_out[B.out] = nB;
  }
  // final rows: fields past each row's end hold Y in the stored layout
  if (a.final_rows && A.chain == 0 && A.kt == g.K - 1) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      a.final_rows[A.it.rows_off + r * 4 + A.cls] = (st[r] & HALF_LO) | ~HALF_LO;
  }
  if (a.final_rows && has_b && B.chain == 0 && B.kt == g.K - 1) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      a.final_rows[B.it.rows_off + r * 4 + B.cls] = (st[r] >> 16) | ~HALF_LO;
  }
}

template <int LMIN, int NOISE>
__device__ __forceinline__ void dispatch_pair(const RunArgs& a, const GroupDesc& g, int L,
                                              int64_t t, bool has_b, uint32_t (*lds)[512],
                                              int col) {
  if constexpr (LMIN <= PAIR_L_MAX) {
    if (L == LMIN) {
      run_pair<LMIN, NOISE>(a, g, t, has_b, lds, col);
      return;
    }
    dispatch_pair<LMIN + 1, NOISE>(a, g, L, t, has_b, lds, col);
  }
}

template <int NOISE>
__device__ __forceinline__ void pair_persistent(const RunArgs& a) {
  __shared__ uint32_t lds_tbl[9][512];
  const int col = threadIdx.x;
  const int lane = threadIdx.x & 63;
  while (true) {
    uint32_t tile = 0;
    if (lane == 0) tile = atomicAdd(a.queue, 1u);
    tile = __builtin_amdgcn_readfirstlane(tile);  // lane 0 is active: the loop is wave-uniform
    if ((int64_t)tile >= a.n_tiles) break;
    const TileDesc td = a.tiles[tile];
    const GroupDesc g = a.groups[td.group];
    if (td.L < 2 || td.L > PAIR_L_MAX) continue;
    const int64_t t = td.first_task + lane;
    if (t < g.n_tasks) dispatch_pair<2, NOISE>(a, g, td.L, t, t + 64 < g.n_tasks, lds_tbl, col);
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PAIR_WAVES)))
chains_pair_kernel(const RunArgs a) {
  pair_persistent<0>(a);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PAIR_WAVES)))
chains_pair_flip_kernel(const RunArgs a) {
  pair_persistent<1>(a);
}

}  // namespace

hipError_t launch_chains_pair(const RunArgs& a, int waves, int wg, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  if (!a.items || !a.tiles || !a.tables || a.trace || a.resume_rows || a.state_rows)
    return hipErrorInvalidValue;
  const int per_wg = wg / 64;
  const int blocks = (waves + per_wg - 1) / per_wg;
  if (a.noise == MCMC_NOISE_BITPHASE)
    hipLaunchKernelGGL(chains_pair_flip_kernel, dim3((unsigned)blocks), dim3((unsigned)wg), 0, s,
                       a);
  else if (a.noise == MCMC_NOISE_DEPOLARIZING)
    hipLaunchKernelGGL(chains_pair_kernel, dim3((unsigned)blocks), dim3((unsigned)wg), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mcmc
