// Colour-phased Metropolis chains, one chain per lane (Sec. IV, Sec. IV.A,
// Sec. V of arXiv:1302.2669).
//
// Mapping.  Every lane owns one chain (syndrome, class, temperature, replica)
// and keeps its whole configuration in VGPRs as packed 2-bit Pauli fields
// (device_common.h): 2L-1 row words for L <= 16, twice that up to L = 25.
// The code distance is a template parameter, so every row, word, field and
// Philox block index below is a compile-time constant and the state never
// leaves registers; the kernel has no barrier and no shared state between
// lanes.  The only LDS use is a per-lane copy of the acceptance thresholds.
//
// One sweep = the four colour phases of Sec. V's grouping in order.  Within a
// phase the sites share no qubit, so a whole grid row of same-coloured sites
// is evaluated at once with word-parallel (SWAR) arithmetic:
//   per neighbour direction, a star qubit contributes c = 2[I] + [z] and a
//   plaquette qubit c = 2[I] + [x] (so c - 1 = its change of weight), summed
//   over the four neighbour words into one 4-bit nibble per site:
//   t = Delta n + 4 in [0, 8];
// then per site: the Philox word u, accept = t <= 4 || u < A[t-4], and the
// accepted sites' masks flip the x (star) or z (plaquette) bits of the three
// touched rows with a handful of XORs.  The weight change of the row is the
// sum of accepted nibbles minus 4 per accepted site.
//
// Accumulation: n after every colour phase of a counted sweep is added to S
// (int64); A counts accepted moves.  No cross-lane reduction is needed.
//
// Noise models (template parameter NOISE): 0 = depolarizing, n = number of
// non-identity qubits (the c above); 1 = independent bit/phase flips, n =
// number of x parts + z parts, so a star qubit contributes c = 2[x = 0] and a
// plaquette qubit c = 2[z = 0].  Under NOISE 1 the padding Y of a row end
// would read as c = 0, so the one padded field a star reads (the east end of
// its odd row) is forced to c = 1 there.
#pragma once

#include "device_common.h"
#include "internal.h"

namespace mcmc {

__device__ __forceinline__ uint32_t c_star(uint32_t v) {
  const uint32_t z = (v >> 1) & 0x55555555u;
  const uint32_t id = ~(v | (v >> 1)) & 0x55555555u;
  return (id << 1) | z;
}
__device__ __forceinline__ uint32_t c_plaq(uint32_t v) {
  const uint32_t x = v & 0x55555555u;
  const uint32_t id = ~(v | (v >> 1)) & 0x55555555u;
  return (id << 1) | x;
}

// Independent bit/phase flips: c = 2[x = 0] (star), 2[z = 0] (plaquette).
__device__ __forceinline__ uint32_t c_star_flip(uint32_t v) { return ~(v << 1) & 0xAAAAAAAAu; }
__device__ __forceinline__ uint32_t c_plaq_flip(uint32_t v) { return ~v & 0xAAAAAAAAu; }

template <int NOISE>
__device__ __forceinline__ uint32_t c_star_of(uint32_t v) {
  if constexpr (NOISE == 1) return c_star_flip(v);
  else return c_star(v);
}
template <int NOISE>
__device__ __forceinline__ uint32_t c_plaq_of(uint32_t v) {
  if constexpr (NOISE == 1) return c_plaq_flip(v);
  else return c_plaq(v);
}

// Sum of the eight nibbles of v.
__device__ __forceinline__ uint32_t nibble_sum(uint32_t v, uint32_t acc) {
  const uint32_t b = (v & 0x0F0F0F0Fu) + ((v >> 4) & 0x0F0F0F0Fu);
  return __builtin_amdgcn_sad_u8(b, 0u, acc);
}

// acc = 2 * acc + (u < thr): the comparison result lands directly in the
// running bit mask (the first site pushed ends in the highest bit).
__device__ __forceinline__ uint32_t push_accept(uint32_t acc, uint32_t u, uint32_t thr) {
  asm("v_cmp_lt_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
      : "+v"(acc)
      : "v"(u), "v"(thr)
      : "vcc");
  return acc;
}

// Bits 0..7 of x moved to bits 0, 4, ..., 28 (one per nibble).
__device__ __forceinline__ uint32_t spread_nibbles(uint32_t x) {
  x = (x | (x << 12)) & 0x000F000Fu;
  x = (x | (x << 6)) & 0x03030303u;
  return (x | (x << 3)) & 0x11111111u;
}

// Nibble-LSB mask of the sites of one row in word w: sites j = par, par+2, ...
// below `limit` fields, at nibble (j % 16) / 2 of word j / 16.
__host__ __device__ constexpr uint32_t site_nibbles(int par, int limit, int w) {
  uint32_t m = 0;
  for (int j = par; j < limit; j += 2)
    if (j / 16 == w) m |= 1u << (4 * ((j % 16) / 2));
  return m;
}

// Rank (position within its colour, row-major) of the first site of row i.
template <int L>
__host__ __device__ constexpr int star_row_rank(int i, int par_of_row0) {
  // stars of colour with (i' + j) & 1 == phi: row i' holds (L - par + 1) / 2
  // of them, par = (i' + phi) & 1
  int r = 0;
  for (int ii = 0; ii < i; ++ii) r += (L - ((ii + par_of_row0) & 1) + 1) / 2;
  return r;
}
template <int L>
__host__ __device__ constexpr int plaq_row_rank(int i, int par_of_row0) {
  int r = 0;
  for (int ii = 0; ii < i; ++ii) r += (L - 1 - ((ii + par_of_row0) & 1) + 1) / 2;
  return r;
}

// Row fence: every state word is passed through an empty asm statement, so no
// computation of a later row can be hoisted above this point.  Without it the
// compiler precomputes partial neighbour sums of many rows ahead and keeps
// them live, which costs far more occupancy than the latency it hides.
// The row's weight change and accept count are fenced too, so that their
// computation is not sunk to the end of the phase.
template <int R, int W>
__device__ __forceinline__ void row_fence(uint32_t (&st)[R][W], int32_t& dn, int32_t& acc) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int w = 0; w < W; ++w) asm volatile("" : "+v"(st[r][w]));
  asm volatile("" : "+v"(dn), "+v"(acc));
}
// Philox blocks two at a time (interleaved rounds, more independent work per
// wave) unless the including kernel turns it off; the words are identical.
#ifndef MCMC_PAIRED_PHILOX
#define MCMC_PAIRED_PHILOX 1
#endif
#ifndef MCMC_ROW_FENCE
#define MCMC_ROW_FENCE() row_fence(st, dn, acc_total)
#endif

// The item (syndrome) behind index `idx` of a group: from the plan's table, or
// implicit for a uniform batch.
__device__ __forceinline__ ItemDesc item_of(const RunArgs& a, int64_t idx, int RW) {
  if (a.items) return a.items[idx];
  ItemDesc it;
  it.orig = idx;
  it.syn_off = 0;
  it.rows_off = idx * RW * 4;
  it.chain_off = idx * 4 * (int64_t)a.g0.K * a.g0.C;
  it.corr_off = 0;
  it.table_off = 0;
  it.beta_bar = 0.0;
  it.sid = a.syndrome_ids ? a.syndrome_ids[idx] : (uint32_t)idx;
  it.group = 0;
  return it;
}

// One chain (lane) of group g: task t of the group.  lds_tbl is this
// workgroup's threshold table, column `col` belongs to this lane.
template <int L, int NOISE>
__device__ __forceinline__ void run_chain(const RunArgs& a, const GroupDesc& g, int64_t t,
                                          uint32_t (*lds_tbl)[256], const int col) {
  using G = Geo<L>;
  constexpr int R = G::R, W = G::W, S = G::S;
  const int lane = col;
  const int K = g.K, C = g.C;

  // task -> (item, class, temperature, replica)
  const int64_t per_item = 4 * (int64_t)K * C;
  const int64_t item_local = t / per_item;
  const int rem = (int)(t - item_local * per_item);
  const int chain = rem % C;
  const int kt = (rem / C) % K;
  const int cls = rem / (C * K);
  const ItemDesc it = item_of(a, g.first_item + item_local, G::RW);
  const int64_t out = it.chain_off + rem;   // per-chain output slot

  // this lane's thresholds: entry t = Delta + 4; t <= 4 is never read
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    uint32_t v = 0xFFFFFFFFu;
    if (e > 4) v = a.tables ? a.tables[it.table_off + kt * 4 + (e - 5)] : a.table0[kt][e - 5];
    lds_tbl[e][lane] = v;
  }

  uint32_t st[R][W];
  int32_t n;
  int64_t Ssum = 0, Acnt = 0;
  if (a.resume_rows) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int w = 0; w < W; ++w)
        st[r][w] = a.resume_rows[(int64_t)(r * W + w) * a.total_chains + out];
    n = a.resume_n[out];
    Ssum = a.resume_S[out];
    Acnt = a.resume_A[out];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int w = 0; w < W; ++w) st[r][w] = a.init_rows[it.rows_off + (r * W + w) * 4 + cls];
    n = a.init_n[it.orig * 4 + cls];
  }

  ChainRng rng;
  rng.init(a.k0, a.k1, it.sid, ((uint32_t)cls << 28) | ((uint32_t)(kt + 1) << 20) | (uint32_t)chain);

  int16_t* trace = a.trace ? a.trace + out * a.trace_len : nullptr;
  int64_t tpos = 0;

  for (int sweep = g.sweep_begin; sweep < g.sweep_end; ++sweep) {
    rng.begin_sweep((uint32_t)sweep);
    uint4 blk = make_uint4(0, 0, 0, 0);
    uint4 blk_next = make_uint4(0, 0, 0, 0);
#if MCMC_PAIRED_PHILOX == 4
    uint4 quad[4];
#endif
    int32_t dn = 0;     // weight change of the current phase
    int32_t acc_total = 0;

    auto end_phase = [&]() {
      n += dn;
      dn = 0;
      if (sweep >= g.burn) Ssum += n;
      if (trace) trace[tpos++] = (int16_t)n;
    };

    // Accept decisions of one row's sites (nibble m of `sum` holds Delta n + 4
    // of site m): Philox words in draw order, thresholds from LDS, then
    // u < A[Delta] folded into a bit mask, OR the sites with Delta n <= 0
    // (t + 3 < 8).  Leaves the nibble-LSB accept masks in acc and adds the
    // row's weight change and accept count.
    auto decide_row = [&](auto PAR, auto NSITE, auto D0, auto LIMIT, const uint32_t (&sum)[W],
                          uint32_t (&acc)[W]) {
      constexpr int par = decltype(PAR)::value, nsite = decltype(NSITE)::value;
      constexpr int d0 = decltype(D0)::value, limit = decltype(LIMIT)::value;
      // bit (nsite-1-m) of `rbits`: u_m < A[Delta_m], pushed in site order so
      // that only one draw and one threshold are live at a time
      uint32_t rbits = 0;
      static_for<nsite>([&](auto MM) {
        constexpr int m = decltype(MM)::value;
        constexpr int j = par + 2 * m;
        constexpr int w = j / 16, nib = (j % 16) / 2;
        constexpr int d = d0 + m;
#if MCMC_PAIRED_PHILOX == 4
        // blocks four at a time while four remain in the sweep
        if constexpr ((d & 15) == 0 && d / 4 + 3 < S) {
          rng.template block_quad<d / 4>(quad);
          blk = quad[0];
        } else if constexpr ((d & 3) == 0 && (d & ~15) / 4 + 3 < S) {
          blk = quad[(d / 4) & 3];
        } else if constexpr ((d & 3) == 0) {
          blk = rng.template block<d / 4>();
        }
#elif MCMC_PAIRED_PHILOX
        // blocks two at a time (the second waits in blk_next); a lone last
        // block of the sweep is computed alone
        if constexpr ((d & 7) == 0) {
          if constexpr (d / 4 + 1 < S) rng.template block_pair<d / 4>(blk, blk_next);
          else blk = rng.template block<d / 4>();
        } else if constexpr ((d & 7) == 4) {
          blk = blk_next;
        }
#else
        if constexpr ((d & 3) == 0) blk = rng.template block<d / 4>();
#endif
        const uint32_t thr = lds_tbl[(sum[w] >> (4 * nib)) & 15u][lane];
        rbits = push_accept(rbits, word_of(blk, d & 3), thr);
      });
      const uint32_t bits = __builtin_bitreverse32(rbits) >> (32 - nsite);  // bit m: site m
      static_for<W>([&](auto WW) {
        constexpr int w = decltype(WW)::value;
        constexpr uint32_t sites = site_nibbles(par, limit, w);
        const uint32_t low = ~(sum[w] + 0x33333333u) >> 3;  // nibble LSB: t <= 4
        acc[w] = (spread_nibbles((bits >> (8 * w)) & 0xFFu) | low) & sites;
        const uint32_t nm = (acc[w] << 4) - acc[w];
        const int32_t cnt = (int32_t)__builtin_popcount(acc[w]);
        dn += (int32_t)nibble_sum(sum[w] & nm, 0u) - 4 * cnt;
        acc_total += cnt;
      });
    };

    // ---------------- stars: colours 0 and 1 ----------------
    static_for<2>([&](auto PH) {
      constexpr int phi = decltype(PH)::value;
      static_for<L - 1>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int par = (i + phi) & 1;
        constexpr int nsite = (L - par + 1) / 2;
        constexpr int rank0 = star_row_rank<L>(i, phi);
        uint32_t cO[W], sum[W], acc[W];
        static_for<W>([&](auto WW) {
          constexpr int w = decltype(WW)::value;
          cO[w] = c_star_of<NOISE>(st[2 * i + 1][w]);
          if constexpr (NOISE == 1) cO[w] |= 0x55555555u & ~field_mask(L - 1, w);  // pad: c = 1
        });
        static_for<W>([&](auto WW) {
          constexpr int w = decltype(WW)::value;
          const uint32_t cN = c_star_of<NOISE>(st[2 * i][w]);
          const uint32_t cS = c_star_of<NOISE>(st[2 * i + 2][w]);
          uint32_t cWest;
          if constexpr (w == 0) cWest = (cO[0] << 2) | 1u;
          else cWest = (cO[w] << 2) | (cO[w - 1] >> 30);
          constexpr uint32_t M = 0x33333333u;
          sum[w] = ((cN >> (2 * par)) & M) + ((cS >> (2 * par)) & M) +
                   ((cO[w] >> (2 * par)) & M) + ((cWest >> (2 * par)) & M);
        });
        decide_row(std::integral_constant<int, par>{}, std::integral_constant<int, nsite>{},
                   std::integral_constant<int, phi * S + rank0>{},
                   std::integral_constant<int, L>{}, sum, acc);
        uint32_t ax[W];
        static_for<W>([&](auto WW) { ax[decltype(WW)::value] = acc[decltype(WW)::value] << (2 * par); });
        static_for<W>([&](auto WW) {
          constexpr int w = decltype(WW)::value;
          st[2 * i][w] ^= ax[w];
          st[2 * i + 2][w] ^= ax[w];
          uint32_t westward = ax[w] >> 2;
          if constexpr (w + 1 < W) westward |= ax[w + 1] << 30;
          st[2 * i + 1][w] ^= (ax[w] | westward) & field_mask(L - 1, w) & 0x55555555u;
        });
        MCMC_ROW_FENCE();
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
          uint32_t cE[W], sum[W], acc[W];
          static_for<W>([&](auto WW) { cE[decltype(WW)::value] = c_plaq_of<NOISE>(st[2 * i][decltype(WW)::value]); });
          static_for<W>([&](auto WW) {
            constexpr int w = decltype(WW)::value;
            uint32_t cN = 0x55555555u, cS = 0x55555555u;
            if constexpr (i > 0) cN = c_plaq_of<NOISE>(st[2 * i - 1][w]);
            if constexpr (i < L - 1) cS = c_plaq_of<NOISE>(st[2 * i + 1][w]);
            uint32_t cEast = cE[w] >> 2;
            if constexpr (w + 1 < W) cEast |= cE[w + 1] << 30;
            constexpr uint32_t M = 0x33333333u;
            sum[w] = ((cN >> (2 * par)) & M) + ((cS >> (2 * par)) & M) +
                     ((cE[w] >> (2 * par)) & M) + ((cEast >> (2 * par)) & M);
          });
          decide_row(std::integral_constant<int, par>{}, std::integral_constant<int, nsite>{},
                     std::integral_constant<int, phi * S + rank0>{},
                     std::integral_constant<int, L - 1>{}, sum, acc);
          uint32_t az[W];
          static_for<W>([&](auto WW) { az[decltype(WW)::value] = acc[decltype(WW)::value] << (2 * par + 1); });
          static_for<W>([&](auto WW) {
            constexpr int w = decltype(WW)::value;
            if constexpr (i > 0) st[2 * i - 1][w] ^= az[w];
            if constexpr (i < L - 1) st[2 * i + 1][w] ^= az[w];
            uint32_t eastward = az[w] << 2;
            if constexpr (w > 0) eastward |= az[w - 1] >> 30;
            st[2 * i][w] ^= az[w] | eastward;
          });
          MCMC_ROW_FENCE();
        }
      });
      end_phase();
    });
    Acnt += acc_total;
  }

  a.S_out[out] = Ssum;
  a.A_out[out] = Acnt;
  a.n_out[out] = n;
  if (a.state_rows) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int w = 0; w < W; ++w) a.state_rows[(int64_t)(r * W + w) * a.total_chains + out] = st[r][w];
  }
  if (a.final_rows && chain == 0 && kt == K - 1) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int w = 0; w < W; ++w) a.final_rows[it.rows_off + (r * W + w) * 4 + cls] = st[r][w];
  }
}


// Persistent tile loop over the L range [LMIN, LMAX]: every wave takes the
// next tile from the launch's queue (tiles are ordered longest first by the
// planner) and runs the code of that tile's L; tiles of another L range are
// skipped.  Every wave leaves once the queue is exhausted.
template <int LMIN, int LMAX, int NOISE>
__device__ __forceinline__ void dispatch_tile(const RunArgs& a, const GroupDesc& g, int L, int64_t t,
                                              uint32_t (*lds_tbl)[256], int col) {
  if constexpr (LMIN <= LMAX) {
    if (L == LMIN) {
      run_chain<LMIN, NOISE>(a, g, t, lds_tbl, col);
      return;
    }
    dispatch_tile<LMIN + 1, LMAX, NOISE>(a, g, L, t, lds_tbl, col);
  }
}

template <int LMIN, int LMAX, int NOISE = 0>
__device__ __forceinline__ void chains_persistent(const RunArgs& a) {
  __shared__ uint32_t lds_tbl[9][256];
  const int col = threadIdx.x;
  const int lane = threadIdx.x & 63;
  while (true) {
    uint32_t tile = 0;
    if (lane == 0) tile = atomicAdd(a.queue, 1u);
    tile = __builtin_amdgcn_readfirstlane(tile);  // lane 0 is active: the loop is wave-uniform
    GroupDesc g;
    int L;
    int64_t first;
    if (a.tile_cum) {
      const uint32_t c0 = a.tile_cum[0], c1 = a.tile_cum[1], c2 = a.tile_cum[2];
      if (tile >= c2) break;
      const int gi = tile < c0 ? 0 : (tile < c1 ? 1 : 2);
      g = a.groups[gi];
      L = g.L;
      first = (int64_t)(tile - (gi == 0 ? 0u : (gi == 1 ? c0 : c1))) * TILE;
    } else if ((int64_t)tile >= a.n_tiles) {
      break;
    } else if (a.tiles) {
      const TileDesc td = a.tiles[tile];
      g = a.groups[td.group];
      L = td.L;
      first = td.first_task;
    } else {
      g = a.g0;
      L = a.g0.L;
      first = (int64_t)tile * TILE;
    }
    if (L < LMIN || L > LMAX) continue;
    const int64_t t = first + lane;
    if (t < g.n_tasks) dispatch_tile<LMIN, LMAX, NOISE>(a, g, L, t, lds_tbl, col);
  }
}

}  // namespace mcmc
