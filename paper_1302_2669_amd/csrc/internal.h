// Internal interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/mcmcdec.h"
#include "device_common.h"

namespace mcmc {

// Offsets of the pieces of a chain-state buffer holding T chains of a
// distance-L code (struct of arrays, every piece 256-byte aligned):
//   rows [RW][T] uint32 (word-major), n [T] int32, S [T] int64, A [T] int64.
struct ChainStateLayout {
  size_t rows, n, S, A, bytes;
};
ChainStateLayout chain_state_layout(int L, int64_t T);

// ---------------------------------------------------------------------------
// Work description of a chain launch.  Chains are grouped by everything that
// shapes the kernel's code and loop (L, temperatures, chains per class, sweep
// range); a group's chains are numbered item-major:
//   task = item_local * (4*K*C) + (cls*K + k)*C + chain.
// A wave takes a tile of 64 consecutive tasks of one group.  Uniform batches
// (mcmc_decode_batch) describe one group implicitly; mixed batches carry
// explicit group, item and tile tables built by the host planner.
// ---------------------------------------------------------------------------
struct GroupDesc {
  int32_t L, K, C, burn, sweep_begin, sweep_end;
  int32_t first_item, n_items;  // items of the group in plan order
  int64_t n_tasks;              // n_items * 4 * K * C
};

struct ItemDesc {               // one syndrome, plan order
  int64_t orig;                 // caller's index (outputs indexed by it)
  int64_t syn_off;              // byte offset of its syndrome in the input
  int64_t rows_off;             // word offset of its [RW][4] start / final-row block
  int64_t chain_off;            // first per-chain output slot
  int64_t corr_off;             // byte offset of its correction output
  int64_t table_off;            // uint32 offset of its [K][4] thresholds
  double beta_bar;
  uint32_t sid;                 // Philox counter word 2 (also the sample id)
  int32_t group;
  uint32_t err_thr;             // floor(p 2^32), for sampling this item's errors
  int32_t noise;                // MCMC_NOISE_* of this syndrome
  double beta_star;             // its K = 1 temperature (beta_bar for K > 1)
};

struct TileDesc {
  int32_t group;
  int32_t L;
  int64_t first_task;           // within the group
};

constexpr int TILE = 64;        // tasks per tile (one wave)

struct RunArgs {
  // explicit plan, or all nullptr for a uniform batch
  const GroupDesc* groups;
  const ItemDesc* items;
  const TileDesc* tiles;
  const uint32_t* tables;
  // uniform batch: group g0 with items s = 0..n-1
  GroupDesc g0;
  const uint32_t* syndrome_ids;  // [n] or nullptr (=> s)
  uint32_t table0[MCMC_TEMPS_MAX][4];
  int64_t n_tiles;
  // device-built plan: cumulative tile counts of groups 0, 1, 2 (tile t of
  // group g covers tasks (t - tiles before g) * TILE ...); when set, tiles and
  // n_tiles are not used by the kernel
  const uint32_t* tile_cum;
  uint32_t* queue;               // tile counter of this launch, zero at start
  int32_t lmin, lmax;            // L range compiled into the launched kernel
  uint32_t k0, k1;               // Philox key
  const uint32_t* init_rows;     // class starts, [RW][4] block per item
  const int32_t* init_n;         // [orig*4 + cls]
  int64_t* S_out;                // per chain (chain_off + rem)
  int64_t* A_out;
  int32_t* n_out;
  uint32_t* final_rows;          // chain 0 at k = K of every class, [RW][4] per item, or nullptr
  int64_t total_chains;          // uniform batch: chain-state stride
  uint32_t* state_rows;          // uniform batch only: [RW][total_chains] final states, or nullptr
  const uint32_t* resume_rows;   // uniform batch only
  const int32_t* resume_n;
  const int64_t* resume_S;
  const int64_t* resume_A;
  int16_t* trace;                // [chain][trace_len] or nullptr
  int64_t trace_len;
  int32_t noise;                 // MCMC_NOISE_*: selects the kernel family
};

// Persistent chain kernels, one per L range, each with the register budget
// of its largest code: L 2..13 (6 waves per SIMD), 14..16 (5), and the
// two-word-row ranges 17..19, 20..22, 23..25 (3).  `waves` is the persistent
// grid in waves, `wg` the workgroup size (64, 128 or 256).
constexpr int N_RANGES = 5;
constexpr int RANGE_LO[N_RANGES] = {2, 14, 17, 20, 23};
constexpr int RANGE_HI[N_RANGES] = {13, 16, 19, 22, 25};
constexpr int RANGE_WAVES[N_RANGES] = {5, 5, 3, 3, 3};
inline int range_of(int L) {
  for (int r = 0; r < N_RANGES; ++r)
    if (L >= RANGE_LO[r] && L <= RANGE_HI[r]) return r;
  return -1;
}
inline bool range_is_wide(int r) { return RANGE_LO[r] > 16; }
template <int R>
hipError_t launch_chains_range(const RunArgs& a, int waves, int wg, hipStream_t s);
// The same ranges under independent bit/phase flips (energy = x parts +
// z parts).
template <int R>
hipError_t launch_chains_flip_range(const RunArgs& a, int waves, int wg, hipStream_t s);
// Picks the kernel of `range` for a.noise.
hipError_t launch_chains(int range, const RunArgs& a, int waves, int wg, hipStream_t s);
// The second chain mapping: two chains per lane for codes up to PAIR_L_MAX,
// plans only (a.items, a.tiles, a.tables; no trace, resume or state export);
// a.tiles are pair tiles of 2 * TILE tasks.  PAIR_WAVES: the kernel's
// register-limited waves per SIMD.
constexpr int PAIR_L_MAX = 8;
constexpr int PAIR_WAVES = 5;
hipError_t launch_chains_pair(const RunArgs& a, int waves, int wg, hipStream_t s);
// Random-scan chains of a uniform batch (g0, table0, a.noise; no trace):
// one 64-lane workgroup per 64 chains, each lane's state in LDS.
hipError_t launch_chains_random(const RunArgs& a, hipStream_t s);
size_t random_scan_lds_bytes(int L);
hipError_t launch_zero(uint32_t* p, int64_t n, hipStream_t s);

// Class starts of syndromes given either implicitly (L, n: syndrome s at
// s*n_stab, block at s*RW*4) or by the plan's item table.
struct StartArgs {
  const uint8_t* syn;
  const ItemDesc* items;         // nullptr => implicit
  const GroupDesc* groups;
  int64_t n;
  int32_t L;                     // implicit only
  uint32_t* rows;                // [RW][4] per item, or nullptr
  int32_t* weights;              // [orig*4 + cls], or nullptr
  uint8_t* bytes;                // [orig][4][n_q] (implicit only), or nullptr
  int32_t noise;                 // weights count x|z (0) or x + z parts (1)
  int32_t max_L;                 // with items: the largest L among them
};
hipError_t launch_init(const StartArgs& a, hipStream_t s);
hipError_t launch_init_matching(const StartArgs& a, hipStream_t s);
// Exact minimum-weight matching starts (MCMC_INIT_MWPM): one workgroup per
// syndrome, dynamic LDS sized for the largest L.  The launches of the larger
// capacities go to a per-device side stream forked from and joined to s; the
// first call on a device that is not capturing creates it when may_create
// (callers that must not create runtime objects pass false: then, as under a
// capture before the stream exists, every launch goes to s in order).
hipError_t launch_init_mwpm(const StartArgs& a, hipStream_t s, bool may_create = true);
// Creates the current device's side stream of launch_init_mwpm now (for
// callers that capture the starts into a graph later).
hipError_t mwpm_prepare_overlap();
// The start kernel of an MCMC_INIT_* mode.
hipError_t launch_init_mode(uint32_t init, const StartArgs& a, hipStream_t s,
                            bool may_create = true);

// Rate bin of the gap route: floor(p * 100) in fp32 (p already fp32), capped
// to [0, MCMC_GAP_BINS - 1]; the gate kernel and the host fit share it.
__host__ __device__ inline int gap_bin(float p) {
  const float q = p * 100.0f;
  const int k = (int)floorf(q);
  return k < 0 ? 0 : (k > MCMC_GAP_BINS - 1 ? MCMC_GAP_BINS - 1 : k);
}

// Second-smallest minus smallest of four class start weights.
__host__ __device__ inline int32_t start_weight_gap(const int32_t* x) {
  const int32_t a = x[0] < x[1] ? x[0] : x[1], b = x[0] < x[1] ? x[1] : x[0];
  const int32_t c = x[2] < x[3] ? x[2] : x[3], d = x[2] < x[3] ? x[3] : x[2];
  const int32_t lo = a < c ? a : c, hi_lo = a < c ? c : a, lo_hi = b < d ? b : d;
  return (hi_lo < lo_hi ? hi_lo : lo_hi) - lo;
}

#ifdef __HIPCC__
// Syndrome s of a start launch: its L, input bytes, start block and caller index.
struct StartItem {
  int L;
  int noise;                    // energy counted as x|z (0) or x + z parts (1)
  const uint8_t* sy;
  int64_t rows_off, orig;
};
__device__ inline StartItem start_item(const StartArgs& a, int64_t s) {
  StartItem r;
  if (a.items) {
    const ItemDesc it = a.items[s];
    r.L = a.groups[it.group].L;
    r.noise = it.noise;
    r.sy = a.syn + it.syn_off;
    r.rows_off = it.rows_off;
    r.orig = it.orig;
  } else {
    r.L = a.L;
    r.noise = a.noise;
    r.sy = a.syn + s * (int64_t)(2 * a.L * (a.L - 1));
    r.rows_off = s * (int64_t)words_per_config(a.L) * 4;
    r.orig = s;
  }
  return r;
}

#endif

hipError_t launch_unpack(int L, int noise, const uint32_t* rows, int64_t count, int64_t stride,
                         uint8_t* out, int32_t* weights, hipStream_t s);

struct DecideArgs {
  const ItemDesc* items;       // nullptr => uniform batch (g0, beta_bar)
  const GroupDesc* groups;
  GroupDesc g0;
  double beta_bar;             // uniform batch
  double beta_star;            // uniform batch: the K = 1 temperature (beta_bar by default)
  int32_t noise;               // uniform batch: beta=0 endpoint 3/4 n_q (0) or n_q (1)
  int32_t samples_per_sweep;   // uniform batch: n samples per sweep, 0 => 4 (colour phases)
  double ln2;                  // log 2 from the host's libm
  int64_t n;
  const int64_t* S;            // per chain
  const int32_t* n_final;      // per chain
  const uint32_t* final_rows;  // [RW][4] per item, or nullptr
  double* class_prob;          // [n][4] (caller's index)
  double* mean_n;              // [n][4] or nullptr
  uint8_t* chosen;             // [n]
  uint8_t* correction;         // uniform: [n][n_q]; plan: at item corr_off; or nullptr
  const uint8_t* flip;         // [n] (caller's index): class composed with the decision, or nullptr
};
hipError_t launch_decide(const DecideArgs& a, hipStream_t s);

hipError_t launch_sample(int L, int noise, uint32_t threshold, uint32_t k0, uint32_t k1,
                         const uint32_t* ids,
                         uint32_t id_base, int64_t n, uint8_t* syn, uint8_t* true_class,
                         uint8_t* errors, hipStream_t s);
// One sample per plan item (its L, p, id; syndrome written at syn_off, class at orig).
hipError_t launch_sample_items(const ItemDesc* items, const GroupDesc* groups, int64_t n,
                               uint32_t k0, uint32_t k1, uint8_t* syn, uint8_t* true_class,
                               hipStream_t s);

// ---- imperfect measurements (space-time hypotheses) ---------------------------
// LDS of one 64-chain workgroup of the space-time kernel (lattice tables)
// must stay within this.
// Codes up to this L run the register-interval kernel, larger ones the
// streaming-window kernel (spacetime_win.h, one translation unit per L).
constexpr int SPACETIME_FAST_L_MAX = 12;
constexpr int SPACETIME_WIN_L_MIN = SPACETIME_FAST_L_MAX + 1;
constexpr int SPACETIME_WIN_L_MAX = MCMC_L_MAX;
struct SpaceTimeArgs {
  int32_t L, T, chains, burn, sweep_end;
  int64_t n;                    // observation histories
  int64_t n_tasks;              // n * 4 * chains
  const uint32_t* ids;          // [n] or nullptr (=> i)
  const uint8_t* obs;           // [n][T][n_stab] observed outcomes
  const uint8_t* reps;          // [i*4 + cls][n_q] matching starts of the last round
  const int32_t* rep_weight;    // [i*4 + cls]
  uint32_t k0, k1;
  uint32_t sp_thr[4];           // spatial moves: A[Delta n], Delta n = 1..4
  uint32_t t_thr[25];           // time moves: [(dn+2)*5 + dm+2]
  uint32_t t_always;            // bit (dn+2)*5 + dm+2: dn + xi dm <= 0
  double xi, beta_bar;
  int64_t *Sn, *Sm, *A;         // [n][4][chains]
  int32_t *n_final, *m_final;
  uint8_t* final_c;             // [n][4][n_q] accumulated error of chain 0, or nullptr
  double *class_prob, *mean_n, *mean_m;
  uint8_t* chosen;
  uint8_t* correction;          // [n][n_q] or nullptr
  uint32_t* state;              // hypotheses: [words per chain][n_tasks]
};
hipError_t launch_spacetime_sample(int L, int T, uint32_t thr_d, uint32_t thr_m, uint32_t k0,
                                   uint32_t k1, uint32_t id_base, int64_t n, uint8_t* obs,
                                   uint8_t* true_class, hipStream_t s);
// Copies the last round of every history: last [n][n_stab].
hipError_t launch_spacetime_last(int64_t n, int T, int nstab, const uint8_t* obs, uint8_t* last,
                                 hipStream_t s);
hipError_t launch_spacetime_chains(const SpaceTimeArgs& a, hipStream_t s);
hipError_t launch_spacetime_decide(const SpaceTimeArgs& a, hipStream_t s);

// ---- device-built budget plans ----------------------------------------------
// One code size, three groups by sweep budget: 0 = sweeps[0] (full), 1 =
// sweeps[1] (short), 2 = sweeps[2] (none); route r of syndrome i puts it in
// group 0 (r = 2), 1 (r = 1) or 2 (r = 0).
struct BudgetArgs {
  int64_t n;
  const uint8_t* route;         // [n]
  const uint32_t* ids;          // [n] syndrome ids
  const double* beta;           // [n] beta_bar per syndrome (tables [n][K][4]), or nullptr
  double beta0;                 // beta_bar when beta is nullptr
  int64_t table0_off;           // offset of the one table [K][4] when beta is nullptr
  int32_t L, K, C, burn;
  int32_t sweeps[3];
  uint32_t* counts;             // [8] scratch, cleared here
  GroupDesc* groups;            // [3] out
  ItemDesc* items;              // [n] out
  uint32_t* tile_cum;           // [3] out: cumulative tiles of groups 0..2
};
hipError_t launch_budget_plan(const BudgetArgs& a, hipStream_t s);

// ---- gate network -----------------------------------------------------------
// Offsets (in floats) of the parameter blocks in the flat fp32 vector.
struct CnnOffsets {
  int64_t W1, b1, W2, b2, W3, b3, Wh, bh, total;
};
// Byte offsets of the buffers in a gate-network workspace for L and batch B.
struct CnnWorkspace {
  size_t x0, a1, a2, a3, wb1, wb2, wb3, wt2, wt3, whb, dz, dp3, dp2, dp1, part, partb, hpart,
      loss, bytes;
};
// Byte offsets of the bf16 weight copies (the workspace of cnn_infer).
struct CnnWeights {
  size_t wb1, wb2, wb3, wt2, wt3, whb, bytes;
};
CnnOffsets cnn_offsets(int L);
CnnWeights cnn_weights(int L);
// Samples per workgroup of the fused inference kernel on the current device
// (0 if one sample does not fit in its LDS).
int cnn_infer_group(int L);
// Logits of the forward pass with every activation kept on chip; identical
// to cnn_forward's.
hipError_t cnn_infer(int L, int64_t B, const float* prm, const uint8_t* syn, const float* p,
                     float* logits, char* ws, hipStream_t s);
CnnWorkspace cnn_workspace(int L, int64_t B);
hipError_t cnn_forward(int L, int64_t B, const float* prm, const uint8_t* syn, const float* p,
                       float* logits, char* ws, hipStream_t s);
hipError_t cnn_backward(int L, int64_t B, const float* prm, const float* logits, const float* tgt,
                        const int32_t* budget, float wb, float* grads, float* loss, char* ws,
                        hipStream_t s);
hipError_t cnn_adam(int64_t n, float* prm, const float* g, float* m, float* v, float lr, float b1,
                    float b2, float eps, float c1, float c2, hipStream_t s);
// route, argmax class, confidences [B][3] (or nullptr) and, when flip is
// not nullptr, the class to compose with the start decision (class route)
// The start-weight gap route of the gate (table == nullptr: off): weights
// [B][4] class start weights, p [B] fp32 rates, table [MCMC_GAP_BINS].
struct GapRoute {
  const int32_t* weights = nullptr;
  const float* p = nullptr;
  const uint8_t* table = nullptr;
};
hipError_t cnn_gate(int64_t B, const float* logits, float thr, bool class_route, uint8_t* route,
                    uint8_t* cls, float* conf, uint8_t* flip, const GapRoute& gap,
                    hipStream_t s);
// flag[i] = route[i] == 1 && the replica margin z of the short run's decision
// (per-chain sums sum_n, [4][K][C] per syndrome) is below thr
hipError_t cnn_escalate_flags(int64_t n, const uint8_t* route, const int64_t* sum_n, int K, int C,
                              double thr, uint8_t* flag, hipStream_t s);
// dst[k][0..row) = src[idx[k]][0..row), k < n
hipError_t cnn_gather(int64_t n, int row, const int32_t* idx, const uint8_t* src, uint8_t* dst,
                      hipStream_t s);
// dst[idx[k]] = src[k], k < n
hipError_t cnn_scatter(int64_t n, const int32_t* idx, const uint8_t* src, uint8_t* dst,
                       hipStream_t s);
// training support (cnn_train.hip)
hipError_t cnn_init_params(int L, uint64_t seed, float* prm, hipStream_t s);
hipError_t gate_budget_labels(int64_t n, const uint8_t* d0, const uint8_t* d1, const uint8_t* d2,
                              int32_t* budget, hipStream_t s);
// out[i][k] = prob[i][k ^ (start[i] & 3)]
hipError_t gate_relative_targets(int64_t n, const uint8_t* start, const float* prob, float* out,
                                 hipStream_t s);
int permutation_half_bits(int64_t n);
hipError_t cnn_permutation(int64_t n, uint64_t seed, uint32_t epoch, int32_t* perm,
                           hipStream_t s);
// acc[0] (+)= sum of loss[0..B) in index order (reset: acc[0] = 0 first)
hipError_t cnn_loss_sum(int64_t B, const float* loss, double* acc, bool reset, hipStream_t s);
// corr[idx[k]][..] = reps[k][cls[idx[k]]][..], rows of n_q bytes
hipError_t cnn_pick(int64_t n, int nq, const int32_t* idx, const uint8_t* cls,
                    const uint8_t* reps, uint8_t* corr, hipStream_t s);

}  // namespace mcmc
