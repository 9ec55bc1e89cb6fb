/*
 * mcmcdec — single-temperature MCMC decoder for the planar surface code on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: A. Hutter, J. R. Wootton, D. Loss, "An efficient Markov chain Monte
 * Carlo algorithm for the surface code", arXiv:1302.2669.  Given the anyon
 * configuration (syndrome) of a distance-L planar code under depolarizing
 * noise, the decoder runs Metropolis chains over the stabilizer-equivalent
 * error configurations of each of the four logical classes (Sec. IV), turns
 * the chain averages of the error count n into class probabilities with the
 * thermodynamic-integration identity (Eq. main), and picks the most likely
 * class (Sec. IV.A).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Lattice   (2L-1)x(2L-1) grid; data qubits on cells (r,c) with r+c even,
 *            numbered row-major: n_q = 2L^2-2L+1.  Stars (sigma^x stabilizers)
 *            on (r odd, c even), plaquettes (sigma^z) on (r even, c odd);
 *            n_stab = 2L(L-1) (Sec. II).  Sites: stars row-major, then
 *            plaquettes row-major.
 *  Pauli     one byte per qubit: bit 0 = x part, bit 1 = z part
 *            (0=I, 1=X, 2=Z, 3=Y).
 *  Syndrome  one byte per site, 0 = unlit, nonzero = lit.  A star is lit by an
 *            odd number of z parts on its qubits, a plaquette by x parts.
 *            Every syndrome is valid.
 *  Class     bx + 2*bz, bx = parity of x parts on grid column 0, bz = parity
 *            of z parts on grid row 0 (0=I, 1=X-bar, 2=Z-bar, 3=Y-bar).
 *  Colours   a sweep applies colour 0 (stars, i+j even), 1 (stars, odd),
 *            2 (plaquettes, even), 3 (plaquettes, odd); sites of one colour
 *            share no qubit (Sec. V's four groups).
 *  Random    Philox4x32-10, key = (seed lo, seed hi).  Draw d of a sweep
 *            (d = colour*L(L-1)/2 + rank of the site in its colour) is word
 *            d&3 at counter (d>>2, sweep, syndrome_id,
 *            cls<<28 | temp<<20 | chain); temp runs 1..K.
 *  Accept    Delta n <= 0, or u < A_k[Delta n] with
 *            A_k[D] = floor(2^32 exp(-beta_k D)), beta_k = k*beta_bar/K,
 *            beta_bar = -log((p/3)/(1-p)) (Eq. betaBar, Sec. IV).
 *  Noise     depolarizing (default): n = number of non-identity qubits.
 *            Independent bit/phase flips (Eq. pauliChannel with
 *            p_b = p_p = p, Sec. IV.A's last paragraph): n = number of x
 *            parts + number of z parts (Y counts twice), beta_bar =
 *            log((1-p)/p), and the single temperature beta* = 0.85 beta_bar
 *            unless the caller sets another scale.
 *
 * Pointers
 * --------
 *  Arguments named d_* are DEVICE pointers owned by the caller; h_* are host
 *  pointers.  `stream` is a hipStream_t (NULL = the default stream).  Calls
 *  that take a stream are asynchronous: they validate, enqueue kernels and
 *  return; results are ready after the stream is synchronised.  No entry point
 *  allocates device memory: scratch space comes in through `d_workspace`,
 *  sized by mcmc_workspace_size().
 *
 * Errors
 * ------
 *  Every entry point returns MCMC_OK (0) or a negative mcmc_status and never
 *  throws.  Invalid arguments are rejected before anything is enqueued.  A
 *  failed kernel launch returns MCMC_EDEVICE; faults inside kernels surface at
 *  the caller's next stream synchronisation.
 */
#ifndef MCMCDEC_H
#define MCMCDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mcmc_status {
  MCMC_OK = 0,
  MCMC_EINVAL = -1,     /* malformed argument (NULL where required, bad flag) */
  MCMC_ERANGE = -2,     /* argument outside the supported range               */
  MCMC_ENOMEM = -3,     /* host allocation failed                              */
  MCMC_EDEVICE = -4,    /* HIP runtime error (launch failure, bad device ptr)  */
  MCMC_EWORKSPACE = -5  /* workspace pointer NULL or smaller than required     */
};

#define MCMC_L_MIN 2
#define MCMC_L_MAX 25
#define MCMC_TEMPS_MAX 64
#define MCMC_CHAINS_MAX (1 << 20)
#define MCMC_SWEEPS_MAX (1 << 28)

/* noise models (mcmc_params.noise) */
#define MCMC_NOISE_DEPOLARIZING 0u /* X, Y, Z with p/3 each; 0 < p < 0.75        */
#define MCMC_NOISE_BITPHASE 1u     /* x part and z part each with p,
                                      independently; 0 < p < 0.5               */

/* flags */
#define MCMC_TRACE 1u  /* write n after every colour phase to d_trace          */
#define MCMC_RESUME 2u /* start from d_chain_state instead of the class starts */
#define MCMC_RANDOM_SCAN 4u /* Sec. IV's chain: each step applies the Metropolis
                               rule to one stabilizer chosen uniformly at random
                               (Philox block t>>1 of sweep s at counter (t>>1, s,
                               syndrome_id, 2<<30 | cls<<28 | temp<<20 | chain),
                               word 2(t&1) -> site floor(u n_stab / 2^32), word
                               2(t&1)+1 -> acceptance); n_stab steps per sweep,
                               n summed after every step (d_sum_n counts
                               n_stab samples per sweep).  Not with MCMC_TRACE. */

/* class starts (Sec. IV: one starting configuration per class, consistent
 * with the syndrome) */
#define MCMC_INIT_CANONICAL 0u /* every anyon's string to the left (plaquettes) or
                                  top (stars) boundary, times the logicals     */
#define MCMC_INIT_MATCHING 1u  /* greedy matching per anyon type plus the
                                  cheapest parity change per class (an
                                  approximation of Sec. III's enhanced matching) */
#define MCMC_INIT_MWPM 2u      /* Sec. III's enhanced matching, exact: per anyon
                                  type and line parity the part with the fewest
                                  errors of that type (a minimum-weight perfect
                                  matching of the lit sites and the boundaries the
                                  parity needs, under shortest-path distances);
                                  class c = x part of parity c&1 + z part of
                                  parity c>>1.  Ties between equal-weight
                                  matchings go to the smallest sum of a per-pair
                                  key (from the ends' splitmix64 keys); paths
                                  are fixed per pair (see
                                  mcmc_init_representatives).  With no counted
                                  sweep the decision is the enhanced-matching
                                  decoder (fewest errors, Y counting once). */

typedef struct mcmc_params {
  int32_t L;           /* code distance, MCMC_L_MIN..MCMC_L_MAX                  */
  int32_t n_temps;     /* K: 1 (beta* = beta_bar, Sec. IV.A) or even 2..64
                          (beta_k = k beta_bar/K, Simpson's rule, Sec. IV.A)    */
  int32_t chains;      /* independent chains per class and temperature, >= 1   */
  int32_t burn;        /* uncounted sweeps at the start, >= 0                   */
  int32_t sweeps;      /* counted sweeps, >= 0: the chain covers absolute sweeps
                          [0, burn + sweeps)                                    */
  int32_t sweep_begin; /* with MCMC_RESUME: first absolute sweep of this call
                          (the state in d_chain_state is the one after sweep
                          sweep_begin-1); must be 0 otherwise                   */
  double p;            /* error rate of the noise model (beta_bar > 0)          */
  uint64_t seed;       /* Philox key                                            */
  uint32_t flags;      /* MCMC_TRACE | MCMC_RESUME | MCMC_RANDOM_SCAN           */
  uint32_t init;       /* MCMC_INIT_CANONICAL or MCMC_INIT_MATCHING             */
  uint32_t noise;      /* MCMC_NOISE_DEPOLARIZING (0) or MCMC_NOISE_BITPHASE    */
  uint32_t reserved;   /* must be 0                                             */
  double beta_scale;   /* K = 1: beta* = beta_scale * beta_bar, in (0, 4];
                          0 selects the model's default (1 depolarizing, 0.85
                          bit/phase flips).  K > 1: must be 0 or 1 (the ladder
                          runs to beta_bar).  With beta* < beta_bar the
                          estimator integrates the trapezoid over [0, beta*]
                          and holds <n> at its beta* value up to beta_bar.   */
} mcmc_params;

/* Human-readable name of a status code (static string). */
const char* mcmc_strerror(int status);

/* ABI version of this header: 0x00010500 for 1.5. */
int32_t mcmc_abi_version(void);

/* n_q and n_stab of a distance-L code (Sec. II: n_stab = 2L(L-1),
 * Sec. IV.A: n_q = n_stab + 1).  Host only.  ERANGE outside L_MIN..L_MAX. */
int mcmc_geometry(int32_t L, int32_t* h_n_qubits, int32_t* h_n_stab);

/* Host export of the lattice tables, for checking against other
 * implementations.  h_supports [n_stab][4] qubit indices, -1 padded
 * (weight-3 boundary stabilizers); h_colour [n_stab] 0..3; h_draw [n_stab]
 * the draw number d of each site within a sweep.  Any pointer may be NULL. */
int mcmc_lattice(int32_t L, int32_t* h_supports, int32_t* h_colour, int32_t* h_draw);

/* The uint32 acceptance thresholds A_k[1..4] for k = 1..n_temps, row-major
 * [n_temps][4], computed in double precision on the host (Eq. betaBar,
 * Sec. IV).  ERANGE if p is outside (0, 0.75) or n_temps outside 1..64. */
int mcmc_acceptance_table(double p, int32_t n_temps, uint32_t* h_table);

/* The thresholds a decode with *h_prm uses: [n_temps][4] for its noise
 * model, rate and beta_scale (beta_k = k beta_bar/K, or beta* for K = 1).
 * Same errors as mcmc_workspace_size for the parameters it reads. */
int mcmc_params_table(const mcmc_params* h_prm, uint32_t* h_table);

/* Bytes of device workspace mcmc_decode_batch needs for n syndromes. */
int mcmc_workspace_size(const mcmc_params* h_prm, int64_t n, size_t* h_bytes);

/* Bytes of a chain-state buffer for n syndromes (every chain's packed
 * configuration, weight, energy sum and accept count). */
int mcmc_chain_state_size(const mcmc_params* h_prm, int64_t n, size_t* h_bytes);

/*
 * Decode n syndromes of one (L, p) with the same sweep budget.
 *
 *  d_syndromes   [n][n_stab] uint8                       (required)
 *  d_syndrome_ids[n] uint32 Philox counter word 2, NULL => i (required to be
 *                distinct for independent chains across calls)
 *  d_class_prob  [n][4] double   estimated P(E) (Eq. main with the closed-form
 *                beta=0 endpoint, 3/4 n_q depolarizing or n_q bit/phase;
 *                trapezoid for K=1, Simpson for even K)
 *  d_mean_n      [n][4] double   pooled <n> at the highest temperature index
 *                (beta_bar for K > 1, beta* for K = 1)
 *  d_sum_n       [n][4][K][chains] int64  sum of n after every counted colour
 *                phase, or NULL
 *  d_accepts     [n][4][K][chains] int64  accepted moves (burn-in included), or NULL
 *  d_chosen      [n] uint8       the decided class: the one with the largest
 *                estimated Z_E, i.e. the smallest integer key
 *                sum_{k<K} w_k S_{E,k} + S_{E,K} (w_k = 4 odd k, 2 even k);
 *                ties to the lowest class.  For K=1 this is argmin <n>
 *                (Sec. IV.A).                                       (required)
 *  d_correction  [n][n_q] uint8  final configuration of chain 0 of the chosen
 *                class at k = K, or NULL
 *  d_chain_state chain-state buffer (mcmc_chain_state_size) or NULL: read at
 *                start with MCMC_RESUME, written at the end when non-NULL
 *  d_trace       [n][4][K][chains][4*(burn+sweeps-sweep_begin)] int16, n after
 *                every colour phase; required with MCMC_TRACE (may be NULL when
 *                that length is 0), must be NULL without it
 *  d_workspace   >= mcmc_workspace_size() bytes, 256-byte aligned
 *
 * Output per syndrome depends only on its bytes, its id and *h_prm; never on
 * n, batch order or the launch configuration.
 */
int mcmc_decode_batch(const uint8_t* d_syndromes, const uint32_t* d_syndrome_ids, int64_t n,
                      const mcmc_params* h_prm, double* d_class_prob, double* d_mean_n,
                      int64_t* d_sum_n, int64_t* d_accepts, uint8_t* d_chosen,
                      uint8_t* d_correction, void* d_chain_state, int16_t* d_trace,
                      void* d_workspace, size_t workspace_bytes, void* stream);

/*
 * mcmc_decode_batch for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as mcmc_decode_batch, without the
 * workspace: the decode's scratch (mcmc_workspace_size bytes) lives in a
 * buffer of MCMC_NOALLOC_SCRATCH_BYTES inside the library, one per device,
 * reserved when the library's code is loaded on that device and held until the
 * process ends; nothing is allocated per call.  A decode needing more than
 * that (at L = 13 with 4 x 4 chains, more than about 59000 syndromes) returns
 * MCMC_EWORKSPACE before anything is enqueued.  Every call on a device shares
 * that device's buffer and keeps nothing in it between calls: calls ordered on
 * one stream are safe, calls that overlap on one device (other streams, other
 * host threads) race and corrupt each other's results.
 */
#define MCMC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mcmc_decode_batch_noalloc(const uint8_t* d_syndromes, const uint32_t* d_syndrome_ids,
                              int64_t n, const mcmc_params* h_prm, double* d_class_prob,
                              double* d_mean_n, int64_t* d_sum_n, int64_t* d_accepts,
                              uint8_t* d_chosen, uint8_t* d_correction, void* d_chain_state,
                              int16_t* d_trace, void* stream);

/* The four class starting configurations (Sec. IV: one chain start per
 * class, consistent with the syndrome) of n syndromes: d_reps [n][4][n_q]
 * uint8, row k of class k; `init` is MCMC_INIT_CANONICAL, MCMC_INIT_MATCHING
 * or MCMC_INIT_MWPM.  Asynchronous; needs no workspace.
 *
 * MCMC_INIT_MWPM in full (Sec. III).  Per anyon type (plaquettes: x parts,
 * left/right boundaries, parity = x parts on grid column 0; stars: z parts,
 * top/bottom, parity = z parts on grid row 0) and parity b, the vertex set is
 * the lit sites (i, j) of the type plus NEAR (left/top) if b = 1 plus FAR
 * (right/bottom) if (lit count + b) is odd, and the distances are
 *   d(a, a') = min(|di| + |dj|, near(a) + near(a'), far(a) + far(a')),
 *   d(a, NEAR) = near(a), d(a, FAR) = far(a), d(NEAR, FAR) = L,
 * near/far = j+1 / L-1-j (plaquettes), i+1 / L-1-i (stars).  The matching
 * minimises the sum of W = d 2^53 + 2 t over its pairs, t = the top 43 bits
 * of the 64-bit product K(a) K(a') of the ends' keys, K = splitmix64 at the
 * vertex id (id = site index, NEAR 4094, FAR 4095), so the total distance is
 * the minimum and ties go to the smallest t sum.  Pair a < a' (site order): direct path if the
 * Manhattan distance is d (plaquettes along a's grid row to the column of
 * a', then along that column; stars along a's grid column to the row of a',
 * then along that row), else both strings to the nearer boundary (NEAR on a
 * tie); boundary matches are straight strings and NEAR-FAR is the logical
 * string (X on grid row 0, Z on grid column 0).
 *
 * Resources: the syndromes too large for the first launch of the matching
 * starts are solved on a non-blocking stream of the library's, forked from
 * `stream` and joined back to it with two events.  That stream and the two
 * events are created once per device, on the first MCMC_INIT_MWPM call that
 * is not under a stream capture (or by mcmc_plan_create / mcmc_gated_create
 * with MCMC_INIT_MWPM), and kept until the process ends; until then, and
 * always for mcmc_decode_batch_noalloc, every launch goes to `stream` in
 * order.  The same holds for mcmc_decode_batch, plans and the gated decoder
 * with MCMC_INIT_MWPM starts. */
int mcmc_init_representatives(int32_t L, uint32_t init, const uint8_t* d_syndromes, int64_t n,
                              uint8_t* d_reps, void* stream);

/* The weights of the four class starts of n syndromes (the same starts as
 * mcmc_init_representatives): d_weights [n][4] int32, entry k the number of
 * qubits on which class k's start is not the identity (depolarizing weight).
 * Asynchronous; needs no workspace.  ERANGE / EINVAL as
 * mcmc_init_representatives. */
int mcmc_start_weights(int32_t L, uint32_t init, const uint8_t* d_syndromes, int64_t n,
                       int32_t* d_weights, void* stream);

/* Unpack a chain-state buffer into d_states [n][4][K][chains][n_q] uint8 and
 * d_weights [n][4][K][chains] int32, each chain's energy n under the noise
 * model of *h_prm (either pointer may be NULL). */
int mcmc_unpack_chain_state(const mcmc_params* h_prm, int64_t n, const void* d_chain_state,
                            uint8_t* d_states, int32_t* d_weights, void* stream);

/*
 * Depolarizing errors (Eq. pauliChannel, X/Y/Z with p/3 each) for sample ids
 * d_sample_ids[i] (NULL => id_base + i).  Qubit q of sample s draws
 * Philox(ctr = (q>>1, 0, s, 1<<30), key = seed) words 2(q&1), 2(q&1)+1 =
 * (u0, u1): hit iff u0 < floor(p 2^32); type (u1*3)>>32 -> X, Y, Z.
 *  d_syndromes [n][n_stab] uint8, d_true_class [n] uint8 (required),
 *  d_errors    [n][n_q] uint8 or NULL.
 */
int mcmc_sample_errors(int32_t L, double p, uint64_t seed, const uint32_t* d_sample_ids,
                       uint32_t id_base, int64_t n, uint8_t* d_syndromes, uint8_t* d_true_class,
                       uint8_t* d_errors, void* stream);

/* The same for a chosen noise model.  MCMC_NOISE_DEPOLARIZING is
 * mcmc_sample_errors.  MCMC_NOISE_BITPHASE (Eq. pauliChannel with
 * p_b = p_p = p, 0 < p < 0.5): the same two words, x part iff
 * u0 < floor(p 2^32), z part iff u1 < floor(p 2^32).  EINVAL for another
 * model. */
int mcmc_sample_errors_model(int32_t L, uint32_t noise, double p, uint64_t seed,
                             const uint32_t* d_sample_ids, uint32_t id_base, int64_t n,
                             uint8_t* d_syndromes, uint8_t* d_true_class, uint8_t* d_errors,
                             void* stream);

/*
 * Mixed batches (syndromes of different L, noise model, p, sweep budget,
 * chains and temperature count in one decode).  A plan is built once on the
 * host from an array of items; executing it enqueues the class starts, the
 * persistent chain kernels (one per L range and noise model its syndromes
 * fall in; ranges 2-13, 14-16 on the caller's stream and 17-19, 20-22, 23-25
 * on side streams, as mcmc_tuning.concurrent sets; waves take 64-chain tiles
 * from an atomic queue, longest tiles first) and the estimator, with no host
 * synchronisation.  The same sequence can be recorded into a HIP graph once
 * and replayed (mcmc_plan_graph_launch).  Per-syndrome results are identical
 * to mcmc_decode_batch with that syndrome's parameters and id, whatever the
 * batch composition or launch shape.
 */
typedef struct mcmc_item {
  int32_t L;            /* MCMC_L_MIN..MCMC_L_MAX                                  */
  int32_t sweeps;       /* counted sweeps, >= 0                                    */
  int32_t burn;         /* uncounted sweeps, >= 0                                  */
  int32_t chains;       /* chains per class and temperature, >= 1                  */
  int32_t n_temps;      /* 1 or even 2..64                                         */
  uint32_t syndrome_id; /* Philox counter word 2 of this syndrome's chains         */
  double p;             /* error rate of its noise model (as mcmc_params.p)        */
  int64_t syn_offset;   /* byte offset of its n_stab(L) syndrome bytes in the input */
  int64_t corr_offset;  /* byte offset of its n_q(L) correction bytes in the output */
  uint32_t noise;       /* MCMC_NOISE_DEPOLARIZING (0) or MCMC_NOISE_BITPHASE      */
  uint32_t reserved;    /* must be 0                                               */
  double beta_scale;    /* as mcmc_params.beta_scale (0: the model's default)      */
} mcmc_item;

/* Launch shape of a plan: workgroup size (64, 128 or 256) of the L <= 16
 * kernels (narrow) and of the L >= 17 kernels (wide); the persistent grid of
 * each kernel in waves per SIMD, as an offset (narrow -4..8, wide -2..8)
 * from the occupancy its register budget allows; the streams: all kernels
 * one after the other on the caller's stream (0), the L >= 17 kernels on one
 * side stream beside the L <= 16 ones (1), or each of the three L >= 17
 * kernels on a side stream of its own (2), joined to the caller's stream
 * before the estimator; and the chain mapping of codes with L <= 8: one
 * chain per lane (pair_small 0) or two chains per lane, the rows of both in
 * the same registers (1).  Never changes results. */
typedef struct mcmc_tuning {
  int32_t wg_narrow, occ_narrow;
  int32_t wg_wide, occ_wide;
  int32_t concurrent;
  int32_t pair_small;
} mcmc_tuning;

typedef struct mcmc_plan mcmc_plan; /* opaque */

/* Build a plan for n items (host array, copied).  Allocates the plan's device
 * tables (hipMalloc) and four streams; *plan receives the handle.  ERANGE /
 * EINVAL for an invalid item (checked before anything is allocated). */
int mcmc_plan_create(const mcmc_item* h_items, int64_t n, uint64_t seed, uint32_t init,
                     mcmc_plan** plan);
int mcmc_plan_destroy(mcmc_plan* plan);
/* Replace the plan's items (same rules as mcmc_plan_create; seed, init and
 * tuning kept).  Reuses the plan's device tables when they are large enough,
 * else reallocates them; recorded graphs are dropped.  Synchronous copies.
 * Invalid items leave the plan unchanged; a failed allocation or copy
 * (EDEVICE) leaves it empty (executions then do nothing). */
int mcmc_plan_rebuild(mcmc_plan* plan, const mcmc_item* h_items, int64_t n);

/* Total chains (length of the per-chain outputs), workspace bytes, and the
 * number of stabilizer updates one execution performs.  Any pointer may be NULL. */
int mcmc_plan_info(const mcmc_plan* plan, int64_t* h_total_chains, size_t* h_workspace_bytes,
                   int64_t* h_total_updates);
int mcmc_plan_get_tuning(const mcmc_plan* plan, mcmc_tuning* h_tuning);
int mcmc_plan_set_tuning(mcmc_plan* plan, const mcmc_tuning* h_tuning);

/*
 * Decode the plan's syndromes.  Outputs are indexed by the item's position in
 * the array given to mcmc_plan_create:
 *  d_class_prob [n][4] f64, d_mean_n [n][4] f64 or NULL, d_chosen [n] u8;
 *  d_sum_n / d_accepts: per chain, item i's [4][K][chains] block after those
 *  of items 0..i-1 (or NULL); d_correction: at each item's corr_offset (or NULL).
 */
int mcmc_plan_execute(mcmc_plan* plan, const uint8_t* d_syndromes, double* d_class_prob,
                      double* d_mean_n, int64_t* d_sum_n, int64_t* d_accepts, uint8_t* d_chosen,
                      uint8_t* d_correction, void* d_workspace, size_t workspace_bytes,
                      void* stream);

/* Same, through a HIP graph recorded on first use for this set of pointers
 * and replayed afterwards (the plan keeps the instantiated graphs). */
int mcmc_plan_graph_launch(mcmc_plan* plan, const uint8_t* d_syndromes, double* d_class_prob,
                           double* d_mean_n, int64_t* d_sum_n, int64_t* d_accepts,
                           uint8_t* d_chosen, uint8_t* d_correction, void* d_workspace,
                           size_t workspace_bytes, void* stream);

/* Samples for the plan's items (the rule of mcmc_sample_errors_model with
 * each item's L, noise model and p, sample id = its syndrome_id): syndromes
 * written at the items' syn_offset in d_syndromes, classes to d_true_class [n]. */
int mcmc_plan_sample(const mcmc_plan* plan, uint64_t seed, uint8_t* d_syndromes,
                     uint8_t* d_true_class, void* stream);

/* Pick the launch shape by timing whole executions of the plan (coordinate
 * search over workgroup size, grid sizes and stream overlap), synchronising
 * `stream`.  With cache_path, a stored shape for the same workload signature
 * (device CU count and the plan's groups) is reused, and a new one appended.
 * The chosen shape is written to *h_result when non-NULL. */
int mcmc_plan_autotune(mcmc_plan* plan, const uint8_t* d_syndromes, double* d_class_prob,
                       double* d_mean_n, int64_t* d_sum_n, int64_t* d_accepts, uint8_t* d_chosen,
                       uint8_t* d_correction, void* d_workspace, size_t workspace_bytes,
                       void* stream, const char* cache_path, mcmc_tuning* h_result);

/*
 * Gate network.  Not part of the paper's method: a small convolutional
 * network over the syndrome of one code size, trained on the decoder's own
 * class probabilities, that predicts the four class log-probabilities and a
 * sweep budget (0, short, full) so that easy syndromes skip most or all of
 * the Metropolis sweeps.  The chains themselves are unchanged.
 *
 *  Input    [L][L][3] planes per syndrome: lit star (i, j) at (i, j) (row L-1
 *           empty), lit plaquette (i, j) at (i, j) (column L-1 empty), and
 *           the syndrome's depolarizing rate p in every cell.
 *  Body     three 3x3 convolutions with 32 channels, zero padding, bias and
 *           ReLU; tap t = 3(dy+1) + (dx+1), weights W[c_out][t][c_in].
 *  Head     linear map of the flattened last activation (feature =
 *           (y L + x) 32 + c) to 7 logits: classes 0..3, budgets 0..2.
 *  Params   one fp32 vector in the order W1 [32][9][3], b1 [32], W2
 *           [32][9][32], b2, W3 [32][9][32], b3, Wh [7][32 L^2], bh [7]
 *           (mcmc_cnn_param_count floats).
 *  Numerics every matrix product takes bfloat16 operands (weights, input
 *           planes, ReLU outputs and back-propagated pre-activation
 *           gradients rounded to nearest even) with fp32 accumulation on the
 *           matrix cores; biases, logits, loss, gradients and the optimizer
 *           are fp32.  Every reduction has a fixed order: results do not
 *           depend on the launch or on timing.
 */
#define MCMC_CNN_BATCH_MAX (1 << 24)

/* Number of fp32 parameters for distance L. */
int mcmc_cnn_param_count(int32_t L, int64_t* h_count);
/* Device workspace bytes of mcmc_cnn_forward / mcmc_cnn_backward for a batch. */
int mcmc_cnn_workspace_size(int32_t L, int64_t batch, size_t* h_bytes);
/* Byte offsets in that workspace of the bfloat16 [batch L^2][channels]
 * tensors x0 (8 channels, 3 used), a1, a2, a3 (the three ReLU outputs) and
 * the pre-activation gradients of conv3, conv2, conv1 (32 channels), in that
 * order, h_offsets[7].  For inspection in tests. */
int mcmc_cnn_workspace_offsets(int32_t L, int64_t batch, int64_t* h_offsets);

/*
 * Forward pass: d_syndromes [batch][n_stab] uint8, d_p [batch] fp32,
 * d_params as above, d_logits [batch][8] fp32 (entries 0..6 written; 7 is
 * left as is).  The workspace keeps the activations for mcmc_cnn_backward.
 */
int mcmc_cnn_forward(int32_t L, int64_t batch, const float* d_params, const uint8_t* d_syndromes,
                     const float* d_p, float* d_logits, void* d_workspace, size_t workspace_bytes,
                     void* stream);

/*
 * Inference only: the same logits as mcmc_cnn_forward, bit for bit, from one
 * fused kernel that keeps a group of samples' activations in LDS through all
 * layers (nothing kept for a backward pass).  The workspace holds bf16 copies
 * of the weights (mcmc_cnn_infer_workspace_size bytes).  EDEVICE if the
 * device's LDS per workgroup cannot hold one sample.
 */
int mcmc_cnn_infer_workspace_size(int32_t L, size_t* h_bytes);
int mcmc_cnn_infer(int32_t L, int64_t batch, const float* d_params, const uint8_t* d_syndromes,
                   const float* d_p, float* d_logits, void* d_workspace, size_t workspace_bytes,
                   void* stream);

/*
 * Loss and gradients of the batch just run forward (same L, batch, params,
 * inputs and workspace, in stream order).  Loss per sample: soft
 * cross-entropy of the class logits against d_class_target [batch][4] fp32
 * plus budget_weight times the cross-entropy of the budget logits against
 * d_budget [batch] int32 in 0..2 (values outside are clamped); the objective
 * is the batch mean.  d_grads [param_count] fp32 receives its gradient;
 * d_loss [batch] fp32 the per-sample losses, or NULL.
 */
int mcmc_cnn_backward(int32_t L, int64_t batch, const float* d_params, const float* d_logits,
                      const float* d_class_target, const int32_t* d_budget, float budget_weight,
                      float* d_grads, float* d_loss, void* d_workspace, size_t workspace_bytes,
                      void* stream);

/* One Adam step number `step` (>= 1) over n_params floats, in place on
 * d_params, d_m, d_v: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * w -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
int mcmc_cnn_step(int64_t n_params, int64_t step, float lr, float beta1, float beta2, float eps,
                  float* d_params, const float* d_grads, float* d_m, float* d_v, void* stream);

/*
 * Initial parameters for distance L: He-normal weights (standard deviation
 * sqrt(2 / fan-in), fan-in 27, 288, 288 and 32 L^2 for W1, W2, W3, Wh) and
 * zero biases.  Weight i of the flat vector is
 * sqrt(-2 ln((a + 1) 2^-32)) cos(2 pi b 2^-32) sqrt(2 / fan-in), computed in
 * double and rounded to float, where (a, b) are words 2(i&1), 2(i&1)+1 of
 * Philox4x32-10 at counter (i >> 1, 0, 0, 3<<30 | 3<<28 | 0xFE<<20), key =
 * seed (Box-Muller).
 */
int mcmc_cnn_init(int32_t L, uint64_t seed, float* d_params, void* stream);

/*
 * Budget labels of the gate from three decisions of each syndrome (no
 * sweep, short budget, full budget): d_budget[i] = 0 if d_zero[i] ==
 * d_full[i], else 1 if d_short[i] == d_full[i], else 2.
 */
int mcmc_gate_budget_labels(int64_t n, const uint8_t* d_zero, const uint8_t* d_short,
                            const uint8_t* d_full, int32_t* d_budget, void* stream);

/*
 * Class targets of the gate read relative to each syndrome's start decision
 * (the class whose start has the fewest errors, i.e. the no-sweep decision):
 * d_targets[i][k] = d_class_prob[i][k ^ (d_start_class[i] & 3)], f32 [n][4].
 * Classes are indexed by the two logical parities (bit 0: X-bar, bit 1:
 * Z-bar), so XOR composes two classes and entry 0 is the probability that
 * the start decision is the right class.  The two arrays must not overlap
 * (EINVAL).
 */
int mcmc_gate_relative_targets(int64_t n, const uint8_t* d_start_class, const float* d_class_prob,
                               float* d_targets, void* stream);

/*
 * The keyed shuffle of training epoch `epoch`: d_perm [n] a permutation of
 * 0..n-1.  With b the smallest even number >= 2 for which 2^b >= n and
 * h = b/2, position i maps through a 4-round Feistel network on b bits
 * ((l, r) -> (r, l xor F_k(r)), l the high h bits), F_k(r) = the low h bits
 * of word 0 of Philox4x32-10 at counter (r, k, epoch, 3<<30 | 3<<28 | 0xFD<<20),
 * key = seed, repeated (cycle walking) until the value is below n.
 */
int mcmc_cnn_permutation(int64_t n, uint64_t seed, uint32_t epoch, int32_t* d_perm,
                         void* stream);

/*
 * One training epoch on the device: the samples (syndromes [n][n_stab],
 * rates [n] fp32, class targets [n][4] fp32, budget labels [n] int32) are
 * taken in the order of mcmc_cnn_permutation(n, seed, epoch) in mini-batches
 * of `batch` (the last partial batch dropped); each batch runs
 * mcmc_cnn_forward, mcmc_cnn_backward and one Adam step (mcmc_cnn_step) with
 * step number *h_step + 1 and learning rate
 * lr + (lr_final - lr) * *h_step / max(1, total_steps - 1), then *h_step is
 * incremented.  d_loss_sum[0] receives the sum of the epoch's per-sample
 * losses (added batch by batch in sample order).  The workspace holds the
 * permutation, the gathered batch, logits, gradients and the network's own
 * workspace (mcmc_cnn_train_workspace_size).
 */
typedef struct mcmc_train_config {
  float lr, lr_final;     /* learning rate at the first and last step           */
  float beta1, beta2, eps;
  float budget_weight;    /* weight of the budget term of the loss              */
  int64_t batch;          /* samples per step, 1..MCMC_CNN_BATCH_MAX             */
  int64_t total_steps;    /* steps of the whole run (for the learning rate)      */
  uint64_t seed;          /* key of the shuffle                                  */
} mcmc_train_config;
int mcmc_cnn_train_workspace_size(int32_t L, int64_t n, int64_t batch, size_t* h_bytes);
int mcmc_cnn_train_epoch(int32_t L, int64_t n, const mcmc_train_config* h_cfg, uint32_t epoch,
                         int64_t* h_step, float* d_params, float* d_m, float* d_v,
                         const uint8_t* d_syndromes, const float* d_p,
                         const float* d_class_target, const int32_t* d_budget,
                         double* d_loss_sum, void* d_workspace, size_t workspace_bytes,
                         void* stream);

/*
 * Gate from logits [batch][8]: d_class = argmax of the class logits (ties to
 * the lowest); with q = softmax of the budget logits and c = the largest
 * entry of the class softmax, d_confidence [batch][3] = (q0, q0 + q1, c) (or
 * NULL): the predicted probabilities that no sweep, and that at most the
 * short budget, already give the full-budget decision, and the class head's
 * confidence.  d_route = 0 if q0 >= threshold, else 1 if q0 + q1 >=
 * threshold, else 2.  With class_route != 0 (a class head trained on targets
 * relative to the start decision, mcmc_gate_relative_targets) the route is
 * also 0 when c >= threshold: the answer is then the start decision composed
 * with d_class.
 */
int mcmc_cnn_gate(int64_t batch, const float* d_logits, float threshold, int32_t class_route,
                  uint8_t* d_route, uint8_t* d_class, float* d_confidence, void* stream);

/*
 * Gated decoder for one code size.  The network (mcmc_cnn_infer) runs on the
 * whole batch and its gate sets each syndrome's sweep budget: route 0 = no
 * counted sweep (the decision from the class starts alone), 1 =
 * sweeps_short, 2 = sweeps_full.  All syndromes then run as one mixed plan
 * (one persistent launch of every budget).  Every output is exactly that of
 * mcmc_decode_batch with the syndrome's p, id and final budget; the network
 * only chooses the budget, except under class_route (below).
 *
 * class_route != 0: the class head is read relative to the start decision
 * (mcmc_cnn_gate); a syndrome it is confident on takes route 0 and its answer
 * is the no-sweep decision composed with the predicted class, its correction
 * the start of that class.  Not combined with escalation (EINVAL).
 *
 * escalate > 0: a route-1 syndrome whose short-run decision has a replica
 * margin below `escalate` is decoded again with sweeps_full (route 3): its
 * chains are keyed by sweep, so this extends the same chains.  The margin:
 * each replica r (chain index) has, per class e, its share of the decision
 * key, sum_k w_k S[e][k][r] (w = 4, 2, ..., 4, 1 as in the decision, 1 for
 * K = 1); with m_e and v_e the mean and sample variance of those over the C
 * replicas, b the decided class and s the runner-up, z = (m_s - m_b) /
 * sqrt((v_b + v_s) / C) (infinite if the spread is zero and m_s > m_b, zero
 * if m_s = m_b).  Needs chains >= 2.
 */
/*
 * The start-weight gap route (not in the paper; a rule beside the network).
 * The gap of a syndrome is the second-smallest minus the smallest of its
 * four class start weights (mcmc_start_weights); its rate bin is
 * floor(p * 100) computed in fp32 (p rounded to fp32, the product rounded to
 * fp32), capped at MCMC_GAP_BINS - 1.  With a table set, a syndrome the
 * network does not send to route 0 takes route 0 (the no-sweep decision,
 * class unchanged) when its gap is at least its bin's entry; an entry of
 * MCMC_GAP_NEVER never does.
 */
#define MCMC_GAP_BINS 50
#define MCMC_GAP_NEVER 255u

/* Fit of the gap table from labelled samples: h_table [MCMC_GAP_BINS]
 * receives, per rate bin, the smallest G < MCMC_GAP_NEVER such that among
 * the bin's samples with gap >= G at least min_count remain and the number
 * whose budget label (mcmc_gate_budget_labels) is not 0 is at most
 * max_miss times their count (compared in double); MCMC_GAP_NEVER if none.
 * h_p [n] host rates, d_weights [n][4] and d_budget [n] device arrays.
 * Copies them to the host and waits on the stream.  EINVAL on null pointers,
 * ERANGE on n < 0, max_miss outside [0, 1], min_count < 1 or a rate that
 * mcmc_gated_decode would reject. */
int mcmc_gate_fit_gap_table(int64_t n, const double* h_p, const int32_t* d_weights,
                            const int32_t* d_budget, double max_miss, int32_t min_count,
                            uint8_t* h_table, void* stream);

typedef struct mcmc_gate_config {
  int32_t L;            /* code distance                                           */
  int32_t n_temps;      /* K of the Metropolis routes (1 or even)                  */
  int32_t chains;       /* chains per class and temperature                        */
  int32_t burn;         /* uncounted sweeps                                        */
  int32_t sweeps_short; /* counted sweeps of route 1                               */
  int32_t sweeps_full;  /* counted sweeps of route 2                               */
  double p;             /* rate used when no per-syndrome rates are given          */
  uint64_t seed;        /* Philox key of the chains                                */
  uint32_t init;        /* MCMC_INIT_CANONICAL, _MATCHING or _MWPM                  */
  float threshold;      /* minimum gate confidence for routes 0 and 1             */
  float escalate;       /* route-1 syndromes with a replica margin below this
                           take the full budget; 0 = never                        */
  int64_t max_batch;    /* largest batch a call may pass                           */
  int32_t class_route;  /* 1: the class head, relative to the start decision,
                           may answer (route 0); 0: the budget head alone         */
} mcmc_gate_config;

typedef struct mcmc_gated mcmc_gated; /* opaque */

/* Build a gated decoder; allocates its plan's device tables (sized for
 * max_batch syndromes) and pinned host staging buffers. */
int mcmc_gated_create(const mcmc_gate_config* h_cfg, mcmc_gated** gated);
int mcmc_gated_destroy(mcmc_gated* gated);
/* Device workspace bytes of mcmc_gated_decode (any batch up to max_batch). */
int mcmc_gated_workspace_size(const mcmc_gated* gated, size_t* h_bytes);
/* The decoder's internal plan (for mcmc_plan_set_tuning / get_tuning). */
int mcmc_gated_plan(mcmc_gated* gated, mcmc_plan** h_plan);
/* The gap route's table of the decoder: h_table [MCMC_GAP_BINS] (copied,
 * the call waits for the copy), or NULL to switch the route off (the
 * default).  Not while a decode of this decoder is in flight (the device
 * copy of the table is shared by its calls).  The decoder then computes every syndrome's class starts before
 * the gate (with escalation, in a launch of their own that only counts the
 * weights, before the plan's). */
int mcmc_gated_set_gap_table(mcmc_gated* gated, const uint8_t* h_table);

/*
 * Decode n <= max_batch syndromes d_syndromes [n][n_stab] with network
 * parameters d_params.  h_ids [n] host syndrome ids (NULL => i), h_p [n] host
 * rates (NULL => the configured p).  Outputs: d_chosen [n] (required),
 * d_route [n] (0..3) and d_logits [n][8] (or NULL), d_correction [n][n_q]
 * (or NULL), h_counts [4] syndromes per final route (or NULL).
 * Without escalation the routes become a three-group plan on the device and
 * the persistent kernel reads its tile ranges there: the call enqueues
 * everything and returns (it waits on the stream only to fill h_counts, and
 * on its own host-to-device copies of the previous call before reusing their
 * staging buffers).  With escalation it waits for the gate and for the short
 * runs' estimates to build each plan on the host, and returns with the
 * stream drained.
 */
int mcmc_gated_decode(mcmc_gated* gated, const float* d_params, const uint8_t* d_syndromes,
                      const uint32_t* h_ids, const double* h_p, int64_t n, uint8_t* d_chosen,
                      uint8_t* d_route, float* d_logits, uint8_t* d_correction,
                      int64_t* h_counts, void* d_workspace, size_t workspace_bytes,
                      void* stream);

/*
 * Imperfect stabilizer measurements (Sec. VI).  Stabilizers are measured in
 * `rounds` = T rounds; before round t every data qubit suffers depolarizing
 * noise of rate p (interval t) and every outcome of rounds 0..T-2 is wrong
 * with probability p_m; the last round is perfect.  Round t reports
 * s_t = syn(E_0 ... E_t) xor M_t.  A hypothesis (E_0..E_{T-1}, M_0..M_{T-2})
 * with n data errors and m wrong outcomes has weight exp(-beta_bar (n + xi m)),
 * xi = log((1-p_m)/p_m) / beta_bar.  Chains (one per class and replica, at
 * beta_bar) move by spatial stabilizers within an interval and by Sec. VI's
 * time moves (a Pauli on one qubit in intervals t and t+1 with the outcomes
 * of round t that it anticommutes with toggled).  A sweep is every spatial
 * move (t = 0..T-1, sites in order) then every time move (t = 0..T-2,
 * qubits in order, X before Z); move (t, k) uses draw d = t n_stab + k and
 * move (t, q, P) d = T n_stab + 2 t (n_q + 1) + 2 q + (P == Z), word d & 3 of
 * Philox at (d >> 2, sweep, id, 3<<30 | cls<<28 | 1<<20 | chain).  A move with
 * E = dn + xi dm <= 0 is taken, else iff u < floor(2^32 exp(-beta_bar E)).
 * n and m are summed after each half of a counted sweep; the decision is the
 * class with the smallest S_n + xi S_m (float64), ties to the lowest class.
 * Class starts: every flipped outcome before the last round blamed on the
 * measurement (M_t = s_t, t < T-1), no data error before the last interval,
 * and E_{T-1} the class-c MCMC_INIT_MATCHING start of s_{T-1}.
 * The hypotheses, T ceil(n_q/16) + (T-1) ceil(n_stab/32) words per chain,
 * live in the workspace; up to L = 13 the chains keep their current
 * intervals in registers.
 */
#define MCMC_ROUNDS_MAX 64

typedef struct mcmc_spacetime_params {
  int32_t L;          /* MCMC_L_MIN..MCMC_L_MAX                               */
  int32_t rounds;     /* T, 1..MCMC_ROUNDS_MAX (T = 1: one perfect round)      */
  int32_t chains;     /* chains per class, >= 1                                */
  int32_t burn;       /* uncounted sweeps, >= 0                                */
  int32_t sweeps;     /* counted sweeps, >= 0                                  */
  int32_t reserved;   /* must be 0                                             */
  double p;           /* depolarizing rate per interval, 0 < p < 0.75          */
  double p_m;         /* outcome error rate, 0 < p_m < 0.5                     */
  uint64_t seed;      /* Philox key                                            */
} mcmc_spacetime_params;

/* Bytes of device workspace for n observation histories. */
int mcmc_spacetime_workspace_size(const mcmc_spacetime_params* h_prm, int64_t n,
                                  size_t* h_bytes);

/* Host tables of a decode: spatial thresholds [4] (Delta n = 1..4), time-move
 * thresholds [25] at (dn+2)*5 + dm+2, the always-accept mask (bit (dn+2)*5 +
 * dm+2 set iff dn + xi dm <= 0) and xi.  Any pointer may be NULL. */
int mcmc_spacetime_tables(const mcmc_spacetime_params* h_prm, uint32_t* h_spatial,
                          uint32_t* h_time, uint32_t* h_always, double* h_xi);

/*
 * Decode n observation histories d_obs [n][T][n_stab] uint8 (nonzero = -1
 * outcome).  d_ids [n] Philox counter word 2 (NULL => i).  Outputs (device):
 * d_class_prob [n][4] (Eq. main, trapezoid on [0, beta_bar], beta = 0
 * endpoint 3/4 n_q T + xi n_stab (T-1)/2), d_mean_n / d_mean_m [n][4] pooled
 * <n>, <m> (or NULL), d_sum_n / d_sum_m / d_accepts [n][4][chains] int64 (or
 * NULL), d_chosen [n] (required), d_correction [n][n_q] the accumulated data
 * error of chain 0 of the chosen class (or NULL).  Asynchronous on `stream`.
 * ERANGE for n > 2^28 or n * 4 * chains > 2^36.
 */
int mcmc_decode_spacetime(const uint8_t* d_obs, const uint32_t* d_ids, int64_t n,
                          const mcmc_spacetime_params* h_prm, double* d_class_prob,
                          double* d_mean_n, double* d_mean_m, int64_t* d_sum_n, int64_t* d_sum_m,
                          int64_t* d_accepts, uint8_t* d_chosen, uint8_t* d_correction,
                          void* d_workspace, size_t workspace_bytes, void* stream);

/* Samples of the model for ids id_base + i: interval t's data errors follow
 * mcmc_sample_errors' rule with counter word 1 = 1 + t; outcome k of round
 * t < T-1 is wrong iff word k & 3 of Philox at (k >> 2, 0x80000000 | t, id,
 * 1<<30) is below floor(p_m 2^32).  d_obs [n][T][n_stab], d_true_class [n]
 * (class of E_0 ... E_{T-1}). */
int mcmc_sample_spacetime(int32_t L, int32_t rounds, double p, double p_m, uint64_t seed,
                          uint32_t id_base, int64_t n, uint8_t* d_obs, uint8_t* d_true_class,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MCMCDEC_H */
