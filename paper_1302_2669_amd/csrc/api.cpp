// C-ABI of libmcmcdec (declared in include/mcmcdec.h): argument validation,
// host-side tables, workspace carving and kernel enqueueing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>


#include "../../include/mcmcdec.h"
#include "device_common.h"
#include "host_common.h"
#include "internal.h"

#include <algorithm>
#include <mutex>

namespace mcmc {

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  if (dev >= 64) dev = 63;
  if (cached[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

ChainStateLayout chain_state_layout(int L, int64_t T) {
  ChainStateLayout c{};
  size_t off = 0;
  c.rows = off; off = align_up(off + (size_t)words_per_config(L) * T * sizeof(uint32_t));
  c.n = off;    off = align_up(off + (size_t)T * sizeof(int32_t));
  c.S = off;    off = align_up(off + (size_t)T * sizeof(int64_t));
  c.A = off;    off = align_up(off + (size_t)T * sizeof(int64_t));
  c.bytes = off;
  return c;
}

hipError_t launch_chains(int range, const RunArgs& a, int waves, int wg, hipStream_t s) {
  if (a.noise == MCMC_NOISE_BITPHASE) {
    switch (range) {
      case 0: return launch_chains_flip_range<0>(a, waves, wg, s);
      case 1: return launch_chains_flip_range<1>(a, waves, wg, s);
      case 2: return launch_chains_flip_range<2>(a, waves, wg, s);
      case 3: return launch_chains_flip_range<3>(a, waves, wg, s);
      case 4: return launch_chains_flip_range<4>(a, waves, wg, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.noise != MCMC_NOISE_DEPOLARIZING) return hipErrorInvalidValue;
  switch (range) {
    case 0: return launch_chains_range<0>(a, waves, wg, s);
    case 1: return launch_chains_range<1>(a, waves, wg, s);
    case 2: return launch_chains_range<2>(a, waves, wg, s);
    case 3: return launch_chains_range<3>(a, waves, wg, s);
    case 4: return launch_chains_range<4>(a, waves, wg, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mcmc

// Scratch of mcmc_decode_batch_noalloc: one copy on every device the library
// runs on, held until the process ends.  Host code uses only the per-device
// address that hipGetSymbolAddress returns for it, never this name.
static __device__ __align__(256) uint8_t scratch[MCMC_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// address of the current device's scratch; looked up once per device, with
// that device current
int scratch_on_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MCMC_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MCMC_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MCMC_OK;
}

}  // namespace

namespace {

using namespace mcmc;

int check_params(const mcmc_params* prm, int64_t n) {
  if (!prm) return MCMC_EINVAL;
  if (n < 0) return MCMC_ERANGE;
  if (!valid_L(prm->L)) return MCMC_ERANGE;
  if (!valid_noise(prm->noise) || prm->reserved != 0) return MCMC_EINVAL;
  if (!valid_rate(prm->noise, prm->p)) return MCMC_ERANGE;
  if (prm->n_temps < 1 || prm->n_temps > MCMC_TEMPS_MAX) return MCMC_ERANGE;
  if (prm->n_temps != 1 && (prm->n_temps % 2) != 0) return MCMC_EINVAL;
  if (prm->n_temps == 1) {
    if (!(prm->beta_scale >= 0.0 && prm->beta_scale <= 4.0)) return MCMC_ERANGE;  // NaN too
  } else if (prm->beta_scale != 0.0 && prm->beta_scale != 1.0) {
    return MCMC_ERANGE;
  }
  if (prm->chains < 1 || prm->chains > MCMC_CHAINS_MAX) return MCMC_ERANGE;
  if (prm->burn < 0 || prm->sweeps < 0) return MCMC_ERANGE;
  if ((int64_t)prm->burn + prm->sweeps > MCMC_SWEEPS_MAX) return MCMC_ERANGE;
  if (prm->flags & ~(MCMC_TRACE | MCMC_RESUME | MCMC_RANDOM_SCAN)) return MCMC_EINVAL;
  if ((prm->flags & MCMC_RANDOM_SCAN) && (prm->flags & MCMC_TRACE)) return MCMC_EINVAL;
  if (prm->init != MCMC_INIT_CANONICAL && prm->init != MCMC_INIT_MATCHING &&
      prm->init != MCMC_INIT_MWPM)
    return MCMC_EINVAL;
  if (prm->flags & MCMC_RESUME) {
    if (prm->sweep_begin < 0 || prm->sweep_begin > prm->burn + prm->sweeps) return MCMC_ERANGE;
  } else if (prm->sweep_begin != 0) {
    return MCMC_EINVAL;
  }
  // chains and tiles must fit the counters (tile index is 32-bit)
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  if (n > 0 && (T / n / 4 / prm->n_temps != prm->chains || T > ((int64_t)1 << 38)))
    return MCMC_ERANGE;
  return MCMC_OK;
}

struct WorkspaceLayout {
  size_t queue, init_rows, init_n, S, A, n_final, final_rows, bytes;
};

WorkspaceLayout workspace_layout(const mcmc_params* prm, int64_t n) {
  const int RW = words_per_config(prm->L);
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  WorkspaceLayout w{};
  size_t off = 0;
  w.queue = off;      off = align_up(off + kQueueSlots * sizeof(uint32_t));
  w.init_rows = off;  off = align_up(off + (size_t)RW * n * 4 * sizeof(uint32_t));
  w.init_n = off;     off = align_up(off + (size_t)n * 4 * sizeof(int32_t));
  w.S = off;          off = align_up(off + (size_t)T * sizeof(int64_t));
  w.A = off;          off = align_up(off + (size_t)T * sizeof(int64_t));
  w.n_final = off;    off = align_up(off + (size_t)T * sizeof(int32_t));
  w.final_rows = off; off = align_up(off + (size_t)RW * n * 4 * sizeof(uint32_t));
  w.bytes = off;
  return w;
}

}  // namespace

extern "C" {

const char* mcmc_strerror(int status) {
  switch (status) {
    case MCMC_OK: return "ok";
    case MCMC_EINVAL: return "invalid argument";
    case MCMC_ERANGE: return "argument out of range";
    case MCMC_ENOMEM: return "out of host memory";
    case MCMC_EDEVICE: return "HIP runtime error";
    case MCMC_EWORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
  }
}

int32_t mcmc_abi_version(void) { return 0x00010500; }

int mcmc_geometry(int32_t L, int32_t* n_qubits, int32_t* n_stab) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (n_qubits) *n_qubits = 2 * L * L - 2 * L + 1;
  if (n_stab) *n_stab = 2 * L * (L - 1);
  return MCMC_OK;
}

int mcmc_lattice(int32_t L, int32_t* supports, int32_t* colour, int32_t* draw) {
  if (!valid_L(L)) return MCMC_ERANGE;
  const int side = 2 * L - 1;
  const int nstar = L * (L - 1);
  const int S = nstar / 2;
  auto q = [side](int r, int c) { return (r * side + c) / 2; };
  int rank[4] = {0, 0, 0, 0};
  for (int s = 0; s < 2 * nstar; ++s) {
    int r, c, col;
    if (s < nstar) {
      const int i = s / L, j = s % L;
      r = 2 * i + 1; c = 2 * j; col = (i + j) & 1;
    } else {
      const int i = (s - nstar) / (L - 1), j = (s - nstar) % (L - 1);
      r = 2 * i; c = 2 * j + 1; col = 2 + ((i + j) & 1);
    }
    if (supports) {
      int k = 0;
      const int dr[4] = {-1, 1, 0, 0}, dc[4] = {0, 0, -1, 1};
      for (int d = 0; d < 4; ++d) {
        const int rr = r + dr[d], cc = c + dc[d];
        if (rr >= 0 && rr < side && cc >= 0 && cc < side) supports[s * 4 + k++] = q(rr, cc);
      }
      for (; k < 4; ++k) supports[s * 4 + k] = -1;
    }
    if (colour) colour[s] = col;
    if (draw) draw[s] = col * S + rank[col];
    rank[col]++;
  }
  return MCMC_OK;
}

int mcmc_acceptance_table(double p, int32_t n_temps, uint32_t* table) {
  if (!table) return MCMC_EINVAL;
  if (!valid_p(p) || n_temps < 1 || n_temps > MCMC_TEMPS_MAX) return MCMC_ERANGE;
  fill_table(p, n_temps, table);
  return MCMC_OK;
}

int mcmc_params_table(const mcmc_params* prm, uint32_t* table) {
  if (!table) return MCMC_EINVAL;
  const int st = check_params(prm, 0);
  if (st != MCMC_OK) return st;
  fill_params_table(prm, table);
  return MCMC_OK;
}

int mcmc_workspace_size(const mcmc_params* prm, int64_t n, size_t* bytes) {
  if (!bytes) return MCMC_EINVAL;
  const int st = check_params(prm, n);
  if (st != MCMC_OK) return st;
  *bytes = workspace_layout(prm, n).bytes;
  return MCMC_OK;
}

int mcmc_chain_state_size(const mcmc_params* prm, int64_t n, size_t* bytes) {
  if (!bytes) return MCMC_EINVAL;
  const int st = check_params(prm, n);
  if (st != MCMC_OK) return st;
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  *bytes = chain_state_layout(prm->L, T).bytes;
  return MCMC_OK;
}

// mcmc_decode_batch; may_create: the matching starts may create their side
// stream (not for the entry point that allocates nothing)
static int decode_batch(const uint8_t* syndromes, const uint32_t* syndrome_ids, int64_t n,
                        const mcmc_params* prm, double* class_prob, double* mean_n,
                        int64_t* sum_n, int64_t* accepts, uint8_t* chosen, uint8_t* correction,
                        void* chain_state, int16_t* trace, void* workspace,
                        size_t workspace_bytes, void* stream, bool may_create) {
  int st = check_params(prm, n);
  if (st != MCMC_OK) return st;
  if (n == 0) return MCMC_OK;
  if (!syndromes || !class_prob || !chosen) return MCMC_EINVAL;
  const bool do_trace = (prm->flags & MCMC_TRACE) != 0;
  const bool resume = (prm->flags & MCMC_RESUME) != 0;
  const int64_t trace_len = 4 * (int64_t)(prm->burn + prm->sweeps - prm->sweep_begin);
  if (!do_trace && trace) return MCMC_EINVAL;
  if (do_trace && !trace && trace_len > 0) return MCMC_EINVAL;
  if (resume && !chain_state) return MCMC_EINVAL;
  const WorkspaceLayout wl = workspace_layout(prm, n);
  if (!workspace || workspace_bytes < wl.bytes) return MCMC_EWORKSPACE;
  if (((uintptr_t)workspace % kAlign) != 0) return MCMC_EWORKSPACE;
  if (chain_state && ((uintptr_t)chain_state % kAlign) != 0) return MCMC_EINVAL;

  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int L = prm->L;
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  uint32_t* queue = (uint32_t*)(ws + wl.queue);
  uint32_t* init_rows = (uint32_t*)(ws + wl.init_rows);
  int32_t* init_n = (int32_t*)(ws + wl.init_n);
  int64_t* S = sum_n ? sum_n : (int64_t*)(ws + wl.S);
  int64_t* A = accepts ? accepts : (int64_t*)(ws + wl.A);
  int32_t* nf = (int32_t*)(ws + wl.n_final);
  uint32_t* final_rows = correction ? (uint32_t*)(ws + wl.final_rows) : nullptr;

  st = hip_status(launch_zero(queue, kQueueSlots, s));
  if (st != MCMC_OK) return st;
  if (!resume) {
    StartArgs sa{};
    sa.syn = syndromes;
    sa.n = n;
    sa.L = L;
    sa.rows = init_rows;
    sa.weights = init_n;
    sa.noise = (int32_t)prm->noise;
    st = hip_status(launch_init_mode(prm->init, sa, s, may_create));
    if (st != MCMC_OK) return st;
  }

  RunArgs a{};
  a.g0.L = L;
  a.g0.K = prm->n_temps;
  a.g0.C = prm->chains;
  a.g0.burn = prm->burn;
  a.g0.sweep_begin = prm->sweep_begin;
  a.g0.sweep_end = prm->burn + prm->sweeps;
  a.g0.first_item = 0;
  a.g0.n_items = (int32_t)n;
  a.g0.n_tasks = T;
  a.syndrome_ids = syndrome_ids;
  fill_params_table(prm, &a.table0[0][0]);
  a.noise = (int32_t)prm->noise;
  a.n_tiles = (T + TILE - 1) / TILE;
  a.queue = queue;
  a.lmin = a.lmax = L;
  a.k0 = (uint32_t)(prm->seed & 0xFFFFFFFFull);
  a.k1 = (uint32_t)(prm->seed >> 32);
  a.init_rows = init_rows;
  a.init_n = init_n;
  a.S_out = S;
  a.A_out = A;
  a.n_out = nf;
  a.final_rows = final_rows;
  a.total_chains = T;
  a.trace = (do_trace && trace_len > 0) ? trace : nullptr;
  a.trace_len = trace_len;
  if (chain_state) {
    const ChainStateLayout cl = chain_state_layout(L, T);
    char* cs = (char*)chain_state;
    a.state_rows = (uint32_t*)(cs + cl.rows);
    if (resume) {
      a.resume_rows = (const uint32_t*)(cs + cl.rows);
      a.resume_n = (const int32_t*)(cs + cl.n);
      a.resume_S = (const int64_t*)(cs + cl.S);
      a.resume_A = (const int64_t*)(cs + cl.A);
    }
  }
  const bool random_scan = (prm->flags & MCMC_RANDOM_SCAN) != 0;
  if (random_scan) {
    st = hip_status(launch_chains_random(a, s));
  } else {
    const int range = range_of(L);
    const int64_t waves = std::min<int64_t>(a.n_tiles, default_waves(range, device_cus()));
    st = hip_status(launch_chains(range, a, (int)waves, 256, s));
  }
  if (st != MCMC_OK) return st;

  if (chain_state) {  // n, S, A of every chain next to the rows
    const ChainStateLayout cl = chain_state_layout(L, T);
    char* cs = (char*)chain_state;
    st = hip_status(hipMemcpyAsync(cs + cl.n, nf, (size_t)T * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
    if (st == MCMC_OK)
      st = hip_status(hipMemcpyAsync(cs + cl.S, S, (size_t)T * sizeof(int64_t),
                                     hipMemcpyDeviceToDevice, s));
    if (st == MCMC_OK)
      st = hip_status(hipMemcpyAsync(cs + cl.A, A, (size_t)T * sizeof(int64_t),
                                     hipMemcpyDeviceToDevice, s));
    if (st != MCMC_OK) return st;
  }

  DecideArgs d{};
  d.g0 = a.g0;
  d.beta_bar = beta_bar_of(prm->noise, prm->p);
  d.beta_star = beta_top(prm);
  d.noise = (int32_t)prm->noise;
  d.samples_per_sweep = random_scan ? n_stab(L) : 4;
  d.ln2 = log(2.0);
  d.n = n;
  d.S = S;
  d.n_final = nf;
  d.final_rows = final_rows;
  d.class_prob = class_prob;
  d.mean_n = mean_n;
  d.chosen = chosen;
  d.correction = correction;
  return hip_status(launch_decide(d, s));
}

int mcmc_decode_batch(const uint8_t* syndromes, const uint32_t* syndrome_ids, int64_t n,
                      const mcmc_params* prm, double* class_prob, double* mean_n, int64_t* sum_n,
                      int64_t* accepts, uint8_t* chosen, uint8_t* correction, void* chain_state,
                      int16_t* trace, void* workspace, size_t workspace_bytes, void* stream) {
  return decode_batch(syndromes, syndrome_ids, n, prm, class_prob, mean_n, sum_n, accepts, chosen,
                      correction, chain_state, trace, workspace, workspace_bytes, stream, true);
}

int mcmc_decode_batch_noalloc(const uint8_t* syndromes, const uint32_t* syndrome_ids, int64_t n,
                              const mcmc_params* prm, double* class_prob, double* mean_n,
                              int64_t* sum_n, int64_t* accepts, uint8_t* chosen,
                              uint8_t* correction, void* chain_state, int16_t* trace,
                              void* stream) {
  const int st = check_params(prm, n);
  if (st != MCMC_OK) return st;
  if (n == 0) return MCMC_OK;
  if (workspace_layout(prm, n).bytes > MCMC_NOALLOC_SCRATCH_BYTES) return MCMC_EWORKSPACE;
  void* ws = nullptr;
  const int sst = scratch_on_current_device(&ws);
  if (sst != MCMC_OK) return sst;
  // the same kernels as mcmc_decode_batch, with the device's scratch as the
  // workspace (its tile counter is zeroed by a kernel at the start of every call)
  return decode_batch(syndromes, syndrome_ids, n, prm, class_prob, mean_n, sum_n, accepts, chosen,
                      correction, chain_state, trace, ws, MCMC_NOALLOC_SCRATCH_BYTES, stream, false);
}

int mcmc_init_representatives(int32_t L, uint32_t init, const uint8_t* syndromes, int64_t n,
                              uint8_t* reps, void* stream) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (init != MCMC_INIT_CANONICAL && init != MCMC_INIT_MATCHING && init != MCMC_INIT_MWPM)
    return MCMC_EINVAL;
  if (n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!syndromes || !reps) return MCMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  StartArgs sa{};
  sa.syn = syndromes;
  sa.n = n;
  sa.L = L;
  sa.bytes = reps;
  return hip_status(launch_init_mode(init, sa, s));
}

int mcmc_start_weights(int32_t L, uint32_t init, const uint8_t* syndromes, int64_t n,
                       int32_t* weights, void* stream) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (init != MCMC_INIT_CANONICAL && init != MCMC_INIT_MATCHING && init != MCMC_INIT_MWPM)
    return MCMC_EINVAL;
  if (n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!syndromes || !weights) return MCMC_EINVAL;
  StartArgs sa{};
  sa.syn = syndromes;
  sa.n = n;
  sa.L = L;
  sa.weights = weights;
  return hip_status(launch_init_mode(init, sa, (hipStream_t)stream));
}

int mcmc_unpack_chain_state(const mcmc_params* prm, int64_t n, const void* chain_state,
                            uint8_t* states, int32_t* weights, void* stream) {
  const int st = check_params(prm, n);
  if (st != MCMC_OK) return st;
  if (n == 0) return MCMC_OK;
  if (!chain_state) return MCMC_EINVAL;
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  const ChainStateLayout cl = chain_state_layout(prm->L, T);
  return hip_status(launch_unpack(prm->L, (int)prm->noise,
                                  (const uint32_t*)((const char*)chain_state + cl.rows), T, T,
                                  states, weights, (hipStream_t)stream));
}

int mcmc_sample_errors_model(int32_t L, uint32_t noise, double p, uint64_t seed,
                             const uint32_t* sample_ids, uint32_t id_base, int64_t n,
                             uint8_t* syndromes, uint8_t* true_class, uint8_t* errors,
                             void* stream) {
  if (!valid_noise(noise)) return MCMC_EINVAL;
  if (!valid_L(L) || !valid_rate(noise, p) || n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!syndromes || !true_class) return MCMC_EINVAL;
  if (n > 0x7FFFFFFF) return MCMC_ERANGE;
  const uint32_t thr = (uint32_t)floor(ldexp(p, 32));
  return hip_status(launch_sample(L, (int)noise, thr, (uint32_t)(seed & 0xFFFFFFFFull),
                                  (uint32_t)(seed >> 32), sample_ids, id_base, n, syndromes,
                                  true_class, errors, (hipStream_t)stream));
}

int mcmc_sample_errors(int32_t L, double p, uint64_t seed, const uint32_t* sample_ids,
                       uint32_t id_base, int64_t n, uint8_t* syndromes, uint8_t* true_class,
                       uint8_t* errors, void* stream) {
  return mcmc_sample_errors_model(L, MCMC_NOISE_DEPOLARIZING, p, seed, sample_ids, id_base, n,
                                  syndromes, true_class, errors, stream);
}

}  // extern "C"
