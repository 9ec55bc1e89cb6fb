// C-ABI of libmcmcdec (declared in include/mcmcdec.h): argument validation,
// host-side tables, workspace carving and kernel enqueueing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/mcmcdec.h"
#include "device_common.h"
#include "internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool valid_L(int32_t L) { return L >= MCMC_L_MIN && L <= MCMC_L_MAX; }

// beta_bar = -log((p/3)/(1-p))  (Eq. betaBar)
double beta_bar(double p) { return -log((p / 3.0) / (1.0 - p)); }

bool valid_p(double p) { return p > 0.0 && p < 0.75; }  // false for NaN

int check_params(const mcmc_params* prm, int64_t n) {
  if (!prm) return MCMC_EINVAL;
  if (n < 0) return MCMC_ERANGE;
  if (!valid_L(prm->L)) return MCMC_ERANGE;
  if (!valid_p(prm->p)) return MCMC_ERANGE;
  if (prm->n_temps < 1 || prm->n_temps > MCMC_TEMPS_MAX) return MCMC_ERANGE;
  if (prm->n_temps != 1 && (prm->n_temps % 2) != 0) return MCMC_EINVAL;
  if (prm->chains < 1 || prm->chains > MCMC_CHAINS_MAX) return MCMC_ERANGE;
  if (prm->burn < 0 || prm->sweeps < 0) return MCMC_ERANGE;
  if ((int64_t)prm->burn + prm->sweeps > MCMC_SWEEPS_MAX) return MCMC_ERANGE;
  if (prm->flags & ~(MCMC_TRACE | MCMC_RESUME)) return MCMC_EINVAL;
  if (prm->init != MCMC_INIT_CANONICAL && prm->init != MCMC_INIT_MATCHING) return MCMC_EINVAL;
  if (prm->flags & MCMC_RESUME) {
    if (prm->sweep_begin < 0 || prm->sweep_begin > prm->burn + prm->sweeps) return MCMC_ERANGE;
  } else if (prm->sweep_begin != 0) {
    return MCMC_EINVAL;
  }
  // task count must fit the 1-D grid (blocks of 256 lanes, 32-bit block index)
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  if (n > 0 && (T / n / 4 / prm->n_temps != prm->chains || T > ((int64_t)1 << 38)))
    return MCMC_ERANGE;
  return MCMC_OK;
}

struct WorkspaceLayout {
  size_t init_rows, init_n, S, A, n_final, corr_rows, bytes;
};

WorkspaceLayout workspace_layout(const mcmc_params* prm, int64_t n) {
  const int RW = mcmc::words_per_config(prm->L);
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  WorkspaceLayout w{};
  size_t off = 0;
  w.init_rows = off; off = align_up(off + (size_t)RW * n * 4 * sizeof(uint32_t));
  w.init_n = off;    off = align_up(off + (size_t)n * 4 * sizeof(int32_t));
  w.S = off;         off = align_up(off + (size_t)T * sizeof(int64_t));
  w.A = off;         off = align_up(off + (size_t)T * sizeof(int64_t));
  w.n_final = off;   off = align_up(off + (size_t)T * sizeof(int32_t));
  w.corr_rows = off; off = align_up(off + (size_t)RW * n * 4 * sizeof(uint32_t));
  w.bytes = off;
  return w;
}

void fill_table(double p, int32_t K, uint32_t* out) {
  const double bb = beta_bar(p);
  for (int k = 1; k <= K; ++k) {
    const double beta = ((double)k * bb) / (double)K;
    for (int d = 1; d <= 4; ++d) {
      const double w = exp(-(beta * (double)d));
      out[(k - 1) * 4 + (d - 1)] = (uint32_t)floor(ldexp(w, 32));
    }
  }
}

int hip_status(hipError_t e) { return e == hipSuccess ? MCMC_OK : MCMC_EDEVICE; }

}  // namespace

namespace mcmc {

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

}  // namespace mcmc

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

int32_t mcmc_abi_version(void) { return 0x00010000; }

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
  *bytes = mcmc::chain_state_layout(prm->L, T).bytes;
  return MCMC_OK;
}

int mcmc_decode_batch(const uint8_t* syndromes, const uint32_t* syndrome_ids, int64_t n,
                      const mcmc_params* prm, double* class_prob, double* mean_n, int64_t* sum_n,
                      int64_t* accepts, uint8_t* chosen, uint8_t* correction, void* chain_state,
                      int16_t* trace, void* workspace, size_t workspace_bytes, void* stream) {
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
  uint32_t* init_rows = (uint32_t*)(ws + wl.init_rows);
  int32_t* init_n = (int32_t*)(ws + wl.init_n);
  int64_t* S = sum_n ? sum_n : (int64_t*)(ws + wl.S);
  int64_t* A = accepts ? accepts : (int64_t*)(ws + wl.A);
  int32_t* nf = (int32_t*)(ws + wl.n_final);
  uint32_t* corr_rows = correction ? (uint32_t*)(ws + wl.corr_rows) : nullptr;

  if (!resume) {
    st = hip_status(prm->init == MCMC_INIT_MATCHING
                        ? mcmc::launch_init_matching(L, syndromes, n, init_rows, init_n, nullptr, s)
                        : mcmc::launch_init(L, syndromes, n, init_rows, init_n, nullptr, s));
    if (st != MCMC_OK) return st;
  }

  mcmc::ChainArgs a{};
  a.init_rows = init_rows;
  a.init_n = init_n;
  a.syndrome_ids = syndrome_ids;
  a.n = n;
  a.K = prm->n_temps;
  a.C = prm->chains;
  a.burn = prm->burn;
  a.sweep_begin = prm->sweep_begin;
  a.sweep_end = prm->burn + prm->sweeps;
  a.k0 = (uint32_t)(prm->seed & 0xFFFFFFFFull);
  a.k1 = (uint32_t)(prm->seed >> 32);
  fill_table(prm->p, prm->n_temps, &a.table[0][0]);
  a.S_out = S;
  a.A_out = A;
  a.n_out = nf;
  a.corr_rows = corr_rows;
  a.trace = trace_len > 0 ? trace : nullptr;
  a.trace_len = trace_len;
  if (chain_state) {
    const mcmc::ChainStateLayout cl = mcmc::chain_state_layout(L, T);
    char* cs = (char*)chain_state;
    a.state_rows = (uint32_t*)(cs + cl.rows);
    if (resume) {
      a.resume_rows = (const uint32_t*)(cs + cl.rows);
      a.resume_n = (const int32_t*)(cs + cl.n);
      a.resume_S = (const int64_t*)(cs + cl.S);
      a.resume_A = (const int64_t*)(cs + cl.A);
    }
  }
  st = hip_status(mcmc::launch_chain(L, a, s, do_trace && trace_len > 0, resume));
  if (st != MCMC_OK) return st;

  if (chain_state) {  // n, S, A of every chain next to the rows
    const mcmc::ChainStateLayout cl = mcmc::chain_state_layout(L, T);
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

  mcmc::DecideArgs d{};
  d.S = S;
  d.n_final = nf;
  d.corr_rows = corr_rows;
  d.n = n;
  d.K = prm->n_temps;
  d.C = prm->chains;
  d.L = L;
  d.sweeps = prm->sweeps;
  d.beta_bar = beta_bar(prm->p);
  const int nq = 2 * L * L - 2 * L + 1;
  const int nstab = 2 * L * (L - 1);
  d.f0 = 0.75 * (double)nq;
  d.log_z0 = (double)nstab * log(2.0);
  d.class_prob = class_prob;
  d.mean_n = mean_n;
  d.chosen = chosen;
  d.correction = correction;
  return hip_status(mcmc::launch_decide(d, s));
}

int mcmc_init_representatives(int32_t L, uint32_t init, const uint8_t* syndromes, int64_t n,
                              uint8_t* reps, void* stream) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (init != MCMC_INIT_CANONICAL && init != MCMC_INIT_MATCHING) return MCMC_EINVAL;
  if (n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!syndromes || !reps) return MCMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  return hip_status(init == MCMC_INIT_MATCHING
                        ? mcmc::launch_init_matching(L, syndromes, n, nullptr, nullptr, reps, s)
                        : mcmc::launch_init(L, syndromes, n, nullptr, nullptr, reps, s));
}

int mcmc_unpack_chain_state(const mcmc_params* prm, int64_t n, const void* chain_state,
                            uint8_t* states, int32_t* weights, void* stream) {
  const int st = check_params(prm, n);
  if (st != MCMC_OK) return st;
  if (n == 0) return MCMC_OK;
  if (!chain_state) return MCMC_EINVAL;
  const int64_t T = n * 4 * (int64_t)prm->n_temps * prm->chains;
  const mcmc::ChainStateLayout cl = mcmc::chain_state_layout(prm->L, T);
  return hip_status(mcmc::launch_unpack(prm->L, (const uint32_t*)((const char*)chain_state + cl.rows),
                                        T, T, states, weights, (hipStream_t)stream));
}

int mcmc_sample_errors(int32_t L, double p, uint64_t seed, const uint32_t* sample_ids,
                       uint32_t id_base, int64_t n, uint8_t* syndromes, uint8_t* true_class,
                       uint8_t* errors, void* stream) {
  if (!valid_L(L) || !valid_p(p) || n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!syndromes || !true_class) return MCMC_EINVAL;
  if (n > 0x7FFFFFFF) return MCMC_ERANGE;
  const uint32_t thr = (uint32_t)floor(ldexp(p, 32));
  return hip_status(mcmc::launch_sample(L, thr, (uint32_t)(seed & 0xFFFFFFFFull),
                                        (uint32_t)(seed >> 32), sample_ids, id_base, n, syndromes,
                                        true_class, errors, (hipStream_t)stream));
}

}  // extern "C"
