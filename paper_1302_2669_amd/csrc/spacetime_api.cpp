// C-ABI of the imperfect-measurement decoder (declared in include/mcmcdec.h):
// validation, host tables, workspace carving and kernel enqueueing.
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/mcmcdec.h"
#include "device_common.h"
#include "host_common.h"
#include "internal.h"

namespace {

using namespace mcmc;

int check_st(const mcmc_spacetime_params* prm, int64_t n) {
  if (!prm) return MCMC_EINVAL;
  if (prm->reserved != 0) return MCMC_EINVAL;
  // n <= 2^28 keeps every grid of the decode (n n_stab / 256 blocks for the
  // last-round copy) within 32-bit block counts
  if (n < 0 || n > ((int64_t)1 << 28) || !valid_L(prm->L)) return MCMC_ERANGE;
  if (prm->rounds < 1 || prm->rounds > MCMC_ROUNDS_MAX) return MCMC_ERANGE;
  if (!valid_p(prm->p) || !(prm->p_m > 0.0 && prm->p_m < 0.5)) return MCMC_ERANGE;
  if (prm->chains < 1 || prm->chains > MCMC_CHAINS_MAX) return MCMC_ERANGE;
  if (prm->burn < 0 || prm->sweeps < 0) return MCMC_ERANGE;
  if ((int64_t)prm->burn + prm->sweeps > MCMC_SWEEPS_MAX) return MCMC_ERANGE;
  const int64_t T = n * 4 * (int64_t)prm->chains;
  if (n > 0 && (T / n / 4 != prm->chains || T > ((int64_t)1 << 36))) return MCMC_ERANGE;
  return MCMC_OK;
}

struct StLayout {
  size_t ds, reps, rep_w, Sn, Sm, A, nf, mf, fc, state, bytes;
};

StLayout st_layout(const mcmc_spacetime_params* prm, int64_t n) {
  const int L = prm->L, T = prm->rounds;
  const int64_t nq = n_qubits(L), ns = n_stab(L);
  const int64_t chains = n * 4 * (int64_t)prm->chains;
  StLayout w{};
  size_t off = 0;
  w.ds = off;    off = align_up(off + (size_t)(n * ns));
  w.reps = off;  off = align_up(off + (size_t)(n * 4 * nq));
  w.rep_w = off; off = align_up(off + (size_t)(n * 4) * sizeof(int32_t));
  w.Sn = off;    off = align_up(off + (size_t)chains * sizeof(int64_t));
  w.Sm = off;    off = align_up(off + (size_t)chains * sizeof(int64_t));
  w.A = off;     off = align_up(off + (size_t)chains * sizeof(int64_t));
  w.nf = off;    off = align_up(off + (size_t)chains * sizeof(int32_t));
  w.mf = off;    off = align_up(off + (size_t)chains * sizeof(int32_t));
  w.fc = off;    off = align_up(off + (size_t)(n * 4 * nq));
  w.state = off;   // the hypotheses, word-major over all chains
  {
    const int64_t words = (int64_t)T * ((nq + 15) / 16) + (int64_t)(T - 1) * ((ns + 31) / 32);
    off = align_up(off + (size_t)(words * chains) * sizeof(uint32_t));
  }
  w.bytes = off;
  return w;
}

}  // namespace

extern "C" {

int mcmc_spacetime_workspace_size(const mcmc_spacetime_params* prm, int64_t n, size_t* bytes) {
  if (!bytes) return MCMC_EINVAL;
  const int st = check_st(prm, n);
  if (st != MCMC_OK) return st;
  *bytes = st_layout(prm, n).bytes;
  return MCMC_OK;
}

int mcmc_spacetime_tables(const mcmc_spacetime_params* prm, uint32_t* h_spatial,
                          uint32_t* h_time, uint32_t* h_always, double* h_xi) {
  const int st = check_st(prm, 0);
  if (st != MCMC_OK) return st;
  const double bb = beta_bar(prm->p);
  const double xi = log((1.0 - prm->p_m) / prm->p_m) / bb;
  if (h_spatial) fill_row(bb, h_spatial);
  uint32_t always = 0;
  for (int dn = -2; dn <= 2; ++dn)
    for (int dm = -2; dm <= 2; ++dm) {
      const int e = (dn + 2) * 5 + (dm + 2);
      const double en = (double)dn + xi * (double)dm;
      uint32_t thr = 0;
      if (en <= 0.0) always |= 1u << e;
      else thr = (uint32_t)floor(ldexp(exp(-(bb * en)), 32));
      if (h_time) h_time[e] = thr;
    }
  if (h_always) *h_always = always;
  if (h_xi) *h_xi = xi;
  return MCMC_OK;
}

int mcmc_decode_spacetime(const uint8_t* obs, const uint32_t* ids, int64_t n,
                          const mcmc_spacetime_params* prm, double* class_prob, double* mean_n,
                          double* mean_m, int64_t* sum_n, int64_t* sum_m, int64_t* accepts,
                          uint8_t* chosen, uint8_t* correction, void* workspace,
                          size_t workspace_bytes, void* stream) {
  int st = check_st(prm, n);
  if (st != MCMC_OK) return st;
  if (n == 0) return MCMC_OK;
  if (!obs || !class_prob || !chosen) return MCMC_EINVAL;
  const StLayout wl = st_layout(prm, n);
  if (!workspace || workspace_bytes < wl.bytes) return MCMC_EWORKSPACE;
  if (((uintptr_t)workspace % kAlign) != 0) return MCMC_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int L = prm->L, T = prm->rounds;

  uint8_t* last = (uint8_t*)(ws + wl.ds);
  st = hip_status(launch_spacetime_last(n, T, n_stab(L), obs, last, s));
  if (st != MCMC_OK) return st;
  StartArgs sa{};
  sa.syn = last;
  sa.n = n;
  sa.L = L;
  sa.weights = (int32_t*)(ws + wl.rep_w);
  sa.bytes = (uint8_t*)(ws + wl.reps);
  st = hip_status(launch_init_matching(sa, s));
  if (st != MCMC_OK) return st;

  SpaceTimeArgs a{};
  a.L = L;
  a.T = T;
  a.chains = prm->chains;
  a.burn = prm->burn;
  a.sweep_end = prm->burn + prm->sweeps;
  a.n = n;
  a.n_tasks = n * 4 * (int64_t)prm->chains;
  a.ids = ids;
  a.obs = obs;
  a.reps = sa.bytes;
  a.rep_weight = sa.weights;
  a.k0 = (uint32_t)(prm->seed & 0xFFFFFFFFull);
  a.k1 = (uint32_t)(prm->seed >> 32);
  st = mcmc_spacetime_tables(prm, a.sp_thr, a.t_thr, &a.t_always, &a.xi);
  if (st != MCMC_OK) return st;
  a.beta_bar = beta_bar(prm->p);
  a.Sn = sum_n ? sum_n : (int64_t*)(ws + wl.Sn);
  a.Sm = sum_m ? sum_m : (int64_t*)(ws + wl.Sm);
  a.A = accepts ? accepts : (int64_t*)(ws + wl.A);
  a.n_final = (int32_t*)(ws + wl.nf);
  a.m_final = (int32_t*)(ws + wl.mf);
  a.final_c = correction ? (uint8_t*)(ws + wl.fc) : nullptr;
  a.class_prob = class_prob;
  a.mean_n = mean_n;
  a.mean_m = mean_m;
  a.chosen = chosen;
  a.correction = correction;
  a.state = (uint32_t*)(ws + wl.state);
  st = hip_status(launch_spacetime_chains(a, s));
  if (st != MCMC_OK) return st;
  return hip_status(launch_spacetime_decide(a, s));
}

int mcmc_sample_spacetime(int32_t L, int32_t rounds, double p, double p_m, uint64_t seed,
                          uint32_t id_base, int64_t n, uint8_t* obs, uint8_t* true_class,
                          void* stream) {
  if (!valid_L(L) || rounds < 1 || rounds > MCMC_ROUNDS_MAX || !valid_p(p) ||
      !(p_m > 0.0 && p_m < 0.5) || n < 0 || n > 0x7FFFFFFF)
    return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!obs || !true_class) return MCMC_EINVAL;
  const uint32_t thr_d = (uint32_t)floor(ldexp(p, 32));
  const uint32_t thr_m = (uint32_t)floor(ldexp(p_m, 32));
  return hip_status(launch_spacetime_sample(L, rounds, thr_d, thr_m,
                                            (uint32_t)(seed & 0xFFFFFFFFull),
                                            (uint32_t)(seed >> 32), id_base, n, obs, true_class,
                                            (hipStream_t)stream));
}

}  // extern "C"
