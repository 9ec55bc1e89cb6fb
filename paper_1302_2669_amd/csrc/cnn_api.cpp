// C-ABI of the gate network and of the gated decoder.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "device_common.h"
#include "host_common.h"

using namespace mcmc;

namespace {

bool cnn_batch_ok(int64_t batch) { return batch >= 0 && batch <= MCMC_CNN_BATCH_MAX; }

int check_ws(const void* ws, size_t have, size_t need) {
  if (need == 0) return MCMC_OK;
  if (!ws || have < need || ((uintptr_t)ws % kAlign) != 0) return MCMC_EWORKSPACE;
  return MCMC_OK;
}

}  // namespace

extern "C" {

int mcmc_cnn_param_count(int32_t L, int64_t* h_count) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (!h_count) return MCMC_EINVAL;
  *h_count = cnn_offsets(L).total;
  return MCMC_OK;
}

int mcmc_cnn_workspace_size(int32_t L, int64_t batch, size_t* h_bytes) {
  if (!valid_L(L) || !cnn_batch_ok(batch)) return MCMC_ERANGE;
  if (!h_bytes) return MCMC_EINVAL;
  *h_bytes = batch == 0 ? 0 : cnn_workspace(L, batch).bytes;
  return MCMC_OK;
}

int mcmc_cnn_workspace_offsets(int32_t L, int64_t batch, int64_t* h_offsets) {
  if (!valid_L(L) || !cnn_batch_ok(batch)) return MCMC_ERANGE;
  if (!h_offsets) return MCMC_EINVAL;
  const CnnWorkspace w = cnn_workspace(L, batch);
  const size_t o[7] = {w.x0, w.a1, w.a2, w.a3, w.dp3, w.dp2, w.dp1};
  for (int i = 0; i < 7; ++i) h_offsets[i] = (int64_t)o[i];
  return MCMC_OK;
}

int mcmc_cnn_forward(int32_t L, int64_t batch, const float* d_params, const uint8_t* d_syndromes,
                     const float* d_p, float* d_logits, void* d_workspace, size_t workspace_bytes,
                     void* stream) {
  if (!valid_L(L) || !cnn_batch_ok(batch)) return MCMC_ERANGE;
  if (batch == 0) return MCMC_OK;
  if (!d_params || !d_syndromes || !d_p || !d_logits) return MCMC_EINVAL;
  const int st = check_ws(d_workspace, workspace_bytes, cnn_workspace(L, batch).bytes);
  if (st != MCMC_OK) return st;
  return hip_status(cnn_forward(L, batch, d_params, d_syndromes, d_p, d_logits,
                                (char*)d_workspace, (hipStream_t)stream));
}

int mcmc_cnn_infer_workspace_size(int32_t L, size_t* h_bytes) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (!h_bytes) return MCMC_EINVAL;
  *h_bytes = cnn_weights(L).bytes;
  return MCMC_OK;
}

int mcmc_cnn_infer(int32_t L, int64_t batch, const float* d_params, const uint8_t* d_syndromes,
                   const float* d_p, float* d_logits, void* d_workspace, size_t workspace_bytes,
                   void* stream) {
  if (!valid_L(L) || !cnn_batch_ok(batch)) return MCMC_ERANGE;
  if (batch == 0) return MCMC_OK;
  if (!d_params || !d_syndromes || !d_p || !d_logits) return MCMC_EINVAL;
  const int st = check_ws(d_workspace, workspace_bytes, cnn_weights(L).bytes);
  if (st != MCMC_OK) return st;
  if (cnn_infer_group(L) < 1) return MCMC_EDEVICE;
  return hip_status(cnn_infer(L, batch, d_params, d_syndromes, d_p, d_logits, (char*)d_workspace,
                              (hipStream_t)stream));
}

int mcmc_cnn_backward(int32_t L, int64_t batch, const float* d_params, const float* d_logits,
                      const float* d_class_target, const int32_t* d_budget, float budget_weight,
                      float* d_grads, float* d_loss, void* d_workspace, size_t workspace_bytes,
                      void* stream) {
  if (!valid_L(L) || !cnn_batch_ok(batch)) return MCMC_ERANGE;
  if (batch == 0) return MCMC_OK;
  if (!d_params || !d_logits || !d_class_target || !d_budget || !d_grads) return MCMC_EINVAL;
  if (!(budget_weight >= 0.0f) || !isfinite(budget_weight)) return MCMC_ERANGE;
  const int st = check_ws(d_workspace, workspace_bytes, cnn_workspace(L, batch).bytes);
  if (st != MCMC_OK) return st;
  return hip_status(cnn_backward(L, batch, d_params, d_logits, d_class_target, d_budget,
                                 budget_weight, d_grads, d_loss, (char*)d_workspace,
                                 (hipStream_t)stream));
}

int mcmc_cnn_step(int64_t n_params, int64_t step, float lr, float beta1, float beta2, float eps,
                  float* d_params, const float* d_grads, float* d_m, float* d_v, void* stream) {
  if (n_params < 0 || step < 1) return MCMC_ERANGE;
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return MCMC_ERANGE;
  if (n_params == 0) return MCMC_OK;
  if (!d_params || !d_grads || !d_m || !d_v) return MCMC_EINVAL;
  // bias corrections 1 - beta^t in double on the host
  const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
  return hip_status(cnn_adam(n_params, d_params, d_grads, d_m, d_v, lr, beta1, beta2, eps, c1, c2,
                             (hipStream_t)stream));
}

int mcmc_cnn_init(int32_t L, uint64_t seed, float* d_params, void* stream) {
  if (!valid_L(L)) return MCMC_ERANGE;
  if (!d_params) return MCMC_EINVAL;
  return hip_status(cnn_init_params(L, seed, d_params, (hipStream_t)stream));
}

int mcmc_gate_budget_labels(int64_t n, const uint8_t* d_zero, const uint8_t* d_short,
                            const uint8_t* d_full, int32_t* d_budget, void* stream) {
  if (n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!d_zero || !d_short || !d_full || !d_budget) return MCMC_EINVAL;
  return hip_status(gate_budget_labels(n, d_zero, d_short, d_full, d_budget,
                                       (hipStream_t)stream));
}

int mcmc_gate_relative_targets(int64_t n, const uint8_t* d_start_class, const float* d_class_prob,
                               float* d_targets, void* stream) {
  if (n < 0) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!d_start_class || !d_class_prob || !d_targets) return MCMC_EINVAL;
  // the permutation reads a row while writing it: the buffers must not overlap
  const char* a = (const char*)d_class_prob;
  const char* b = (const char*)d_targets;
  const size_t bytes = (size_t)n * 4 * sizeof(float);
  if (a < b + bytes && b < a + bytes) return MCMC_EINVAL;
  return hip_status(gate_relative_targets(n, d_start_class, d_class_prob, d_targets,
                                          (hipStream_t)stream));
}

int mcmc_cnn_permutation(int64_t n, uint64_t seed, uint32_t epoch, int32_t* d_perm,
                         void* stream) {
  if (!cnn_batch_ok(n)) return MCMC_ERANGE;
  if (n == 0) return MCMC_OK;
  if (!d_perm) return MCMC_EINVAL;
  return hip_status(cnn_permutation(n, seed, epoch, d_perm, (hipStream_t)stream));
}

namespace {

// Training workspace: the epoch's permutation, the gathered batch, logits,
// gradients, per-sample losses, then the network's own workspace.
struct TrainWorkspace {
  size_t perm, syn, p, tgt, bud, logits, grads, loss, net, bytes;
};

TrainWorkspace train_workspace(int L, int64_t n, int64_t B) {
  TrainWorkspace w{};
  size_t off = 0;
  const int ns = 2 * L * (L - 1);
  w.perm = off;   off = align_up(off + (size_t)n * sizeof(int32_t));
  w.syn = off;    off = align_up(off + (size_t)B * ns);
  w.p = off;      off = align_up(off + (size_t)B * sizeof(float));
  w.tgt = off;    off = align_up(off + (size_t)B * 4 * sizeof(float));
  w.bud = off;    off = align_up(off + (size_t)B * sizeof(int32_t));
  w.logits = off; off = align_up(off + (size_t)B * 8 * sizeof(float));
  w.grads = off;  off = align_up(off + (size_t)cnn_offsets(L).total * sizeof(float));
  w.loss = off;   off = align_up(off + (size_t)B * sizeof(float));
  w.net = off;    off = align_up(off + cnn_workspace(L, B).bytes);
  w.bytes = off;
  return w;
}

bool train_config_ok(const mcmc_train_config* c) {
  return c && c->batch >= 1 && c->batch <= MCMC_CNN_BATCH_MAX && c->total_steps >= 1 &&
         c->lr >= 0.0f && c->lr_final >= 0.0f && isfinite(c->lr) && isfinite(c->lr_final) &&
         c->beta1 >= 0.0f && c->beta1 < 1.0f && c->beta2 >= 0.0f && c->beta2 < 1.0f &&
         c->eps > 0.0f && c->budget_weight >= 0.0f && isfinite(c->budget_weight);
}

}  // namespace

int mcmc_cnn_train_workspace_size(int32_t L, int64_t n, int64_t batch, size_t* h_bytes) {
  if (!valid_L(L) || !cnn_batch_ok(n) || batch < 1 || batch > MCMC_CNN_BATCH_MAX)
    return MCMC_ERANGE;
  if (!h_bytes) return MCMC_EINVAL;
  *h_bytes = train_workspace(L, n, batch).bytes;
  return MCMC_OK;
}

int mcmc_cnn_train_epoch(int32_t L, int64_t n, const mcmc_train_config* h_cfg, uint32_t epoch,
                         int64_t* h_step, float* d_params, float* d_m, float* d_v,
                         const uint8_t* d_syndromes, const float* d_p,
                         const float* d_class_target, const int32_t* d_budget,
                         double* d_loss_sum, void* d_workspace, size_t workspace_bytes,
                         void* stream) {
  if (!valid_L(L) || !cnn_batch_ok(n)) return MCMC_ERANGE;
  if (!h_cfg || !h_step) return MCMC_EINVAL;
  if (!train_config_ok(h_cfg) || *h_step < 0) return MCMC_ERANGE;
  if (!d_params || !d_m || !d_v || !d_loss_sum) return MCMC_EINVAL;
  if (n > 0 && (!d_syndromes || !d_p || !d_class_target || !d_budget)) return MCMC_EINVAL;
  const int64_t B = h_cfg->batch;
  const TrainWorkspace w = train_workspace(L, n, B);
  int st = check_ws(d_workspace, workspace_bytes, w.bytes);
  if (st != MCMC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)d_workspace;
  int32_t* perm = (int32_t*)(ws + w.perm);
  uint8_t* bsyn = (uint8_t*)(ws + w.syn);
  float* bp = (float*)(ws + w.p);
  float* btgt = (float*)(ws + w.tgt);
  int32_t* bbud = (int32_t*)(ws + w.bud);
  float* logits = (float*)(ws + w.logits);
  float* grads = (float*)(ws + w.grads);
  float* loss = (float*)(ws + w.loss);
  char* net = ws + w.net;
  const int ns = 2 * L * (L - 1);
  const int64_t P = cnn_offsets(L).total;
  st = hip_status(cnn_loss_sum(0, loss, d_loss_sum, true, s));
  if (st != MCMC_OK) return st;
  st = hip_status(cnn_permutation(n, h_cfg->seed, epoch, perm, s));
  if (st != MCMC_OK) return st;
  for (int64_t at = 0; at + B <= n; at += B) {
    const int32_t* idx = perm + at;
    st = hip_status(cnn_gather(B, ns, idx, d_syndromes, bsyn, s));
    if (st == MCMC_OK) st = hip_status(cnn_gather(B, 4, idx, (const uint8_t*)d_p, (uint8_t*)bp, s));
    if (st == MCMC_OK)
      st = hip_status(cnn_gather(B, 16, idx, (const uint8_t*)d_class_target, (uint8_t*)btgt, s));
    if (st == MCMC_OK)
      st = hip_status(cnn_gather(B, 4, idx, (const uint8_t*)d_budget, (uint8_t*)bbud, s));
    if (st == MCMC_OK) st = hip_status(cnn_forward(L, B, d_params, bsyn, bp, logits, net, s));
    if (st == MCMC_OK)
      st = hip_status(cnn_backward(L, B, d_params, logits, btgt, bbud, h_cfg->budget_weight,
                                   grads, loss, net, s));
    if (st != MCMC_OK) return st;
    // learning rate falls linearly from lr to lr_final over total_steps steps
    const int64_t t = *h_step;
    const double frac = (double)t / (double)std::max<int64_t>(1, h_cfg->total_steps - 1);
    const float lr = (float)((double)h_cfg->lr + ((double)h_cfg->lr_final - h_cfg->lr) * frac);
    const float c1 = (float)(1.0 - pow((double)h_cfg->beta1, (double)(t + 1)));
    const float c2 = (float)(1.0 - pow((double)h_cfg->beta2, (double)(t + 1)));
    st = hip_status(cnn_adam(P, d_params, grads, d_m, d_v, lr, h_cfg->beta1, h_cfg->beta2,
                             h_cfg->eps, c1, c2, s));
    if (st == MCMC_OK) st = hip_status(cnn_loss_sum(B, loss, d_loss_sum, false, s));
    if (st != MCMC_OK) return st;
    *h_step = t + 1;
  }
  return MCMC_OK;
}

int mcmc_cnn_gate(int64_t batch, const float* d_logits, float threshold, int32_t class_route,
                  uint8_t* d_route, uint8_t* d_class, float* d_confidence, void* stream) {
  if (!cnn_batch_ok(batch)) return MCMC_ERANGE;
  if (!(threshold >= 0.0f && threshold <= 1.0f)) return MCMC_ERANGE;
  if (batch == 0) return MCMC_OK;
  if (!d_logits || !d_route || !d_class) return MCMC_EINVAL;
  return hip_status(
      cnn_gate(batch, d_logits, threshold, class_route != 0, d_route, d_class, d_confidence,
               nullptr, GapRoute{}, (hipStream_t)stream));
}

}  // extern "C"

// ---- gated decoder ------------------------------------------------------------

struct mcmc_gated {
  mcmc_gate_config cfg{};
  mcmc_plan* plan = nullptr;
  size_t plan_ws = 0;
  int nq = 0, ns = 0;
  // pinned host staging
  uint8_t* h_route = nullptr;
  uint8_t* h_flag = nullptr;
  int32_t* h_idx = nullptr;   // escalated batch indices
  float* h_pf = nullptr;
  std::vector<mcmc_item> items;
  // device-built budget plan (the path without escalation): groups [3],
  // items [N], tables [N][K][4], beta_bar [N], ids [N], counters [8],
  // cumulative tiles [4]; pinned staging of ids, tables, beta and counts
  void* dblock = nullptr;
  GroupDesc* d_groups = nullptr;
  ItemDesc* d_items = nullptr;
  uint32_t* d_tables = nullptr;
  double* d_beta = nullptr;
  uint32_t* d_ids = nullptr;
  uint32_t* d_counts = nullptr;
  uint32_t* d_tile_cum = nullptr;
  uint8_t* d_gap = nullptr;          // gap route thresholds [MCMC_GAP_BINS]
  bool gap_on = false;
  uint32_t* h_ids = nullptr;
  uint32_t* h_tab = nullptr;
  double* h_beta = nullptr;
  uint32_t* h_cnt = nullptr;
  hipEvent_t staged = nullptr;       // the last call's host-to-device copies
  bool staged_pending = false;
};

namespace {

struct GatedWorkspace {
  size_t cnn, logits, pf, route, cls, flip, conf, flag, idx, prob, chosen, plan;
  // device-built path: queue, class starts, per-chain sums, final rows
  size_t q, irows, in_n, S, A, nf, frows, bytes;
};

GatedWorkspace gated_workspace(const mcmc_gated* g) {
  const int64_t n = g->cfg.max_batch;
  GatedWorkspace w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  w.cnn = take(cnn_weights(g->cfg.L).bytes);
  w.logits = take((size_t)n * 8 * sizeof(float));
  w.pf = take((size_t)n * sizeof(float));
  w.route = take((size_t)n);
  w.cls = take((size_t)n);
  w.flip = take((size_t)n);
  w.conf = take((size_t)n * 3 * sizeof(float));
  w.flag = take((size_t)n);
  w.idx = take((size_t)n * sizeof(int32_t));
  w.prob = take((size_t)n * 4 * sizeof(double));
  w.chosen = take((size_t)n);
  w.plan = take(g->plan_ws);
  const int64_t chains = n * 4 * (int64_t)g->cfg.n_temps * g->cfg.chains;
  const int64_t rows = n * (int64_t)words_per_config(g->cfg.L) * 4;
  w.q = take(kQueueSlots * sizeof(uint32_t));
  w.irows = take((size_t)rows * sizeof(uint32_t));
  w.in_n = take((size_t)n * 4 * sizeof(int32_t));
  w.S = take((size_t)chains * sizeof(int64_t));
  w.A = take((size_t)chains * sizeof(int64_t));
  w.nf = take((size_t)chains * sizeof(int32_t));
  w.frows = take((size_t)rows * sizeof(uint32_t));
  w.bytes = off;
  return w;
}

void free_gated(mcmc_gated* g) {
  if (!g) return;
  if (g->plan) mcmc_plan_destroy(g->plan);
  if (g->h_route) (void)hipHostFree(g->h_route);
  if (g->h_flag) (void)hipHostFree(g->h_flag);
  if (g->h_idx) (void)hipHostFree(g->h_idx);
  if (g->h_pf) (void)hipHostFree(g->h_pf);
  if (g->h_ids) (void)hipHostFree(g->h_ids);
  if (g->h_tab) (void)hipHostFree(g->h_tab);
  if (g->h_beta) (void)hipHostFree(g->h_beta);
  if (g->h_cnt) (void)hipHostFree(g->h_cnt);
  if (g->staged) {
    (void)hipEventSynchronize(g->staged);
    (void)hipEventDestroy(g->staged);
  }
  if (g->dblock) (void)hipFree(g->dblock);
  delete g;
}

mcmc_item make_item(const mcmc_gate_config& c, int32_t sweeps, uint32_t id, double p, int64_t i,
                    int ns, int nq) {
  mcmc_item it{};
  it.L = c.L;
  it.sweeps = sweeps;
  it.burn = c.burn;
  it.chains = c.chains;
  it.n_temps = c.n_temps;
  it.syndrome_id = id;
  it.p = p;
  it.syn_offset = i * ns;
  it.corr_offset = i * nq;
  return it;
}

}  // namespace

extern "C" {

int mcmc_gated_create(const mcmc_gate_config* h_cfg, mcmc_gated** out) {
  if (!out || !h_cfg) return MCMC_EINVAL;
  *out = nullptr;
  const mcmc_gate_config& c = *h_cfg;
  if (!valid_L(c.L) || !valid_p(c.p)) return MCMC_ERANGE;
  if (c.max_batch < 1 || c.max_batch > MCMC_CNN_BATCH_MAX) return MCMC_ERANGE;
  if (!(c.threshold >= 0.0f && c.threshold <= 1.0f)) return MCMC_ERANGE;
  if (!(c.escalate >= 0.0f && c.escalate <= 1e6f)) return MCMC_ERANGE;
  if (c.escalate > 0.0f && c.chains < 2) return MCMC_ERANGE;  // the margin needs replicas
  if (c.class_route != 0 && c.class_route != 1) return MCMC_EINVAL;
  if (c.class_route && c.escalate > 0.0f) return MCMC_EINVAL;
  if (c.sweeps_short < 0 || c.sweeps_full < 0) return MCMC_ERANGE;
  if (c.init != MCMC_INIT_CANONICAL && c.init != MCMC_INIT_MATCHING && c.init != MCMC_INIT_MWPM)
    return MCMC_EINVAL;
  if (cnn_infer_group(c.L) < 1) return MCMC_EDEVICE;
  mcmc_gated* g = new (std::nothrow) mcmc_gated();
  if (!g) return MCMC_ENOMEM;
  g->cfg = c;
  mcmc_geometry(c.L, &g->nq, &g->ns);
  // reserve the plan's device block for a whole batch (every budget has the
  // same number of chains and tiles per syndrome)
  try {
    g->items.resize((size_t)c.max_batch);
  } catch (...) {
    free_gated(g);
    return MCMC_ENOMEM;
  }
  for (int64_t i = 0; i < c.max_batch; ++i)
    g->items[i] = make_item(c, c.sweeps_full, (uint32_t)i, c.p, i, g->ns, g->nq);
  int st = mcmc_plan_create(g->items.data(), c.max_batch, c.seed, c.init, &g->plan);
  if (st != MCMC_OK) {
    free_gated(g);
    return st;
  }
  st = mcmc_plan_info(g->plan, nullptr, &g->plan_ws, nullptr);
  const size_t n = (size_t)c.max_batch;
  bool ok = st == MCMC_OK;
  ok = ok && hipHostMalloc((void**)&g->h_route, n, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&g->h_flag, n, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&g->h_idx, n * 4, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&g->h_pf, n * 4, hipHostMallocDefault) == hipSuccess;
  // device-built budget plan storage
  const size_t K4 = 4 * (size_t)c.n_temps;
  const size_t sz_g = align_up(3 * sizeof(GroupDesc)), sz_i = align_up(n * sizeof(ItemDesc));
  // tables: one per syndrome, then the configured rate's at slot N
  const size_t sz_t = align_up((n + 1) * K4 * 4), sz_b = align_up(n * 8), sz_id = align_up(n * 4);
  const size_t sz_c = align_up(8 * 4), sz_tc = align_up(4 * 4), sz_gap = align_up(MCMC_GAP_BINS);
  ok = ok && hipMalloc(&g->dblock, sz_g + sz_i + sz_t + sz_b + sz_id + sz_c + sz_tc + sz_gap) ==
                 hipSuccess;
  if (ok) {
    char* b = (char*)g->dblock;
    g->d_groups = (GroupDesc*)b;
    g->d_items = (ItemDesc*)(b + sz_g);
    g->d_tables = (uint32_t*)(b + sz_g + sz_i);
    g->d_beta = (double*)(b + sz_g + sz_i + sz_t);
    g->d_ids = (uint32_t*)(b + sz_g + sz_i + sz_t + sz_b);
    g->d_counts = (uint32_t*)(b + sz_g + sz_i + sz_t + sz_b + sz_id);
    g->d_tile_cum = (uint32_t*)(b + sz_g + sz_i + sz_t + sz_b + sz_id + sz_c);
    g->d_gap = (uint8_t*)(b + sz_g + sz_i + sz_t + sz_b + sz_id + sz_c + sz_tc);
  }
  ok = ok && hipHostMalloc((void**)&g->h_ids, n * 4, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&g->h_tab, n * K4 * 4, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&g->h_beta, n * 8, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&g->h_cnt, 8 * 4, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&g->staged, hipEventDisableTiming) == hipSuccess;
  if (ok) {
    // the configured rate's table after the per-syndrome slots, for batches
    // without their own rates
    fill_table(c.p, c.n_temps, g->h_tab);
    ok = hipMemcpy(g->d_tables + n * K4, g->h_tab, K4 * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    free_gated(g);
    return st != MCMC_OK ? st : MCMC_EDEVICE;
  }
  if (c.init == MCMC_INIT_MWPM) (void)mwpm_prepare_overlap();
  *out = g;
  return MCMC_OK;
}

int mcmc_gated_destroy(mcmc_gated* g) {
  free_gated(g);
  return MCMC_OK;
}

int mcmc_gated_workspace_size(const mcmc_gated* g, size_t* h_bytes) {
  if (!g || !h_bytes) return MCMC_EINVAL;
  *h_bytes = gated_workspace(g).bytes;
  return MCMC_OK;
}

int mcmc_gated_plan(mcmc_gated* g, mcmc_plan** h_plan) {
  if (!g || !h_plan) return MCMC_EINVAL;
  *h_plan = g->plan;
  return MCMC_OK;
}

int mcmc_gated_set_gap_table(mcmc_gated* g, const uint8_t* h_table) {
  if (!g) return MCMC_EINVAL;
  if (!h_table) {
    g->gap_on = false;
    return MCMC_OK;
  }
  if (hipMemcpy(g->d_gap, h_table, MCMC_GAP_BINS, hipMemcpyHostToDevice) != hipSuccess)
    return MCMC_EDEVICE;
  g->gap_on = true;
  return MCMC_OK;
}

int mcmc_gate_fit_gap_table(int64_t n, const double* h_p, const int32_t* d_weights,
                            const int32_t* d_budget, double max_miss, int32_t min_count,
                            uint8_t* h_table, void* stream) {
  if (!h_table || (n > 0 && (!h_p || !d_weights || !d_budget))) return MCMC_EINVAL;
  if (n < 0 || !(max_miss >= 0.0 && max_miss <= 1.0) || min_count < 1) return MCMC_ERANGE;
  for (int64_t i = 0; i < n; ++i)
    if (!valid_p(h_p[i])) return MCMC_ERANGE;
  std::vector<int32_t> w, bud;
  try {
    w.resize((size_t)n * 4);
    bud.resize((size_t)n);
  } catch (...) {
    return MCMC_ENOMEM;
  }
  const hipStream_t s = (hipStream_t)stream;
  if (n > 0 &&
      (hipMemcpyAsync(w.data(), d_weights, (size_t)n * 16, hipMemcpyDeviceToHost, s) !=
           hipSuccess ||
       hipMemcpyAsync(bud.data(), d_budget, (size_t)n * 4, hipMemcpyDeviceToHost, s) !=
           hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    return MCMC_EDEVICE;
  // per bin and gap value: samples and misses (budget label != 0); gaps at
  // or above MCMC_GAP_NEVER are counted in the last slot
  constexpr int NG = (int)MCMC_GAP_NEVER + 1;
  std::vector<int64_t> cnt((size_t)MCMC_GAP_BINS * NG, 0), miss((size_t)MCMC_GAP_BINS * NG, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t gap = start_weight_gap(&w[(size_t)i * 4]);
    const int k = gap_bin((float)h_p[i]);
    const size_t at = (size_t)k * NG + (size_t)std::min<int32_t>(gap, NG - 1);
    ++cnt[at];
    miss[at] += bud[(size_t)i] != 0;
  }
  for (int k = 0; k < MCMC_GAP_BINS; ++k) {
    // counts of gap >= G from the top down, then the smallest qualifying G
    int64_t c_ge[NG + 1], m_ge[NG + 1];
    c_ge[NG] = m_ge[NG] = 0;
    for (int G = NG - 1; G >= 0; --G) {
      c_ge[G] = c_ge[G + 1] + cnt[(size_t)k * NG + G];
      m_ge[G] = m_ge[G + 1] + miss[(size_t)k * NG + G];
    }
    h_table[k] = (uint8_t)MCMC_GAP_NEVER;
    for (int G = 0; G < (int)MCMC_GAP_NEVER && c_ge[G] >= min_count; ++G) {
      if ((double)m_ge[G] <= max_miss * (double)c_ge[G]) {
        h_table[k] = (uint8_t)G;
        break;
      }
    }
  }
  return MCMC_OK;
}

}  // extern "C"

namespace {

// The gated decode without escalation, with no host synchronisation: the
// gate's routes are turned into a three-group plan on the device
// (launch_budget_plan) and the persistent kernel reads its tile ranges there.
int gated_decode_device(mcmc_gated* g, const float* d_params, const uint8_t* d_syndromes,
                        const uint32_t* h_ids, const double* h_p, int64_t n, uint8_t* d_chosen,
                        uint8_t* route, float* logits, uint8_t* d_correction, int64_t* h_counts,
                        char* ws, const GatedWorkspace& wl, hipStream_t s) {
  const mcmc_gate_config& c = g->cfg;
  // the previous call's copies out of the staging buffers must be done
  if (g->staged_pending && hipEventSynchronize(g->staged) != hipSuccess) return MCMC_EDEVICE;
  for (int64_t i = 0; i < n; ++i) {
    g->h_pf[i] = (float)(h_p ? h_p[i] : c.p);
    g->h_ids[i] = h_ids ? h_ids[i] : (uint32_t)i;
  }
  float* pf = (float*)(ws + wl.pf);
  bool ok = hipMemcpyAsync(pf, g->h_pf, (size_t)n * 4, hipMemcpyHostToDevice, s) == hipSuccess;
  ok = ok && hipMemcpyAsync(g->d_ids, g->h_ids, (size_t)n * 4, hipMemcpyHostToDevice, s) ==
                 hipSuccess;
  if (h_p) {
    fill_tables_parallel(h_p, n, c.n_temps, g->h_tab, g->h_beta);
    ok = ok && hipMemcpyAsync(g->d_tables, g->h_tab, (size_t)n * 4 * c.n_temps * 4,
                              hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(g->d_beta, g->h_beta, (size_t)n * 8, hipMemcpyHostToDevice, s) ==
                   hipSuccess;
  }
  ok = ok && hipEventRecord(g->staged, s) == hipSuccess;
  if (!ok) return MCMC_EDEVICE;
  g->staged_pending = true;

  // the class starts, in syndrome order (the plan's items keep each
  // syndrome's start rows and weights at its own offsets), before the gate,
  // which may read their weights
  uint32_t* queue = (uint32_t*)(ws + wl.q);
  uint32_t* irows = (uint32_t*)(ws + wl.irows);
  int32_t* in_n = (int32_t*)(ws + wl.in_n);
  StartArgs sa{};
  sa.syn = d_syndromes;
  sa.n = n;
  sa.L = c.L;
  sa.rows = irows;
  sa.weights = in_n;
  sa.max_L = c.L;
  int st = hip_status(launch_init_mode(c.init, sa, s));
  if (st != MCMC_OK) return st;

  st = hip_status(cnn_infer(c.L, n, d_params, d_syndromes, pf, logits, ws + wl.cnn, s));
  if (st != MCMC_OK) return st;
  uint8_t* flip = c.class_route ? (uint8_t*)(ws + wl.flip) : nullptr;
  GapRoute gap{};
  if (g->gap_on) gap = GapRoute{in_n, pf, g->d_gap};
  st = hip_status(cnn_gate(n, logits, c.threshold, c.class_route != 0, route,
                           (uint8_t*)(ws + wl.cls), (float*)(ws + wl.conf), flip, gap, s));
  if (st != MCMC_OK) return st;

  BudgetArgs ba{};
  ba.n = n;
  ba.route = route;
  ba.ids = g->d_ids;
  ba.beta = h_p ? g->d_beta : nullptr;
  ba.beta0 = beta_bar(c.p);
  ba.table0_off = c.max_batch * 4 * (int64_t)c.n_temps;
  ba.L = c.L;
  ba.K = c.n_temps;
  ba.C = c.chains;
  ba.burn = c.burn;
  ba.sweeps[0] = c.sweeps_full;
  ba.sweeps[1] = c.sweeps_short;
  ba.sweeps[2] = 0;
  ba.counts = g->d_counts;
  ba.groups = g->d_groups;
  ba.items = g->d_items;
  ba.tile_cum = g->d_tile_cum;
  st = hip_status(launch_budget_plan(ba, s));
  if (st != MCMC_OK) return st;

  int64_t* S = (int64_t*)(ws + wl.S);
  int32_t* nf = (int32_t*)(ws + wl.nf);
  uint32_t* frows = d_correction ? (uint32_t*)(ws + wl.frows) : nullptr;
  st = hip_status(launch_zero(queue, kQueueSlots, s));
  if (st != MCMC_OK) return st;

  const int r = range_of(c.L);
  const int64_t per_item = 4 * (int64_t)c.n_temps * c.chains;
  const int64_t max_tiles = (n * per_item + TILE - 1) / TILE + 3;
  RunArgs a{};
  a.groups = g->d_groups;
  a.items = g->d_items;
  a.tables = g->d_tables;
  a.tile_cum = g->d_tile_cum;
  a.n_tiles = max_tiles;
  a.queue = queue + r;
  a.lmin = RANGE_LO[r];
  a.lmax = RANGE_HI[r];
  a.k0 = (uint32_t)(c.seed & 0xFFFFFFFFull);
  a.k1 = (uint32_t)(c.seed >> 32);
  a.init_rows = irows;
  a.init_n = in_n;
  a.S_out = S;
  a.A_out = (int64_t*)(ws + wl.A);
  a.n_out = nf;
  a.final_rows = frows;
  a.total_chains = n * per_item;
  const int64_t waves = std::min<int64_t>(max_tiles, (int64_t)device_cus() * 4 * RANGE_WAVES[r]);
  st = hip_status(launch_chains(r, a, (int)waves, 256, s));
  if (st != MCMC_OK) return st;

  DecideArgs d{};
  d.items = g->d_items;
  d.groups = g->d_groups;
  d.ln2 = log(2.0);
  d.n = n;
  d.S = S;
  d.n_final = nf;
  d.final_rows = frows;
  d.class_prob = (double*)(ws + wl.prob);
  d.mean_n = nullptr;
  d.chosen = d_chosen;
  d.correction = d_correction;
  d.flip = flip;
  st = hip_status(launch_decide(d, s));
  if (st != MCMC_OK) return st;
  if (h_counts) {
    if (hipMemcpyAsync(g->h_cnt, g->d_counts, 3 * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return MCMC_EDEVICE;
    h_counts[0] = g->h_cnt[2];    // no sweep
    h_counts[1] = g->h_cnt[1];    // short budget
    h_counts[2] = g->h_cnt[0];    // full budget
    h_counts[3] = 0;
  }
  return MCMC_OK;
}

}  // namespace

extern "C" {

int mcmc_gated_decode(mcmc_gated* g, const float* d_params, const uint8_t* d_syndromes,
                      const uint32_t* h_ids, const double* h_p, int64_t n, uint8_t* d_chosen,
                      uint8_t* d_route, float* d_logits, uint8_t* d_correction,
                      int64_t* h_counts, void* d_workspace, size_t workspace_bytes,
                      void* stream) {
  if (!g) return MCMC_EINVAL;
  const mcmc_gate_config& c = g->cfg;
  if (n < 0 || n > c.max_batch) return MCMC_ERANGE;
  if (h_counts) h_counts[0] = h_counts[1] = h_counts[2] = h_counts[3] = 0;
  if (n == 0) return MCMC_OK;
  if (!d_params || !d_syndromes || !d_chosen) return MCMC_EINVAL;
  if (h_p)
    for (int64_t i = 0; i < n; ++i)
      if (!valid_p(h_p[i])) return MCMC_ERANGE;
  const GatedWorkspace wl = gated_workspace(g);
  int st = check_ws(d_workspace, workspace_bytes, wl.bytes);
  if (st != MCMC_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)d_workspace;
  float* logits = d_logits ? d_logits : (float*)(ws + wl.logits);
  uint8_t* route = d_route ? d_route : (uint8_t*)(ws + wl.route);
  if (c.escalate <= 0.0f)
    return gated_decode_device(g, d_params, d_syndromes, h_ids, h_p, n, d_chosen, route, logits,
                               d_correction, h_counts, ws, wl, s);
  // escalation: the routes come back to the host to build each plan
  if (g->staged_pending) {
    if (hipEventSynchronize(g->staged) != hipSuccess) return MCMC_EDEVICE;
    g->staged_pending = false;
  }
  float* pf = (float*)(ws + wl.pf);
  double* prob = (double*)(ws + wl.prob);

  // network pass and gate
  for (int64_t i = 0; i < n; ++i) g->h_pf[i] = (float)(h_p ? h_p[i] : c.p);
  if (hipMemcpyAsync(pf, g->h_pf, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return MCMC_EDEVICE;
  st = hip_status(cnn_infer(c.L, n, d_params, d_syndromes, pf, logits, ws + wl.cnn, s));
  if (st != MCMC_OK) return st;
  GapRoute gap{};
  if (g->gap_on) {  // the start weights alone (the plan makes its own starts)
    int32_t* in_n = (int32_t*)(ws + wl.in_n);
    StartArgs sa{};
    sa.syn = d_syndromes;
    sa.n = n;
    sa.L = c.L;
    sa.weights = in_n;
    sa.max_L = c.L;
    st = hip_status(launch_init_mode(c.init, sa, s));
    if (st != MCMC_OK) return st;
    gap = GapRoute{in_n, pf, g->d_gap};
  }
  st = hip_status(cnn_gate(n, logits, c.threshold, false, route, (uint8_t*)(ws + wl.cls),
                           (float*)(ws + wl.conf), nullptr, gap, s));
  if (st != MCMC_OK) return st;
  if (hipMemcpyAsync(g->h_route, route, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess)
    return MCMC_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return MCMC_EDEVICE;

  // one plan, item i = syndrome i with the sweep budget of its route
  const int32_t budget[3] = {0, c.sweeps_short, c.sweeps_full};
  int64_t cnt[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    const uint8_t r = g->h_route[i] > 2 ? 2 : g->h_route[i];
    ++cnt[r];
    const uint32_t id = h_ids ? h_ids[i] : (uint32_t)i;
    g->items[i] = make_item(c, budget[r], id, h_p ? h_p[i] : c.p, i, g->ns, g->nq);
  }
  st = mcmc_plan_rebuild(g->plan, g->items.data(), n);
  if (st != MCMC_OK) return st;
  size_t need = 0;
  mcmc_plan_info(g->plan, nullptr, &need, nullptr);
  if (need > g->plan_ws) return MCMC_EWORKSPACE;
  // per-chain sums of every item (item i's [4][K][C] block at i 4KC)
  int64_t* sums = (int64_t*)(ws + wl.S);
  st = mcmc_plan_execute(g->plan, d_syndromes, prob, nullptr, sums, nullptr, d_chosen,
                         d_correction, ws + wl.plan, g->plan_ws, stream);
  if (st != MCMC_OK) return st;

  // short-budget syndromes whose decision margin across the replicas is
  // small: full budget (the chains are keyed by sweep, so this continues the
  // same chains)
  int64_t m = 0;
  if (c.escalate > 0.0f && cnt[1] > 0) {
    uint8_t* flag = (uint8_t*)(ws + wl.flag);
    st = hip_status(cnn_escalate_flags(n, route, sums, c.n_temps, c.chains, (double)c.escalate,
                                       flag, s));
    if (st != MCMC_OK) return st;
    if (hipMemcpyAsync(g->h_flag, flag, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess)
      return MCMC_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return MCMC_EDEVICE;
    for (int64_t i = 0; i < n; ++i) {
      if (!g->h_flag[i]) continue;
      const uint32_t id = h_ids ? h_ids[i] : (uint32_t)i;
      g->items[m] = make_item(c, c.sweeps_full, id, h_p ? h_p[i] : c.p, i, g->ns, g->nq);
      g->h_idx[m++] = (int32_t)i;
      g->h_route[i] = 3;
    }
    if (m > 0) {
      int32_t* idx = (int32_t*)(ws + wl.idx);
      uint8_t* chosen_sub = (uint8_t*)(ws + wl.chosen);
      if (hipMemcpyAsync(idx, g->h_idx, (size_t)m * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return MCMC_EDEVICE;
      st = mcmc_plan_rebuild(g->plan, g->items.data(), m);
      if (st != MCMC_OK) return st;
      st = mcmc_plan_execute(g->plan, d_syndromes, prob, nullptr, nullptr, nullptr, chosen_sub,
                             d_correction, ws + wl.plan, g->plan_ws, stream);
      if (st != MCMC_OK) return st;
      st = hip_status(cnn_scatter(m, idx, chosen_sub, d_chosen, s));
      if (st != MCMC_OK) return st;
      if (hipMemcpyAsync(route, g->h_route, (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess)
        return MCMC_EDEVICE;
    }
  }
  if (h_counts) {
    h_counts[0] = cnt[0];
    h_counts[1] = cnt[1] - m;
    h_counts[2] = cnt[2];
    h_counts[3] = m;
  }
  // the staging buffers are reused by the next call
  if (hipStreamSynchronize(s) != hipSuccess) return MCMC_EDEVICE;
  return MCMC_OK;
}

}  // extern "C"
