// Mixed batches: syndromes of different L, p, sweep budget and chain count
// decoded together (the batched-launch pattern).  A plan is built once on the
// host: items are grouped by (L, K, chains, burn, sweeps, noise model); groups
// get 64-chain tiles; the tiles of each kernel range and noise model are
// ordered longest first (LPT) so that the persistent kernels' atomic queues
// hand out long tiles before short ones; per-syndrome acceptance tables are
// computed in FP64 on the host exactly as for a uniform batch.  Execution
// enqueues queue reset -> class starts -> persistent chain kernels (one per
// kernel range and noise model, on up to four streams joined again) ->
// estimator; the same sequence can be captured once into a HIP graph and
// replayed.  Outputs depend only on each syndrome's bytes, id and parameters,
// never on the plan's grouping, order or launch shape.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mcmcdec.h"
#include "device_common.h"
#include "host_common.h"
#include "internal.h"

namespace mcmc {

void fill_tables_parallel(const double* p, int64_t n, int32_t K, uint32_t* tables, double* beta) {
  auto fill = [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      uint32_t* dst = tables + i * 4 * (int64_t)K;
      if (i > lo && p[i] == p[i - 1]) {
        std::copy(dst - 4 * K, dst, dst);
        beta[i] = beta[i - 1];
      } else {
        fill_table(p[i], K, dst);
        beta[i] = beta_bar(p[i]);
      }
    }
  };
  const int64_t kChunk = 4096;
  const int workers = (int)std::min<int64_t>(
      std::max(1u, std::min(16u, std::thread::hardware_concurrency())), (n + kChunk - 1) / kChunk);
  if (workers <= 1) {
    fill(0, n);
    return;
  }
  std::vector<std::thread> pool;
  const int64_t per = (n + workers - 1) / workers;
  for (int w = 0; w < workers; ++w) {
    const int64_t lo = w * per, hi = std::min(n, lo + per);
    if (lo < hi) pool.emplace_back(fill, lo, hi);
  }
  for (auto& t : pool) t.join();
}

}  // namespace mcmc

using namespace mcmc;

struct GraphEntry {
  std::vector<const void*> key;
  hipGraphExec_t exec = nullptr;
};

struct mcmc_plan {
  int64_t n = 0;
  uint64_t seed = 0;
  uint32_t init = MCMC_INIT_MATCHING;
  int device = 0;
  std::vector<GroupDesc> groups;
  std::vector<ItemDesc> items;       // plan order
  std::vector<TileDesc> tiles;       // by kernel range, each longest first
  std::vector<uint32_t> tables;
  // tiles by launch slot: kernel range r under noise model m is slot m * N_RANGES + r
  static constexpr int kSlots = 2 * N_RANGES;
  int64_t range_first[kSlots] = {0}, range_tiles[kSlots] = {0};
  // codes of at most PAIR_L_MAX: their one-chain tiles close slot (m, 0)
  // (small_tiles[m] of them), and the same tasks as 128-task pair tiles for
  // the two-chains-per-lane kernel (pair_first[m], pair_tiles[m])
  int64_t small_tiles[2] = {0}, pair_first[2] = {0}, pair_tiles[2] = {0};
  std::vector<int> group_noise;      // noise model of each group
  int64_t total_chains = 0, total_rows = 0, total_updates = 0;
  size_t corr_bytes = 0;
  // device copies
  void* dev = nullptr;
  size_t dev_bytes = 0;
  GroupDesc* d_groups = nullptr;
  ItemDesc* d_items = nullptr;
  TileDesc* d_tiles = nullptr;
  uint32_t* d_tables = nullptr;
  // launch shape
  mcmc_tuning tuning{};
  // side streams: the two-word-row kernels together (concurrent 1) or one
  // per two-word-row range (concurrent 2), forked from and joined to the
  // caller's stream
  static constexpr int kSides = N_RANGES - 2;
  hipStream_t side[kSides] = {nullptr};
  hipEvent_t join[kSides] = {nullptr};
  hipStream_t capture = nullptr;     // stream used to record graphs
  hipEvent_t fork = nullptr;
  std::vector<GraphEntry> graphs;
};
static_assert(RANGE_LO[1] <= 16 && RANGE_LO[N_RANGES - mcmc_plan::kSides] > 16,
              "one side stream per two-word-row range, which are the last kSides");

namespace {

struct PlanWorkspace {
  size_t queue, init_rows, init_n, S, A, n_final, final_rows, bytes;
};

PlanWorkspace plan_workspace(const mcmc_plan* p) {
  PlanWorkspace w{};
  size_t off = 0;
  w.queue = off;      off = align_up(off + kQueueSlots * sizeof(uint32_t));
  w.init_rows = off;  off = align_up(off + (size_t)p->total_rows * sizeof(uint32_t));
  w.init_n = off;     off = align_up(off + (size_t)p->n * 4 * sizeof(int32_t));
  w.S = off;          off = align_up(off + (size_t)p->total_chains * sizeof(int64_t));
  w.A = off;          off = align_up(off + (size_t)p->total_chains * sizeof(int64_t));
  w.n_final = off;    off = align_up(off + (size_t)p->total_chains * sizeof(int32_t));
  w.final_rows = off; off = align_up(off + (size_t)p->total_rows * sizeof(uint32_t));
  w.bytes = off;
  return w;
}

int check_item(const mcmc_item& it) {
  if (!valid_noise(it.noise) || it.reserved != 0) return MCMC_EINVAL;
  if (!valid_L(it.L) || !valid_rate(it.noise, it.p)) return MCMC_ERANGE;
  if (it.n_temps < 1 || it.n_temps > MCMC_TEMPS_MAX) return MCMC_ERANGE;
  if (it.n_temps != 1 && (it.n_temps % 2) != 0) return MCMC_EINVAL;
  if (it.n_temps == 1) {
    if (!(it.beta_scale >= 0.0 && it.beta_scale <= 4.0)) return MCMC_ERANGE;  // NaN too
  } else if (it.beta_scale != 0.0 && it.beta_scale != 1.0) {
    return MCMC_ERANGE;
  }
  if (it.chains < 1 || it.chains > MCMC_CHAINS_MAX) return MCMC_ERANGE;
  if (it.burn < 0 || it.sweeps < 0 || (int64_t)it.burn + it.sweeps > MCMC_SWEEPS_MAX)
    return MCMC_ERANGE;
  if (it.syn_offset < 0 || it.corr_offset < 0) return MCMC_ERANGE;
  return MCMC_OK;
}

void release_graphs(mcmc_plan* p) {
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
}

int enqueue(mcmc_plan* p, const uint8_t* syn, double* prob, double* mean_n, int64_t* sum_n,
            int64_t* accepts, uint8_t* chosen, uint8_t* correction, void* workspace,
            hipStream_t s) {
  const PlanWorkspace wl = plan_workspace(p);
  char* ws = (char*)workspace;
  uint32_t* queue = (uint32_t*)(ws + wl.queue);
  uint32_t* init_rows = (uint32_t*)(ws + wl.init_rows);
  int32_t* init_n = (int32_t*)(ws + wl.init_n);
  int64_t* S = sum_n ? sum_n : (int64_t*)(ws + wl.S);
  int64_t* A = accepts ? accepts : (int64_t*)(ws + wl.A);
  int32_t* nf = (int32_t*)(ws + wl.n_final);
  uint32_t* final_rows = correction ? (uint32_t*)(ws + wl.final_rows) : nullptr;

  int st = hip_status(launch_zero(queue, kQueueSlots, s));
  if (st != MCMC_OK) return st;
  StartArgs sa{};
  sa.syn = syn;
  sa.items = p->d_items;
  sa.groups = p->d_groups;
  sa.n = p->n;
  sa.rows = init_rows;
  sa.weights = init_n;
  for (const GroupDesc& g : p->groups) sa.max_L = std::max(sa.max_L, g.L);
  st = hip_status(launch_init_mode(p->init, sa, s));
  if (st != MCMC_OK) return st;

  RunArgs a{};
  a.groups = p->d_groups;
  a.items = p->d_items;
  a.tables = p->d_tables;
  a.k0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
  a.k1 = (uint32_t)(p->seed >> 32);
  a.init_rows = init_rows;
  a.init_n = init_n;
  a.S_out = S;
  a.A_out = A;
  a.n_out = nf;
  a.final_rows = final_rows;
  a.total_chains = p->total_chains;

  const mcmc_tuning& tu = p->tuning;
  const int cus = device_cus();
  auto run_range = [&](int slot, hipStream_t on) -> int {
    const int r = slot % N_RANGES, m = slot / N_RANGES;
    // the small codes of range 0 under the two-chains-per-lane mapping
    const bool pair = r == 0 && tu.pair_small != 0 && p->small_tiles[m] > 0;
    if (pair) {
      RunArgs ra = a;
      ra.noise = m;
      ra.tiles = p->d_tiles + p->pair_first[m];
      ra.n_tiles = p->pair_tiles[m];
      ra.queue = queue + mcmc_plan::kSlots + m;
      ra.lmin = 2;
      ra.lmax = PAIR_L_MAX;
      const int per_simd = std::max(1, PAIR_WAVES + tu.occ_narrow);
      const int64_t waves = std::min<int64_t>(ra.n_tiles, (int64_t)cus * 4 * per_simd);
      const int st2 = hip_status(launch_chains_pair(ra, (int)waves, tu.wg_narrow, on));
      if (st2 != MCMC_OK) return st2;
    }
    const int64_t n_tiles = p->range_tiles[slot] - (pair ? p->small_tiles[m] : 0);
    if (n_tiles == 0) return MCMC_OK;
    RunArgs ra = a;
    ra.noise = m;
    ra.tiles = p->d_tiles + p->range_first[slot];
    ra.n_tiles = n_tiles;
    ra.queue = queue + slot;
    ra.lmin = RANGE_LO[r];
    ra.lmax = RANGE_HI[r];
    const bool wide = range_is_wide(r);
    // occupancy offset from the kernel's own register-limited occupancy
    const int per_simd = std::max(1, RANGE_WAVES[r] + (wide ? tu.occ_wide : tu.occ_narrow));
    const int wg = wide ? tu.wg_wide : tu.wg_narrow;
    const int64_t waves = std::min<int64_t>(n_tiles, (int64_t)cus * 4 * per_simd);
    return hip_status(launch_chains(r, ra, (int)waves, wg, on));
  };
  // stream of each kernel range: the caller's, or a side stream for the
  // two-word-row ranges (all on side 0, or range r on side r - 2)
  bool used[N_RANGES] = {false};
  for (int slot = 0; slot < mcmc_plan::kSlots; ++slot)
    if (p->range_tiles[slot] != 0) used[slot % N_RANGES] = true;
  bool narrow = false, wide = false;
  for (int r = 0; r < N_RANGES; ++r)
    if (used[r]) (range_is_wide(r) ? wide : narrow) = true;
  int side_of[N_RANGES];
  for (int r = 0; r < N_RANGES; ++r) {
    side_of[r] = -1;
    if (!used[r] || !range_is_wide(r) || tu.concurrent == 0) continue;
    if (tu.concurrent == 1 && !narrow) continue;   // the wide kernels alone: one stream
    side_of[r] = tu.concurrent == 1 ? 0 : r - (N_RANGES - mcmc_plan::kSides);
  }
  bool forked[mcmc_plan::kSides] = {false};
  bool any_side = false;
  for (int r = 0; r < N_RANGES; ++r)
    if (side_of[r] >= 0) any_side = forked[side_of[r]] = true;
  if (any_side) {
    if (hipEventRecord(p->fork, s) != hipSuccess) return MCMC_EDEVICE;
    for (int i = 0; i < mcmc_plan::kSides; ++i)
      if (forked[i] && hipStreamWaitEvent(p->side[i], p->fork, 0) != hipSuccess)
        return MCMC_EDEVICE;
  }
  for (int r = N_RANGES - 1; r >= 0; --r) {   // longest tiles first
    for (int m = 0; m < 2; ++m) {
      st = run_range(m * N_RANGES + r, side_of[r] >= 0 ? p->side[side_of[r]] : s);
      if (st != MCMC_OK) return st;
    }
  }
  for (int i = 0; i < mcmc_plan::kSides; ++i) {
    if (!forked[i]) continue;
    if (hipEventRecord(p->join[i], p->side[i]) != hipSuccess) return MCMC_EDEVICE;
    if (hipStreamWaitEvent(s, p->join[i], 0) != hipSuccess) return MCMC_EDEVICE;
  }

  DecideArgs d{};
  d.items = p->d_items;
  d.groups = p->d_groups;
  d.ln2 = log(2.0);
  d.n = p->n;
  d.S = S;
  d.n_final = nf;
  d.final_rows = final_rows;
  d.class_prob = prob;
  d.mean_n = mean_n;
  d.chosen = chosen;
  d.correction = correction;
  return hip_status(launch_decide(d, s));
}

int check_exec(const mcmc_plan* p, const uint8_t* syn, const double* prob, const uint8_t* chosen,
               const void* workspace, size_t workspace_bytes) {
  if (!p) return MCMC_EINVAL;
  if (p->n == 0) return MCMC_OK;
  if (!syn || !prob || !chosen) return MCMC_EINVAL;
  const PlanWorkspace wl = plan_workspace(p);
  if (!workspace || workspace_bytes < wl.bytes || ((uintptr_t)workspace % kAlign) != 0)
    return MCMC_EWORKSPACE;
  return MCMC_OK;
}

// Workload signature for the tuning cache: device CU count and the multiset
// of (L, K, chains, burn, sweeps, items) groups.
std::string plan_signature(const mcmc_plan* p) {
  std::string s = "cus=" + std::to_string(device_cus());
  for (size_t i = 0; i < p->groups.size(); ++i) {
    const GroupDesc& g = p->groups[i];
    s += ";" + std::to_string(g.L) + "," + std::to_string(g.K) + "," + std::to_string(g.C) + "," +
         std::to_string(g.burn) + "," + std::to_string(g.sweep_end - g.burn) + "," +
         std::to_string(g.n_items) + (p->group_noise[i] ? ",b" : "");
  }
  return s;
}

bool read_cache(const char* path, const std::string& sig, mcmc_tuning* t) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[1 << 16];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char* tab = strchr(line, '\t');
    if (!tab) continue;
    *tab = 0;
    if (sig != line) continue;
    mcmc_tuning v{};
    if (sscanf(tab + 1, "%d %d %d %d %d %d", &v.wg_narrow, &v.occ_narrow, &v.wg_wide,
               &v.occ_wide, &v.concurrent, &v.pair_small) == 6) {
      *t = v;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void write_cache(const char* path, const std::string& sig, const mcmc_tuning& t) {
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s\t%d %d %d %d %d %d\n", sig.c_str(), t.wg_narrow, t.occ_narrow, t.wg_wide,
          t.occ_wide, t.concurrent, t.pair_small);
  fclose(f);
}

}  // namespace

extern "C" {

namespace {

// (Re)build the plan's groups, items, tiles and tables from an item array
// (already validated) and copy them to the device, growing the plan's device
// block only when it is too small.
int build_plan_into(mcmc_plan* p, const mcmc_item* items, int64_t n);

// Empty plan: executes nothing.  The state a failed build leaves behind, so
// that no later call uses descriptors that were never uploaded.
void clear_plan(mcmc_plan* p) {
  p->n = 0;
  p->groups.clear();
  p->group_noise.clear();
  p->items.clear();
  p->tiles.clear();
  p->tables.clear();
  p->total_chains = p->total_rows = p->total_updates = 0;
  for (int r = 0; r < mcmc_plan::kSlots; ++r) p->range_first[r] = p->range_tiles[r] = 0;
  for (int m = 0; m < 2; ++m) p->small_tiles[m] = p->pair_first[m] = p->pair_tiles[m] = 0;
}

int build_plan(mcmc_plan* p, const mcmc_item* items, int64_t n) {
  const int st = build_plan_into(p, items, n);
  if (st != MCMC_OK) clear_plan(p);
  return st;
}

int build_plan_into(mcmc_plan* p, const mcmc_item* items, int64_t n) {
  release_graphs(p);
  p->n = n;
  p->groups.clear();
  p->group_noise.clear();
  p->items.clear();
  p->tiles.clear();
  p->tables.clear();
  p->total_chains = p->total_rows = p->total_updates = 0;
  for (int r = 0; r < mcmc_plan::kSlots; ++r) p->range_first[r] = p->range_tiles[r] = 0;
  for (int m = 0; m < 2; ++m) p->small_tiles[m] = p->pair_first[m] = p->pair_tiles[m] = 0;

  // groups: (L, K, C, burn, sweeps) -> items, in order of first appearance
  // (a batch has few distinct keys: linear search with a last-hit cache)
  using Key = std::tuple<int, int, int, int, int, int>;   // L, K, C, burn, sweeps, noise
  std::vector<std::pair<Key, std::vector<int64_t>>> by_key;
  size_t last = 0;
  for (int64_t i = 0; i < n; ++i) {
    const mcmc_item& it = items[i];
    const Key k{it.L, it.n_temps, it.chains, it.burn, it.sweeps, (int)it.noise};
    if (by_key.empty() || by_key[last].first != k) {
      last = by_key.size();
      for (size_t j = 0; j < by_key.size(); ++j)
        if (by_key[j].first == k) {
          last = j;
          break;
        }
      if (last == by_key.size()) by_key.push_back({k, {}});
    }
    by_key[last].second.push_back(i);
  }
  // per-chain cost of a group: (burn + sweeps) * n_stab; most costly first,
  // equal costs in key order
  std::vector<size_t> order(by_key.size());
  for (size_t j = 0; j < order.size(); ++j) order[j] = j;
  auto cost = [&](size_t j) {
    const Key& k = by_key[j].first;
    return ((int64_t)std::get<3>(k) + std::get<4>(k)) * n_stab(std::get<0>(k));
  };
  std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    const int64_t ca = cost(a), cb = cost(b);
    return ca != cb ? ca > cb : by_key[a].first < by_key[b].first;
  });

  // per-chain outputs, start blocks and table rows in the caller's order
  std::vector<int64_t> chain_off(n), rows_off(n), table_off(n);
  int64_t c_acc = 0, r_acc = 0, t_acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    chain_off[i] = c_acc;
    rows_off[i] = r_acc;
    table_off[i] = t_acc;
    c_acc += 4 * (int64_t)items[i].n_temps * items[i].chains;
    r_acc += (int64_t)words_per_config(items[i].L) * 4;
    t_acc += 4 * (int64_t)items[i].n_temps;
  }
  p->total_chains = c_acc;
  p->total_rows = r_acc;

  // acceptance tables and beta_bar per item, in parallel over contiguous
  // chunks (an item with the rate and ladder of the one before copies its rows)
  p->tables.resize((size_t)t_acc);
  std::vector<double> bbar(n), bstar(n);
  auto fill = [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      const mcmc_item& it = items[i];
      uint32_t* dst = p->tables.data() + table_off[i];
      const mcmc_item* prev = i > lo ? &items[i - 1] : nullptr;
      if (prev && it.p == prev->p && it.n_temps == prev->n_temps && it.noise == prev->noise &&
          it.beta_scale == prev->beta_scale) {
        std::copy(dst - 4 * it.n_temps, dst, dst);
        bbar[i] = bbar[i - 1];
        bstar[i] = bstar[i - 1];
      } else {
        // the same tables and temperatures as a uniform decode of this item
        mcmc_params prm{};
        prm.p = it.p;
        prm.n_temps = it.n_temps;
        prm.noise = it.noise;
        prm.beta_scale = it.beta_scale;
        fill_params_table(&prm, dst);
        bbar[i] = beta_bar_of(it.noise, it.p);
        bstar[i] = beta_top(&prm);
      }
    }
  };
  const int64_t kChunk = 4096;
  const int workers = (int)std::min<int64_t>(
      std::max(1u, std::min(16u, std::thread::hardware_concurrency())), (n + kChunk - 1) / kChunk);
  if (workers <= 1) {
    fill(0, n);
  } else {
    std::vector<std::thread> pool;
    const int64_t per = (n + workers - 1) / workers;
    for (int w = 0; w < workers; ++w) {
      const int64_t lo = w * per, hi = std::min(n, lo + per);
      if (lo < hi) pool.emplace_back(fill, lo, hi);
    }
    for (auto& t : pool) t.join();
  }

  p->items.reserve(n);
  for (size_t j : order) {
    const Key& k = by_key[j].first;
    const std::vector<int64_t>& members = by_key[j].second;
    GroupDesc g{};
    g.L = std::get<0>(k);
    g.K = std::get<1>(k);
    g.C = std::get<2>(k);
    g.burn = std::get<3>(k);
    g.sweep_begin = 0;
    g.sweep_end = std::get<3>(k) + std::get<4>(k);
    g.first_item = (int32_t)p->items.size();
    g.n_items = (int32_t)members.size();
    g.n_tasks = (int64_t)members.size() * 4 * g.K * g.C;
    const int gid = (int)p->groups.size();
    for (int64_t i : members) {
      const mcmc_item& src = items[i];
      ItemDesc it{};
      it.orig = i;
      it.syn_off = src.syn_offset;
      it.rows_off = rows_off[i];
      it.chain_off = chain_off[i];
      it.corr_off = src.corr_offset;
      it.table_off = table_off[i];
      it.beta_bar = bbar[i];
      it.beta_star = bstar[i];
      it.noise = (int32_t)src.noise;
      it.sid = src.syndrome_id;
      it.group = gid;
      it.err_thr = (uint32_t)floor(ldexp(src.p, 32));
      p->items.push_back(it);
      p->total_updates += 4 * (int64_t)src.n_temps * src.chains *
                          ((int64_t)src.burn + src.sweeps) * n_stab(src.L);
    }
    p->groups.push_back(g);
    p->group_noise.push_back(std::get<5>(k));
  }
  // tiles per launch slot (kernel range and noise model), each slot longest
  // first (groups are already in descending cost order)
  for (int slot = 0; slot < mcmc_plan::kSlots; ++slot) {
    const int r = slot % N_RANGES, m = slot / N_RANGES;
    p->range_first[slot] = (int64_t)p->tiles.size();
    // in range 0 the codes the pair kernel can take come last
    for (int part = 0; part < 2; ++part) {
      const int64_t before = (int64_t)p->tiles.size();
      for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const GroupDesc& g = p->groups[gi];
        if (range_of(g.L) != r || p->group_noise[gi] != m) continue;
        if ((g.L <= PAIR_L_MAX) != (part == 1)) continue;
        for (int64_t f = 0; f < g.n_tasks; f += TILE)
          p->tiles.push_back(TileDesc{(int32_t)gi, g.L, f});
      }
      if (r == 0 && part == 1) p->small_tiles[m] = (int64_t)p->tiles.size() - before;
    }
    p->range_tiles[slot] = (int64_t)p->tiles.size() - p->range_first[slot];
  }
  for (int m = 0; m < 2; ++m) {
    p->pair_first[m] = (int64_t)p->tiles.size();
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
      const GroupDesc& g = p->groups[gi];
      if (g.L > PAIR_L_MAX || p->group_noise[gi] != m) continue;
      for (int64_t f = 0; f < g.n_tasks; f += 2 * TILE)
        p->tiles.push_back(TileDesc{(int32_t)gi, g.L, f});
    }
    p->pair_tiles[m] = (int64_t)p->tiles.size() - p->pair_first[m];
  }
  if ((int64_t)p->tiles.size() > 0xFFFFFFFFll) return MCMC_ERANGE;

  // device copies in one block
  const size_t gsz = align_up(p->groups.size() * sizeof(GroupDesc) + 1);
  const size_t isz = align_up(p->items.size() * sizeof(ItemDesc) + 1);
  const size_t tsz = align_up(p->tiles.size() * sizeof(TileDesc) + 1);
  const size_t bsz = align_up(p->tables.size() * sizeof(uint32_t) + 1);
  const size_t need = gsz + isz + tsz + bsz;
  if (need > p->dev_bytes) {
    if (p->dev) (void)hipFree(p->dev);
    p->dev = nullptr;
    p->dev_bytes = 0;
    if (hipMalloc(&p->dev, need) != hipSuccess) return MCMC_EDEVICE;
    p->dev_bytes = need;
  }
  char* base = (char*)p->dev;
  p->d_groups = (GroupDesc*)base;
  p->d_items = (ItemDesc*)(base + gsz);
  p->d_tiles = (TileDesc*)(base + gsz + isz);
  p->d_tables = (uint32_t*)(base + gsz + isz + tsz);
  bool ok = true;
  if (!p->groups.empty())
    ok &= hipMemcpy(p->d_groups, p->groups.data(), p->groups.size() * sizeof(GroupDesc),
                    hipMemcpyHostToDevice) == hipSuccess;
  if (!p->items.empty())
    ok &= hipMemcpy(p->d_items, p->items.data(), p->items.size() * sizeof(ItemDesc),
                    hipMemcpyHostToDevice) == hipSuccess;
  if (!p->tiles.empty())
    ok &= hipMemcpy(p->d_tiles, p->tiles.data(), p->tiles.size() * sizeof(TileDesc),
                    hipMemcpyHostToDevice) == hipSuccess;
  if (!p->tables.empty())
    ok &= hipMemcpy(p->d_tables, p->tables.data(), p->tables.size() * sizeof(uint32_t),
                    hipMemcpyHostToDevice) == hipSuccess;
  return ok ? MCMC_OK : MCMC_EDEVICE;
}

int check_items(const mcmc_item* items, int64_t n) {
  if (n < 0 || n > ((int64_t)1 << 31)) return MCMC_ERANGE;
  if (n > 0 && !items) return MCMC_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    const int st = check_item(items[i]);
    if (st != MCMC_OK) return st;
  }
  return MCMC_OK;
}

}  // namespace

int mcmc_plan_create(const mcmc_item* items, int64_t n, uint64_t seed, uint32_t init,
                     mcmc_plan** out) {
  if (!out) return MCMC_EINVAL;
  *out = nullptr;
  if (init != MCMC_INIT_CANONICAL && init != MCMC_INIT_MATCHING && init != MCMC_INIT_MWPM)
    return MCMC_EINVAL;
  int st = check_items(items, n);
  if (st != MCMC_OK) return st;
  mcmc_plan* p = new (std::nothrow) mcmc_plan();
  if (!p) return MCMC_ENOMEM;
  p->seed = seed;
  p->init = init;
  (void)hipGetDevice(&p->device);
  st = build_plan(p, items, n);
  if (st != MCMC_OK) {
    mcmc_plan_destroy(p);
    return st;
  }
  bool ok = true;
  for (int i = 0; i < mcmc_plan::kSides; ++i) {
    ok &= hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking) == hipSuccess;
    ok &= hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming) == hipSuccess;
  }
  ok &= hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) == hipSuccess;
  ok &= hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    mcmc_plan_destroy(p);
    return MCMC_EDEVICE;
  }
  p->tuning.wg_narrow = 256;
  p->tuning.wg_wide = 256;
  p->tuning.occ_narrow = 0;
  p->tuning.occ_wide = 0;
  p->tuning.pair_small = 1;   // measured faster at every L <= 8 (1.02-1.7x)
  p->tuning.concurrent = 2;
  // the matching starts' side stream exists before any capture of the plan
  // (without it the starts run their launches in order)
  if (init == MCMC_INIT_MWPM) (void)mwpm_prepare_overlap();
  *out = p;
  return MCMC_OK;
}

int mcmc_plan_rebuild(mcmc_plan* p, const mcmc_item* items, int64_t n) {
  if (!p) return MCMC_EINVAL;
  const int st = check_items(items, n);
  if (st != MCMC_OK) return st;
  return build_plan(p, items, n);
}

int mcmc_plan_destroy(mcmc_plan* p) {
  if (!p) return MCMC_OK;
  release_graphs(p);
  if (p->fork) (void)hipEventDestroy(p->fork);
  for (int i = 0; i < mcmc_plan::kSides; ++i) {
    if (p->join[i]) (void)hipEventDestroy(p->join[i]);
    if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
  }
  if (p->capture) (void)hipStreamDestroy(p->capture);
  if (p->dev) (void)hipFree(p->dev);
  delete p;
  return MCMC_OK;
}

int mcmc_plan_info(const mcmc_plan* p, int64_t* total_chains, size_t* workspace_bytes,
                   int64_t* total_updates) {
  if (!p) return MCMC_EINVAL;
  if (total_chains) *total_chains = p->total_chains;
  if (workspace_bytes) *workspace_bytes = plan_workspace(p).bytes;
  if (total_updates) *total_updates = p->total_updates;
  return MCMC_OK;
}

int mcmc_plan_get_tuning(const mcmc_plan* p, mcmc_tuning* t) {
  if (!p || !t) return MCMC_EINVAL;
  *t = p->tuning;
  return MCMC_OK;
}

int mcmc_plan_set_tuning(mcmc_plan* p, const mcmc_tuning* t) {
  if (!p || !t) return MCMC_EINVAL;
  auto wg_ok = [](int wg) { return wg == 64 || wg == 128 || wg == 256; };
  if (!wg_ok(t->wg_narrow) || !wg_ok(t->wg_wide)) return MCMC_EINVAL;
  if (t->occ_narrow < -4 || t->occ_narrow > 8 || t->occ_wide < -2 || t->occ_wide > 8)
    return MCMC_ERANGE;
  if (t->concurrent < 0 || t->concurrent > 2) return MCMC_EINVAL;
  if (t->pair_small != 0 && t->pair_small != 1) return MCMC_EINVAL;
  p->tuning = *t;
  release_graphs(p);  // captured graphs hold the old launch shape
  return MCMC_OK;
}

int mcmc_plan_execute(mcmc_plan* p, const uint8_t* syndromes, double* class_prob,
                      double* mean_n, int64_t* sum_n, int64_t* accepts, uint8_t* chosen,
                      uint8_t* correction, void* workspace, size_t workspace_bytes,
                      void* stream) {
  int st = check_exec(p, syndromes, class_prob, chosen, workspace, workspace_bytes);
  if (st != MCMC_OK || p->n == 0) return st;
  return enqueue(p, syndromes, class_prob, mean_n, sum_n, accepts, chosen, correction, workspace,
                 (hipStream_t)stream);
}

int mcmc_plan_graph_launch(mcmc_plan* p, const uint8_t* syndromes, double* class_prob,
                           double* mean_n, int64_t* sum_n, int64_t* accepts, uint8_t* chosen,
                           uint8_t* correction, void* workspace, size_t workspace_bytes,
                           void* stream) {
  int st = check_exec(p, syndromes, class_prob, chosen, workspace, workspace_bytes);
  if (st != MCMC_OK || p->n == 0) return st;
  const std::vector<const void*> key = {syndromes, class_prob, mean_n, sum_n, accepts,
                                        chosen, correction, workspace};
  hipGraphExec_t exec = nullptr;
  for (auto& g : p->graphs)
    if (g.key == key) exec = g.exec;
  if (!exec) {
    if (hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return MCMC_EDEVICE;
    st = enqueue(p, syndromes, class_prob, mean_n, sum_n, accepts, chosen, correction, workspace,
                 p->capture);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->capture, &graph);
    if (st != MCMC_OK || e != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return st != MCMC_OK ? st : MCMC_EDEVICE;
    }
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return MCMC_EDEVICE;
    p->graphs.push_back(GraphEntry{key, exec});
  }
  return hip_status(hipGraphLaunch(exec, (hipStream_t)stream));
}

int mcmc_plan_sample(const mcmc_plan* p, uint64_t seed, uint8_t* syndromes, uint8_t* true_class,
                     void* stream) {
  if (!p) return MCMC_EINVAL;
  if (p->n == 0) return MCMC_OK;
  if (!syndromes || !true_class) return MCMC_EINVAL;
  return hip_status(launch_sample_items(p->d_items, p->d_groups, p->n,
                                        (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32),
                                        syndromes, true_class, (hipStream_t)stream));
}

int mcmc_plan_autotune(mcmc_plan* p, const uint8_t* syndromes, double* class_prob,
                       double* mean_n, int64_t* sum_n, int64_t* accepts, uint8_t* chosen,
                       uint8_t* correction, void* workspace, size_t workspace_bytes, void* stream,
                       const char* cache_path, mcmc_tuning* result) {
  int st = check_exec(p, syndromes, class_prob, chosen, workspace, workspace_bytes);
  if (st != MCMC_OK) return st;
  const std::string sig = plan_signature(p);
  mcmc_tuning best = p->tuning;
  if (cache_path && read_cache(cache_path, sig, &best)) {
    st = mcmc_plan_set_tuning(p, &best);
    if (st == MCMC_OK && result) *result = p->tuning;
    return st;
  }
  if (p->n == 0) {
    if (result) *result = p->tuning;
    return MCMC_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return MCMC_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return MCMC_EDEVICE;
  }
  auto time_of = [&](const mcmc_tuning& t, float* ms) -> int {
    p->tuning = t;
    if (hipEventRecord(e0, s) != hipSuccess) return MCMC_EDEVICE;
    int r = enqueue(p, syndromes, class_prob, mean_n, sum_n, accepts, chosen, correction,
                    workspace, s);
    if (r != MCMC_OK) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return MCMC_EDEVICE;
    return hip_status(hipEventElapsedTime(ms, e0, e1));
  };
  // coordinate search from the plan's current shape; every candidate decodes the
  // whole batch, and all candidates give identical outputs
  float best_ms = 0.0f, again = 0.0f;
  st = time_of(best, &best_ms);  // also warms up the code objects
  if (st == MCMC_OK) st = time_of(best, &best_ms);
  if (st == MCMC_OK) st = time_of(best, &again);
  best_ms = std::min(best_ms, again);
  // each move is applied to the best shape found so far
  const std::vector<std::function<void(mcmc_tuning&)>> moves = {
      [](mcmc_tuning& t) { t.wg_narrow = t.wg_wide = 64; },
      [](mcmc_tuning& t) { t.wg_narrow = t.wg_wide = 128; },
      [](mcmc_tuning& t) { t.occ_narrow = -1; },
      [](mcmc_tuning& t) { t.occ_narrow = 1; },
      [](mcmc_tuning& t) { t.occ_wide = -1; },
      [](mcmc_tuning& t) { t.occ_wide = 1; },
      [](mcmc_tuning& t) { t.concurrent = 0; },
      [](mcmc_tuning& t) { t.concurrent = 1; },
      [](mcmc_tuning& t) { t.concurrent = 2; },
      [](mcmc_tuning& t) { t.pair_small = 1 - t.pair_small; },
  };
  for (size_t i = 0; st == MCMC_OK && i < moves.size(); ++i) {
    mcmc_tuning cand = best;
    moves[i](cand);
    if (memcmp(&cand, &best, sizeof cand) == 0) continue;
    // the shorter of two executions: kernels on several streams interleave
    // differently from run to run
    float ms = 0.0f, ms2 = 0.0f;
    st = time_of(cand, &ms);
    if (st == MCMC_OK) st = time_of(cand, &ms2);
    ms = std::min(ms, ms2);
    if (st == MCMC_OK && ms < best_ms * 0.98f) {
      best_ms = ms;
      best = cand;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->tuning = best;
  release_graphs(p);
  if (st != MCMC_OK) return st;
  if (cache_path) write_cache(cache_path, sig, best);
  if (result) *result = best;
  return MCMC_OK;
}

}  // extern "C"
