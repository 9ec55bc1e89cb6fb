// Minimum-weight matching class starts (arXiv:1302.2669, Sec. III and Sec. IV).
//
// Sec. III decodes each anyon type on its own by minimum-weight matching and
// forces the other line parity with an extra boundary anyon; the 2 x 2
// combinations are the four class hypotheses, and Sec. IV starts each class's
// chain from its hypothesis.  Each (type, parity) problem is solved exactly
// (mwpm_solver.h): a minimum T-join of the lattice graph, i.e. a minimum-weight
// perfect matching of the lit sites and the boundary vertices the parity
// needs, under shortest-path distances, ties broken by a per-pair splitmix64
// key so that the optimum is unique.
//
// Paths: a matched anyon pair a < a' (site order) whose Manhattan distance is
// its distance takes the direct path (plaquettes: along a's grid row to the
// column of a', then along that column; stars: along a's grid column to the
// row of a', then along that row), else both anyons go to the nearer
// boundary option (NEAR on a tie); anyon-boundary matches take the straight
// string and NEAR-FAR the logical string.  Class c = x part of parity c & 1
// with z part of parity c >> 1.
//
// One workgroup per syndrome.  Its two waves each solve one anyon type (both
// parities, the second from the first's solution) with the whole solver state
// in LDS (at large L one wave takes both types in turn), XOR their parts into
// bit planes, and the workgroup packs the four class starts.  Up to three
// launches by problem size (capacity tiers); the larger two, which hold few
// syndromes but long solves, run on a side stream beside the first.
#include <mutex>

#include "device_common.h"
#include "internal.h"

#define MW_FN __device__ __forceinline__
#define MW_HD __host__ __device__ inline
#include "mwpm_solver.h"

namespace mcmc {

namespace {

struct Wave64 {
  static constexpr int N = 64;
  int lane;
  MW_FN void sync() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  MW_FN int uni(int x) const { return __builtin_amdgcn_readfirstlane(x); }
  MW_FN int64_t uni64(int64_t x) const {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
  }
  // one step of an unsigned minimum over the wave: combine with the value DPP
  // control CTRL brings in (lanes it does not reach keep the identity)
  template <int CTRL, int ROWS>
  MW_FN static uint32_t min_step(uint32_t v) {
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, CTRL, ROWS, 0xf, false);
    return o < v ? o : v;
  }
  // unsigned minimum of v over the wave: prefix minima within each row of 16
  // lanes (row_shr 1, 2, 4, 8), then row 0's result into row 1 and row 2's
  // into row 3 (row_bcast:15), then row 1's into rows 2 and 3
  // (row_bcast:31); lane 63 holds the minimum.
  MW_FN static uint32_t wave_min(uint32_t v) {
    v = min_step<0x111, 0xf>(v);
    v = min_step<0x112, 0xf>(v);
    v = min_step<0x114, 0xf>(v);
    v = min_step<0x118, 0xf>(v);
    v = min_step<0x142, 0xa>(v);
    v = min_step<0x143, 0xc>(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
  }
  // smallest (signed) key over the wave and the idx of the lowest lane
  // holding it: the minimum of the high words (sign bit flipped, so that the
  // unsigned order is the signed one), then, only when several lanes share
  // it, the minimum of their low words
  MW_FN void argmin(int64_t& key, int& idx) const {
    const uint32_t lo = (uint32_t)key, hi = (uint32_t)((uint64_t)key >> 32) ^ 0x80000000u;
    const uint32_t mh = wave_min(hi);
    uint64_t at = __ballot(hi == mh);
    uint32_t ml;
    if (__popcll(at) > 1) {
      ml = wave_min(hi == mh ? lo : 0xFFFFFFFFu);
      at = __ballot(hi == mh && lo == ml);
    } else {
      ml = (uint32_t)__builtin_amdgcn_readlane((int)lo, __builtin_ctzll(at));
    }
    idx = __builtin_amdgcn_readlane(idx, __builtin_ctzll(at));
    key = (int64_t)(((uint64_t)(mh ^ 0x80000000u) << 32) | ml);
  }
  // one step of the grouped minimum: (hi, lo, ix) from the lane DPP control
  // CTRL names, lexicographically unsigned (unreached lanes bring all ones)
  template <int CTRL, int ROWS>
  MW_FN static void seg_step(uint32_t& hi, uint32_t& lo, uint32_t& ix) {
    const uint32_t oh = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)hi, CTRL, ROWS, 0xf, false);
    const uint32_t ol = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)lo, CTRL, ROWS, 0xf, false);
    const uint32_t oi = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)ix, CTRL, ROWS, 0xf, false);
    const bool take = oh < hi || (oh == hi && (ol < lo || (ol == lo && oi < ix)));
    hi = take ? oh : hi;
    lo = take ? ol : lo;
    ix = take ? oi : ix;
  }
  // smallest (signed key, idx >= 0) within each aligned group of 2^lg lanes
  // (lg wave-uniform, 0..6), left in the group's last lane: the prefix
  // minima of wave_min stopped after lg steps, each lane then holding the
  // minimum over the 2^lg lanes ending at it
  MW_FN void seg_argmin(int64_t& key, int& idx, int lg) const {
    uint32_t lo = (uint32_t)key, hi = (uint32_t)((uint64_t)key >> 32) ^ 0x80000000u;
    uint32_t ix = (uint32_t)idx;
    if (lg >= 1) seg_step<0x111, 0xf>(hi, lo, ix);
    if (lg >= 2) seg_step<0x112, 0xf>(hi, lo, ix);
    if (lg >= 3) seg_step<0x114, 0xf>(hi, lo, ix);
    if (lg >= 4) seg_step<0x118, 0xf>(hi, lo, ix);
    if (lg >= 5) seg_step<0x142, 0xa>(hi, lo, ix);
    if (lg >= 6) seg_step<0x143, 0xc>(hi, lo, ix);
    key = (int64_t)(((uint64_t)(hi ^ 0x80000000u) << 32) | lo);
    idx = (int)ix;
  }
  MW_FN bool any(bool p) const { return __ballot(p) != 0ull; }
  MW_FN int compact(bool take, int& count) const {
    const uint64_t bal = __ballot(take);
    const int slot = count + __popcll(bal & ((1ull << lane) - 1ull));
    count += __popcll(bal);
    return slot;
  }
  MW_FN void xor_word(uint32_t* p, uint32_t v) const { atomicXor(p, v); }
};

// waves per workgroup: one per anyon type when both states fit in 64 KB,
// else one wave taking the types in turn
int mwpm_waves(int cap) { return 2 * mw::region_bytes(cap) <= 64 * 1024 ? 2 : 1; }

size_t mwpm_lds(int cap) {
  return mwpm_waves(cap) * mw::region_bytes(cap) + (4 * mw::ROWS + 4) * sizeof(uint32_t);
}

// Capacity of the first launch: two 64-vertex states and the planes take
// 11.4 KB of LDS, so 14 two-wave workgroups (7 waves per SIMD) fit in a
// compute unit's 160 KB; at L = 13, p = 0.15 this holds 99% of the
// syndromes.
constexpr int MWPM_FAST_CAP = 64;

// Capacity of the launch after it (5 waves per SIMD at most): the problems
// of the typical syndromes of the larger codes (lit sites of one type up to
// about 2/5 of them, at least 85); the rare larger syndromes go to a last
// launch sized for a fully lit code.
int mwpm_small_capacity(int L) {
  const int full = mw::capacity(L);
  int c = 2 * L * (L - 1) / 5 + 8;
  if (c < 88) c = 88;
  c = (c + 3) & ~3;
  return c < full ? c : full;
}

// vertices of the second-parity problem of a type with k lit sites (the
// larger of the two): k + NEAR + FAR, or k + FAR + NEAR + the dummy
__device__ __forceinline__ int max_vertices(int k) { return (k & 1) ? k + 3 : k + 2; }

}  // namespace

// Wave w solves anyon types w, w + waves (0 plaquettes / x parts, 1 stars /
// z parts): parity 0 from the start, then parity 1 from parity 0's solution;
// problem p = 2 type + parity paints plane p.  A launch takes the syndromes
// whose larger problem needs more than `lo` and at most `hi` vertices, in a
// state sized for `cap`.  WPE is the register budget in waves per SIMD: 7
// (72 VGPRs, some spills) for the launch of capacity MWPM_FAST_CAP, whose
// LDS allows 7; 5 (96 VGPRs, a few spills) for the larger capacities, whose
// LDS allows at most 5 (at 4 waves, 117 VGPRs and none, the kernel is 15%
// slower; at 8, 64 VGPRs, the scalar spills make it 28% slower than at 7).
template <int WPE, int CAP>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(WPE)))
init_mwpm_kernel(const StartArgs a, int cap_arg, int waves, int lo, int hi) {
  // CAP != 0: the capacity as a compile-time constant, so that every solver
  // array sits at a constant offset from the wave's region
  const int cap = CAP ? CAP : cap_arg;
  extern __shared__ __align__(16) uint8_t mw_lds[];
  __shared__ int lit[2];
  const int64_t s = blockIdx.x;
  if (s >= a.n) return;
  const StartItem si = start_item(a, s);
  const int L = si.L;
  const int nsite = L * (L - 1);
  if (threadIdx.x < 2) lit[threadIdx.x] = 0;
  __syncthreads();
  int cs = 0, cp = 0;
  for (int t = threadIdx.x; t < nsite; t += blockDim.x) {
    cs += si.sy[t] != 0;
    cp += si.sy[nsite + t] != 0;
  }
  if (cs) atomicAdd(&lit[1], cs);
  if (cp) atomicAdd(&lit[0], cp);
  __syncthreads();
  const int need = max(max_vertices(lit[0]), max_vertices(lit[1]));
  if (need <= lo || need > hi) return;  // another launch takes it
  const int wave = threadIdx.x >> 6;
  const size_t region = mw::region_bytes(cap);
  uint32_t* planes = reinterpret_cast<uint32_t*>(mw_lds + waves * region);  // [4][ROWS]
  int* wsum = reinterpret_cast<int*>(planes + 4 * mw::ROWS);
  for (int k = threadIdx.x; k < 4 * mw::ROWS; k += blockDim.x) planes[k] = 0u;
  if (threadIdx.x < 4) wsum[threadIdx.x] = 0;
  __syncthreads();
  if (wave < waves) {
    mw::Solver<Wave64> m;
    m.wv.lane = threadIdx.x & 63;
    m.carve(mw_lds + wave * region, cap);
    for (int t = wave; t < 2; t += waves) {
      m.load(si.sy, L, t != 0, 0);
      m.solve();
      m.wv.sync();
      m.paint(planes + (2 * t) * mw::ROWS, 0);
      m.wv.sync();
      m.solve_other_parity(si.sy);
      m.wv.sync();
      m.paint(planes + (2 * t + 1) * mw::ROWS, 1);
      m.wv.sync();
    }
  }
  __syncthreads();
  // class c: x part of parity c & 1 (problem c & 1), z part of parity c >> 1
  // (problem 2 + (c >> 1))
  const int R = 2 * L - 1, W = words_per_row(L);
  const int nq = 2 * L * L - 2 * L + 1, side_len = 2 * L - 1;
  for (int t = threadIdx.x; t < 4 * R; t += blockDim.x) {
    const int cls = t / R, r = t % R;
    const uint32_t xb = planes[(cls & 1) * mw::ROWS + r];
    const uint32_t zb = planes[(2 + (cls >> 1)) * mw::ROWS + r];
    const int fields = (r & 1) ? L - 1 : L;
    const uint32_t valid = fields >= 32 ? ~0u : ((1u << fields) - 1u);
    atomicAdd(&wsum[cls], si.noise ? __builtin_popcount(xb & valid) + __builtin_popcount(zb & valid)
                                    : __builtin_popcount((xb | zb) & valid));
    if (a.rows) {
      for (int w = 0; w < W; ++w) {
        uint32_t word = 0;
        for (int f = 0; f < 16; ++f) {
          const int kk = 16 * w + f;
          const uint32_t code = kk < fields ? (((xb >> kk) & 1u) | (((zb >> kk) & 1u) << 1)) : 3u;
          word |= code << (2 * f);
        }
        a.rows[si.rows_off + (r * W + w) * 4 + cls] = word;
      }
    }
    if (a.bytes) {
      uint8_t* out = a.bytes + (si.orig * 4 + cls) * nq + (r * side_len + (r & 1)) / 2;
      for (int kk = 0; kk < fields; ++kk)
        out[kk] = (uint8_t)(((xb >> kk) & 1u) | (((zb >> kk) & 1u) << 1));
    }
  }
  __syncthreads();
  if (a.weights && threadIdx.x < 4) a.weights[si.orig * 4 + threadIdx.x] = wsum[threadIdx.x];
}

namespace {

// Per device: the side stream of the larger tiers and the events that fork
// it from and join it to the caller's stream.  Created on first use outside
// a stream capture (or by mwpm_prepare_overlap) and kept until the process
// ends; the mutex orders concurrent callers' fork-launch-join sequences.
struct Overlap {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kOverlapDevices = 64;
std::mutex g_overlap_mu;
Overlap g_overlap[kOverlapDevices];

// the current device's entry, created if `create`; null if it does not exist
// (or cannot be made)
Overlap* overlap_entry(bool create) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kOverlapDevices) return nullptr;
  Overlap& o = g_overlap[dev];
  if (o.side || !create) return o.side ? &o : nullptr;
  Overlap n;
  if (hipStreamCreateWithFlags(&n.side, hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&n.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&n.join, hipEventDisableTiming) != hipSuccess) {
    if (n.fork) (void)hipEventDestroy(n.fork);
    (void)hipStreamDestroy(n.side);
    return nullptr;
  }
  o = n;
  return &o;
}

hipError_t launch_tier(const StartArgs& a, int cap, int lo, int hi, hipStream_t s) {
  const size_t lds = mwpm_lds(cap);
  // the capacity compiled in only where the launch's is exactly that one
  // (smaller codes have smaller single-tier capacities)
  const bool fast = cap <= MWPM_FAST_CAP, fixed = cap == MWPM_FAST_CAP;
  const void* fn = fixed  ? reinterpret_cast<const void*>(init_mwpm_kernel<7, MWPM_FAST_CAP>)
                   : fast ? reinterpret_cast<const void*>(init_mwpm_kernel<7, 0>)
                          : reinterpret_cast<const void*>(init_mwpm_kernel<5, 0>);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lds);
    if (e != hipSuccess) return e;
  }
  if (fixed)
    hipLaunchKernelGGL((init_mwpm_kernel<7, MWPM_FAST_CAP>), dim3((unsigned)a.n), dim3(128), lds,
                       s, a, cap, mwpm_waves(cap), lo, hi);
  else if (fast)
    hipLaunchKernelGGL((init_mwpm_kernel<7, 0>), dim3((unsigned)a.n), dim3(128), lds, s, a, cap,
                       mwpm_waves(cap), lo, hi);
  else
    hipLaunchKernelGGL((init_mwpm_kernel<5, 0>), dim3((unsigned)a.n), dim3(128), lds, s, a, cap,
                       mwpm_waves(cap), lo, hi);
  return hipGetLastError();
}

}  // namespace

hipError_t mwpm_prepare_overlap() {
  std::lock_guard<std::mutex> lock(g_overlap_mu);
  return overlap_entry(true) ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t launch_init_mwpm(const StartArgs& a, hipStream_t s, bool may_create) {
  if (a.n == 0) return hipSuccess;
  const int L = a.items ? a.max_L : a.L;
  if (L < MCMC_L_MIN || L > MCMC_L_MAX) return hipErrorInvalidValue;
  // capacity tiers: the 7-wave launch, the typical syndromes of the larger
  // codes, a fully lit code
  const int full = mw::capacity(L), mid = mwpm_small_capacity(L);
  int caps[3], nt = 0;
  if (mid > MWPM_FAST_CAP) caps[nt++] = MWPM_FAST_CAP;
  caps[nt++] = mid;
  if (full > mid) caps[nt++] = full;
  int lo[3], hi[3];
  for (int t = 0; t < nt; ++t) {
    lo[t] = t ? caps[t - 1] : 0;
    hi[t] = t + 1 < nt ? caps[t] : 0x7fffffff;
  }
  if (nt == 1) return launch_tier(a, caps[0], lo[0], hi[0], s);
  // the later tiers on the side stream, launched first so that their few long
  // workgroups start at once; without a side stream, in order on s
  std::lock_guard<std::mutex> lock(g_overlap_mu);
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap_status) != hipSuccess) cap_status = hipStreamCaptureStatusNone;
  const Overlap* o = overlap_entry(may_create && cap_status == hipStreamCaptureStatusNone);
  hipError_t e = hipSuccess;
  if (o) {
    if ((e = hipEventRecord(o->fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(o->side, o->fork, 0)) != hipSuccess) return e;
    for (int t = 1; t < nt; ++t)
      if ((e = launch_tier(a, caps[t], lo[t], hi[t], o->side)) != hipSuccess) return e;
    if ((e = launch_tier(a, caps[0], lo[0], hi[0], s)) != hipSuccess) return e;
    if ((e = hipEventRecord(o->join, o->side)) != hipSuccess) return e;
    return hipStreamWaitEvent(s, o->join, 0);
  }
  for (int t = 0; t < nt; ++t)
    if ((e = launch_tier(a, caps[t], lo[t], hi[t], s)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace mcmc
