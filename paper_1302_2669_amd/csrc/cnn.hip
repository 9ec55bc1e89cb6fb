// Gate network kernels: a small convolutional network over the syndrome
// planes of one code size, trained on the decoder's own class probabilities
// to predict the class and a sweep budget (the learned-gate pattern grown on
// the decoder; not part of the paper's method).
//
// Layout: activations channels-last [pixel][channel] in bfloat16 (pixel =
// sample*L*L + y*L + x); master parameters fp32 in the order W1 [32][9][3],
// b1, W2 [32][9][32], b2, W3 [32][9][32], b3, Wh [7][L*L*32], bh [7].
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (bf16 operands,
// fp32 accumulation): forward M = pixels, N = 32 output channels,
// K = 9 taps x input channels; backward-data the same with the taps mirrored
// and the weight roles transposed; weight gradients M = 32, N = taps x input
// channels, K = pixels, split over pixel chunks and reduced in a fixed order.
// Lane layout of the 16x16x32 MFMA: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16] and D[4(l/16)+i][l%16], i = 0..3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "host_common.h"
#include "internal.h"

namespace mcmc {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32;

__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 lds8(const bf16* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int tap_dy(int t) { return t / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

// ---- input planes ----------------------------------------------------------
// x0[pixel][8]: 0 lit star (i, j) at (i, j), 1 lit plaquette (i, j) at (i, j),
// 2 the sample's p, 3..7 zero.
__global__ void encode_kernel(int L, int64_t B, const uint8_t* __restrict__ syn,
                              const float* __restrict__ p, bf16* __restrict__ x0) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = B * L * L;
  if (pix >= P) return;
  const int64_t b = pix / (L * L);
  const int r = (int)(pix - b * L * L), y = r / L, x = r % L;
  const uint8_t* s = syn + b * (int64_t)(2 * L * (L - 1));
  const int ns = L * (L - 1);
  const float star = (y < L - 1 && s[y * L + x]) ? 1.0f : 0.0f;
  const float plaq = (x < L - 1 && s[ns + y * (L - 1) + x]) ? 1.0f : 0.0f;
  bf16* o = x0 + pix * 8;
  o[0] = (bf16)star;
  o[1] = (bf16)plaq;
  o[2] = (bf16)p[b];
  for (int c = 3; c < 8; ++c) o[c] = (bf16)0.0f;
}

// ---- parameter casts -------------------------------------------------------
// wb1 [32][96] (k = tap*8 + ci, ci < 3), wb2/wb3 [32][288] (k = tap*32 + ci),
// wt2/wt3 [32 ci][288 (tap*32 + co)] = W[co][tap][ci], whb [16][L*L*32].
__global__ void cast_kernel(int L, const float* __restrict__ prm, const CnnOffsets off,
                            bf16* __restrict__ wb1, bf16* __restrict__ wb2, bf16* __restrict__ wb3,
                            bf16* __restrict__ wt2, bf16* __restrict__ wt3, bf16* __restrict__ whb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kh = (int64_t)L * L * CH;
  if (i < 32 * 96) {
    const int co = (int)(i / 96), k = (int)(i % 96), tap = k / 8, ci = k % 8;
    wb1[i] = (bf16)((tap < 9 && ci < 3) ? prm[off.W1 + (co * 9 + tap) * 3 + ci] : 0.0f);
  }
  if (i < 32 * 288) {
    wb2[i] = (bf16)prm[off.W2 + i];
    wb3[i] = (bf16)prm[off.W3 + i];
    const int ci = (int)(i / 288), k = (int)(i % 288), tap = k / 32, co = k % 32;
    wt2[i] = (bf16)prm[off.W2 + (co * 9 + tap) * 32 + ci];
    wt3[i] = (bf16)prm[off.W3 + (co * 9 + tap) * 32 + ci];
  }
  if (i < 16 * kh) {
    const int o = (int)(i / kh);
    whb[i] = (bf16)(o < 7 ? prm[off.Wh + i] : 0.0f);
  }
}

// ---- convolution as implicit GEMM -------------------------------------------
// Forward (MIRROR = false): out[p][n] = relu(sum_{tap,ci} in[p + tap][ci] *
// w[n][tap*CIN + ci] + bias[n]).  Backward data (MIRROR = true): out[p][n] =
// (sum_{tap,c} in[p - tap][c] * w[n][tap*CIN + c]) * (mask[p][n] > 0).
// One wave computes 16 pixels x 32 channels; 4 waves per workgroup.
template <int CIN, bool MIRROR>
__global__ void __launch_bounds__(256) conv_kernel(int L, int64_t P, const bf16* __restrict__ in,
                                                   const bf16* __restrict__ w,
                                                   const float* __restrict__ bias,
                                                   const bf16* __restrict__ mask,
                                                   bf16* __restrict__ out) {
  constexpr int KP = (9 * CIN + 31) / 32 * 32;
  constexpr int CHUNKS = CIN / 8;
  const int lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t pm = tile * 16 + (lane & 15);
  const int LL = L * L;
  int64_t b = 0;
  int y = 0, x = 0;
  if (pm < P) {
    b = pm / LL;
    const int r = (int)(pm - b * LL);
    y = r / L;
    x = r % L;
  }
  f32x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  const int grp = lane >> 4;
  const int n = lane & 15;
#pragma unroll
  for (int s = 0; s < KP / 32; ++s) {
    const int g = 4 * s + grp;
    const int tap = g / CHUNKS, cc = g % CHUNKS;
    bf16x8 a = zero8();
    if (tap < 9 && pm < P) {
      int dy = tap_dy(tap), dx = tap_dx(tap);
      if (MIRROR) { dy = -dy; dx = -dx; }
      const int yy = y + dy, xx = x + dx;
      if (yy >= 0 && yy < L && xx >= 0 && xx < L)
        a = load8(in + ((b * LL + yy * L + xx) * CIN + cc * 8));
    }
    const bf16x8 w0 = load8(w + (int64_t)n * KP + s * 32 + 8 * grp);
    const bf16x8 w1 = load8(w + (int64_t)(n + 16) * KP + s * 32 + 8 * grp);
    // weights as the A operand: D[channel][pixel], so lane (n, grp) ends
    // with channels 4 grp .. 4 grp + 3 (and + 16) of pixel n
    acc0 = mfma(w0, a, acc0);
    acc1 = mfma(w1, a, acc1);
  }
  if (pm >= P) return;
  bf16x8 o;   // channels 4 grp + i at o[i], 16 + 4 grp + i at o[4 + i]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c0 = 4 * grp + i, c1 = 16 + 4 * grp + i;
    float v0 = acc0[i], v1 = acc1[i];
    if (!MIRROR) {
      v0 = fmaxf(v0 + bias[c0], 0.0f);
      v1 = fmaxf(v1 + bias[c1], 0.0f);
    } else {
      v0 = (float)mask[pm * CH + c0] > 0.0f ? v0 : 0.0f;
      v1 = (float)mask[pm * CH + c1] > 0.0f ? v1 : 0.0f;
    }
    o[i] = (bf16)v0;
    o[4 + i] = (bf16)v1;
  }
  const uint4 ov = __builtin_bit_cast(uint4, o);
  *reinterpret_cast<uint2*>(out + pm * CH + 4 * grp) = make_uint2(ov.x, ov.y);
  *reinterpret_cast<uint2*>(out + pm * CH + 16 + 4 * grp) = make_uint2(ov.z, ov.w);
}

// ---- weight gradients ------------------------------------------------------
// Workgroup w handles samples [w*G, (w+1)*G) in order and writes
// part[w][co][c] = sum over its samples and pixels of dpre[p][co] *
// in[p + tap(c)][ci(c)] (c = tap*CIN + ci < 9*CIN; columns up to KP are zero)
// and partb[w][co] = sum of dpre[p][co].  Each sample is staged in LDS
// channel-major on its image padded by one zero pixel on every side
// ((L+2)^2 positions, rounded up to a multiple of 32): the MFMA k index runs
// over padded positions, so a tap is a constant offset of dy*(L+2)+dx and no
// bounds test is needed (padding positions hold zeros in both operands).
constexpr int WG_THREADS = 256;

struct WgradGeom {
  int PW, PS, KPAD, DSTR, OFF, ISTR;
};
__host__ __device__ inline WgradGeom wgrad_geom(int L) {
  WgradGeom g;
  g.PW = L + 2;
  g.PS = g.PW * g.PW;
  g.KPAD = (g.PS + 31) / 32 * 32;
  g.DSTR = g.KPAD + 8;                       // 16-byte rows, 16 lanes on disjoint banks
  g.OFF = (g.PW + 1 + 7) / 8 * 8;            // room for the most negative tap offset
  int istr = g.OFF + g.KPAD + g.PW + 1 + 1;
  istr = (istr + 1) / 2 * 2;
  if (((istr / 2) & 1) == 0) istr += 2;      // odd word stride: 16 lanes, 16 banks
  g.ISTR = istr;
  return g;
}
template <int CIN>
inline size_t wgrad_lds_bytes(int L) {
  const WgradGeom g = wgrad_geom(L);
  return ((size_t)CH * g.DSTR + (size_t)CIN * g.ISTR) * 2;
}

template <int CIN>
__global__ void __launch_bounds__(WG_THREADS) conv_wgrad_kernel(int L, int64_t B, int G,
                                                                const bf16* __restrict__ dpre,
                                                                const bf16* __restrict__ in,
                                                                float* __restrict__ part,
                                                                float* __restrict__ partb) {
  constexpr int KP = (9 * CIN + 31) / 32 * 32;
  constexpr int NT = KP / 16;                 // column tiles
  constexpr int TILES = 2 * NT;               // x 2 row tiles of 16 output channels
  constexpr int TPW = (TILES + 3) / 4;        // tiles per wave
  extern __shared__ __align__(16) unsigned char wsm[];
  const WgradGeom gm = wgrad_geom(L);
  bf16* dT = reinterpret_cast<bf16*>(wsm);            // [CH][DSTR]
  bf16* iT = dT + CH * gm.DSTR;                       // [CIN][ISTR]
  __shared__ float runs[8][CH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane >> 4, n = lane & 15;
  const int LL = L * L;
  const int64_t s0 = (int64_t)blockIdx.x * G;
  const int64_t s1 = s0 + G < B ? s0 + G : B;
  f32x4 acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = f32x4{0, 0, 0, 0};
  float bsum = 0.0f;
  const int nwords = (CH * gm.DSTR + CIN * gm.ISTR) / 2;
  for (int64_t smp = s0; smp < s1; ++smp) {
    __syncthreads();
    for (int i = tid; i < nwords; i += WG_THREADS) reinterpret_cast<uint32_t*>(wsm)[i] = 0u;
    __syncthreads();
    const int64_t pix0 = smp * LL;
    for (int i = tid; i < LL * CH; i += WG_THREADS) {
      const int r = i / CH, co = i % CH;
      const int q = (r / L + 1) * gm.PW + (r % L + 1);
      dT[co * gm.DSTR + q] = dpre[(pix0 + r) * CH + co];
    }
    for (int i = tid; i < LL * CIN; i += WG_THREADS) {
      const int r = i / CIN, ci = i % CIN;
      const int q = (r / L + 1) * gm.PW + (r % L + 1);
      iT[ci * gm.ISTR + gm.OFF + q] = in[(pix0 + r) * CIN + ci];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int t = wave + 4 * u;
      if (t >= TILES) continue;
      const int mt = t / NT, nt = t % NT;
      const int co = mt * 16 + n;
      const int c = nt * 16 + n;
      const bool col_ok = c < 9 * CIN;
      const int tap = col_ok ? c / CIN : 4, ci = col_ok ? c % CIN : 0;
      const int shift = tap_dy(tap) * gm.PW + tap_dx(tap);
      const bf16* arow = dT + co * gm.DSTR + 8 * grp;
      const bf16* brow = iT + ci * gm.ISTR + gm.OFF + shift + 8 * grp;
      for (int k = 0; k < gm.KPAD; k += 32) {
        const bf16x8 a = lds8(arow + k);
        bf16x8 bb;
#pragma unroll
        for (int j = 0; j < 8; ++j) bb[j] = brow[k + j];
        if (!col_ok) bb = zero8();
        acc[u] = mfma(a, bb, acc[u]);
      }
    }
    // bias: 8 runs of the padded row per channel, in run order
    {
      const int co = tid & 31, run = tid >> 5;
      const int per = gm.KPAD / 8;
      float s = 0.0f;
      for (int j = 0; j < per; ++j) s += (float)dT[co * gm.DSTR + run * per + j];
      runs[run][co] = s;
    }
    __syncthreads();
    if (tid < CH) {
      float s = 0.0f;
      for (int r = 0; r < 8; ++r) s += runs[r][tid];
      bsum += s;
    }
  }
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = wave + 4 * u;
    if (t >= TILES) continue;
    const int mt = t / NT, nt = t % NT;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      part[((int64_t)blockIdx.x * CH + mt * 16 + 4 * grp + i) * KP + nt * 16 + n] = acc[u][i];
  }
  if (tid < CH) partb[(int64_t)blockIdx.x * CH + tid] = bsum;
}

// Samples per weight-gradient workgroup: enough workgroups to fill the chip
// twice, at most one sample each for small batches.
inline int wgrad_group(int64_t B) {
  const int64_t target = 512;
  return (int)(B <= target ? 1 : (B + target - 1) / target);
}

// grad W[co][tap][ci] (ci < cin_real) and grad b[co] from the per-workgroup
// partials: a workgroup takes 16 outputs (index i: the W entries, then the
// 32 biases) and 16 row segments; segment g adds rows g, g+16, ... in order,
// and the 16 segment sums are added in segment order.
constexpr int RED_OUT = 16, RED_SEG = 16;

template <int CIN>
__global__ void __launch_bounds__(RED_OUT * RED_SEG) wgrad_reduce_kernel(
    int64_t rows, int cin_real, const float* __restrict__ part, const float* __restrict__ partb,
    float* __restrict__ gW, float* __restrict__ gb) {
  constexpr int KP = (9 * CIN + 31) / 32 * 32;
  __shared__ float seg_sum[RED_SEG][RED_OUT];
  const int o = threadIdx.x % RED_OUT, g = threadIdx.x / RED_OUT;
  const int nW = CH * 9 * cin_real;
  const int i = blockIdx.x * RED_OUT + o;
  float acc = 0.0f;
  if (i < nW) {
    const int co = i / (9 * cin_real), rem = i % (9 * cin_real);
    const int c = (rem / cin_real) * CIN + rem % cin_real;
    for (int64_t k = g; k < rows; k += RED_SEG) acc += part[(k * CH + co) * KP + c];
  } else if (i < nW + CH) {
    for (int64_t k = g; k < rows; k += RED_SEG) acc += partb[k * CH + (i - nW)];
  }
  seg_sum[g][o] = acc;
  __syncthreads();
  if (g == 0 && i < nW + CH) {
    float t = seg_sum[0][o];
    for (int j = 1; j < RED_SEG; ++j) t += seg_sum[j][o];
    if (i < nW) gW[i] = t;
    else gb[i - nW] = t;
  }
}

// ---- head ----------------------------------------------------------------
// logits[b][o] = sum_f a3[b][f] * whb[o][f] + bh[o], o < 7; 16 samples per
// wave.  The sum over the L*L pixel steps (32 features each) runs as 8
// interleaved MFMA chains, chain j taking steps j, j+8, ..., added in chain
// order at the end; the fused inference kernel uses the same order, so both
// give the same bits.
constexpr int HEAD_CHAINS = 8;

// One workgroup of HEAD_CHAINS waves per 16 samples: wave j runs chain j and
// the chains are added in order through LDS.
__global__ void __launch_bounds__(64 * HEAD_CHAINS) head_fwd_kernel(
    int L, int64_t B, const bf16* __restrict__ a3, const bf16* __restrict__ whb,
    const float* __restrict__ bh, float* __restrict__ logits) {
  __shared__ float part[HEAD_CHAINS][16][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, grp = lane >> 4, n = lane & 15;
  const int64_t tile = blockIdx.x;
  const int64_t bm = tile * 16 + n;
  const int LL = L * L;
  const int64_t kh = (int64_t)LL * CH;
  f32x4 acc = {0, 0, 0, 0};
  for (int st0 = wave; st0 < LL; st0 += 8 * HEAD_CHAINS) {
    bf16x8 aq[8], bq[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int st = st0 + j * HEAD_CHAINS;
      aq[j] = (st < LL && bm < B) ? load8(a3 + bm * kh + st * 32 + 8 * grp) : zero8();
      bq[j] = (st < LL && n < 7) ? load8(whb + (int64_t)n * kh + st * 32 + 8 * grp) : zero8();
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (st0 + j * HEAD_CHAINS < LL) acc = mfma(aq[j], bq[j], acc);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) part[wave][4 * grp + i][n] = acc[i];
  __syncthreads();
  if (threadIdx.x < 16 * 8) {
    const int row = threadIdx.x >> 3, o = threadIdx.x & 7;
    const int64_t bo = tile * 16 + row;
    if (bo < B && o < 7) {
      float t = part[0][row][o];
      for (int j = 1; j < HEAD_CHAINS; ++j) t = t + part[j][row][o];
      logits[bo * 8 + o] = t + bh[o];
    }
  }
}

// ---- fused inference -----------------------------------------------------
// One workgroup (8 waves) runs S samples through the three convolutions and
// the head with every activation in LDS; only the syndromes, rates, weights
// and logits touch global memory.  Same operations in the same order as the
// layered kernels above (conv: per-pixel tap/chunk k-steps on MFMA, bias,
// ReLU, bf16; head: 8 interleaved chains), so the logits are identical.
constexpr int INFER_THREADS = 512;
constexpr int INFER_WAVES = INFER_THREADS / 64;
static_assert(INFER_WAVES == HEAD_CHAINS, "both head paths add the same chains in the same order");
constexpr int ASTR = 40;      // bf16 per pixel of a 32-channel activation (80 B: 16 lanes
                              // reading 16 B each at this stride hit disjoint banks)
constexpr int W1STR = 104;    // bf16 per row of conv1 weights (96 used)
constexpr int W23STR = 296;   // bf16 per row of conv2/conv3 weights (288 used)
constexpr int INFER_WEIGHT_BYTES = 32 * W1STR * 2 + 2 * 32 * W23STR * 2;
constexpr int INFER_PART_BYTES = INFER_WAVES * 256 * 4 + 16;   // + a 16-byte zero slot


// One convolution over the group's pixels, LDS to LDS.  Each wave takes two
// 16-pixel tiles per trip (four independent MFMA chains).  Weights are the
// A operand (held in VGPRs for the layer), activations the B operand, so a
// lane ends with four consecutive channels of one pixel and writes them in
// one 8-byte store.  A tap outside the image (or a pixel past the group) is
// read from a 16-byte slot of zeros: the validity of the nine taps of a
// lane's pixel is a 9-bit mask computed once per tile.
template <int CIN, int WSTR, int INSTR>
__device__ __forceinline__ void conv_lds(int L, int LL, int npix, const bf16* in, const bf16* w,
                                         const float* __restrict__ bias, bf16* out,
                                         const bf16* zslot) {
  constexpr int KP = (9 * CIN + 31) / 32 * 32;
  constexpr int STEPS = KP / 32;
  constexpr int CHUNKS = CIN / 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, grp = lane >> 4, n = lane & 15;
  bf16x8 w0[STEPS], w1[STEPS];
#pragma unroll
  for (int st = 0; st < STEPS; ++st) {
    w0[st] = lds8(w + n * WSTR + st * 32 + 8 * grp);
    w1[st] = lds8(w + (n + 16) * WSTR + st * 32 + 8 * grp);
  }
  float bias0[4], bias1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bias0[i] = bias[4 * grp + i];
    bias1[i] = bias[16 + 4 * grp + i];
  }
  const int ntiles = (npix + 15) / 16;
  for (int t0 = wave; t0 < ntiles; t0 += 2 * INFER_WAVES) {
    int q[2];
    uint32_t valid[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      q[u] = (t0 + u * INFER_WAVES) * 16 + n;
      const bool ok = q[u] < npix;
      const int r = ok ? q[u] % LL : 0;
      const int y = r / L, x = r - (r / L) * L;
      uint32_t m = 0;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + tap_dy(tap), xx = x + tap_dx(tap);
        m |= (uint32_t)(yy >= 0 && yy < L && xx >= 0 && xx < L) << tap;
      }
      valid[u] = ok ? m : 0u;
    }
    f32x4 acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
#pragma unroll
    for (int st = 0; st < STEPS; ++st) {
      const int g = 4 * st + grp;
      const int tap = g / CHUNKS, cc = g % CHUNKS;
      const int toff = (tap_dy(tap) * L + tap_dx(tap)) * INSTR + cc * 8;
      bf16x8 xa[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool in_img = tap < 9 && ((valid[u] >> tap) & 1u);
        xa[u] = lds8(in_img ? in + q[u] * INSTR + toff : zslot);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        acc[u][0] = mfma(w0[st], xa[u], acc[u][0]);
        acc[u][1] = mfma(w1[st], xa[u], acc[u][1]);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (q[u] >= npix) continue;
      bf16x8 o;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o[i] = (bf16)fmaxf(acc[u][0][i] + bias0[i], 0.0f);
        o[4 + i] = (bf16)fmaxf(acc[u][1][i] + bias1[i], 0.0f);
      }
      const uint4 ov = __builtin_bit_cast(uint4, o);
      *reinterpret_cast<uint2*>(out + q[u] * ASTR + 4 * grp) = make_uint2(ov.x, ov.y);
      *reinterpret_cast<uint2*>(out + q[u] * ASTR + 16 + 4 * grp) = make_uint2(ov.z, ov.w);
    }
  }
}

__global__ void __launch_bounds__(INFER_THREADS) infer_kernel(
    int L, int S, int64_t B, const uint8_t* __restrict__ syn, const float* __restrict__ p,
    const bf16* __restrict__ wb1, const bf16* __restrict__ wb2, const bf16* __restrict__ wb3,
    const bf16* __restrict__ whb, const float* __restrict__ b1, const float* __restrict__ b2,
    const float* __restrict__ b3, const float* __restrict__ bh, float* __restrict__ logits,
    int64_t n_groups) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int LL = L * L, npix = S * LL, nst = 2 * L * (L - 1), ns = L * (L - 1);
  bf16* w1s = reinterpret_cast<bf16*>(smem);
  bf16* w2s = w1s + 32 * W1STR;
  bf16* w3s = w2s + 32 * W23STR;
  float* part = reinterpret_cast<float*>(w3s + 32 * W23STR);     // [waves][16][16]
  bf16* zslot = reinterpret_cast<bf16*>(part + INFER_WAVES * 256);
  bf16* bufA = zslot + 8;
  bf16* bufB = bufA + npix * ASTR;
  const int tid = threadIdx.x;

  for (int i = tid; i < 32 * 12; i += INFER_THREADS) {
    const int r = i / 12, c = i % 12;
    *reinterpret_cast<uint4*>(w1s + r * W1STR + c * 8) =
        *reinterpret_cast<const uint4*>(wb1 + r * 96 + c * 8);
  }
  for (int i = tid; i < 32 * 36; i += INFER_THREADS) {
    const int r = i / 36, c = i % 36;
    *reinterpret_cast<uint4*>(w2s + r * W23STR + c * 8) =
        *reinterpret_cast<const uint4*>(wb2 + r * 288 + c * 8);
    *reinterpret_cast<uint4*>(w3s + r * W23STR + c * 8) =
        *reinterpret_cast<const uint4*>(wb3 + r * 288 + c * 8);
  }
  if (tid < 8) zslot[tid] = (bf16)0.0f;
  // persistent: the weights stay in LDS while the workgroup walks its groups
  // of S samples (the barriers between the stages already order every
  // buffer's reuse from one group to the next)
  for (int64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
  const int64_t s0 = grp * S;
  const int nsm = (int)min((int64_t)S, B - s0);
  // input planes, 8 channels per pixel (the layout of the layered x0)
  for (int q = tid; q < npix; q += INFER_THREADS) {
    const int sm = q / LL, r = q - sm * LL, y = r / L, x = r - (r / L) * L;
    bf16x8 v = zero8();
    if (sm < nsm) {
      const uint8_t* sy = syn + (s0 + sm) * nst;
      v[0] = (bf16)((y < L - 1 && sy[y * L + x]) ? 1.0f : 0.0f);
      v[1] = (bf16)((x < L - 1 && sy[ns + y * (L - 1) + x]) ? 1.0f : 0.0f);
      v[2] = (bf16)p[s0 + sm];
    }
    *reinterpret_cast<uint4*>(bufA + q * 8) = __builtin_bit_cast(uint4, v);
  }
  __syncthreads();
  conv_lds<8, W1STR, 8>(L, LL, npix, bufA, w1s, b1, bufB, zslot);
  __syncthreads();
  conv_lds<32, W23STR, ASTR>(L, LL, npix, bufB, w2s, b2, bufA, zslot);
  __syncthreads();
  conv_lds<32, W23STR, ASTR>(L, LL, npix, bufA, w3s, b3, bufB, zslot);
  __syncthreads();

  // head: wave j runs chain j over pixel steps j, j+8, ...
  {
    const int lane = tid & 63, wave = tid >> 6, grp = lane >> 4, n = lane & 15;
    const int64_t kh = (int64_t)LL * CH;
    f32x4 acc = {0, 0, 0, 0};
    // eight of this chain's steps per trip: their weight loads (from L2) are
    // all in flight before the first product; rows 7..15 of the padded head
    // weights are zero and not read
    for (int st0 = wave; st0 < LL; st0 += 8 * INFER_WAVES) {
      bf16x8 bq[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int st = st0 + j * INFER_WAVES;
        bq[j] = (st < LL && n < 7) ? load8(whb + (int64_t)n * kh + st * 32 + 8 * grp) : zero8();
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int st = st0 + j * INFER_WAVES;
        if (st < LL) {
          const bf16x8 a = n < nsm ? lds8(bufB + (n * LL + st) * ASTR + 8 * grp) : zero8();
          acc = mfma(a, bq[j], acc);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) part[wave * 256 + (4 * grp + i) * 16 + n] = acc[i];
  }
  __syncthreads();
  if (tid < 16 * 8) {
    const int row = tid >> 3, o = tid & 7;
    if (row < nsm && o < 7) {
      float t = part[row * 16 + o];
      for (int j = 1; j < INFER_WAVES; ++j) t = t + part[j * 256 + row * 16 + o];
      logits[(s0 + row) * 8 + o] = t + bh[o];
    }
  }
  }
}

// Loss and dL/dlogits per sample (soft cross-entropy on the 4 class logits,
// weighted cross-entropy on the 3 budget logits), averaged over the batch.
__global__ void loss_kernel(int64_t B, const float* __restrict__ logits,
                            const float* __restrict__ tgt, const int32_t* __restrict__ budget,
                            float wb, float* __restrict__ dz, float* __restrict__ loss) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float* z = logits + b * 8;
  float m = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
  float e[4], se = 0.0f;
  for (int k = 0; k < 4; ++k) { e[k] = expf(z[k] - m); se += e[k]; }
  float lc = 0.0f;
  for (int k = 0; k < 4; ++k) {
    const float pk = e[k] / se;
    lc -= tgt[b * 4 + k] * ((z[k] - m) - logf(se));
    dz[b * 8 + k] = (pk - tgt[b * 4 + k]) / (float)B;
  }
  const float mb = fmaxf(fmaxf(z[4], z[5]), z[6]);
  float eb[3], sb = 0.0f;
  for (int k = 0; k < 3; ++k) { eb[k] = expf(z[4 + k] - mb); sb += eb[k]; }
  const int y = min(max(budget[b], 0), 2);
  const float lb = -((z[4 + y] - mb) - logf(sb));
  for (int k = 0; k < 3; ++k)
    dz[b * 8 + 4 + k] = wb * (eb[k] / sb - (k == y ? 1.0f : 0.0f)) / (float)B;
  dz[b * 8 + 7] = 0.0f;
  loss[b] = lc + wb * lb;
}

// grad Wh[o][f] = sum_b dz[b][o] a3[b][f]; grad bh[o] = sum_b dz[b][o].
// grad Wh[o][f] = sum_b dz[b][o] a3[b][f]: the batch is cut into
// HEAD_SEGS contiguous segments (blockIdx.y), each summed in batch order into
// hpart[seg][o][f]; head_wgrad_reduce adds the segments in order.
constexpr int HEAD_SEGS = 8;

__global__ void head_wgrad_kernel(int L, int64_t B, const float* __restrict__ dz,
                                  const bf16* __restrict__ a3, float* __restrict__ hpart) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kh = (int64_t)L * L * CH;
  if (f >= kh) return;
  const int seg = blockIdx.y;
  const int64_t per = (B + HEAD_SEGS - 1) / HEAD_SEGS;
  const int64_t b0 = seg * per, b1 = b0 + per < B ? b0 + per : B;
  float s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = b0; b < b1; ++b) {
    const float a = (float)a3[b * kh + f];
#pragma unroll
    for (int o = 0; o < 7; ++o) s[o] += dz[b * 8 + o] * a;
  }
#pragma unroll
  for (int o = 0; o < 7; ++o) hpart[((int64_t)seg * 7 + o) * kh + f] = s[o];
}

__global__ void head_wgrad_reduce_kernel(int L, int64_t B, const float* __restrict__ hpart,
                                         const float* __restrict__ dz, float* __restrict__ gWh,
                                         float* __restrict__ gbh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kh = (int64_t)L * L * CH;
  if (i < 7 * kh) {
    float t = hpart[i];
    for (int seg = 1; seg < HEAD_SEGS; ++seg) t += hpart[(int64_t)seg * 7 * kh + i];
    gWh[i] = t;
  }
  if (i < 7) {
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t b = 0;
    for (; b + 8 <= B; b += 8)
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += dz[(b + j) * 8 + i];
    for (int j = 0; b < B; ++b, ++j) s[j] += dz[b * 8 + i];
    float t = s[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) t += s[j];
    gbh[i] = t;
  }
}

// dpre3[b][f] = (sum_o dz[b][o] whb[o][f]) * (a3[b][f] > 0), rounded to bf16.
__global__ void head_dgrad_kernel(int L, int64_t B, const float* __restrict__ dz,
                                  const bf16* __restrict__ whb, const bf16* __restrict__ a3,
                                  bf16* __restrict__ dpre) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kh = (int64_t)L * L * CH;
  if (i >= B * kh) return;
  const int64_t b = i / kh, f = i - b * kh;
  float s = 0.0f;
  for (int o = 0; o < 7; ++o) s += dz[b * 8 + o] * (float)whb[o * kh + f];
  dpre[i] = (bf16)((float)a3[i] > 0.0f ? s : 0.0f);
}

__global__ void adam_kernel(int64_t n, float* __restrict__ prm, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mm = b1 * m[i] + (1.0f - b1) * g[i];
  const float vv = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
  m[i] = mm;
  v[i] = vv;
  prm[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Gate: class = argmax of the class logits (ties to the lowest); budget
// probabilities q = softmax of the budget logits; conf = (q0, q0 + q1, c),
// the probabilities that 0 and that at most the short budget reach the
// full-budget decision, and c = the class softmax's largest entry.
// route = 0 if q0 >= thr, else 1 if q0 + q1 >= thr, else 2.  With
// class_route the class head is read relative to the start decision: when
// c >= thr the route is 0 and flip = the argmax class (the class to compose
// with the start decision), else flip = 0.
__global__ void gate_kernel(int64_t B, const float* __restrict__ logits, float thr,
                            int class_route, uint8_t* __restrict__ route,
                            uint8_t* __restrict__ cls, float* __restrict__ conf,
                            uint8_t* __restrict__ flip, const GapRoute gap) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float* z = logits + b * 8;
  int best = 0;
  for (int k = 1; k < 4; ++k)
    if (z[k] > z[best]) best = k;
  float ec = 0.0f;
  for (int k = 0; k < 4; ++k) ec += expf(z[k] - z[best]);
  const float cmax = 1.0f / ec;
  const float m = fmaxf(fmaxf(z[4], z[5]), z[6]);
  const float e0 = expf(z[4] - m), e1 = expf(z[5] - m), e2 = expf(z[6] - m);
  const float sum = (e0 + e1) + e2;
  const float q0 = e0 / sum, q01 = (e0 + e1) / sum;
  uint8_t r = (uint8_t)(q0 >= thr ? 0 : (q01 >= thr ? 1 : 2));
  uint8_t f = 0;
  if (class_route && cmax >= thr) {
    r = 0;
    f = (uint8_t)best;
  }
  if (gap.table && r != 0) {  // the start-weight gap route: the no-sweep decision
    const int t = gap.table[gap_bin(gap.p[b])];
    if (t != (int)MCMC_GAP_NEVER && start_weight_gap(gap.weights + 4 * b) >= t) r = 0;
  }
  route[b] = r;
  cls[b] = (uint8_t)best;
  if (flip) flip[b] = f;
  if (conf) {
    conf[3 * b] = q0;
    conf[3 * b + 1] = q01;
    conf[3 * b + 2] = cmax;
  }
}

// Escalation margin of syndrome i from its short run's per-chain sums
// (block [4][K][C] at i 4KC): replica r's key of class e is the decision key
// restricted to that replica, sum_k w_k S[e][k][r] (w = 4, 2, ..., 4, 1 as in
// the decision; 1 for K = 1).  m_e = mean over the C replicas, v_e = their
// sample variance; with b the decided class (least m, ties to the lowest)
// and s the runner-up, z = (m_s - m_b) / sqrt((v_b + v_s) / C) (+inf when
// the spread is zero and m_s > m_b, 0 when m_s = m_b).
// flag[i] = route[i] == 1 && z < thr.
__global__ void escalate_kernel(int64_t n, const uint8_t* __restrict__ route,
                                const int64_t* __restrict__ sum_n, int K, int C, double thr,
                                uint8_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (route[i] != 1) {
    flag[i] = 0;
    return;
  }
  const int64_t* blk = sum_n + i * 4 * (int64_t)K * C;
  double mean[4], var[4];
  for (int e = 0; e < 4; ++e) {
    double s1 = 0.0;
    for (int r = 0; r < C; ++r) {
      int64_t key = 0;
      for (int k = 0; k < K; ++k) {
        const int64_t w = k + 1 == K ? 1 : ((k + 1) % 2 == 1 ? 4 : 2);
        key += w * blk[((int64_t)e * K + k) * C + r];
      }
      s1 += (double)key;
    }
    mean[e] = s1 / (double)C;
    double s2 = 0.0;
    for (int r = 0; r < C; ++r) {
      int64_t key = 0;
      for (int k = 0; k < K; ++k) {
        const int64_t w = k + 1 == K ? 1 : ((k + 1) % 2 == 1 ? 4 : 2);
        key += w * blk[((int64_t)e * K + k) * C + r];
      }
      const double d = (double)key - mean[e];
      s2 += d * d;
    }
    var[e] = s2 / (double)(C - 1);
  }
  int b = 0;
  for (int e = 1; e < 4; ++e)
    if (mean[e] < mean[b]) b = e;
  int s = b == 0 ? 1 : 0;
  for (int e = 0; e < 4; ++e)
    if (e != b && mean[e] < mean[s]) s = e;
  const double gap = mean[s] - mean[b];
  const double se = sqrt((var[b] + var[s]) / (double)C);
  bool esc;
  if (se > 0.0) esc = gap / se < thr;
  else esc = !(gap > 0.0);
  flag[i] = (uint8_t)esc;
}

__global__ void gather_kernel(int64_t n, int row, const int32_t* __restrict__ idx,
                              const uint8_t* __restrict__ src, uint8_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * row) return;
  const int64_t k = i / row;
  dst[i] = src[(int64_t)idx[k] * row + (i - k * row)];
}

__global__ void scatter_kernel(int64_t n, const int32_t* __restrict__ idx,
                               const uint8_t* __restrict__ src, uint8_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = src[i];
}

__global__ void pick_kernel(int64_t n, int nq, const int32_t* __restrict__ idx,
                            const uint8_t* __restrict__ cls, const uint8_t* __restrict__ reps,
                            uint8_t* __restrict__ corr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nq) return;
  const int64_t k = i / nq;
  const int q = (int)(i - k * nq);
  const int64_t o = idx[k];
  corr[o * nq + q] = reps[(k * 4 + cls[o]) * nq + q];
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

CnnOffsets cnn_offsets(int L) {
  CnnOffsets o{};
  const int64_t kh = (int64_t)L * L * CH;
  o.W1 = 0;
  o.b1 = o.W1 + CH * 9 * 3;
  o.W2 = o.b1 + CH;
  o.b2 = o.W2 + CH * 9 * CH;
  o.W3 = o.b2 + CH;
  o.b3 = o.W3 + CH * 9 * CH;
  o.Wh = o.b3 + CH;
  o.bh = o.Wh + 7 * kh;
  o.total = o.bh + 7;
  return o;
}

CnnWorkspace cnn_workspace(int L, int64_t B) {
  CnnWorkspace w{};
  const int64_t P = B * L * L, kh = (int64_t)L * L * CH;
  const int64_t chunks = (B + wgrad_group(B) - 1) / wgrad_group(B);   // weight-gradient rows
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) / 256 * 256;
    return at;
  };
  w.x0 = take((size_t)P * 8 * 2);
  w.a1 = take((size_t)P * CH * 2);
  w.a2 = take((size_t)P * CH * 2);
  w.a3 = take((size_t)P * CH * 2);
  w.wb1 = take(32 * 96 * 2);
  w.wb2 = take(32 * 288 * 2);
  w.wb3 = take(32 * 288 * 2);
  w.wt2 = take(32 * 288 * 2);
  w.wt3 = take(32 * 288 * 2);
  w.whb = take((size_t)16 * kh * 2);
  w.dz = take((size_t)B * 8 * 4);
  w.dp3 = take((size_t)P * CH * 2);
  w.dp2 = take((size_t)P * CH * 2);
  w.dp1 = take((size_t)P * CH * 2);
  w.part = take((size_t)chunks * CH * 288 * 4);
  w.partb = take((size_t)chunks * CH * 4);
  w.hpart = take((size_t)HEAD_SEGS * 7 * kh * 4);
  w.loss = take((size_t)B * 4);
  w.bytes = off;
  return w;
}

CnnWeights cnn_weights(int L) {
  CnnWeights w{};
  const int64_t kh = (int64_t)L * L * CH;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) / 256 * 256;
    return at;
  };
  w.wb1 = take(32 * 96 * 2);
  w.wb2 = take(32 * 288 * 2);
  w.wb3 = take(32 * 288 * 2);
  w.wt2 = take(32 * 288 * 2);
  w.wt3 = take(32 * 288 * 2);
  w.whb = take((size_t)16 * kh * 2);
  w.bytes = off;
  return w;
}

int cnn_infer_group(int L) {
  int dev = 0, maxlds = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
      hipSuccess)
    return 0;
  const int per = 2 * L * L * ASTR * 2;
  const int S = (maxlds - INFER_WEIGHT_BYTES - INFER_PART_BYTES) / per;
  return S < 1 ? 0 : (S > 16 ? 16 : S);
}

hipError_t cnn_infer(int L, int64_t B, const float* prm, const uint8_t* syn, const float* p,
                     float* logits, char* ws, hipStream_t s) {
  const CnnWeights wl = cnn_weights(L);
  const CnnOffsets off = cnn_offsets(L);
  const int64_t kh = (int64_t)L * L * CH;
  const int S = cnn_infer_group(L);
  if (S < 1) return hipErrorInvalidConfiguration;
  const int64_t n_cast = 16 * kh > 32 * 288 ? 16 * kh : 32 * 288;
  bf16* wb1 = reinterpret_cast<bf16*>(ws + wl.wb1);
  bf16* wb2 = reinterpret_cast<bf16*>(ws + wl.wb2);
  bf16* wb3 = reinterpret_cast<bf16*>(ws + wl.wb3);
  bf16* whb = reinterpret_cast<bf16*>(ws + wl.whb);
  hipLaunchKernelGGL(cast_kernel, dim3(blocks_for(n_cast, 256)), dim3(256), 0, s, L, prm, off, wb1,
                     wb2, wb3, reinterpret_cast<bf16*>(ws + wl.wt2),
                     reinterpret_cast<bf16*>(ws + wl.wt3), whb);
  const size_t lds = (size_t)INFER_WEIGHT_BYTES + INFER_PART_BYTES +
                     (size_t)2 * S * L * L * ASTR * 2;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&infer_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int64_t groups = (B + S - 1) / S;
  const int per_cu = std::max<int>(1, std::min<int>(4, (int)(163840 / lds)));
  const int64_t wgs = std::min<int64_t>(groups, (int64_t)device_cus() * per_cu);
  hipLaunchKernelGGL(infer_kernel, dim3((unsigned)wgs), dim3(INFER_THREADS), lds, s, L, S, B, syn,
                     p, wb1, wb2, wb3, whb, prm + off.b1, prm + off.b2, prm + off.b3, prm + off.bh,
                     logits, groups);
  return hipGetLastError();
}

#define WSP(T, name) reinterpret_cast<T*>(ws + wl.name)

hipError_t cnn_forward(int L, int64_t B, const float* prm, const uint8_t* syn, const float* p,
                       float* logits, char* ws, hipStream_t s) {
  const CnnWorkspace wl = cnn_workspace(L, B);
  const CnnOffsets off = cnn_offsets(L);
  const int64_t P = B * L * L, kh = (int64_t)L * L * CH;
  hipLaunchKernelGGL(encode_kernel, dim3(blocks_for(P, 256)), dim3(256), 0, s, L, B, syn, p,
                     WSP(bf16, x0));
  // one thread per entry of the largest of the cast arrays
  const int64_t n_cast = 16 * kh > 32 * 288 ? 16 * kh : 32 * 288;
  hipLaunchKernelGGL(cast_kernel, dim3(blocks_for(n_cast, 256)), dim3(256), 0, s, L, prm, off,
                     WSP(bf16, wb1), WSP(bf16, wb2), WSP(bf16, wb3), WSP(bf16, wt2),
                     WSP(bf16, wt3), WSP(bf16, whb));
  const unsigned g = blocks_for((P + 15) / 16, 4);
  hipLaunchKernelGGL((conv_kernel<8, false>), dim3(g), dim3(256), 0, s, L, P, WSP(bf16, x0),
                     WSP(bf16, wb1), prm + off.b1, nullptr, WSP(bf16, a1));
  hipLaunchKernelGGL((conv_kernel<32, false>), dim3(g), dim3(256), 0, s, L, P, WSP(bf16, a1),
                     WSP(bf16, wb2), prm + off.b2, nullptr, WSP(bf16, a2));
  hipLaunchKernelGGL((conv_kernel<32, false>), dim3(g), dim3(256), 0, s, L, P, WSP(bf16, a2),
                     WSP(bf16, wb3), prm + off.b3, nullptr, WSP(bf16, a3));
  hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)((B + 15) / 16)), dim3(64 * HEAD_CHAINS), 0, s,
                     L, B,
                     WSP(bf16, a3), WSP(bf16, whb), prm + off.bh, logits);
  return hipGetLastError();
}

hipError_t cnn_backward(int L, int64_t B, const float* prm, const float* logits, const float* tgt,
                        const int32_t* budget, float wb, float* grads, float* loss, char* ws,
                        hipStream_t s) {
  const CnnWorkspace wl = cnn_workspace(L, B);
  const CnnOffsets off = cnn_offsets(L);
  const int64_t P = B * L * L, kh = (int64_t)L * L * CH;
  const int G = wgrad_group(B);
  const int64_t chunks = (B + G - 1) / G;
  const size_t lds32 = wgrad_lds_bytes<32>(L), lds8 = wgrad_lds_bytes<8>(L);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&conv_wgrad_kernel<32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds32);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&conv_wgrad_kernel<8>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds8);
  float* lossv = loss ? loss : WSP(float, loss);
  hipLaunchKernelGGL(loss_kernel, dim3(blocks_for(B, 256)), dim3(256), 0, s, B, logits, tgt,
                     budget, wb, WSP(float, dz), lossv);
  hipLaunchKernelGGL(head_wgrad_kernel, dim3(blocks_for(kh, 256), HEAD_SEGS), dim3(256), 0, s, L,
                     B, WSP(float, dz), WSP(bf16, a3), WSP(float, hpart));
  hipLaunchKernelGGL(head_wgrad_reduce_kernel, dim3(blocks_for(7 * kh, 256)), dim3(256), 0, s, L,
                     B, WSP(float, hpart), WSP(float, dz), grads + off.Wh, grads + off.bh);
  hipLaunchKernelGGL(head_dgrad_kernel, dim3(blocks_for(B * kh, 256)), dim3(256), 0, s, L, B,
                     WSP(float, dz), WSP(bf16, whb), WSP(bf16, a3), WSP(bf16, dp3));
  const unsigned g = blocks_for((P + 15) / 16, 4);
  // conv3: weights, then data back into a2's gradient
  hipLaunchKernelGGL((conv_wgrad_kernel<32>), dim3((unsigned)chunks), dim3(WG_THREADS), lds32, s,
                     L, B, G,
                     WSP(bf16, dp3), WSP(bf16, a2), WSP(float, part), WSP(float, partb));
  hipLaunchKernelGGL((wgrad_reduce_kernel<32>), dim3(blocks_for(CH * 9 * CH + CH, RED_OUT)),
                     dim3(RED_OUT * RED_SEG), 0,
                     s, chunks, CH, WSP(float, part), WSP(float, partb), grads + off.W3,
                     grads + off.b3);
  hipLaunchKernelGGL((conv_kernel<32, true>), dim3(g), dim3(256), 0, s, L, P, WSP(bf16, dp3),
                     WSP(bf16, wt3), nullptr, WSP(bf16, a2), WSP(bf16, dp2));
  // conv2
  hipLaunchKernelGGL((conv_wgrad_kernel<32>), dim3((unsigned)chunks), dim3(WG_THREADS), lds32, s,
                     L, B, G,
                     WSP(bf16, dp2), WSP(bf16, a1), WSP(float, part), WSP(float, partb));
  hipLaunchKernelGGL((wgrad_reduce_kernel<32>), dim3(blocks_for(CH * 9 * CH + CH, RED_OUT)),
                     dim3(RED_OUT * RED_SEG), 0,
                     s, chunks, CH, WSP(float, part), WSP(float, partb), grads + off.W2,
                     grads + off.b2);
  hipLaunchKernelGGL((conv_kernel<32, true>), dim3(g), dim3(256), 0, s, L, P, WSP(bf16, dp2),
                     WSP(bf16, wt2), nullptr, WSP(bf16, a1), WSP(bf16, dp1));
  // conv1: weights only
  hipLaunchKernelGGL((conv_wgrad_kernel<8>), dim3((unsigned)chunks), dim3(WG_THREADS), lds8, s,
                     L, B, G,
                     WSP(bf16, dp1), WSP(bf16, x0), WSP(float, part), WSP(float, partb));
  hipLaunchKernelGGL((wgrad_reduce_kernel<8>), dim3(blocks_for(CH * 9 * 3 + CH, RED_OUT)),
                     dim3(RED_OUT * RED_SEG), 0, s,
                     chunks, 3, WSP(float, part), WSP(float, partb), grads + off.W1,
                     grads + off.b1);
  return hipGetLastError();
}

hipError_t cnn_adam(int64_t n, float* prm, const float* g, float* m, float* v, float lr, float b1,
                    float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, prm, g, m, v, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t cnn_gate(int64_t B, const float* logits, float thr, bool class_route, uint8_t* route,
                    uint8_t* cls, float* conf, uint8_t* flip, const GapRoute& gap,
                    hipStream_t s) {
  hipLaunchKernelGGL(gate_kernel, dim3(blocks_for(B, 256)), dim3(256), 0, s, B, logits, thr,
                     class_route ? 1 : 0, route, cls, conf, flip, gap);
  return hipGetLastError();
}

hipError_t cnn_escalate_flags(int64_t n, const uint8_t* route, const int64_t* sum_n, int K, int C,
                              double thr, uint8_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(escalate_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, route, sum_n,
                     K, C, thr, flag);
  return hipGetLastError();
}

hipError_t cnn_gather(int64_t n, int row, const int32_t* idx, const uint8_t* src, uint8_t* dst,
                      hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n * row, 256)), dim3(256), 0, s, n, row, idx,
                     src, dst);
  return hipGetLastError();
}

hipError_t cnn_scatter(int64_t n, const int32_t* idx, const uint8_t* src, uint8_t* dst,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, idx, src, dst);
  return hipGetLastError();
}

hipError_t cnn_pick(int64_t n, int nq, const int32_t* idx, const uint8_t* cls,
                    const uint8_t* reps, uint8_t* corr, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(pick_kernel, dim3(blocks_for(n * nq, 256)), dim3(256), 0, s, n, nq, idx, cls,
                     reps, corr);
  return hipGetLastError();
}

}  // namespace mcmc
