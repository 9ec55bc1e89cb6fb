// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/mcmcdec.h"
#include "internal.h"

namespace mcmc {

constexpr size_t kAlign = 256;

// Tile-queue counters at the head of every workspace, one per chain kernel
// range; all of them are zeroed before each launch sequence.
constexpr int kQueueSlots = 16;
static_assert(kQueueSlots >= 2 * N_RANGES + 2,
              "one queue counter per kernel range and noise model, and per pair launch");

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bool valid_L(int32_t L) { return L >= MCMC_L_MIN && L <= MCMC_L_MAX; }

// beta_bar = -log((p/3)/(1-p))  (Eq. betaBar)
inline double beta_bar(double p) { return -log((p / 3.0) / (1.0 - p)); }

inline bool valid_p(double p) { return p > 0.0 && p < 0.75; }  // false for NaN

inline int n_qubits(int L) { return 2 * L * L - 2 * L + 1; }
inline int n_stab(int L) { return 2 * L * (L - 1); }

// A[Delta] = floor(2^32 exp(-beta Delta)), Delta = 1..4.
inline void fill_row(double beta, uint32_t* out) {
  for (int d = 1; d <= 4; ++d) {
    const double w = exp(-(beta * (double)d));
    out[d - 1] = (uint32_t)floor(ldexp(w, 32));
  }
}

// A_k[Delta] = floor(2^32 exp(-beta_k Delta)), beta_k = k beta_bar / K, row k-1.
inline void fill_table(double p, int32_t K, uint32_t* out) {
  const double bb = beta_bar(p);
  for (int k = 1; k <= K; ++k) fill_row(((double)k * bb) / (double)K, out + (k - 1) * 4);
}

// ---- noise models -----------------------------------------------------------
// Independent bit/phase flips with rate q on each part: a configuration with
// m flipped parts has relative weight (q/(1-q))^m, so beta_bar = log((1-q)/q).
inline bool valid_noise(uint32_t noise) {
  return noise == MCMC_NOISE_DEPOLARIZING || noise == MCMC_NOISE_BITPHASE;
}
inline bool valid_rate(uint32_t noise, double p) {
  return noise == MCMC_NOISE_BITPHASE ? (p > 0.0 && p < 0.5) : valid_p(p);
}
inline double beta_bar_of(uint32_t noise, double p) {
  return noise == MCMC_NOISE_BITPHASE ? log((1.0 - p) / p) : beta_bar(p);
}
// beta* / beta_bar of the single-temperature decoder (0 selects the model's
// default: the paper finds 0.85 best under independent flips).
inline double beta_scale_of(uint32_t noise, double scale) {
  if (scale != 0.0) return scale;
  return noise == MCMC_NOISE_BITPHASE ? 0.85 : 1.0;
}
// The highest sampled temperature: beta* for K = 1, beta_bar otherwise.
inline double beta_top(const mcmc_params* prm) {
  const double bb = beta_bar_of(prm->noise, prm->p);
  return prm->n_temps == 1 ? beta_scale_of(prm->noise, prm->beta_scale) * bb : bb;
}
// Thresholds [K][4] of a uniform decode.
inline void fill_params_table(const mcmc_params* prm, uint32_t* out) {
  const int K = prm->n_temps;
  if (K == 1) {
    fill_row(beta_top(prm), out);
    return;
  }
  const double bb = beta_bar_of(prm->noise, prm->p);
  for (int k = 1; k <= K; ++k) fill_row(((double)k * bb) / (double)K, out + (k - 1) * 4);
}

// Tables [n][K][4] and beta_bar [n] of n rates, on up to 16 host threads
// (each value is computed exactly as fill_table / beta_bar compute it).
void fill_tables_parallel(const double* p, int64_t n, int32_t K, uint32_t* tables, double* beta);

inline int hip_status(hipError_t e) { return e == hipSuccess ? MCMC_OK : MCMC_EDEVICE; }

// Compute units of the current device (cached per device).
int device_cus();

// Default persistent grid: enough waves to fill every SIMD at the kernel's
// occupancy.
inline int default_waves(int range, int cus) { return cus * 4 * RANGE_WAVES[range]; }

}  // namespace mcmc
