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
constexpr int kQueueSlots = 8;
static_assert(kQueueSlots >= N_RANGES, "one queue counter per kernel range");

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bool valid_L(int32_t L) { return L >= MCMC_L_MIN && L <= MCMC_L_MAX; }

// beta_bar = -log((p/3)/(1-p))  (Eq. betaBar)
inline double beta_bar(double p) { return -log((p / 3.0) / (1.0 - p)); }

inline bool valid_p(double p) { return p > 0.0 && p < 0.75; }  // false for NaN

inline int n_qubits(int L) { return 2 * L * L - 2 * L + 1; }
inline int n_stab(int L) { return 2 * L * (L - 1); }

// A_k[Delta] = floor(2^32 exp(-beta_k Delta)), beta_k = k beta_bar / K, row k-1.
inline void fill_table(double p, int32_t K, uint32_t* out) {
  const double bb = beta_bar(p);
  for (int k = 1; k <= K; ++k) {
    const double beta = ((double)k * bb) / (double)K;
    for (int d = 1; d <= 4; ++d) {
      const double w = exp(-(beta * (double)d));
      out[(k - 1) * 4 + (d - 1)] = (uint32_t)floor(ldexp(w, 32));
    }
  }
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
