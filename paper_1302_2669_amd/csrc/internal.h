// Internal interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcmcdec.h"

namespace mcmc {

// Offsets of the pieces of a chain-state buffer holding T chains of a
// distance-L code (struct of arrays, every piece 256-byte aligned):
//   rows [RW][T] uint32 (word-major), n [T] int32, S [T] int64, A [T] int64.
struct ChainStateLayout {
  size_t rows, n, S, A, bytes;
};
ChainStateLayout chain_state_layout(int L, int64_t T);

struct ChainArgs {
  const uint32_t* init_rows;   // [RW][n*4] word-major class starts
  const int32_t* init_n;       // [n*4] their weights
  const uint32_t* syndrome_ids;// [n] or nullptr (=> index)
  int64_t n;                   // syndromes
  int32_t K, C;                // temperatures, chains per class and temperature
  int32_t burn, sweep_begin, sweep_end;
  uint32_t k0, k1;             // Philox key
  uint32_t table[MCMC_TEMPS_MAX][4];  // acceptance thresholds A_k[1..4], row k-1
  int64_t* S_out;              // [T]
  int64_t* A_out;              // [T]
  int32_t* n_out;              // [T]
  uint32_t* state_rows;        // [RW][T] final configurations, or nullptr
  const uint32_t* resume_rows; // [RW][T] with resume
  const int32_t* resume_n;
  const int64_t* resume_S;
  const int64_t* resume_A;
  uint32_t* corr_rows;         // [RW][n*4]: chain 0 at k = K of every class, or nullptr
  int16_t* trace;              // [T][trace_len] or nullptr
  int64_t trace_len;
};

template <int L>
hipError_t launch_chain_L(const ChainArgs& a, hipStream_t s, bool trace, bool resume);
hipError_t launch_chain(int L, const ChainArgs& a, hipStream_t s, bool trace, bool resume);

// rows ([RW][n*4] word-major), weights ([n*4]) and bytes ([n*4][n_q]) may each be nullptr.
hipError_t launch_init(int L, const uint8_t* syn, int64_t n, uint32_t* rows, int32_t* weights,
                       uint8_t* bytes, hipStream_t s);
// Greedy-matching class starts, same outputs as launch_init.
hipError_t launch_init_matching(int L, const uint8_t* syn, int64_t n, uint32_t* rows,
                                int32_t* weights, uint8_t* bytes, hipStream_t s);
hipError_t launch_unpack(int L, const uint32_t* rows, int64_t count, int64_t stride,
                         uint8_t* out, int32_t* weights, hipStream_t s);

struct DecideArgs {
  const int64_t* S;            // [n][4][K][C]
  const int32_t* n_final;      // [n][4][K][C]
  const uint32_t* corr_rows;   // [RW][n*4] or nullptr
  int64_t n;
  int32_t K, C, L, sweeps;
  double beta_bar, f0, log_z0; // f0 = 3/4 n_q, log_z0 = n_stab log 2
  double* class_prob;          // [n][4]
  double* mean_n;              // [n][4] or nullptr
  uint8_t* chosen;             // [n]
  uint8_t* correction;         // [n][n_q] or nullptr
};
hipError_t launch_decide(const DecideArgs& a, hipStream_t s);

hipError_t launch_sample(int L, uint32_t threshold, uint32_t k0, uint32_t k1, const uint32_t* ids,
                         uint32_t id_base, int64_t n, uint8_t* syn, uint8_t* true_class,
                         uint8_t* errors, hipStream_t s);

}  // namespace mcmc
