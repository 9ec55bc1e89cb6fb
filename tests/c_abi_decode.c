/*
 * The decoder driven from plain C through the C-ABI alone (no Python, no
 * torch): sample depolarizing errors on the device, decode them, copy the
 * decisions back, and print them with the logical error rate.
 *
 *   c_abi_decode L p sweeps chains n seed out.txt
 *
 * out.txt receives one line per syndrome: "<chosen> <true class>".  Exit
 * status 0 on success, 1 on any library or runtime error (message on stderr).
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/mcmcdec.h"

static int fail(const char* what, int status) {
  fprintf(stderr, "%s: %s (%d)\n", what, mcmc_strerror(status), status);
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 8) {
    fprintf(stderr, "usage: %s L p sweeps chains n seed out.txt\n", argv[0]);
    return 1;
  }
  mcmc_params prm;
  memset(&prm, 0, sizeof prm);               /* depolarizing, default beta* */
  prm.L = atoi(argv[1]);
  prm.p = atof(argv[2]);
  prm.sweeps = atoi(argv[3]);
  prm.chains = atoi(argv[4]);
  prm.n_temps = 1;
  prm.init = MCMC_INIT_MATCHING;
  const int64_t n = atoll(argv[5]);
  prm.seed = strtoull(argv[6], NULL, 0);

  int32_t nq = 0, ns = 0;
  int st = mcmc_geometry(prm.L, &nq, &ns);
  if (st != MCMC_OK) return fail("mcmc_geometry", st);
  size_t ws_bytes = 0;
  st = mcmc_workspace_size(&prm, n, &ws_bytes);
  if (st != MCMC_OK) return fail("mcmc_workspace_size", st);

  uint8_t *d_syn = NULL, *d_true = NULL, *d_chosen = NULL;
  double* d_prob = NULL;
  void* d_ws = NULL;
  if (hipMalloc((void**)&d_syn, (size_t)n * ns) != hipSuccess ||
      hipMalloc((void**)&d_true, (size_t)n) != hipSuccess ||
      hipMalloc((void**)&d_chosen, (size_t)n) != hipSuccess ||
      hipMalloc((void**)&d_prob, (size_t)n * 4 * sizeof(double)) != hipSuccess ||
      hipMalloc(&d_ws, ws_bytes ? ws_bytes : 1) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  st = mcmc_sample_errors(prm.L, prm.p, prm.seed, NULL, 0, n, d_syn, d_true, NULL, NULL);
  if (st != MCMC_OK) return fail("mcmc_sample_errors", st);
  st = mcmc_decode_batch(d_syn, NULL, n, &prm, d_prob, NULL, NULL, NULL, d_chosen, NULL, NULL,
                         NULL, d_ws, ws_bytes, NULL);
  if (st != MCMC_OK) return fail("mcmc_decode_batch", st);

  uint8_t* chosen = (uint8_t*)malloc((size_t)n);
  uint8_t* truth = (uint8_t*)malloc((size_t)n);
  if (!chosen || !truth) return 1;
  if (hipMemcpy(chosen, d_chosen, (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(truth, d_true, (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "hipMemcpy failed\n");
    return 1;
  }
  FILE* f = fopen(argv[7], "w");
  if (!f) return 1;
  int64_t wrong = 0;
  for (int64_t i = 0; i < n; ++i) {
    fprintf(f, "%d %d\n", chosen[i], truth[i]);
    wrong += chosen[i] != truth[i];
  }
  fclose(f);
  printf("ok n=%lld logical_error=%.6f\n", (long long)n, (double)wrong / (double)n);
  free(chosen);
  free(truth);
  hipFree(d_syn);
  hipFree(d_true);
  hipFree(d_chosen);
  hipFree(d_prob);
  hipFree(d_ws);
  return 0;
}
