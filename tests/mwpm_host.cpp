// Host build of the library's class-start matching solver (the kernel's own
// source in mwpm_solver.h, run with a one-lane wave policy), for checking it
// against the oracle on the CPU, under the address and undefined-behaviour
// sanitizers.
//
// stdin:  int32 L, int32 n, then n syndromes of n_stab bytes.
// stdout: per syndrome and problem p = 0..3 (type p >> 1, parity p & 1,
//         solved as the kernel does: parity 1 from parity 0's solution):
//         int32 failed, then 2L-1 uint32 bit rows of the part.
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../include/mcmcdec.h"

#define MW_FN inline
#define MW_HD inline
#include "../paper_1302_2669_amd/csrc/mwpm_solver.h"

struct Wave1 {
  static constexpr int N = 1;
  int lane = 0;
  void sync() const {}
  void argmin(int64_t&, int&) const {}
  void seg_argmin(int64_t&, int&, int) const {}
  bool any(bool p) const { return p; }
  int compact(bool take, int& count) const {
    const int slot = count;
    count += take ? 1 : 0;
    return slot;
  }
  void xor_word(uint32_t* p, uint32_t v) const { *p ^= v; }
  int uni(int x) const { return x; }
  int64_t uni64(int64_t x) const { return x; }
};

int main() {
  int32_t L = 0, n = 0;
  if (fread(&L, 4, 1, stdin) != 1 || fread(&n, 4, 1, stdin) != 1) return 2;
  if (L < MCMC_L_MIN || L > MCMC_L_MAX || n < 0) return 2;
  const int nstab = 2 * L * (L - 1);
  const int rows = 2 * L - 1;
  const int cap = mcmc::mw::capacity(L);
  // exactly the solver's region, so that an access past it is reported
  std::vector<uint8_t> syn(nstab);
  for (int s = 0; s < n; ++s) {
    if (fread(syn.data(), 1, nstab, stdin) != (size_t)nstab) return 3;
    for (int t = 0; t < 2; ++t) {  // as the kernel: parity 0, then parity 1 from it
      uint8_t* region = static_cast<uint8_t*>(malloc(mcmc::mw::region_bytes(cap)));
      mcmc::mw::Solver<Wave1> m;
      m.carve(region, cap);
      m.load(syn.data(), L, t != 0, 0);
      for (int parity = 0; parity < 2; ++parity) {
        if (parity) m.solve_other_parity(syn.data());
        else m.solve();
        std::vector<uint32_t> plane(rows, 0u);
        m.paint(plane.data(), parity);
        const int32_t failed = m.fail ? 1 : 0;
        fwrite(&failed, 4, 1, stdout);
        fwrite(plane.data(), 4, rows, stdout);
      }
      free(region);
    }
  }
  return 0;
}
