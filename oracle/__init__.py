"""Plain CPU oracle for the single-temperature MCMC surface-code decoder.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use it.  It shares no code, tables or constants with the HIP library; the two
are written independently from the same conventions, so that agreement between
them is evidence rather than tautology.

Paper: A. Hutter, J. R. Wootton, D. Loss, "An efficient Markov chain Monte
Carlo algorithm for the surface code" (arXiv:1302.2669).

Modules
-------
geometry   planar code of distance L, supports, colours, logical lines (Sec. II)
philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11)
tables     beta-bar (Eq. betaBar), temperature ladder, uint32 acceptance table
sampler    depolarizing or independent bit/phase-flip errors (Eq. pauliChannel),
           syndromes, true class
init       one syndrome-consistent representative per logical class
chains     colour-phased Metropolis chains (Sec. IV, Sec. IV.A, Sec. V)
estimator  thermodynamic integration (Eq. main) and the class decision
enumerate  exact class partition functions by enumerating stabilizer products
decoder    the whole decode, composed from the above
spacetime  imperfect measurements (Sec. VI): sampler, starts, chains, decode
cnn        the gate network in float64 (forward, backward, Adam, bf16 rounding)

Every floating-point quantity is float64.  Integer work uses numpy integer
arrays; nothing here is blocked, fused or reordered beyond the paper's steps.
"""
