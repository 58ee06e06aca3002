"""FP64 CPU oracle for the per-event squared matrix element |M|^2.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code, table or constant generator with the HIP implementation.

What it computes follows the workflow of the paper (Sec. IV.a/IV.b: random
numbers -> RAMBO phase-space sampling -> SIGMAKIN matrix element), with every
step written from its textbook or published definition:

* ``philox``   Philox4x32-10 counter-based random numbers (Salmon, Moraes,
               Dror, Shaw, SC'11) and the bits->double map.
* ``rambo``    RAMBO massless sampling and massive rescaling (Kleiss,
               Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359).
* ``lorentz``  explicit 4x4 Dirac algebra, helicity spinors, polarisation
               vectors (helicity formalism of Sec. II).
* ``colour``   SU(3) generators, structure constants and colour matrices by
               brute-force traces (colour-flow decomposition of Sec. II).
* ``amplitudes`` Feynman-rule amplitudes: e+e- -> mu+mu- (Fig. 1) written
               out, gg -> tt~ written out with explicit colour indices, and a
               recursion over subsets of gluons for t t~ + n gluons in two
               forms: colour-dressed with explicit adjoint indices (plain
               definition) and colour-decomposed onto T-strings (the
               dual-amplitude form of Sec. II).
* ``me``       |M|^2 = (1/IDEN) sum over helicities and colours, the sampling
               chain, and d(|M|^2 w)/dr by reverse-mode differentiation.

All arithmetic is float64 / complex128 (numpy for the integer RNG, torch CPU
for the physics so that autograd supplies the reverse-mode gradient).
"""
