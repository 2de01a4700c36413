"""Reference oracle for the uniform sparse FFT (usFFT) hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU
restatement of what the method computes (Kaemmerer, Potts, Taubert, "The
uniform sparse FFT with application to PDEs with random coefficients",
Alg. 1 and Sec. 2-3).  It exists so that the HIP implementation can be
checked against something written independently from the paper.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never does, and it shares no code, tables or
constants with the HIP path.

Modules
  rng      counter-based SplitMix64 draws (tails y', lattice generators z)
  fem      P1 finite elements on the uniform triangulated unit square,
           element-by-element assembly, banded Cholesky solve
  lattice  admissible lattice sizes and the multiple rank-1 lattice planner
  dft      naive DFTs (1-D detection, lattice bins)
  select   per-node selection, uniform OR over nodes, set join
  usfft    Alg. 1 driver, trigonometric-polynomial sampler, evaluation
  fem_mesh P1 elements on a general triangulation, sparse direct solve
  periodization  tent and lognormal maps of the affine / lognormal models
  evaluation     error measures, variance, sensitivity indices and
                 expectation of the approximation (Sec. 4, 4.1)

Every function states the passage it follows.  Parity status of each part is
listed in the module headers; "parity unpinned" marks parts whose only check
is seed-matched agreement with the HIP path.
"""
