"""CPU oracle for the even-odd preconditioned Wilson/clover operator and BiCGStab.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or run
anything in this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark do. It shares no code with the GPU library.

It is written as the plain definitions, in float64/complex128 NumPy, with full
4x4 gamma matrices, full 3x3 links and full 12x12 site matrices, and none of
the GPU path's devices (no spin projection, no two-row links, no chiral
blocks, no even-odd storage).

Modules:

* ``dirac``   -- lattice geometry, the gamma basis, the hopping term, the
  Wilson operator, the clover term, the parity blocks of Eq. (1) and the
  Schur complement.
* ``solvers`` -- BiCGStab, CG and the FP64 defect-correction outer loop.
* ``sampled`` -- the same operators evaluated at a list of sites only, for
  checks on lattices too large for the whole-field oracle.
* ``dense``   -- brute-force 12V x 12V matrix of the operator for tiny
  lattices (an independent, loop-by-loop construction used as a pin).
* ``freefield`` -- momentum-space closed forms for unit links.
* ``sap``     -- the Schwarz alternating procedure preconditioner (block
  decomposition, Dirichlet block operator, minimal-residual block solves)
  and flexible BiCGStab.
* ``staggered`` -- the staggered operator, its even-odd normal system and CG.
* ``dwf``     -- the Moebius domain-wall operator (Shamir as a special case),
  its adjoint and the normal-equation solve.
* ``mg``      -- the two-level aggregation multigrid: chiral aggregation of
  test vectors, the coarse operator P^dag D P, the SAP-smoothed setup, the
  two-level preconditioner and its flexible BiCGStab solve.

Parity status: every function here is pinned by a CPU test (``tests/
test_oracle_*.py``) except the overall sign and trace convention of the clover
term, which no invariant can fix ("parity unpinned"; see ``dirac.clover``).
"""
