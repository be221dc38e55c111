"""Plain FP64 CPU oracle for RGDBEK (randomized greedy double block extended
Kaczmarz), arXiv 2509.19267.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP implementation in ``paper_2509_19267_amd``; the two meet only through
the seeded input generators in ``workloads``, which hold none of the
method's arithmetic.

Modules
  philox   Philox4x64-10 counter-based generator (Salmon et al., SC'11).
  lnfun    the natural logarithm used for the exponential selection keys.
  select   block selection: draw k distinct indices with probability
           proportional to the residual weights (Section 2, Algorithm 1).
  blockls  the two pseudoinverse block projections (the GDBEK update rule
           that RGDBEK reuses, Section 1 / Section 2).
  rgdbek   Algorithm 1 iterated step by step, plus the stopping tests, the
           extended-residual refinement loop and the adjoint/gradient
           formulas.
  refsol   closed-form references (pseudoinverse solution and optimal
           residual, Theorem 2.3 notation).

Every function is written from the paper's definitions in FP64; where the
paper is silent the reading taken is stated in the function's docstring.
"""
