"""FP64 CPU oracle for the Split-SPCP hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct NumPy implementation of what
the GPU path computes.  It exists to check the HIP library; it is not part of
the product.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it.  It shares no code with the HIP
path (no kernels, headers, helpers, tables or pre/post-processing); both sides
only consume the same seeded inputs from ``paper_1702_02241_amd.synth``.

Contents (each function cites the passage it follows):

* ``objective`` -- Huber marginal phi, objective f(U,V), gradient (Sec. 1
  "Marginalization in S", eq. PhiDef, eq. smoothNC; Sec. 3.2 eq. diff;
  Sec. 5 eq. Thm5).
* ``lbfgs``     -- L-BFGS with memory 10 and a strong-Wolfe line search
  (Sec. 5.1; algorithm from Nocedal & Wright, which the paper cites).
* ``convex``    -- FISTA with singular-value thresholding on the convex
  problem eq. genConvex (Sec. 1: proximal gradient methods apply).
* ``certificate`` -- the convergence certificate of Sec. 3.4 (exact and
  efficient forms, the factor-based SVD of its footnote, the gap bound
  eq. Fbound with F_bound).
* ``rsvd``      -- randomized SVD initialisation (Sec. 4.2).
* ``mlp``       -- two-layer MLP forward/backward/Adam used to check the
  warm-start network kernels.

Parity status per function is listed in each module header.
"""
from . import objective, lbfgs, convex, certificate, rsvd, mlp  # noqa: F401
