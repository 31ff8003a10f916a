"""Plain FP64 CPU oracle for the randomized small-block Lanczos null-space method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding or the autograd wrapper) may import, call, link or execute
anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it is written from the paper (Kressner & Shao, "On a randomized
small-block Lanczos method for large-scale null space computations") with
NumPy/SciPy primitives only, favouring obviously-correct code over speed.

Modules
  exact     -- exact null spaces (closed forms, dense SVD) and principal angles
  operator  -- B = A^T A + eps D applied matrix-free (Sec. 1.2)
  lanczos   -- Algorithm 1 (full reorthogonalisation) and Algorithm 2
               (thick restart, W-recurrence partial reorthogonalisation)
  refine    -- Rayleigh-Ritz with the unperturbed A^T A (Remark after Alg. 1)
               followed by a range-restricted CG projection onto null(A)
  backward  -- gradient of a loss on the null projector w.r.t. A's nonzeros

Pinned by tests/test_oracle_*.py against closed forms, invariants, bounds the
paper proves, brute force on tiny inputs and the values the paper prints for
its worked example (the null space dimensions plain block Lanczos reports on
the diagonal matrix of Sec. 1, its first table).  Parity unpinned: iteration
and matvec counts of the method itself (they depend on rounding order and on
random draws the paper does not print).
"""
