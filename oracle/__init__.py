"""FP64 CPU oracle for the MDC / Marchenko / LSQR path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may use it.  It shares no code with the HIP library (no kernels,
headers, helpers or tables); both sides only draw their seeded inputs from
`paper_2011_11120_amd.synth`, which holds none of the method's arithmetic.

Modules
  mdc        -- Eq.2-4 (Theory): orthogonal real DFT with truncation, the
                per-frequency kernel product and its conjugate transpose,
                zero-padded inverse; plus the time-domain definition (Eq.1)
                as brute-force circular sums for tiny inputs.
  marchenko  -- Eq.5 (receiver-side redatuming): the 2x2 block operator with
                the time-space window, its adjoint, the data vector, and the
                Neumann series (forward-only scheme).
  lsqr       -- LSQR (Paige & Saunders 1982) with fixed iteration count and
                CGLS (the paper's solver, Applications section) as cross-check.
  power      -- power iteration for the spectral norm of a kernel slice.

Every function is pinned by `tests/test_oracle_*.py` against something other
than itself (brute force, closed forms, numpy/scipy routines, invariants).
"""
