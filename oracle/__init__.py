"""Plain FP64 CPU oracle of the FD-Helmholtz ORAS-FGMRES solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path: the only common module
is ``inputs`` (seeded velocity models and sources, no solver arithmetic).

What it computes (citations are to the paper, Dolean et al., EAGE 2021,
arXiv 2103.14921):
  * operator.py  -- the 27-point mixed-grid FD discretisation of the Helmholtz
                    equation (eq. eqh / eq1, FD-vs-FE section) with PML on the
                    sides and bottom and a homogeneous Dirichlet top; the
                    least-squares dispersion fit of the stencil weights.
  * dd.py        -- the overlapping box decomposition, Boolean restriction R_i,
                    Boolean partition of unity D_i, local operators A_i with
                    absorbing (Robin) interface conditions, banded-LU local
                    solves and the one-level ORAS preconditioner (eq. oras).
  * coarse.py    -- the coarse space Z (trilinear at 2h), E = Z^T A Z, the
                    coarse one-level ORAS and the fixed 10-iteration coarse
                    GMRES, and the two-level preconditioner (eq. 2lvl).
  * krylov.py    -- right-preconditioned flexible GMRES with CGS2 and complex
                    Givens rotations (GMRES of the domain-decomposition
                    section).
  * analytic.py  -- closed-form Green's functions (homogeneous medium, image
                    source, linear velocity gradient) used as pins.
  * solve.py     -- the whole solve for many right-hand sides.

Every function that has no independent pin says "parity unpinned" in its
docstring; none do at present.
"""
