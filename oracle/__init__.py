"""CPU FP64 oracle for the matrix-free global stability method.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only the tests, the smoke check and the
bench's CPU-baseline leg use it.  It shares no code with the HIP library;
the two meet only at the seeded arrays produced by ``synth``.

Contents (each function cites the passage of the paper it follows):
  operator   -- thermodynamics, FD stencils, the discrete right-hand side
                N(q) of the Navier-Stokes system in (p, u_i, s) form, its
                exact linearisation by complex step, the Frechet quotient
                of eq. (frechet) and a brute-force dense Jacobian.
  krylov     -- restarted GMRES with CGS2 (Section "Iterative solvers").
  arnoldi    -- implicitly restarted Arnoldi (Algorithm 1) with the
                Ritz-estimate test (eq. ritz_estimate) and the Cayley
                transformation (eq. cayley_transform / cayley_arnoldi).
  refine     -- FP64 outer / FP32 inner iterative refinement of the Cayley
                system (an added precision form, not from the paper).
  blockjac   -- block-Jacobi preconditioner (Section "Preconditioning").
  fourier_pc -- mean-flow preconditioner: J of the base averaged over the
                periodic axes, solved exactly (Section "Preconditioning",
                Conclusions).
  modes      -- x-Fourier blocks A_k of J for bases uniform along x, read
                off the operator on a seven-point-long grid (the spectrum
                of J is the union of theirs).
  philox     -- Philox4x32-10 counter-based generator (Salmon et al. 2011)
                plus Box-Muller, for the seeded block noise.
"""
