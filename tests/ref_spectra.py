"""Leading eigenvalues of the oracle's operator under the Cayley transform
(test helper; CPU only).

The oracle's sparse Jacobian (coloured complex-step probing) restricted to
the interior DOFs, a sparse LU of J - sigma I (SuperLU), and ARPACK's
implicitly restarted Arnoldi on C = (J - sigma I)^{-1} (J - mu I) for the
eigenvalues of largest |theta| (eq. cayley_transform), back-transformed by
lambda = (sigma theta - mu)/(theta - 1).  Library routines on the oracle's
operator only: no GPU code.  For grids where the dense Jacobian is out of
reach; on small grids tests/test_oracle_solvers.py checks it against the
dense LAPACK spectrum.  Only eigenvalues separated from the |theta| ~ 1 ring
are reliable (ring members differ by ~1e-5 in |theta| and ARPACK settles on
any of them).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as ssl

from oracle import operator as op


def cayley_leading(prob, q0, k, sigma=0.2, mu=-0.2, tol=1e-14, ncv=None, seed=0):
    """(lam, theta) of the k eigenvalues of C with largest |theta|, largest
    first."""
    S = op.sparse_jacobian(prob, q0)
    idx = op.interior_index(prob)
    A = S[idx][:, idx].tocsc()
    n = A.shape[0]
    lu = ssl.splu((A - sigma * sp.identity(n, format="csc")).tocsc())
    C = ssl.LinearOperator((n, n), matvec=lambda v: lu.solve(A @ v - mu * v), dtype=np.float64)
    v0 = np.random.default_rng(seed).standard_normal(n)
    th = ssl.eigs(C, k=k, which="LM", tol=tol, ncv=ncv or max(2 * k + 1, 40), v0=v0,
                  return_eigenvectors=False, maxiter=100000)
    th = th[np.argsort(-np.abs(th), kind="stable")]
    lam = (sigma * th - mu) / (th - 1.0)
    return lam, th


def mode_leading(prob, q0, k=1, sigma=0.25, n=4):
    """Eigenvalues of the x-Fourier block A_k of the oracle's operator
    (oracle/modes.py; bases uniform along x) nearest sigma, by ARPACK in
    shift-invert mode on the sparse banded block, largest real part first.
    Grid-size independent in cost along x, so it serves full-size 2D grids."""
    from oracle import modes
    A = modes.mode_matrix(prob, q0, k, sparse=True)
    lam = ssl.eigs(A.tocsc(), k=n, sigma=sigma, which="LM", tol=1e-14, return_eigenvectors=False,
                   v0=np.ones(A.shape[0], dtype=complex))
    return lam[np.argsort(-lam.real, kind="stable")]
