"""x-Fourier blocks of the operator for bases uniform along x (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

For a base state that does not vary along the periodic x axis (every 2D
workload: the tanh layer), the discrete operator commutes with shifts along
x.  The perturbation exp(i theta_k i) phi_j (i the x index, theta_k =
2 pi k / Nx) is mapped to exp(i theta_k i) (A_k phi)_j, so the spectrum of J
(Section "Stability analysis") is the union over k of the spectra of the
(Ny-2) nv square matrices

    A_k[(j, v), (j', v')] = sum_{dx=-3..3} J[(v, j, x0 + dx), (v', j', x0)] e^{-i theta_k dx}.

J's coefficients do not depend on x0 and reach three points along x, so they
are read off the operator on a grid of the same spacing that is seven
points long (offsets -3 .. 3 do not alias there), here from the oracle's
coloured-probe sparse Jacobian.  The interior rows j = 1 .. Ny-2 are the
unknowns, in the order u = (j-1) nv + v.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import operator as opr

NARROW = 7   # 2 * reach + 1


def narrow_problem(prob):
    """The problem on a grid of the same x spacing, NARROW points long."""
    nx, ny, nz = prob.n
    lx, ly, lz = prob.length
    return dataclasses.replace(prob, n=(NARROW, ny, nz), length=(lx * NARROW / nx, ly, lz))


def _check(prob, q0):
    if prob.ndim != 2:
        raise ValueError("mode blocks are built for 2D problems")
    q0 = np.asarray(q0, dtype=np.float64)
    if not np.array_equal(q0, np.broadcast_to(q0[..., :1], q0.shape)):
        raise ValueError("the base state varies along x")
    return q0


def stencil(prob, q0):
    """(rows u, columns u', offsets dx, values): the entries
    J[(v, j, dx), (v', j', 0)] with interior j, j'."""
    q0 = _check(prob, q0)
    pn = narrow_problem(prob)
    qn = np.broadcast_to(q0[..., :1], pn.shape).copy()
    S = opr.sparse_jacobian(pn, qn).tocsc()
    nv, ny = prob.nv, prob.n[1]
    # columns: a unit at (v', j', x = 0) of the narrow grid
    vp, jp = np.meshgrid(np.arange(nv), np.arange(1, ny - 1), indexing="ij")
    cols = ((vp * ny + jp) * NARROW).ravel()
    sub = S[:, cols].tocoo()
    r, c, val = sub.row, sub.col, sub.data
    i = r % NARROW
    j = (r // NARROW) % ny
    v = r // (NARROW * ny)
    keep = (j >= 1) & (j <= ny - 2)
    u = (j[keep] - 1) * nv + v[keep]
    up = (jp.ravel()[c[keep]] - 1) * nv + vp.ravel()[c[keep]]
    dx = np.where(i[keep] <= NARROW // 2, i[keep], i[keep] - NARROW)
    return u, up, dx, val[keep]


def mode_matrix(prob, q0, k, sparse=False, st=None):
    """A_k (dense complex array, or scipy CSR with sparse=True); st: a
    precomputed stencil(prob, q0)."""
    import scipy.sparse as sp
    u, up, dx, val = st if st is not None else stencil(prob, q0)
    theta = 2.0 * np.pi * k / prob.n[0]
    n = (prob.n[1] - 2) * prob.nv
    A = sp.coo_matrix((val * np.exp(-1j * theta * dx), (u, up)), shape=(n, n)).tocsr()
    return A if sparse else A.toarray()
