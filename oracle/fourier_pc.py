"""Mean-flow preconditioner (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Section "Preconditioning" builds the preconditioner from the operator itself
(a local block-Jacobi scheme), and the Conclusions point to a cheaper
approximate operator as the way to a better one.  This preconditioner keeps
the full operator but of an approximate base state: the base averaged over
the periodic directions (x, and z in 3D), q_bar(y) = mean over x, z of
q0(x, y, z).  For that base the discrete operator commutes with shifts along
the periodic axes, so it is block diagonal in their Fourier modes, each block
banded in y; the library solves it mode by mode.  Here it is the plain
definition:

    M(s) = P (J(q_bar) - s I) P on the interior DOFs,   z = M(s)^{-1} r,

with a dense Jacobian and a dense solve.  For bases that do not vary along
the periodic axes (every 2D workload) q_bar = q0 and M(s) = J - s I exactly.
"""
from __future__ import annotations

import numpy as np

from . import operator as opr


def mean_base(prob, q0):
    """q0 averaged over the periodic axes (x, and z in 3D), broadcast back
    to the grid: a base state that depends on y only."""
    q0 = np.asarray(q0, dtype=np.float64)
    axes = (-1,) if prob.ndim == 2 else (-1, -3)
    m = q0.mean(axis=axes, keepdims=True)
    return np.broadcast_to(m, q0.shape).copy()


def operator_matrix(prob, q0, shift):
    """Dense M(s) = J(q_bar) - s I on the interior DOFs."""
    J = opr.dense_jacobian(prob, mean_base(prob, q0))
    return J - shift * np.eye(J.shape[0])


def apply(prob, q0, shift, r, M=None):
    """z = M(s)^{-1} r on the interior, 0 on the wall rows."""
    if M is None:
        M = operator_matrix(prob, q0, shift)
    idx = opr.interior_index(prob)
    rv = np.asarray(r, dtype=np.float64).ravel()
    z = np.zeros(prob.ndof)
    z[idx] = np.linalg.solve(M, rv[idx])
    return z.reshape(prob.shape)
