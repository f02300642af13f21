"""FP64 outer / FP32 inner iterative refinement of the Cayley system (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

An added precision form, not from the paper: the linear system of eq.
(cayley_arnoldi), (J - sigma I) y = b, is solved by classical iterative
refinement.  Each sweep computes the FP64 residual r = b - A y, solves the
correction equation A d = r/||r|| in single precision with restarted GMRES
to a loose inner tolerance, and adds ||r|| d to y in FP64.  The sweeps stop
when ||r|| <= tol ||b|| (true FP64 residual) or after max_outer sweeps.
"""
from __future__ import annotations

import numpy as np

from .krylov import gmres


def ir_solve(apply_A64, apply_A32, b, tol=1e-10, inner_tol=1e-4,
             inner_restart=30, max_outer=10, inner_max_matvec=10 ** 6):
    """Returns (y, info) with info: outer, inner_matvecs, relres, history."""
    b = np.asarray(b, dtype=np.float64).ravel()
    bnorm = float(np.linalg.norm(b))
    y = np.zeros_like(b)
    info = dict(outer=0, inner_matvecs=0, matvecs64=0, relres=0.0,
                converged=False, history=[])
    if bnorm == 0.0:
        info["converged"] = True
        return y, info
    r = b.copy()
    while True:
        rnorm = float(np.linalg.norm(r))
        info["relres"] = rnorm / bnorm
        info["history"].append(rnorm / bnorm)
        if rnorm <= tol * bnorm:
            info["converged"] = True
            return y, info
        if info["outer"] >= max_outer:
            return y, info
        r32 = (r / rnorm).astype(np.float32)
        d, inner = gmres(apply_A32, r32, restart=inner_restart, tol=inner_tol,
                         max_matvec=inner_max_matvec, dtype=np.float32)
        info["inner_matvecs"] += inner["matvecs"]
        y = y + rnorm * d.astype(np.float64)
        r = b - apply_A64(y)
        info["matvecs64"] += 1
        info["outer"] += 1
