"""Restarted GMRES with classical Gram-Schmidt applied twice (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Section "Iterative solvers": the Cayley system (eq. cayley_arnoldi) is solved
by restarted GMRES (Saad & Schultz 1986).  The paper leaves the variant open;
this follows the plain textbook method:

  * initial guess x0 (zero by default), residual relative to ||b||_2;
  * Arnoldi with CGS2: h = V^T w; w -= V h; h2 = V^T w; w -= V h2; h += h2;
  * Givens rotations on the (j+1) x j Hessenberg matrix, residual estimate
    |g_{j+1}|;
  * right preconditioning x = M^{-1} u, in the flexible form (the
    preconditioned directions Z are stored) so that an inexact or
    lower-precision M^{-1} is allowed;
  * after each cycle the true residual b - A x is recomputed and the method
    restarts unless it meets the tolerance or the matvec budget is spent.

With dtype=float32 every vector and every vector operation is single
precision (the inner solver of the precision form); the (m+1) x m least
squares problem is kept in double precision.
"""
from __future__ import annotations

import math

import numpy as np


def givens(a, b):
    """Rotation (c, s) with [c s; -s c] [a; b] = [r; 0], r = hypot(a, b)."""
    if b == 0.0:
        return 1.0, 0.0
    r = math.hypot(a, b)
    return a / r, b / r


def gmres(apply_A, b, x0=None, restart=40, tol=1e-12, max_matvec=10 ** 6,
          precond=None, breakdown_tol=1e-14, record=False, dtype=np.float64):
    """Solve A x = b.  Returns (x, info).

    info: iters (Arnoldi steps), matvecs (applications of A, including the
    residual ones), cycles, relres (true ||b - A x|| / ||b||), converged,
    breakdown, history (residual estimates if record)."""
    b = np.asarray(b, dtype=dtype).ravel()
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n, dtype) if x0 is None else np.array(x0, dtype=dtype).ravel()
    info = dict(iters=0, matvecs=0, cycles=0, relres=0.0, converged=False,
                breakdown=False, history=[])
    if bnorm == 0.0:
        info.update(converged=True)
        return np.zeros(n, dtype), info
    M = (lambda v: v) if precond is None else precond
    m = restart
    while True:
        if x0 is None and info["cycles"] == 0:
            r = b.copy()
        else:
            r = b - apply_A(x)
            info["matvecs"] += 1
        beta = float(np.linalg.norm(r))
        info["relres"] = beta / bnorm
        if beta <= tol * bnorm:
            info["converged"] = True
            return x, info
        if info["matvecs"] >= max_matvec:
            return x, info
        V = np.zeros((n, m + 1), dtype)
        Z = np.zeros((n, m), dtype)
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        jdone = 0
        stop = False
        for j in range(m):
            Z[:, j] = M(V[:, j])
            w = apply_A(Z[:, j])
            info["matvecs"] += 1
            info["iters"] += 1
            wnorm0 = float(np.linalg.norm(w))
            # CGS2
            h = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            hnext = float(np.linalg.norm(w))
            H[:j + 1, j] = h
            H[j + 1, j] = hnext
            # previous rotations on column j
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            jdone = j + 1
            if record:
                info["history"].append(abs(g[j + 1]) / bnorm)
            if hnext <= breakdown_tol * wnorm0:
                info["breakdown"] = True
                stop = True
                break
            V[:, j + 1] = w / hnext
            if abs(g[j + 1]) <= tol * bnorm or info["matvecs"] >= max_matvec:
                stop = True
                break
        # least squares: R y = g
        R = H[:jdone, :jdone]
        y = np.zeros(jdone)
        for i in range(jdone - 1, -1, -1):
            y[i] = (g[i] - R[i, i + 1:jdone] @ y[i + 1:]) / R[i, i]
        x = x + Z[:, :jdone] @ y.astype(dtype)
        info["cycles"] += 1
        # the true residual is recomputed at the top of the loop (also after a
        # breakdown, where the Krylov space held the exact solution)
        x0 = x


def lgmres(apply_A, b, x0=None, inner_m=30, outer_k=3, tol=1e-12, max_matvec=10 ** 6,
           precond=None, breakdown_tol=1e-14, dtype=np.float64):
    """LGMRES(m, k) (Section "Iterative solvers": GMRES whose restart cycles
    are augmented with error approximations, after Baker, Jessup & Manteuffel).

    Each cycle builds, from the current residual r, the space spanned by m
    Krylov directions M^{-1} v_1 .. M^{-1} v_m followed by the stored
    corrections of the previous cycles, newest first (at most k of them,
    fewer in the first cycles).  The Arnoldi process runs over this sequence
    of directions d_j in the flexible form: w = A d_j is orthogonalised by CGS2
    against v_1 .. v_j, giving column j of the Hessenberg matrix and v_{j+1};
    the iterate becomes x + D y with y the least-squares solution, and the
    correction D y is stored as the newest augmentation vector.  Its image
    A D y is not recomputed: it equals r_old - r_new, the difference of the
    true residuals at the start of consecutive cycles, so an augmentation
    step costs no operator product.  With k = 0 the method is GMRES(m).
    Returns (x, info) as gmres does."""
    b = np.asarray(b, dtype=dtype).ravel()
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n, dtype) if x0 is None else np.array(x0, dtype=dtype).ravel()
    info = dict(iters=0, matvecs=0, cycles=0, relres=0.0, converged=False, breakdown=False)
    if bnorm == 0.0:
        info.update(converged=True)
        return np.zeros(n, dtype), info
    M = (lambda v: v) if precond is None else precond
    aug = []                      # stored corrections, newest first
    aug_A = []                    # their images under A
    first = x0 is None
    r_prev = None
    while True:
        if first:
            r = b.copy()
            first = False
        else:
            r = b - apply_A(x)
            info["matvecs"] += 1
        if r_prev is not None and outer_k > 0:
            aug_A = [r_prev - r] + aug_A[:outer_k - 1]
        beta = float(np.linalg.norm(r))
        info["relres"] = beta / bnorm
        if beta <= tol * bnorm:
            info["converged"] = True
            return x, info
        if info["matvecs"] >= max_matvec:
            return x, info
        mt = inner_m + len(aug)
        V = np.zeros((n, mt + 1), dtype)
        D = np.zeros((n, mt), dtype)
        H = np.zeros((mt + 1, mt))
        cs = np.zeros(mt)
        sn = np.zeros(mt)
        g = np.zeros(mt + 1)
        g[0] = beta
        V[:, 0] = r / beta
        jdone = 0
        for j in range(mt):
            if j < inner_m:
                D[:, j] = M(V[:, j])
                w = apply_A(D[:, j])
                info["matvecs"] += 1
            else:
                D[:, j] = aug[j - inner_m]
                w = aug_A[j - inner_m].copy()
            info["iters"] += 1
            wnorm0 = float(np.linalg.norm(w))
            h = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            hnext = float(np.linalg.norm(w))
            H[:j + 1, j] = h
            H[j + 1, j] = hnext
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            jdone = j + 1
            if hnext <= breakdown_tol * wnorm0:
                info["breakdown"] = True
                break
            V[:, j + 1] = w / hnext
            if abs(g[j + 1]) <= tol * bnorm or info["matvecs"] >= max_matvec:
                break
        R = H[:jdone, :jdone]
        y = np.zeros(jdone)
        for i in range(jdone - 1, -1, -1):
            y[i] = (g[i] - R[i, i + 1:jdone] @ y[i + 1:]) / R[i, i]
        dx = D[:, :jdone] @ y.astype(dtype)
        x = x + dx
        info["cycles"] += 1
        if outer_k > 0:
            aug = [dx] + aug[:outer_k - 1]
            r_prev = r
