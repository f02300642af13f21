"""Implicitly restarted Arnoldi with the Cayley transformation (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Follows Section "Implicitly restarted Arnoldi method", Algorithm 1, with the
Ritz-estimate test of eq. (ritz_estimate), applied to the Cayley operator
C = (J - sigma I)^{-1} (J - mu I) of eq. (cayley_transform).  Readings:

  * real arithmetic: a complex-conjugate pair of shifts is applied as one
    double-shift QR step; the kept dimension k grows by one when the k-th
    and (k+1)-th Ritz values form a conjugate pair, so no pair is split;
  * the p = m - k shifts are the unwanted Ritz values (exact shifts);
  * wanted = largest |theta| (eigenvalues of J with Re lambda > 0 map to
    |theta| > 1 when mu = -sigma);
  * the restart keeps H_k = H_m(1:k,1:k) after the QR steps (the printed
    "H_m Q(1:k,1:k)" is read this way), v_{k+1} = (V_m Q)(:,k+1) and the
    scalar multiplying f_m is Q(m,k) (printed as sigma_k, renamed here to
    avoid the clash with the Cayley sigma);
  * ||H_m|| in the test is the Frobenius norm; eps_m = 2^-52;
  * orthogonalisation is classical Gram-Schmidt applied twice.

The QR steps use the explicit textbook form H - s I = QR, H <- Q^T H Q
(for a pair: (H - s I)(H - conj(s) I) = QR), which is what the implicit
bulge chase computes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

EPS_MACHINE = 2.0 ** -52


def cayley_theta(lam, sigma, mu):
    """theta = (lambda - mu)/(lambda - sigma): eigenvalue of C for an
    eigenvalue lambda of J (eq. cayley_transform)."""
    return (lam - mu) / (lam - sigma)


def cayley_lambda(theta, sigma, mu):
    """Inverse map lambda = (sigma theta - mu)/(theta - 1)."""
    return (sigma * theta - mu) / (theta - 1.0)


def _cgs2(V, w):
    h = V.T @ w
    w = w - V @ h
    h2 = V.T @ w
    w = w - V @ h2
    return w, h + h2


def _sort_wanted(theta):
    """Order Ritz values by decreasing |theta|; conjugate partners adjacent,
    positive imaginary part first."""
    key = np.lexsort((-theta.imag, -theta.real, -np.round(np.abs(theta), 13)))
    return key


def _kept(theta_sorted, nev):
    k = nev
    if k < len(theta_sorted):
        a = theta_sorted[k - 1]
        b = theta_sorted[k]
        if a.imag != 0.0 and b.imag != 0.0 and abs(b - np.conj(a)) <= 1e-12 * max(1.0, abs(a)):
            k += 1
    return k


def _apply_shifts(H, shifts):
    """QR steps with the given shifts (conjugate pairs as one double step).
    Returns (H_new, Q)."""
    m = H.shape[0]
    Q = np.eye(m)
    i = 0
    shifts = list(shifts)
    while i < len(shifts):
        s = shifts[i]
        if abs(s.imag) > 0.0 and i + 1 < len(shifts) and abs(shifts[i + 1] - np.conj(s)) <= 1e-12 * max(1.0, abs(s)):
            Mshift = H @ H - 2.0 * s.real * H + (abs(s) ** 2) * np.eye(m)
            i += 2
        else:
            Mshift = H - s.real * np.eye(m)
            i += 1
        Qj, _ = np.linalg.qr(Mshift)
        H = Qj.T @ H @ Qj
        Q = Q @ Qj
    # H is upper Hessenberg up to rounding; clear the rounding below it
    H = np.triu(H, -1)
    return H, Q


def arnoldi_extend(op, V, H, j0, m):
    """Arnoldi steps j0 .. m-1 (0-based): V[:, j+1], H[:j+2, j]."""
    nops = 0
    for j in range(j0, m):
        w = op(V[:, j])
        nops += 1
        w, h = _cgs2(V[:, :j + 1], w)
        beta = float(np.linalg.norm(w))
        H[:j + 1, j] = h
        H[j + 1, j] = beta
        if beta == 0.0:
            raise RuntimeError("Arnoldi breakdown: invariant subspace found")
        V[:, j + 1] = w / beta
    return nops


def iram(op, v0, nev=6, ncv=30, tol=1e-10, max_restarts=500):
    """Algorithm 1.  op applies the (transformed) operator to a vector.

    Returns dict(theta: wanted Ritz values (nev, complex), Y: their unit
    eigenvectors of H_m, V: basis (n x m), ritz_est, converged, restarts,
    nops, nconv)."""
    v0 = np.asarray(v0, dtype=np.float64).ravel()
    n = v0.size
    m = ncv
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = v0 / np.linalg.norm(v0)
    nops = arnoldi_extend(op, V, H, 0, m)
    restarts = 0
    while True:
        Hm = H[:m, :m]
        theta, Y = sla.eig(Hm)
        order = _sort_wanted(theta)
        theta = theta[order]
        Y = Y[:, order]
        Y = Y / np.linalg.norm(Y, axis=0)
        rnorm = abs(H[m, m - 1])
        est = rnorm * np.abs(Y[m - 1, :])
        hnorm = np.linalg.norm(Hm, "fro")
        ok = est[:nev] <= np.maximum(EPS_MACHINE * hnorm, tol * np.abs(theta[:nev]))
        nconv = int(np.sum(ok))
        if nconv >= nev or restarts >= max_restarts:
            return dict(theta=theta[:nev], Y=Y[:, :nev], V=V[:, :m].copy(),
                        ritz_est=est[:nev], converged=bool(nconv >= nev),
                        restarts=restarts, nops=nops, nconv=nconv,
                        H=Hm.copy(), f_norm=rnorm)
        k = _kept(theta, nev)
        shifts = theta[k:]
        Hs, Q = _apply_shifts(Hm.copy(), shifts)
        beta_hat = Hs[k, k - 1]
        s = Q[m - 1, k - 1]
        VQ = V[:, :m] @ Q
        f_m = H[m, m - 1] * V[:, m]
        f_k = VQ[:, k] * beta_hat + f_m * s
        Hn = np.zeros((m + 1, m))
        Hn[:k, :k] = Hs[:k, :k]
        fk_norm = float(np.linalg.norm(f_k))
        Vn = np.zeros((n, m + 1))
        Vn[:, :k] = VQ[:, :k]
        Vn[:, k] = f_k / fk_norm
        Hn[k, k - 1] = fk_norm
        V, H = Vn, Hn
        nops += arnoldi_extend(op, V, H, k, m)
        restarts += 1


def ritz_pairs(res, sigma=None, mu=None):
    """Ritz vectors x_i = V_m y_i (complex) and, when sigma/mu are given,
    the eigenvalues of J by the inverse Cayley map."""
    X = res["V"] @ res["Y"]
    if sigma is None:
        return res["theta"], X
    return cayley_lambda(res["theta"], sigma, mu), X


def cayley_operator_dense(J, sigma, mu):
    """Exact Cayley application w = (J - sigma I)^{-1}(J - mu I) v by one LU
    factorisation of the dense J - sigma I."""
    n = J.shape[0]
    lu = sla.lu_factor(J - sigma * np.eye(n))
    return lambda v: sla.lu_solve(lu, J @ v - mu * v)
