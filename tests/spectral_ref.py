"""Spectral reference right-hand side on an all-periodic grid (test helper).

An independent restatement of the governing equations (Section "Governing
equations", eq. navier_stokes) in their printed, un-expanded form, used to pin
the oracle's discrete N(q):

* the stress tensor tau_ij = 2 mu (s_ij - s_kk delta_ij / 3) (mu_v = 0) is
  assembled as a field and its divergence d_j tau_ij is taken directly;
* the heat flux divergence d_j(lambda d_j T) is the derivative of the assembled
  flux lambda(T) d_j T;
* the dissipation is Phi = tau_ij s_ij;
* the pressure equation keeps the printed factor p/c_v in front of
  Ds/Dt = (heat + Phi)/(rho T) (with the material derivative on the left and
  the physical sign of the entropy source, as the oracle reads them).

Derivatives are Fourier-spectral (exact for band-limited fields, spectrally
accurate for the smooth periodic fields the tests use), so the oracle's
6th-order finite differences must converge to this at 6th order.  Nothing
here is shared with the oracle: the expanded viscous form, the chain rule for
grad mu and grad lambda and the (gamma - 1) simplification are exactly what
this reference does *not* use.

The derivative operator maps real fields to real fields (the Nyquist mode of
odd derivatives is dropped), so the function is complex-analytic in q and its
complex-step derivative is the exact derivative of this reference.
"""
from __future__ import annotations

import numpy as np


def _dspec_real(f, axis, length):
    """Spectral first derivative of a real field along `axis` (period `length`)."""
    n = f.shape[axis]
    k = 2.0 * np.pi * np.fft.rfftfreq(n, d=length / n)
    if n % 2 == 0:
        k[-1] = 0.0                          # odd derivative: drop the Nyquist mode
    shape = [1] * f.ndim
    shape[axis] = k.size
    F = np.fft.rfft(f, axis=axis)
    return np.fft.irfft(1j * k.reshape(shape) * F, n=n, axis=axis)


def _dspec(f, axis, length):
    """The same derivative applied to the real and imaginary parts separately,
    so that rounding in the (large) real part never leaks into the (tiny)
    imaginary part of a complex-step evaluation."""
    return (_dspec_real(f.real, axis, length)
            + 1j * _dspec_real(f.imag, axis, length))


def rhs_spectral(prob, q):
    """N(q) of the un-expanded equations with spectral derivatives.

    `prob` must be periodic in every axis; q has shape (nv, [Nz,] Ny, Nx)."""
    nd = prob.ndim
    assert all(b == 0 for b in prob.bc[:nd]), "spectral reference needs a periodic grid"
    g = float(prob.gamma)
    mach = float(prob.mach)
    R = 1.0 / (g * mach * mach)              # gas constant, rho_ref = T_ref = 1
    p_ref = R                                # p_ref = rho_ref R T_ref
    cv = R / (g - 1.0)
    cp = cv + R
    mu_ref = 1.0 / prob.re if prob.re > 0 else 0.0
    S = float(prob.sutherland)
    pr = float(prob.pr)

    q = np.asarray(q, dtype=complex)
    p = q[0]
    u = [q[1 + i] for i in range(nd)]
    s = q[nd + 1]

    def D(f, a):
        return _dspec(f, -1 - a, prob.length[a])

    # ideal gas with the entropy measured from the reference state:
    # s = cv ln(p/p_ref) - cp ln(rho/rho_ref)
    rho = np.exp((cv * np.log(p / p_ref) - s) / cp)
    T = p / (rho * R)
    mu = mu_ref * T ** 1.5 * (1.0 + S) / (T + S)          # Sutherland
    lam = cp * mu / pr                                    # Prandtl number
    c2 = g * p / rho                                      # speed of sound squared

    grad_u = [[D(u[i], j) for j in range(nd)] for i in range(nd)]
    sij = [[0.5 * (grad_u[i][j] + grad_u[j][i]) for j in range(nd)] for i in range(nd)]
    skk = sum(sij[k][k] for k in range(nd))
    tau = [[2.0 * mu * (sij[i][j] - (skk / 3.0 if i == j else 0.0)) for j in range(nd)]
           for i in range(nd)]
    div_tau = [sum(D(tau[i][j], j) for j in range(nd)) for i in range(nd)]
    heat = sum(D(lam * D(T, j), j) for j in range(nd))
    phi = sum(tau[i][j] * sij[i][j] for i in range(nd) for j in range(nd))

    Ds_Dt = (heat + phi) / (rho * T)                      # entropy equation
    adv = lambda f: sum(u[j] * D(f, j) for j in range(nd))
    Np = -adv(p) - rho * c2 * skk + (p / cv) * Ds_Dt
    Nu = [-adv(u[i]) - D(p, i) / rho + div_tau[i] / rho for i in range(nd)]
    Ns = -adv(s) + Ds_Dt
    return np.stack([Np] + Nu + [Ns])


def smooth_state(prob, which=0):
    """Smooth periodic fields with O(1) variations of T, shear, non-zero
    divergence and every velocity component active (all wave numbers <= 2)."""
    nd = prob.ndim
    nx, ny, nz = prob.n
    ax = [2 * np.pi * np.arange(prob.n[a]) / prob.n[a] for a in range(nd)]
    if nd == 2:
        Y, X = np.meshgrid(ax[1], ax[0], indexing="ij")
        Z = 0.0 * X
    else:
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    g = float(prob.gamma)
    p_ref = 1.0 / (g * prob.mach ** 2)
    cp = g * p_ref / (g - 1.0)
    ph = 0.7 * which
    q = np.zeros(prob.shape)
    q[0] = p_ref * (1.0 + 0.15 * np.sin(X + 2 * Y + ph) + 0.1 * np.cos(Y - Z))
    q[1] = 0.6 * np.sin(Y + ph) + 0.3 * np.cos(X - Y) + 0.2 * np.sin(Z)
    q[2] = 0.4 * np.cos(X + ph) + 0.2 * np.sin(X + Y + Z)
    if nd == 3:
        q[3] = 0.3 * np.sin(Y + Z + ph) + 0.25 * np.cos(X) * np.cos(Z)
    q[nd + 1] = cp * (0.25 * np.sin(X + ph) * np.cos(Y) + 0.1 * np.cos(2 * Y) + 0.05 * np.sin(X + Z))
    return q
