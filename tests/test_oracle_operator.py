"""Pins of the oracle operator against closed forms (CPU only).

The oracle is checked against facts that do not come from its own code:
modified wavenumbers and polynomial exactness of the stencils, ideal-gas
identities, closed-form right-hand sides of parallel base flows, the Fourier
symbol of the linearised equations about a uniform state, and finite
differences of N itself for the complex-step derivative.
"""
import numpy as np
import pytest

import synth
from oracle import operator as op

P, W = op.BC_PERIODIC, op.BC_WALL


# ---------------------------------------------------------------- stencils
@pytest.mark.parametrize("m", [1, 3, 7])
def test_periodic_stencils_modified_wavenumber(m):
    n, L = 32, 5.0
    h = L / n
    x = np.arange(n) * h
    k = 2 * np.pi * m / L
    f = np.sin(k * x)[None, :]
    kt = (1.5 * np.sin(k * h) - 0.3 * np.sin(2 * k * h) + np.sin(3 * k * h) / 30.0) / h
    kh2 = (49.0 / 18 - 3 * np.cos(k * h) + 0.3 * np.cos(2 * k * h) - np.cos(3 * k * h) / 45.0) / h ** 2
    np.testing.assert_allclose(op.d1(f, 0, h, P)[0], kt * np.cos(k * x), atol=1e-12 * k)
    np.testing.assert_allclose(op.d2(f, 0, h, P)[0], -kh2 * np.sin(k * x), atol=1e-11 * k * k)


def _poly_rows(deg, n=14, h=0.37):
    y = np.arange(n) * h + 0.3
    f = (y ** deg)[:, None] * np.ones((1, 3))
    d1 = (deg * y ** (deg - 1) if deg > 0 else 0 * y)[:, None]
    d2 = (deg * (deg - 1) * y ** (deg - 2) if deg > 1 else 0 * y)[:, None]
    return y, f, d1, d2, h


@pytest.mark.parametrize("deg", range(0, 8))
def test_wall_axis_polynomial_exactness(deg):
    y, f, d1x, d2x, h = _poly_rows(deg)
    D1 = op.d1(f, 1, h, W)
    D2 = op.d2(f, 1, h, W)
    n = len(y)
    scale = max(1.0, np.abs(f).max())
    rows6 = slice(3, n - 3)
    if deg <= 6:
        np.testing.assert_allclose(D1[rows6], np.broadcast_to(d1x, f.shape)[rows6], atol=1e-9 * scale)
    if deg <= 7:
        np.testing.assert_allclose(D2[rows6], np.broadcast_to(d2x, f.shape)[rows6], atol=1e-8 * scale)
    for j in (2, n - 3):
        if deg <= 4:
            np.testing.assert_allclose(D1[j], np.broadcast_to(d1x, f.shape)[j], atol=1e-9 * scale)
        if deg <= 5:
            np.testing.assert_allclose(D2[j], np.broadcast_to(d2x, f.shape)[j], atol=1e-8 * scale)
    for j in (1, n - 2):
        if deg <= 2:
            np.testing.assert_allclose(D1[j], np.broadcast_to(d1x, f.shape)[j], atol=1e-9 * scale)
        if deg <= 3:
            np.testing.assert_allclose(D2[j], np.broadcast_to(d2x, f.shape)[j], atol=1e-8 * scale)
    # wall rows are never updated
    assert np.all(D1[0] == 0) and np.all(D1[-1] == 0)


def test_wall_axis_orders_are_tight():
    # the 6th-order rows are not exact for degree 7 (D1): the pin above is tight
    y, f, d1x, _, h = _poly_rows(7)
    D1 = op.d1(f, 1, h, W)
    assert np.abs(D1[3:-3] - d1x[3:-3]).max() > 1e-6


# ---------------------------------------------------------- thermodynamics
@pytest.mark.parametrize("mach", [0.1, 0.3, 0.5, 0.9])
def test_reference_state(mach):
    prob = synth.mixing_layer_2d(8, 8, mach, 500.0)
    c = op.Constants(prob)
    p = np.array(1.0 / (1.4 * mach ** 2))
    rho = op.density(c, p, np.array(0.0))
    T = op.temperature(c, p, rho)
    assert abs(rho - 1.0) < 1e-15 and abs(T - 1.0) < 1e-14
    assert abs(1.4 * p / rho - 1.0 / mach ** 2) < 1e-12          # c^2 = gamma p / rho
    assert abs(op.viscosity(c, 1.0) - 1.0 / 500.0) < 1e-18
    assert abs(c.cp - 1.0 / (0.4 * mach ** 2)) < 1e-12


def test_thermo_partials_closed_form():
    prob = synth.mixing_layer_2d(8, 8, 0.5, 1000.0)
    c = op.Constants(prob)
    rng = np.random.default_rng(0)
    p = c.p_ref * (1 + 0.3 * rng.random(5))
    s = 0.5 * rng.standard_normal(5)
    h = 1e-30
    rho = op.density(c, p, s)
    T = op.temperature(c, p, rho)
    drho_dp = np.imag(op.density(c, p + 1j * h, s)) / h
    drho_ds = np.imag(op.density(c, p, s + 1j * h)) / h
    T_of = lambda pp, ss: op.temperature(c, pp, op.density(c, pp, ss))
    dT_dp = np.imag(T_of(p + 1j * h, s)) / h
    dT_ds = np.imag(T_of(p, s + 1j * h)) / h
    np.testing.assert_allclose(drho_dp, rho / (c.gamma * p), rtol=1e-13)
    np.testing.assert_allclose(drho_ds, -rho / c.cp, rtol=1e-13)
    np.testing.assert_allclose(dT_dp, T / p * (1 - 1 / c.gamma), rtol=1e-13)
    np.testing.assert_allclose(dT_ds, T / c.cp, rtol=1e-13)
    Tq = 0.7 + rng.random(5)
    dmu = np.imag(op.viscosity(c, Tq + 1j * h)) / h
    np.testing.assert_allclose(op.dviscosity(c, Tq), dmu, rtol=1e-13)


# ------------------------------------------------------ N(q) closed forms
@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_state_is_steady(ndim):
    prob = (synth.mixing_layer_2d(12, 11, 0.4, 800.0) if ndim == 2
            else synth.mixing_layer_3d(8, 9, 8, 0.4, 800.0))
    q = np.zeros(prob.shape)
    q[0] = synth.base_pressure(prob) * 1.3
    q[1] = 0.7
    q[-1] = 0.2
    assert np.abs(op.rhs(prob, q)).max() < 1e-12


@pytest.mark.parametrize("ndim", [2, 3])
def test_inviscid_parallel_flow_is_steady(ndim):
    prob = (synth.mixing_layer_2d(12, 31, 0.5, 0.0) if ndim == 2
            else synth.mixing_layer_3d(8, 17, 8, 0.5, 0.0))
    assert np.abs(op.rhs(prob, synth.base_flow(prob))).max() < 1e-13


def test_viscous_tanh_closed_form():
    # rho = T = 1, v = 0, uniform p and s: only shear terms survive
    prob = synth.mixing_layer_2d(12, 31, 0.3, 500.0)
    q0 = synth.base_flow(prob)
    c = op.Constants(prob)
    h = op.spacings(prob)
    u = q0[1]
    Du = op.d1(u, 1, h[1], W)
    D2u = op.d2(u, 1, h[1], W)
    N = op.rhs(prob, q0)
    mu0 = 1.0 / 500.0
    m = op.interior_mask(prob)
    np.testing.assert_allclose(N[1], mu0 * D2u * m, atol=1e-15)
    assert np.abs(N[2]).max() < 1e-15
    np.testing.assert_allclose(N[0], (c.gamma - 1) * mu0 * Du ** 2 * m, atol=1e-15)
    np.testing.assert_allclose(N[3], mu0 * Du ** 2 * m, atol=1e-15)


# --------------------------------------------------------------- Jv checks
@pytest.mark.parametrize("ndim", [2, 3])
def test_cstep_matches_central_difference(ndim):
    prob = (synth.mixing_layer_2d(12, 13, 0.3, 500.0) if ndim == 2
            else synth.mixing_layer_3d(8, 11, 8, 0.5, 1000.0))
    q0 = synth.random_base(prob, 3)
    v = synth.random_vector(prob, 4)
    y = op.jv_cstep(prob, q0, v)
    e = 1e-5
    vp = op.project(prob, v)
    yc = (op.rhs(prob, q0 + e * vp) - op.rhs(prob, q0 - e * vp)) / (2 * e)
    assert np.linalg.norm(y - yc) / np.linalg.norm(y) < 1e-8


def test_frechet_quotient_error_bound():
    prob = synth.config0()
    q0 = synth.base_flow(prob)
    v = synth.random_vector(prob, 0)
    v = v / np.linalg.norm(v)
    y = op.jv_cstep(prob, q0, v)
    yf = op.jv_frechet(prob, q0, v)
    rel = np.linalg.norm(yf - y) / np.linalg.norm(y)
    assert 1e-12 < rel < 1e-6        # first-order quotient with eps = sqrt(eps_m)


def test_linearity_and_projection():
    prob = synth.mixing_layer_2d(12, 13, 0.3, 500.0)
    q0 = synth.random_base(prob, 5)
    v = synth.random_vector(prob, 6)
    w = synth.random_vector(prob, 7)
    a, b = 0.7, -1.9
    lhs = op.jv_cstep(prob, q0, a * v + b * w)
    rhs_ = a * op.jv_cstep(prob, q0, v) + b * op.jv_cstep(prob, q0, w)
    assert np.linalg.norm(lhs - rhs_) / np.linalg.norm(lhs) < 1e-13
    # wall entries of the input are ignored and those of the output are zero
    v2 = v.copy()
    v2[:, 0, :] = 5.0
    y2 = op.jv_cstep(prob, q0, v2)
    assert np.array_equal(y2, op.jv_cstep(prob, q0, v))
    assert np.all(y2[:, 0, :] == 0) and np.all(y2[:, -1, :] == 0)


# ------------------------------------------------ Fourier symbol, uniform flow
def _symbol_eigs(prob, U, viscous):
    """Eigenvalues of the linearised equations about p = p_ref, u = (U,0,0),
    s = 0 on an all-periodic grid, per wave vector (Fourier analysis)."""
    nd = prob.ndim
    c = op.Constants(prob)
    h = op.spacings(prob)
    g, p0 = c.gamma, c.p_ref
    mu0 = c.mu_ref if viscous else 0.0
    lam0 = c.cp * mu0 / c.pr
    Tp, Ts = (1 - 1 / g) / p0, 1.0 / c.cp
    ks = []
    for a in range(nd):
        n = prob.n[a]
        kk = 2 * np.pi * np.fft.fftfreq(n, d=h[a])
        kt = (1.5 * np.sin(kk * h[a]) - 0.3 * np.sin(2 * kk * h[a]) + np.sin(3 * kk * h[a]) / 30) / h[a]
        k2 = (49 / 18 - 3 * np.cos(kk * h[a]) + 0.3 * np.cos(2 * kk * h[a]) - np.cos(3 * kk * h[a]) / 45) / h[a] ** 2
        ks.append((kt, k2))
    out = []
    import itertools
    for idx in itertools.product(*[range(prob.n[a]) for a in range(nd)]):
        kt = np.array([ks[a][0][idx[a]] for a in range(nd)])
        k2 = np.array([ks[a][1][idx[a]] for a in range(nd)])
        nv = nd + 2
        A = np.zeros((nv, nv), complex)
        adv = -1j * U * kt[0]
        for r in range(nv):
            A[r, r] += adv
        for i in range(nd):
            A[0, 1 + i] += -g * p0 * 1j * kt[i]
            A[1 + i, 0] += -1j * kt[i]                       # rho0 = 1
            A[1 + i, 1 + i] += -mu0 * k2.sum() - mu0 / 3 * k2[i]
            for j in range(nd):
                if j != i:
                    A[1 + i, 1 + j] += -mu0 / 3 * kt[i] * kt[j]
        q = -lam0 * k2.sum()                                 # Q' = q (Tp p' + Ts s')
        A[0, 0] += (g - 1) * q * Tp
        A[0, nv - 1] += (g - 1) * q * Ts
        A[nv - 1, 0] += q * Tp
        A[nv - 1, nv - 1] += q * Ts
        out.extend(np.linalg.eigvals(A))
    return np.array(out)


@pytest.mark.parametrize("ndim,viscous", [(2, False), (2, True), (3, False), (3, True)])
def test_uniform_flow_spectrum_equals_fourier_symbol(ndim, viscous):
    re = 50.0 if viscous else 0.0
    if ndim == 2:
        prob = synth.mixing_layer_2d(12, 10, 0.5, re, lx=7.0, ly=6.0, bc_y=P)
    else:
        prob = synth.mixing_layer_3d(7, 6, 6, 0.5, re, lx=5.0, ly=4.0, lz=4.5, bc_y=P)
    U = 0.7
    q0 = np.zeros(prob.shape)
    q0[0] = synth.base_pressure(prob)
    q0[1] = U
    J = op.dense_jacobian(prob, q0)
    lam = np.linalg.eigvals(J)
    sym = _symbol_eigs(prob, U, viscous)
    assert len(sym) == len(lam)
    scale = np.abs(sym).max()
    # every dense eigenvalue has a symbol eigenvalue next to it and vice versa
    d1 = np.abs(lam[:, None] - sym[None, :]).min(axis=1)
    d2 = np.abs(sym[:, None] - lam[None, :]).min(axis=1)
    assert d1.max() < 1e-9 * scale and d2.max() < 1e-9 * scale
    if not viscous:
        # textbook acoustics: -i U kx and -i U kx +- i c |k| with c = 1/M
        assert np.abs(lam.real).max() < 1e-9 * scale


def test_sparse_jacobian_equals_dense():
    prob = synth.mixing_layer_2d(16, 14, 0.3, 500.0)
    q0 = synth.random_base(prob, 1)
    S = op.sparse_jacobian(prob, q0).toarray()
    J = op.dense_jacobian(prob, q0, interior_only=False)
    assert np.array_equal(S, J)
