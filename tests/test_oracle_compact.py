"""Pins of the oracle's compact first derivative and the compact operator (CPU).

The compact scheme (Lele's tridiagonal 6th-order first derivative, 4th-order
Pade rows next to a wall, 3rd-order one-sided rows at a wall) is checked
against facts that do not come from its code:
* its Fourier symbol: inserting e^{ikx} into the scheme gives
  k' h = (a sin kh + (b/2) sin 2kh) / (1 + 2 alpha cos kh);
* 6th-order convergence on a periodic grid, and 3rd order (the closure's)
  with walls; exactness for cubics with walls (every row is exact for them)
  and inexactness for a quartic at the wall row (the closure is 3rd order);
* the compact operator N(q) converges to the independent spectral
  restatement of the equations at 6th order, closer than the explicit one;
* planted mistakes in a copy of the scheme are caught.
"""
import numpy as np
import pytest

import synth
from oracle import operator as op
from spectral_ref import rhs_spectral, smooth_state

P, W = synth.BC_PERIODIC, synth.BC_WALL
ALPHA, A, B = 1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0


def symbol(kh):
    return (A * np.sin(kh) + 0.5 * B * np.sin(2 * kh)) / (1.0 + 2.0 * ALPHA * np.cos(kh))


@pytest.mark.parametrize("n", [32, 27])
def test_fourier_symbol(n):
    L = 2 * np.pi
    h = L / n
    x = np.arange(n) * h
    for k in (1, 3, 7, n // 2 - 1):
        f = np.stack([np.sin(k * x), np.cos(k * x)])
        d = op.d1_compact(f, 0, h, P)
        kp = symbol(k * h) / h
        np.testing.assert_allclose(d[0], kp * np.cos(k * x), atol=1e-12 * max(1.0, kp))
        np.testing.assert_allclose(d[1], -kp * np.sin(k * x), atol=1e-12 * max(1.0, kp))


def _err_periodic(n):
    L = 2 * np.pi
    h = L / n
    x = np.arange(n) * h
    f = np.exp(np.sin(x))
    return np.abs(op.d1_compact(f, 0, h, P) - np.cos(x) * f).max()


def _err_wall(n):
    y = np.linspace(-1.0, 1.0, n)
    h = y[1] - y[0]
    f = np.exp(np.sin(2 * y))[:, None] * np.ones((1, 3))
    return np.abs(op.d1_compact(f, 1, h, W) - (2 * np.cos(2 * y) * np.exp(np.sin(2 * y)))[:, None]).max()


def test_convergence_orders():
    r6 = _err_periodic(24) / _err_periodic(48)
    assert 50 < r6 < 80, r6                       # 2^6 = 64
    r3 = _err_wall(41) / _err_wall(81)
    assert 6 < r3 < 12, r3                        # closure order 3: 2^3 = 8


def test_walls_exact_for_cubics_not_quartics():
    ny = 17
    y = np.linspace(-1.5, 2.0, ny)
    h = y[1] - y[0]
    f = (y ** 3 - 2 * y)[:, None] * np.ones((1, 2))
    np.testing.assert_allclose(op.d1_compact(f, 1, h, W), (3 * y ** 2 - 2)[:, None] * np.ones((1, 2)),
                               rtol=0, atol=1e-12)
    g = (y ** 4)[:, None]
    assert abs(op.d1_compact(g, 1, h, W)[0, 0] - 4 * y[0] ** 3) > 1e-3


def _prob(n, scheme):
    return synth.Problem(ndim=2, n=(n, n, 1), length=(2 * np.pi, 2.6 * np.pi, 1.0), mach=0.5, re=20.0,
                         bc=(P, P, P), scheme=scheme)


def _op_err(n, scheme, linear):
    prob = _prob(n, scheme)
    q0 = smooth_state(prob, 0)
    if linear:
        v = smooth_state(prob, 1) - q0
        a = op.jv_cstep(prob, q0, v)
        b = np.imag(rhs_spectral(prob, q0 + 1e-30j * v)) / 1e-30
    else:
        a, b = op.rhs(prob, q0), rhs_spectral(prob, q0).real
    return np.array([np.abs(a[k] - b[k]).max() / np.abs(b[k]).max() for k in range(prob.nv)])


@pytest.mark.parametrize("linear", [False, True], ids=["N", "Jv"])
def test_compact_operator_converges_to_spectral_reference(linear):
    c64, c128 = _op_err(64, 1, linear), _op_err(128, 1, linear)
    e128 = _op_err(128, 0, linear)
    ratio = c64 / c128
    print("\ncompact errors", c64, "->", c128, "ratios", ratio, "explicit at 128", e128)
    assert np.all(ratio > 30) and np.all(ratio < 100)
    # the 2nd-derivative (heat, viscous) parts are explicit in both schemes,
    # so the gain is in the components the wave terms dominate (u, v), and
    # no component gets worse
    assert np.all(c128 < 1.1 * e128)
    assert np.min(c128 / e128) < 0.2


@pytest.mark.parametrize("what", ["alpha", "b", "closure"])
def test_planted_mistake_is_caught(what, monkeypatch):
    good = op.compact_matrices

    def bad(n, periodic):
        A_, B_ = good(n, periodic)
        if what == "alpha":
            A_ = A_ + np.diag(np.full(n - 1, 0.01), 1)
        elif what == "b":
            B_ = B_.copy()
            B_[5, 7] *= 1.05
        else:
            if periodic:
                return A_, B_
            B_ = B_.copy()
            B_[0, 2] = 0.4
        return A_, B_

    monkeypatch.setattr(op, "compact_matrices", bad)
    caught = False
    try:
        test_fourier_symbol(32)
        test_walls_exact_for_cubics_not_quartics()
        test_convergence_orders()
    except AssertionError:
        caught = True
    assert caught


@pytest.mark.slow
def test_compact_resolves_the_kh_mode_at_lower_resolution():
    """Temporal mixing layer (M 0.5, Re 1000, alpha 0.4 box): the leading
    (Kelvin-Helmholtz) eigenvalue of the compact operator on a 32 x 30 grid
    is at least twice as close to the resolved value (explicit operator on
    192 x 190, from its x-Fourier block) as the explicit operator's on the
    same 32 x 30 grid."""
    import sys
    from ref_spectra import mode_leading
    fine = synth.mixing_layer_2d(192, 190, 0.5, 1000.0)
    ref = mode_leading(fine, synth.base_flow(fine))[0].real
    pe = synth.mixing_layer_2d(32, 30, 0.5, 1000.0)
    lam_e = mode_leading(pe, synth.base_flow(pe))[0].real
    pc = synth.mixing_layer_2d(32, 30, 0.5, 1000.0, scheme=synth.SCHEME_COMPACT)
    ev = np.linalg.eigvals(op.dense_jacobian(pc, synth.base_flow(pc)))
    lam_c = ev[np.argmax(ev.real)].real
    print("\nresolved %.6f  explicit %.6f  compact %.6f" % (ref, lam_e, lam_c), file=sys.stderr)
    assert abs(lam_c - ref) * 2 < abs(lam_e - ref)
