"""Pins of the oracle's y-grid stretching (CPU).

Rows at y = (Ly/2) sinh(beta eta)/sinh(beta) of a uniform eta grid; the
operator's y derivatives follow by the chain rule with the analytic metric.
Checked against facts that do not come from that code:
* beta -> 0 is the uniform grid: the operator (N and Jv, both schemes) at
  beta = 1e-4 differs from the uniform one by O(beta^2) only;
* on the stretched grid D_y and D_yy of tanh(y) converge at 6th order (the
  interior stencils' order in eta) to the exact derivatives;
* the Kelvin-Helmholtz growth rate (M 0.5, Re 1000) on 30 stretched rows is
  far closer to the resolved value (uniform grid of 380 rows) than on 30
  uniform rows, and 60 stretched rows reach it;
* planted mistakes in the metric are caught.
"""
import numpy as np
import pytest

import synth
from oracle import operator as op

C = synth.SCHEME_COMPACT


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("scheme", [synth.SCHEME_EXPLICIT, C], ids=["explicit", "compact"])
def test_tiny_stretch_is_the_uniform_operator(scheme):
    pu = synth.mixing_layer_2d(12, 17, 0.5, 400.0, scheme=scheme)
    ps = synth.mixing_layer_2d(12, 17, 0.5, 400.0, scheme=scheme, stretch=1e-4)
    q0 = synth.random_base(pu, 1)
    v = synth.random_vector(pu, 2)
    n_u, n_s = op.rhs(pu, q0), op.rhs(ps, q0)
    assert 0.0 < _rel(n_s, n_u) < 1e-7
    j_u, j_s = op.jv_cstep(pu, q0, v), op.jv_cstep(ps, q0, v)
    assert 0.0 < _rel(j_s, j_u) < 1e-7
    # a real stretch is a different operator
    p3 = synth.mixing_layer_2d(12, 17, 0.5, 400.0, scheme=scheme, stretch=3.0)
    assert _rel(op.jv_cstep(p3, q0, v), j_u) > 1e-2


def _deriv_errors(ny, beta=3.0):
    p = synth.mixing_layer_2d(8, ny, 0.5, 100.0, stretch=beta)
    y = synth.grid_y(p)
    f = np.tanh(y)[:, None] * np.ones((1, 8))
    sech2 = 1.0 / np.cosh(y) ** 2
    e1 = np.abs(op.deriv(p, f, 1) - sech2[:, None])[3:ny - 3].max()
    e2 = np.abs(op.deriv2(p, f, 1) - (-2.0 * np.tanh(y) * sech2)[:, None])[3:ny - 3].max()
    return e1, e2


def test_stretched_derivatives_sixth_order():
    e33, e65, e129 = _deriv_errors(33), _deriv_errors(65), _deriv_errors(129)
    for k in range(2):
        for a, b in ((e33, e65), (e65, e129)):
            assert 40.0 < a[k] / b[k] < 80.0, (k, a, b)     # 2^6 = 64
    assert e129[0] < 1e-7 and e129[1] < 1e-7


@pytest.mark.parametrize("what", ["sign", "scale", "drop"])
def test_planted_metric_mistakes_are_caught(what, monkeypatch):
    good = op.y_metrics

    def bad(prob):
        iyp, mq = good(prob)
        if what == "sign":
            return iyp, -mq
        if what == "scale":
            return 0.5 * iyp, mq
        return iyp, 0.0 * mq

    monkeypatch.setattr(op, "y_metrics", bad)
    with pytest.raises(AssertionError):
        test_stretched_derivatives_sixth_order()


def test_stretch_needs_walls():
    p = synth.mixing_layer_2d(8, 12, 0.5, 100.0, bc_y=synth.BC_PERIODIC, stretch=2.0)
    with pytest.raises(ValueError):
        op.rhs(p, synth.base_flow(p))


def test_stretched_grid_resolves_the_kh_mode():
    from ref_spectra import mode_leading

    def lead(ny, beta):
        p = synth.mixing_layer_2d(32, ny, 0.5, 1000.0, stretch=beta)
        return mode_leading(p, synth.base_flow(p))[0].real

    ref = lead(380, 0.0)
    e_uniform = abs(lead(30, 0.0) - ref)
    e_stretch = abs(lead(30, 3.0) - ref)
    assert e_stretch * 10.0 < e_uniform, (e_stretch, e_uniform)
    assert abs(lead(60, 3.0) - ref) < 3e-5
