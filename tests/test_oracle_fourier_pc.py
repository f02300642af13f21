"""Pins of the oracle's mean-flow preconditioner (CPU).

The preconditioner is the operator of the base state averaged over the
periodic axes, M(s) = P (J(q_bar) - s I) P.  Checked against facts that do
not come from its code: the averaged base does not vary along the periodic
axes and keeps their means; for that base the operator commutes with the
periodic shifts (so it decouples into Fourier modes, each coupling only
y-rows within the stencil reach: the structure the GPU solver relies on);
for a base that does not vary along x it is the operator itself, so
preconditioned GMRES converges in one step; on a varying base it still
cuts the iteration count."""
import numpy as np
import pytest

import synth
from oracle import fourier_pc as fpc
from oracle import krylov
from oracle import operator as op


def test_mean_base_is_homogeneous_and_keeps_the_means():
    prob = synth.mixing_layer_3d(8, 9, 7, 0.5, 1000.0)
    q0 = synth.random_base(prob, 5)
    qb = fpc.mean_base(prob, q0)
    assert np.array_equal(qb, np.roll(qb, 3, axis=-1))          # x
    assert np.array_equal(qb, np.roll(qb, 2, axis=-3))          # z
    np.testing.assert_allclose(qb.sum(axis=(-1, -3)), q0.sum(axis=(-1, -3)), rtol=1e-14)
    # a base that does not vary along x and z is returned unchanged
    q1 = synth.base_flow(prob)
    np.testing.assert_allclose(fpc.mean_base(prob, q1), q1, rtol=0, atol=1e-15)


@pytest.mark.parametrize("ndim", [2, 3])
def test_mean_flow_operator_commutes_with_periodic_shifts(ndim):
    prob = (synth.mixing_layer_2d(12, 13, 0.5, 800.0) if ndim == 2
            else synth.mixing_layer_3d(9, 11, 8, 0.5, 800.0))
    q0 = synth.random_base(prob, 6)
    qb = fpc.mean_base(prob, q0)
    v = synth.random_vector(prob, 7)
    for axis in ([-1] if ndim == 2 else [-1, -3]):
        lhs = op.jv_cstep(prob, qb, np.roll(v, 1, axis=axis))
        rhs = np.roll(op.jv_cstep(prob, qb, v), 1, axis=axis)
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
    # coupling in y is limited to the stencil reach: a unit perturbation at
    # row j moves rows j-3 .. j+3 only
    e = np.zeros(prob.shape)
    j0 = 6
    e[(1,) + ((0,) if ndim == 3 else ()) + (j0, 0)] = 1.0
    y = op.jv_cstep(prob, qb, e)
    rows = np.nonzero(np.abs(y).sum(axis=tuple(a for a in range(y.ndim) if a != y.ndim - 2)))[0]
    assert rows.min() >= j0 - 3 and rows.max() <= j0 + 3


def test_exact_for_parallel_flow_one_gmres_step():
    prob = synth.mixing_layer_2d(16, 14, 0.5, 1000.0)
    q0 = synth.base_flow(prob)
    sigma = 0.2
    M = fpc.operator_matrix(prob, q0, sigma)
    idx = op.interior_index(prob)
    J = op.dense_jacobian(prob, q0)
    np.testing.assert_allclose(M, J - sigma * np.eye(J.shape[0]), rtol=0, atol=1e-13 * np.abs(J).max())
    b = synth.random_vector(prob, 1, stream=1).ravel()[idx]
    A = lambda x: J @ x - sigma * x   # noqa: E731
    Minv = lambda x: np.linalg.solve(M, x)   # noqa: E731
    x, info = krylov.gmres(A, b, restart=20, tol=1e-10, precond=Minv)
    assert info["converged"] and info["matvecs"] <= 2


def test_cuts_iterations_on_a_varying_base():
    prob = synth.mixing_layer_2d(16, 14, 0.5, 1000.0)
    q0 = synth.base_flow(prob)
    q0 = q0 + 0.02 * synth.random_base(prob, 3) * np.array([0, 1, 1, 0])[:, None, None]
    sigma = 0.2
    J = op.dense_jacobian(prob, q0)
    M = fpc.operator_matrix(prob, q0, sigma)
    idx = op.interior_index(prob)
    b = synth.random_vector(prob, 2, stream=1).ravel()[idx]
    A = lambda x: J @ x - sigma * x   # noqa: E731
    _, plain = krylov.gmres(A, b, restart=40, tol=1e-10, max_matvec=20000)
    xp, pre = krylov.gmres(A, b, restart=40, tol=1e-10, precond=lambda x: np.linalg.solve(M, x))
    assert pre["converged"]
    assert pre["matvecs"] * 10 < plain["matvecs"]
    xs = np.linalg.solve(J - sigma * np.eye(J.shape[0]), b)
    assert np.linalg.norm(xp - xs) / np.linalg.norm(xs) < 1e-8


# ---- x-Fourier blocks of the operator (oracle/modes.py) ----

def test_mode_blocks_map_fourier_perturbations():
    """J applied to Re(e^{i theta_k i} phi_j) is Re(e^{i theta_k i} (A_k phi)_j)
    for a random complex phi (the defining property, checked with the full
    operator on the full grid)."""
    from oracle import modes
    prob = synth.mixing_layer_2d(12, 11, 0.5, 800.0)
    q0 = synth.base_flow(prob)
    nv, ny, nx = prob.nv, prob.n[1], prob.n[0]
    rng = np.random.default_rng(3)
    for k in (0, 1, 5, 6):
        A = modes.mode_matrix(prob, q0, k)
        phi = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
        ph = np.exp(2j * np.pi * k * np.arange(nx) / nx)
        def field(w):
            f = np.zeros(prob.shape, dtype=complex)
            f[:, 1:ny - 1, :] = w.reshape(ny - 2, nv).T[:, :, None] * ph[None, None, :]
            return f
        lhs = op.jv_cstep(prob, q0, field(phi).real)
        rhs = field(A @ phi).real
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max(), k


def test_mode_spectra_union_is_the_dense_spectrum():
    """The union over k of the spectra of A_k is the spectrum of the dense
    Jacobian; A_{Nx-k} = conj(A_k)."""
    from oracle import modes
    prob = synth.mixing_layer_2d(8, 10, 0.4, 600.0)
    q0 = synth.base_flow(prob)
    ev = np.linalg.eigvals(op.dense_jacobian(prob, q0))
    st = modes.stencil(prob, q0)
    parts = [np.linalg.eigvals(modes.mode_matrix(prob, q0, k, st=st)) for k in range(prob.n[0])]
    em = np.concatenate(parts)
    assert len(em) == len(ev)
    scale = np.abs(ev).max()
    for lam in ev:
        assert np.min(np.abs(em - lam)) < 1e-9 * scale
    for lam in em:
        assert np.min(np.abs(ev - lam)) < 1e-9 * scale
    A1 = modes.mode_matrix(prob, q0, 1, st=st)
    A7 = modes.mode_matrix(prob, q0, 7, st=st)
    np.testing.assert_allclose(A7, A1.conj(), rtol=0, atol=1e-14 * np.abs(A1).max())


def test_mode_blocks_refuse_x_varying_bases():
    from oracle import modes
    prob = synth.mixing_layer_2d(8, 10, 0.4, 600.0)
    with pytest.raises(ValueError):
        modes.mode_matrix(prob, synth.random_base(prob, 1), 1)
