"""Pins of the oracle's iterative parts (GMRES, IRAM, Cayley, IR, block-Jacobi,
Philox) against library routines, invariants and known answers (CPU only)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import arnoldi as ar
from oracle import blockjac as bj
from oracle import krylov as kr
from oracle import operator as op
from oracle import philox
from oracle import refine

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def small():
    prob = synth.mixing_layer_2d(12, 12, 0.3, 500.0)
    q0 = synth.random_base(prob, 11)
    J = op.dense_jacobian(prob, q0)
    return prob, q0, J


@pytest.fixture(scope="module")
def kh24():
    prob = synth.mixing_layer_2d(24, 24, 0.3, 500.0)
    q0 = synth.base_flow(prob)
    J = op.dense_jacobian(prob, q0)
    return prob, q0, J, np.linalg.eigvals(J)


# ------------------------------------------------------------------- GMRES
def test_gmres_matches_direct_solve(small):
    prob, q0, J = small
    n = J.shape[0]
    A = J - 0.2 * np.eye(n)
    b = np.random.default_rng(0).standard_normal(n)
    x, info = kr.gmres(lambda v: A @ v, b, restart=40, tol=1e-12)
    xs = np.linalg.solve(A, b)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1.01e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12 * np.linalg.cond(A)


def test_gmres_residual_monotone_and_restart(small):
    prob, q0, J = small
    n = J.shape[0]
    A = J - 0.2 * np.eye(n)
    b = np.random.default_rng(1).standard_normal(n)
    x, info = kr.gmres(lambda v: A @ v, b, restart=200, tol=1e-10, record=True)
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 1e-15)             # minimal residual within a cycle
    x2, info2 = kr.gmres(lambda v: A @ v, b, restart=25, tol=1e-10)
    assert info2["converged"] and info2["cycles"] > 1
    assert np.linalg.norm(x2 - x) / np.linalg.norm(x) < 1e-8


def test_gmres_exact_preconditioner_one_step(small):
    prob, q0, J = small
    n = J.shape[0]
    A = J - 0.2 * np.eye(n)
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(2).standard_normal(n)
    x, info = kr.gmres(lambda v: A @ v, b, restart=10, tol=1e-10, precond=lambda v: Ainv @ v)
    assert info["converged"] and info["iters"] == 1


def test_gmres_zero_rhs_and_budget(small):
    prob, q0, J = small
    n = J.shape[0]
    x, info = kr.gmres(lambda v: J @ v, np.zeros(n))
    assert info["converged"] and np.all(x == 0) and info["matvecs"] == 0
    b = np.random.default_rng(3).standard_normal(n)
    x, info = kr.gmres(lambda v: J @ v - 0.2 * v, b, restart=5, tol=1e-14, max_matvec=7)
    assert not info["converged"] and info["matvecs"] <= 8


def test_gmres_happy_breakdown_on_eigenvector():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    A = Q @ np.diag(np.arange(1, 31.0)) @ Q.T
    b = Q[:, 3]
    x, info = kr.gmres(lambda v: A @ v, b, restart=10, tol=1e-12)
    assert info["breakdown"] and info["iters"] == 1 and info["converged"]
    np.testing.assert_allclose(x, b / 4.0, atol=1e-14)


def test_gmres_float32_inner(small):
    prob, q0, J = small
    n = J.shape[0]
    A32 = (J - 0.2 * np.eye(n)).astype(np.float32)
    b = np.random.default_rng(5).standard_normal(n).astype(np.float32)
    x, info = kr.gmres(lambda v: A32 @ v, b, restart=30, tol=1e-4, dtype=np.float32)
    assert x.dtype == np.float32 and info["converged"]
    assert np.linalg.norm(b - A32 @ x) <= 2e-4 * np.linalg.norm(b)


# -------------------------------------------------------------------- IRAM
def _known_spectrum_matrix(n=200, seed=0):
    rng = np.random.default_rng(seed)
    lead = [10.0, 8.0 + 3.0j, 8.0 - 3.0j, -7.5, 6.0 + 1.0j, 6.0 - 1.0j]
    rest = 2.0 * rng.random(n - len(lead)) - 1.0
    D = np.zeros((n, n))
    D[0, 0] = 10.0
    D[1:3, 1:3] = [[8.0, 3.0], [-3.0, 8.0]]
    D[3, 3] = -7.5
    D[4:6, 4:6] = [[6.0, 1.0], [-1.0, 6.0]]
    D[6:, 6:] = np.diag(rest)
    S = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    return S @ D @ np.linalg.inv(S), np.array(lead)


def test_iram_known_dominant_eigenvalues():
    A, lead = _known_spectrum_matrix()
    v0 = np.random.default_rng(1).standard_normal(A.shape[0])
    res = ar.iram(lambda v: A @ v, v0, nev=6, ncv=20, tol=1e-12, max_restarts=200)
    assert res["converged"]
    got = res["theta"]
    for lam in lead:
        assert np.min(np.abs(got - lam)) < 1e-9 * 10
    assert np.all(np.abs(np.abs(got[:-1]) - np.abs(got[1:])) >= -1e-12)   # sorted by |theta|


def test_iram_arnoldi_relation_after_restarts():
    A, _ = _known_spectrum_matrix(seed=2)
    n = A.shape[0]
    v0 = np.random.default_rng(3).standard_normal(n)
    res = ar.iram(lambda v: A @ v, v0, nev=4, ncv=12, tol=1e-14, max_restarts=5)
    assert res["restarts"] >= 1
    V, H = res["V"], res["H"]
    m = V.shape[1]
    # A V_m = V_m H_m + f_m e_m^T with ||f_m|| = f_norm, f_m orthogonal to V_m
    R = A @ V - V @ H
    assert np.linalg.norm(R[:, :-1]) < 1e-11 * np.linalg.norm(A)
    assert abs(np.linalg.norm(R[:, -1]) - res["f_norm"]) < 1e-10 * np.linalg.norm(A)
    assert np.linalg.norm(V.T @ V - np.eye(m)) < 1e-13
    assert np.linalg.norm(V.T @ R[:, -1]) < 1e-10 * np.linalg.norm(A)


def test_cayley_spectral_mapping(small):
    prob, q0, J = small
    n = J.shape[0]
    sigma, mu = 0.2, -0.2
    C = np.linalg.solve(J - sigma * np.eye(n), J - mu * np.eye(n))
    lamJ = np.linalg.eigvals(J)
    lamC = np.linalg.eigvals(C)
    th = ar.cayley_theta(lamJ, sigma, mu)
    d = np.abs(lamC[:, None] - th[None, :]).min(axis=1)
    assert d.max() < 1e-10 * np.abs(th).max()
    # back-transform is the inverse map
    np.testing.assert_allclose(ar.cayley_lambda(th, sigma, mu), lamJ, atol=1e-10)


def test_cayley_iram_finds_kh_pair(kh24):
    prob, q0, J, lam = kh24
    idx = op.interior_index(prob)
    v0 = synth.random_vector(prob, 0).ravel()[idx]
    res = ar.iram(ar.cayley_operator_dense(J, 0.2, -0.2), v0, nev=2, ncv=20,
                  tol=1e-10, max_restarts=50)
    assert res["converged"]
    l, X = ar.ritz_pairs(res, 0.2, -0.2)
    for i in range(2):
        assert np.min(np.abs(lam - l[i])) < 1e-10
        r = np.linalg.norm(J @ X[:, i] - l[i] * X[:, i]) / np.linalg.norm(X[:, i])
        assert r < 1e-8 * abs(l[i])
    # the KH mode of the symmetric layer is real and double
    assert abs(l[0].imag) < 1e-10 and abs(l[0] - l[1]) < 1e-9
    assert 0.1 < l[0].real < 0.2


def test_cayley_iram_with_gmres_inner(kh24):
    prob, q0, J, lam = kh24
    idx = op.interior_index(prob)
    n = J.shape[0]
    A = J - 0.2 * np.eye(n)

    def C(v):
        x, info = kr.gmres(lambda z: A @ z, J @ v + 0.2 * v, restart=60, tol=1e-12)
        return x
    v0 = synth.random_vector(prob, 0).ravel()[idx]
    res = ar.iram(C, v0, nev=2, ncv=12, tol=1e-10, max_restarts=20)
    l = ar.cayley_lambda(res["theta"], 0.2, -0.2)
    assert res["converged"]
    for i in range(2):
        assert np.min(np.abs(lam - l[i])) / abs(l[i]) < 1e-8


# ---------------------------------------------------------------------- IR
def test_iterative_refinement_reaches_fp64_solution(small):
    prob, q0, J = small
    n = J.shape[0]
    A = J - 0.2 * np.eye(n)
    A32 = A.astype(np.float32)
    b = np.random.default_rng(6).standard_normal(n)
    y, info = refine.ir_solve(lambda v: A @ v, lambda v: A32 @ v, b, tol=1e-10,
                              inner_tol=1e-4, inner_restart=30)
    assert info["converged"]
    h = info["history"]
    assert all(h[i + 1] < h[i] for i in range(len(h) - 1))
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(y - xs) / np.linalg.norm(xs) < 1e-10 * np.linalg.cond(A)


# -------------------------------------------------------------- block-Jacobi
def test_probed_blocks_equal_dense_submatrices():
    prob = synth.mixing_layer_2d(16, 16, 0.3, 500.0)
    q0 = synth.random_base(prob, 8)
    lay = bj.block_layout(prob, 4, 4)
    Jfull = op.dense_jacobian(prob, q0, interior_only=False)
    Bd = bj.blocks_from_dense(prob, Jfull, lay)
    Bp = bj.blocks_by_probing(prob, lambda v: op.jv_cstep(prob, q0, v), lay)
    assert np.abs(Bp - Bd).max() <= 1e-12 * np.abs(Bd).max()


def test_probed_blocks_3d():
    prob = synth.mixing_layer_3d(8, 8, 8, 0.5, 1000.0)
    q0 = synth.random_base(prob, 9)
    lay = bj.block_layout(prob, 4, 4, 1)
    assert bj.probe_colours(prob, lay) == (2, 2, 4)
    Jfull = op.dense_jacobian(prob, q0, interior_only=False)
    Bd = bj.blocks_from_dense(prob, Jfull, lay)
    Bp = bj.blocks_by_probing(prob, lambda v: op.jv_cstep(prob, q0, v), lay)
    assert np.abs(Bp - Bd).max() <= 1e-12 * np.abs(Bd).max()


def test_block_apply_inverts_block_diagonal():
    prob = synth.mixing_layer_2d(8, 8, 0.3, 500.0)
    q0 = synth.random_base(prob, 10)
    lay = bj.block_layout(prob, 4, 4)
    Jfull = op.dense_jacobian(prob, q0, interior_only=False)
    B = bj.blocks_from_dense(prob, Jfull, lay)
    wall = bj.block_wall_mask(prob, lay)
    Bs = bj.shifted_blocks(B, 0.15, 0.1, 0.01, seed=3, wall=wall)
    r = synth.random_vector(prob, 1)
    z = bj.apply(prob, Bs, lay, r)
    idx = bj.block_dof_index(prob, lay)
    zb = z.ravel()[idx]
    rb = r.ravel()[idx]
    # B_b z_b = r_b for every block (wall entries of r are 0, so are those of z)
    np.testing.assert_allclose(np.einsum("bij,bj->bi", Bs, zb), rb, atol=1e-10)
    assert np.all(z.reshape(prob.shape)[:, 0, :] == 0)


def test_wall_dofs_are_identity_in_blocks():
    # at shift == diag_add and without noise, a wall block's interior part is
    # exactly P_b J P_b^T on the interior DOFs: the preconditioner must apply
    # its inverse there (no Schur complement from the wall DOFs)
    prob = synth.mixing_layer_2d(8, 8, 0.3, 500.0)
    q0 = synth.random_base(prob, 11)
    lay = bj.block_layout(prob, 4, 4)
    Jfull = op.dense_jacobian(prob, q0, interior_only=False)
    B = bj.blocks_from_dense(prob, Jfull, lay)
    wall = bj.block_wall_mask(prob, lay)
    assert wall.any() and not wall.all()
    Bs = bj.shifted_blocks(B, 0.1, 0.1, 0.0, seed=3, wall=wall)
    r = synth.random_vector(prob, 2)
    z = bj.apply(prob, Bs, lay, r)
    idx = bj.block_dof_index(prob, lay)
    for b in range(lay["nblocks"]):
        inn = ~wall[b]
        Bi = Jfull[np.ix_(idx[b][inn], idx[b][inn])]
        np.testing.assert_allclose(z.ravel()[idx[b][inn]], np.linalg.solve(Bi, r.ravel()[idx[b][inn]]),
                                   rtol=1e-10, atol=1e-12)
        # the wall DOFs of the shifted block form an identity block
        assert np.array_equal(Bs[b][np.ix_(wall[b], wall[b])], np.eye(wall[b].sum()))
        assert not Bs[b][np.ix_(wall[b], inn)].any() and not Bs[b][np.ix_(inn, wall[b])].any()


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        vals = [int(t, 16) for t in r]
        ctr = np.array(vals[0:4], dtype=np.uint64)
        key = np.array(vals[4:6], dtype=np.uint64)
        out = philox.philox4x32_10(ctr, key)
        assert [int(v) for v in out] == vals[6:10]


def test_block_noise_is_standard_normal():
    z = philox.block_noise(seed=3, nb=80, blocks=np.arange(40))
    assert z.shape == (40, 80, 80)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    z2 = philox.block_noise(seed=3, nb=80, blocks=np.arange(20, 40))
    assert np.array_equal(z[20:], z2)                   # counter-based: any subset
    z3 = philox.block_noise(seed=4, nb=80, blocks=np.arange(20, 40))
    assert not np.array_equal(z2, z3)


# ---------------------------------------------------------------------------
# LGMRES (Section "Iterative solvers": restart cycles augmented with error
# approximations)
# ---------------------------------------------------------------------------
def _convection_diffusion(N=40, eps=0.02):
    import scipy.sparse as sp
    h = 1.0 / (N + 1)
    I = sp.eye(N)
    e = np.ones(N)
    D2 = sp.diags([e[:-1], -2 * e, e[:-1]], [-1, 0, 1]) / h ** 2
    D1 = sp.diags([-e[:-1], e[:-1]], [-1, 1]) / (2 * h)
    return (-eps * (sp.kron(I, D2) + sp.kron(D2, I)) + sp.kron(I, D1) + 0.5 * sp.kron(D1, I)).tocsr()


def test_lgmres_without_augmentation_is_gmres(small):
    prob, q0, J = small
    idx = op.interior_index(prob)
    A = J - 0.2 * np.eye(J.shape[0])
    b = synth.random_vector(prob, 51).ravel()[idx]
    xg, ig = kr.gmres(lambda v: A @ v, b, restart=9, tol=1e-11, max_matvec=50000)
    xl, il = kr.lgmres(lambda v: A @ v, b, inner_m=9, outer_k=0, tol=1e-11, max_matvec=50000)
    assert np.array_equal(xg, xl)
    assert (ig["iters"], ig["matvecs"], ig["cycles"]) == (il["iters"], il["matvecs"], il["cycles"])


def test_lgmres_solution_and_library_routine():
    """LGMRES(17, 3) reaches the direct solution of a nonsymmetric
    convection-diffusion system, as scipy's lgmres (the same method, which
    also reuses the corrections' images) does, with about the same number of
    operator products."""
    import scipy.sparse.linalg as ssl
    A = _convection_diffusion()
    b = np.random.default_rng(5).standard_normal(A.shape[0])
    xd = ssl.spsolve(A.tocsc(), b)
    x, info = kr.lgmres(lambda v: A @ v, b, inner_m=17, outer_k=3, tol=1e-10, max_matvec=20000)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-7
    count = [0]

    def mv(v):
        count[0] += 1
        return A @ v
    xs, flag = ssl.lgmres(ssl.LinearOperator(A.shape, matvec=mv), b, rtol=1e-10, inner_m=17, outer_k=3,
                          maxiter=2000)
    assert flag == 0
    assert np.linalg.norm(xs - x) / np.linalg.norm(xd) < 1e-7
    assert abs(info["matvecs"] - count[0]) <= 0.05 * count[0]


def test_lgmres_needs_fewer_products_on_a_cayley_system():
    prob = synth.mixing_layer_2d(32, 32, 0.5, 1000.0)
    S = op.sparse_jacobian(prob, synth.base_flow(prob)).tocsr()
    idx = op.interior_index(prob)
    import scipy.sparse as sp
    A = (S[idx][:, idx] - 0.2 * sp.eye(len(idx))).tocsr()
    b = synth.random_vector(prob, 1).ravel()[idx]
    _, ig = kr.gmres(lambda v: A @ v, b, restart=40, tol=1e-10, max_matvec=60000)
    xl, il = kr.lgmres(lambda v: A @ v, b, inner_m=37, outer_k=3, tol=1e-10, max_matvec=60000)
    assert ig["converged"] and il["converged"]
    assert np.linalg.norm(b - A @ xl) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert il["matvecs"] < 0.8 * ig["matvecs"]


def test_cayley_leading_reference_matches_dense_spectrum():
    """The sparse ARPACK reference the GPU sweep test uses (tests/ref_spectra)
    against the dense LAPACK spectrum of the oracle's Jacobian on the 24x24
    case (tests/golden): the separated leading pair (the KH mode, |theta| =
    6.0) is the same to 1e-10.  Beyond it the spectrum is a ring of
    |theta| ~ 1 whose members differ by 1e-5 in |theta|; ARPACK settles on
    any of them, so the reference is used for separated eigenvalues only."""
    import numpy as _np
    from ref_spectra import cayley_leading
    prob = synth.mixing_layer_2d(24, 24, 0.3, 500.0)
    lam, th = cayley_leading(prob, synth.base_flow(prob), 4)
    a = _np.loadtxt(os.path.join(GOLDEN, "spectrum_kh_24x24_M0.3_Re500.txt"))
    ref = a[:, 0] + 1j * a[:, 1]
    for l in lam[:2]:
        assert abs(l - ref[0]) < 1e-10 * abs(ref[0])
    assert _np.all(_np.abs(th[:2]) > 5.0) and _np.all(_np.abs(th[2:]) < 1.01)

