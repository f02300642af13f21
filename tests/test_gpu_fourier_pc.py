"""Parity of the HIP mean-flow preconditioner with the oracle's dense one.

M(s) = P (J(q_bar) - s I) P with q_bar the base averaged over the periodic
axes.  The library builds it from operator probes, factors one banded matrix
per Fourier mode and shift, and applies it through DFTs; the oracle solves
the dense M(s) assembled from its own complex-step Jacobian.

Tolerances: FP64 factors and FP64 vectors 1e-12 cond(M); FP32 factors or
FP32 vectors 8 (kl + ku + 1 + nx + nz) 2^-24 cond(M), the bound of a
backward-stable FP32 banded solve plus the FP32 DFT sums."""
import numpy as np
import pytest

import synth
from oracle import fourier_pc as fpc
from oracle import operator as op
from gpu_util import dev, host, need_gpu, rel, torch

pytestmark = pytest.mark.gpu

SHIFTS = [0.05, 0.2, 0.35]

CASES = [
    ("2d", synth.mixing_layer_2d(16, 14, 0.5, 1000.0)),
    # odd nx: no Nyquist mode; 34 interior rows: many window slides
    ("2d-odd-tall", synth.mixing_layer_2d(15, 36, 0.3, 500.0)),
    # 5 interior rows, fewer than the 7 probe colours; order 20, barely
    # more than the LU window's 16 rows
    ("2d-five-rows", synth.mixing_layer_2d(12, 7, 0.5, 1000.0)),
    ("3d", synth.mixing_layer_3d(8, 9, 8, 0.5, 800.0)),
    ("3d-odd", synth.mixing_layer_3d(9, 10, 7, 0.5, 800.0)),
]


def tol_for(prob, cond, f32):
    if not f32:
        return 1e-12 * cond
    nv = prob.nv
    kw = 8 * nv - 1
    return 8 * (kw + prob.n[0] + prob.n[2]) * 2.0 ** -24 * cond


@pytest.mark.parametrize("name,prob", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fprec", ["f64", "f32"])
def test_mean_flow_apply_parity(name, prob, fprec):
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, SA_PC_MEAN_FLOW, Context
    q0 = synth.random_base(prob, 51)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup(SHIFTS, factor_prec=SA_F64 if fprec == "f64" else SA_F32, kind=SA_PC_MEAN_FLOW)
    r = synth.random_vector(prob, 52)
    # wall entries of r are ignored
    rw = r.copy()
    rw[:, synth.wall_mask(prob)] = 7.0
    for s, sig in enumerate(SHIFTS):
        M = fpc.operator_matrix(prob, q0, sig)
        ref = fpc.apply(prob, q0, sig, r, M=M)
        cond = np.linalg.cond(M)
        z = torch.full((prob.ndof,), np.nan, dtype=torch.float64, device="cuda:0")
        ctx.precond_apply(s, dev(rw), z)
        zh = host(z)
        err = rel(zh, ref)
        assert err < tol_for(prob, cond, fprec == "f32"), (s, err, cond)
        assert np.all(zh.reshape(prob.shape)[:, synth.wall_mask(prob)] == 0.0)
        z32 = torch.full((prob.ndof,), np.nan, dtype=torch.float32, device="cuda:0")
        ctx.precond_apply(s, dev(rw, torch.float32), z32)
        err32 = rel(host(z32), ref)
        assert err32 < tol_for(prob, cond, True), (s, err32, cond)


def test_mean_flow_apply_several_vectors():
    """nrhs vectors with one shift equal the same vectors one at a time."""
    need_gpu()
    from paper_1502_03701_amd import SA_F64, SA_PC_MEAN_FLOW, Context
    prob = synth.mixing_layer_3d(8, 9, 8, 0.5, 800.0)
    q0 = synth.random_base(prob, 53)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup(SHIFTS, factor_prec=SA_F64, kind=SA_PC_MEAN_FLOW)
    r = synth.random_vector(prob, 54, nrhs=3)
    z = torch.empty(3 * prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.precond_apply(1, dev(r), z, nrhs=3)
    zh = host(z).reshape(3, -1)
    for i in range(3):
        zi = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
        ctx.precond_apply(1, dev(r[i]), zi)
        assert np.array_equal(host(zi), zh[i])


def test_mean_flow_rejects_what_it_cannot_do():
    need_gpu()
    from paper_1502_03701_amd import SA_F64, SA_PC_MEAN_FLOW, Context, SAError
    ctx = Context()
    prob = synth.mixing_layer_2d(16, 14, 0.5, 1000.0)
    ctx.base_set(prob, dev(synth.base_flow(prob)))
    with pytest.raises(SAError):
        ctx.precond_setup([0.2], kind=7)
    ctx.precond_setup([0.2, 0.3], factor_prec=SA_F64, kind=SA_PC_MEAN_FLOW)
    r = dev(synth.random_vector(prob, 1, nrhs=3))
    z = torch.empty_like(r)
    with pytest.raises(SAError):   # at most nshift vectors per call
        ctx.precond_apply(0, r, z, nrhs=3)
    with pytest.raises(SAError):
        ctx.precond_apply(2, r[:prob.ndof], z[:prob.ndof])
    # no walls in y: no banded structure
    per = synth.mixing_layer_2d(16, 16, 0.5, 1000.0, bc_y=synth.BC_PERIODIC)
    ctx3 = Context()
    ctx3.base_set(per, dev(synth.base_flow(per)))
    with pytest.raises(SAError):
        ctx3.precond_setup([0.2], kind=SA_PC_MEAN_FLOW)


def test_parallel_flow_is_solved_in_one_step():
    """For a base that does not vary along x, q_bar = q0 and M(s) = J - s I:
    preconditioned GMRES converges after one product (2D workload of the
    48 x 48 mixing layer, M 0.3, Re 500)."""
    need_gpu()
    from paper_1502_03701_amd import SA_F64, SA_PC_MEAN_FLOW, Context
    prob = synth.config0()
    q0 = synth.base_flow(prob)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup([0.2], factor_prec=SA_F64, kind=SA_PC_MEAN_FLOW)
    b = synth.random_vector(prob, 61, stream=1)
    x = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda:0")
    _, info = ctx.gmres_solve([0.2], dev(b), x, restart=40, tol=1e-10, use_precond=True)
    assert info[0]["status"] == 0 and info[0]["matvecs"] <= 3, info[0]
    J = op.dense_jacobian(prob, q0)
    idx = op.interior_index(prob)
    xs = np.linalg.solve(J - 0.2 * np.eye(J.shape[0]), b.ravel()[idx])
    assert rel(host(x)[idx], xs) < 1e-9


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_noisy_3d_base_converges_in_a_few_products(prec):
    """3D tanh layer with 1e-3 spanwise noise: q_bar removes the noise, so
    the preconditioned operator is the identity up to O(1e-3) and GMRES
    needs a handful of products where plain GMRES(40) needs hundreds; both
    reach the same solution."""
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, SA_MIXED, SA_PC_MEAN_FLOW, Context
    prob = synth.mixing_layer_3d(24, 25, 16, 0.5, 1000.0)
    q0 = synth.base_flow(prob, seed=2, w_noise=1e-3)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    b = dev(synth.random_vector(prob, 62, stream=1))
    x0 = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda:0")
    plain = ctx.gmres_solve([0.2], b, x0, restart=40, tol=1e-10)[1][0]
    ctx.precond_setup([0.2], factor_prec=SA_F64 if prec == "f64" else SA_F32, kind=SA_PC_MEAN_FLOW)
    x1 = torch.zeros_like(x0)
    kw = dict(prec=SA_MIXED, inner_tol=1e-4) if prec == "mixed" else {}
    pre = ctx.gmres_solve([0.2], b, x1, restart=40, tol=1e-10, use_precond=True, **kw)[1][0]
    assert plain["status"] == 0 and pre["status"] == 0, (plain, pre)
    # refinement: 3 outer sweeps, each a residual product and 2 - 3 inner ones
    assert pre["matvecs"] <= (12 if prec == "f64" else 24), (pre, plain)
    assert pre["matvecs"] * 10 < plain["matvecs"], (pre, plain)
    assert rel(host(x1), host(x0)) < 1e-8
    # true residual of the preconditioned solution
    y = torch.empty_like(x1)
    ctx.op_apply(x1, y, shift=0.2)
    assert rel(host(y), host(b)) < 2e-10


def test_eigs_with_mean_flow_preconditioner_match():
    """Cayley-IRAM with preconditioned inner solves on the 48 x 48 workload
    (M 0.3, Re 500, Arnoldi dimension 30, 6 eigenpairs): the four separated
    leading eigenvalues match the oracle's dense spectrum within 1e-8, and a
    Cayley solve costs a few products (M(sigma) is the operator itself for
    this parallel base; plain GMRES needs thousands)."""
    need_gpu()
    from test_gpu_eigs import check, golden
    from paper_1502_03701_amd import SA_F64, SA_MIXED, SA_NOT_CONVERGED, SA_PC_MEAN_FLOW, Context, arnoldi_eigs
    prob = synth.config0()
    q0 = synth.base_flow(prob)
    v0 = dev(synth.random_vector(prob, 0))
    ref = golden("c0_48x48_M0.3_Re500")
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup([0.2], factor_prec=SA_F64, kind=SA_PC_MEAN_FLOW)
    for prec in (SA_F64, SA_MIXED):
        rc, out = arnoldi_eigs([ctx], [v0], nev=6, ncv=30, lin_tol=1e-12, use_precond=True, prec=prec,
                               max_restarts=20)
        r = out[0]
        assert rc in (0, SA_NOT_CONVERGED)
        check(r["lam"][:4], ref, 2)
        # FP64: one Krylov step and the residual products; refinement: about
        # four sweeps of a residual product and two FP32 steps to 1e-12
        per = 5 if prec == SA_F64 else 16
        assert r["n_matvec"] <= per * r["n_cayley"], (r["n_matvec"], r["n_cayley"])


def test_fp32_solve_after_fp64_solve_stays_finite():
    """A preconditioned FP32 solve that converges in a few steps, run after an
    FP64 solve on the same context: its unused basis columns hold the FP64
    run's bytes, which read as FP32 may be non-finite; the solution update
    must not touch them."""
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, SA_PC_MEAN_FLOW, Context
    prob = synth.mixing_layer_3d(24, 25, 16, 0.5, 1000.0)
    ctx = Context()
    ctx.base_set(prob, dev(synth.base_flow(prob, seed=2, w_noise=1e-3)))
    ctx.precond_setup([0.2], factor_prec=SA_F32, kind=SA_PC_MEAN_FLOW)
    b = dev(synth.random_vector(prob, 62, stream=1))
    x = torch.zeros_like(b)
    assert ctx.gmres_solve([0.2], b, x, restart=40, tol=1e-10, use_precond=True)[1][0]["status"] == 0
    for graph in (True, False):
        x32 = torch.zeros(prob.ndof, dtype=torch.float32, device="cuda:0")
        _, info = ctx.gmres_solve([0.2], b.float(), x32, restart=40, tol=1e-5, use_precond=True, prec=SA_F32,
                                  use_graph=graph)
        assert info[0]["status"] == 0 and info[0]["matvecs"] <= 8, info[0]
        assert bool(torch.isfinite(x32).all())
        assert rel(host(x32), host(x)) < 1e-4


@pytest.mark.slow
@pytest.mark.parametrize("fprec", ["f64", "f32"])
def test_full_size_3d_residual(fprec):
    """256 x 128 x 128, 5 variables, tanh layer without noise (q_bar = q0,
    so M(s) = J - s I): the residual of the applied inverse, measured with
    the operator kernel, bounds the whole path at full size."""
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, SA_PC_MEAN_FLOW, Context
    prob = synth.config2()
    ctx = Context()
    ctx.base_set(prob, dev(synth.base_flow(prob)))
    ctx.precond_setup([0.2], factor_prec=SA_F64 if fprec == "f64" else SA_F32, kind=SA_PC_MEAN_FLOW)
    g = torch.Generator(device="cuda:0").manual_seed(5)
    r = torch.randn(prob.ndof, dtype=torch.float64, device="cuda:0", generator=g)
    r.view(prob.shape)[:, :, [0, -1], :] = 0.0
    z = torch.empty_like(r)
    ctx.precond_apply(0, r, z)
    y = torch.empty_like(r)
    ctx.op_apply(z, y, shift=0.2)
    res = float(torch.linalg.norm(y - r) / torch.linalg.norm(r))
    assert res < (1e-9 if fprec == "f64" else 1e-3), res


def test_sweep_problems_full_size_against_mode_oracle():
    """Three problems of the 48-flow sweep at their full size (the smallest
    and the largest side, and one between), run concurrently on their own
    streams in the mixed form with the mean-flow preconditioner: the
    leading (Kelvin-Helmholtz) pair of each against the leading eigenvalue
    of the oracle's x-Fourier block k = 1 (the x-wavenumber of the box),
    within 1e-8."""
    need_gpu()
    from ref_spectra import mode_leading
    from paper_1502_03701_amd import SA_F32, SA_MIXED, SA_PC_MEAN_FLOW, Context, arnoldi_eigs
    items = synth.config4_sweep()
    sides = [it.problem.n[0] for it in items]
    pick = [int(np.argmin(sides)), int(np.argmax(sides)), 11]
    streams = [torch.cuda.Stream() for _ in pick]
    ctxs, v0s = [], []
    for i, st in zip(pick, streams):
        it = items[i]
        c = Context(stream=st)
        c.base_set(it.problem, dev(synth.base_flow(it.problem)))
        c.precond_setup([0.2], factor_prec=SA_F32, kind=SA_PC_MEAN_FLOW)
        ctxs.append(c)
        v0s.append(dev(synth.random_vector(it.problem, it.seed)))
    torch.cuda.synchronize()
    rc, res = arnoldi_eigs(ctxs, v0s, nev=2, ncv=16, tol=1e-10, max_restarts=60, restart=30, lin_tol=1e-12,
                           prec=SA_MIXED, inner_tol=1e-4, use_precond=True)
    assert rc == 0
    for i, r in zip(pick, res):
        it = items[i]
        ref = mode_leading(it.problem, synth.base_flow(it.problem))[0]
        got = max(r["lam"][:2], key=lambda z: z.real)
        assert r["nconv"] >= 2
        assert abs(got - ref) < 1e-8 * abs(ref), (it.problem.n, got, ref)
        assert all(abs(l - ref) < 1e-8 * abs(ref) for l in r["lam"][:2])
