"""Parity of the HIP operator with compact first derivatives (sa_problem
scheme = SA_SCHEME_COMPACT) with the oracle's compact operator (exact
complex-step linearisation of the same discrete N).  Bar: 1e-12 normwise
relative in FP64, 1e-5 in FP32; eigenvalues against the dense spectrum of
the oracle's compact Jacobian within 1e-8."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import operator as op
from gpu_util import dev, host, need_gpu, rel, torch

pytestmark = pytest.mark.gpu
C = synth.SCHEME_COMPACT

CASES = [
    ("2d-wall", synth.mixing_layer_2d(16, 14, 0.5, 1000.0, scheme=C), "random"),
    ("2d-ragged", synth.mixing_layer_2d(15, 11, 0.3, 400.0, scheme=C), "random"),
    ("2d-periodic", synth.mixing_layer_2d(12, 12, 0.4, 600.0, bc_y=synth.BC_PERIODIC, scheme=C), "random"),
    ("2d-inviscid", synth.mixing_layer_2d(16, 21, 0.9, 0.0, scheme=C), "tanh"),
    ("3d-wall", synth.mixing_layer_3d(8, 9, 8, 0.5, 800.0, scheme=C), "random"),
    ("3d-periodic", synth.mixing_layer_3d(9, 8, 7, 0.4, 500.0, bc_y=synth.BC_PERIODIC, scheme=C), "random"),
]


def base_for(prob, kind, seed=7):
    if kind == "tanh":
        return synth.base_flow(prob)
    return synth.random_base(prob, seed)


@pytest.mark.parametrize("name,prob,kind", CASES, ids=[c[0] for c in CASES])
def test_compact_jv_parity(name, prob, kind):
    need_gpu()
    from paper_1502_03701_amd import Context
    q0 = base_for(prob, kind)
    v = synth.random_vector(prob, 3)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    explicit = op.jv_cstep(dataclasses.replace(prob, scheme=synth.SCHEME_EXPLICIT), q0, v)
    for shift in (0.0, 0.2):
        ref = op.jv_cstep(prob, q0, v) - shift * op.project(prob, v)
        y = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
        ctx.op_apply(dev(v), y, shift=shift)
        assert rel(host(y), ref) < 1e-12, name
        y32 = torch.empty(prob.ndof, dtype=torch.float32, device="cuda:0")
        ctx.op_apply(dev(v, torch.float32), y32, shift=shift)
        assert rel(host(y32), ref) < 1e-5, name
    # the compact operator is a different operator: far from the explicit one
    assert rel(op.jv_cstep(prob, q0, v), explicit) > 1e-4


def test_compact_batch_and_wall_inputs():
    """Several vectors in one call equal single calls; wall entries of x
    (here NaN) are ignored and y is 0 there."""
    need_gpu()
    from paper_1502_03701_amd import Context
    prob = synth.mixing_layer_3d(8, 9, 8, 0.5, 800.0, scheme=C)
    q0 = synth.random_base(prob, 8)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    v = synth.random_vector(prob, 9, nrhs=3)
    vw = v.copy()
    for r in range(3):
        vw[r][:, synth.wall_mask(prob)] = np.nan
    y = torch.empty(3 * prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.op_apply(dev(vw), y, shift=0.1, nrhs=3)
    yh = host(y).reshape(3, *prob.shape)
    for r in range(3):
        ref = op.jv_cstep(prob, q0, v[r]) - 0.1 * op.project(prob, v[r])
        assert rel(yh[r], ref) < 1e-12
        assert np.all(yh[r][:, synth.wall_mask(prob)] == 0.0)


def test_compact_gmres_with_explicit_mean_flow_preconditioner():
    """GMRES on the compact operator, right-preconditioned by the explicit
    operator of the x-averaged base (a cheaper approximate operator): the
    solution of the compact system to 1e-10, in far fewer products than
    without the preconditioner."""
    need_gpu()
    from paper_1502_03701_amd import SA_F64, SA_PC_MEAN_FLOW, Context
    prob = synth.mixing_layer_2d(24, 22, 0.5, 1000.0, scheme=C)
    q0 = synth.base_flow(prob)
    b = synth.random_vector(prob, 11, stream=1)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    x0 = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda:0")
    plain = ctx.gmres_solve([0.2], dev(b), x0, restart=40, tol=1e-10, max_matvec=200000)[1][0]
    ctx.precond_setup([0.2], factor_prec=SA_F64, kind=SA_PC_MEAN_FLOW)
    x1 = torch.zeros_like(x0)
    pre = ctx.gmres_solve([0.2], dev(b), x1, restart=40, tol=1e-10, use_precond=True)[1][0]
    assert pre["status"] == 0, pre
    J = op.dense_jacobian(prob, q0)
    idx = op.interior_index(prob)
    xs = np.linalg.solve(J - 0.2 * np.eye(J.shape[0]), b.ravel()[idx])
    assert rel(host(x1)[idx], xs) < 1e-8
    assert pre["matvecs"] * 5 < plain["matvecs"], (pre, plain)


def test_compact_eigenvalues_against_dense_spectrum():
    """Leading eigenvalues of the compact operator (2D mixing layer 24 x 22,
    M 0.5, Re 1000, KH pair) from Cayley-IRAM, FP64 and mixed, against the
    dense LAPACK spectrum of the oracle's compact Jacobian."""
    need_gpu()
    from paper_1502_03701_amd import SA_F64, SA_MIXED, SA_PC_MEAN_FLOW, Context, arnoldi_eigs
    prob = synth.mixing_layer_2d(24, 22, 0.5, 1000.0, scheme=C)
    q0 = synth.base_flow(prob)
    ev = np.linalg.eigvals(op.dense_jacobian(prob, q0))
    lead = ev[np.argmax(ev.real)]
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup([0.2], factor_prec=SA_F64, kind=SA_PC_MEAN_FLOW)
    v0 = dev(synth.random_vector(prob, 0))
    for prec in (SA_F64, SA_MIXED):
        rc, res = arnoldi_eigs([ctx], [v0], nev=2, ncv=16, tol=1e-11, max_restarts=60, lin_tol=1e-12,
                               use_precond=True, prec=prec)
        r = res[0]
        assert r["nconv"] >= 2, r
        for lam in r["lam"][:2]:
            assert np.min(np.abs(ev - lam)) < 1e-8 * abs(lam), (lam, lead)
        assert abs(max(r["lam"][:2], key=lambda z: z.real) - lead) < 1e-8 * abs(lead)
