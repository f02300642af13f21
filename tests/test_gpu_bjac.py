"""Parity of the HIP block-Jacobi preconditioner (coloured probing, seeded
noise, batched LU with partial pivoting, block solves) with the oracle's
blocks (dense-Jacobian submatrices, Philox noise) and plain batched solves.

FP64 factors: 1e-12 x cond.  FP32 factors: the bound of a backward-stable
FP32 solve, 8 nb 2^-24 cond, is used as the tolerance."""
import numpy as np
import pytest

import synth
from oracle import blockjac as bj
from oracle import operator as op
from gpu_util import dev, host, need_gpu, rel, torch

pytestmark = pytest.mark.gpu


def oracle_blocks(prob, q0, bx, by, bz, shifts, diag_add, noise_std, seed):
    lay = bj.block_layout(prob, bx, by, bz)
    Jfull = op.dense_jacobian(prob, q0, interior_only=False)
    B = bj.blocks_from_dense(prob, Jfull, lay)
    return lay, [bj.shifted_blocks(B, s, diag_add, noise_std, seed) for s in shifts]


CASES = [
    ("2d", synth.mixing_layer_2d(16, 16, 0.3, 500.0), (4, 4, 1)),
    ("2d-rect", synth.mixing_layer_2d(24, 12, 0.5, 1000.0), (4, 2, 1)),
    ("3d", synth.mixing_layer_3d(8, 8, 8, 0.5, 1000.0), (4, 4, 1)),
    # order 40: not a multiple of 16, so FP32 factors take the unblocked kernel
    ("2d-nb40", synth.mixing_layer_2d(20, 12, 0.5, 1000.0), (5, 2, 1)),
]


@pytest.mark.parametrize("name,prob,blk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fprec", ["f64", "f32"])
def test_block_apply_parity(name, prob, blk, fprec):
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, Context
    shifts = [0.05, 0.2, 0.35]
    q0 = synth.random_base(prob, 41)
    lay, Bs = oracle_blocks(prob, q0, *blk, shifts, 0.1, 0.01, 3)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup(shifts, *blk, diag_add=0.1, noise_std=0.01, seed=3,
                      factor_prec=SA_F64 if fprec == "f64" else SA_F32)
    r = synth.random_vector(prob, 42)
    for s in range(len(shifts)):
        ref = bj.apply(prob, Bs[s], lay, r)
        cond = max(np.linalg.cond(B) for B in Bs[s])
        z = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
        ctx.precond_apply(s, dev(r), z)
        tol = 1e-12 * cond if fprec == "f64" else 8 * lay["nb"] * 2.0 ** -24 * cond
        assert rel(host(z), ref) < tol, (s, cond)
        z32 = torch.empty(prob.ndof, dtype=torch.float32, device="cuda:0")
        ctx.precond_apply(s, dev(r, torch.float32), z32)
        assert rel(host(z32), ref) < max(tol, 8 * lay["nb"] * 2.0 ** -24 * cond)


def test_preconditioned_gmres_converges():
    need_gpu()
    from paper_1502_03701_amd import SA_F64, Context
    prob = synth.mixing_layer_2d(16, 16, 0.3, 500.0)
    q0 = synth.random_base(prob, 43)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup([0.2], 4, 4, 1, diag_add=0.0, noise_std=0.0, factor_prec=SA_F64)
    b = synth.random_vector(prob, 44)
    x = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda:0")
    rc, info = ctx.gmres_solve([0.2], dev(b), x, restart=40, tol=1e-10, use_precond=True)
    assert rc == 0 and info[0]["relres"] <= 1e-10
    J = op.dense_jacobian(prob, q0)
    idx = op.interior_index(prob)
    A = J - 0.2 * np.eye(J.shape[0])
    xr = np.zeros(prob.ndof)
    xr[idx] = np.linalg.solve(A, b.ravel()[idx])
    assert rel(host(x), xr) < 1e-10 * np.linalg.cond(A)


def test_singular_block_and_errors():
    need_gpu()
    from paper_1502_03701_amd import SA_F64, Context, SAError
    from paper_1502_03701_amd import _native as n
    prob = synth.mixing_layer_2d(16, 16, 0.3, 500.0)
    ctx = Context()
    ctx.base_set(prob, dev(synth.base_flow(prob)))
    r = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda:0")
    with pytest.raises(SAError) as e:
        ctx.precond_apply(0, r, torch.zeros_like(r))
    assert e.value.code == n.SA_ESTATE
    # wall DOFs have zero rows; diag_add = shift and no noise leaves them singular
    with pytest.raises(SAError) as e:
        ctx.precond_setup([0.2], 4, 4, 1, diag_add=0.2, noise_std=0.0, factor_prec=SA_F64)
    assert e.value.code == n.SA_ESINGULAR
    with pytest.raises(SAError) as e:
        ctx.precond_setup([0.2], 5, 4, 1)
    assert e.value.code == n.SA_EINVAL
