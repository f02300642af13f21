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
    wall = bj.block_wall_mask(prob, lay)
    return lay, [bj.shifted_blocks(B, s, diag_add, noise_std, seed, wall=wall) for s in shifts]


CASES = [
    ("2d", synth.mixing_layer_2d(16, 16, 0.3, 500.0), (4, 4, 1)),
    ("2d-rect", synth.mixing_layer_2d(24, 12, 0.5, 1000.0), (4, 2, 1)),
    ("3d", synth.mixing_layer_3d(8, 8, 8, 0.5, 1000.0), (4, 4, 1)),
    # order 40: not a multiple of 16, so FP32 factors take the unblocked kernel
    ("2d-nb40", synth.mixing_layer_2d(20, 12, 0.5, 1000.0), (5, 2, 1)),
    # 5 block rows between the walls, 2 probe colours in y: colours of
    # unequal size (3 and 2 block rows)
    ("2d-ragged-colours", synth.mixing_layer_2d(16, 20, 0.3, 500.0), (4, 4, 1)),
]


@pytest.mark.parametrize("name,prob,blk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("fprec", ["f64", "f32"])
def test_block_apply_parity(name, prob, blk, fprec):
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, Context
    # 0.1 == diag_add: the interior part of a wall block is then unshifted
    shifts = [0.05, 0.1, 0.35]
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


@pytest.mark.parametrize("fprec", ["f64", "f32"])
def test_wall_blocks_invert_their_interior_part(fprec):
    """At shift == diag_add and without noise, each block's interior part is
    the interior submatrix of the dense Jacobian: the preconditioner must
    apply exactly its inverse on the interior DOFs of wall blocks (the wall
    DOFs, not unknowns of P J P, stay an identity and add no Schur term)."""
    need_gpu()
    from paper_1502_03701_amd import SA_F32, SA_F64, Context
    prob = synth.mixing_layer_2d(16, 16, 0.3, 500.0)
    q0 = synth.random_base(prob, 45)
    lay = bj.block_layout(prob, 4, 4, 1)
    Jfull = op.dense_jacobian(prob, q0, interior_only=False)
    idx = bj.block_dof_index(prob, lay)
    wall = bj.block_wall_mask(prob, lay)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup([0.1], 4, 4, 1, diag_add=0.1, noise_std=0.0,
                      factor_prec=SA_F64 if fprec == "f64" else SA_F32)
    r = synth.random_vector(prob, 46)
    z = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.precond_apply(0, dev(r), z)
    zh = host(z)
    nwall = 0
    for b in range(lay["nblocks"]):
        if not wall[b].any():
            continue
        nwall += 1
        inn = ~wall[b]
        Bi = Jfull[np.ix_(idx[b][inn], idx[b][inn])]
        ref = np.linalg.solve(Bi, r.ravel()[idx[b][inn]])
        cond = np.linalg.cond(Bi)
        tol = 1e-12 * cond if fprec == "f64" else 8 * lay["nb"] * 2.0 ** -24 * cond
        assert rel(zh[idx[b][inn]], ref) < tol, (b, cond)
        assert np.all(zh[idx[b][wall[b]]] == 0)
    assert nwall == 2 * lay["nbx"]


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
    # a fluid at rest without viscosity: the entropy rows of J vanish, so
    # diag_add = shift without noise leaves every block exactly singular
    rest = synth.mixing_layer_2d(16, 16, 0.3, 0.0)
    q_rest = synth.base_flow(rest)
    q_rest[1] = 0.0
    ctx.base_set(rest, dev(q_rest))
    with pytest.raises(SAError) as e:
        ctx.precond_setup([0.2], 4, 4, 1, diag_add=0.2, noise_std=0.0, factor_prec=SA_F64)
    assert e.value.code == n.SA_ESINGULAR
    with pytest.raises(SAError) as e:
        ctx.precond_setup([0.2], 5, 4, 1)
    assert e.value.code == n.SA_EINVAL


def test_full_size_3d_sampled_blocks():
    """256x128x128 with 4x4x1-cell blocks (262 144 blocks of order 80), the 8
    benchmark shifts and FP32 factors, as timed: the GPU preconditioner's
    output on sampled blocks (walls, periodic seams, interior) against the
    oracle's solve with that block.  Each block comes from the oracle's
    complex-step operator on a periodic window around it (rows >= 6 cells
    from the window's cut faces, so the window's operator equals the full
    grid's there) plus the Philox noise of its global block index."""
    need_gpu()
    from oracle import philox
    from paper_1502_03701_amd import Context
    prob = synth.config2()
    q0 = synth.base_flow(prob, seed=2, w_noise=1e-3)
    shifts = synth.config3_shifts()
    nx, ny, nz = prob.n
    lay = bj.block_layout(prob, 4, 4, 1)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    ctx.precond_setup(shifts, 4, 4, 1, diag_add=0.1, noise_std=0.01, seed=3)
    r = synth.random_vector(prob, 43)
    Z = {}
    for s in (0, 7):
        z = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
        ctx.precond_apply(s, dev(r), z)
        Z[s] = host(z).reshape(prob.shape)
    ctx.close()
    dx, dz = prob.length[0] / nx, prob.length[2] / nz
    M, WX, WZ = 6, 16, 13          # margin, window width in x and z
    for ib, jb, kb in [(0, 0, 0), (63, 31, 127), (17, 13, 64), (40, 1, 5)]:
        ii = (4 * ib - M + np.arange(WX)) % nx
        kk = (kb - M + np.arange(WZ)) % nz
        sub = synth.mixing_layer_3d(WX, ny, WZ, prob.mach, prob.re, lx=WX * dx, ly=prob.length[1], lz=WZ * dz)
        qs = q0[:, kk][:, :, :, ii]
        # local DOF l = var*16 + 4*cy + cx of the block, in window coordinates
        l = np.arange(80)
        var, cy, cx = l // 16, (l % 16) // 4, l % 4
        wflat = ((var * WZ + M) * ny + (4 * jb + cy)) * WX + (M + cx)
        B = np.zeros((80, 80))
        for c in range(80):
            e = np.zeros(sub.ndof)
            e[wflat[c]] = 1.0
            B[:, c] = op.jv_cstep(sub, qs, e.reshape(sub.shape)).ravel()[wflat]
        b = (kb * lay["nby"] + jb) * lay["nbx"] + ib
        E = philox.block_noise(3, 80, [b])[0]
        gflat = ((var * nz + kb) * ny + (4 * jb + cy)) * nx + (4 * ib + cx)
        wall = (4 * jb + cy == 0) | (4 * jb + cy == ny - 1)
        for s in (0, 7):
            Bs = B + 0.01 * E + (0.1 - shifts[s]) * np.eye(80)
            # wall DOFs: identity rows and columns (not unknowns of P J P)
            Bs[wall, :] = 0.0
            Bs[:, wall] = 0.0
            Bs[wall, wall] = 1.0
            ref = np.linalg.solve(Bs, r.ravel()[gflat])
            ref[wall] = 0.0
            got = Z[s].ravel()[gflat]
            tol = 8 * 80 * 2.0 ** -24 * np.linalg.cond(Bs)
            assert rel(got, ref) < tol, (ib, jb, kb, s)
