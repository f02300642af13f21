"""Parity of the HIP operator y = (J - s I) x with the oracle's exact
(complex-step) linearisation.  Bar: 1e-12 normwise relative in FP64, 1e-5 in
FP32."""
import numpy as np
import pytest

import synth
from oracle import operator as op
from gpu_util import dev, host, need_gpu, rel, torch

pytestmark = pytest.mark.gpu

CASES = [
    ("c0", synth.config0(), "tanh"),
    ("2d-ragged-wall", synth.mixing_layer_2d(37, 29, 0.5, 1000.0), "random"),
    ("2d-periodic", synth.mixing_layer_2d(20, 18, 0.3, 300.0, bc_y=synth.BC_PERIODIC), "random"),
    ("2d-inviscid", synth.mixing_layer_2d(16, 21, 0.9, 0.0), "random"),
    ("3d-small", synth.mixing_layer_3d(12, 11, 10, 0.5, 1000.0), "random"),
    ("3d-reduced", synth.mixing_layer_3d(32, 16, 16, 0.5, 1000.0), "noise"),
    ("3d-periodic", synth.mixing_layer_3d(9, 8, 7, 0.4, 500.0, bc_y=synth.BC_PERIODIC), "random"),
]


def base_for(prob, kind, seed=7):
    if kind == "tanh":
        return synth.base_flow(prob)
    if kind == "noise":
        return synth.base_flow(prob, seed=seed, w_noise=1e-3)
    return synth.random_base(prob, seed)


@pytest.fixture(scope="module")
def ctxs():
    need_gpu()
    from paper_1502_03701_amd import Context
    return Context


@pytest.mark.parametrize("name,prob,kind", CASES, ids=[c[0] for c in CASES])
def test_jv_fp64_parity(ctxs, name, prob, kind):
    q0 = base_for(prob, kind)
    v = synth.random_vector(prob, 3)
    ctx = ctxs()
    ctx.base_set(prob, dev(q0))
    for shift in (0.0, 0.2):
        y = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
        ctx.op_apply(dev(v), y, shift=shift)
        ref = op.jv_cstep(prob, q0, v) - shift * op.project(prob, v)
        assert rel(host(y), ref) < 1e-12, name


@pytest.mark.parametrize("name,prob,kind", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_jv_fp32_parity(ctxs, name, prob, kind):
    q0 = base_for(prob, kind)
    v = synth.random_vector(prob, 4)
    ctx = ctxs()
    ctx.base_set(prob, dev(q0))
    y = torch.empty(prob.ndof, dtype=torch.float32, device="cuda:0")
    ctx.op_apply(dev(v, torch.float32), y, shift=0.2)
    ref = op.jv_cstep(prob, q0, v) - 0.2 * op.project(prob, v)
    assert rel(host(y), ref) < 1e-5


VARIANT_CASES = [
    ("2d-ragged-wall", synth.mixing_layer_2d(37, 29, 0.5, 1000.0), "random"),
    ("3d-small", synth.mixing_layer_3d(12, 11, 10, 0.5, 1000.0), "random"),
    ("3d-periodic", synth.mixing_layer_3d(9, 8, 7, 0.4, 500.0, bc_y=synth.BC_PERIODIC), "random"),
    # 40 planes: a ragged last z chunk for the chunk depths 16 and 32
    ("3d-zragged", synth.mixing_layer_3d(20, 13, 40, 0.5, 800.0), "noise"),
    # nx, ny multiples of 16: the 16 x 16 tiles cover the plane exactly (the
    # FP64 prefetch kernels' branch-free instantiation), z ragged as above
    ("3d-exact-tiles", synth.mixing_layer_3d(32, 16, 40, 0.5, 1000.0), "noise"),
    # uniform thermodynamic state (the iso kernels run): 2D parallel flow with
    # ragged tiles, and a small 3D grid with spanwise noise and ragged tiles
    ("2d-tanh-ragged", synth.mixing_layer_2d(37, 29, 0.5, 1000.0), "tanh"),
    ("3d-noise-ragged", synth.mixing_layer_3d(21, 19, 11, 0.5, 1000.0), "noise"),
]
NVAR = 12


@pytest.mark.parametrize("variant", range(NVAR))
@pytest.mark.parametrize("name,prob,kind", VARIANT_CASES, ids=[c[0] for c in VARIANT_CASES])
def test_jv_every_kernel_variant(ctxs, name, prob, kind, variant):
    """Each operator kernel variant the autotuner may pick, pinned, in both
    precisions, against the oracle (also with two right-hand sides).  NaN on
    both wall rows of the input must be ignored (the operator is P J P)."""
    from paper_1502_03701_amd import SA_F32, SA_F64
    q0 = base_for(prob, kind)
    v = synth.random_vector(prob, 5, nrhs=2)
    ctx = ctxs()
    ctx.base_set(prob, dev(q0))
    ctx.set_jv_variant(SA_F64, variant)
    ctx.set_jv_variant(SA_F32, variant)
    assert ctx.jv_variant(SA_F64)[0] == variant and ctx.jv_variant(SA_F32)[0] == variant
    ref = np.stack([op.jv_cstep(prob, q0, v[r]) - 0.1 * op.project(prob, v[r]) for r in range(2)])
    if prob.bc[1] == synth.BC_WALL:
        v = v.copy()
        v[..., 0, :] = np.nan
        v[..., -1, :] = np.nan
    y = torch.empty(2 * prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.op_apply(dev(v), y, shift=0.1, nrhs=2)
    assert rel(host(y), ref.ravel()) < 1e-12, (name, variant)
    y32 = torch.empty(2 * prob.ndof, dtype=torch.float32, device="cuda:0")
    ctx.op_apply(dev(v, torch.float32), y32, shift=0.1, nrhs=2)
    assert rel(host(y32), ref.ravel()) < 1e-5, (name, variant)
    if prob.bc[1] == synth.BC_WALL:   # wall rows: exactly zero (+0 or -0), in both precisions
        for out in (host(y), host(y32)):
            w = out.reshape((2,) + prob.shape)
            assert np.all(w[..., 0, :] == 0) and np.all(w[..., -1, :] == 0), (name, variant)


def test_autotuner_picks_a_measured_variant(ctxs):
    from paper_1502_03701_amd import SA_F32, SA_F64, SAError
    prob = synth.mixing_layer_3d(32, 16, 40, 0.5, 1000.0)
    ctx = ctxs()
    ctx.base_set(prob, dev(synth.base_flow(prob, seed=1, w_noise=1e-3)))
    for prec in (SA_F64, SA_F32):
        var, times = ctx.jv_variant(prec)
        assert 0 <= var < NVAR
        assert all(t > 0 for t in times.values())      # uniform p0, s0: the iso kernels are timed too
        assert list(times.values())[var] == min(times.values())
    with pytest.raises(SAError):
        ctx.set_jv_variant(SA_F64, NVAR)


def test_uniform_state_detection(ctxs):
    """The iso kernels are timed (and may be picked) only for base states
    whose pressure and entropy are the same at every point."""
    from paper_1502_03701_amd import SA_F32, SA_F64
    prob = synth.mixing_layer_3d(16, 12, 10, 0.5, 1000.0)
    from paper_1502_03701_amd._native import JV_VARIANTS
    ctx = ctxs()
    iso = [n for n in JV_VARIANTS if n.startswith("iso")]
    for q0, expect in [(synth.base_flow(prob, seed=3, w_noise=1e-3), True), (synth.random_base(prob, 2), False)]:
        ctx.base_set(prob, dev(q0))
        for prec in (SA_F64, SA_F32):
            var, times = ctx.jv_variant(prec)
            assert all((times[n] > 0) == expect for n in iso), (expect, times)
            if not expect:
                assert not JV_VARIANTS[var].startswith("iso")
    # a base whose entropy varies in one point only is not of that class
    q0 = synth.base_flow(prob)
    q0[-1, 4, 5, 6] = 1e-9
    ctx.base_set(prob, dev(q0))
    assert all(ctx.jv_variant(SA_F64)[1][n] == 0 for n in iso)


def test_jv_multi_rhs_and_wall_inputs_ignored(ctxs):
    prob = synth.mixing_layer_2d(24, 19, 0.5, 800.0)
    q0 = synth.random_base(prob, 9)
    V = synth.random_vector(prob, 5, nrhs=3)
    ctx = ctxs()
    ctx.base_set(prob, dev(q0))
    Vw = V.copy()
    Vw[:, :, 0, :] = 3.0           # garbage on the wall rows of the input
    y = torch.empty(3 * prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.op_apply(dev(Vw), y, shift=0.1, nrhs=3)
    Y = host(y).reshape((3,) + prob.shape)
    for r in range(3):
        ref = op.jv_cstep(prob, q0, V[r]) - 0.1 * op.project(prob, V[r])
        assert rel(Y[r], ref) < 1e-12
        assert np.all(Y[r][:, 0, :] == 0) and np.all(Y[r][:, -1, :] == 0)


@pytest.mark.parametrize("variant", [None, 8, 0], ids=["autotuned", "iso_z32", "prefetch_z32"])
def test_jv_full_size_3d_sampled_windows(ctxs, variant):
    """256x128x128 (the 3D benchmark grid), the kernels bench.py times (the
    autotuned ones) and the iso and general 32-plane kernels pinned: compare
    windows of the full-size GPU output, FP64 and FP32, with the oracle
    evaluated on the window (valid >= 3 cells away from the window's cut
    faces, full y range with the walls)."""
    from paper_1502_03701_amd import SA_F32, SA_F64
    prob = synth.config2()
    q0 = synth.base_flow(prob, seed=2, w_noise=1e-3)
    v = synth.random_vector(prob, 2)
    ctx = ctxs()
    if variant is not None:
        ctx.set_jv_variant(SA_F64, variant)
        ctx.set_jv_variant(SA_F32, variant)
    ctx.base_set(prob, dev(q0))
    print("\nvariants:", ctx.jv_variant(SA_F64)[0], ctx.jv_variant(SA_F32)[0])
    y = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.op_apply(dev(v), y, shift=0.2)
    Y = host(y).reshape(prob.shape)
    y32 = torch.empty(prob.ndof, dtype=torch.float32, device="cuda:0")
    ctx.op_apply(dev(v, torch.float32), y32, shift=0.2)
    Y32 = host(y32).reshape(prob.shape)
    rng = np.random.default_rng(0)
    nx, ny, nz = prob.n
    W = 14
    dx = prob.length[0] / nx
    dz = prob.length[2] / nz
    for _ in range(3):
        i0 = int(rng.integers(0, nx))
        k0 = int(rng.integers(0, nz))
        ii = (i0 + np.arange(W)) % nx
        kk = (k0 + np.arange(W)) % nz
        sub = synth.mixing_layer_3d(W, ny, W, prob.mach, prob.re, lx=W * dx, ly=prob.length[1], lz=W * dz)
        qs = q0[:, kk][:, :, :, ii]
        vs = v[:, kk][:, :, :, ii]
        ref = op.jv_cstep(sub, qs, vs) - 0.2 * op.project(sub, vs)
        inner = (slice(None), slice(3, W - 3), slice(None), slice(3, W - 3))
        assert rel(Y[:, kk][:, :, :, ii][inner], ref[inner]) < 1e-12
        assert rel(Y32[:, kk][:, :, :, ii][inner], ref[inner]) < 1e-5


def test_jv_deterministic_rerun(ctxs):
    prob = synth.mixing_layer_3d(16, 12, 10, 0.5, 1000.0)
    q0 = synth.random_base(prob, 1)
    v = synth.random_vector(prob, 1)
    ctx = ctxs()
    ctx.base_set(prob, dev(q0))
    y1 = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
    y2 = torch.empty_like(y1)
    ctx.op_apply(dev(v), y1)
    ctx.op_apply(dev(v), y2)
    assert torch.equal(y1, y2)


def test_errors(ctxs):
    from paper_1502_03701_amd import SAError
    from paper_1502_03701_amd import _native as n
    ctx = ctxs()
    x = torch.zeros(100, dtype=torch.float64, device="cuda:0")
    rc = ctx.lib.sa_op_apply(ctx.h, 0, 1, n._ptr(x), n._ptr(x), 0.0)
    assert rc == n.SA_ESTATE
    prob = synth.mixing_layer_2d(12, 12, 0.3, 500.0)
    q0 = synth.base_flow(prob)
    q0[0, 3, 3] = np.nan
    with pytest.raises(SAError) as e:
        ctx.base_set(prob, dev(q0))
    assert e.value.code == n.SA_ENONFINITE
    bad = synth.mixing_layer_2d(6, 12, 0.3, 500.0)
    with pytest.raises(SAError) as e:
        ctx.base_set(bad, dev(synth.base_flow(bad)))
    assert e.value.code == n.SA_EINVAL


def test_jv_full_size_2d_every_output(ctxs):
    """512 x 512 (the 2D benchmark grid, n = 1 048 576), the autotuned
    kernels: every output of the FP64 product against the oracle to 1e-12,
    the FP32 product to 1e-5."""
    from paper_1502_03701_amd import SA_F32, SA_F64
    prob = synth.config1()
    q0 = synth.base_flow(prob)
    v = synth.random_vector(prob, 8)
    ctx = ctxs()
    ctx.base_set(prob, dev(q0))
    assert ctx.jv_variant(SA_F64)[0] >= 0 and ctx.jv_variant(SA_F32)[0] >= 0   # tuned, not defaulted
    ref = op.jv_cstep(prob, q0, v) - 0.2 * op.project(prob, v)
    y = torch.empty(prob.ndof, dtype=torch.float64, device="cuda:0")
    ctx.op_apply(dev(v), y, shift=0.2)
    assert rel(host(y), ref) < 1e-12
    y32 = torch.empty(prob.ndof, dtype=torch.float32, device="cuda:0")
    ctx.op_apply(dev(v, torch.float32), y32, shift=0.2)
    assert rel(host(y32), ref) < 1e-5
