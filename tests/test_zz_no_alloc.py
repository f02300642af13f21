"""The allocation-free GMRES entry point (sa_gmres_solve_noalloc) against the
allocating one (sa_gmres_solve) through the C ABI.

Both run the same kernels in the same order (restart cycles as plain
launches), so the solutions, residuals and counts must agree bit for bit.
Two calls in a row share the device's scratch array, the second with a
smaller problem; a third uses the refinement form, and a solve whose
workspace exceeds the scratch is refused with SA_EINVAL."""
import numpy as np
import pytest

import synth
from gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu


def _pair(ctx, prob, sigmas, b, **kw):
    ns = len(sigmas)
    out = []
    for noalloc in (False, True):
        x = torch.zeros(ns * prob.ndof, dtype=torch.float64, device="cuda:0")
        rc, info = ctx.gmres_solve(sigmas, b, x, use_graph=False, noalloc=noalloc, **kw)
        out.append((rc, info, host(x)))
    return out


def test_noalloc_matches_allocating_solve_twice():
    need_gpu()
    from paper_1502_03701_amd import SA_MIXED, Context
    # call 1: two shifts in lockstep on a 24 x 20 grid
    pa = synth.mixing_layer_2d(24, 20, 0.3, 500.0)
    ca = Context()
    ca.base_set(pa, dev(synth.random_base(pa, 61)))
    ba = synth.random_vector(pa, 62, stream=1, nrhs=2)
    (rc0, i0, x0), (rc1, i1, x1) = _pair(ca, pa, [0.2, 0.35], dev(ba), restart=20, tol=1e-8,
                                         max_matvec=3000)
    print("call 1:", rc0, [i["iters"] for i in i0], [i["relres"] for i in i0])
    assert rc0 == rc1 and i0 == i1
    assert np.array_equal(x0, x1)
    assert max(i["relres"] for i in i1) <= 1e-8 or rc1 == 1
    # call 2: a smaller problem (16 x 12), one shift, LGMRES
    pb = synth.mixing_layer_2d(16, 12, 0.5, 1000.0)
    cb = Context()
    cb.base_set(pb, dev(synth.random_base(pb, 63)))
    bb = synth.random_vector(pb, 64, stream=1)
    (rc0, i0, x0), (rc1, i1, x1) = _pair(cb, pb, [0.2], dev(bb), restart=15, augment=2, tol=1e-9,
                                         max_matvec=3000)
    print("call 2:", rc0, i0[0]["iters"], i0[0]["relres"])
    assert rc0 == rc1 and i0 == i1
    assert np.array_equal(x0, x1)
    # call 3: FP32 GMRES inside FP64 refinement on the same small problem
    (rc0, i0, x0), (rc1, i1, x1) = _pair(cb, pb, [0.2], dev(bb), restart=15, tol=1e-10, max_matvec=5000,
                                         prec=SA_MIXED, inner_tol=1e-4)
    print("call 3:", rc0, i0[0]["outer"], i0[0]["relres"])
    assert rc0 == rc1 and i0 == i1
    assert np.array_equal(x0, x1)
    ca.close()
    cb.close()


def test_noalloc_refuses_oversize_workspace():
    need_gpu()
    from paper_1502_03701_amd import Context, SAError
    from paper_1502_03701_amd import _native as n
    prob = synth.mixing_layer_2d(256, 256, 0.5, 1000.0)   # n = 262 144: 41 columns are 86 MB
    ctx = Context()
    ctx.base_set(prob, dev(synth.base_flow(prob)))
    b = dev(synth.random_vector(prob, 65, stream=1))
    x = torch.zeros_like(b)
    with pytest.raises(SAError) as e:
        ctx.gmres_solve([0.2], b, x, restart=40, noalloc=True)
    assert e.value.code == n.SA_EINVAL and "scratch" in str(e.value)
    ctx.close()
