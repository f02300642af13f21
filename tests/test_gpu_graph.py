"""Captured GMRES cycles (hipGraph replay) give bit-for-bit the results of the
plain launches.  Each graph is replayed several times, with other eager work
(operator calls, solves into other buffers, torch kernels) and synchronisations
between the replays, and every replay is checked against the eager result."""
import numpy as np
import pytest

import synth
from gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    need_gpu()
    from paper_1502_03701_amd import Context
    prob = synth.mixing_layer_2d(16, 14, 0.3, 500.0)
    q0 = synth.random_base(prob, 41)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    return prob, q0, ctx


def _eager_noise(ctx, prob, k):
    """Unrelated work on the same stream between graph replays."""
    v = dev(synth.random_vector(prob, 100 + k))
    y = torch.empty_like(v)
    ctx.op_apply(v, y, shift=0.1 * k)
    t = torch.randn(4096, device="cuda:0").cumsum(0)
    torch.cuda.synchronize()
    return float(t[-1]) + float(y.sum())


def _check_replays(ctx, prob, solve, ref_x, ref_info, n_replay=3):
    for k in range(n_replay):
        _eager_noise(ctx, prob, k)
        x, info = solve()
        assert np.array_equal(host(x), ref_x), "replay %d differs" % k
        for a, b in zip(info, ref_info):
            assert a["iters"] == b["iters"] and a["matvecs"] == b["matvecs"]
            assert a["relres"] == b["relres"] and a["status"] == b["status"]


@pytest.mark.parametrize("restart,max_matvec", [(7, 10 ** 5), (9, 31)])
def test_graph_fp64_multishift(setup, restart, max_matvec):
    prob, q0, ctx = setup
    sig = [0.05, 0.2, 0.35]
    B = dev(synth.random_vector(prob, 42, nrhs=3))

    def solve(graph):
        X = torch.zeros(3 * prob.ndof, dtype=torch.float64, device="cuda:0")
        rc, info = ctx.gmres_solve(sig, B, X, restart=restart, tol=1e-10, max_matvec=max_matvec,
                                   use_graph=graph)
        return X, info

    Xe, ie = solve(False)
    assert ie[0]["cycles"] >= 3
    _check_replays(ctx, prob, lambda: solve(True), host(Xe), ie)


def test_graph_fp32_preconditioned_and_mixed(setup):
    """The small-block preconditioner stalls GMRES on this case (the oracle's
    preconditioned GMRES(6) stays near relres 0.96 for 17000 steps), so the
    preconditioned solves run on a small matvec budget: only equality of the
    two launch modes is checked there."""
    prob, q0, ctx = setup
    from paper_1502_03701_amd import SA_F32, SA_MIXED
    sig = [0.1, 0.3]
    ctx.precond_setup(sig, 4, 2, 1, diag_add=0.1, noise_std=0.01, seed=5)
    B = synth.random_vector(prob, 43, nrhs=2)
    B32 = dev(B, torch.float32)

    def solve32(graph):
        X = torch.zeros(2 * prob.ndof, dtype=torch.float32, device="cuda:0")
        rc, info = ctx.gmres_solve(sig, B32, X, restart=6, tol=1e-5, max_matvec=150, prec=SA_F32,
                                   use_precond=True, use_graph=graph)
        return X, info

    Xe, ie = solve32(False)
    assert ie[0]["cycles"] >= 2
    _check_replays(ctx, prob, lambda: solve32(True), host(Xe), ie)

    B64 = dev(B)
    for pc, budget in ((False, 10 ** 5), (True, 200)):
        def solvem(graph):
            X = torch.zeros(2 * prob.ndof, dtype=torch.float64, device="cuda:0")
            rc, info = ctx.gmres_solve(sig, B64, X, restart=8, tol=1e-10, max_matvec=budget, prec=SA_MIXED,
                                       inner_tol=1e-3, max_outer=30, use_precond=pc, use_graph=graph)
            return X, info

        Xe, ie = solvem(False)
        if not pc:
            assert ie[0]["outer"] >= 2 and ie[0]["status"] == 0
        _check_replays(ctx, prob, lambda: solvem(True), host(Xe), ie)


def test_graph_dropped_on_new_base(setup):
    """A second base state of the same grid reuses every buffer address; the
    cached graphs (which bake in the operator constants) must not be reused."""
    prob, q0, _ = setup
    from paper_1502_03701_amd import Context
    ctx = Context()
    b = dev(synth.random_vector(prob, 44))
    out = {}
    for mach in (0.3, 0.6):
        p = synth.mixing_layer_2d(16, 14, mach, 500.0)
        ctx.base_set(p, dev(synth.random_base(p, 45)))
        for graph in (True, False):
            x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda:0")
            ctx.gmres_solve([0.2], b, x, restart=5, tol=1e-10, max_matvec=600, use_graph=graph)
            out[mach, graph] = host(x)
    assert np.array_equal(out[0.3, True], out[0.3, False])
    assert np.array_equal(out[0.6, True], out[0.6, False])
    assert not np.array_equal(out[0.3, True], out[0.6, True])


def test_graph_eigs(setup):
    prob, q0, _ = setup
    from paper_1502_03701_amd import Context, arnoldi_eigs
    p = synth.mixing_layer_2d(24, 24, 0.3, 500.0)
    ctx = Context()
    ctx.base_set(p, dev(synth.base_flow(p)))
    v0 = dev(synth.random_vector(p, 0))
    res = {}
    for graph in (False, True, True):
        rc, r = arnoldi_eigs([ctx], [v0], nev=2, ncv=16, sigma=0.2, mu=-0.2, tol=1e-10, max_restarts=50,
                             restart=40, lin_tol=1e-12, use_graph=graph)
        assert rc == 0
        _eager_noise(ctx, p, 1)
        res.setdefault(graph, []).append(r[0])
    for r in res[True]:
        assert r["lam"] == res[False][0]["lam"]
        assert r["n_matvec"] == res[False][0]["n_matvec"]
