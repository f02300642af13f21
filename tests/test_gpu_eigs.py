"""Parity of the HIP Cayley-IRAM eigenpairs with the oracle's dense spectrum
(LAPACK eigenvalues of the oracle's Jacobian, tests/golden/spectrum_*.txt).

Rule for degenerate eigenvalues (the KH mode of the symmetric layer is an
exact double eigenvalue; Krylov methods return one or two copies depending
on rounding): every returned lambda must lie within 1e-8 (relative, floor
1e-3) of an eigenvalue of the dense spectrum, and the distinct returned
values (clustered at 1e-6) must be the leading distinct eigenvalues by
|theta|."""
import os

import numpy as np
import pytest

import synth
from gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    a = np.loadtxt(os.path.join(GOLDEN, "spectrum_%s.txt" % name))
    return a[:, 0] + 1j * a[:, 1]


def distinct(vals, tol=1e-6):
    out = []
    for v in vals:
        if all(abs(v - u) > tol * max(abs(u), 1e-3) for u in out):
            out.append(v)
    return out


def check(lams, ref, n_leading):
    for l in lams:
        d = np.min(np.abs(ref - l)) / max(abs(l), 1e-3)
        assert d < 1e-8, (l, d)
    got = distinct(lams)
    want = distinct(ref)[:n_leading]
    for w in want:
        assert any(abs(w - g) < 1e-8 * max(abs(w), 1e-3) for g in got), (w, got)


def run(prob, nev, ncv, prec=0, max_restarts=50, evecs=False, lin_tol=1e-12, restart=40):
    from paper_1502_03701_amd import Context, arnoldi_eigs
    q0 = synth.base_flow(prob)
    ctx = Context()
    ctx.base_set(prob, dev(q0))
    v0 = dev(synth.random_vector(prob, 0))
    ev = None
    if evecs:
        ev = [(torch.zeros(nev * prob.ndof, dtype=torch.float64, device="cuda:0"),
               torch.zeros(nev * prob.ndof, dtype=torch.float64, device="cuda:0"))]
    rc, res = arnoldi_eigs([ctx], [v0], nev=nev, ncv=ncv, sigma=0.2, mu=-0.2, tol=1e-10,
                           max_restarts=max_restarts, restart=restart, lin_tol=lin_tol,
                           prec=prec, inner_tol=1e-4, max_outer=20, evecs=ev)
    return rc, res[0], ev


def test_kh_pair_fp64():
    need_gpu()
    prob = synth.mixing_layer_2d(24, 24, 0.3, 500.0)
    rc, r, ev = run(prob, nev=2, ncv=16, evecs=True)
    assert rc == 0 and r["nconv"] >= 2
    check(r["lam"], golden("kh_24x24_M0.3_Re500"), 1)
    assert all(x < 1e-8 for x in r["resid"])
    assert all(abs(l.imag) < 1e-9 for l in r["lam"])


def test_kh_pair_mixed_matches_fp64():
    need_gpu()
    from paper_1502_03701_amd import SA_MIXED
    prob = synth.mixing_layer_2d(32, 32, 0.5, 1000.0)
    rc64, r64, _ = run(prob, nev=2, ncv=16)
    rcm, rm, _ = run(prob, nev=2, ncv=16, prec=SA_MIXED)
    assert rc64 == 0 and rcm == 0
    ref = golden("kh_32x32_M0.5_Re1000")
    check(r64["lam"], ref, 1)
    check(rm["lam"], ref, 1)
    for a, b in zip(sorted(r64["lam"], key=abs), sorted(rm["lam"], key=abs)):
        assert abs(a - b) / abs(a) < 1e-8


def test_restart_budget_partial_result():
    need_gpu()
    from paper_1502_03701_amd import SA_NOT_CONVERGED
    prob = synth.mixing_layer_2d(24, 24, 0.3, 500.0)
    rc, r, _ = run(prob, nev=6, ncv=10, max_restarts=0)
    assert rc == SA_NOT_CONVERGED and r["restarts"] == 0
    assert r["n_cayley"] == 10


def test_bad_options():
    need_gpu()
    from paper_1502_03701_amd import Context, SAError, arnoldi_eigs
    prob = synth.mixing_layer_2d(12, 12, 0.3, 500.0)
    ctx = Context()
    ctx.base_set(prob, dev(synth.base_flow(prob)))
    v0 = dev(synth.random_vector(prob, 0))
    with pytest.raises(SAError):
        arnoldi_eigs([ctx], [v0], nev=6, ncv=7)
    with pytest.raises(SAError):
        arnoldi_eigs([ctx], [v0], nev=2, ncv=10, sigma=0.3, mu=0.3)


@pytest.mark.slow
def test_c0_leading_four():
    """C0 (48x48, M=0.3, Re=500): the KH pair and its harmonic (two double
    eigenvalues, |theta| = 11.0 and 2.24); the remaining spectrum lies in
    the |theta| ~ 1 ring."""
    need_gpu()
    rc, r, _ = run(synth.config0(), nev=4, ncv=20, lin_tol=1e-12)
    assert rc == 0
    check(r["lam"], golden("c0_48x48_M0.3_Re500"), 2)


def test_concurrent_problems_match_sequential():
    """Problems on pairwise distinct streams run concurrently (one host
    thread each) and give the same eigenvalues, bit for bit, as the same
    problems run in turn on one stream."""
    need_gpu()
    from paper_1502_03701_amd import Context, arnoldi_eigs
    items = synth.config4_reduced(count=3, sides=(16, 20))
    def setup(streams):
        ctxs, v0s = [], []
        for it, st in zip(items, streams):
            c = Context(stream=st)
            c.base_set(it.problem, dev(synth.base_flow(it.problem)))
            ctxs.append(c)
            v0s.append(dev(synth.random_vector(it.problem, it.seed)))
        return ctxs, v0s
    kw = dict(nev=2, ncv=12, sigma=0.2, mu=-0.2, tol=1e-9, max_restarts=40, restart=30, lin_tol=1e-11)
    ctxs, v0s = setup([torch.cuda.current_stream()] * len(items))
    rc1, r1 = arnoldi_eigs(ctxs, v0s, **kw)
    streams = [torch.cuda.Stream() for _ in items]
    ctxs2, v0s2 = setup(streams)
    torch.cuda.synchronize()
    rc2, r2 = arnoldi_eigs(ctxs2, v0s2, **kw)
    assert rc1 == rc2
    for a, b in zip(r1, r2):
        assert a["lam"] == b["lam"] and a["n_matvec"] == b["n_matvec"]
        assert a["seconds"] > 0 and b["seconds"] > 0
    # a mix of shared and distinct streams is refused
    from paper_1502_03701_amd import SAError
    with pytest.raises(SAError):
        arnoldi_eigs([ctxs[0], ctxs[1], ctxs2[2]], v0s, **kw)
