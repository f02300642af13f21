"""Pin of the oracle's viscous, heat-conduction and dissipation terms (CPU).

The closed-form pins of test_oracle_operator.py use uniform temperature or
parallel flows, where every mu'(T) and lambda'(T) term, and the dependence of
mu and lambda on a perturbed temperature, drop out.  Here the oracle's discrete
N(q) (expanded viscous form, chain rule for grad mu and grad lambda, the
(gamma - 1) form of the pressure equation's heat term) is compared with an
independent restatement of eq. navier_stokes in its printed, un-expanded form
(assembled tau_ij, d_j tau_ij, d_j(lambda d_j T), Phi = tau_ij s_ij, the factor
p/c_v) with Fourier-spectral derivatives, on all-periodic grids and smooth
fields with O(1) temperature variation, shear and divergence.  The 6th-order
differences must converge to it at 6th order in every component: the error
falls by about 2^6 = 64 per grid doubling.  The same holds for the linearised
operator: the oracle's complex-step J(q0)v against the complex-step
derivative of the spectral reference about the same non-uniform base.

A term with a wrong sign, coefficient or factor leaves an O(1) error that does
not converge; the last test plants four such mistakes in a copy of the oracle
and checks that each one is caught.
"""
import types

import numpy as np
import pytest

import synth
from oracle import operator as op
from spectral_ref import rhs_spectral, smooth_state

P = synth.BC_PERIODIC


def _prob(ndim, n, re=20.0):
    # unequal periods, so that a spacing mix-up between axes shows
    if ndim == 2:
        return synth.Problem(ndim=2, n=(n, n, 1), length=(2 * np.pi, 2.6 * np.pi, 1.0),
                             mach=0.5, re=re, bc=(P, P, P))
    return synth.Problem(ndim=3, n=(n, n, n), length=(2 * np.pi, 2.6 * np.pi, 1.6 * np.pi),
                         mach=0.5, re=re, bc=(P, P, P))


# grid pairs (n, 2n) in the asymptotic range of the 6th-order stencils
GRIDS = {2: (64, 128), 3: (24, 48)}
# error after refinement (relative to the component's max), and the
# accepted band for the error ratio of one doubling (2^6 = 64)
FINE_TOL = {2: 1e-7, 3: 2e-5}
RATIO_BAND = (30.0, 100.0)


def _jv_spectral(prob, q0, v, h=1e-30):
    return np.imag(rhs_spectral(prob, q0 + 1j * h * v)) / h


def _errors(mod, ndim, linear):
    out = []
    for n in GRIDS[ndim]:
        prob = _prob(ndim, n)
        q0 = smooth_state(prob, 0)
        if linear:
            v = smooth_state(prob, 1) - q0
            a, b = mod.jv_cstep(prob, q0, v), _jv_spectral(prob, q0, v)
        else:
            a, b = mod.rhs(prob, q0), rhs_spectral(prob, q0).real
        out.append(np.array([np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()
                             for k in range(prob.nv)]))
    return out[0], out[1]


def _converges(mod, ndim, linear):
    coarse, fine = _errors(mod, ndim, linear)
    ratio = coarse / fine
    ok = bool(np.all(fine < FINE_TOL[ndim]) and np.all(ratio > RATIO_BAND[0])
              and np.all(ratio < RATIO_BAND[1]))
    return ok, coarse, fine, ratio


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("linear", [False, True], ids=["N", "Jv"])
def test_oracle_converges_to_spectral_reference(ndim, linear):
    ok, coarse, fine, ratio = _converges(op, ndim, linear)
    print(f"\n{ndim}D {'Jv' if linear else 'N'}: errors {coarse} -> {fine}, ratios {ratio}")
    assert ok


@pytest.mark.parametrize("ndim", [2, 3])
def test_spectral_reference_is_resolved(ndim):
    # the reference on n and on 2n points agrees at the common points far
    # better than the finite differences do, so the convergence above measures
    # the finite differences, not the reference
    n = GRIDS[ndim][0]
    pc, pf = _prob(ndim, n), _prob(ndim, 2 * n)
    coarse = rhs_spectral(pc, smooth_state(pc)).real
    fine = rhs_spectral(pf, smooth_state(pf)).real
    fd = op.rhs(pc, smooth_state(pc))
    sub = fine[(slice(None),) + (slice(None, None, 2),) * ndim]
    for k in range(coarse.shape[0]):
        ref_err = np.abs(sub[k] - coarse[k]).max()
        assert ref_err < 0.05 * np.abs(fd[k] - coarse[k]).max()
        assert ref_err < (1e-10 if ndim == 2 else 1e-5) * np.abs(coarse[k]).max()


def test_spectral_reference_uniform_state_is_steady():
    prob = _prob(3, 12)
    q = np.zeros(prob.shape)
    q[0] = 1.3 / (1.4 * 0.25)
    q[1], q[2], q[3], q[4] = 0.4, -0.2, 0.1, 0.3
    assert np.abs(rhs_spectral(prob, q)).max() < 1e-12


# planted mistakes: (description, exact text in the oracle, replacement)
MUTATIONS = [
    ("sign of the -2/3 grad T div u term of the stress divergence",
     "(cross - (2.0 / 3.0) * DT[i] * theta)", "(cross + (2.0 / 3.0) * DT[i] * theta)"),
    ("coefficient of lambda'(T) |grad T|^2 in the heat flux divergence",
     "Q = lam * LT + dlam *", "Q = lam * LT + 0.5 * dlam *"),
    ("coefficient of div(u)^2 in the dissipation",
     "- (2.0 / 3.0) * theta * theta)", "- (1.0 / 3.0) * theta * theta)"),
    ("heat / (rho T) replaced by heat / rho in the entropy equation",
     "heat / (rho * T)", "heat / rho"),
]


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(what, old, new):
    src = open(op.__file__).read()
    assert src.count(old) == 1, f"oracle text for '{what}' not found"
    mutant = types.ModuleType("oracle_operator_mutant")
    exec(compile(src.replace(old, new), "oracle_operator_mutant", "exec"), mutant.__dict__)
    for ndim in (2, 3):
        for linear in (False, True):
            ok, *_ = _converges(mutant, ndim, linear)
            assert not ok, f"{what} not caught ({ndim}D, {'Jv' if linear else 'N'})"
