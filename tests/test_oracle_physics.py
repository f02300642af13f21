"""Physics pin: the Kelvin-Helmholtz growth rate of the tanh layer against
the growth rates the paper prints (Section "Validation", Table 2).

Inviscid cases, alpha = 2 pi / 15.83 (L1 = 15.83 delta, Section "Numerical
Experiments"), walls at y = +-15.  The discrete operator differs from the
paper's (explicit instead of compact staggered differences, walls instead of
non-reflective boundaries), so the check is a band around the printed values,
not equality.  The symmetric layer makes the KH eigenvalue real and double.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as ssl

import synth
from oracle import operator as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_growth_rates.txt")


def table2():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            t = line.split()
            out[t[0]] = dict(mach=float(t[1]), re=float(t[2]), computed=float(t[4]),
                             blumen=float(t[5]), mack=float(t[6]))
    return out


def kh_eigenvalues(mach, guess, ny=256):
    prob = synth.mixing_layer_2d(8, ny, mach, 0.0, lx=15.83)
    S = op.sparse_jacobian(prob, synth.base_flow(prob))
    idx = op.interior_index(prob)
    Si = S[idx][:, idx].tocsc()
    w = ssl.eigs(Si, k=4, sigma=guess, return_eigenvectors=False)
    return w[np.argsort(-w.real)][:2]


@pytest.mark.parametrize("case,band", [("V01", 0.005), ("V02", 0.002)])
def test_kh_growth_rate_against_table2(case, band):
    ref = table2()[case]
    lam = kh_eigenvalues(ref["mach"], ref["mack"] + 0.003)
    assert np.all(np.abs(lam.imag) < 1e-8)                 # real
    assert abs(lam[0] - lam[1]) < 1e-8                      # double
    assert abs(lam[0].real - ref["mack"]) < band
    assert abs(lam[0].real - ref["computed"]) < band + 0.002
