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


def kh_eigenvalues(mach, guess, ny=256, nx=8, lx=15.83, re=0.0):
    prob = synth.mixing_layer_2d(nx, ny, mach, re, lx=lx)
    S = op.sparse_jacobian(prob, synth.base_flow(prob))
    idx = op.interior_index(prob)
    Si = S[idx][:, idx].tocsc()
    w = ssl.eigs(Si, k=4, sigma=guess, return_eigenvectors=False)
    return w[np.argsort(-w.real)][:2]


# The validation domain holds one wavelength of the least stable mode
# (Section "Model problem").  At M = 0.1 and 0.5 that is L1 = 15.83
# (alpha = 0.397, Section "Numerical Experiments").  At M = 0.9 the least
# stable wavenumber lies near alpha = 0.2 (this discretisation: growth
# 0.0535 / 0.0548 / 0.0551 / 0.0551 / 0.0545 at alpha = 0.17 / 0.19 / 0.2 /
# 0.21 / 0.23, the same to 1e-5 on 512 and 1024 points in y), while at
# alpha = 0.397 the leading eigenvalues are complex and change with the
# resolution; so the M = 0.9 rows use alpha = 0.2.  The 16 x 64 rows run on
# a uniform grid (dy = 0.48) where the paper stretched its grid to a minimum
# spacing of 0.08 delta, hence the wider bands there.
#   case: (nx, ny, Lx, band around Mack's value, band around the paper's)
ROWS = {
    "V01": (8, 256, 15.83, 0.005, 0.007),
    "V02": (8, 256, 15.83, 0.002, 0.002),
    "V03": (8, 512, 2 * np.pi / 0.2, 0.001, 0.001),
    "V05": (16, 64, 15.83, 0.005, 0.005),
    "V06": (16, 64, 15.83, 0.002, 0.003),
    "V07": (16, 64, 2 * np.pi / 0.2, 0.008, 0.008),
}


@pytest.mark.parametrize("case", sorted(ROWS))
def test_kh_growth_rate_against_table2(case):
    ref = table2()[case]
    nx, ny, lx, band_mack, band_paper = ROWS[case]
    lam = kh_eigenvalues(ref["mach"], ref["mack"] + 0.003, ny=ny, nx=nx, lx=lx)
    print(f"\n{case}: M={ref['mach']} {nx}x{ny} Lx={lx:.3f}: {lam[0].real:.5f} "
          f"(paper {ref['computed']}, Mack {ref['mack']})")
    assert np.all(np.abs(lam.imag) < 1e-8)                 # real
    assert abs(lam[0] - lam[1]) < 1e-8                      # double
    assert abs(lam[0].real - ref["mack"]) < band_mack
    assert abs(lam[0].real - ref["computed"]) < band_paper


@pytest.mark.parametrize("case,ny,nx", [("V04", 256, 8), ("V08", 64, 16)])
def test_viscous_rows_damp_the_kh_mode(case, ny, nx):
    """V04 / V08 (M = 0.5, Re = 1000).  With Re read on delta and u_inf
    (mu_ref = 1/Re) the viscous terms lower the growth rate by about 1 %
    (0.1395 on 8 x 256, against 0.1412 inviscid), whereas the paper prints
    0.1273 / 0.1270 (Mack 0.1271); this discretisation gives that rate only
    near Re = 100 (0.1267).  The paper states neither the scales of its
    Reynolds number nor its viscous base state, so the printed value is not
    pinned (parity unpinned); this test checks the sign and size of the
    viscous correction and that the mode stays real and double."""
    ref = table2()[case]
    inv = kh_eigenvalues(0.5, 0.144, ny=ny, nx=nx)
    visc = kh_eigenvalues(0.5, 0.142, ny=ny, nx=nx, re=ref["re"])
    print(f"\n{case}: inviscid {inv[0].real:.5f}, Re={ref['re']:.0f} {visc[0].real:.5f} "
          f"(paper {ref['computed']})")
    assert np.all(np.abs(visc.imag) < 1e-8) and abs(visc[0] - visc[1]) < 1e-8
    assert 0.0005 < inv[0].real - visc[0].real < 0.005
