"""Write the reference spectra the eigen parity tests compare against.

Calls only the oracle (dense Jacobian by complex step) and LAPACK (scipy's
eigvals) -- no GPU code.  Output: one text file per case with the 12
eigenvalues of J of largest |theta|, theta = (lam - mu)/(lam - sigma),
sigma = 0.2, mu = -0.2.  Run:  python tests/golden/make_spectra.py
"""
import os
import sys

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import operator as op  # noqa: E402

CASES = {
    "c0_48x48_M0.3_Re500": (synth.config0(), "tanh"),
    "kh_24x24_M0.3_Re500": (synth.mixing_layer_2d(24, 24, 0.3, 500.0), "tanh"),
    "kh_32x32_M0.5_Re1000": (synth.mixing_layer_2d(32, 32, 0.5, 1000.0), "tanh"),
    # reduced 3D: the workload's base (tanh layer plus 1e-3 N(0,1) spanwise
    # velocity from seed 2) on a 16 x 16 x 8 grid (n = 8 960 interior DOFs)
    "3d_16x16x8_M0.5_Re1000_w": (synth.mixing_layer_3d(16, 16, 8, 0.5, 1000.0), "tanh_w"),
}


def main(names=None):
    for name, (prob, kind) in CASES.items():
        if names and name not in names:
            continue
        q0 = synth.base_flow(prob, seed=2, w_noise=1e-3) if kind == "tanh_w" else synth.base_flow(prob)
        J = op.dense_jacobian(prob, q0, batch=256)
        lam = sla.eigvals(J)
        th = (lam + 0.2) / (lam - 0.2)
        o = np.argsort(-np.abs(th), kind="stable")[:12]
        path = os.path.join(HERE, "spectrum_%s.txt" % name)
        with open(path, "w") as f:
            f.write("# eigenvalues of the oracle's dense J (LAPACK), largest |theta| first\n")
            f.write("# written by tests/golden/make_spectra.py; sigma = 0.2, mu = -0.2\n")
            f.write("# re im |theta|\n")
            for i in o:
                f.write("%.17e %.17e %.17e\n" % (lam[i].real, lam[i].imag, abs(th[i])))
        print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1:])
