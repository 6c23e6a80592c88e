"""Write the stored expected values of the full-size parity tests.

Every number written here comes from the FP64 CPU oracle (oracle/gdm_oracle.py)
on the seeded inputs of gdm_inputs; nothing is taken from the GPU path.

    python tests/golden/make_golden.py config4_adjoint   # ~2-3 min on 8 cores
    python tests/golden/make_golden.py config2_samples   # ~2-4 min, ~8 GB RAM

config4_adjoint.npz: loss L = sigma_sca + (1/P) sum_p |E_tot(r_p)|^2 / |E0|^2 of
  the 2000-cell cuboid (10 x 10 x 20 cells, 8 nm, eps 10+0.05i, 700 nm, 4096
  probes) and its gradient w.r.t. all 6000 cell coordinates, Re/Im eps of every
  cell and the wavelength (the oracle's hand-written FP64 adjoint).
config2_samples.npz: the 12 000-unknown random-aspect cuboid (seed 2, 66 plane
  waves): cross sections of every RHS, the 2-norm of every column of q and F,
  and q, F at 97 seeded sample unknowns for every RHS.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gdm_inputs as gi  # noqa: E402
from oracle import gdm_oracle as O  # noqa: E402


def config4_adjoint():
    w = gi.config4()
    g = O.adjoint_gradient(w)
    np.savez_compressed(os.path.join(HERE, "config4_adjoint.npz"), r=g["r"], eps_re=g["eps_re"],
                        eps_im=g["eps_im"], wavelength=np.array([g["wavelength"]]), loss=np.array([g["loss"]]))


def config2_samples():
    w = gi.config2()
    s = O.simulate(w)
    n = s["q"].shape[0]
    idx = np.sort(np.random.default_rng(1234).choice(n, size=97, replace=False))
    np.savez_compressed(os.path.join(HERE, "config2_samples.npz"), idx=idx, q=s["q"][idx].T, F=s["F"][idx].T,
                        q_norm=np.linalg.norm(s["q"], axis=0), F_norm=np.linalg.norm(s["F"], axis=0),
                        ext=s["ext"], sca=s["sca"], abs=s["abs"], rad=s["rad"])


if __name__ == "__main__":
    jobs = {"config4_adjoint": config4_adjoint, "config2_samples": config2_samples}
    for name in sys.argv[1:] or list(jobs):
        print("writing", name, flush=True)
        jobs[name]()
