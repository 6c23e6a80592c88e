"""Write the stored expected values of the full-size parity tests.

Every number written here comes from the FP64 CPU oracle (oracle/gdm_oracle.py)
on the seeded inputs of gdm_inputs; nothing is taken from the GPU path.

    python tests/golden/make_golden.py config4_adjoint   # ~2-3 min on 8 cores
    python tests/golden/make_golden.py config2_samples   # ~2-4 min, ~8 GB RAM
    python tests/golden/make_golden.py config3_samples   # ~10-20 min

config4_adjoint.npz: loss L = sigma_sca + (1/P) sum_p |E_tot(r_p)|^2 / |E0|^2 of
  the 2000-cell cuboid (10 x 10 x 20 cells, 8 nm, eps 10+0.05i, 700 nm, 4096
  probes) and its gradient w.r.t. all 6000 cell coordinates, Re/Im eps of every
  cell and the wavelength (the oracle's hand-written FP64 adjoint).
config2_samples.npz: the 12 000-unknown random-aspect cuboid (seed 2, 66 plane
  waves): cross sections of every RHS, the 2-norm of every column of q and F,
  and q, F at 97 seeded sample unknowns for every RHS.
config3_samples.npz: 64 seeded (structure, wavelength) items of the 32-structure
  x 128-wavelength batch (Drude-Lorentz permittivities, 10 nm cells): the
  extinction, scattering and absorption cross sections of both polarisations.
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


def config3_samples():
    """64 seeded (structure, wavelength) items of the 32 x 128 batch: oracle
    cross sections (ext, sca, abs) of both polarisations."""
    w = gi.config3()
    rng = np.random.default_rng(3333)
    ns, nw = w["eps"].shape
    items = sorted({(int(a), int(b)) for a, b in zip(rng.integers(0, ns, 200), rng.integers(0, nw, 200))})
    items = [items[i] for i in sorted(rng.choice(len(items), 64, replace=False))]
    cs = np.zeros((64, len(w["khat"]), 3))
    r_eff, a_eff = np.zeros((0, 3)), np.zeros((0, 6, 6), dtype=np.complex128)
    for t, (si, li) in enumerate(items):
        r = w["structs"][si]["r_cell"]
        wl = dict(r_cell=r, step=w["step"], eps_cell=np.full(len(r), w["eps"][si, li]), n_env=w["n_env"],
                  wavelength=float(w["wavelengths"][li]), khat=w["khat"], e0=w["e0"], r_eff=r_eff, alpha_eff=a_eff)
        sim = O.simulate(wl)
        cs[t, :, 0], cs[t, :, 1], cs[t, :, 2] = sim["ext"], sim["sca"], sim["abs"]
        print(f"  item {t}: structure {si} ({len(r)} cells), wavelength {li}", flush=True)
    np.savez_compressed(os.path.join(HERE, "config3_samples.npz"), items=np.array(items), cs=cs)


if __name__ == "__main__":
    jobs = {"config4_adjoint": config4_adjoint, "config2_samples": config2_samples,
            "config3_samples": config3_samples}
    for name in sys.argv[1:] or list(jobs):
        print("writing", name, flush=True)
        jobs[name]()
