"""GPU parity of the point-dipole sources, the LDOS and the scattered Green's
tensor of the structured environment (gdm_dipole_sources, gdm_ldos,
gdm_green_tensor through the C-ABI) against the FP64 oracle.

Tolerances: the incident field of a source within 1e-13 relative (a closed
form per dipole); the LDOS within 1e-10 absolute (values of order 1) and the
Green's tensor within 1e-10 of its largest entry, in FP64 mode and after FP32
LU + FP64 refinement (the bar of the method's FP64 mode).
"""
import sys

import numpy as np
import pytest

import gdm_inputs as gi
from oracle import gdm_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_09545_amd import gdm
    c = gdm.Context(0)
    yield c
    c.close()


def workload(which):
    if which == "cells":
        w = dict(gi.config1())
        w["r_cell"] = gi.cuboid_cells(4, 3, 3, 15.0)
        w["step"] = 15.0
        w["eps_cell"] = np.full(len(w["r_cell"]), 9.0 + 0.4j)
        w["eps_cell"][::4] += 3.0
        w["n_env"] = 1.2
        w["wavelength"] = 520.0
        return w
    if which == "mixed":
        return gi.small_mixed()
    raise ValueError(which)


SOURCES = np.array([[30.0, -20.0, 65.0], [-45.0, 35.0, -58.0], [0.0, 0.0, 90.0]])
POINTS = np.array([[-50.0, 10.0, 80.0], [5.0, 60.0, -40.0], [70.0, -70.0, 0.0], [0.0, 0.0, 90.0]])


def setup(ctx, w, prec):
    r_eff = w.get("r_eff")
    ne = 0 if r_eff is None else len(r_eff)
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]),
                      torch.as_tensor(r_eff) if ne else None, torch.as_tensor(w["alpha_eff"]) if ne else None)
    ctx.factorize(w["wavelength"], prec)


@pytest.mark.parametrize("which", ["cells", "mixed"])
def test_dipole_source_field_matches_oracle(ctx, which):
    from paper_2505_09545_amd import gdm
    w = workload(which)
    say("dipole sources", which)
    setup(ctx, w, gdm.PREC_FP64)
    rng = np.random.default_rng(3)
    d = rng.standard_normal((len(SOURCES), 6)) + 1j * rng.standard_normal((len(SOURCES), 6))
    f0 = ctx.dipole_sources(torch.as_tensor(SOURCES), torch.as_tensor(d)).cpu().numpy()
    D = O.Dipoles(w)
    ref = O.dipole_source_at_dipoles(D, SOURCES, d).T
    assert np.max(np.abs(f0 - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("which", ["cells", "mixed"])
def test_ldos_and_green_tensor_match_oracle(ctx, which, prec):
    w = workload(which)
    say("ldos / green", which, "prec", prec)
    setup(ctx, w, prec)
    tol = 1e-14 if prec == 1 else 0.0
    L = ctx.ldos(torch.as_tensor(SOURCES), tol=tol).cpu().numpy()
    Lo = O.ldos(w, SOURCES)
    print("  ldos range", float(L.min()), float(L.max()), flush=True)
    assert np.max(np.abs(L - Lo)) < 1e-10
    G = ctx.green_tensor(torch.as_tensor(SOURCES), torch.as_tensor(POINTS), tol=tol).cpu().numpy()
    Go, _ = O.green_scattered(w, SOURCES, POINTS)
    assert np.max(np.abs(G - Go)) < 1e-10 * np.max(np.abs(Go))


def test_ldos_radiative_lossless_energy_balance(ctx):
    """With lossless cells and the radiative self-term the GPU LDOS equals the
    oracle's far-field power ratio (energy conservation, the oracle's pin)."""
    from paper_2505_09545_amd import gdm
    w = workload("cells")
    w["eps_cell"] = np.full(len(w["r_cell"]), 9.0 + 0j)
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]), None, None,
                      selfterm=gdm.SELF_RADIATIVE)
    ctx.factorize(w["wavelength"], gdm.PREC_FP64)
    say("ldos radiative lossless")
    L = ctx.ldos(torch.as_tensor(SOURCES[:1])).cpu().numpy()
    Lo = O.ldos(w, SOURCES[:1], mode="radiative")
    assert np.max(np.abs(L - Lo)) < 1e-10


def test_sources_errors(ctx):
    from paper_2505_09545_amd import gdm
    w = workload("cells")
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]))
    say("sources: errors")
    with pytest.raises(gdm.GDMError) as ei:  # structure replaced: no factors
        ctx.ldos(torch.as_tensor(SOURCES))
    assert ei.value.status == gdm.GDM_E_STATE
    ctx.factorize(w["wavelength"])
    with pytest.raises(gdm.GDMError) as ei:  # a source on a cell
        ctx.ldos(torch.as_tensor(w["r_cell"][:1]))
    assert ei.value.status == gdm.GDM_E_PROBE_AT_DIPOLE
    with pytest.raises(gdm.GDMError) as ei:  # a point on a cell
        ctx.green_tensor(torch.as_tensor(SOURCES[:1]), torch.as_tensor(w["r_cell"][3:4]))
    assert ei.value.status == gdm.GDM_E_PROBE_AT_DIPOLE
