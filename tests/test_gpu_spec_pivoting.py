"""Speculative partial pivoting (the default panel mode of gdm_factorize):
the diagonal taken as every column's pivot, each checked against the partial
pivoting rule, the factorisation repeated with the pivot search when a check
fails.  Dielectric structures pass every check (their coupling matrices keep
the diagonal as partial pivoting's choice); a plasmonic sphere near its
dipole resonance (eps = -2 + 0.1i) does not and must fall back.  Either way
the results equal the oracle's within 1e-10 and those of the pivot search.
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


def relcol(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def workload(which):
    if which == "config1":
        return gi.config1()
    if which == "mixed":
        return gi.small_mixed()
    if which == "config4_cells":  # 8 x 8 x 16 cells, n = 3072: 24 blocks of 128 (config1: 771, a 3-column tail)
        w = dict(gi.config4())
        w["r_cell"] = gi.cuboid_cells(8, 8, 16, 8.0)
        w["eps_cell"] = np.full(len(w["r_cell"]), 10.0 + 0.05j)
        w["eps_cell"][::5] += 3.0 + 0.2j
        return w
    if which == "plasmonic":
        w = gi.config1()
        return dict(w, eps_cell=np.full(len(w["r_cell"]), -2.0 + 0.1j))
    if which == "plasmonic_eps4":
        w = gi.config1()
        return dict(w, eps_cell=np.full(len(w["r_cell"]), -4.0 + 0.5j))
    raise ValueError(which)


def factor_and_solve(ctx, w, prec, mode):
    from paper_2505_09545_amd import gdm
    r_eff = w.get("r_eff")
    ne = 0 if r_eff is None else len(r_eff)
    ctx.set_pivoting(mode)
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]),
                      torch.as_tensor(r_eff) if ne else None, torch.as_tensor(w["alpha_eff"]) if ne else None)
    before = ctx.pivot_fallbacks()
    ctx.factorize(w["wavelength"], prec)
    fell_back = ctx.pivot_fallbacks() - before
    khat, e0, e2 = gdm.plane_wave_inputs(w, ctx)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve(f0, tol=1e-14 if prec == gdm.PREC_FP32_IR else 0.0)
    ctx.set_pivoting(0)
    return q.cpu().numpy(), f.cpu().numpy(), fell_back


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("which,expect_fallback", [("config1", 0), ("mixed", 0), ("config4_cells", 0),
                                                    ("plasmonic", 1), ("plasmonic_eps4", 1)])
def test_speculative_pivots_match_oracle_and_pivot_search(ctx, which, expect_fallback, prec):
    w = workload(which)
    say("speculative pivoting", which, "prec", prec)
    q0, f0, fb0 = factor_and_solve(ctx, w, prec, 0)
    print("  n", ctx.n, "fallbacks", fb0, flush=True)
    assert fb0 == expect_fallback
    q1, f1, fb1 = factor_and_solve(ctx, w, prec, 1)
    assert fb1 == 0
    sim = O.simulate(w)
    assert relcol(q0, sim["q"].T) < 1e-10
    assert relcol(f0, sim["F"].T) < 1e-10
    # same pivots, same algorithm: the two modes agree to rounding
    assert relcol(q0, q1) < (1e-12 if prec == 0 else 1e-10)
