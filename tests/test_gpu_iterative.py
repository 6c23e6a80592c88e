"""GPU parity of the matrix-free iterative solver (gdm_solve_iterative through
the C-ABI) against the FP64 oracle.  The Krylov method reaches the solution of
the same linear system the oracle solves with LAPACK, so the oracle pins it.

Tolerances: moments, fields and cross sections within 1e-10 relative (the bar
of the method's FP64 mode), with GMRES run to a relative residual of 1e-13
(the forward error is at most the condition number, ~10^2 here, times that).
At n = 69 000 (no dense oracle) every sampled residual row is bounded by the
residual's 2-norm the solver reports plus the FP64 rounding of the row's terms.
"""
import os
import sys

import numpy as np
import pytest

import gdm_inputs as gi
from oracle import gdm_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
    if which == "config4_small":
        w = dict(gi.config4())
        w["r_cell"] = gi.cuboid_cells(4, 5, 6, 8.0)
        w["eps_cell"] = np.full(len(w["r_cell"]), 10.0 + 0.05j)
        w["eps_cell"][::3] += 2.0 + 0.3j
        w["khat"] = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]])
        w["e0"] = np.array([[1.0, 0.0, 0.0], [0.0, 1.0j, 0.0]], dtype=np.complex128)
        w["r_probe"] = gi.probe_plane(12, 12, 200.0, 200.0, -150.0)
        return w
    if which == "config5_replica":
        return gi.config5(sub=(48, 52), probes=40)
    raise ValueError(which)


def setup(ctx, w):
    r_eff = w.get("r_eff")
    ne = 0 if r_eff is None else len(r_eff)
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]),
                      torch.as_tensor(r_eff) if ne else None, torch.as_tensor(w["alpha_eff"]) if ne else None)
    ctx.set_wavelength(w["wavelength"])


@pytest.mark.parametrize("which", ["config1", "mixed", "config4_small", "config5_replica"])
def test_iterative_matches_oracle(ctx, which):
    from paper_2505_09545_amd import gdm
    w = workload(which)
    say("iterative vs oracle", which)
    setup(ctx, w)
    khat, e0, e2 = gdm.plane_wave_inputs(w, ctx)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve_iterative(w["wavelength"], f0, tol=1e-13)
    print("  n", ctx.n, "products", ctx.info.ir_iters, "relres", ctx.info.backward_err, flush=True)
    assert ctx.info.backward_err <= 1e-13
    sim = O.simulate(w)
    assert relcol(q.cpu().numpy(), sim["q"].T) < 1e-10
    assert relcol(f.cpu().numpy(), sim["F"].T) < 1e-10
    cs = ctx.cross_sections(f0, q, f, e2, want_ff=True).cpu().numpy()
    for col, key in ((0, "ext"), (1, "sca"), (2, "abs"), (3, "rad")):
        assert np.max(np.abs(cs[:, col] - sim[key]) / np.abs(sim[key])) < 1e-10, key
    rp = w.get("r_probe")
    if rp is not None and len(rp):
        E, H = ctx.fields(q, torch.as_tensor(rp))
        Es, Hs = O.scattered_fields(sim["D"], sim["q"], rp)
        assert relcol(E.cpu().numpy(), Es) < 1e-10
        assert relcol(H.cpu().numpy(), Hs) < 1e-10


def test_iterative_config2_vs_golden(ctx):
    """n = 12 000 (the benchmark structure), the two normal-incidence plane
    waves: moments and fields against the oracle values stored for them."""
    from paper_2505_09545_amd import gdm
    ref = np.load(os.path.join(GOLDEN, "config2_samples.npz"))
    w = gi.config2()
    w = dict(w, khat=w["khat"][:2], e0=w["e0"][:2])
    say("iterative config2, 2 RHS")
    setup(ctx, w)
    khat, e0, e2 = gdm.plane_wave_inputs(w, ctx)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve_iterative(w["wavelength"], f0, tol=1e-13)
    print("  products", ctx.info.ir_iters, "relres", ctx.info.backward_err, flush=True)
    qn = torch.linalg.vector_norm(q, dim=1).cpu().numpy()
    assert np.max(np.abs(qn - ref["q_norm"][:2]) / ref["q_norm"][:2]) < 1e-10
    idx = torch.as_tensor(ref["idx"], device=q.device)
    assert np.max(np.abs(q[:, idx].cpu().numpy() - ref["q"][:2]) / ref["q_norm"][:2, None]) < 1e-10
    assert np.max(np.abs(f[:, idx].cpu().numpy() - ref["F"][:2]) / ref["F_norm"][:2, None]) < 1e-10
    cs = ctx.cross_sections(f0, q, f, e2).cpu().numpy()
    for col, key in ((0, "ext"), (1, "sca"), (2, "abs")):
        assert np.max(np.abs(cs[:, col] - ref[key][:2]) / np.abs(ref[key][:2])) < 1e-10, key


def test_iterative_config5_full_size_residual_rows(ctx):
    """n = 69 000 without any n^2 storage: residual rows by the oracle's direct
    per-pair sums; |F0_u - (M F)_u| <= relres ||F0||_2 + 1e-12 (scale), where
    scale is the sum of the moduli of the row's terms."""
    from paper_2505_09545_amd import gdm
    w = gi.config5()
    say("iterative config5 n = 69000")
    setup(ctx, w)
    assert ctx.n == 69000
    khat, e0, e2 = gdm.plane_wave_inputs(w, ctx)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve_iterative(w["wavelength"], f0, tol=1e-13)
    relres = ctx.info.backward_err
    print("  products", ctx.info.ir_iters, "relres", relres, flush=True)
    assert relres <= 1e-13
    F0 = f0[0].cpu().numpy()
    F = f[0].cpu().numpy()
    D = O.Dipoles(w)
    rng = np.random.default_rng(57)
    rows = np.sort(np.concatenate([rng.choice(3 * D.nc, 20, replace=False),
                                   3 * D.nc + rng.choice(3 * D.ne, 20, replace=False),
                                   3 * D.N + rng.choice(3 * D.ne, 20, replace=False)]))
    MF, scale = O.matvec_rows(D, rows, F)
    res = np.abs(F0[rows] - MF)
    bound = relres * np.linalg.norm(F0) * 1.01 + 1e-12 * (scale + np.abs(F0[rows]))
    print("  max residual / bound", float(np.max(res / bound)), flush=True)
    assert np.all(res <= bound)


def test_iterative_stops_at_max_iter_with_noconv(ctx):
    from paper_2505_09545_amd import gdm
    w = workload("config1")
    setup(ctx, w)
    khat, e0, e2 = gdm.plane_wave_inputs(w, ctx)
    f0 = ctx.incident_planewave(khat, e0)
    say("iterative max_iter 3")
    with pytest.raises(gdm.GDMError) as ei:
        ctx.solve_iterative(w["wavelength"], f0, tol=1e-13, max_iter=3)
    assert ei.value.status == gdm.GDM_E_NOCONV
    assert ctx.info.ir_iters == 3 and ctx.info.backward_err > 1e-13
    with pytest.raises(gdm.GDMError) as ei:
        ctx.solve_iterative(w["wavelength"], f0, restart=5000)
    assert ei.value.status == gdm.GDM_E_ARG
