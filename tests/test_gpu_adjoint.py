"""GPU parity of the hand-written adjoint (gdm_adjoint through the C-ABI, and
the torch.autograd.Function over it) against the FP64 oracle's adjoint and
against central finite differences of the GPU forward pass.

Loss (the paper's resonance-search example shape): L = sigma_sca +
(1/P) sum_p |E_tot(r_p)|^2 / |E0|^2, summed over RHS.

Tolerances:
  * vs the oracle gradient: per parameter group (positions, Re eps, Im eps,
    wavelength) max |g - g_ref| / max |g_ref| <= 1e-9 in FP64 mode and after
    FP32 LU + FP64 refinement of both the forward and the transposed solve.
    The gradient is a sum of O(N^2) pair terms of alternating sign; 1e-9 leaves
    a factor ~100 over the FP64 round-off seen on these sizes (~1e-11).
  * vs central differences (h = 1e-4 nm for coordinates and wavelength, 1e-4
    for Re/Im eps): max |g - g_FD| / max |g_FD| <= 1e-6 over the sampled
    entries of each group.
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


def small_cells():
    """config-4 recipe at a size the oracle finishes in seconds: 4 x 5 x 6 cells
    (8 nm, eps 10+0.05i, 700 nm), two plane waves, 12 x 12 probes."""
    w = dict(gi.config4())
    w["r_cell"] = gi.cuboid_cells(4, 5, 6, 8.0)
    w["eps_cell"] = np.full(len(w["r_cell"]), 10.0 + 0.05j)
    w["eps_cell"][::3] += 2.0 + 0.3j  # non-uniform, so every eps entry has its own gradient
    w["khat"] = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]])
    w["e0"] = np.array([[1.0, 0.0, 0.0], [0.0, 1.0j, 0.0]], dtype=np.complex128)
    w["r_probe"] = gi.probe_plane(12, 12, 200.0, 200.0, -150.0)
    return w


def workload(which):
    if which == "cells":
        return small_cells()
    return gi.small_mixed(seed=31, n_cell_side=3, n_eff=5)


def setup(ctx, w, selfterm=0):
    ne = len(w["r_eff"])
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]),
                      torch.as_tensor(w["r_eff"]) if ne else None,
                      torch.as_tensor(w["alpha_eff"]) if ne else None, selfterm)


def gpu_loss_and_grad(ctx, w, prec, selfterm=0, want_grad=True):
    """Forward on the GPU, loss in FP64 on the host, then gdm_adjoint."""
    setup(ctx, w, selfterm)
    tol = 1e-14 if prec == 1 else 0.0
    ctx.factorize(w["wavelength"], prec)
    dev = ctx.device
    khat = torch.as_tensor(w["khat"], dtype=torch.float64, device=dev)
    e0 = torch.as_tensor(w["e0"], dtype=torch.complex128, device=dev)
    e2 = (e0.abs() ** 2).sum(dim=1)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve(f0, tol=tol)
    cs = ctx.cross_sections(f0, q, f, e2)
    rp = torch.as_tensor(w["r_probe"], dtype=torch.float64, device=dev)
    P = len(rp)
    Ei, _ = ctx.planewave(khat, e0, rp, want_h=False)
    Es, _ = ctx.fields(q, rp, want_h=False)
    E = Ei + Es
    L = float(cs[:, 1].sum()) + float(((E.abs() ** 2).sum(dim=(1, 2)) / e2).sum()) / P
    if not want_grad:
        return L, None
    g_sigma = torch.zeros((len(khat), 3), dtype=torch.float64, device=dev)
    g_sigma[:, 1] = 1.0
    g_e = E.conj() / (P * e2[:, None, None])
    gr, geps, gwl = ctx.adjoint(khat, e0, f0, q, f, g_sigma=g_sigma, r_probe=rp, g_e=g_e, tol=tol)
    return L, dict(r=gr.cpu().numpy(), eps_re=geps[:, 0].cpu().numpy(), eps_im=geps[:, 1].cpu().numpy(),
                   wavelength=float(gwl.cpu().numpy()[0]))


def rel_group(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check_vs_oracle(g, ref, nc, tol):
    assert rel_group(g["r"], ref["r"]) <= tol, ("r", rel_group(g["r"], ref["r"]))
    assert rel_group(g["eps_re"][:nc], ref["eps_re"]) <= tol, ("eps_re", rel_group(g["eps_re"][:nc], ref["eps_re"]))
    assert rel_group(g["eps_im"][:nc], ref["eps_im"]) <= tol, ("eps_im", rel_group(g["eps_im"][:nc], ref["eps_im"]))
    assert abs(g["wavelength"] - ref["wavelength"]) <= tol * abs(ref["wavelength"]), (g["wavelength"],
                                                                                      ref["wavelength"])


@pytest.mark.parametrize("which", ["cells", "mixed"])
@pytest.mark.parametrize("prec", [0, 1])
def test_adjoint_matches_oracle(ctx, which, prec):
    say("adjoint vs oracle", which, "prec", prec)
    w = workload(which)
    L, g = gpu_loss_and_grad(ctx, w, prec)
    ref = O.adjoint_gradient(w)
    assert abs(L - ref["loss"]) <= 1e-10 * abs(ref["loss"])
    check_vs_oracle(g, ref, len(w["r_cell"]), 1e-9)
    if prec == 1:
        assert ctx.info.backward_err <= 1e-14


def test_adjoint_radiative_selfterm(ctx):
    say("adjoint radiative self-term")
    w = small_cells()
    L, g = gpu_loss_and_grad(ctx, w, 0, selfterm=1)
    ref = O.adjoint_gradient(w, mode="radiative")
    check_vs_oracle(g, ref, len(w["r_cell"]), 1e-9)


def test_adjoint_cross_section_only_and_field_only(ctx):
    """The two loss terms separately (g_e NULL / g_sigma NULL) add up to the full gradient."""
    say("adjoint split terms")
    w = workload("mixed")
    _, full = gpu_loss_and_grad(ctx, w, 0)
    dev = ctx.device
    khat = torch.as_tensor(w["khat"], dtype=torch.float64, device=dev)
    e0 = torch.as_tensor(w["e0"], dtype=torch.complex128, device=dev)
    e2 = (e0.abs() ** 2).sum(dim=1)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve(f0)
    rp = torch.as_tensor(w["r_probe"], dtype=torch.float64, device=dev)
    Ei, _ = ctx.planewave(khat, e0, rp, want_h=False)
    Es, _ = ctx.fields(q, rp, want_h=False)
    g_sigma = torch.zeros((len(khat), 3), dtype=torch.float64, device=dev)
    g_sigma[:, 1] = 1.0
    a = ctx.adjoint(khat, e0, f0, q, f, g_sigma=g_sigma)
    b = ctx.adjoint(khat, e0, f0, q, f, r_probe=rp, g_e=(Ei + Es).conj() / (len(rp) * e2[:, None, None]))
    for i, key in ((0, "r"), (2, "wavelength")):
        s = (a[i] + b[i]).cpu().numpy()
        assert np.max(np.abs(s - full[key])) <= 1e-12 * np.max(np.abs(full[key]))
    s = (a[1] + b[1]).cpu().numpy()
    assert np.max(np.abs(s[:, 0] - full["eps_re"])) <= 1e-12 * np.max(np.abs(full["eps_re"]))


def test_adjoint_vs_finite_differences(ctx):
    say("adjoint vs FD")
    w = small_cells()
    L0, g = gpu_loss_and_grad(ctx, w, 0)
    rng = np.random.default_rng(7)
    h = 1e-4
    # positions: 9 sampled coordinates
    cells = rng.choice(len(w["r_cell"]), 9, replace=False)
    fd, ad = [], []
    for i, c in enumerate(cells):
        a = i % 3
        wp, wm = dict(w), dict(w)
        wp["r_cell"] = w["r_cell"].copy()
        wm["r_cell"] = w["r_cell"].copy()
        wp["r_cell"][c, a] += h
        wm["r_cell"][c, a] -= h
        fd.append((gpu_loss_and_grad(ctx, wp, 0, want_grad=False)[0] -
                   gpu_loss_and_grad(ctx, wm, 0, want_grad=False)[0]) / (2 * h))
        ad.append(g["r"][c, a])
    assert rel_group(ad, fd) <= 1e-6, (ad, fd)
    # permittivity: 4 cells, Re and Im
    for part, key in ((1.0, "eps_re"), (1j, "eps_im")):
        fd, ad = [], []
        for c in cells[:4]:
            wp, wm = dict(w), dict(w)
            wp["eps_cell"] = w["eps_cell"].copy()
            wm["eps_cell"] = w["eps_cell"].copy()
            wp["eps_cell"][c] += part * h
            wm["eps_cell"][c] -= part * h
            fd.append((gpu_loss_and_grad(ctx, wp, 0, want_grad=False)[0] -
                       gpu_loss_and_grad(ctx, wm, 0, want_grad=False)[0]) / (2 * h))
            ad.append(g[key][c])
        assert rel_group(ad, fd) <= 1e-6, (key, ad, fd)
    # wavelength
    wp, wm = dict(w), dict(w)
    wp["wavelength"] = w["wavelength"] + h
    wm["wavelength"] = w["wavelength"] - h
    fd = (gpu_loss_and_grad(ctx, wp, 0, want_grad=False)[0] - gpu_loss_and_grad(ctx, wm, 0, want_grad=False)[0]) / (
        2 * h)
    assert abs(g["wavelength"] - fd) <= 1e-6 * abs(fd), (g["wavelength"], fd)


def test_autograd_function(ctx):
    """GDMFunction + torch.autograd on the same loss equals the oracle gradient,
    including effective-dipole positions (mixed system)."""
    say("autograd function")
    from paper_2505_09545_amd.autograd import GDMSetup, gdm_forward
    w = workload("mixed")
    dev = ctx.device
    rc = torch.tensor(w["r_cell"], dtype=torch.float64, device=dev, requires_grad=True)
    eps = torch.tensor(w["eps_cell"], dtype=torch.complex128, device=dev, requires_grad=True)
    re = torch.tensor(w["r_eff"], dtype=torch.float64, device=dev, requires_grad=True)
    wl = torch.tensor(w["wavelength"], dtype=torch.float64, device=dev, requires_grad=True)
    e0 = torch.as_tensor(w["e0"], dtype=torch.complex128, device=dev)
    sim = GDMSetup(ctx, step=w["step"], n_env=w["n_env"], khat=torch.as_tensor(w["khat"], device=dev), e0=e0,
                   r_probe=torch.as_tensor(w["r_probe"], dtype=torch.float64, device=dev),
                   alpha_eff=torch.as_tensor(w["alpha_eff"], device=dev))
    sig, E = gdm_forward(rc, eps, wl, sim, r_eff=re)
    e2 = (e0.abs() ** 2).sum(dim=1)
    L = sig[:, 1].sum() + ((E.abs() ** 2).sum(dim=(1, 2)) / e2).sum() / E.shape[1]
    # use the context for something else in between: backward must restore its factors
    setup(ctx, small_cells())
    ctx.factorize(500.0)
    L.backward()
    ref = O.adjoint_gradient(w)
    nc = len(w["r_cell"])
    g = dict(r=np.concatenate([rc.grad.cpu().numpy(), re.grad.cpu().numpy()]),
             eps_re=eps.grad.real.cpu().numpy(), eps_im=eps.grad.imag.cpu().numpy(),
             wavelength=float(wl.grad.cpu()))
    assert abs(float(L.detach()) - ref["loss"]) <= 1e-10 * abs(ref["loss"])
    check_vs_oracle(g, ref, nc, 1e-9)


def test_adjoint_full_config4_vs_golden(ctx):
    """Full-size config 4 (2000 cells, 4096 probes, n = 6000) against the stored
    oracle gradient (tests/golden/make_golden.py), FP64 and FP32 + refinement."""
    say("adjoint full config4")
    path = os.path.join(GOLDEN, "config4_adjoint.npz")
    ref = dict(np.load(path))
    w = gi.config4()
    L, g = gpu_loss_and_grad(ctx, w, 0)
    assert abs(L - float(ref["loss"][0])) <= 1e-10 * abs(float(ref["loss"][0]))
    ref["wavelength"] = float(ref["wavelength"][0])
    check_vs_oracle(g, ref, len(w["r_cell"]), 1e-9)
    L32, g32 = gpu_loss_and_grad(ctx, w, 1)
    check_vs_oracle(g32, ref, len(w["r_cell"]), 1e-9)


def test_adjoint_full_config4_finite_differences(ctx):
    """Full-size config 4 (n = 6000) in FP64: the GPU adjoint against central
    differences of the GPU forward on a seeded sample -- 64 coordinates (every
    axis, cells spread over the cuboid), Re and Im of the permittivity of 8
    cells, and the wavelength; max |g - g_FD| / max |g_FD| <= 1e-6 per group
    (h = 1e-4 nm or 1e-4, truncation error ~1e-8 of the loss' scale)."""
    say("adjoint full config4: finite differences")
    w = gi.config4()
    L, g = gpu_loss_and_grad(ctx, w, 0)
    rng = np.random.default_rng(11)
    h = 1e-4

    def fd_of(mod):
        wp, wm = mod(+h), mod(-h)
        return (gpu_loss_and_grad(ctx, wp, 0, want_grad=False)[0] -
                gpu_loss_and_grad(ctx, wm, 0, want_grad=False)[0]) / (2 * h)

    cells = rng.choice(len(w["r_cell"]), 64, replace=False)
    fd, ad = [], []
    for i, c in enumerate(cells):
        a = i % 3

        def mod(d, c=c, a=a):
            r = w["r_cell"].copy()
            r[c, a] += d
            return dict(w, r_cell=r)
        fd.append(fd_of(mod))
        ad.append(g["r"][c, a])
    print("  coordinates: max rel", rel_group(ad, fd), flush=True)
    assert rel_group(ad, fd) <= 1e-6
    for part, key in ((1.0, "eps_re"), (1j, "eps_im")):
        fd, ad = [], []
        for c in cells[:8]:
            def mod(d, c=c):
                e = np.array(w["eps_cell"], dtype=np.complex128, copy=True)
                e[c] += part * d
                return dict(w, eps_cell=e)
            fd.append(fd_of(mod))
            ad.append(g[key][c])
        print(" ", key, "max rel", rel_group(ad, fd), flush=True)
        assert rel_group(ad, fd) <= 1e-6
    fdw = fd_of(lambda d: dict(w, wavelength=w["wavelength"] + d))
    print("  wavelength", g["wavelength"], fdw, flush=True)
    assert abs(g["wavelength"] - fdw) <= 1e-6 * abs(fdw)


def test_adjoint_state_and_argument_errors(ctx):
    say("adjoint errors")
    from paper_2505_09545_amd import gdm
    w = small_cells()
    setup(ctx, w)
    dev = ctx.device
    z = torch.zeros((1, ctx.n), dtype=torch.complex128, device=dev)
    k = torch.tensor([[0.0, 0.0, 1.0]], dtype=torch.float64, device=dev)
    e = torch.tensor([[1.0, 0.0, 0.0]], dtype=torch.complex128, device=dev)
    with pytest.raises(gdm.GDMError) as ex:  # set_structure dropped the factors
        ctx.adjoint(k, e, z, z, z, g_sigma=torch.ones((1, 3), dtype=torch.float64, device=dev))
    assert ex.value.status == gdm.GDM_E_STATE
