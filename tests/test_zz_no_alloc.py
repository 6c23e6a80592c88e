"""gdm_fields_noalloc (the probe-field entry point that allocates nothing)
against gdm_fields, both through the C-ABI, on two calls in a row, the second
with a smaller input; plus the size limit of its static scratch array.

The two entry points run the same kernels with the same dipole splits, so the
results must agree bit for bit; both are also held to the oracle's FP64 fields
(relative 1e-10 per RHS column, the bar of the FP64 mode).
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


def relcol(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def small_structure():
    """config-4 recipe at 4 x 5 x 6 cells (120 dipoles: four dipole splits of
    32, 32, 32 and 24 when there are few probes), two plane waves."""
    w = dict(gi.config4())
    w["r_cell"] = gi.cuboid_cells(4, 5, 6, 8.0)
    w["eps_cell"] = np.full(len(w["r_cell"]), 10.0 + 0.05j)
    w["khat"] = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]])
    w["e0"] = np.array([[1.0, 0.0, 0.0], [0.0, 1.0j, 0.0]], dtype=np.complex128)
    return w


@pytest.fixture(scope="module")
def solved():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_09545_amd import gdm
    ctx = gdm.Context(0)
    w = small_structure()
    out = gdm.run_forward(ctx, w, prec=gdm.PREC_FP64, probes=False)
    torch.cuda.synchronize()
    sim = O.simulate(w)
    yield gdm, ctx, w, out["q"], sim
    ctx.close()


def nan_like(t):
    return torch.full_like(t, complex(float("nan"), float("nan")))


def test_noalloc_matches_gdm_fields_on_two_calls(solved):
    gdm, ctx, w, q, sim = solved
    dev = ctx.device
    # call 1: 64 x 64 probes, 2 RHS, E and H (several dipole splits: the scratch holds partial sums)
    rp1 = torch.as_tensor(gi.probe_plane(64, 64, 200.0, 200.0, -150.0), dtype=torch.float64, device=dev)
    say("noalloc call 1: n_rhs 2, probes", rp1.shape[0], "with H")
    E_ref, H_ref = ctx.fields(q, rp1)
    E1, H1 = nan_like(E_ref), nan_like(H_ref)
    ctx.fields_noalloc(q, rp1, E1, H1)
    torch.cuda.synchronize()
    assert torch.equal(E1, E_ref) and torch.equal(H1, H_ref)
    Es, Hs = O.scattered_fields(sim["D"], sim["q"], rp1.cpu().numpy())
    assert relcol(E1.cpu().numpy(), Es) <= 1e-10
    assert relcol(H1.cpu().numpy(), Hs) <= 1e-10
    # call 2, smaller: 300 probes of another plane, 1 RHS, E only (the array
    # still holds call 1's partial sums)
    rp2 = torch.as_tensor(gi.probe_plane(20, 15, 120.0, 90.0, 95.0), dtype=torch.float64, device=dev)
    q2 = q[1:2].contiguous()
    say("noalloc call 2: n_rhs 1, probes", rp2.shape[0], "E only")
    E_ref2, _ = ctx.fields(q2, rp2, want_h=False)
    E2 = nan_like(E_ref2)
    ctx.fields_noalloc(q2, rp2, E2, None)
    torch.cuda.synchronize()
    assert torch.equal(E2, E_ref2)
    Es2, _ = O.scattered_fields(sim["D"], sim["q"][:, 1:2], rp2.cpu().numpy())
    assert relcol(E2.cpu().numpy(), Es2) <= 1e-10


def test_noalloc_rejects_sizes_beyond_its_array(solved):
    gdm, ctx, w, q, sim = solved
    dev = ctx.device
    # 2 RHS x 50 000 probes in 4 dipole splits with H: 2 * 48 * 4 * 2 * 50 000 B
    # = 38.4 MB of partial sums > 32 MiB (host-side check: no kernel runs)
    rp = torch.as_tensor(gi.probe_plane(250, 200, 400.0, 400.0, -150.0), dtype=torch.float64, device=dev)
    E = nan_like(torch.empty((2, rp.shape[0], 3), dtype=torch.complex128, device=dev))
    H = nan_like(E)
    say("noalloc over-size request: n_rhs 2, probes", rp.shape[0])
    with pytest.raises(gdm.GDMError) as ei:
        ctx.fields_noalloc(q, rp, E, H)
    assert ei.value.status == gdm.GDM_E_ARG
    torch.cuda.synchronize()
    assert torch.isnan(E.real).all() and torch.isnan(H.real).all()
    # the same probes without H (19.2 MB) fit, and agree with gdm_fields
    say("noalloc same probes, E only")
    E_ref, _ = ctx.fields(q, rp, want_h=False)
    ctx.fields_noalloc(q, rp, E, None)
    torch.cuda.synchronize()
    assert torch.equal(E, E_ref)
