"""GPU parity of the HIP hot path (through the C-ABI) against the FP64 oracle.

Tolerances: FP64 results (moments, fields, cross sections) within 1e-10
relative (per RHS column, 2-norm; cross sections absolute-relative), the bar of
the method's FP64 mode; FP32 + FP64 refinement to the same 1e-10; the assembled
matrix elementwise within 1e-13 of the oracle's FP64 matrix (FP64 storage) or
one FP32 rounding (FP32 storage); the stand-alone GEMM / LU within a few
hundred units of roundoff of the respective precision times the problem scale.
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
    """max over RHS of ||a - b|| / ||b|| (rows = RHS)."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def oracle_q_rhs_major(sim):
    return sim["q"].T, sim["F"].T, sim["F0"].T


# ---------------------------------------------------------------------------
# GEMM (trailing update) against numpy
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("m,n,k,mode,trans", [(64, 64, 8, 0, 0), (200, 131, 77, 0, 0), (333, 70, 129, 1, 0),
                                              (129, 66, 300, 0, 1), (70, 5, 260, 1, 1), (1, 1, 1, 0, 0),
                                              # >= 2 tiles of 64 x 64 per CU: the large tile, k not a
                                              # multiple of its 4 complex k per stage
                                              (1500, 1430, 130, 0, 0), (1430, 1500, 131, 1, 0),
                                              (1500, 1400, 66, 0, 1),
                                              # small tiles with the whole k range (64 <= k <= 128) loaded
                                              # up front: exact, ragged and chunked (FP64: two halves) k
                                              (256, 66, 128, 0, 0), (300, 40, 64, 1, 1), (190, 97, 100, 1, 0),
                                              (130, 66, 96, 0, 1)])
def test_gemm_matches_numpy(ctx, dtype, m, n, k, mode, trans):
    say("gemm", dtype, m, n, k, mode, trans)
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    ndt = np.complex128 if dtype == "c128" else np.complex64
    lda_rows = (k if trans else m) + 3
    A = (rng.standard_normal((lda_rows, (m if trans else k))) + 1j * rng.standard_normal((lda_rows, (m if trans else k)))).astype(ndt)
    B = (rng.standard_normal((k + 1, n)) + 1j * rng.standard_normal((k + 1, n))).astype(ndt)
    C = (rng.standard_normal((m + 2, n)) + 1j * rng.standard_normal((m + 2, n))).astype(ndt)
    # column-major storage = transpose of row-major tensors
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    tB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    tC = torch.from_numpy(np.ascontiguousarray(C.T)).cuda()
    ctx.gemm(mode, trans, m, n, k, tA, lda_rows, tB, k + 1, tC, m + 2)
    torch.cuda.synchronize()
    got = tC.cpu().numpy().T
    Ad = A.astype(np.complex128)
    opA = (Ad[:k, :m].T if trans else Ad[:m, :k])
    prod = opA @ B[:k].astype(np.complex128)
    exp = C.astype(np.complex128).copy()
    exp[:m] = (exp[:m] - prod) if mode == 0 else prod
    eps = 2.2e-16 if dtype == "c128" else 1.2e-7
    scale = np.abs(opA) @ np.abs(B[:k]) + np.abs(C[:m])
    assert np.all(np.abs(got[:m] - exp[:m]) <= 8 * (k + 2) * eps * scale + 1e-300)
    assert np.array_equal(got[m:], C[m:])  # rows beyond m untouched


# ---------------------------------------------------------------------------
# LU + solve on random matrices (several blocks, ragged tail)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (37, 3), (300, 5), (777, 66), (777, 133)])
def test_getrf_getrs_random(ctx, dtype, n, nrhs):
    say("getrf/getrs", dtype, n, nrhs)
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A += np.eye(n) * 2.0  # keep it comfortably non-singular; pivoting is still exercised
    Bm = rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).to(tdt).cuda()
    ipiv = ctx.getrf(tA)
    for trans in (0, 1):
        tB = torch.from_numpy(np.ascontiguousarray(Bm.T)).to(tdt).cuda()
        ctx.getrs(tA, tB, trans)
        torch.cuda.synchronize()
        X = tB.cpu().numpy().T.astype(np.complex128)
        op = A.T if trans else A
        ref = np.linalg.solve(op, Bm)
        cond = np.linalg.cond(A)
        tol = (1e-12 if dtype == "c128" else 5e-5) * max(1.0, cond / 10)
        assert relcol(X.T, ref.T) < tol, (trans, relcol(X.T, ref.T), cond)
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)


def test_getrf_pivots_match_lapack(ctx):
    """Partial pivoting picks the row of largest |re|+|im| (ties to the lowest
    index): on a matrix whose pivots are unambiguous the pivot sequence is
    LAPACK's (zgetrf with the izamax rule)."""
    say("pivot order")
    import scipy.linalg as sla
    n = 300
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    ctx.set_pivoting(1)  # partial pivoting (also the default)
    try:
        piv = ctx.getrf(tA).cpu().numpy()
    finally:
        ctx.set_pivoting(0)
    _, lp = sla.lu_factor(A)
    # LAPACK's izamax uses |re| + |im| as well
    assert np.array_equal(piv, lp)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("pb", [1, 2, 4, 8])
@pytest.mark.parametrize("n", [3, 131, 1000, 2601])
def test_getrf_pivoting_widths(ctx, dtype, pb, n):
    """Every pivoting mode (columns per exchange 1: partial pivoting; 2, 4, 8:
    tournament; FP64 caps it at 4) on random matrices: ragged last panel (n not
    a multiple of the 128-column panel nor of the inner width), panels over
    one to ~80 workgroups.  P A = L U is checked through the solves of both
    op(A): the normwise backward error ||A x - b|| / (||A|| ||x|| + ||b||) of
    every column within a small multiple of the precision's unit roundoff."""
    say("getrf pivoting", dtype, pb, n)
    rng = np.random.default_rng(1000 + n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Bm = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    u = 1.1e-16 if dtype == "c128" else 6e-8
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).to(tdt).cuda()
    ctx.set_pivoting(pb)
    try:
        ipiv = ctx.getrf(tA).cpu().numpy()
    finally:
        ctx.set_pivoting(0)
    assert np.all(ipiv >= np.arange(n)) and np.all(ipiv < n)
    ndt = np.complex128 if dtype == "c128" else np.complex64
    As = A.astype(ndt).astype(np.complex128)  # the matrix and RHS as stored
    Bs = Bm.astype(ndt).astype(np.complex128)
    for trans in (0, 1):
        tB = torch.from_numpy(np.ascontiguousarray(Bm.T)).to(tdt).cuda()
        ctx.getrs(tA, tB, trans)
        torch.cuda.synchronize()
        X = tB.cpu().numpy().T.astype(np.complex128)
        op = As.T if trans else As
        r = op @ X - Bs
        norm_op = np.abs(op).sum(axis=1).max()
        be = np.max(np.abs(r).max(axis=0) / (norm_op * np.abs(X).max(axis=0) + np.abs(Bs).max(axis=0)))
        assert be < 30 * u * np.sqrt(n), (trans, be)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("pb", [1, 4, 8])
def test_getrf_zero_column_reports_its_index(ctx, dtype, pb):
    """An exactly zero column makes that column's pivot zero whatever the row
    interchanges: GDM_E_SINGULAR with bad_index = the column (here 37 and 200,
    the first reported)."""
    from paper_2505_09545_amd import gdm
    say("getrf zero column", dtype, pb)
    n = 300
    rng = np.random.default_rng(77)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A[:, 37] = 0
    A[:, 200] = 0
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).to(tdt).cuda()
    ctx.set_pivoting(pb)
    try:
        with pytest.raises(gdm.GDMError) as ei:
            ctx.getrf(tA)
    finally:
        ctx.set_pivoting(0)
    assert ei.value.status == gdm.GDM_E_SINGULAR
    assert ctx.info.bad_index == 37


# ---------------------------------------------------------------------------
# assembly (step a)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["config1", "mixed"])
def test_assembly_matches_oracle(ctx, which):
    say("assembly", which)
    w = gi.config1() if which == "config1" else gi.small_mixed(seed=21, n_cell_side=4, n_eff=9)
    from paper_2505_09545_amd import gdm
    gdm.run_forward  # binding present
    ctx.set_environment(w["n_env"])
    ne = len(w["r_eff"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]),
                      torch.as_tensor(w["r_eff"]) if ne else None, torch.as_tensor(w["alpha_eff"]) if ne else None)
    M = ctx.assemble(w["wavelength"]).cpu().numpy()
    Mo = O.assemble(O.Dipoles(w))
    err = np.abs(M - Mo)
    assert np.max(err) <= 1e-13 * np.max(np.abs(Mo)), np.max(err) / np.max(np.abs(Mo))
    assert np.all(err <= 1e-13 * np.abs(Mo) + 1e-15 * np.max(np.abs(Mo)))
    M32 = ctx.assemble(w["wavelength"], torch.complex64).cpu().numpy().astype(np.complex128)
    # FP64 arithmetic rounded once to FP32: within one FP32 rounding of the oracle
    assert np.all(np.abs(M32.real - Mo.real) <= 6.0e-8 * np.abs(Mo.real) + 1e-300)
    assert np.all(np.abs(M32.imag - Mo.imag) <= 6.0e-8 * np.abs(Mo.imag) + 1e-300)


# ---------------------------------------------------------------------------
# full forward path (steps a, b, c + cross sections) against the oracle
# ---------------------------------------------------------------------------
def _forward(ctx, w, prec, tol=0.0, want_ff=True):
    from paper_2505_09545_amd import gdm
    return gdm.run_forward(ctx, w, prec=prec, tol=tol, want_ff=want_ff)


@pytest.mark.parametrize("which", ["config1", "mixed", "config4_small", "config2_66rhs"])
@pytest.mark.parametrize("prec", [0, 1])
def test_forward_matches_oracle(ctx, which, prec):
    say("forward", which, "prec", prec)
    if which == "config1":
        w = gi.config1()
    elif which == "config2_66rhs":
        # the config-2 recipe at 600 cells (n = 1800) with all 66 plane waves:
        # solves over 66 RHS (three column tiles) and, in FP32+IR, residuals as
        # one 64-column tile plus a 2-column remainder on the side stream
        w = gi.config2(ncell=600)
    elif which == "mixed":
        w = gi.small_mixed(seed=22, n_cell_side=5, n_eff=12)
    else:
        w = dict(gi.config4())
        w["r_cell"] = gi.cuboid_cells(6, 7, 9, 8.0)
        w["eps_cell"] = np.full(len(w["r_cell"]), 10 + 0.05j)
        w["r_probe"] = w["r_probe"][::7]
    out = _forward(ctx, w, prec)
    sim = O.simulate(w)
    D = sim["D"]
    q, F, F0 = oracle_q_rhs_major(sim)
    assert relcol(out["f0"].cpu().numpy(), F0) < 1e-13
    assert relcol(out["q"].cpu().numpy(), q) < 1e-10
    assert relcol(out["f"].cpu().numpy(), F) < 1e-10
    cs = out["cs"].cpu().numpy()
    e2 = np.sum(np.abs(w["e0"]) ** 2, axis=1)
    ff = O.sca_farfield_doublesum(D, sim["q"], e2)
    for col, ref in ((0, sim["ext"]), (1, sim["sca"]), (2, sim["abs"]), (3, sim["rad"]), (4, ff)):
        assert np.max(np.abs(cs[:, col] - ref) / np.abs(ref)) < 1e-10, (col, cs[:, col], ref)
    if len(w["r_probe"]):
        Es, Hs = O.scattered_fields(D, sim["q"], w["r_probe"])
        assert relcol(out["E_sca"].cpu().numpy(), Es) < 1e-10
        assert relcol(out["H_sca"].cpu().numpy(), Hs) < 1e-10
    if prec == 1:
        assert out["info"].backward_err <= 1e-14


def test_planewave_points(ctx):
    say("planewave points")
    w = gi.config2(ncell=1000, n_random_pw=5)
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"][:10]), w["step"], torch.as_tensor(w["eps_cell"][:10]))
    ctx.factorize(w["wavelength"])
    pts = gi.fibonacci_sphere(77, 130.0)
    E, H = ctx.planewave(torch.as_tensor(w["khat"]), torch.as_tensor(w["e0"]), torch.as_tensor(pts))
    k0 = 2 * np.pi / w["wavelength"]
    Eo, Ho = O.planewave(pts, w["khat"], w["e0"], k0, w["n_env"])
    assert np.max(np.abs(E.cpu().numpy() - Eo)) < 1e-14
    assert np.max(np.abs(H.cpu().numpy() - Ho)) < 1e-14


def test_total_fields_and_intensity(ctx):
    """gdm_fields_total = the oracle's incident plane wave plus its scattered
    field at the probes (1e-10 per RHS column, E and H), and
    gdm_planewave_intensity = sum |e0_a|^2 (to rounding), on the 257-cell
    sphere with both polarisations plus a tilted, elliptically polarised wave."""
    say("total fields")
    from paper_2505_09545_amd import gdm
    w = dict(gi.config1())
    w["khat"] = np.vstack([w["khat"], [[0.6, 0.0, 0.8]]])
    w["e0"] = np.vstack([w["e0"], [[0.8, 0.3j, -0.6]]]).astype(np.complex128)
    out = gdm.run_forward(ctx, w, prec=gdm.PREC_FP64, probes=False)
    khat, e0, e2 = gdm.plane_wave_inputs(w, ctx)
    assert np.allclose(e2.cpu().numpy(), np.sum(np.abs(w["e0"]) ** 2, axis=1), rtol=1e-15, atol=0)
    E, H = ctx.fields_total(out["q"], khat, e0, torch.as_tensor(w["r_probe"]))
    sim = O.simulate(w)
    Es, Hs = O.scattered_fields(sim["D"], sim["q"], w["r_probe"])
    k0 = 2 * np.pi / w["wavelength"]
    Ei, Hi = O.planewave(w["r_probe"], w["khat"], w["e0"], k0, w["n_env"])
    assert relcol(E.cpu().numpy(), Es + Ei) < 1e-10
    assert relcol(H.cpu().numpy(), Hs + Hi) < 1e-10


# ---------------------------------------------------------------------------
# error paths (forced from the host; every kernel still exits normally)
# ---------------------------------------------------------------------------
def test_singular_cell_reports_singular(ctx):
    """A single cell at the Clausius-Mossotti pole eps = -2 eps_env makes
    1 - S alpha = 0 exactly: the factorisation reports a zero pivot."""
    say("singular")
    from paper_2505_09545_amd import gdm
    ctx.set_environment(1.0)
    ctx.set_structure(torch.zeros((1, 3), dtype=torch.float64), 10.0, torch.tensor([-2.0 + 0j]))
    with pytest.raises(gdm.GDMError) as e:
        ctx.factorize(500.0)
    assert e.value.status == gdm.GDM_E_SINGULAR
    assert ctx.info.bad_index == 0


def test_probe_on_dipole_is_rejected(ctx):
    say("probe at dipole")
    from paper_2505_09545_amd import gdm
    w = gi.config1()
    out = _forward(ctx, dict(w, r_probe=np.zeros((0, 3))), 0, want_ff=False)
    with pytest.raises(gdm.GDMError) as e:
        ctx.fields(out["q"], torch.as_tensor(w["r_cell"][5:6]))
    assert e.value.status == gdm.GDM_E_PROBE_AT_DIPOLE


def test_argument_errors(ctx):
    say("argument errors")
    from paper_2505_09545_amd import gdm
    with pytest.raises(gdm.GDMError) as e:
        ctx.set_environment(-1.0)
    assert e.value.status == gdm.GDM_E_ARG
    with pytest.raises(gdm.GDMError) as e:
        ctx.factorize(-5.0)
    assert e.value.status == gdm.GDM_E_ARG


def test_profile_tag_mask(ctx):
    """gdm_profile_mask times only the launches of the tags it is given (the
    benchmark's timed region keeps events on the update GEMM only);
    gdm_profile(ctx, 1) times every tag; a mask outside [0, 2^tags) is an
    argument error."""
    say("profile tag mask")
    from paper_2505_09545_amd import gdm
    w = gi.config1()
    ctx.profile(True, tags=["update", "panel"])
    gdm.run_forward(ctx, w, prec=gdm.PREC_FP32_IR, tol=1e-14, probes=False)
    p = ctx.profile_read()
    ctx.profile(False)
    assert p["update"]["launches"] > 0 and p["panel"]["launches"] > 0
    assert all(p[t]["launches"] == 0 for t in gdm.Context.PROF_TAGS if t not in ("update", "panel")), p
    ctx.profile(True)
    gdm.run_forward(ctx, w, prec=gdm.PREC_FP32_IR, tol=1e-14, probes=False)
    p = ctx.profile_read()
    ctx.profile(False)
    for t in ("update", "lookahead", "panel", "panel_l21", "assemble", "trsm", "solve", "resid"):
        assert p[t]["launches"] > 0 and p[t]["ms"] > 0, (t, p[t])
    with pytest.raises(gdm.GDMError) as e:
        ctx._check(ctx._call("gdm_profile_mask", ctx.h, 1 << len(gdm.Context.PROF_TAGS)))
    assert e.value.status == gdm.GDM_E_ARG


# ---------------------------------------------------------------------------
# full size: the 12 000-unknown benchmark workload against stored oracle values
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pivoting", [1, 4])
@pytest.mark.parametrize("prec", [1, 0])
def test_full_config2_vs_golden(ctx, prec, pivoting):
    """n = 12 000, 66 RHS, in the launch configuration bench.py times (partial
    pivoting), and with tournament pivoting over 4 columns: every cross
    section, the 2-norm of every column of q and F, and q, F at 97 seeded sample
    unknowns of every RHS against tests/golden/config2_samples.npz (written by
    tests/golden/make_golden.py from the oracle)."""
    import os
    say("full config2", "prec", prec, "pivoting", pivoting)
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_samples.npz"))
    w = gi.config2()
    from paper_2505_09545_amd import gdm
    ctx.set_pivoting(pivoting)
    try:
        out = gdm.run_forward(ctx, w, prec=prec, tol=1e-14 if prec == 1 else 0.0, probes=False)
    finally:
        ctx.set_pivoting(0)
    q = out["q"]
    f = out["f"]
    qn = torch.linalg.vector_norm(q, dim=1).cpu().numpy()
    fn = torch.linalg.vector_norm(f, dim=1).cpu().numpy()
    assert np.max(np.abs(qn - ref["q_norm"]) / ref["q_norm"]) < 1e-10
    assert np.max(np.abs(fn - ref["F_norm"]) / ref["F_norm"]) < 1e-10
    idx = torch.as_tensor(ref["idx"], device=q.device)
    qs = q[:, idx].cpu().numpy()
    fs = f[:, idx].cpu().numpy()
    # per RHS column: sampled entries within 1e-10 of the column norm
    assert np.max(np.abs(qs - ref["q"]) / ref["q_norm"][:, None]) < 1e-10
    assert np.max(np.abs(fs - ref["F"]) / ref["F_norm"][:, None]) < 1e-10
    cs = out["cs"].cpu().numpy()
    for col, key in ((0, "ext"), (1, "sca"), (2, "abs"), (3, "rad")):
        assert np.max(np.abs(cs[:, col] - ref[key]) / np.abs(ref[key])) < 1e-10, key
    if prec == 1:
        assert out["info"].backward_err <= 1e-14


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_config2_assembly_sampled(ctx, dtype):
    """The 12 000 x 12 000 matrix of the benchmark workload, read right after the
    (asynchronous) assembly call: the blocks between 64 seeded sample dipoles
    equal the oracle's assembly of the structure made of those dipoles alone
    (an off-diagonal block depends only on its two dipoles, a diagonal block on
    its own)."""
    say("full config2 assembly", dtype)
    w = gi.config2()
    ctx.set_environment(w["n_env"])
    ctx.set_structure(torch.as_tensor(w["r_cell"]), w["step"], torch.as_tensor(w["eps_cell"]))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    M = ctx.assemble(w["wavelength"], tdt)
    idx = np.sort(np.random.default_rng(99).choice(len(w["r_cell"]), 64, replace=False))
    u = torch.as_tensor((3 * idx[:, None] + np.arange(3)[None, :]).ravel(), device=M.device)
    got = M[u][:, u].cpu().numpy().astype(np.complex128)
    del M
    sub = dict(w, r_cell=w["r_cell"][idx], eps_cell=w["eps_cell"][idx])
    ref = O.assemble(O.Dipoles(sub))
    if dtype == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    else:
        # FP64 arithmetic rounded once to FP32, per real component
        assert np.all(np.abs(got.real - ref.real) <= 6.0e-8 * np.abs(ref.real) + 1e-300)
        assert np.all(np.abs(got.imag - ref.imag) <= 6.0e-8 * np.abs(ref.imag) + 1e-300)
