"""Plain FP64 CPU oracle for the Green's Dyadic Method (GDM) hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import or run this module.  The product
(the HIP library and its Python binding) never calls it and shares no code
with it.

What it computes, each function citing the passage of arXiv:2505.09545 it
follows (sections / equations of the paper):

* Green's dyad blocks G^Ep, G^Hp, G^Em, G^Hm of a homogeneous lossless medium
  (Sec. "Formalism and implementation", Eq. superprop_G).  The paper defers
  their explicit form to its pyGDM reference; the forms used here follow from
  Maxwell's equations in Gaussian units with exp(-i w t) and are pinned in the
  tests by the vector Helmholtz equation, the curl relations between blocks,
  the static dipole limit and the radiative limit.
* cubic-cell polarisability alpha = (eps - eps_env) d^3 / (4 pi) (Sec. "Volume
  discretization polarizabilities") and the cubic self-term
  S^Ep = -4 pi / (3 eps_env d^3) I (Eq. selfterm_SEp_cubic); zero self-terms for
  effective point dipoles (same section, last paragraph).
* the discretised coupled system F_i = F0_i + sum_j G(r_i, r_j) alpha_j F_j
  (Eq. LPS_6by6_discrete) written as M F = F0 with M = I - G~ A
  (Eq. GDM_system_of_equations, read as in the design notes), with electric and
  magnetic unknowns separated and the magnetic unknowns of mesh cells removed
  (Sec. "Hybrid discretization GDM", Fig. coupling_matrix).
* solution by LU decomposition (Sec. "Numerical solution"): LAPACK zgetrf /
  zgetrs through SciPy.
* scattered fields by re-propagation of the dipole moments (Sec.
  "Observables", first item).
* extinction / absorption / scattering cross sections (Sec. "Observables"),
  plus the far-field scattering cross section by the exact double sum and by
  quadrature of the far-field amplitude.
* gradients of a scalar loss by a hand-written FP64 adjoint (the paper obtains
  them by automatic differentiation, Sec. "Example: Autograd for resonance
  search").
* point-dipole sources, the scattered part of the structured environment's
  Green's tensor and the electric / magnetic LDOS (Sec. "Observables";
  Appendix, illumination classes), from the same linear system; the paper
  defers their formulas to references, the normalisation used here follows
  from the power a dipole emits and is pinned by energy conservation (LDOS
  times the host's emitted power = far-field power of source plus structure,
  lossless cells with the radiative self-term) and by reciprocity.
* exact multipole moments (electric and magnetic dipoles and quadrupoles) of
  the cells' polarisation and their scattering and extinction cross sections
  (Sec. "Observables"); the paper names the exact-moment construction by
  reference only, the forms used here are pinned by projecting the far field on
  the l = 1, 2 electric / magnetic multipole subspaces (scattering) and by the
  optical theorem on those projections (extinction).
* extraction of an effective electric-magnetic dipole pair from a discretised
  structure (Sec. "Extraction of effective models"): moments by the exact
  multipole decomposition, alpha_eff = F0^+ P by least squares; pinned by the
  one-cell case (the cell's dressed polarisability exactly) and by the
  extracted model reproducing the full simulation of a small particle.
* global polarisability matrices (Sec. "Extraction of effective models";
  Fig. reference_system): M effective pairs whose moments are q_g = alpha_G F_g
  with one non-local 6M x 6M alpha_G, not coupled among themselves; their
  absorption also subtracts the group's mutual radiation (the paper's own code
  leaves GPM absorption to ext minus the far-field integral, Sec.
  "Implementation technical details"; the two agree exactly).  Extraction by
  scattered-field matching at probes and alpha_G = F0^+ P.  Pinned by the
  exact GPM of a cluster of coupled point dipoles (whole-system results
  unchanged, extraction returns it) and by a rod whose near field needs
  several pairs.

Units: nm, nm^2.  Complex values are numpy complex128.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np
import scipy.linalg as sla
import scipy.special as sps

FOUR_PI = 4.0 * math.pi


# ----------------------------------------------------------------------------
# wave numbers and Green's tensors  (Eq. superprop_G)
# ----------------------------------------------------------------------------
def wavenumbers(wavelength: float, n_env: float):
    """k0 = 2 pi / lambda0 (Sec. "Effective polarizabilities ..."), k = n_env k0."""
    k0 = 2.0 * math.pi / wavelength
    return k0, n_env * k0, n_env * n_env


def cross_matrix(v: np.ndarray) -> np.ndarray:
    """[v]_x such that [v]_x @ w = v x w, for v of shape (..., 3)."""
    z = np.zeros(v.shape[:-1])
    return np.stack([np.stack([z, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], z, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def green_ep(R: np.ndarray, k0: float, n_env: float) -> np.ndarray:
    """Electric field at r from an electric dipole at r', R = r - r' (..., 3).

    G^Ep = exp(ikR)/eps_env [ (k^2/R + ik/R^2 - 1/R^3) I
                              + (-k^2/R - 3ik/R^2 + 3/R^3) Rhat Rhat^T ]."""
    k = n_env * k0
    eps = n_env * n_env
    Rn = np.linalg.norm(R, axis=-1)
    Rh = R / Rn[..., None]
    ph = np.exp(1j * k * Rn) / eps
    a = (k * k / Rn + 1j * k / Rn ** 2 - 1.0 / Rn ** 3) * ph
    b = (-k * k / Rn - 3j * k / Rn ** 2 + 3.0 / Rn ** 3) * ph
    return a[..., None, None] * np.eye(3) + b[..., None, None] * (Rh[..., :, None] * Rh[..., None, :])


def green_hp(R: np.ndarray, k0: float, n_env: float) -> np.ndarray:
    """Magnetic field at r from an electric dipole at r':
    G^Hp = k0 k exp(ikR)/R (1 + i/(kR)) [Rhat]_x."""
    k = n_env * k0
    Rn = np.linalg.norm(R, axis=-1)
    Rh = R / Rn[..., None]
    h = k0 * k * np.exp(1j * k * Rn) / Rn * (1.0 + 1j / (k * Rn))
    return h[..., None, None] * cross_matrix(Rh)


def green6(R: np.ndarray, k0: float, n_env: float) -> np.ndarray:
    """6x6 dyad [[G^Ep, G^Em], [G^Hp, G^Hm]] with G^Em = -G^Hp and
    G^Hm = eps_env G^Ep (duality of the magnetic-dipole fields, mu = 1)."""
    eps = n_env * n_env
    gep = green_ep(R, k0, n_env)
    ghp = green_hp(R, k0, n_env)
    top = np.concatenate([gep, -ghp], axis=-1)
    bot = np.concatenate([ghp, eps * gep], axis=-1)
    return np.concatenate([top, bot], axis=-2)


def dgreen6_dR(R: np.ndarray, k0: float, n_env: float) -> np.ndarray:
    """Analytic derivative d G6(R) / d R_a, returned with shape (..., 3[a], 6, 6)."""
    k = n_env * k0
    eps = n_env * n_env
    Rn = np.linalg.norm(R, axis=-1)
    Rh = R / Rn[..., None]
    phi = np.exp(1j * k * Rn)
    # G^Ep = phi/eps (A I + Bq R R^T)
    A = k * k / Rn + 1j * k / Rn ** 2 - 1.0 / Rn ** 3
    A_R = -k * k / Rn ** 2 - 2j * k / Rn ** 3 + 3.0 / Rn ** 4
    Bq = -k * k / Rn ** 3 - 3j * k / Rn ** 4 + 3.0 / Rn ** 5
    Bq_R = 3 * k * k / Rn ** 4 + 12j * k / Rn ** 5 - 15.0 / Rn ** 6
    phi_R = 1j * k * phi
    I3 = np.eye(3)
    RR = R[..., :, None] * R[..., None, :]
    shp = R.shape[:-1]
    dE = np.zeros(shp + (3, 3, 3), dtype=np.complex128)
    dH = np.zeros(shp + (3, 3, 3), dtype=np.complex128)
    u = k0 * k * phi * (1.0 / Rn ** 2 + 1j / (k * Rn ** 3))
    u_R = k0 * k * (phi_R * (1.0 / Rn ** 2 + 1j / (k * Rn ** 3))
                    + phi * (-2.0 / Rn ** 3 - 3j / (k * Rn ** 4)))
    cx = cross_matrix(R)
    for a in range(3):
        ea = np.zeros(3)
        ea[a] = 1.0
        dRR = ea[:, None] * R[..., None, :] + R[..., :, None] * ea[None, :]
        termA = ((phi_R * A + phi * A_R) * Rh[..., a])[..., None, None] * I3
        termB = ((phi_R * Bq + phi * Bq_R) * Rh[..., a])[..., None, None] * RR
        termC = (phi * Bq)[..., None, None] * dRR
        dE[..., a, :, :] = (termA + termB + termC) / eps
        dH[..., a, :, :] = (u_R * Rh[..., a])[..., None, None] * cx + u[..., None, None] * cross_matrix(ea)
    top = np.concatenate([dE, -dH], axis=-1)
    bot = np.concatenate([dH, eps * dE], axis=-1)
    return np.concatenate([top, bot], axis=-2)


def dgreen6_dk0(R: np.ndarray, k0: float, n_env: float) -> np.ndarray:
    """Analytic derivative d G6 / d k0 at fixed R and n_env (k = n_env k0)."""
    k = n_env * k0
    eps = n_env * n_env
    Rn = np.linalg.norm(R, axis=-1)
    phi = np.exp(1j * k * Rn)
    dphi = 1j * n_env * Rn * phi
    A = k * k / Rn + 1j * k / Rn ** 2 - 1.0 / Rn ** 3
    dA = n_env * (2 * k / Rn + 1j / Rn ** 2)
    Bq = -k * k / Rn ** 3 - 3j * k / Rn ** 4 + 3.0 / Rn ** 5
    dBq = n_env * (-2 * k / Rn ** 3 - 3j / Rn ** 4)
    RR = R[..., :, None] * R[..., None, :]
    dE = ((dphi * A + phi * dA)[..., None, None] * np.eye(3)
          + (dphi * Bq + phi * dBq)[..., None, None] * RR) / eps
    # G^Hp = u(R) [R]_x with u = phi (n k0^2 / R^2 + i k0 / R^3)
    w = n_env * k0 * k0 / Rn ** 2 + 1j * k0 / Rn ** 3
    dw = 2 * n_env * k0 / Rn ** 2 + 1j / Rn ** 3
    du = dphi * w + phi * dw
    dH = du[..., None, None] * cross_matrix(R)
    top = np.concatenate([dE, -dH], axis=-1)
    bot = np.concatenate([dH, eps * dE], axis=-1)
    return np.concatenate([top, bot], axis=-2)


# ----------------------------------------------------------------------------
# dipoles: polarisabilities, self-terms, unknown layout
# ----------------------------------------------------------------------------
def cell_alpha(eps_cell, step: float, n_env: float):
    """alpha_pE = chi_ee d^3 / (4 pi) with chi_ee = eps - eps_env
    (Sec. "Volume discretization polarizabilities")."""
    return (np.asarray(eps_cell, dtype=np.complex128) - n_env * n_env) * step ** 3 / FOUR_PI


def cell_selfterm(step: float, n_env: float, k0: float, mode: str = "static") -> complex:
    """S^Ep = -I 4 pi / (3 eps_env d^3) (Eq. selfterm_SEp_cubic).  mode
    'radiative' adds i (2/3) k^3 / eps_env (radiation reaction; an option, not
    the paper's method)."""
    eps = n_env * n_env
    s = -FOUR_PI / (3.0 * eps * step ** 3) + 0j
    if mode == "radiative":
        k = n_env * k0
        s += 1j * (2.0 / 3.0) * k ** 3 / eps
    return s


class Dipoles:
    """All point dipoles of a simulation: N_c mesh cells then N_e effective
    ED+MD dipoles.  Unknown layout (Sec. "Hybrid discretization GDM"):
    [E of all N_c + N_e dipoles | H of the N_e effective dipoles]."""

    def __init__(self, wl: Dict, wavelength: float = None, mode: str = "static",
                 eps_cell=None, r_cell=None, r_eff=None):
        self.n_env = float(wl["n_env"])
        self.eps_env = self.n_env ** 2
        self.wavelength = float(wl["wavelength"] if wavelength is None else wavelength)
        self.k0, self.k, _ = wavenumbers(self.wavelength, self.n_env)
        self.step = float(wl["step"])
        self.mode = mode
        rc = np.asarray(wl["r_cell"] if r_cell is None else r_cell, dtype=np.float64)
        re = np.asarray(wl["r_eff"] if r_eff is None else r_eff, dtype=np.float64).reshape(-1, 3)
        self.nc, self.ne = len(rc), len(re)
        self.N = self.nc + self.ne
        self.pos = np.concatenate([rc, re], axis=0)
        eps_c = wl["eps_cell"] if eps_cell is None else eps_cell
        self.eps_cell = np.asarray(eps_c, dtype=np.complex128)
        a_c = cell_alpha(self.eps_cell, self.step, self.n_env)
        self.alpha6 = np.zeros((self.N, 6, 6), dtype=np.complex128)
        for a in range(3):
            self.alpha6[: self.nc, a, a] = a_c
        if self.ne:
            self.alpha6[self.nc:] = np.asarray(wl["alpha_eff"], dtype=np.complex128)
        self.S6 = np.zeros((self.N, 6, 6), dtype=np.complex128)
        s = cell_selfterm(self.step, self.n_env, self.k0, mode)
        for a in range(3):
            self.S6[: self.nc, a, a] = s
        # unknown index of (dipole, 6-component); -1 where the unknown is removed
        self.idx = -np.ones((self.N, 6), dtype=np.int64)
        self.idx[:, 0:3] = 3 * np.arange(self.N)[:, None] + np.arange(3)[None, :]
        self.idx[self.nc:, 3:6] = 3 * self.N + 3 * np.arange(self.ne)[:, None] + np.arange(3)[None, :]
        self.n = 3 * self.N + 3 * self.ne
        self.rho = np.concatenate([np.zeros(self.nc), np.ones(self.ne)])  # radiative reaction in alpha
        # GPM groups (Sec. "Extraction of effective models": a global polarisability
        # matrix over M effective dipoles): wl["gpm"] = [(first, M, alpha [6M, 6M]), ...]
        # with `first` an index among the effective dipoles; members' own alpha_eff is
        # not used, their moments are q_g = alpha_G F_g (blocks ordered (dipole, p, m)),
        # and members of one group do not couple through G~ (alpha_G holds that).
        self.groups = []
        self.gid = -np.ones(self.N, dtype=np.int64)
        for g, (first, M, aG) in enumerate(wl.get("gpm", []) or []):
            mem = self.nc + int(first) + np.arange(int(M))
            aG = np.asarray(aG, dtype=np.complex128).reshape(6 * int(M), 6 * int(M))
            assert np.all(self.gid[mem] < 0) and mem[-1] < self.N
            self.gid[mem] = g
            self.alpha6[mem] = 0.0
            self.groups.append((mem, aG))

    def group_cols(self, mem) -> np.ndarray:
        """Reduced indices of a group's unknowns, ordered (dipole, component)."""
        return self.idx[mem].reshape(-1)

    def q_of(self, F: np.ndarray) -> np.ndarray:
        """q = A F in the reduced layout (local blocks, then the GPM groups)."""
        q = self.from6(np.einsum("dab,db...->da...", self.alpha6, self.to6(F)))
        for mem, aG in self.groups:
            cols = self.group_cols(mem)
            q[cols] = np.tensordot(aG, F[cols], axes=(1, 0))
        return q

    def comps(self, d: int):
        return np.arange(6) if d >= self.nc else np.arange(3)

    def alpha_matrix(self) -> np.ndarray:
        """A in the reduced layout (q = A F): block diagonal, plus the GPM blocks."""
        A = np.zeros((self.n, self.n), dtype=np.complex128)
        for d in range(self.N):
            c = self.comps(d)
            ii = self.idx[d, c]
            A[np.ix_(ii, ii)] = self.alpha6[d][np.ix_(c, c)]
        for mem, aG in self.groups:
            cols = self.group_cols(mem)
            A[np.ix_(cols, cols)] = aG
        return A

    def to6(self, x: np.ndarray) -> np.ndarray:
        """Reduced vector(s) [n, ...] -> per-dipole 6-vectors [N, 6, ...] (zeros where removed)."""
        out = np.zeros((self.N, 6) + x.shape[1:], dtype=np.complex128)
        out[:, 0:3] = x[: 3 * self.N].reshape((self.N, 3) + x.shape[1:])
        if self.ne:
            out[self.nc:, 3:6] = x[3 * self.N:].reshape((self.ne, 3) + x.shape[1:])
        return out

    def from6(self, y: np.ndarray) -> np.ndarray:
        x = np.zeros((self.n,) + y.shape[2:], dtype=np.complex128)
        x[: 3 * self.N] = y[:, 0:3].reshape((3 * self.N,) + y.shape[2:])
        if self.ne:
            x[3 * self.N:] = y[self.nc:, 3:6].reshape((3 * self.ne,) + y.shape[2:])
        return x


# ----------------------------------------------------------------------------
# the coupled system  (Eq. LPS_6by6_discrete, Eq. GDM_system_of_equations)
# ----------------------------------------------------------------------------
def coupling_greens(D: Dipoles, chunk: int = 64) -> np.ndarray:
    """G~ in the reduced layout: G~[idx(i,a), idx(j,b)] = G6(r_i - r_j)[a, b]
    for i != j and S6_i[a, b] for i == j."""
    n, N = D.n, D.N
    G = np.zeros((n, n), dtype=np.complex128)
    rows_all = D.idx  # [N, 6]
    for i0 in range(0, N, chunk):
        i1 = min(N, i0 + chunk)
        R = D.pos[i0:i1, None, :] - D.pos[None, :, :]
        same = np.all(R == 0.0, axis=-1)
        Rs = np.where(same[..., None], 1.0, R)
        g6 = green6(Rs, D.k0, D.n_env)  # [c, N, 6, 6]
        for li, i in enumerate(range(i0, i1)):
            g6[li, i] = D.S6[i]
        # electric rows of the chunk
        for a_lo, a_hi, row_sel in ((0, 3, slice(i0, i1)), (3, 6, slice(max(i0, D.nc), i1))):
            r_d = np.arange(N)[row_sel]
            if len(r_d) == 0:
                continue
            rr = rows_all[r_d, a_lo:a_hi].reshape(-1)
            blk = g6[r_d - i0, :, a_lo:a_hi, :]  # [ri, N, 3, 6]
            # electric columns of all dipoles
            ce = rows_all[:, 0:3].reshape(-1)
            G[np.ix_(rr, ce)] = blk[:, :, :, 0:3].transpose(0, 2, 1, 3).reshape(len(rr), 3 * N)
            if D.ne:
                cm = rows_all[D.nc:, 3:6].reshape(-1)
                G[np.ix_(rr, cm)] = blk[:, D.nc:, :, 3:6].transpose(0, 2, 1, 3).reshape(len(rr), 3 * D.ne)
    for mem, _ in D.groups:  # no coupling inside a GPM group
        cols = D.group_cols(mem)
        G[np.ix_(cols, cols)] = 0.0
    return G


def apply_alpha_right(D: Dipoles, G: np.ndarray) -> np.ndarray:
    """G~ A for the block-diagonal A (column mixing within each dipole)."""
    out = np.empty_like(G)
    # cells: alpha_pE is scalar times I
    a_c = D.alpha6[: D.nc, 0, 0]
    out[:, : 3 * D.nc] = G[:, : 3 * D.nc] * np.repeat(a_c, 3)[None, :]
    for d in range(D.nc, D.N):
        c = D.idx[d]
        out[:, c] = G[:, c] @ D.alpha6[d]
    for mem, aG in D.groups:
        cols = D.group_cols(mem)
        out[:, cols] = G[:, cols] @ aG
    return out


def assemble(D: Dipoles) -> np.ndarray:
    """M = I - G~ A (n x n, complex128)."""
    G = coupling_greens(D)
    M = -apply_alpha_right(D, G)
    M[np.diag_indices(D.n)] += 1.0
    return M


def matvec_rows(D: Dipoles, rows: np.ndarray, x: np.ndarray):
    """(M x)[rows] for selected unknowns without forming M: with q = A x,
    (M x)_u = x_u - [sum_{j != i} G6(r_i - r_j) q_j + S6_i q_i]_c for u = idx(i, c)
    (Eq. GDM_system_of_equations read as M = I - G~ A).  Also returns
    sum of the moduli of the terms, |x_u| + sum |G6_ij q_j|_c + |S6_i q_i|_c,
    a scale for round-off bounds.  x: [n] (one vector)."""
    rows = np.asarray(rows, dtype=np.int64)
    q6 = D.to6(D.q_of(x))  # [N, 6]
    # (dipole, component) of every requested unknown
    where = {int(D.idx[d, c]): (d, c) for d in range(D.N) for c in range(6) if D.idx[d, c] >= 0}
    out = np.zeros(len(rows), dtype=np.complex128)
    scale = np.zeros(len(rows))
    for t, u in enumerate(rows):
        i, c = where[int(u)]
        R = D.pos[i][None, :] - D.pos
        R[i] = 1.0  # placeholder, replaced by the self-term below
        g = green6(R, D.k0, D.n_env)[:, c, :]  # [N, 6]
        terms = np.einsum("jb,jb->j", g, q6)
        terms[i] = D.S6[i][c] @ q6[i]
        if D.gid[i] >= 0:  # no coupling inside a GPM group
            terms[(D.gid == D.gid[i]) & (np.arange(D.N) != i)] = 0.0
        out[t] = x[u] - np.sum(terms)
        scale[t] = abs(x[u]) + np.sum(np.abs(terms))
    return out, scale


# ----------------------------------------------------------------------------
# illumination  (Appendix, 3D illuminations: plane wave)
# ----------------------------------------------------------------------------
def planewave(r: np.ndarray, khat: np.ndarray, e0: np.ndarray, k0: float, n_env: float):
    """E0(r) = e0 exp(i k khat.r), H0 = n_env khat x E0; returns E, H [n_pw, P, 3]."""
    k = n_env * k0
    khat = np.atleast_2d(khat)
    e0 = np.atleast_2d(e0)
    ph = np.exp(1j * k * (r @ khat.T)).T  # [n_pw, P]
    E = ph[:, :, None] * e0[:, None, :]
    H = n_env * np.cross(khat[:, None, :], E)
    return E, H


def incident_at_dipoles(D: Dipoles, khat, e0) -> np.ndarray:
    """F0 in the reduced layout, [n, n_pw]."""
    E, H = planewave(D.pos, khat, e0, D.k0, D.n_env)
    F6 = np.concatenate([E, H], axis=-1).transpose(1, 2, 0)  # [N, 6, n_pw]
    return D.from6(F6)


# ----------------------------------------------------------------------------
# solve  (Sec. "Numerical solution": LU decomposition)
# ----------------------------------------------------------------------------
def solve(M: np.ndarray, F0: np.ndarray):
    lu = sla.lu_factor(M, check_finite=False)
    return sla.lu_solve(lu, F0, check_finite=False), lu


def simulate(wl: Dict, mode: str = "static", wavelength: float = None, eps_cell=None,
             r_cell=None, keep_matrix: bool = False) -> Dict:
    """Full forward pass: dipoles, assembly, LU solve, q = A F, cross sections."""
    D = Dipoles(wl, wavelength, mode, eps_cell=eps_cell, r_cell=r_cell)
    M = assemble(D)
    F0 = incident_at_dipoles(D, wl["khat"], wl["e0"])
    F, lu = solve(M, F0)
    q = D.q_of(F)
    out = dict(D=D, F0=F0, F=F, q=q, lu=lu)
    out.update(cross_sections(D, F0, F, q, np.sum(np.abs(np.atleast_2d(wl["e0"])) ** 2, axis=1)))
    if keep_matrix:
        out["M"] = M
    return out


# ----------------------------------------------------------------------------
# observables  (Sec. "Observables")
# ----------------------------------------------------------------------------
def cross_sections(D: Dipoles, F0, F, q, e0_norm2) -> Dict:
    """Per RHS: ext = C sum Im(F0^* . q); abs = C sum [Im(F^* . q) - rho (2/3) k^3
    (|p|^2/eps_env + |m|^2)]; sca = ext - abs; rad = C sum (2/3) k^3 (|p|^2/eps_env + |m|^2);
    with C = 4 pi k0 / (n_env |E0|^2)."""
    C = FOUR_PI * D.k0 / (D.n_env * np.asarray(e0_norm2, dtype=np.float64))
    q6 = D.to6(q)
    w = np.concatenate([np.full(3, 1.0 / D.eps_env), np.ones(3)])
    prad = (2.0 / 3.0) * D.k ** 3 * np.einsum("c,dcr->dr", w, np.abs(q6) ** 2)  # [N, rhs]
    ext = C * np.sum(np.imag(np.conj(F0) * q), axis=0)
    absr = C * (np.sum(np.imag(np.conj(F) * q), axis=0) - np.sum(D.rho[:, None] * prad, axis=0))
    # a GPM group radiates as a whole: also subtract its members' mutual terms
    # Im sum_{i != j in g} q_i^H G6(r_i - r_j) q_j (the self terms are in prad)
    for mem, _ in D.groups:
        R = D.pos[mem][:, None, :] - D.pos[mem][None, :, :]
        same = np.eye(len(mem), dtype=bool)
        g6 = green6(np.where(same[..., None], 1.0, R), D.k0, D.n_env)
        g6[same] = 0.0
        qg = q6[mem]
        absr = absr - C * np.imag(np.einsum("iar,ijab,jbr->r", np.conj(qg), g6, qg))
    rad = C * np.sum(prad, axis=0)
    return dict(ext=ext, abs=absr, sca=ext - absr, rad=rad)


def sca_farfield_doublesum(D: Dipoles, q, e0_norm2, chunk: int = 256) -> np.ndarray:
    """sigma_sca,ff = C Im sum_{i,j} q_i^H G^_ij q_j, G^_ij = G6(r_i - r_j) (i != j),
    G^_ii = i (2/3) k^3 diag(I/eps_env, I): the exact power radiated by the dipoles."""
    C = FOUR_PI * D.k0 / (D.n_env * np.asarray(e0_norm2, dtype=np.float64))
    q6 = D.to6(q)  # [N, 6, rhs]
    tot = np.zeros(q6.shape[2])
    diag = 1j * (2.0 / 3.0) * D.k ** 3 * np.concatenate([np.full(3, 1.0 / D.eps_env), np.ones(3)])
    for i0 in range(0, D.N, chunk):
        i1 = min(D.N, i0 + chunk)
        R = D.pos[i0:i1, None, :] - D.pos[None, :, :]
        same = np.all(R == 0.0, axis=-1)
        g6 = green6(np.where(same[..., None], 1.0, R), D.k0, D.n_env)
        g6[same] = 0.0
        s = np.einsum("iar,ijab,jbr->r", np.conj(q6[i0:i1]), g6, q6)
        s += np.einsum("iar,a,iar->r", np.conj(q6[i0:i1]), diag, q6[i0:i1])
        tot += np.imag(s)
    return C * tot


def farfield_amplitude(D: Dipoles, q, nhat: np.ndarray) -> np.ndarray:
    """A(n) with E_sca -> exp(ikR)/R A(n): sum_j exp(-ik n.r_j) [(k^2/eps)(n x p_j) x n
    - k0 k (n x m_j)]; returns [n_dir, 3, rhs]."""
    q6 = D.to6(q)
    p, m = q6[:, 0:3], q6[:, 3:6]
    ph = np.exp(-1j * D.k * (nhat @ D.pos.T))  # [dir, N]
    P = np.einsum("dj,jar->dar", ph, p)
    Mm = np.einsum("dj,jar->dar", ph, m)
    n3 = nhat[:, :, None]
    nxp = np.cross(n3, P, axis=1)
    return (D.k ** 2 / D.eps_env) * np.cross(nxp, n3, axis=1) - D.k0 * D.k * np.cross(n3, Mm, axis=1)


def sca_farfield_quadrature(D: Dipoles, q, e0_norm2, n_theta: int = 96, n_phi: int = 192):
    """sigma_sca = (1/|E0|^2) \\oint |A(n)|^2 dOmega by Gauss-Legendre in cos(theta)
    times the uniform rule in phi."""
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * math.pi * np.arange(n_phi) / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    nhat = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wx[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).reshape(-1)
    A = farfield_amplitude(D, q, nhat)
    return np.einsum("d,dar->r", w, np.abs(A) ** 2) / np.asarray(e0_norm2, dtype=np.float64)


def scattered_fields(D: Dipoles, q, r_probe: np.ndarray, chunk: int = 512):
    """E_sca, H_sca at probes by re-propagation sum_j G6(r_p - r_j) q_j
    (Sec. "Observables"); returns E, H [rhs, P, 3]."""
    q6 = D.to6(q)  # [N, 6, rhs]
    P = len(r_probe)
    out = np.zeros((q6.shape[2], P, 6), dtype=np.complex128)
    for p0 in range(0, P, chunk):
        p1 = min(P, p0 + chunk)
        R = r_probe[p0:p1, None, :] - D.pos[None, :, :]
        g6 = green6(R, D.k0, D.n_env)
        out[:, p0:p1, :] = np.einsum("pjab,jbr->rpa", g6, q6)
    return out[..., 0:3], out[..., 3:6]


# ----------------------------------------------------------------------------
# local dipole sources, Green's tensor and LDOS of the structured environment
# (Sec. "Observables": electric and magnetic LDOS and Green's tensors in a
# nano-structured environment; Appendix, illumination classes: electric and
# magnetic point-dipole sources)
# ----------------------------------------------------------------------------
def dipole_source_at_dipoles(D: Dipoles, r_src, d_src) -> np.ndarray:
    """F0 [n, n_src] of point dipole sources d_src = (p, m) [n_src, 6] at r_src
    [n_src, 3]: the source's own field G6(r_i - r_s) d_s at every dipole, in the
    reduced layout."""
    R = D.pos[:, None, :] - np.asarray(r_src, dtype=np.float64)[None, :, :]
    g6 = green6(R, D.k0, D.n_env)  # [N, S, 6, 6]
    return D.from6(np.einsum("nsab,sb->nas", g6, np.asarray(d_src, dtype=np.complex128)))


def green_scattered(wl: Dict, r_src, r_pts, mode: str = "static"):
    """Scattered part of the 6x6 Green's tensor of the structured environment,
    G_sca[s, p, row, c]: the field (row 0-2 E, 3-5 H) at r_pts[p] that the
    structure scatters under the unit source component c (p_x, p_y, p_z, m_x,
    m_y, m_z) at r_src[s] -- the solve of M F = G(., r_s) e_c, q = A F, then
    re-propagation.  Returns (G_sca [S, P, 6, 6], D)."""
    D = Dipoles(wl, mode=mode)
    M = assemble(D)
    r_src = np.asarray(r_src, dtype=np.float64).reshape(-1, 3)
    S = len(r_src)
    d = np.tile(np.eye(6, dtype=np.complex128), (S, 1))  # RHS 6 s + c
    F0 = dipole_source_at_dipoles(D, np.repeat(r_src, 6, axis=0), d)
    F, _ = solve(M, F0)
    q = D.q_of(F)
    r_pts = np.asarray(r_pts, dtype=np.float64).reshape(-1, 3)
    E, H = scattered_fields(D, q, r_pts)  # [6 S, P, 3]
    G = np.concatenate([E, H], axis=-1).reshape(S, 6, len(r_pts), 6)
    return G.transpose(0, 2, 3, 1), D


def ldos(wl: Dict, r_src, mode: str = "static") -> np.ndarray:
    """Partial LDOS of electric and magnetic point dipoles at r_src along x, y,
    z relative to the homogeneous host, [S, 2, 3]: a unit dipole d emits
    (omega/2) Im(d^* . F(r_s)) with F its total field at itself; the host's part
    is the radiation reaction Im G^Ep(0) = (2/3) k^3/eps_env I (Im G^Hm(0) =
    (2/3) k^3 I), so rho_e,a/rho_0 = 1 + (3/2)(eps_env/k^3) Im G_sca^Ep_aa(r_s,
    r_s) and rho_m,a/rho_0 = 1 + (3/2)(1/k^3) Im G_sca^Hm_aa(r_s, r_s)."""
    G, D = green_scattered(wl, r_src, r_src, mode)
    S = G.shape[0]
    out = np.zeros((S, 2, 3))
    k3 = D.k ** 3
    for s in range(S):
        for a in range(3):
            out[s, 0, a] = 1.0 + 1.5 * D.eps_env / k3 * G[s, s, a, a].imag
            out[s, 1, a] = 1.0 + 1.5 / k3 * G[s, s, 3 + a, 3 + a].imag
    return out


# ----------------------------------------------------------------------------
# exact multipole decomposition up to quadrupoles (Sec. "Observables": exact
# multipole decomposition of the polarisation inside a discretised structure and
# of the scattering and extinction cross sections; Sec. "Implementation
# technical details", which names the exact-moment and extinction references)
# ----------------------------------------------------------------------------
def multipole_center(D: Dipoles) -> np.ndarray:
    """Default expansion point: the mean position of the mesh cells."""
    return np.mean(D.pos[:D.nc], axis=0)


def multipole_moments(D: Dipoles, q, r0=None) -> Dict:
    """Exact electric / magnetic dipole and quadrupole moments of the mesh
    cells' polarisation (their electric dipoles p_j at r_j; effective dipoles
    are not part of the discretised structure and are left out), about r0.

    With R = r_j - r0, x = k|R| and spherical Bessel functions j_n(x) (SciPy),
    summed over cells, in the Gaussian convention of farfield_amplitude:
      p   = p_j j0 + (k^2/2) [3 (R.p_j) R - R^2 p_j] j2/x^2
      m   = -i k0 (3/2) (R x p_j) j1/x
      Qe  = 3 { [3 (R p_j^T + p_j R^T) - 2 (R.p_j) I] j1/x
                + 2 k^2 [5 (R.p_j) R R^T - R^2 (R p_j^T + p_j R^T) - R^2 (R.p_j) I] j3/x^3 }
      Qm  = -i k0 15 [R (R x p_j)^T + (R x p_j) R^T] j2/x^2
    (the current of a dipole is -i omega p; at x -> 0 these become the
    long-wavelength moments: p, m = -(i k0/2) sum R x p, the traceless
    quadrupoles).  Returns dict p [rhs,3], m [rhs,3], Qe [rhs,3,3], Qm [rhs,3,3]
    and r0."""
    r0 = multipole_center(D) if r0 is None else np.asarray(r0, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    if q.ndim == 1:
        q = q[:, None]
    nc = D.nc
    P = q[:3 * nc].reshape(nc, 3, -1)  # [nc, 3, rhs]
    R = D.pos[:nc] - r0[None, :]
    rr = np.linalg.norm(R, axis=1)
    x = D.k * rr
    xs = np.where(x > 0, x, 1.0)
    j0 = sps.spherical_jn(0, x)
    # j_n(x)/x^n at x = 0: 1 / (2n+1)!!
    w1 = np.where(x > 0, sps.spherical_jn(1, xs) / xs, 1.0 / 3.0)
    w2 = np.where(x > 0, sps.spherical_jn(2, xs) / xs ** 2, 1.0 / 15.0)
    w3 = np.where(x > 0, sps.spherical_jn(3, xs) / xs ** 3, 1.0 / 105.0)
    k, k0 = D.k, D.k0
    Rp = np.einsum("ja,jar->jr", R, P)  # R.p
    R2 = rr ** 2
    I3 = np.eye(3)
    p = np.einsum("j,jar->ra", j0, P) + (k ** 2 / 2) * np.einsum(
        "j,jar->ra", w2, 3 * Rp[:, None, :] * R[:, :, None] - R2[:, None, None] * P)
    RxP = np.cross(R[:, :, None], P, axis=1)  # [nc, 3, rhs]
    m = -1j * k0 * 1.5 * np.einsum("j,jar->ra", w1, RxP)
    RPt = np.einsum("ja,jbr->jabr", R, P)
    sym = RPt + RPt.transpose(0, 2, 1, 3)  # R p^T + p R^T
    RR = np.einsum("ja,jb->jab", R, R)
    t1 = 3 * sym - 2 * Rp[:, None, None, :] * I3[None, :, :, None]
    t3 = (5 * Rp[:, None, None, :] * RR[:, :, :, None] - R2[:, None, None, None] * sym
          - (R2[:, None] * Rp)[:, None, None, :] * I3[None, :, :, None])
    Qe = 3 * (np.einsum("j,jabr->rab", w1, t1) + 2 * k ** 2 * np.einsum("j,jabr->rab", w3, t3))
    RXt = np.einsum("ja,jbr->jabr", R, RxP)
    Qm = -1j * k0 * 15 * np.einsum("j,jabr->rab", w2, RXt + RXt.transpose(0, 2, 1, 3))
    return dict(p=p, m=m, Qe=Qe, Qm=Qm, r0=r0)


def multipole_cross_sections(D: Dipoles, q, khat=None, e0=None, r0=None) -> Dict:
    """Scattering cross sections of the four multipoles (exact moments above):
      ED (8 pi/3) k^4/eps^2 |p|^2, MD (8 pi/3) k0^2 k^2 |m|^2,
      EQ (pi/45) k^6/eps^2 sum|Qe_ab|^2, MQ (pi/45) k0^2 k^4 sum|Qm_ab|^2,
    each over |E0|^2 -- the powers of the far-field patterns
    (k^2/eps)(n x p) x n, -k0 k n x m, -(i k^3/(6 eps))(n x Qe n) x n and
    (i k0 k^2/6) n x (Qm n) (farfield_amplitude's convention).  With a plane
    wave (khat, e0) also the extinction of each: C Im(E0*(r0).p),
    C Im(H0*(r0).m), (C/6) Im(sum_ab d_a E0*_b(r0) Qe_ab),
    (C/6) Im(sum_ab d_a H0*_b(r0) Qm_ab), C = 4 pi k0/(n_env |E0|^2) (the
    incident field and its gradient at r0 against each moment).
    Returns dict sca [rhs, 4] and, with a plane wave, ext [rhs, 4]
    (order ED, MD, EQ, MQ)."""
    mo = multipole_moments(D, q, r0)
    k, k0, eps = D.k, D.k0, D.eps_env
    sca = np.stack([(8 * math.pi / 3) * k ** 4 / eps ** 2 * np.sum(np.abs(mo["p"]) ** 2, axis=1),
                    (8 * math.pi / 3) * k0 ** 2 * k ** 2 * np.sum(np.abs(mo["m"]) ** 2, axis=1),
                    (math.pi / 45) * k ** 6 / eps ** 2 * np.sum(np.abs(mo["Qe"]) ** 2, axis=(1, 2)),
                    (math.pi / 45) * k0 ** 2 * k ** 4 * np.sum(np.abs(mo["Qm"]) ** 2, axis=(1, 2))], axis=1)
    out = dict(sca=None, ext=None, moments=mo)
    if khat is None:
        out["sca"] = sca
        return out
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    e0 = np.atleast_2d(np.asarray(e0, dtype=np.complex128))
    e2 = np.sum(np.abs(e0) ** 2, axis=1)
    out["sca"] = sca / e2[:, None]
    E, H = planewave(mo["r0"][None, :], khat, e0, k0, D.n_env)  # [rhs, 1, 3]
    Es, Hs = np.conj(E[:, 0]), np.conj(H[:, 0])
    gE = -1j * k * khat[:, :, None] * Es[:, None, :]  # d_a E0*_b
    gH = -1j * k * khat[:, :, None] * Hs[:, None, :]
    C = FOUR_PI * k0 / (D.n_env * e2)
    out["ext"] = np.stack([C * np.imag(np.sum(Es * mo["p"], axis=1)),
                           C * np.imag(np.sum(Hs * mo["m"], axis=1)),
                           C / 6 * np.imag(np.sum(gE * mo["Qe"], axis=(1, 2))),
                           C / 6 * np.imag(np.sum(gH * mo["Qm"], axis=(1, 2)))], axis=1)
    return out


# ----------------------------------------------------------------------------
# effective models: extraction of one effective electric-magnetic dipole pair
# (Sec. "Extraction of effective models": illuminate, simulate, extract the
# dipole moments -- for one pair in 3D by the exact multipole decomposition --
# and fit alpha_eff by least squares, alpha_eff = F0^+ P)
# ----------------------------------------------------------------------------
def illumination_at_point(D: Dipoles, r0, khat, e0, r_src, d_src) -> np.ndarray:
    """(E0, H0) at r0 of each illumination, [N, 6]: the plane waves (khat, e0)
    first, then the point-dipole sources d_src [n_src, 6] at r_src (their own
    field G6(r0 - r_s) d_s)."""
    r0 = np.asarray(r0, dtype=np.float64)
    rows = []
    if khat is not None and len(np.atleast_2d(khat)):
        E, H = planewave(r0[None, :], khat, e0, D.k0, D.n_env)
        rows.append(np.concatenate([E[:, 0], H[:, 0]], axis=1))
    if r_src is not None and len(np.atleast_2d(r_src)):
        rs = np.atleast_2d(np.asarray(r_src, dtype=np.float64))
        g = green6(r0[None, :] - rs, D.k0, D.n_env)  # [S, 6, 6]
        rows.append(np.einsum("sab,sb->sa", g, np.atleast_2d(np.asarray(d_src, dtype=np.complex128))))
    return np.concatenate(rows, axis=0)


def extract_dipole_pair(wl: Dict, khat, e0, r_src=None, d_src=None, r0=None, mode: str = "static"):
    """Effective 6x6 polarisability of the structure about r0 (default: the
    cells' mean position): for every illumination the full system is solved,
    the exact electric and magnetic dipole moments (p, m) about r0 are taken
    (multipole_moments) and stacked as the rows of P [N, 6]; the rows of F0
    [N, 6] are the illuminations' (E0, H0) at r0.  alpha_eff minimises
    ||F0 alpha_eff^T - P|| (least squares, LAPACK through NumPy), so that
    (p, m) ~ alpha_eff (E0, H0).  Returns (alpha_eff [6, 6], relative residual
    ||F0 alpha_eff^T - P||_F / ||P||_F, r0)."""
    D = Dipoles(wl, mode=mode)
    M = assemble(D)
    cols = []
    if khat is not None and len(np.atleast_2d(khat)):
        cols.append(incident_at_dipoles(D, khat, e0))
    if r_src is not None and len(np.atleast_2d(r_src)):
        cols.append(dipole_source_at_dipoles(D, r_src, d_src))
    F0 = np.concatenate(cols, axis=1)
    F, _ = solve(M, F0)
    q = D.q_of(F)
    mo = multipole_moments(D, q, r0)
    P = np.concatenate([mo["p"], mo["m"]], axis=1)  # [N, 6]
    A = illumination_at_point(D, mo["r0"], khat, e0, r_src, d_src)
    X, *_ = np.linalg.lstsq(A, P, rcond=None)
    res = np.linalg.norm(A @ X - P) / np.linalg.norm(P)
    return X.T, float(res), mo["r0"]


def extract_gpm(wl: Dict, r_gpm, khat, e0, r_src=None, d_src=None, r_probe=None, mode: str = "static"):
    """Global polarisability matrix (6M x 6M) of the structure for M dipole
    pairs at r_gpm [M, 3] (Sec. "Extraction of effective models"): for every
    illumination the full system is solved and the scattered (E, H) at the
    probes r_probe [P, 3] is computed (scattered_fields); the moments
    (p_j, m_j) of the M pairs are the least-squares fit of that field by
    sum_j G6(r_p - r_j) (p_j, m_j) (both E and H matched); with the rows of
    F0 [N, 6M] the illuminations' (E0, H0) at the M positions and the rows of
    P [N, 6M] the fitted moments, alpha_G minimises ||F0 alpha_G^T - P||.
    Returns (alpha_G [6M, 6M] ordered (pair, p then m), relative residual of
    the field fit (all illuminations), relative residual of the alpha fit)."""
    D = Dipoles(wl, mode=mode)
    M = assemble(D)
    cols = []
    if khat is not None and len(np.atleast_2d(khat)):
        cols.append(incident_at_dipoles(D, khat, e0))
    if r_src is not None and len(np.atleast_2d(r_src)):
        cols.append(dipole_source_at_dipoles(D, r_src, d_src))
    F0 = np.concatenate(cols, axis=1)
    F, _ = solve(M, F0)
    q = D.q_of(F)
    rp = np.asarray(r_probe, dtype=np.float64).reshape(-1, 3)
    rg = np.asarray(r_gpm, dtype=np.float64).reshape(-1, 3)
    Es, Hs = scattered_fields(D, q, rp)  # [N, P, 3] each
    Y = np.concatenate([Es, Hs], axis=2).reshape(Es.shape[0], -1).T  # [6P, N]
    G = green6(rp[:, None, :] - rg[None, :, :], D.k0, D.n_env)  # [P, M, 6, 6]
    G = G.transpose(0, 2, 1, 3).reshape(6 * len(rp), 6 * len(rg))
    Q, *_ = np.linalg.lstsq(G, Y, rcond=None)  # [6M, N]
    res_field = np.linalg.norm(G @ Q - Y) / np.linalg.norm(Y)
    A = np.concatenate([illumination_at_point(D, r, khat, e0, r_src, d_src) for r in rg], axis=1)
    P = Q.T  # [N, 6M]
    X, *_ = np.linalg.lstsq(A, P, rcond=None)
    res_alpha = np.linalg.norm(A @ X - P) / np.linalg.norm(P)
    return X.T, float(res_field), float(res_alpha)


# ----------------------------------------------------------------------------
# adjoint gradient of a scalar loss (FP64 reference gradient)
# ----------------------------------------------------------------------------
def loss_sca_plus_nearfield(wl: Dict, w_sca: float = 1.0, w_nf: float = None,
                            wavelength=None, eps_cell=None, r_cell=None, mode="static") -> float:
    """L = w_sca sigma_sca + w_nf sum_p |E_tot(r_p)|^2 / |E0|^2, summed over RHS
    (default w_nf = 1 / number of probes)."""
    sim = simulate(wl, mode, wavelength, eps_cell, r_cell)
    D = sim["D"]
    P = len(wl["r_probe"])
    w_nf = (1.0 / P if P else 0.0) if w_nf is None else w_nf
    L = w_sca * float(np.sum(sim["sca"]))
    if P and w_nf:
        E_inc, _ = planewave(wl["r_probe"], wl["khat"], wl["e0"], D.k0, D.n_env)
        Es, _ = scattered_fields(D, sim["q"], wl["r_probe"])
        e2 = np.sum(np.abs(np.atleast_2d(wl["e0"])) ** 2, axis=1)
        L += w_nf * float(np.sum(np.sum(np.abs(E_inc + Es) ** 2, axis=(1, 2)) / e2))
    return L


def adjoint_gradient(wl: Dict, w_sca: float = 1.0, w_nf: float = None, mode="static") -> Dict:
    """Gradient of ``loss_sca_plus_nearfield`` w.r.t. every dipole position,
    Re/Im of every cell permittivity and the wavelength.

    Adjoint identity (M F = F0, q = A F, dL = 2 Re[g . dz] for Wirtinger
    partials g of the real loss):
      M^T lam = g_F + A^T g_qe,   g_qe = g_q + sum_p g_Ep G_pj,
      dL = 2 Re[(lam + g_F0) . dF0 + lam . dG~ q + (lam^T G~ + g_qe) dA F
                + g_Ep . (dE0_p + dG_p q)] + explicit dependence through C(k0)."""
    D = Dipoles(wl, None, mode)
    assert not D.groups, "the gradient is written for local polarisabilities"
    M = assemble(D)
    Gt = coupling_greens(D)
    F0 = incident_at_dipoles(D, wl["khat"], wl["e0"])
    F, lu = solve(M, F0)
    q = D.q_of(F)
    e2 = np.sum(np.abs(np.atleast_2d(wl["e0"])) ** 2, axis=1)  # [rhs]
    C = FOUR_PI * D.k0 / (D.n_env * e2)  # [rhs]
    nrhs = F0.shape[1]
    rp = np.asarray(wl["r_probe"], dtype=np.float64).reshape(-1, 3)
    P = len(rp)
    w_nf = (1.0 / P if P else 0.0) if w_nf is None else w_nf
    wq = np.concatenate([np.full(3, 1.0 / D.eps_env), np.ones(3)])
    q6 = D.to6(q)
    # Wirtinger partials of sigma_sca = ext - abs
    g_q = w_sca * C[None, :] * (np.conj(F0) / 2j - np.conj(F) / 2j)
    g_q6 = D.to6(g_q) + w_sca * C[None, None, :] * (2.0 / 3.0) * D.k ** 3 * (
        D.rho[:, None, None] * wq[None, :, None] * np.conj(q6))
    g_q = D.from6(g_q6)
    g_F = w_sca * C[None, :] * (np.conj(q) / 2j)
    g_F0 = w_sca * C[None, :] * (-np.conj(q) / 2j)
    # probes
    if P and w_nf:
        E_inc, H_inc = planewave(rp, wl["khat"], wl["e0"], D.k0, D.n_env)
        Es, _ = scattered_fields(D, q, rp)
        Etot = E_inc + Es  # [rhs, P, 3]
        g_Ep = w_nf * np.conj(Etot) / e2[:, None, None]
        # g_qe contribution: sum_p g_Ep[r,p,a] G6(r_p - r_j)[a, b]
        acc = np.zeros((D.N, 6, nrhs), dtype=np.complex128)
        for p0 in range(0, P, 256):
            p1 = min(P, p0 + 256)
            g6 = green6(rp[p0:p1, None, :] - D.pos[None, :, :], D.k0, D.n_env)
            acc += np.einsum("rpa,pjab->jbr", g_Ep[:, p0:p1], g6[:, :, 0:3, :])
        g_qe = g_q + D.from6(acc)
    else:
        g_Ep = None
        g_qe = g_q
    A = D.alpha_matrix()
    lam = sla.lu_solve(lu, g_F + A.T @ g_qe, trans=1, check_finite=False)
    v = Gt.T @ lam + g_qe  # (lam^T G~ + g_qe)^T
    # permittivity of cells: dA_j = d^3/(4 pi) deps I3
    v6 = D.to6(v)
    F6 = D.to6(F)
    s = np.sum(v6[: D.nc, 0:3] * F6[: D.nc, 0:3], axis=(1, 2)) * D.step ** 3 / FOUR_PI
    g_eps_re = 2.0 * np.real(s)
    g_eps_im = 2.0 * np.real(1j * s)
    # positions
    lam6 = D.to6(lam)
    lg6 = D.to6(lam + g_F0)
    F06 = D.to6(F0)
    g_r = np.zeros((D.N, 3))
    khat = np.atleast_2d(wl["khat"])
    # incident phase: dF0_m / dr_m,a = i k khat_a F0_m
    for a in range(3):
        g_r[:, a] += 2.0 * np.real(np.einsum("dcr,dcr,r->d", lg6, F06, 1j * D.k * khat[:, a]))
    # pair terms
    for i0 in range(0, D.N, 64):
        i1 = min(D.N, i0 + 64)
        R = D.pos[i0:i1, None, :] - D.pos[None, :, :]
        same = np.all(R == 0.0, axis=-1)
        dg = dgreen6_dR(np.where(same[..., None], 1.0, R), D.k0, D.n_env)  # [c, N, 3, 6, 6]
        dg[same] = 0.0
        # rows i in chunk (m = i): lam_i^T dG(r_i - r_j) q_j
        t1 = np.einsum("iar,ijxab,jbr->ix", lam6[i0:i1], dg, q6)
        g_r[i0:i1] += 2.0 * np.real(t1)
        # columns j (m = j): - lam_i^T dG(r_i - r_j) q_j
        t2 = np.einsum("iar,ijxab,jbr->jx", lam6[i0:i1], dg, q6)
        g_r -= 2.0 * np.real(t2)
    if g_Ep is not None:
        for p0 in range(0, P, 128):
            p1 = min(P, p0 + 128)
            dg = dgreen6_dR(rp[p0:p1, None, :] - D.pos[None, :, :], D.k0, D.n_env)
            t = np.einsum("rpa,pjxab,jbr->jx", g_Ep[:, p0:p1], dg[:, :, :, 0:3, :], q6)
            g_r -= 2.0 * np.real(t)
    # wavelength through k0
    dLdk0 = 0.0
    for i0 in range(0, D.N, 64):
        i1 = min(D.N, i0 + 64)
        R = D.pos[i0:i1, None, :] - D.pos[None, :, :]
        same = np.all(R == 0.0, axis=-1)
        dg = dgreen6_dk0(np.where(same[..., None], 1.0, R), D.k0, D.n_env)
        dg[same] = 0.0
        dLdk0 += 2.0 * np.real(np.einsum("iar,ijab,jbr->", lam6[i0:i1], dg, q6))
    if D.mode == "radiative":
        dS = 1j * 2.0 * D.k ** 2 * D.n_env / D.eps_env
        dLdk0 += 2.0 * np.real(dS * np.sum(lam6[: D.nc, 0:3] * q6[: D.nc, 0:3]))
    kr = D.pos @ khat.T  # [N, rhs]
    dLdk0 += 2.0 * np.real(np.sum(lg6 * (1j * D.n_env * kr)[:, None, :] * F06))
    # explicit dependence through C(k0) (sigma proportional to k0) and (2/3) k^3
    sig = cross_sections(D, F0, F, q, e2)
    prad_eff = (2.0 / 3.0) * D.k ** 3 * np.einsum("c,dcr->r", wq, D.rho[:, None, None] * np.abs(q6) ** 2)
    dLdk0 += w_sca * float(np.sum(sig["sca"] / D.k0))
    dLdk0 += w_sca * float(np.sum(C * prad_eff * 3.0 / D.k0))
    if g_Ep is not None:
        E_inc, _ = planewave(rp, wl["khat"], wl["e0"], D.k0, D.n_env)
        dEinc = E_inc * (1j * D.n_env * (rp @ khat.T)).T[:, :, None]
        dLdk0 += 2.0 * np.real(np.sum(g_Ep * dEinc))
        for p0 in range(0, P, 256):
            p1 = min(P, p0 + 256)
            dg = dgreen6_dk0(rp[p0:p1, None, :] - D.pos[None, :, :], D.k0, D.n_env)
            dLdk0 += 2.0 * np.real(np.einsum("rpa,pjab,jbr->", g_Ep[:, p0:p1], dg[:, :, 0:3, :], q6))
    g_wl = dLdk0 * (-D.k0 / D.wavelength)
    return dict(r=g_r, eps_re=g_eps_re, eps_im=g_eps_im, wavelength=g_wl,
                loss=w_sca * float(np.sum(sig["sca"])) + (
                    w_nf * float(np.sum(np.sum(np.abs(Etot) ** 2, axis=(1, 2)) / e2)) if g_Ep is not None else 0.0))
