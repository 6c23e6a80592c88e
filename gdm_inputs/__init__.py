"""Seeded synthetic workloads for the Green's Dyadic Method (GDM) hot path.

This module only builds inputs: dipole positions, cell step, permittivities,
effective polarisability tensors, plane-wave directions/polarisations and probe
points.  It holds none of the method's arithmetic (no Green's tensors, no
linear algebra, no observables), so that both the CPU oracle and the HIP path
can be fed from it without sharing code.

The structures follow the kinds of workload the paper simulates: volume
discretisations of spheres and cuboids on a cubic grid (Sec. "Volume
discretization polarizabilities"), lattices of effective point dipoles mixed
with a discretised structure (Sec. "Hybrid discretization GDM", Fig.
"coupling_matrix"), plane-wave illuminations (Appendix, 3D illuminations) and
probe planes / spheres for near and far fields (Sec. "Observables").

Units: lengths and wavelengths in nm.  Time convention exp(-i w t).
Every random draw uses ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

HC_EV_NM = 1239.84193  # hbar*omega [eV] = HC_EV_NM / lambda [nm]


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------
def sphere_cells(radius_nm: float, step_nm: float) -> np.ndarray:
    """Cubic-grid nodes d*(i,j,k) with |r| <= radius (node at the origin)."""
    m = int(math.floor(radius_nm / step_nm)) + 1
    ax = np.arange(-m, m + 1)
    i, j, k = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * step_nm
    keep = np.sum(pts * pts, axis=1) <= radius_nm * radius_nm * (1 + 1e-12)
    return np.ascontiguousarray(pts[keep])


def cuboid_cells(na: int, nb: int, nc: int, step_nm: float) -> np.ndarray:
    """na x nb x nc cells, centred on the origin, C order (x slowest)."""
    ax = [(np.arange(n) - (n - 1) / 2.0) * step_nm for n in (na, nb, nc)]
    x, y, z = np.meshgrid(*ax, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))


def ellipsoid_cells(semi: np.ndarray, step_nm: float) -> np.ndarray:
    """Grid nodes (node at the origin) inside the ellipsoid with semi-axes ``semi``."""
    m = [int(math.floor(s / step_nm)) + 1 for s in semi]
    ax = [np.arange(-mm, mm + 1) * step_nm for mm in m]
    x, y, z = np.meshgrid(*ax, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    keep = np.sum((pts / semi[None, :]) ** 2, axis=1) <= 1.0 + 1e-12
    return np.ascontiguousarray(pts[keep])


def box_cells(half: np.ndarray, step_nm: float) -> np.ndarray:
    """Grid nodes (node at the origin) inside the box |x_a| <= half_a."""
    m = [int(math.floor(h / step_nm + 1e-12)) for h in half]
    ax = [np.arange(-mm, mm + 1) * step_nm for mm in m]
    x, y, z = np.meshgrid(*ax, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))


def zcylinder_cells(radii: np.ndarray, half_h: float, step_nm: float) -> np.ndarray:
    """Grid nodes inside an elliptic cylinder along z (semi-axes radii[0:2], half height)."""
    m = [int(math.floor(r / step_nm)) + 1 for r in radii[:2]]
    mz = int(math.floor(half_h / step_nm + 1e-12))
    ax = [np.arange(-mm, mm + 1) * step_nm for mm in m] + [np.arange(-mz, mz + 1) * step_nm]
    x, y, z = np.meshgrid(*ax, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    keep = (pts[:, 0] / radii[0]) ** 2 + (pts[:, 1] / radii[1]) ** 2 <= 1.0 + 1e-12
    return np.ascontiguousarray(pts[keep])


def fibonacci_sphere(n: int, radius_nm: float) -> np.ndarray:
    """Deterministic golden-angle spiral of n points on a sphere."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - 2.0 * (i + 0.5) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius_nm * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def probe_plane(nx: int, ny: int, half_x: float, half_y: float, z_nm: float) -> np.ndarray:
    x = np.linspace(-half_x, half_x, nx)
    y = np.linspace(-half_y, half_y, ny)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), np.full(X.size, z_nm)], axis=1))


def random_planewaves(rng: np.random.Generator, n: int):
    """n plane waves: direction uniform on the sphere, real linear polarisation
    orthogonal to it (normalised Gaussian draws)."""
    k = rng.standard_normal((n, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    g = rng.standard_normal((n, 3))
    e = g - np.sum(g * k, axis=1, keepdims=True) * k
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    return k, e.astype(np.complex128)


def normal_incidence_xy():
    khat = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    e0 = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], dtype=np.complex128)
    return khat, e0


def _empty_eff():
    return np.zeros((0, 3)), np.zeros((0, 6, 6), dtype=np.complex128)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def config1() -> Dict:
    """Sphere r=40 nm on a 10 nm grid (257 cells), eps 12+0.1i, vacuum,
    lambda 600 nm, +z plane waves polarised x and y, 1000 probes on a 200 nm
    sphere (Fibonacci lattice).  No random numbers."""
    r = sphere_cells(40.0, 10.0)
    khat, e0 = normal_incidence_xy()
    r_eff, a_eff = _empty_eff()
    return dict(name="sphere257_eps12_l600", r_cell=r, step=10.0,
                eps_cell=np.full(len(r), 12.0 + 0.1j), n_env=1.0, wavelength=600.0,
                khat=khat, e0=e0, r_probe=fibonacci_sphere(1000, 200.0),
                r_eff=r_eff, alpha_eff=a_eff)


def _cuboid_triples(ncell: int, max_ratio: float) -> List[tuple]:
    out = []
    for a in range(1, ncell + 1):
        if ncell % a:
            continue
        for b in range(1, ncell // a + 1):
            if (ncell // a) % b:
                continue
            c = ncell // (a * b)
            if max(a, b, c) <= max_ratio * min(a, b, c):
                out.append((a, b, c))
    return out


def config2(seed: int = 2, ncell: int = 4000, n_random_pw: int = 64) -> Dict:
    """Random-aspect cuboid of ``ncell`` cells on a 5 nm grid, per-cell eps with
    Re ~ U[2,16], Im ~ U[0,1], n_env 1.33, lambda 550 nm, RHS: +z x/y plus
    ``n_random_pw`` random plane waves."""
    rng = np.random.default_rng(seed)
    triples = _cuboid_triples(ncell, 8.0)
    a, b, c = triples[int(rng.integers(len(triples)))]
    r = cuboid_cells(a, b, c, 5.0)
    eps = rng.uniform(2.0, 16.0, len(r)) + 1j * rng.uniform(0.0, 1.0, len(r))
    k0, e0 = normal_incidence_xy()
    k1, e1 = random_planewaves(rng, n_random_pw)
    r_eff, a_eff = _empty_eff()
    return dict(name=f"cuboid{a}x{b}x{c}_d5_nenv1.33_l550", r_cell=r, step=5.0, eps_cell=eps,
                n_env=1.33, wavelength=550.0, khat=np.concatenate([k0, k1]),
                e0=np.concatenate([e0, e1]), r_probe=np.zeros((0, 3)),
                r_eff=r_eff, alpha_eff=a_eff, dims=(a, b, c))


def drude_lorentz(wavelength_nm, p: Dict) -> np.ndarray:
    """eps(w) = eps_inf - wp^2/(w^2 + i gD w) + de * wL^2/(wL^2 - w^2 - i gL w), w in eV."""
    w = HC_EV_NM / np.asarray(wavelength_nm, dtype=np.float64)
    return (p["eps_inf"] - p["wp"] ** 2 / (w * w + 1j * p["gD"] * w)
            + p["de"] * p["wL"] ** 2 / (p["wL"] ** 2 - w * w - 1j * p["gL"] * w))


def _shape_cells(shape: str, ratios: np.ndarray, scale: float, step: float) -> np.ndarray:
    semi = scale * ratios
    if shape == "ellipsoid":
        return ellipsoid_cells(semi, step)
    if shape == "cuboid":
        return box_cells(semi, step)
    return zcylinder_cells(semi, semi[2], step)


def config3(seed: int = 3, n_struct: int = 32, n_wl: int = 128) -> Dict:
    """32 random structures (ellipsoid / cuboid / z-cylinder) of 300..3000 cells on
    a 10 nm grid, each with its own Drude-Lorentz permittivity, 128 wavelengths
    in 400..900 nm, +z plane waves polarised x and y."""
    rng = np.random.default_rng(seed)
    step = 10.0
    shapes = ("ellipsoid", "cuboid", "zcylinder")
    structs = []
    while len(structs) < n_struct:
        shape = shapes[int(rng.integers(3))]
        n_target = int(rng.integers(300, 3001))
        ratios = rng.uniform(0.5, 2.0, 3)
        lo, hi = 1.0, 400.0
        for _ in range(60):  # bisect the scale on the cell count
            mid = 0.5 * (lo + hi)
            if len(_shape_cells(shape, ratios, mid, step)) < n_target:
                lo = mid
            else:
                hi = mid
        cand = [_shape_cells(shape, ratios, s, step) for s in (lo, hi)]
        best = min(cand, key=lambda c: abs(len(c) - n_target))
        if not (300 <= len(best) <= 3000):
            continue
        dl = dict(eps_inf=rng.uniform(1.5, 3.0), de=rng.uniform(1.0, 6.0),
                  wL=rng.uniform(4.0, 5.5), gL=rng.uniform(0.05, 0.3),
                  wp=rng.uniform(0.0, 1.5), gD=rng.uniform(0.05, 0.2))
        structs.append(dict(shape=shape, r_cell=best, dl=dl))
    wl = np.linspace(400.0, 900.0, n_wl)
    eps = np.stack([drude_lorentz(wl, s["dl"]) for s in structs])  # [n_struct][n_wl]
    khat, e0 = normal_incidence_xy()
    return dict(name="batch32x128", structs=structs, step=step, wavelengths=wl, eps=eps,
                n_env=1.0, khat=khat, e0=e0)


def config4() -> Dict:
    """Cuboid 10x10x20 cells, 8 nm grid (N = 2000), eps 10+0.05i, vacuum,
    lambda 700 nm, +z x-polarised, 64x64 probes on z = -150 nm."""
    r = cuboid_cells(10, 10, 20, 8.0)
    r_eff, a_eff = _empty_eff()
    return dict(name="cuboid10x10x20_d8_l700", r_cell=r, step=8.0,
                eps_cell=np.full(len(r), 10.0 + 0.05j), n_env=1.0, wavelength=700.0,
                khat=np.array([[0.0, 0.0, 1.0]]), e0=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128),
                r_probe=probe_plane(64, 64, 200.0, 200.0, -150.0), r_eff=r_eff, alpha_eff=a_eff)


def mie_like_alpha6(rng: np.random.Generator, n: int, wavelength: float, n_env: float,
                    a_nm: float = 50.0, eps_s: float = 12.0) -> np.ndarray:
    """Seeded random 6x6 polarisabilities scaled like a small dielectric sphere.

    Electric part: quasistatic sphere polarisability with radiative correction;
    magnetic part a quarter of it; both perturbed by 10 % complex Gaussian noise
    in every entry (an input recipe, not part of the method)."""
    eps_env = n_env * n_env
    k = 2.0 * math.pi / wavelength * n_env
    ae0 = eps_env * a_nm ** 3 * (eps_s - eps_env) / (eps_s + 2 * eps_env)
    ae = 1.0 / (1.0 / ae0 - 1j * (2.0 / 3.0) * k ** 3 / eps_env)
    am0 = 0.25 * ae0 / eps_env
    am = 1.0 / (1.0 / am0 - 1j * (2.0 / 3.0) * k ** 3)
    base = np.diag(np.array([ae, ae, ae, am, am, am], dtype=np.complex128))
    X = rng.standard_normal((n, 6, 6))
    Y = rng.standard_normal((n, 6, 6))
    return base[None, :, :] * (1.0 + 0.1 * (X + 1j * Y))


def config5(seed: int = 5, lattice: int = 100, sub: tuple = None, probes: int = 1000) -> Dict:
    """3000-cell cuboid (15x20x10, 6 nm grid, eps 6+0.2i) inside a 100x100
    lattice (period 300 nm, z = 0) of effective ED+MD dipoles with seeded 6x6
    polarisabilities; lambda 650 nm, +z x-polarised; probes on z = -100 nm.

    ``sub=(i0, i1)`` keeps only lattice sites i, j in [i0, i1) (with the same
    per-site draws as the full lattice), the reduced replica used where the
    dense FP64 oracle does not fit in memory."""
    rng = np.random.default_rng(seed)
    wl, n_env = 650.0, 1.0
    a6 = mie_like_alpha6(rng, lattice * lattice, wl, n_env)
    ii, jj = np.meshgrid(np.arange(lattice), np.arange(lattice), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    c = (lattice - 1) / 2.0
    r_eff = np.stack([(ii - c) * 300.0, (jj - c) * 300.0, np.zeros(ii.size)], axis=1)
    if sub is not None:
        keep = (ii >= sub[0]) & (ii < sub[1]) & (jj >= sub[0]) & (jj < sub[1])
        r_eff, a6 = r_eff[keep], a6[keep]
    r = cuboid_cells(15, 20, 10, 6.0)
    half = 15000.0 * (lattice / 100.0)
    return dict(name="hybrid3000_lattice%d" % lattice, r_cell=r, step=6.0,
                eps_cell=np.full(len(r), 6.0 + 0.2j), n_env=n_env, wavelength=wl,
                khat=np.array([[0.0, 0.0, 1.0]]), e0=np.array([[1.0, 0.0, 0.0]], dtype=np.complex128),
                r_probe=probe_plane(probes, probes, half, half, -100.0),
                r_eff=np.ascontiguousarray(r_eff), alpha_eff=np.ascontiguousarray(a6))


def small_mixed(seed: int = 11, n_cell_side: int = 3, n_eff: int = 4) -> Dict:
    """A small cells + 6x6-dipoles system for exercising the 6N layout."""
    rng = np.random.default_rng(seed)
    r = cuboid_cells(n_cell_side, n_cell_side, n_cell_side, 8.0)
    eps = 4.0 + rng.uniform(0, 8, len(r)) + 1j * rng.uniform(0, 0.5, len(r))
    wl, n_env = 600.0, 1.2
    ang = np.arange(n_eff) * 2 * math.pi / max(n_eff, 1)
    r_eff = np.stack([160 * np.cos(ang), 160 * np.sin(ang), 20.0 * np.arange(n_eff)], axis=1)
    a6 = mie_like_alpha6(rng, n_eff, wl, n_env, a_nm=30.0)
    k, e = random_planewaves(rng, 3)
    return dict(name="mixed_small", r_cell=r, step=8.0, eps_cell=eps, n_env=n_env,
                wavelength=wl, khat=k, e0=e, r_probe=fibonacci_sphere(50, 400.0),
                r_eff=r_eff, alpha_eff=a6)
