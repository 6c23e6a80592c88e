"""torch.autograd.Function over the GDM hot path (forward and hand-written adjoint
in libgdm; this module only marshals tensors).

    sim = GDMSetup(ctx, step=8.0, n_env=1.0, khat=..., e0=..., r_probe=...)
    sigma, E = GDMFunction.apply(r_cell, eps_cell, wavelength, None, sim)
    loss = sigma[:, 1].sum() + (E.abs() ** 2).sum() / P
    loss.backward()        # r_cell.grad, eps_cell.grad, wavelength.grad

Outputs: sigma [n_rhs, 3] = (extinction, scattering, absorption) in nm^2 and the
TOTAL electric field E = E_inc + E_sca [n_rhs, P, 3] at the probes.  Inputs that
can carry gradients: cell positions r_cell [n_cell, 3] (float64), cell
permittivities eps_cell [n_cell] (complex128), the wavelength (0-d float64
tensor, nm) and the effective-dipole positions r_eff [n_eff, 3] (or None).  The
paper differentiates its PyTorch solver with autograd (Sec. "Example: Autograd
for resonance search"); here the backward pass is the adjoint of include/gdm.h,
which reuses the LU factors of the forward pass.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import gdm


@dataclass
class GDMSetup:
    """Non-differentiable settings of one GDMFunction call."""
    ctx: "gdm.Context"
    step: float
    n_env: float
    khat: torch.Tensor            # [n_rhs, 3] float64
    e0: torch.Tensor              # [n_rhs, 3] complex128
    r_probe: torch.Tensor = None  # [P, 3] float64 (None: no field output)
    alpha_eff: torch.Tensor = None  # [n_eff, 6, 6] complex128
    prec: int = gdm.PREC_FP64
    tol: float = 0.0
    selfterm: int = gdm.SELF_STATIC


def _forward(sim: GDMSetup, r_cell, eps_cell, wl: float, r_eff):
    c = sim.ctx
    c.set_environment(sim.n_env)
    c.set_structure(r_cell, sim.step, eps_cell, r_eff, sim.alpha_eff, sim.selfterm)
    c.factorize(wl, sim.prec)
    khat = c._dev(sim.khat, torch.float64, None, "khat").reshape(-1, 3)
    e0 = c._dev(sim.e0, torch.complex128, None, "e0").reshape(-1, 3)
    f0 = c.incident_planewave(khat, e0)
    q, f = c.solve(f0, tol=sim.tol)
    e2 = c.planewave_intensity(e0)
    cs = c.cross_sections(f0, q, f, e2)[:, :3].contiguous()
    if sim.r_probe is not None and len(sim.r_probe):
        E, _ = c.fields_total(q, khat, e0, sim.r_probe, want_h=False)
    else:
        E = torch.zeros((len(khat), 0, 3), dtype=torch.complex128, device=c.device)
    return khat, e0, f0, q, f, cs, E


class GDMFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, r_cell, eps_cell, wavelength, r_eff, sim: GDMSetup):
        wl = float(wavelength)
        khat, e0, f0, q, f, cs, E = _forward(sim, r_cell.detach(), eps_cell.detach(), wl,
                                             None if r_eff is None else r_eff.detach())
        fctx.sim = sim
        fctx.wl = wl
        fctx.has_eff = r_eff is not None
        fctx.state = sim.ctx.state_id
        fctx.wl_shape = wavelength.shape if isinstance(wavelength, torch.Tensor) else None
        fctx.save_for_backward(r_cell, eps_cell, r_eff if r_eff is not None else torch.empty(0), khat, e0, f0, q, f)
        return cs, E

    @staticmethod
    def backward(fctx, g_cs, g_E):
        sim = fctx.sim
        r_cell, eps_cell, r_eff, khat, e0, f0, q, f = fctx.saved_tensors
        c = sim.ctx
        if c.state_id != fctx.state:
            # the context was used for another system since this forward: restore the factors
            _, _, f0, q, f, _, _ = _forward(sim, r_cell.detach(), eps_cell.detach(), fctx.wl,
                                            r_eff.detach() if fctx.has_eff else None)
        g_sigma = None if g_cs is None else g_cs.detach().to(torch.float64).contiguous()
        g_e = None
        if g_E is not None and g_E.numel():
            g_e = (g_E.detach().conj() * 0.5).contiguous()  # torch passes 2 conj(dL/dE)
        grad_r, grad_eps2, grad_wl = c.adjoint(khat, e0, f0, q, f, g_sigma=g_sigma,
                                               r_probe=sim.r_probe if g_e is not None else None, g_e=g_e,
                                               tol=sim.tol)
        nc = r_cell.shape[0]
        g_rc = grad_r[:nc].to(r_cell.dtype)
        g_eps = torch.complex(grad_eps2[:, 0], grad_eps2[:, 1]).to(eps_cell.dtype)
        g_wl = grad_wl.reshape(fctx.wl_shape) if fctx.wl_shape is not None else None
        g_re = grad_r[nc:].to(r_eff.dtype) if fctx.has_eff else None
        return g_rc, g_eps, g_wl, g_re, None


def gdm_forward(r_cell, eps_cell, wavelength, sim: GDMSetup, r_eff=None):
    """Differentiable forward: returns (sigma [n_rhs, 3], E_total [n_rhs, P, 3])."""
    return GDMFunction.apply(r_cell, eps_cell, wavelength, r_eff, sim)
