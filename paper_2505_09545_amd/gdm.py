"""Thin ctypes binding of libgdm (include/gdm.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of libgdm.so.  Torch tensors are used as device buffers; each context runs on
its own stream, ordered with the caller's current torch stream around every
call.  There is no CPU fallback: importing this module without the built
library raises.

Layouts follow the C header: complex arrays are torch.complex128 tensors
(interleaved re/im doubles); vectors in the unknown layout are [n_rhs, n];
dense matrices are column-major, i.e. returned as the transpose of a
row-major tensor.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdm.so")

GDM_OK, GDM_E_ARG, GDM_E_OOM, GDM_E_DEVICE, GDM_E_SINGULAR, GDM_E_NOCONV, GDM_E_PROBE_AT_DIPOLE, GDM_E_STATE = range(8)
STATUS_NAMES = ["OK", "E_ARG", "E_OOM", "E_DEVICE", "E_SINGULAR", "E_NOCONV", "E_PROBE_AT_DIPOLE", "E_STATE"]
PREC_FP64, PREC_FP32_IR = 0, 1
SELF_STATIC, SELF_RADIATIVE = 0, 1

EXPORTED = ["gdm_create", "gdm_destroy", "gdm_last_error", "gdm_set_memory_limit", "gdm_memory_used", "gdm_set_pivoting",
            "gdm_pivot_fallbacks",
            "gdm_set_environment", "gdm_set_structure", "gdm_set_gpm", "gdm_extract_gpm",
            "gdm_num_unknowns", "gdm_assemble", "gdm_factorize", "gdm_set_wavelength", "gdm_solve_iterative", "gdm_incident_planewave", "gdm_solve",
            "gdm_planewave", "gdm_fields", "gdm_fields_total", "gdm_planewave_intensity", "gdm_fields_noalloc", "gdm_cross_sections", "gdm_multipoles", "gdm_extract_dipole_pair", "gdm_dipole_sources", "gdm_ldos", "gdm_green_tensor", "gdm_adjoint", "gdm_batch_spectra", "gdm_batch_tuning", "gdm_getrf", "gdm_getrs", "gdm_gemm", "gdm_sync",
            "gdm_profile", "gdm_profile_mask", "gdm_profile_read"]


class GDMInfo(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int32), ("backward_err", ctypes.c_double), ("bad_index", ctypes.c_int64),
                ("ms_assemble", ctypes.c_float), ("ms_factor", ctypes.c_float), ("ms_solve", ctypes.c_float),
                ("ms_ir", ctypes.c_float)]


class GDMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgdm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libgdm.so not found at {path}; build it with python -m paper_2505_09545_amd.build")
    lib = ctypes.CDLL(path)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "gdm_create": ([ctypes.c_int, P, ctypes.POINTER(P)], ctypes.c_int),
        "gdm_destroy": ([P], None),
        "gdm_last_error": ([P], ctypes.c_char_p),
        "gdm_set_memory_limit": ([P, I64], ctypes.c_int),
        "gdm_memory_used": ([P], I64),
        "gdm_set_pivoting": ([P, I32], ctypes.c_int),
        "gdm_pivot_fallbacks": ([P], I64),
        "gdm_set_environment": ([P, D], ctypes.c_int),
        "gdm_set_structure": ([P, I64, P, D, P, I64, P, P, ctypes.c_int], ctypes.c_int),
        "gdm_num_unknowns": ([P], I64),
        "gdm_set_gpm": ([P, I64, ctypes.POINTER(I64), ctypes.POINTER(I64), P], ctypes.c_int),
        "gdm_extract_gpm": ([P, I64, P, P, I64, P, P, I64, P, I64, P, D, I32, P, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_assemble": ([P, D, ctypes.c_int, P, I64], ctypes.c_int),
        "gdm_factorize": ([P, D, ctypes.c_int, ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_set_wavelength": ([P, D], ctypes.c_int),
        "gdm_solve_iterative": ([P, D, I64, P, D, I32, I32, P, P, ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_incident_planewave": ([P, I64, P, P, P], ctypes.c_int),
        "gdm_solve": ([P, I64, P, D, I32, P, P, ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_planewave": ([P, I64, P, P, I64, P, P, P], ctypes.c_int),
        "gdm_fields": ([P, I64, P, I64, P, P, P], ctypes.c_int),
        "gdm_fields_noalloc": ([P, I64, P, I64, P, P, P], ctypes.c_int),
        "gdm_fields_total": ([P, I64, P, P, P, I64, P, P, P], ctypes.c_int),
        "gdm_planewave_intensity": ([P, I64, P, P], ctypes.c_int),
        "gdm_cross_sections": ([P, I64, P, P, P, P, I32, P], ctypes.c_int),
        "gdm_multipoles": ([P, I64, P, ctypes.POINTER(ctypes.c_double), P, P, P, P], ctypes.c_int),
        "gdm_extract_dipole_pair": ([P, I64, P, P, I64, P, P, ctypes.POINTER(ctypes.c_double), D, I32, P,
                                     ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
        "gdm_dipole_sources": ([P, I64, P, P, P], ctypes.c_int),
        "gdm_ldos": ([P, I64, P, D, I32, P, ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_green_tensor": ([P, I64, P, I64, P, D, I32, P, ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_adjoint": ([P, I64, P, P, P, P, P, P, I64, P, P, D, I32, P, P, P, ctypes.POINTER(GDMInfo)],
                        ctypes.c_int),
        "gdm_batch_spectra": ([P, I64, P, P, P, I64, P, P, I64, P, P, ctypes.c_int, I32, D, ctypes.c_int, P, P,
                               ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_batch_tuning": ([P, P, I32], I32),
        "gdm_getrf": ([P, ctypes.c_int, I64, P, I64, P, ctypes.POINTER(GDMInfo)], ctypes.c_int),
        "gdm_getrs": ([P, ctypes.c_int, ctypes.c_int, I64, I64, P, I64, P, I64], ctypes.c_int),
        "gdm_gemm": ([P, ctypes.c_int, ctypes.c_int, ctypes.c_int, I64, I64, I64, P, I64, P, I64, P, I64],
                     ctypes.c_int),
        "gdm_sync": ([P], ctypes.c_int),
        "gdm_profile": ([P, ctypes.c_int], ctypes.c_int),
        "gdm_profile_mask": ([P, I32], ctypes.c_int),
        "gdm_profile_read": ([P, ctypes.POINTER(ctypes.c_double), I32], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Structure:
    r_cell: torch.Tensor  # [nc, 3] float64
    step: float
    eps_cell: torch.Tensor  # [nc] complex128
    r_eff: torch.Tensor = None  # [ne, 3] float64
    alpha_eff: torch.Tensor = None  # [ne, 6, 6] complex128


class Context:
    """One libgdm context on a CUDA (HIP) device.

    The library's work runs on `stream` (default: a new torch stream of default
    priority owned by this context).  Every call is ordered with the caller's
    current torch stream in both directions: the library stream first waits for
    the current stream (inputs produced there are complete), and afterwards the
    current stream waits for the library stream (outputs are complete before
    torch reads them, and torch's allocator does not reuse their memory early)."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.Stream(device=self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.gdm_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), None)
        self.h = h
        self.info = GDMInfo()
        self._keep = []
        # bumped by every call that replaces the structure or the factors
        self.state_id = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.gdm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        """Call library function `name` ordered with the current torch stream."""
        cur = torch.cuda.current_stream(self.device)
        other = cur.cuda_stream != self.stream.cuda_stream
        if other:
            self.stream.wait_stream(cur)
        st = getattr(self.lib, name)(*args)
        if other:
            cur.wait_stream(self.stream)
        return st

    def _check(self, st, h="self"):
        if st != GDM_OK:
            msg = self.lib.gdm_last_error(self.h if h == "self" else None).decode()
            raise GDMError(st, msg)

    def _dev(self, t, dtype, shape=None, name="array"):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def set_memory_limit(self, nbytes: int = 0):
        """Limit on the device bytes of this context's buffers (0: none); calls
        that would exceed it fail with GDM_E_OOM (include/gdm.h)."""
        self._check(self._call("gdm_set_memory_limit", self.h, int(nbytes)))

    def memory_used(self) -> int:
        return int(self.lib.gdm_memory_used(self.h))

    def set_pivoting(self, columns_per_exchange: int = 0):
        """Panel columns per pivot exchange of the next factorisations
        (include/gdm.h, gdm_set_pivoting): 1 partial pivoting with the search in
        every column, 2/4/8 tournament, 0 the default (speculative partial
        pivoting in factorize)."""
        self._check(self._call("gdm_set_pivoting", self.h, int(columns_per_exchange)))

    def pivot_fallbacks(self) -> int:
        """Factorisations whose speculative pivots failed their check and were
        repeated with the pivot search (gdm_pivot_fallbacks)."""
        return int(self.lib.gdm_pivot_fallbacks(self.h))

    # -- structure / environment ------------------------------------------------
    def set_environment(self, n_env: float):
        self.state_id += 1
        self._check(self._call("gdm_set_environment", self.h, float(n_env)))

    def set_structure(self, r_cell, step, eps_cell, r_eff=None, alpha_eff=None, selfterm=SELF_STATIC):
        nc = 0 if r_cell is None else len(r_cell)
        ne = 0 if r_eff is None else len(r_eff)
        rc = self._dev(r_cell, torch.float64, (nc, 3), "r_cell") if nc else None
        ec = self._dev(eps_cell, torch.complex128, (nc,), "eps_cell") if nc else None
        re = self._dev(r_eff, torch.float64, (ne, 3), "r_eff") if ne else None
        ae = self._dev(alpha_eff, torch.complex128, (ne, 6, 6), "alpha_eff") if ne else None
        self._keep = [rc, ec, re, ae]
        self.state_id += 1
        self._check(self._call("gdm_set_structure", self.h, nc, _ptr(rc), float(step), _ptr(ec), ne, _ptr(re), _ptr(ae),
                                               int(selfterm)))
        self.n_cell, self.n_eff = nc, ne

    def set_gpm(self, groups):
        """Global polarisability matrices (gdm_set_gpm): groups = [(first, alpha_G)]
        with alpha_G [6M, 6M] complex for the effective dipoles [first, first + M);
        an empty list removes the groups."""
        firsts, sizes, mats = [], [], []
        for first, aG in groups:
            aG = self._dev(aG, torch.complex128, None, "alpha_G")
            if aG.dim() != 2 or aG.shape[0] != aG.shape[1] or aG.shape[0] % 6:
                raise ValueError("alpha_G must be [6M, 6M]")
            firsts.append(int(first))
            sizes.append(aG.shape[0] // 6)
            mats.append(aG.reshape(-1))
        ng = len(firsts)
        alpha = torch.cat(mats) if ng else None
        fa = (ctypes.c_int64 * max(ng, 1))(*firsts)
        sa = (ctypes.c_int64 * max(ng, 1))(*sizes)
        self._keep_gpm = alpha
        self.state_id += 1
        self._check(self._call("gdm_set_gpm", self.h, ng, fa, sa, _ptr(alpha)))

    def extract_gpm(self, r_gpm, r_probe, khat=None, e0=None, r_src=None, d_src=None, tol=0.0, max_iter=-1):
        """GPM of the structure for pairs at r_gpm [M, 3] by scattered-field
        matching at r_probe [P, 3] under plane waves (khat, e0) and point sources
        (r_src, d_src) (gdm_extract_gpm; needs factors).  Returns (alpha_G
        [6M, 6M] complex on the device, (field-fit residual, alpha-fit residual))."""
        k = e = rs = ds = None
        npw = nsrc = 0
        if khat is not None:
            k = self._dev(khat, torch.float64, None, "khat").reshape(-1, 3)
            e = self._dev(e0, torch.complex128, (len(k), 3), "e0")
            npw = len(k)
        if r_src is not None:
            rs = self._dev(r_src, torch.float64, None, "r_src").reshape(-1, 3)
            ds = self._dev(d_src, torch.complex128, (len(rs), 6), "d_src")
            nsrc = len(rs)
        rg = self._dev(r_gpm, torch.float64, None, "r_gpm").reshape(-1, 3)
        rp = self._dev(r_probe, torch.float64, None, "r_probe").reshape(-1, 3)
        M = len(rg)
        alpha = torch.empty((6 * M, 6 * M), dtype=torch.complex128, device=self.device)
        res = (ctypes.c_double * 2)(0.0, 0.0)
        self._check(self._call("gdm_extract_gpm", self.h, npw, _ptr(k), _ptr(e), nsrc, _ptr(rs), _ptr(ds), M, _ptr(rg),
                               len(rp), _ptr(rp), float(tol), int(max_iter), _ptr(alpha), res,
                               ctypes.byref(self.info)))
        return alpha, (float(res[0]), float(res[1]))

    @property
    def n(self) -> int:
        return int(self.lib.gdm_num_unknowns(self.h))

    # -- steps ------------------------------------------------------------------------
    def assemble(self, wavelength, dtype=torch.complex128):
        n = self.n
        out = torch.empty((n, n), dtype=dtype, device=self.device)
        self._check(self._call("gdm_assemble", self.h, float(wavelength), 0 if dtype == torch.complex128 else 1,
                                          _ptr(out), n))
        return out.t()  # column-major storage -> M[i, j]

    def factorize(self, wavelength, prec=PREC_FP64):
        self.state_id += 1
        self._check(self._call("gdm_factorize", self.h, float(wavelength), int(prec), ctypes.byref(self.info)))
        return self.info

    def set_wavelength(self, wavelength):
        self.state_id += 1
        self._check(self._call("gdm_set_wavelength", self.h, float(wavelength)))

    def solve_iterative(self, wavelength, f0, tol=0.0, max_iter=0, restart=0, want_field=True):
        """Matrix-free GMRES solve at `wavelength` (include/gdm.h,
        gdm_solve_iterative): returns (q, F); self.info.ir_iters = products with
        M, self.info.backward_err = largest relative residual."""
        f0 = self._dev(f0, torch.complex128, None, "f0")
        if f0.dim() != 2 or f0.shape[1] != self.n:
            raise ValueError(f"f0 must be [n_rhs, {self.n}]")
        q = torch.empty_like(f0)
        f = torch.empty_like(f0) if want_field else None
        self.state_id += 1
        self._check(self._call("gdm_solve_iterative", self.h, float(wavelength), f0.shape[0], _ptr(f0), float(tol),
                               int(max_iter), int(restart), _ptr(q), _ptr(f), ctypes.byref(self.info)))
        return q, f

    def incident_planewave(self, khat, e0):
        k = self._dev(khat, torch.float64, None, "khat").reshape(-1, 3)
        e = self._dev(e0, torch.complex128, None, "e0").reshape(-1, 3)
        if len(k) != len(e):
            raise ValueError("khat and e0 must have the same number of plane waves")
        f0 = torch.empty((len(k), self.n), dtype=torch.complex128, device=self.device)
        self._check(self._call("gdm_incident_planewave", self.h, len(k), _ptr(k), _ptr(e), _ptr(f0)))
        return f0

    def solve(self, f0, tol=0.0, max_iter=-1, want_field=True):
        """Moments q (and fields F) of the right-hand sides f0 [n_rhs, n].  If the
        library runs out of device memory, the right-hand sides are solved in two
        halves, recursively down to one at a time (the paper's restart with a
        smaller batch after an out-of-memory error); self.info then holds the
        largest backward error and correction count over the parts."""
        f0 = self._dev(f0, torch.complex128, None, "f0")
        if f0.dim() != 2 or f0.shape[1] != self.n:
            raise ValueError(f"f0 must be [n_rhs, {self.n}]")
        return self._solve_parts(f0, tol, max_iter, want_field)

    def _solve_parts(self, f0, tol, max_iter, want_field):
        q = torch.empty_like(f0)
        f = torch.empty_like(f0) if want_field else None
        st = self._call("gdm_solve", self.h, f0.shape[0], _ptr(f0), float(tol), int(max_iter), _ptr(q), _ptr(f),
                        ctypes.byref(self.info))
        if st == GDM_E_OOM and f0.shape[0] > 1:
            del q, f
            h = f0.shape[0] // 2
            q1, f1 = self._solve_parts(f0[:h], tol, max_iter, want_field)
            it1, be1 = self.info.ir_iters, self.info.backward_err
            q2, f2 = self._solve_parts(f0[h:], tol, max_iter, want_field)
            self.info.ir_iters = max(it1, self.info.ir_iters)
            self.info.backward_err = max(be1, self.info.backward_err)
            return torch.cat([q1, q2]), (torch.cat([f1, f2]) if want_field else None)
        self._check(st)
        return q, f

    def planewave(self, khat, e0, r, want_h=True):
        k = self._dev(khat, torch.float64, None, "khat").reshape(-1, 3)
        e = self._dev(e0, torch.complex128, None, "e0").reshape(-1, 3)
        r = self._dev(r, torch.float64, None, "r").reshape(-1, 3)
        E = torch.empty((len(k), len(r), 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E) if want_h else None
        self._check(self._call("gdm_planewave", self.h, len(k), _ptr(k), _ptr(e), len(r), _ptr(r), _ptr(E), _ptr(H)))
        return E, H

    def fields(self, q, r_probe, want_h=True):
        """Scattered fields E, H [n_rhs, P, 3] of the moments q at r_probe [P, 3].
        If the library runs out of device memory, the probes are evaluated in
        two halves, recursively down to one probe at a time."""
        q = self._dev(q, torch.complex128, None, "q")
        r = self._dev(r_probe, torch.float64, None, "r_probe").reshape(-1, 3)
        return self._fields_parts(q, r, want_h)

    def _fields_parts(self, q, r, want_h):
        E = torch.empty((q.shape[0], len(r), 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E) if want_h else None
        st = self._call("gdm_fields", self.h, q.shape[0], _ptr(q), len(r), _ptr(r), _ptr(E), _ptr(H))
        if st == GDM_E_OOM and len(r) > 1:
            del E, H
            h = len(r) // 2
            E1, H1 = self._fields_parts(q, r[:h], want_h)
            E2, H2 = self._fields_parts(q, r[h:], want_h)
            return torch.cat([E1, E2], dim=1), (torch.cat([H1, H2], dim=1) if want_h else None)
        self._check(st)
        return E, H

    def fields_total(self, q, khat, e0, r_probe, want_h=True):
        """Total fields E = E_inc + E_sca (and H) [n_rhs, P, 3] at r_probe for the
        moments q of plane waves khat [n_rhs, 3], e0 [n_rhs, 3] (include/gdm.h,
        gdm_fields_total)."""
        q = self._dev(q, torch.complex128, None, "q")
        k = self._dev(khat, torch.float64, (q.shape[0], 3), "khat")
        e = self._dev(e0, torch.complex128, (q.shape[0], 3), "e0")
        r = self._dev(r_probe, torch.float64, None, "r_probe").reshape(-1, 3)
        E = torch.empty((q.shape[0], len(r), 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E) if want_h else None
        self._check(self._call("gdm_fields_total", self.h, q.shape[0], _ptr(q), _ptr(k), _ptr(e), len(r), _ptr(r),
                               _ptr(E), _ptr(H)))
        return E, H

    def planewave_intensity(self, e0):
        """|E0|^2 per plane wave of amplitudes e0 [n_pw, 3] (gdm_planewave_intensity)."""
        e = self._dev(e0, torch.complex128, None, "e0").reshape(-1, 3)
        out = torch.empty(len(e), dtype=torch.float64, device=self.device)
        self._check(self._call("gdm_planewave_intensity", self.h, len(e), _ptr(e), _ptr(out)))
        return out

    def fields_noalloc(self, q, r_probe, E, H=None):
        """gdm_fields_noalloc into caller-allocated outputs E (and H), each
        [n_rhs, P, 3] complex128 on the context's device; allocates nothing on
        the library side (include/gdm.h)."""
        for name, t in (("q", q), ("r_probe", r_probe), ("E", E), ("H", H)):
            if t is not None and (t.device != self.device or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous tensor on {self.device}")
        P = r_probe.shape[0]
        for name, t in (("E", E), ("H", H)):
            if t is not None and (t.dtype != torch.complex128 or tuple(t.shape) != (q.shape[0], P, 3)):
                raise ValueError(f"{name} must be complex128 of shape {(q.shape[0], P, 3)}")
        if q.dtype != torch.complex128 or r_probe.dtype != torch.float64:
            raise ValueError("q must be complex128 and r_probe float64")
        self._check(self._call("gdm_fields_noalloc", self.h, q.shape[0], _ptr(q), P, _ptr(r_probe), _ptr(E), _ptr(H)))

    def cross_sections(self, f0, q, f, e0_norm2, want_ff=False):
        f0 = self._dev(f0, torch.complex128, None, "f0")
        q = self._dev(q, torch.complex128, None, "q")
        f = self._dev(f, torch.complex128, None, "f")
        e2 = self._dev(e0_norm2, torch.float64, (f0.shape[0],), "e0_norm2")
        out = torch.empty((f0.shape[0], 5), dtype=torch.float64, device=self.device)
        self._check(self._call("gdm_cross_sections", self.h, f0.shape[0], _ptr(f0), _ptr(q), _ptr(f), _ptr(e2),
                                                int(bool(want_ff)), _ptr(out)))
        return out

    def multipoles(self, q, r0=None, khat=None, e0=None):
        """Exact multipole moments [n_rhs, 24] complex (p, m, Qe 3x3, Qm 3x3) of
        the mesh cells' polarisation about r0 (default: the cells' mean
        position) and the cross sections [n_rhs, 8] (scattering ED, MD, EQ, MQ,
        then extinction; with plane waves khat, e0 of the RHS) (gdm_multipoles)."""
        q = self._dev(q, torch.complex128, None, "q")
        nr = q.shape[0]
        k = e = None
        if (khat is None) != (e0 is None):
            raise ValueError("khat and e0 go together")
        if khat is not None:
            k = self._dev(khat, torch.float64, (nr, 3), "khat")
            e = self._dev(e0, torch.complex128, (nr, 3), "e0")
        rc = None
        if r0 is not None:
            r0 = [float(v) for v in r0]
            if len(r0) != 3:
                raise ValueError("r0 must have 3 components")
            rc = (ctypes.c_double * 3)(*r0)
        mom = torch.empty((nr, 24), dtype=torch.complex128, device=self.device)
        sig = torch.empty((nr, 8), dtype=torch.float64, device=self.device)
        self._check(self._call("gdm_multipoles", self.h, nr, _ptr(q), rc, _ptr(k) if k is not None else None,
                               _ptr(e) if e is not None else None, _ptr(mom), _ptr(sig)))
        return mom, sig

    def extract_dipole_pair(self, khat=None, e0=None, r_src=None, d_src=None, r0=None, tol=0.0, max_iter=-1):
        """Effective 6x6 polarisability of the structure as one dipole pair at r0
        (default: the cells' mean position) from plane waves (khat, e0) and point
        sources (r_src, d_src), by least squares over the exact dipole moments of
        the responses (gdm_extract_dipole_pair; needs factors).  Returns
        (alpha [6, 6] complex on the device, relative residual)."""
        k = e = rs = ds = None
        npw = nsrc = 0
        if khat is not None:
            k = self._dev(khat, torch.float64, None, "khat").reshape(-1, 3)
            e = self._dev(e0, torch.complex128, (len(k), 3), "e0")
            npw = len(k)
        if r_src is not None:
            rs = self._dev(r_src, torch.float64, None, "r_src").reshape(-1, 3)
            ds = self._dev(d_src, torch.complex128, (len(rs), 6), "d_src")
            nsrc = len(rs)
        rc = None if r0 is None else (ctypes.c_double * 3)(*[float(v) for v in r0])
        alpha = torch.empty((6, 6), dtype=torch.complex128, device=self.device)
        res = ctypes.c_double(0.0)
        self._check(self._call("gdm_extract_dipole_pair", self.h, npw, _ptr(k), _ptr(e), nsrc, _ptr(rs), _ptr(ds), rc,
                               float(tol), int(max_iter), _ptr(alpha), ctypes.byref(res), ctypes.byref(self.info)))
        return alpha, float(res.value)

    def dipole_sources(self, r_src, d_src):
        """Incident field [n_src, n] of point dipoles d_src [n_src, 6] = (p, m) at
        r_src [n_src, 3] on every dipole (gdm_dipole_sources)."""
        r = self._dev(r_src, torch.float64, None, "r_src").reshape(-1, 3)
        d = self._dev(d_src, torch.complex128, (len(r), 6), "d_src")
        f0 = torch.empty((len(r), self.n), dtype=torch.complex128, device=self.device)
        self._check(self._call("gdm_dipole_sources", self.h, len(r), _ptr(r), _ptr(d), _ptr(f0)))
        return f0

    def ldos(self, r_src, tol=0.0, max_iter=-1):
        """Partial electric and magnetic LDOS [n_src, 2, 3] at r_src relative to
        the host (gdm_ldos; needs factors).  After an out-of-memory error the
        points are evaluated in halves."""
        r = self._dev(r_src, torch.float64, None, "r_src").reshape(-1, 3)
        out = torch.empty((len(r), 2, 3), dtype=torch.float64, device=self.device)
        st = self._call("gdm_ldos", self.h, len(r), _ptr(r), float(tol), int(max_iter), _ptr(out),
                        ctypes.byref(self.info))
        if st == GDM_E_OOM and len(r) > 1:
            h = len(r) // 2
            return torch.cat([self.ldos(r[:h], tol, max_iter), self.ldos(r[h:], tol, max_iter)])
        self._check(st)
        return out

    def green_tensor(self, r_src, r_pts, tol=0.0, max_iter=-1):
        """Scattered 6x6 Green's tensor [n_src, n_pts, 6, 6] of the structured
        environment (gdm_green_tensor; needs factors); halves the source points
        after an out-of-memory error."""
        r = self._dev(r_src, torch.float64, None, "r_src").reshape(-1, 3)
        p = self._dev(r_pts, torch.float64, None, "r_pts").reshape(-1, 3)
        G = torch.empty((len(r), len(p), 6, 6), dtype=torch.complex128, device=self.device)
        st = self._call("gdm_green_tensor", self.h, len(r), _ptr(r), len(p), _ptr(p), float(tol), int(max_iter),
                        _ptr(G), ctypes.byref(self.info))
        if st == GDM_E_OOM and len(r) > 1:
            h = len(r) // 2
            return torch.cat([self.green_tensor(r[:h], p, tol, max_iter), self.green_tensor(r[h:], p, tol, max_iter)])
        self._check(st)
        return G

    def adjoint(self, khat, e0, f0, q, f, g_sigma=None, r_probe=None, g_e=None, tol=0.0, max_iter=-1):
        """Reverse pass (include/gdm.h, gdm_adjoint): returns (grad_r [N, 3],
        grad_eps [n_cell, 2] = d/d(Re eps, Im eps), grad_wl [1]).  g_sigma [n_rhs, 3]
        real dL/d(ext, sca, abs); g_e [n_rhs, P, 3] Wirtinger dL/dE_total."""
        k = self._dev(khat, torch.float64, None, "khat").reshape(-1, 3)
        e = self._dev(e0, torch.complex128, None, "e0").reshape(-1, 3)
        f0 = self._dev(f0, torch.complex128, None, "f0")
        q = self._dev(q, torch.complex128, None, "q")
        f = self._dev(f, torch.complex128, None, "f")
        nrhs = f0.shape[0]
        for name, t in (("khat", k), ("e0", e), ("q", q), ("f", f)):
            if t.shape[0] != nrhs:
                raise ValueError(f"{name}: expected {nrhs} rows")
        gs = self._dev(g_sigma, torch.float64, (nrhs, 3), "g_sigma")
        P = 0
        rp = ge = None
        if g_e is not None:
            rp = self._dev(r_probe, torch.float64, None, "r_probe").reshape(-1, 3)
            P = len(rp)
            ge = self._dev(g_e, torch.complex128, (nrhs, P, 3), "g_e")
        N = self.n_cell + self.n_eff
        grad_r = torch.empty((N, 3), dtype=torch.float64, device=self.device)
        grad_eps = torch.empty((max(self.n_cell, 1), 2), dtype=torch.float64, device=self.device)
        grad_wl = torch.empty(1, dtype=torch.float64, device=self.device)
        st = self._call("gdm_adjoint", self.h, nrhs, _ptr(k), _ptr(e), _ptr(f0), _ptr(q), _ptr(f), _ptr(gs), P, _ptr(rp),
                                  _ptr(ge), float(tol), int(max_iter), _ptr(grad_r), _ptr(grad_eps), _ptr(grad_wl),
                                  ctypes.byref(self.info))
        self._check(st)
        return grad_r, grad_eps[: self.n_cell], grad_wl

    def batch_spectra(self, r_cells, step, wavelengths, eps, khat, e0, prec=PREC_FP32_IR, ir_iters=-1, tol=0.0,
                      selfterm=SELF_STATIC, want_be=True):
        """Cross sections of many structures x wavelengths (include/gdm.h,
        gdm_batch_spectra).  r_cells: list of [N_s, 3] cell positions; step: one
        value or one per structure; eps [n_struct, n_wl] complex (one permittivity
        per structure and wavelength).  Returns (cs [n_struct, n_wl, n_pw, 3] =
        (ext, sca, abs), be [n_struct, n_wl] or None)."""
        import numpy as np
        counts = [len(r) for r in r_cells]
        ns = len(counts)
        off = np.zeros(ns + 1, dtype=np.int64)
        off[1:] = np.cumsum(counts)
        rc = self._dev(torch.cat([torch.as_tensor(r, dtype=torch.float64) for r in r_cells]), torch.float64,
                       (int(off[-1]), 3), "r_cells")
        steps = np.broadcast_to(np.asarray(step, dtype=np.float64), (ns,)).copy()
        wl = np.ascontiguousarray(np.asarray(wavelengths, dtype=np.float64).ravel())
        ep = self._dev(eps, torch.complex128, (ns, len(wl)), "eps")
        k = self._dev(khat, torch.float64, None, "khat").reshape(-1, 3)
        e = self._dev(e0, torch.complex128, None, "e0").reshape(-1, 3)
        if len(k) != len(e):
            raise ValueError("khat and e0 must have the same number of plane waves")
        cs = torch.empty((ns, len(wl), len(k), 3), dtype=torch.float64, device=self.device)
        be = torch.empty((ns, len(wl)), dtype=torch.float64, device=self.device) if want_be else None
        host = ctypes.c_void_p  # host arrays: cell offsets, steps, wavelengths
        st = self._call("gdm_batch_spectra", self.h, ns, host(off.ctypes.data), _ptr(rc), host(steps.ctypes.data),
                        len(wl), host(wl.ctypes.data), _ptr(ep), len(k), _ptr(k), _ptr(e), int(prec), int(ir_iters),
                        float(tol), int(selfterm), _ptr(cs), _ptr(be), ctypes.byref(self.info))
        self._check(st)
        return cs, (be if prec == PREC_FP32_IR else None)

    def batch_config(self) -> dict:
        """Measured batch configurations: {smallest n of the size class: (systems
        per group, LU panel width)}."""
        k = int(self.lib.gdm_batch_tuning(self.h, None, 0))
        buf = (ctypes.c_int32 * (3 * max(k, 1)))()
        self.lib.gdm_batch_tuning(self.h, buf, k)
        return {int(buf[3 * i]): (int(buf[3 * i + 1]), int(buf[3 * i + 2])) for i in range(k)}

    # -- dense linear algebra entry points ---------------------------------------------
    def getrf(self, A_colmajor_storage: torch.Tensor):
        """LU of the matrix whose column-major storage is the row-major tensor
        A_colmajor_storage (i.e. the matrix is A_colmajor_storage.T); in place."""
        t = A_colmajor_storage
        n = t.shape[0]
        dtype = 0 if t.dtype == torch.complex128 else 1
        ipiv = torch.empty(n, dtype=torch.int32, device=self.device)
        self.state_id += 1
        self._check(self._call("gdm_getrf", self.h, dtype, n, _ptr(t), t.shape[1], _ptr(ipiv), ctypes.byref(self.info)))
        return ipiv

    def getrs(self, A_storage: torch.Tensor, B_storage: torch.Tensor, trans: int = 0):
        """B_storage: [nrhs, n] row-major = column-major n x nrhs; solved in place."""
        dtype = 0 if A_storage.dtype == torch.complex128 else 1
        n = A_storage.shape[0]
        self._check(self._call("gdm_getrs", self.h, dtype, int(trans), n, B_storage.shape[0], _ptr(A_storage),
                                       A_storage.shape[1], _ptr(B_storage), B_storage.shape[1]))

    def gemm(self, mode, transA, m, n, k, A, lda, B, ldb, C, ldc):
        dtype = 0 if C.dtype == torch.complex128 else 1
        self._check(self._call("gdm_gemm", self.h, dtype, int(mode), int(transA), m, n, k, _ptr(A), lda, _ptr(B), ldb,
                                      _ptr(C), ldc))

    def sync(self):
        self._check(self._call("gdm_sync", self.h))

    PROF_TAGS = ("update", "panel", "assemble", "trsm", "perm", "solve", "resid", "adj_pair", "adj_probe", "fields",
                 "lookahead", "iter_matvec", "panel_l21")

    def profile(self, enable: bool, tags=None):
        """Start (clearing the counters) or stop per-launch event timing; `tags`
        (names from PROF_TAGS) restricts it to those launches."""
        if tags is None or not enable:
            self._check(self._call("gdm_profile", self.h, int(bool(enable))))
        else:
            mask = 0
            for t in tags:
                mask |= 1 << self.PROF_TAGS.index(t)
            self._check(self._call("gdm_profile_mask", self.h, mask))

    def profile_read(self) -> dict:
        nt = 3 * len(self.PROF_TAGS)
        buf = (ctypes.c_double * nt)()
        self._check(self._call("gdm_profile_read", self.h, buf, nt))
        return {t: dict(ms=buf[3 * i], work=buf[3 * i + 1], launches=int(buf[3 * i + 2]))
                for i, t in enumerate(self.PROF_TAGS)}


def plane_wave_inputs(workload: dict, ctx: "Context"):
    """Plane-wave directions and amplitudes of a workload on the context's
    device, and their intensities |E0|^2 (computed by the library)."""
    khat = torch.as_tensor(workload["khat"], dtype=torch.float64, device=ctx.device)
    e0 = torch.as_tensor(workload["e0"], dtype=torch.complex128, device=ctx.device)
    return khat, e0, ctx.planewave_intensity(e0)


def run_forward(ctx: Context, workload: dict, prec=PREC_FP64, tol=0.0, probes=True, want_ff=False):
    """Set up a workload dict (see gdm_inputs) and run the whole forward hot path:
    assembly + LU, incident field, solve, cross sections, probe fields."""
    dev = ctx.device
    r_eff = workload.get("r_eff")
    ne = 0 if r_eff is None else len(r_eff)
    ctx.set_environment(workload["n_env"])
    ctx.set_structure(torch.as_tensor(workload["r_cell"]), workload["step"], torch.as_tensor(workload["eps_cell"]),
                      torch.as_tensor(r_eff) if ne else None,
                      torch.as_tensor(workload["alpha_eff"]) if ne else None)
    ctx.factorize(workload["wavelength"], prec)
    khat, e0, e2 = plane_wave_inputs(workload, ctx)
    f0 = ctx.incident_planewave(khat, e0)
    q, f = ctx.solve(f0, tol=tol)
    out = dict(f0=f0, q=q, f=f, cs=ctx.cross_sections(f0, q, f, e2, want_ff=want_ff), info=ctx.info)
    rp = workload.get("r_probe")
    if probes and rp is not None and len(rp):
        E, H = ctx.fields(q, torch.as_tensor(rp))
        out["E_sca"], out["H_sca"] = E, H
    return out
