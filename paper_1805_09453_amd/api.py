"""Thin Python layer over libgprox (argument marshalling only).

Tensors are torch CUDA (HIP) tensors used as device buffers; the library runs
every step of the method in its own kernels on the context's stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

from . import _lib as L
from .build import LIB


def lib_path() -> str:
    return LIB


class GPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


@dataclass
class Options:
    """Step sizes and stopping rule (gp_opts).  sigma <= 0 means 1/tau; ergodic
    selects the averaged iterates (gap and outputs of the averages)."""
    tau: float
    sigma: float = 0.0
    tol: float = 1e-5
    max_iter: int = 10000
    check_every: int = 10
    norm: int = L.GP_NORM_ISO
    warm_start: bool = False
    ergodic: bool = False

    def c(self) -> L.gp_opts:
        return L.gp_opts(float(self.tau), float(self.sigma), float(self.tol), int(self.max_iter),
                         int(self.check_every), int(self.norm), int(bool(self.warm_start)), int(bool(self.ergodic)))


def _torch():
    import torch
    return torch


def _ptr(t, dtype, shape, name):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class State:
    """A device-resident iterate for pd_step / pd_gap (gp_state plus the tensors it points to)."""

    def __init__(self, kind, ny, nx, h, lam, tau, sigma, norm, f, gpsi, u, p, pbar):
        self.tensors = dict(f=f, gpsi=gpsi, u=u, p=p, pbar=pbar)
        # sigma <= 0 is passed through: the library takes sigma = 1/tau then
        self.c = L.gp_state(kind, ny, nx, norm, h, lam, tau, sigma,
                            ctypes.c_void_p(f.data_ptr()),
                            ctypes.c_void_p(gpsi.data_ptr()) if gpsi is not None else None,
                            ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                            ctypes.c_void_p(pbar.data_ptr()), 0)

    @property
    def iter(self):
        return int(self.c.iter)

    def __getattr__(self, k):
        t = self.__dict__.get("tensors", {})
        if k in t:
            return t[k]
        raise AttributeError(k)


class Context:
    """gp_ctx on a HIP stream (default: torch's current stream on the current device)."""

    def __init__(self, max_ny: int, max_nx: int, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise GPError(L.GP_EHIP, "no GPU available: libgprox has no CPU path")
        self._lib = L.load()
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.max_ny, self.max_nx = max_ny, max_nx
        h = ctypes.c_void_p()
        rc = self._lib.gp_create(ctypes.byref(h), int(max_ny), int(max_nx),
                                 ctypes.c_void_p(self.stream.cuda_stream))
        if rc != L.GP_OK:
            raise GPError(rc, self._lib.gp_strerror(rc).decode())
        self._h = h

    # -- plumbing
    def close(self):
        if getattr(self, "_h", None):
            self._lib.gp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, allow_notconv=False):
        if rc == L.GP_OK or (allow_notconv and rc == L.GP_ENOTCONV):
            return rc
        msg = self._lib.gp_last_error(self._h).decode() or self._lib.gp_strerror(rc).decode()
        raise GPError(rc, msg)

    # -- entry points
    def dct_poisson(self, b, x=None, h=1.0, alpha=0.0):
        torch = _torch()
        ny, nx = b.shape
        x = torch.empty_like(b) if x is None else x
        self._check(self._lib.dct_poisson(self._h, _ptr(b, torch.float32, (ny, nx), "b"),
                                          _ptr(x, torch.float32, (ny, nx), "x"), ny, nx, float(h), float(alpha)))
        return x

    def dct_poisson_f64(self, b, x=None, h=1.0, alpha=0.0):
        torch = _torch()
        ny, nx = b.shape
        x = torch.empty_like(b) if x is None else x
        self._check(self._lib.dct_poisson_f64(self._h, _ptr(b, torch.float64, (ny, nx), "b"),
                                              _ptr(x, torch.float64, (ny, nx), "x"), ny, nx, float(h),
                                              float(alpha)))
        return x

    def rof_solve(self, I, h, lam, opts: Options, u=None, p=None):
        torch = _torch()
        ny, nx = I.shape
        u = torch.empty_like(I) if u is None else u
        p = torch.empty((2, ny, nx), device=I.device, dtype=I.dtype) if p is None else p
        rep = L.gp_report()
        rc = self._lib.rof_solve(self._h, _ptr(I, torch.float32, (ny, nx), "I"),
                                 _ptr(u, torch.float32, (ny, nx), "u"), _ptr(p, torch.float32, (2, ny, nx), "p"),
                                 ny, nx, float(h), float(lam), ctypes.byref(opts.c()), ctypes.byref(rep))
        self._check(rc, allow_notconv=True)
        return u, p, rep.as_dict()

    def emd_solve(self, rho0, rho1, h, opts: Options, phi=None, want_phi=True):
        torch = _torch()
        ny, nx = rho0.shape
        m = torch.empty((2, ny, nx), device=rho0.device, dtype=rho0.dtype)
        if phi is None and want_phi:
            phi = torch.empty_like(rho0)
        rep = L.gp_report()
        rc = self._lib.emd_solve(self._h, _ptr(rho0, torch.float32, (ny, nx), "rho0"),
                                 _ptr(rho1, torch.float32, (ny, nx), "rho1"),
                                 _ptr(m, torch.float32, (2, ny, nx), "m"),
                                 _ptr(phi, torch.float32, (ny, nx), "phi"), ny, nx, float(h),
                                 ctypes.byref(opts.c()), ctypes.byref(rep))
        self._check(rc, allow_notconv=True)
        return m, phi, rep.as_dict()

    # -- 3-D grids
    def dct_poisson3(self, b, x=None, h=1.0, alpha=0.0):
        """(alpha I - Delta) x = b on an [nz][ny][nx] grid (FP32 or FP64 by b's dtype)."""
        torch = _torch()
        nz, ny, nx = b.shape
        x = torch.empty_like(b) if x is None else x
        fn, dt = (self._lib.dct_poisson3_f64, torch.float64) if b.dtype == torch.float64 else \
            (self._lib.dct_poisson3, torch.float32)
        self._check(fn(self._h, _ptr(b, dt, (nz, ny, nx), "b"), _ptr(x, dt, (nz, ny, nx), "x"), nz, ny, nx,
                       float(h), float(alpha)))
        return x

    def rof3_solve(self, I, h, lam, opts: Options, u=None, p=None):
        """ROF on an [nz][ny][nx] volume; returns (u, p [3][nz][ny][nx], report)."""
        torch = _torch()
        nz, ny, nx = I.shape
        u = torch.empty_like(I) if u is None else u
        p = torch.empty((3, nz, ny, nx), device=I.device, dtype=I.dtype) if p is None else p
        rep = L.gp_report()
        rc = self._lib.rof3_solve(self._h, _ptr(I, torch.float32, (nz, ny, nx), "I"),
                                  _ptr(u, torch.float32, (nz, ny, nx), "u"),
                                  _ptr(p, torch.float32, (3, nz, ny, nx), "p"), nz, ny, nx, float(h), float(lam),
                                  ctypes.byref(opts.c()), ctypes.byref(rep))
        self._check(rc, allow_notconv=True)
        return u, p, rep.as_dict()

    def emd3_solve(self, rho0, rho1, h, opts: Options, phi=None, want_phi=True):
        """EMD between [nz][ny][nx] densities; returns (flux m [3][nz][ny][nx], phi, report).
        phi: the warm-start potential when opts.warm_start (overwritten with the certificate's)."""
        torch = _torch()
        nz, ny, nx = rho0.shape
        m = torch.empty((3, nz, ny, nx), device=rho0.device, dtype=rho0.dtype)
        if phi is None and want_phi:
            phi = torch.empty_like(rho0)
        rep = L.gp_report()
        rc = self._lib.emd3_solve(self._h, _ptr(rho0, torch.float32, (nz, ny, nx), "rho0"),
                                  _ptr(rho1, torch.float32, (nz, ny, nx), "rho1"),
                                  _ptr(m, torch.float32, (3, nz, ny, nx), "m"),
                                  _ptr(phi, torch.float32, (nz, ny, nx), "phi"), nz, ny, nx, float(h),
                                  ctypes.byref(opts.c()), ctypes.byref(rep))
        self._check(rc, allow_notconv=True)
        return m, phi, rep.as_dict()

    def emd_setup(self, rho0, rho1, h):
        torch = _torch()
        ny, nx = rho0.shape
        f = torch.empty_like(rho0)
        gpsi = torch.empty((2, ny, nx), device=rho0.device, dtype=rho0.dtype)
        self._check(self._lib.emd_setup(self._h, _ptr(rho0, torch.float32, (ny, nx), "rho0"),
                                        _ptr(rho1, torch.float32, (ny, nx), "rho1"),
                                        _ptr(f, torch.float32, (ny, nx), "f"),
                                        _ptr(gpsi, torch.float32, (2, ny, nx), "gpsi"), ny, nx, float(h)))
        return f, gpsi

    def rof_step_rule(self, I, h, lam, eps, norm=L.GP_NORM_ISO):
        """Section 4.1 step rule on the device: dict with tv = ||I||_TV, grad_l2 = ||grad I||_L2,
        tv_bound (section 3.1 bound on ||u*||_TV), tau = min(tau_continuum, grad_l2) and
        tau_continuum = sqrt(lam) tv / sqrt(eps)."""
        torch = _torch()
        ny, nx = I.shape
        out = L.gp_rof_rule()
        self._check(self._lib.rof_step_rule(self._h, _ptr(I, torch.float32, (ny, nx), "I"), ny, nx, float(h),
                                            float(lam), float(eps), int(norm), ctypes.byref(out)))
        return out.as_dict()

    def make_state(self, kind, f, h, tau, sigma=0.0, lam=0.0, gpsi=None, u=None, p=None, pbar=None,
                   norm=L.GP_NORM_ISO):
        """Wrap caller tensors as a gp_state; missing u/p/pbar start at zero (pbar = p)."""
        torch = _torch()
        ny, nx = f.shape
        ushape = (ny, nx) if kind == L.GP_KIND_ROF else (2, ny, nx)
        u = torch.zeros(ushape, device=f.device, dtype=torch.float32) if u is None else u
        p = torch.zeros((2, ny, nx), device=f.device, dtype=torch.float32) if p is None else p
        pbar = p.clone() if pbar is None else pbar
        _ptr(f, torch.float32, (ny, nx), "f")
        _ptr(u, torch.float32, ushape, "u")
        _ptr(p, torch.float32, (2, ny, nx), "p")
        _ptr(pbar, torch.float32, (2, ny, nx), "pbar")
        if kind == L.GP_KIND_EMD:
            _ptr(gpsi, torch.float32, (2, ny, nx), "gpsi")
        return State(kind, ny, nx, float(h), float(lam), float(tau), float(sigma), int(norm), f, gpsi, u, p, pbar)

    def pd_step(self, st: State, n_iter: int):
        self._check(self._lib.pd_step(self._h, ctypes.byref(st.c), int(n_iter)))

    def profile(self, enable: bool):
        """Start (clear) or stop per-kernel HIP-event timing on this context's stream."""
        self._check(self._lib.gp_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{kernel: {calls, dropped, total_ms, avg_ms, bytes, gbps}} (synchronises)."""
        buf = (L.gp_kstat * 64)()
        n = ctypes.c_int()
        self._check(self._lib.gp_profile_read(self._h, buf, 64, ctypes.byref(n)))
        out = {}
        for k in buf[:min(n.value, 64)]:
            avg = k.total_ms / k.calls if k.calls else 0.0
            out[k.name.decode()] = dict(calls=k.calls, dropped=k.dropped, total_ms=k.total_ms, avg_ms=avg,
                                        bytes=k.bytes, gbps=(k.bytes / (k.total_ms * 1e6)) if k.total_ms else 0.0)
        return out

    def batch_solve(self, problems, opts: Options, outs=None):
        """Solve independent instances together (gp_batch_solve).

        problems: sequence of dicts, ROF: {"kind": GP_KIND_ROF, "I": (ny, nx) tensor, "h", "lam", "tau"};
        EMD: {"kind": GP_KIND_EMD, "rho0", "rho1": (ny, nx) tensors, "h", "tau"}.
        An EMD problem may carry "phi": an (ny, nx) tensor that receives the scaled
        certificate potential.  Returns (outs, reports, rc): outs[i] is u (ROF) or
        the flux m (EMD)."""
        torch = _torch()
        n = len(problems)
        arr = (L.gp_instance * n)()
        keep = []
        outs = [None] * n if outs is None else list(outs)
        for i, q in enumerate(problems):
            kind = int(q["kind"])
            a = q["I"] if kind == L.GP_KIND_ROF else q["rho0"]
            ny, nx = a.shape
            oshape = (ny, nx) if kind == L.GP_KIND_ROF else (2, ny, nx)
            if outs[i] is None:
                outs[i] = torch.empty(oshape, device=a.device, dtype=torch.float32)
            in0 = _ptr(a, torch.float32, (ny, nx), f"problems[{i}] input")
            in1 = _ptr(q["rho1"], torch.float32, (ny, nx), f"problems[{i}].rho1") if kind == L.GP_KIND_EMD else None
            out = _ptr(outs[i], torch.float32, oshape, f"outs[{i}]")
            phi = _ptr(q.get("phi"), torch.float32, (ny, nx), f"problems[{i}].phi") if kind == L.GP_KIND_EMD else None
            arr[i] = L.gp_instance(kind, ny, nx, float(q["h"]), float(q.get("lam", 0.0)), float(q["tau"]),
                                   in0, in1, out, phi)
            keep.append(a)
        reps = (L.gp_report * n)()
        rc = self._lib.gp_batch_solve(self._h, arr, n, ctypes.byref(opts.c()), reps)
        self._check(rc, allow_notconv=True)
        return outs, [r.as_dict() for r in reps], rc

    def get_shape(self, fp64: bool, n: int):
        """(row groups, column groups, tile width) for length-n transforms."""
        r, c, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.gp_get_shape(self._h, int(bool(fp64)), int(n), ctypes.byref(r), ctypes.byref(c),
                                           ctypes.byref(w)))
        return r.value, c.value, w.value

    def set_shape(self, fp64: bool, n: int, row_groups: int = 0, col_groups: int = 0, tile_width: int = 0):
        self._check(self._lib.gp_set_shape(self._h, int(bool(fp64)), int(n), int(row_groups), int(col_groups),
                                           int(tile_width)))

    def get_radix_plan(self, fp64: bool, n: int):
        """Radices of the Stockham passes of length-n transforms (n 7-smooth, not a power of two)."""
        r = (ctypes.c_int * 16)()
        k = ctypes.c_int()
        self._check(self._lib.gp_get_radix_plan(self._h, int(bool(fp64)), int(n), r, ctypes.byref(k)))
        return [r[i] for i in range(k.value)]

    def set_radix_plan(self, fp64: bool, n: int, radices):
        r = (ctypes.c_int * 16)(*[int(x) for x in radices][:16])
        self._check(self._lib.gp_set_radix_plan(self._h, int(bool(fp64)), int(n), r, len(radices)))

    def pd_gap(self, st: State):
        rep = L.gp_report()
        self._check(self._lib.pd_gap(self._h, ctypes.byref(st.c), ctypes.byref(rep)))
        return rep.as_dict()


class WarmStart:
    """The learned warm-start network (ws_net) on a Context's stream."""

    def __init__(self, ctx: Context, max_batch: int, ny: int, nx: int):
        self.ctx, self.max_batch, self.ny, self.nx = ctx, max_batch, ny, nx
        lib = ctx._lib
        h = ctypes.c_void_p()
        ctx._check(lib.ws_create(ctx._h, ctypes.byref(h), int(max_batch), int(ny), int(nx)))
        self._h = h
        self.n_params = int(lib.ws_param_count())

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, blob):
        torch = _torch()
        self.ctx._check(self.ctx._lib.ws_set_params(self.ctx._h, self._h,
                                                    _ptr(blob, torch.float32, (self.n_params,), "blob")))

    def get_params(self):
        torch = _torch()
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self.ctx._check(self.ctx._lib.ws_get_params(self.ctx._h, self._h, _ptr(out, torch.float32, out.shape, "out")))
        return out

    def predict(self, rho0, rho1):
        """rho0, rho1: (B, ny, nx) at the native size -> phi0 (B, ny, nx)."""
        torch = _torch()
        B = rho0.shape[0]
        shp = (B, self.ny, self.nx)
        phi = torch.empty(shp, dtype=torch.float32, device=rho0.device)
        self.ctx._check(self.ctx._lib.ws_predict(self.ctx._h, self._h, _ptr(rho0, torch.float32, shp, "rho0"),
                                                 _ptr(rho1, torch.float32, shp, "rho1"), int(B),
                                                 _ptr(phi, torch.float32, shp, "phi")))
        return phi

    def grads(self, rho0, rho1, phi_star, h, want_grad=False):
        """Loss (float) and, if asked, the FP32 gradient blob."""
        torch = _torch()
        B = rho0.shape[0]
        shp = (B, self.ny, self.nx)
        g = torch.empty(self.n_params, dtype=torch.float32, device=rho0.device) if want_grad else None
        loss = ctypes.c_double()
        self.ctx._check(self.ctx._lib.ws_grads(self.ctx._h, self._h, _ptr(rho0, torch.float32, shp, "rho0"),
                                               _ptr(rho1, torch.float32, shp, "rho1"),
                                               _ptr(phi_star, torch.float32, shp, "phi_star"), int(B), float(h),
                                               _ptr(g, torch.float32, (self.n_params,), "grad"),
                                               ctypes.byref(loss)))
        return (loss.value, g) if want_grad else loss.value

    def adam(self, lr):
        self.ctx._check(self.ctx._lib.ws_adam(self.ctx._h, self._h, float(lr)))

    def train_step(self, rho0, rho1, phi_star, h, lr):
        """grads then adam in one call; returns the batch's loss before the step."""
        torch = _torch()
        B = rho0.shape[0]
        shp = (B, self.ny, self.nx)
        loss = ctypes.c_double()
        self.ctx._check(self.ctx._lib.ws_train_step(self.ctx._h, self._h, _ptr(rho0, torch.float32, shp, "rho0"),
                                                    _ptr(rho1, torch.float32, shp, "rho1"),
                                                    _ptr(phi_star, torch.float32, shp, "phi_star"), int(B), float(h),
                                                    float(lr), ctypes.byref(loss)))
        return loss.value

    def load_params(self, path):
        """Parameters from a raw FP32 file (resets the Adam state)."""
        self.ctx._check(self.ctx._lib.ws_load_params(self.ctx._h, self._h, os.fsencode(path)))

    def save_params(self, path):
        self.ctx._check(self.ctx._lib.ws_save_params(self.ctx._h, self._h, os.fsencode(path)))

    def emd_solve(self, rho0, rho1, h, opts: Options, want_phi=False):
        """emd_solve from the learned start (with fallback); returns (m, phi, report, ws_report)."""
        torch = _torch()
        ny, nx = rho0.shape
        m = torch.empty((2, ny, nx), device=rho0.device, dtype=torch.float32)
        phi = torch.empty_like(rho0) if want_phi else None
        rep, wrep = L.gp_report(), L.ws_report()
        rc = self.ctx._lib.ws_emd_solve(self.ctx._h, self._h, _ptr(rho0, torch.float32, (ny, nx), "rho0"),
                                        _ptr(rho1, torch.float32, (ny, nx), "rho1"),
                                        _ptr(m, torch.float32, (2, ny, nx), "m"),
                                        _ptr(phi, torch.float32, (ny, nx), "phi"), ny, nx, float(h),
                                        ctypes.byref(opts.c()), ctypes.byref(rep), ctypes.byref(wrep))
        self.ctx._check(rc, allow_notconv=True)
        return m, phi, rep.as_dict(), wrep.as_dict()


def dct_poisson_noalloc(b, x=None, h=1.0, alpha=0.0, stream=None):
    """(alpha I - Delta) x = b without a context and without device allocation in
    the library (its workspace is a fixed device array; ny * nx <= 2^20).  x may
    be b (in place) or a caller tensor; a new tensor is allocated here only when
    x is None.  Enqueued on `stream` (default: torch's current stream)."""
    torch = _torch()
    lib = L.load()
    ny, nx = b.shape
    if x is None:
        x = torch.empty_like(b)
    st = torch.cuda.current_stream() if stream is None else stream
    rc = lib.dct_poisson_noalloc(_ptr(b, torch.float32, (ny, nx), "b"), _ptr(x, torch.float32, (ny, nx), "x"), ny,
                                 nx, float(h), float(alpha), ctypes.c_void_p(st.cuda_stream))
    if rc != L.GP_OK:
        raise GPError(rc, f"{lib.gp_strerror(rc).decode()}: {lib.gp_last_error(None).decode()}")
    return x


def emd_step_rule_singular(eps: float, m: float) -> float:
    """Section 4.2 step rule for singular measures, computed by the library:
    min(sqrt(1 / (eps |ln eps|)), 2 m^(1/4)) for a grid of side m."""
    t = L.load().emd_step_rule_singular(float(eps), float(m))
    if t < 0:
        raise ValueError("emd_step_rule_singular needs 0 < eps < 1 and m > 0")
    return t


def ws_downsample(ctx: Context, x, f: int):
    torch = _torch()
    ny, nx = x.shape
    out = torch.empty((ny // f, nx // f), dtype=torch.float32, device=x.device)
    ctx._check(ctx._lib.ws_downsample(ctx._h, _ptr(x, torch.float32, (ny, nx), "x"), ny, nx, int(f),
                                      _ptr(out, torch.float32, out.shape, "out")))
    return out


def ws_upsample(ctx: Context, x, f: int):
    torch = _torch()
    ny, nx = x.shape
    out = torch.empty((ny * f, nx * f), dtype=torch.float32, device=x.device)
    ctx._check(ctx._lib.ws_upsample(ctx._h, _ptr(x, torch.float32, (ny, nx), "x"), ny, nx, int(f),
                                    _ptr(out, torch.float32, out.shape, "out")))
    return out
