"""Python binding of the C ABI (include/ps.h): torch tensors in, device pointers out.

Tensors only provide device memory and the current HIP stream; every step of
the computation runs in the library's HIP kernels.  There is no CPU fallback:
calls raise when the library is not built or no HIP device is present.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PsInfo, check

F64 = torch.float64
PRECISIONS = {"fp64": _lib.PS_FP64, "fp32_refined": _lib.PS_FP32_REFINED, "fp32": _lib.PS_FP32}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != F64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def stream_copy(dst, src):
    """ps_stream_copy of src into dst (same number of bytes; device tensors)."""
    lib = _lib.load()
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("dst and src differ in size")
    check(lib.ps_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n, _stream()))
    return dst


class Plan:
    """One grid (nx, ny, nz, lx, ly, zf) at one precision; owns its device workspace."""

    def __init__(self, nx, ny, nz, lx, ly, zf, precision="fp64", tol=0.0, max_iter=0, flags=0):
        self._lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device")
        torch.cuda.init()
        zf = np.ascontiguousarray(np.asarray(zf, dtype=np.float64))
        if zf.shape != (nz + 1,):
            raise ValueError("zf must have nz+1 entries")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly = float(lx), float(ly)
        self.zf = zf.copy()
        self.precision = precision
        h = ctypes.c_void_p()
        check(self._lib.poisson_plan_create(ctypes.byref(h), self.nx, self.ny, self.nz, self.lx, self.ly,
                                            zf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            PRECISIONS[precision], float(tol), int(max_iter), int(flags)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.poisson_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes
    @property
    def centre_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def face_shape(self):
        return (self.nz + 1, self.ny, self.nx)

    def workspace_bytes(self):
        return int(self._lib.poisson_plan_workspace_bytes(self._h))

    def set_workspace(self, t):
        if t is None:
            check(self._lib.poisson_plan_set_workspace(self._h, None, 0))
        else:
            check(self._lib.poisson_plan_set_workspace(self._h, ctypes.c_void_p(t.data_ptr()),
                                                       t.numel() * t.element_size()))

    # ---- entry points ----
    def solve(self, f, out=None):
        out = torch.empty_like(f) if out is None else out
        info = PsInfo()
        check(self._lib.poisson_solve(self._h, _ptr(f, "f", self.centre_shape), _ptr(out, "phi", self.centre_shape),
                                      _stream(), ctypes.byref(info)))
        return out, info.as_dict()

    def solve_static(self, f, out=None):
        """poisson_solve_static: the same solve with the library's static device scratch
        instead of the plan's workspace (allocates nothing)."""
        out = torch.empty_like(f) if out is None else out
        info = PsInfo()
        check(self._lib.poisson_solve_static(self._h, _ptr(f, "f", self.centre_shape),
                                             _ptr(out, "phi", self.centre_shape), _stream(), ctypes.byref(info)))
        return out, info.as_dict()

    def solve_nosync(self, f, out):
        """poisson_solve without an info record (asynchronous for FP64)."""
        return check(self._lib.poisson_solve(self._h, _ptr(f, "f"), _ptr(out, "phi"), _stream(), None))

    def solve_adjoint(self, g_phi, out=None):
        out = torch.empty_like(g_phi) if out is None else out
        info = PsInfo()
        check(self._lib.poisson_solve_adjoint(self._h, _ptr(g_phi, "g_phi", self.centre_shape),
                                              _ptr(out, "g_rhs", self.centre_shape), _stream(), ctypes.byref(info)))
        return out, info.as_dict()

    def project(self, u, v, w, p=None, phi_out=None, s=1.0, c=0.0, want_info=True):
        info = PsInfo()
        check(self._lib.project(self._h, _ptr(u, "u", self.centre_shape), _ptr(v, "v", self.centre_shape),
                                _ptr(w, "w", self.face_shape), _ptr(p, "p", self.centre_shape),
                                _ptr(phi_out, "phi_out", self.centre_shape), float(s), float(c), _stream(),
                                ctypes.byref(info) if want_info else None))
        return info.as_dict()

    def project_adjoint(self, g_u, g_v, g_w, g_p=None, s=1.0, c=0.0):
        gu = torch.empty_like(g_u)
        gv = torch.empty_like(g_v)
        gw = torch.empty_like(g_w)
        check(self._lib.project_adjoint(self._h, _ptr(g_u, "g_u", self.centre_shape),
                                        _ptr(g_v, "g_v", self.centre_shape), _ptr(g_w, "g_w", self.face_shape),
                                        _ptr(g_p, "g_p", self.centre_shape), _ptr(gu, "gu"), _ptr(gv, "gv"),
                                        _ptr(gw, "gw"), float(s), float(c), _stream(), None))
        return gu, gv, gw

    def cn_solve(self, kind, beta, x):
        shape = self.centre_shape if kind == _lib.PS_CENTER else self.face_shape
        check(self._lib.cn_solve(self._h, int(kind), float(beta), _ptr(x, "rhs_inout", shape), _stream()))
        return x

    def cfl(self, u, v, w, out=None):
        out = torch.empty(1, dtype=F64, device=u.device) if out is None else out
        check(self._lib.ps_cfl(self._h, _ptr(u, "u", self.centre_shape), _ptr(v, "v", self.centre_shape),
                               _ptr(w, "w", self.face_shape), _ptr(out, "cfl"), _stream()))
        return out

    def substep(self, l, dt, nu, kappa, u, v, w, t, p, h_prev=None, h_out=None):
        hp = (ctypes.c_void_p * 4)(*[x.data_ptr() for x in h_prev]) if h_prev is not None else None
        ho = (ctypes.c_void_p * 4)(*[x.data_ptr() for x in h_out]) if h_out is not None else None
        info = PsInfo()
        check(self._lib.rk3_substep(self._h, int(l), float(dt), float(nu), float(kappa),
                                    _ptr(u, "u", self.centre_shape), _ptr(v, "v", self.centre_shape),
                                    _ptr(w, "w", self.face_shape), _ptr(t, "t", self.face_shape),
                                    _ptr(p, "p", self.centre_shape), hp, ho, _stream(), ctypes.byref(info)))
        return info.as_dict()

    def step(self, nu, kappa, u, v, w, t, p, dt=0.0, cfl=1.3, dt_max=float("inf")):
        """One full RK3 step (three substeps); dt <= 0 takes the Courant-limited step
        min(dt_max, cfl / Courant number).  Returns (dt taken, info)."""
        used = ctypes.c_double()
        info = PsInfo()
        check(self._lib.rk3_step(self._h, float(dt), float(cfl), float(dt_max), float(nu), float(kappa),
                                 _ptr(u, "u", self.centre_shape), _ptr(v, "v", self.centre_shape),
                                 _ptr(w, "w", self.face_shape), _ptr(t, "t", self.face_shape),
                                 _ptr(p, "p", self.centre_shape), ctypes.byref(used), _stream(),
                                 ctypes.byref(info)))
        return used.value, info.as_dict()

    def heat_flux(self, w, t, kappa):
        """(mean T on the nz + 1 faces, vertical heat flux on the nz centre planes), device tensors."""
        mean_t = torch.empty(self.nz + 1, dtype=torch.float64, device=w.device)
        flux = torch.empty(self.nz, dtype=torch.float64, device=w.device)
        check(self._lib.ps_heat_flux(self._h, _ptr(w, "w", self.face_shape), _ptr(t, "t", self.face_shape),
                                     float(kappa), _ptr(mean_t, "mean_t"), _ptr(flux, "flux"), _stream()))
        return mean_t, flux

    def substep_adjoint(self, dt, nu, kappa, u, v, w, t, p, g_out, l=1, g_hout=None, want_hprev=False):
        """VJP of substep l at the input state: g_in (five fields), and with want_hprev also the
        cotangent of the previous substep's H (four fields).  g_hout: cotangent of the
        substep's own H output (four fields) or None."""
        g_in = [torch.empty_like(x) for x in (u, v, w, t, p)]
        g_hp = [torch.empty_like(x) for x in (u, v, w, t)] if want_hprev else None
        go = (ctypes.c_void_p * 5)(*[_ptr(x, "g_out").value for x in g_out])
        gho = (ctypes.c_void_p * 4)(*[_ptr(x, "g_hout").value for x in g_hout]) if g_hout is not None else None
        gi = (ctypes.c_void_p * 5)(*[x.data_ptr() for x in g_in])
        ghp = (ctypes.c_void_p * 4)(*[x.data_ptr() for x in g_hp]) if want_hprev else None
        check(self._lib.rk3_substep_adjoint(self._h, int(l), float(dt), float(nu), float(kappa),
                                            _ptr(u, "u", self.centre_shape), _ptr(v, "v", self.centre_shape),
                                            _ptr(w, "w", self.face_shape), _ptr(t, "t", self.face_shape),
                                            _ptr(p, "p", self.centre_shape), go, gho, gi, ghp, _stream(), None))
        return (g_in, g_hp) if want_hprev else g_in

    def step_adjoint(self, dt, nu, kappa, u, v, w, t, p, g_out):
        """VJP of one full RK3 step with fixed dt at the input state (recomputed inside)."""
        g_in = [torch.empty_like(x) for x in (u, v, w, t, p)]
        go = (ctypes.c_void_p * 5)(*[_ptr(x, "g_out").value for x in g_out])
        gi = (ctypes.c_void_p * 5)(*[x.data_ptr() for x in g_in])
        check(self._lib.rk3_step_adjoint(self._h, float(dt), float(nu), float(kappa),
                                         _ptr(u, "u", self.centre_shape), _ptr(v, "v", self.centre_shape),
                                         _ptr(w, "w", self.face_shape), _ptr(t, "t", self.face_shape),
                                         _ptr(p, "p", self.centre_shape), go, gi, _stream(), None))
        return g_in

    # ---- stage access (tests, measurement) ----
    def spectral_layout(self):
        w = ctypes.c_int()
        n = ctypes.c_int()
        check(self._lib.ps_spectral_layout(self._h, ctypes.byref(w), ctypes.byref(n)))
        return w.value, n.value

    def spectral_elems(self):
        return int(self._lib.ps_spectral_elems(self._h))

    def spectral_dtype(self):
        return torch.float64 if self.precision == "fp64" else torch.float32

    def new_spectral(self):
        return torch.empty(self.spectral_elems() * 2, dtype=self.spectral_dtype(), device="cuda")

    def debug_stage(self, stage, inp, out):
        ip = ctypes.c_void_p(inp.data_ptr()) if inp is not None else None
        op = ctypes.c_void_p(out.data_ptr()) if out is not None else None
        check(self._lib.ps_debug_stage(self._h, int(stage), ip, op, _stream()))
        return out

    def spectral_to_canonical(self, buf, which):
        """View a tiled spectral buffer as complex [nz][ny][nx/2+1] (which: 'a' or 'b')."""
        w, nkxb = self.spectral_layout()
        c = torch.view_as_complex(buf.view(-1, 2))
        if which == "a":
            c = c.view(self.nz, nkxb, self.ny, w).permute(0, 2, 1, 3)
        else:
            c = c.view(nkxb, self.ny, self.nz, w).permute(2, 1, 0, 3)
        return c.reshape(self.nz, self.ny, nkxb * w)[:, :, : self.nx // 2 + 1]

    def canonical_to_spectral(self, spec, which):
        w, nkxb = self.spectral_layout()
        full = torch.zeros(self.nz, self.ny, nkxb * w, dtype=spec.dtype, device=spec.device)
        full[:, :, : self.nx // 2 + 1] = spec
        full = full.view(self.nz, self.ny, nkxb, w)
        if which == "a":
            t = full.permute(0, 2, 1, 3)
        else:
            t = full.permute(2, 1, 0, 3)
        return torch.view_as_real(t.contiguous()).reshape(-1).contiguous()


class MultiRes:
    """Temperature grid refining a plan's grid by (rx, ry, rz) (1 or 2 each), with nsub
    temperature RK3 steps per momentum step (the multiple-resolution strategy of Sec. 6)."""

    def __init__(self, plan, rx, ry, rz, nsub=1):
        self.plan = plan
        self._lib = plan._lib
        h = ctypes.c_void_p()
        check(self._lib.mr_create(ctypes.byref(h), plan._h, int(rx), int(ry), int(rz), int(nsub)))
        self._h = h
        self.rx, self.ry, self.rz, self.nsub = int(rx), int(ry), int(rz), int(nsub)
        self.nxf, self.nyf, self.nzf = plan.nx * rx, plan.ny * ry, plan.nz * rz

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def centre_shape(self):
        return (self.nzf, self.nyf, self.nxf)

    @property
    def face_shape(self):
        return (self.nzf + 1, self.nyf, self.nxf)

    def prolong_velocity(self, u, v, w, out=None):
        p = self.plan
        uf, vf, wf = out if out is not None else (
            torch.empty(self.centre_shape, dtype=F64, device=u.device),
            torch.empty(self.centre_shape, dtype=F64, device=u.device),
            torch.empty(self.face_shape, dtype=F64, device=u.device))
        check(self._lib.mr_prolong_velocity(self._h, _ptr(u, "u", p.centre_shape), _ptr(v, "v", p.centre_shape),
                                            _ptr(w, "w", p.face_shape), _ptr(uf, "uf", self.centre_shape),
                                            _ptr(vf, "vf", self.centre_shape), _ptr(wf, "wf", self.face_shape),
                                            _stream()))
        return uf, vf, wf

    def restrict_temperature(self, tf, out=None):
        tc = torch.empty(self.plan.face_shape, dtype=F64, device=tf.device) if out is None else out
        check(self._lib.mr_restrict_temperature(self._h, _ptr(tf, "tf", self.face_shape),
                                                _ptr(tc, "tc", self.plan.face_shape), _stream()))
        return tc

    def temperature_step(self, dt, kappa, vel0, vel1, tf):
        shapes = (self.centre_shape, self.centre_shape, self.face_shape)
        v0 = (ctypes.c_void_p * 3)(*[_ptr(x, "vel0", s).value for x, s in zip(vel0, shapes)])
        v1 = (ctypes.c_void_p * 3)(*[_ptr(x, "vel1", s).value for x, s in zip(vel1, shapes)])
        check(self._lib.mr_temperature_step(self._h, float(dt), float(kappa), v0, v1,
                                            _ptr(tf, "tf", self.face_shape), _stream()))
        return tf

    def step(self, nu, kappa, u, v, w, p, tf, dt=0.0, cfl=1.3, dt_max=float("inf")):
        """One coupled step (momentum on the plan's grid, temperature on this grid), in place.
        Returns (dt taken, info)."""
        pl = self.plan
        used = ctypes.c_double()
        info = PsInfo()
        check(self._lib.rk3_step_mr(self._h, float(dt), float(cfl), float(dt_max), float(nu), float(kappa),
                                    _ptr(u, "u", pl.centre_shape), _ptr(v, "v", pl.centre_shape),
                                    _ptr(w, "w", pl.face_shape), _ptr(p, "p", pl.centre_shape),
                                    _ptr(tf, "tf", self.face_shape), ctypes.byref(used), _stream(),
                                    ctypes.byref(info)))
        return used.value, info.as_dict()


class PoissonSolveFn(torch.autograd.Function):
    """phi = S f with the hand-written adjoint (transposed solve) as its backward."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        phi, _ = plan.solve(f.contiguous())
        return phi

    @staticmethod
    def backward(ctx, g):
        gf, _ = ctx.plan.solve_adjoint(g.contiguous())
        return gf, None


class ProjectFn(torch.autograd.Function):
    """(u, v, w) -> projected (u, v, w); backward = project_adjoint (no stored intermediates)."""

    @staticmethod
    def forward(ctx, u, v, w, plan, s=1.0):
        ctx.plan = plan
        ctx.s = s
        uo, vo, wo = u.clone(), v.clone(), w.clone()
        plan.project(uo, vo, wo, None, None, s, 0.0, want_info=False)
        return uo, vo, wo

    @staticmethod
    def backward(ctx, gu, gv, gw):
        a, b, c = ctx.plan.project_adjoint(gu.contiguous(), gv.contiguous(), gw.contiguous(), None, ctx.s, 0.0)
        return a, b, c, None, None


class SubstepFn(torch.autograd.Function):
    """First RK3 substep (u, v, w, T, p) -> new state with a fixed dt; backward = the
    hand-written substep adjoint, which recomputes what it needs from the saved input."""

    @staticmethod
    def forward(ctx, u, v, w, t, p, plan, dt, nu, kappa):
        ctx.plan, ctx.args = plan, (dt, nu, kappa)
        ctx.save_for_backward(u, v, w, t, p)
        out = [x.clone() for x in (u, v, w, t, p)]
        plan.substep(1, dt, nu, kappa, *out)
        return tuple(out)

    @staticmethod
    def backward(ctx, *g):
        state = ctx.saved_tensors
        g = [torch.zeros_like(x) if gi is None else gi.contiguous() for gi, x in zip(g, state)]
        g_in = ctx.plan.substep_adjoint(*ctx.args, *state, g, l=1)
        return (*g_in, None, None, None, None)


class StepFn(torch.autograd.Function):
    """One full RK3 step with a fixed dt; backward = rk3_step_adjoint (recomputes the
    intermediate substep states from the saved input)."""

    @staticmethod
    def forward(ctx, u, v, w, t, p, plan, dt, nu, kappa):
        ctx.plan, ctx.args = plan, (dt, nu, kappa)
        ctx.save_for_backward(u, v, w, t, p)
        out = [x.clone() for x in (u, v, w, t, p)]
        plan.step(nu, kappa, *out, dt=dt)
        return tuple(out)

    @staticmethod
    def backward(ctx, *g):
        state = ctx.saved_tensors
        g = [torch.zeros_like(x) if gi is None else gi.contiguous() for gi, x in zip(g, state)]
        g_in = ctx.plan.step_adjoint(*ctx.args, *state, g)
        return (*g_in, None, None, None, None)
