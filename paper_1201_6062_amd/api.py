"""Python front end of the TDSE library: plans, propagation, adjoint, autograd.

Thin marshalling over the C ABI (include/tdse.h): tensors are float64 torch
tensors on the GPU, passed by data pointer with torch's current HIP stream.
Every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _capi
from ._capi import TDSE_LANCZOS, TDSE_LENGTH, TDSE_RK4, TDSE_RKF45, TDSE_TAYLOR, TDSE_VELOCITY, TdseError, check

METHODS = {"rk4": TDSE_RK4, "taylor": TDSE_TAYLOR, "lanczos": TDSE_LANCZOS, "rkf45": TDSE_RKF45}
RKF45_SLOTS = (0.0, 0.25, 0.375, 12.0 / 13.0, 1.0, 0.5)
GAUGES = {"length": TDSE_LENGTH, "velocity": TDSE_VELOCITY}


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f64(x, device):
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.asarray(x, dtype=np.float64), device=device)
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def slots_of(method: str) -> int:
    return {"rk4": 3, "rkf45": 6}.get(method, 1)


class Plan:
    """One Hamiltonian (energies [(L+1)N], upper coupling blocks [L, N, N]) and a batch width.

    gauge="length": the blocks are the dipole D_l and field samples are E(t);
    gauge="velocity": the blocks are Q_l of the momentum coupling P = -i Q and
    field samples are the vector potential A(t)."""

    def __init__(self, energies, dipole, batch: int = 1, device="cuda", gauge: str = "length"):
        self._lib = _capi.load()
        self.device = torch.device(device)
        en = _dev_f64(energies, self.device).reshape(-1)
        dip = _dev_f64(dipole, self.device)
        if dip.dim() != 3 or dip.shape[1] != dip.shape[2]:
            raise ValueError("dipole must have shape [lmax, n, n]")
        self.lmax = int(dip.shape[0])
        self.n = int(dip.shape[1]) if self.lmax > 0 else int(en.numel())
        self.batch = int(batch)
        self.energies = en
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self._lib.tdse_create_gauge(ctypes.byref(h), _ptr(en), _ptr(dip) if self.lmax else None,
                                              GAUGES[gauge], self.lmax, self.n, self.batch, _stream(self.device)))
        self.gauge = gauge
        self._h = h

    @property
    def nstates(self) -> int:
        return (self.lmax + 1) * self.n

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tdse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _state(self, c):
        t = _dev_f64(c, self.device)
        return t.reshape(self.batch, 2 * self.nstates)

    def hmul(self, fields, u):
        """y = H(F_b) u_b for each batch column b."""
        f = _dev_f64(fields, self.device).reshape(self.batch)
        u = self._state(u)
        y = torch.empty_like(u)
        check(self._lib.tdse_hmul(self._h, _ptr(f), _ptr(u), _ptr(y), _stream(self.device)))
        return y

    def propagate(self, field, c0, dt: float, method: str = "rk4", order: int = 8,
                  ckpt_every: int = 0, out=None):
        """c(T) for field [B, nsteps, S]; returns cT (and checkpoints if ckpt_every > 0)."""
        m = METHODS[method]
        f = _dev_f64(field, self.device)
        nsteps = f.numel() // (self.batch * slots_of(method))
        f = f.reshape(self.batch, nsteps, slots_of(method)).contiguous()
        c0 = self._state(c0)
        cT = out if out is not None else torch.empty_like(c0)
        ck = None
        if ckpt_every > 0:
            ck = torch.empty(self.batch, nsteps // ckpt_every + 1, 2 * self.nstates,
                             dtype=torch.float64, device=self.device)
        check(self._lib.tdse_propagate(self._h, m, int(order), float(dt), nsteps, _ptr(f), _ptr(c0),
                                       _ptr(cT), _ptr(ck), int(max(ckpt_every, 1)) if ck is not None else 0,
                                       _stream(self.device)))
        return (cT, ck) if ckpt_every > 0 else cT

    def propagate_noalloc(self, field, c0, dt: float, method: str = "rk4", order: int = 8, ckpt=None,
                          ckpt_every: int = 0, out=None):
        """tdse_propagate_noalloc: as propagate (batch-1 plans, RK4 or Taylor),
        with the library's fixed scratch array; allocates nothing on the device
        beyond what the caller passes (out and ckpt must be given for that)."""
        m = METHODS[method]
        f = _dev_f64(field, self.device)
        nsteps = f.numel() // (self.batch * slots_of(method))
        c0 = self._state(c0)
        cT = out if out is not None else torch.empty_like(c0)
        check(self._lib.tdse_propagate_noalloc(self._h, m, int(order), float(dt), nsteps, _ptr(f), _ptr(c0),
                                               _ptr(cT), _ptr(ckpt), int(ckpt_every) if ckpt is not None else 0,
                                               _stream(self.device)))
        return cT

    def propagate_rkf45(self, field, c0, dt: float, ckpt_every: int = 0, out=None):
        """Runge-Kutta-Fehlberg 4(5) over field [B, nsteps, 6] (samples at the six
        stage times); returns (cT, err [B, nsteps]) and the checkpoints if asked."""
        f = _dev_f64(field, self.device)
        nsteps = f.numel() // (self.batch * 6)
        f = f.reshape(self.batch, nsteps, 6).contiguous()
        c0 = self._state(c0)
        cT = out if out is not None else torch.empty_like(c0)
        err = torch.empty(self.batch, nsteps, dtype=torch.float64, device=self.device)
        ck = None
        if ckpt_every > 0:
            ck = torch.empty(self.batch, nsteps // ckpt_every + 1, 2 * self.nstates,
                             dtype=torch.float64, device=self.device)
        check(self._lib.tdse_propagate_rkf45(self._h, float(dt), nsteps, _ptr(f), _ptr(c0), _ptr(cT), _ptr(err),
                                             _ptr(ck), int(max(ckpt_every, 1)) if ck is not None else 0,
                                             _stream(self.device)))
        return (cT, err, ck) if ckpt_every > 0 else (cT, err)

    def propagate_adaptive(self, field_fn, c0, t_final: float, dt0: float, tol: float,
                           dt_min: float = 1e-6, max_steps: int = 100000):
        """tdse_propagate_adaptive: Runge-Kutta-Fehlberg steps with the
        library's step-size control. field_fn(t) gives the field (or vector
        potential) at an array of times; broadcast to [B, 6] per step.
        Returns (c(t_final), accepted step sizes)."""
        c0 = self._state(c0)
        cT = torch.empty_like(c0)
        steps = np.zeros(max(int(max_steps), 1), dtype=np.float64)
        taken = ctypes.c_int64(0)
        slots = np.array(RKF45_SLOTS)
        batch = self.batch

        def fill(t, h, samples, _ctx):
            f = np.asarray(field_fn(t + slots * h), dtype=np.float64)
            np.ctypeslib.as_array(samples, shape=(batch * 6,))[:] = np.broadcast_to(f, (batch, 6)).reshape(-1)

        cb = _capi.FIELD_FN(fill)
        check(self._lib.tdse_propagate_adaptive(self._h, float(t_final), float(dt0), float(tol), float(dt_min),
                                                int(max_steps), cb, None, _ptr(c0), _ptr(cT),
                                                steps.ctypes.data_as(ctypes.c_void_p), ctypes.byref(taken),
                                                _stream(self.device)))
        return cT, list(steps[: taken.value])

    def check_stability(self, method: str, dt: float, fmax: float = 0.0, order: int = 8):
        """tdse_check_stability: (stable?, theta = dt (max|E| + |fmax| ||D||), the method's bound)."""
        th, bd = ctypes.c_double(0.0), ctypes.c_double(0.0)
        st = self._lib.tdse_check_stability(self._h, METHODS[method], int(order), float(dt), float(fmax),
                                            ctypes.byref(th), ctypes.byref(bd))
        if st not in (_capi.TDSE_OK, _capi.TDSE_E_UNSTABLE):
            check(st)
        return st == _capi.TDSE_OK, th.value, bd.value

    def adjoint(self, field, c0, dt: float, lambda_t, ckpt=None, ckpt_every: int = 64,
                method: str = "rk4", order: int = 8, want_lambda0: bool = True):
        """(grad_field [B, nsteps, 3], lambda0 [B, 2n]) for lambda_T = dL/dRe c + i dL/dIm c."""
        m = METHODS[method]
        f = _dev_f64(field, self.device)
        nsteps = f.numel() // (self.batch * slots_of(method))
        f = f.reshape(self.batch, nsteps, slots_of(method)).contiguous()
        c0 = self._state(c0)
        lam = self._state(lambda_t)
        g = torch.empty_like(f)
        l0 = torch.empty_like(c0) if want_lambda0 else None
        check(self._lib.tdse_adjoint(self._h, m, int(order), float(dt), nsteps, _ptr(f), _ptr(c0),
                                     _ptr(ckpt), int(ckpt_every), _ptr(lam), _ptr(g), _ptr(l0),
                                     _stream(self.device)))
        return g, l0


class Group:
    """Several batch-1 plans (any Lmax, N) advanced together, each with its own
    pulse and step count (RK4); every stage-round of all active instances is
    one launch over a shared work list."""

    def __init__(self, plans):
        self._lib = _capi.load()
        self.plans = list(plans)
        self.device = self.plans[0].device
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        check(self._lib.tdse_group_create(ctypes.byref(h), len(self.plans), arr, _stream(self.device)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tdse_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propagate(self, fields, c0s, dt: float):
        """fields[i]: [nsteps_i, 3] RK4 samples; c0s[i]: [2 n_i]. Returns the list of c_i(T)."""
        n = len(self.plans)
        fs = [_dev_f64(f, self.device).reshape(-1, 3).contiguous() for f in fields]
        cs = [p._state(c).reshape(-1).contiguous() for p, c in zip(self.plans, c0s)]
        outs = [torch.empty_like(c) for c in cs]
        nst = (ctypes.c_int64 * n)(*[f.shape[0] for f in fs])
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        cp = (ctypes.c_void_p * n)(*[c.data_ptr() for c in cs])
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        check(self._lib.tdse_group_propagate(self._h, TDSE_RK4, 0, float(dt), nst, fp, cp, op,
                                             _stream(self.device)))
        self._keep = (fs, cs)  # inputs stay referenced until the next call
        return outs


def tune(lmax: int, n: int, batch: int, cache_path: str):
    """Run the autotuner for one problem shape; returns the tuner's summary line."""
    lib = _capi.load()
    check(lib.tdse_tune(int(lmax), int(n), int(batch), cache_path.encode()))
    return lib.tdse_last_error().decode()


def ionization_yield(cT: torch.Tensor, energies) -> torch.Tensor:
    """Y_b = sum over states with E > 0 of |c_b,j|^2 (torch ops; autograd-friendly)."""
    en = torch.as_tensor(energies, dtype=torch.float64, device=cT.device).reshape(-1)
    mask = (en > 0).to(torch.float64)
    c = cT.reshape(cT.shape[0], -1, 2)
    return ((c * c).sum(-1) * mask).sum(-1)


class Propagate(torch.autograd.Function):
    """c(T) = RK4 or Taylor-p map of (field, c0); backward runs the library's
    discrete adjoint from the forward pass's checkpoints."""

    @staticmethod
    def forward(ctx, field, c0, plan: Plan, dt: float, ckpt_every: int = 64, method: str = "rk4",
                order: int = 8):
        cT, ck = plan.propagate(field, c0, dt, method, order=order, ckpt_every=ckpt_every)
        ctx.plan, ctx.dt, ctx.ckpt_every, ctx.method, ctx.order = plan, dt, ckpt_every, method, order
        ctx.save_for_backward(field, c0, ck)
        return cT

    @staticmethod
    def backward(ctx, grad_cT):
        field, c0, ck = ctx.saved_tensors
        plan = ctx.plan
        g, l0 = plan.adjoint(field, c0, ctx.dt, grad_cT.contiguous(), ckpt=ck, ckpt_every=ctx.ckpt_every,
                             method=ctx.method, order=ctx.order)
        return g.reshape(field.shape), l0.reshape(c0.shape), None, None, None, None, None


def piecewise_field(ek: torch.Tensor, steps_per: int, method: str = "rk4") -> torch.Tensor:
    """Per-step samples [B, K * steps_per, S] of piecewise-constant fields
    ek [B, K]: every stage sample of every step in interval k equals ek[:, k].
    Differentiable: the backward sums the per-step, per-slot gradients over
    each interval."""
    rep = torch.repeat_interleave(ek, steps_per, dim=-1)
    return rep.unsqueeze(-1).expand(*rep.shape, slots_of(method)).contiguous()


__all__ = ["Plan", "Group", "Propagate", "piecewise_field", "ionization_yield", "tune", "TdseError", "METHODS"]
