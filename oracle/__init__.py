"""ctypes front end of the plain FP64 CPU oracle (tdse_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product library never does.
Each function propagates pulses one at a time, single-threaded, in the loop
order of the C source. Arrays follow the library's layout: complex vectors
interleaved (re, im), field samples [B, nsteps, S].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdse_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile tdse_oracle.c with gcc into liboracle.so (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        i32, i64, d = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        lib.oracle_dmul.argtypes = [i32, i32, P, P, P]
        lib.oracle_dmul.restype = None
        lib.oracle_hmul.argtypes = [i32, i32, P, P, d, P, P]
        lib.oracle_hmul.restype = None
        lib.oracle_rk4.argtypes = [i32, i32, P, P, d, i64, P, P]
        lib.oracle_rk4.restype = i32
        lib.oracle_taylor.argtypes = [i32, i32, P, P, i32, d, i64, P, P]
        lib.oracle_taylor.restype = i32
        lib.oracle_rk4_tangent.argtypes = [i32, i32, P, P, d, i64, P, P, P, P]
        lib.oracle_rk4_tangent.restype = i32
        lib.oracle_rk4_adjoint.argtypes = [i32, i32, P, P, d, i64, P, P, P, P]
        lib.oracle_rk4_adjoint.restype = i32
        lib.oracle_taylor_adjoint.argtypes = [i32, i32, P, P, i32, d, i64, P, P, P, P]
        lib.oracle_taylor_adjoint.restype = i32
        lib.oracle_rkf45.argtypes = [i32, i32, P, P, d, i64, P, P, P]
        lib.oracle_rkf45.restype = i32
        lib.oracle_set_gauge.argtypes = [i32]
        lib.oracle_set_gauge.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


GAUGES = {"length": 0, "velocity": 1}


class _gauge:
    """Select the coupling gauge of the C oracle for one call (length by default)."""

    def __init__(self, gauge):
        self.code = GAUGES[gauge]

    def __enter__(self):
        _load().oracle_set_gauge(self.code)

    def __exit__(self, *exc):
        _load().oracle_set_gauge(0)
        return False


def _dims_n(energies, dipole, n=None):
    en = _f64(energies)
    dip = _f64(dipole)
    lmax = dip.shape[0]
    n = dip.shape[1] if n is None else n
    if en.size != (lmax + 1) * n:
        raise ValueError("energies size does not match (lmax+1)*n")
    return en, dip, lmax, n


def dmul(energies, dipole, u, n=None, gauge="length"):
    """z = D u for one interleaved complex vector u."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        u = _f64(u)
        z = np.empty_like(u)
        _load().oracle_dmul(lmax, n, _p(dip), _p(u), _p(z))
        return z


def hmul(energies, dipole, field, u, n=None, gauge="length"):
    """y = H(field) u = E o u + field * D u."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        u = _f64(u)
        y = np.empty_like(u)
        _load().oracle_hmul(lmax, n, _p(en), _p(dip), float(field), _p(u), _p(y))
        return y


def rk4(energies, dipole, dt, field, c0, n=None, gauge="length"):
    """RK4 over field[B, nsteps, 3] from c0[B, 2n]; returns c(T) [B, 2n]."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        field = _f64(field)
        c = np.array(c0, dtype=np.float64, copy=True, order="C")
        if field.ndim == 2:
            field = field[None]
        if c.ndim == 1:
            c = c[None]
        assert field.shape[-1] == 3 and field.shape[0] == c.shape[0]
        lib = _load()
        for b in range(c.shape[0]):
            fb = _f64(field[b])
            cb = np.ascontiguousarray(c[b])
            rc = lib.oracle_rk4(lmax, n, _p(en), _p(dip), float(dt), fb.shape[0], _p(fb), _p(cb))
            if rc != 0:
                raise MemoryError("oracle_rk4 allocation failed")
            c[b] = cb
        return c


def taylor(energies, dipole, order, dt, field, c0, n=None, gauge="length"):
    """Taylor-order propagation over field[B, nsteps, 1] (or [B, nsteps])."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        field = _f64(field)
        c = np.array(c0, dtype=np.float64, copy=True, order="C")
        if c.ndim == 1:
            c = c[None]
        if field.ndim == 1:
            field = field[None]
        if field.ndim == 3:
            field = field[..., 0]
        lib = _load()
        for b in range(c.shape[0]):
            fb = _f64(field[b])
            cb = np.ascontiguousarray(c[b])
            rc = lib.oracle_taylor(lmax, n, _p(en), _p(dip), int(order), float(dt), fb.shape[0],
                                   _p(fb), _p(cb))
            if rc != 0:
                raise MemoryError("oracle_taylor allocation failed")
            c[b] = cb
        return c


def rk4_tangent(energies, dipole, dt, field, dfield, c0, dc0=None, n=None, gauge="length"):
    """Returns (c(T), dc(T)) for one pulse: field, dfield [nsteps, 3]."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        field, dfield = _f64(field), _f64(dfield)
        c = np.array(c0, dtype=np.float64, copy=True).reshape(-1)
        dc = np.zeros_like(c) if dc0 is None else np.array(dc0, dtype=np.float64, copy=True).reshape(-1)
        rc = _load().oracle_rk4_tangent(lmax, n, _p(en), _p(dip), float(dt), field.shape[0],
                                        _p(field), _p(dfield), _p(c), _p(dc))
        if rc != 0:
            raise MemoryError("oracle_rk4_tangent allocation failed")
        return c, dc


def rk4_adjoint(energies, dipole, dt, field, c0, lam_t, n=None, gauge="length"):
    """Discrete RK4 adjoint for one pulse. Returns (lambda_0, grad[nsteps, 3])."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        field = _f64(field)
        c0 = _f64(np.asarray(c0).reshape(-1))
        lam = np.array(lam_t, dtype=np.float64, copy=True).reshape(-1)
        grad = np.zeros_like(field)
        rc = _load().oracle_rk4_adjoint(lmax, n, _p(en), _p(dip), float(dt), field.shape[0],
                                        _p(field), _p(c0), _p(lam), _p(grad))
        if rc != 0:
            raise MemoryError("oracle_rk4_adjoint allocation failed")
        return lam, grad


def taylor_adjoint(energies, dipole, order, dt, field, c0, lam_t, n=None, gauge="length"):
    """Discrete Taylor-p adjoint for one pulse (field [nsteps] or [nsteps, 1]).
    Returns (lambda_0, grad[nsteps])."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        field = _f64(np.asarray(field).reshape(-1))
        c0 = _f64(np.asarray(c0).reshape(-1))
        lam = np.array(lam_t, dtype=np.float64, copy=True).reshape(-1)
        grad = np.zeros_like(field)
        rc = _load().oracle_taylor_adjoint(lmax, n, _p(en), _p(dip), int(order), float(dt), field.shape[0],
                                           _p(field), _p(c0), _p(lam), _p(grad))
        if rc != 0:
            raise MemoryError("oracle_taylor_adjoint allocation failed")
        return lam, grad


def rkf45(energies, dipole, dt, field, c0, n=None, gauge="length"):
    """Runge-Kutta-Fehlberg 4(5) over field[B, nsteps, 6]; returns (c(T) [B, 2n],
    err [B, nsteps]) with c advanced by the fifth-order weights (the solution
    the paper propagates, Sec. 5.1) and err the embedded estimate."""
    with _gauge(gauge):
        en, dip, lmax, n = _dims_n(energies, dipole, n)
        field = _f64(field)
        if field.ndim == 2:
            field = field[None]
        c = np.array(c0, dtype=np.float64, copy=True, order="C")
        if c.ndim == 1:
            c = c[None]
        assert field.shape[-1] == 6 and field.shape[0] == c.shape[0]
        err = np.zeros(field.shape[:2])
        lib = _load()
        for b in range(c.shape[0]):
            fb = _f64(field[b])
            cb = np.ascontiguousarray(c[b])
            eb = np.zeros(fb.shape[0])
            rc = lib.oracle_rkf45(lmax, n, _p(en), _p(dip), float(dt), fb.shape[0], _p(fb), _p(cb), _p(eb))
            if rc != 0:
                raise MemoryError("oracle_rkf45 allocation failed")
            c[b] = cb
            err[b] = eb
        return c, err


def positive_mask(energies):
    """Indicator of continuum (E > 0) states, the ionization-yield support."""
    return np.asarray(energies) > 0.0


def ionization_yield(energies, c):
    """Y = sum over E_j > 0 of |c_j|^2, per pulse."""
    c = np.atleast_2d(c)
    m = positive_mask(energies)
    re, im = c[:, 0::2], c[:, 1::2]
    return ((re * re + im * im) * m[None, :]).sum(axis=1)


def yield_seed(energies, c):
    """lambda_T = dY/dRe c + i dY/dIm c = 2 [E > 0] c."""
    m = np.repeat(positive_mask(energies), 2).astype(np.float64)
    return 2.0 * np.atleast_2d(c) * m[None, :]


# ---- short-iterative Lanczos propagator (Krylov; named in Sec. 5.2 as the
# propagator to build on an optimised product)

LANCZOS_BREAKDOWN = 1e-13


def _as_complex(v):
    v = np.asarray(v, dtype=np.float64)
    return v[0::2] + 1j * v[1::2]


def _as_interleaved(z):
    out = np.empty(2 * z.size)
    out[0::2] = z.real
    out[1::2] = z.imag
    return out


def lanczos(energies, dipole, m, dt, field, c0, n=None, gauge="length"):
    """Krylov propagation: with H frozen over step k at the sample field[b, k],
    build the Lanczos basis v_1 = c / |c|, v_{j+1} beta_j = H v_j - alpha_j v_j
    - beta_{j-1} v_{j-1} (alpha_j = <v_j, H v_j>, beta_j = |...|; plain
    three-term recurrence, no reorthogonalisation) for j = 1..m, and set
    c' = |c| V exp(-i dt T) e_1 with T the m x m tridiagonal of the alphas and
    betas, exponentiated through its eigendecomposition. The basis ends early
    (breakdown) once beta_j <= 1e-13 (|alpha_j| + beta_{j-1}).
    field [B, nsteps] or [B, nsteps, 1]; c0 [B, 2n]; returns c(T) [B, 2n]."""
    en, dip, lmax, n = _dims_n(energies, dipole, n)
    c = np.array(c0, dtype=np.float64, copy=True)
    if c.ndim == 1:
        c = c[None]
    f = np.asarray(field, dtype=np.float64)
    if f.ndim == 3:
        f = f[..., 0]
    if f.ndim == 1:
        f = f[None]
    for b in range(c.shape[0]):
        for k in range(f.shape[1]):
            z = _as_complex(c[b])
            beta0 = np.linalg.norm(z)
            if beta0 == 0.0:
                continue
            vs, alphas, betas = [z / beta0], [], []
            for j in range(m):
                w = _as_complex(hmul(en, dip, f[b, k], _as_interleaved(vs[j]), n=n, gauge=gauge))
                a = float(np.real(np.vdot(vs[j], w)))
                w = w - a * vs[j]
                if j > 0:
                    w = w - betas[j - 1] * vs[j - 1]
                alphas.append(a)
                if j == m - 1:
                    break
                bj = float(np.linalg.norm(w))
                if bj <= LANCZOS_BREAKDOWN * (abs(a) + (betas[j - 1] if j > 0 else 0.0)):
                    break
                betas.append(bj)
                vs.append(w / bj)
            kdim = len(alphas)
            t = np.diag(alphas) + np.diag(betas[:kdim - 1], 1) + np.diag(betas[:kdim - 1], -1)
            lam, q = np.linalg.eigh(t)
            y = q @ (np.exp(-1j * dt * lam) * q[0, :])
            c[b] = _as_interleaved(beta0 * sum(y[j] * vs[j] for j in range(kdim)))
    return c
