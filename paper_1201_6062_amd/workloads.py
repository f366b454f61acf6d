"""Seeded synthetic inputs: hydrogen-like Hamiltonians, laser pulses, field samples.

This module only draws and lays out inputs. It performs none of the
propagation arithmetic, so the CPU oracle and the HIP path can both take their
inputs from it without sharing any of the method's code.

Stand-in for the paper's B-spline hydrogen eigenbasis (Sec. 5: 640 explicit
states per partial wave, energies and dipole matrix elements from an external
basis code, not available here):

* energies, per partial wave l: 10 bound levels -1/(2 m^2), m = l+1 .. l+10,
  then a box continuum (pi j / R)^2 / 2, j = 1 .. N-10, R = 200 a.u.;
* dipole block D_l couples l to l+1 (rows: states of l, columns: states of
  l+1); D_l[a, b] = g (l+1) / sqrt((2l+1)(2l+3)) / (1 + |E_l[a] - E_{l+1}[b]|)
  with g ~ N(0, 1) from numpy's default_rng(seed), blocks drawn in order
  l = 0 .. Lmax-1. The l+1 -> l block is D_l transposed, so the full matrix is
  real symmetric (Sec. 3, dipole selection rules; Sec. 5, only the
  superdiagonal blocks are stored).

Pulses follow Sec. 5's sin^2 envelope with a cosine carrier:
E(t) = E0 sin^2(pi t / Tp) cos(w t) for 0 <= t <= Tp, Tp = 2 pi ncyc / w, and
E = 0 outside [0, Tp].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

BOX_RADIUS = 200.0
N_BOUND = 10


def energies(lmax: int, n: int) -> np.ndarray:
    """Field-free energies, shape [(lmax+1)*n], block l at [l*n:(l+1)*n]."""
    out = np.empty((lmax + 1, n), dtype=np.float64)
    for l in range(lmax + 1):
        bound = [-1.0 / (2.0 * m * m) for m in range(l + 1, l + 1 + N_BOUND)]
        cont = [0.5 * (math.pi * j / BOX_RADIUS) ** 2 for j in range(1, max(n - N_BOUND, 0) + 1)]
        out[l] = np.array(bound + cont, dtype=np.float64)[:n]
    return out.reshape(-1)


def dipole(lmax: int, n: int, seed: int, en: np.ndarray | None = None) -> np.ndarray:
    """Upper dipole blocks D_l = D_{l,l+1}, shape [lmax, n, n], row-major."""
    if en is None:
        en = energies(lmax, n)
    e = en.reshape(lmax + 1, n)
    rng = np.random.default_rng(seed)
    out = np.empty((lmax, n, n), dtype=np.float64)
    for l in range(lmax):
        g = rng.standard_normal((n, n))
        ang = (l + 1) / math.sqrt((2 * l + 1) * (2 * l + 3))
        out[l] = g * ang / (1.0 + np.abs(e[l][:, None] - e[l + 1][None, :]))
    return out


def ground_state(lmax: int, n: int, batch: int = 1) -> np.ndarray:
    """c0 = e_0 (lowest bound level of l=0), interleaved complex, [batch, 2*(lmax+1)*n]."""
    c = np.zeros((batch, 2 * (lmax + 1) * n), dtype=np.float64)
    c[:, 0] = 1.0
    return c


def sizing_doubles(n_l: int, n_blocks: int) -> int:
    """Doubles in the paper's packed Hamiltonian: (N_l + N_l^2) per partial wave (Sec. 5)."""
    return (n_l + n_l * n_l) * n_blocks


@dataclass(frozen=True)
class Pulse:
    e0: float
    omega: float
    ncyc: float

    @property
    def duration(self) -> float:
        return 2.0 * math.pi * self.ncyc / self.omega

    def __call__(self, t):
        t = np.asarray(t, dtype=np.float64)
        tp = self.duration
        inside = (t >= 0.0) & (t <= tp)
        val = self.e0 * np.sin(math.pi * t / tp) ** 2 * np.cos(self.omega * t)
        return np.where(inside, val, 0.0)


def nsteps_for(t_final: float, dt: float) -> int:
    """Whole steps covering [0, t_final]: ceil(T/dt) with dt kept (field is 0 past the pulse)."""
    return int(math.ceil(t_final / dt - 1e-9))


RK4_SLOTS = (0.0, 0.5, 1.0)
RKF45_SLOTS = (0.0, 0.25, 0.375, 12.0 / 13.0, 1.0, 0.5)   # Fehlberg stage times / dt


def rk4_samples(pulse, dt: float, nsteps: int) -> np.ndarray:
    """RK4 stage samples per step: E(t_k), E(t_k + dt/2), E(t_k + dt); shape [nsteps, 3]."""
    k = np.arange(nsteps, dtype=np.float64)[:, None]
    t = (k + np.array(RK4_SLOTS)[None, :]) * dt
    return np.ascontiguousarray(pulse(t))


def rkf45_samples(pulse, dt: float, nsteps: int) -> np.ndarray:
    """Runge-Kutta-Fehlberg stage samples per step, E(t_k + c_i dt); shape [nsteps, 6]."""
    k = np.arange(nsteps, dtype=np.float64)[:, None]
    t = (k + np.array(RKF45_SLOTS)[None, :]) * dt
    return np.ascontiguousarray(pulse(t))


def taylor_samples(pulse, dt: float, nsteps: int, where: str = "left") -> np.ndarray:
    """One sample per Taylor step, H frozen at the step's left end (appendix B) or its midpoint."""
    off = {"left": 0.0, "mid": 0.5}[where]
    t = (np.arange(nsteps, dtype=np.float64) + off) * dt
    return np.ascontiguousarray(pulse(t)[:, None])


def random_pulses(rng: np.random.Generator, count: int, ncyc: float = 10.0):
    """E0 log-uniform in [0.01, 0.1], omega uniform in [0.2, 1.0]."""
    out = []
    for _ in range(count):
        e0 = 10.0 ** rng.uniform(-2.0, -1.0)
        w = rng.uniform(0.2, 1.0)
        out.append(Pulse(e0, w, ncyc))
    return out


# --------------------------------------------------------------------------
# The five workloads.


# ---- velocity gauge (Sec. 5): the coupling is -p.A(t)/c with A = -int E dt

# 5-point Gauss-Legendre nodes and weights on [-1, 1]
_GL5_X = np.array([-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831, 0.9061798459386640])
_GL5_W = np.array([0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665,
                   0.2369268850561891])


def _gl5(pulse, a, b):
    """int_a^b E(t) dt by 5-point Gauss-Legendre quadrature (elementwise over a, b)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    mid, half = 0.5 * (a + b), 0.5 * (b - a)
    t = mid[..., None] + half[..., None] * _GL5_X
    return half * (pulse(t) * _GL5_W).sum(axis=-1)


def vector_potential_exact(pulse, t):
    """A(t) = -int_0^t E, closed form for the sin^2 cos pulse (constant after the pulse)."""
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, pulse.duration)
    w, big = pulse.omega, 2.0 * math.pi / pulse.duration
    val = (np.sin(w * t) / w - np.sin((w + big) * t) / (2.0 * (w + big))
           - np.sin((w - big) * t) / (2.0 * (w - big)))
    return -0.5 * pulse.e0 * val


def vector_potential_samples(pulse, dt: float, nsteps: int, method: str = "rk4", where: str = "left"):
    """A(t) at the stage times of each step, accumulated step by step with
    5-point Gauss-Legendre quadrature of E (the paper's velocity-gauge
    procedure). RK4: [nsteps, 3] at t_k, t_k + dt/2, t_k + dt; Taylor:
    [nsteps, 1] at the step's left end or midpoint."""
    k = np.arange(nsteps, dtype=np.float64)
    t0 = k * dt
    a_start = -np.concatenate([[0.0], np.cumsum(_gl5(pulse, t0, t0 + dt))])[:nsteps]
    if method == "rk4":
        a_mid = a_start - _gl5(pulse, t0, t0 + 0.5 * dt)
        a_end = a_start - _gl5(pulse, t0, t0 + dt)
        return np.ascontiguousarray(np.stack([a_start, a_mid, a_end], axis=1))
    if where == "mid":
        return np.ascontiguousarray((a_start - _gl5(pulse, t0, t0 + 0.5 * dt))[:, None])
    return np.ascontiguousarray(a_start[:, None])


def velocity_coupling(energies: np.ndarray, dipole: np.ndarray) -> np.ndarray:
    """Blocks Q_l of the momentum coupling P = -i Q that matches the dipole:
    P = i [H0, D] in this basis, i.e. P_{l,l+1}[a, b] = i (E_l[a] - E_{l+1}[b]) D_l[a, b],
    so Q_l[a, b] = (E_{l+1}[b] - E_l[a]) D_l[a, b] (real; P is Hermitian)."""
    lmax, n = dipole.shape[0], dipole.shape[1]
    e = np.asarray(energies).reshape(lmax + 1, n)
    return np.ascontiguousarray((e[1:, None, :] - e[:-1, :, None]) * dipole)


@dataclass
class Hamiltonian:
    lmax: int
    n: int
    seed: int
    energies: np.ndarray = dc_field(repr=False)
    dipole: np.ndarray = dc_field(repr=False)

    @property
    def nstates(self) -> int:
        return (self.lmax + 1) * self.n


def hamiltonian(lmax: int, n: int, seed: int) -> Hamiltonian:
    en = energies(lmax, n)
    return Hamiltonian(lmax, n, seed, en, dipole(lmax, n, seed, en))


@dataclass
class Workload:
    name: str
    ham: Hamiltonian
    method: str           # "rk4" | "taylor"
    order: int            # Taylor order (0 for RK4)
    dt: float
    nsteps: int
    field: np.ndarray     # [B, nsteps, S]
    c0: np.ndarray        # [B, 2n]
    pulses: list

    @property
    def batch(self) -> int:
        return self.field.shape[0]


def _single(name, lmax, n, seed, pulse, method, dt, order=0, where="left"):
    ham = hamiltonian(lmax, n, seed)
    nst = nsteps_for(pulse.duration, dt)
    if method == "rk4":
        f = rk4_samples(pulse, dt, nst)
    else:
        f = taylor_samples(pulse, dt, nst, where)
    return Workload(name, ham, method, order, dt, nst, f[None], ground_state(lmax, n), [pulse])


def single_small(method: str = "rk4") -> Workload:
    """Lmax=3, N=50, E0=0.05, w=0.5, 10 cycles, dt=0.01, RK4 (12567 steps)."""
    return _single("single_small_L3_N50", 3, 50, 0, Pulse(0.05, 0.5, 10.0), "rk4", 0.01)


def single_large(method: str = "rk4", order: int = 8, where: str = "left") -> Workload:
    """Lmax=15, N=500, E0=0.05, w=0.5, 20 cycles; RK4 dt=0.005, Taylor-8 dt=0.02."""
    p = Pulse(0.05, 0.5, 20.0)
    if method == "rk4":
        return _single("single_L15_N500_rk4", 15, 500, 0, p, "rk4", 0.005)
    return _single(f"single_L15_N500_taylor{order}", 15, 500, 0, p, "taylor", 0.02, order, where)


def batched(count: int = 256, dt: float = 0.005) -> Workload:
    """count pulses sharing the Lmax=15, N=500 Hamiltonian, padded to a common T."""
    ham = hamiltonian(15, 500, 0)
    pulses = random_pulses(np.random.default_rng(1), count)
    t_final = max(p.duration for p in pulses)
    nst = nsteps_for(t_final, dt)
    f = np.stack([rk4_samples(p, dt, nst) for p in pulses])
    return Workload(f"batched_L15_N500_B{count}", ham, "rk4", 0, dt, nst, f,
                    ground_state(15, 500, count), pulses)


@dataclass
class UnevenInstance:
    lmax: int
    n: int
    seed: int
    pulse: Pulse
    nsteps: int


def uneven_specs(count: int = 64, dt: float = 0.005):
    """count instances, Lmax ~ U{7..31}, N ~ U{200..1000}, own H seed and pulse."""
    rng = np.random.default_rng(2)
    out = []
    for i in range(count):
        lmax = int(rng.integers(7, 32))
        n = int(rng.integers(200, 1001))
        e0 = 10.0 ** rng.uniform(-2.0, -1.0)
        w = rng.uniform(0.2, 1.0)
        p = Pulse(e0, w, 10.0)
        out.append(UnevenInstance(lmax, n, 1000 + i, p, nsteps_for(p.duration, dt)))
    return out


ADJ_INTERVALS = 2048
ADJ_STEPS_PER_INTERVAL = 16


def adjoint_pulses(count: int = 32):
    return random_pulses(np.random.default_rng(3), count)


def piecewise_samples(pulse, n_intervals: int = ADJ_INTERVALS, dt: float = 0.01,
                      steps_per: int = ADJ_STEPS_PER_INTERVAL) -> np.ndarray:
    """Piecewise-constant field: E_k = E(midpoint of interval k), interval = steps_per steps."""
    width = steps_per * dt
    mid = (np.arange(n_intervals, dtype=np.float64) + 0.5) * width
    return np.ascontiguousarray(pulse(mid))


def expand_piecewise(ek: np.ndarray, steps_per: int, slots: int = 3) -> np.ndarray:
    """[..., K] interval values -> [..., K*steps_per, slots] per-step stage samples."""
    rep = np.repeat(ek, steps_per, axis=-1)
    return np.ascontiguousarray(np.repeat(rep[..., None], slots, axis=-1))


def collapse_piecewise(g: np.ndarray, steps_per: int) -> np.ndarray:
    """Adjoint of expand_piecewise: sum per-step, per-slot gradients over each interval."""
    s = g.sum(axis=-1)
    return s.reshape(*s.shape[:-1], -1, steps_per).sum(axis=-1)


def random_state(rng: np.random.Generator, nstates: int, batch: int = 1) -> np.ndarray:
    c = rng.standard_normal((batch, 2 * nstates))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    return c
