"""Runge-Kutta-Fehlberg 4(5) on the batched kernels (batch-1 plans through
their batched twin) vs the oracle: c(T) at 1e-10 relative L2 per pulse and the
per-step error estimates to 1e-6 of their largest value (an estimate is the
norm of a combination of the six stage derivatives that nearly cancels, so
its rounding error is about 1e-16 dt |k| in absolute terms); the optional step-size control
replayed step by step in the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1201_6062_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rel_l2(a, b):
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    return np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1))


def make_plan(en, blocks, batch, gauge="length"):
    from paper_1201_6062_amd.api import Plan
    return Plan(en, blocks, batch=batch, gauge=gauge)


def fields(batch, dt, nsteps):
    return np.stack([wl.rkf45_samples(wl.Pulse(0.4 + 0.2 * b, 0.6 + 0.1 * b, 1.5), dt, nsteps) for b in range(batch)])


@pytest.mark.parametrize("lmax,n,batch,nsteps,dt", [(2, 70, 3, 30, 0.1), (3, 130, 1, 25, 0.1), (1, 9, 2, 40, 0.2),
                                                   (15, 500, 4, 4, 0.005)])
def test_rkf45_matches_oracle(lmax, n, batch, nsteps, dt):
    h = wl.hamiltonian(lmax, n, 3)
    f = fields(batch, dt, nsteps)
    c0 = wl.random_state(np.random.default_rng(n), h.nstates, batch)
    cT, err = make_plan(h.energies, h.dipole, batch).propagate_rkf45(f, c0, dt)
    cT, err = cT.cpu().numpy(), err.cpu().numpy()
    for b in sorted({0, batch - 1}):
        ref, eref = oracle.rkf45(h.energies, h.dipole, dt, f[b:b + 1], c0[b:b + 1])
        assert rel_l2(cT[b:b + 1], ref) <= TOL
        assert eref.max() > 1e-12  # well above rounding, so the comparison means something
        assert np.abs(err[b] - eref[0]).max() <= 1e-6 * np.abs(eref).max()


def test_rkf45_256_pulses_sampled():
    """The shape the benchmark times: 256 pulses on the Lmax=15, N=500
    Hamiltonian (the 128x64 tile grid with one K group), three steps taken from
    the middle of the pulses (the field is strong there) from random states;
    pulses 0, 85, 170 and 255 and their error estimates vs the oracle."""
    h, dt, k0, nsteps, batch = wl.hamiltonian(15, 500, 0), 0.005, 20000, 3, 256
    pulses = wl.random_pulses(np.random.default_rng(1), batch)
    f = np.stack([wl.rkf45_samples(p, dt, k0 + nsteps)[k0:] for p in pulses])
    assert np.abs(f).max() > 0.02  # a field well away from zero in this window
    c0 = wl.random_state(np.random.default_rng(11), h.nstates, batch)
    cT, err = make_plan(h.energies, h.dipole, batch).propagate_rkf45(f, c0, dt)
    cT, err = cT.cpu().numpy(), err.cpu().numpy()
    for b in (0, 85, 170, 255):
        ref, eref = oracle.rkf45(h.energies, h.dipole, dt, f[b:b + 1], c0[b:b + 1])
        assert rel_l2(cT[b:b + 1], ref) <= TOL, b
        assert np.abs(err[b] - eref[0]).max() <= 1e-6 * np.abs(eref).max(), b


def test_rkf45_velocity_gauge_and_checkpoints():
    h = wl.hamiltonian(2, 40, 4)
    q = wl.velocity_coupling(h.energies, h.dipole)
    dt, nsteps, k, batch = 0.08, 23, 5, 2
    ps = [wl.Pulse(0.5, 0.6 + 0.2 * b, 1.5) for b in range(batch)]
    # vector potential at the six stage times of every step
    t = (np.arange(nsteps)[:, None] + np.array(wl.RKF45_SLOTS)[None, :]) * dt
    f = np.stack([wl.vector_potential_exact(p, t) for p in ps])
    c0 = wl.random_state(np.random.default_rng(1), h.nstates, batch)
    cT, err, ck = make_plan(h.energies, q, batch, "velocity").propagate_rkf45(f, c0, dt, ckpt_every=k)
    ref, eref = oracle.rkf45(h.energies, q, dt, f, c0, gauge="velocity")
    assert rel_l2(cT.cpu().numpy(), ref) <= TOL
    assert np.abs(err.cpu().numpy() - eref).max() <= 1e-6 * np.abs(eref).max()
    ck = ck.cpu().numpy()
    for j in range(nsteps // k + 1):
        r, _ = oracle.rkf45(h.energies, q, dt, np.ascontiguousarray(f[:, : j * k]), c0, gauge="velocity")
        assert rel_l2(ck[:, j], r) <= TOL, j


def test_rkf45_through_tdse_propagate():
    h = wl.hamiltonian(2, 20, 5)
    dt, nsteps = 0.02, 17
    f = fields(1, dt, nsteps)
    c0 = wl.ground_state(2, 20)
    got = make_plan(h.energies, h.dipole, 1).propagate(f, c0, dt, "rkf45").cpu().numpy()
    ref, _ = oracle.rkf45(h.energies, h.dipole, dt, f, c0)
    assert rel_l2(got, ref) <= TOL


def test_adaptive_step_control_replays_in_the_oracle():
    """The accepted step sequence of the adaptive driver, replayed step by
    step in the oracle, gives the same state; the driver reaches t_final and
    adapts dt to the pulse."""
    h = wl.hamiltonian(2, 30, 6)
    pulse = wl.Pulse(0.6, 0.7, 1.0)
    c0 = wl.ground_state(2, 30)
    plan = make_plan(h.energies, h.dipole, 1)
    cT, steps = plan.propagate_adaptive(lambda t: pulse(t), c0, pulse.duration, 0.05, 1e-9)
    assert abs(sum(steps) - pulse.duration) <= 1e-9 and len(set(np.round(steps, 12))) > 3
    c = c0.copy()
    t = 0.0
    for dt in steps:
        f = pulse(t + np.array(wl.RKF45_SLOTS) * dt)[None, None, :]
        c, _ = oracle.rkf45(h.energies, h.dipole, dt, f, c)
        t += dt
    assert rel_l2(cT.cpu().numpy(), c) <= TOL


def test_rkf45_adjoint_is_unsupported():
    from paper_1201_6062_amd.api import TdseError
    h = wl.hamiltonian(1, 5, 0)
    plan = make_plan(h.energies, h.dipole, 2)
    with pytest.raises(TdseError):
        plan.adjoint(np.zeros((2, 3, 6)), wl.ground_state(1, 5, 2), 0.1, wl.ground_state(1, 5, 2), method="rkf45")
