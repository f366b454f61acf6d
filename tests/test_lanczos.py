"""Short-iterative Lanczos propagator (tdse_propagate with TDSE_LANCZOS) vs
the oracle's Lanczos, on single-vector and batched plans, both gauges.
Bar: relative L2 of c(T) <= 1e-10 per pulse."""
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


def samples(batch, dt, nsteps, gauge="length"):
    ps = [wl.Pulse(0.5 + 0.2 * b, 0.6 + 0.1 * b, 1.5) for b in range(batch)]
    if gauge == "velocity":
        return np.stack([wl.vector_potential_samples(p, dt, nsteps, "taylor", "mid") for p in ps])
    return np.stack([wl.taylor_samples(p, dt, nsteps, "mid") for p in ps])


@pytest.mark.parametrize("lmax,n,batch,m,nsteps", [(2, 130, 1, 8, 30), (3, 50, 1, 12, 25), (1, 7, 1, 1, 40),
                                                  (2, 70, 3, 6, 20), (3, 257, 2, 10, 12), (0, 9, 2, 4, 15),
                                                  (2, 70, 1, 64, 8), (1, 40, 2, 64, 6)])
def test_lanczos_matches_oracle(lmax, n, batch, m, nsteps):
    h = wl.hamiltonian(lmax, n, 2)
    dt = 0.05
    f = samples(batch, dt, nsteps)
    c0 = wl.random_state(np.random.default_rng(m), h.nstates, batch)
    blocks = h.dipole if lmax > 0 else np.zeros((0, n, n))
    got = make_plan(h.energies, blocks, batch).propagate(f, c0, dt, "lanczos", order=m).cpu().numpy()
    ref = oracle.lanczos(h.energies, h.dipole, m, dt, f, c0, n=n)
    assert rel_l2(got, ref) <= TOL


@pytest.mark.parametrize("lmax,n", [(2, 900), (1, 2048)])
def test_lanczos_large_blocks(lmax, n):
    """One pulse with N = 900 (8 tiles per block dimension) and N = 2048 (16,
    the largest): the one-launch Krylov products with their run-time tile
    counts; 3 steps of Krylov dimension 6."""
    h = wl.hamiltonian(lmax, n, 8)
    dt, nsteps, m = 0.02, 3, 6
    f = samples(1, dt, nsteps)
    c0 = wl.random_state(np.random.default_rng(n), h.nstates, 1)
    got = make_plan(h.energies, h.dipole, 1).propagate(f, c0, dt, "lanczos", order=m).cpu().numpy()
    ref = oracle.lanczos(h.energies, h.dipole, m, dt, f, c0, n=n)
    assert rel_l2(got, ref) <= TOL


def test_lanczos_many_segments():
    """One pulse with Lmax=520, N=130 (1042 segments of at most 128 states,
    2080 tiles; 67730 states): more norm and dot parts than one workgroup
    reads in one pass, so the completion and product launches take their
    looping reductions; 3 steps of Krylov dimension 4."""
    h = wl.hamiltonian(520, 130, 4)
    dt, nsteps, m = 0.02, 3, 4
    f = samples(1, dt, nsteps)
    c0 = wl.random_state(np.random.default_rng(21), h.nstates, 1)
    got = make_plan(h.energies, h.dipole, 1).propagate(f, c0, dt, "lanczos", order=m).cpu().numpy()
    ref = oracle.lanczos(h.energies, h.dipole, m, dt, f, c0, n=130)
    assert rel_l2(got, ref) <= TOL


@pytest.mark.parametrize("lmax,n", [(2, 70), (0, 9)])
def test_lanczos_captured_chunks(lmax, n):
    """A single pulse without checkpoints replays captured 64-step chunks:
    150 steps (two chunks and a 22-step tail), then the same plan again with
    another dt, state and field (the chunk graph is reused; dt and the field
    come from the call's descriptor)."""
    h = wl.hamiltonian(lmax, n, 5)
    blocks = h.dipole if lmax > 0 else np.zeros((0, n, n))
    plan = make_plan(h.energies, blocks, 1)
    for dt, seed, nsteps in ((0.05, 1, 150), (0.03, 2, 130)):
        f = samples(1, dt, nsteps)
        c0 = wl.random_state(np.random.default_rng(seed), h.nstates, 1)
        got = plan.propagate(f, c0, dt, "lanczos", order=6).cpu().numpy()
        ref = oracle.lanczos(h.energies, h.dipole, 6, dt, f, c0, n=n)
        assert rel_l2(got, ref) <= TOL, (dt, nsteps)


@pytest.mark.parametrize("batch", [1, 4])
def test_lanczos_velocity_gauge(batch):
    h = wl.hamiltonian(2, 90, 3)
    q = wl.velocity_coupling(h.energies, h.dipole)
    dt, nsteps, m = 0.04, 25, 10
    f = samples(batch, dt, nsteps, "velocity")
    c0 = wl.random_state(np.random.default_rng(5), h.nstates, batch)
    got = make_plan(h.energies, q, batch, "velocity").propagate(f, c0, dt, "lanczos", order=m).cpu().numpy()
    ref = oracle.lanczos(h.energies, q, m, dt, f, c0, gauge="velocity")
    assert rel_l2(got, ref) <= TOL


def test_lanczos_full_size_short():
    """Lmax=15, N=500 single vector and 8 pulses, 6 steps of Krylov dimension 12."""
    h = wl.hamiltonian(15, 500, 0)
    dt, nsteps, m = 0.05, 6, 12
    for batch in (1, 8):
        f = samples(batch, dt, nsteps)
        c0 = wl.ground_state(15, 500, batch)
        got = make_plan(h.energies, h.dipole, batch).propagate(f, c0, dt, "lanczos", order=m).cpu().numpy()
        for b in sorted({0, batch - 1}):
            ref = oracle.lanczos(h.energies, h.dipole, m, dt, f[b:b + 1], c0[b:b + 1])
            assert rel_l2(got[b:b + 1], ref) <= TOL, batch


@pytest.mark.parametrize("batch", [1, 2])
def test_lanczos_checkpoints_and_alias(batch):
    h = wl.hamiltonian(2, 40, 6)
    dt, nsteps, m, k = 0.05, 23, 8, 5
    f = samples(batch, dt, nsteps)
    c0 = wl.random_state(np.random.default_rng(9), h.nstates, batch)
    plan = make_plan(h.energies, h.dipole, batch)
    cT, ck = plan.propagate(f, c0, dt, "lanczos", order=m, ckpt_every=k)
    ck = ck.cpu().numpy()
    for j in range(nsteps // k + 1):
        ref = oracle.lanczos(h.energies, h.dipole, m, dt, np.ascontiguousarray(f[:, : j * k]), c0)
        assert rel_l2(ck[:, j], ref) <= TOL, j
    buf = torch.as_tensor(c0, device="cuda").clone()
    plan.propagate(f, buf, dt, "lanczos", order=m, out=buf)
    assert torch.equal(buf, cT)


def test_lanczos_eigenstate_breakdown_is_exact_phase():
    h = wl.hamiltonian(2, 12, 1)
    c0 = np.zeros((1, 2 * h.nstates))
    c0[0, 2 * 13] = 1.0
    dt, nsteps = 0.7, 25
    got = make_plan(h.energies, h.dipole, 1).propagate(np.zeros((1, nsteps, 1)), c0, dt, "lanczos",
                                                       order=10).cpu().numpy()[0]
    z = got[0::2] + 1j * got[1::2]
    assert abs(z[13] - np.exp(-1j * h.energies[13] * dt * nsteps)) <= 1e-13
    assert np.abs(np.delete(z, 13)).max() <= 1e-15


def test_lanczos_adjoint_is_unsupported():
    from paper_1201_6062_amd.api import TdseError
    h = wl.hamiltonian(1, 5, 0)
    plan = make_plan(h.energies, h.dipole, 1)
    with pytest.raises(TdseError):
        plan.adjoint(np.zeros((1, 3, 1)), wl.ground_state(1, 5), 0.1, wl.ground_state(1, 5), method="lanczos",
                     order=4)
