"""Velocity gauge (Sec. 5: coupling A(t) P with P = -i Q Hermitian) through
every kernel path, vs the CPU oracle in the same gauge. Field samples are the
vector potential by step-wise 5-point Gauss-Legendre quadrature; coupling
blocks are the momentum blocks that match the synthetic dipole (P = i[H0, D]).
Bar: relative L2 of c(T) <= 1e-10; gradients 1e-10 of the largest entry."""
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


def system(lmax, n, seed):
    h = wl.hamiltonian(lmax, n, seed)
    return h, wl.velocity_coupling(h.energies, h.dipole)


def plan(h, q, batch=1):
    from paper_1201_6062_amd.api import Plan
    return Plan(h.energies, q if h.lmax > 0 else np.zeros((0, h.n, h.n)), batch=batch, gauge="velocity")


def a_samples(batch, dt, nsteps, method, seed=0):
    ps = [wl.Pulse(0.6 + 0.3 * b, 0.7 + 0.15 * b, 1.5) for b in range(batch)]
    return np.stack([wl.vector_potential_samples(p, dt, nsteps, method) for p in ps])


@pytest.mark.parametrize("lmax,n,batch", [(1, 1, 1), (2, 3, 1), (3, 130, 1), (15, 500, 1), (2, 70, 3),
                                          (3, 257, 2)])
def test_velocity_hmul(lmax, n, batch):
    h, q = system(lmax, n, 3)
    rng = np.random.default_rng(n)
    u = rng.standard_normal((batch, 2 * h.nstates))
    f = rng.uniform(-1, 1, batch)
    y = plan(h, q, batch).hmul(f, u).cpu().numpy()
    for b in range(batch):
        ref = oracle.hmul(h.energies, q, f[b], u[b], n=n, gauge="velocity")
        assert rel_l2(y[b], ref) <= 1e-13


@pytest.mark.parametrize("path", ["auto", "tiles", "split"])
@pytest.mark.parametrize("lmax,n,nsteps", [(3, 50, 120), (2, 130, 70), (1, 9, 90)])
def test_velocity_rk4_single(lmax, n, nsteps, path, monkeypatch):
    if path != "auto":
        monkeypatch.setenv("TDSE_TILE", f"T={(n + 127) // 128}")
        monkeypatch.setenv("TDSE_SPLIT", "1" if path == "split" else "0")
    h, q = system(lmax, n, 5)
    dt = 0.01
    f = a_samples(1, dt, nsteps, "rk4")
    c0 = wl.random_state(np.random.default_rng(1), h.nstates)
    got = plan(h, q).propagate(f, c0, dt, "rk4").cpu().numpy()
    ref = oracle.rk4(h.energies, q, dt, f, c0, n=n, gauge="velocity")
    assert rel_l2(got, ref) <= TOL


@pytest.mark.parametrize("batch", [1, 4])
def test_velocity_taylor(batch):
    h, q = system(3, 70, 6)
    dt, nsteps, order = 0.02, 40, 8
    f = a_samples(batch, dt, nsteps, "taylor")
    c0 = wl.random_state(np.random.default_rng(2), h.nstates, batch)
    got = plan(h, q, batch).propagate(f, c0, dt, "taylor", order=order).cpu().numpy()
    ref = oracle.taylor(h.energies, q, order, dt, f, c0, n=70, gauge="velocity")
    assert rel_l2(got, ref) <= TOL


def test_velocity_batched_rk4_full_size_short():
    h, q = system(15, 500, 0)
    dt, nsteps, batch = 0.005, 8, 16
    f = a_samples(batch, dt, nsteps, "rk4")
    c0 = wl.ground_state(15, 500, batch)
    got = plan(h, q, batch).propagate(f, c0, dt, "rk4").cpu().numpy()
    for b in (0, 7, 15):
        ref = oracle.rk4(h.energies, q, dt, f[b:b + 1], c0[b:b + 1], gauge="velocity")
        assert rel_l2(got[b:b + 1], ref) <= TOL


@pytest.mark.parametrize("method,batch", [("rk4", 3), ("rk4", 1), ("taylor", 2)])
def test_velocity_adjoint(method, batch):
    h, q = system(2, 13, 7)
    dt, nsteps, order = 0.04, 30, 5
    f = a_samples(batch, dt, nsteps, method)
    c0 = wl.ground_state(2, 13, batch)
    p = plan(h, q, batch)
    cT, ck = p.propagate(f, c0, dt, method, order=order, ckpt_every=8)
    en = torch.as_tensor(h.energies, device="cuda")
    lam = 2.0 * cT * (en > 0).to(torch.float64).repeat_interleave(2)[None, :]
    g, l0 = p.adjoint(f, c0, dt, lam, ckpt=ck, ckpt_every=8, method=method, order=order)
    g, l0 = g.cpu().numpy(), l0.cpu().numpy()
    for b in range(batch):
        if method == "rk4":
            cTb = oracle.rk4(h.energies, q, dt, f[b:b + 1], c0[b:b + 1], gauge="velocity")[0]
            l0r, gr = oracle.rk4_adjoint(h.energies, q, dt, f[b], c0[b], oracle.yield_seed(h.energies, cTb)[0],
                                         gauge="velocity")
        else:
            cTb = oracle.taylor(h.energies, q, order, dt, f[b:b + 1], c0[b:b + 1], gauge="velocity")[0]
            l0r, gr = oracle.taylor_adjoint(h.energies, q, order, dt, f[b], c0[b],
                                            oracle.yield_seed(h.energies, cTb)[0], gauge="velocity")
        g_b = g[b] if method == "rk4" else g[b][..., 0]
        assert np.abs(gr).max() > 1e-7
        assert np.abs(g_b - gr).max() <= 1e-10 * np.abs(gr).max()
        assert np.abs(l0[b] - l0r).max() <= 1e-10 * np.abs(l0r).max()


def test_group_mixed_gauges():
    """A group may hold plans of both gauges; each instance follows its own."""
    from paper_1201_6062_amd.api import Group, Plan
    specs = [(2, 70, 60, "velocity"), (3, 130, 45, "length"), (1, 20, 80, "velocity")]
    plans, fs, cs, refs = [], [], [], []
    for k, (lmax, n, nst, gauge) in enumerate(specs):
        h, q = system(lmax, n, 30 + k)
        blocks = q if gauge == "velocity" else h.dipole
        plans.append(Plan(h.energies, blocks, gauge=gauge))
        p = wl.Pulse(0.5, 0.6 + 0.1 * k, 1.5)
        f = (wl.vector_potential_samples(p, 0.01, nst) if gauge == "velocity" else wl.rk4_samples(p, 0.01, nst))
        c0 = wl.random_state(np.random.default_rng(k), h.nstates)[0]
        fs.append(f)
        cs.append(c0)
        refs.append(oracle.rk4(h.energies, blocks, 0.01, f[None], c0[None], n=n, gauge=gauge)[0])
    out = Group(plans).propagate(fs, cs, 0.01)
    for o, r in zip(out, refs):
        assert rel_l2(o.cpu().numpy(), r) <= TOL
