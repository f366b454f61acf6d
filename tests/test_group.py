"""Uneven multi-instance group (different Lmax, N, pulses and step counts in
one schedule) vs the CPU oracle and vs each instance propagated alone."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1201_6062_amd import workloads as wl

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-10


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def plan_of(h):
    from paper_1201_6062_amd.api import Plan
    return Plan(h.energies, h.dipole if h.lmax else np.zeros((0, h.n, h.n)))


def test_group_small_uneven():
    from paper_1201_6062_amd.api import Group
    shapes = [(2, 130, 90), (3, 50, 70), (1, 7, 0), (0, 9, 40), (4, 257, 33), (2, 64, 129)]
    hs, fs, cs = [], [], []
    for q, (lmax, n, nst) in enumerate(shapes):
        h = wl.hamiltonian(lmax, n, 100 + q)
        p = wl.Pulse(0.1 + 0.02 * q, 0.5 + 0.1 * q, 2.0)
        hs.append(h)
        fs.append(wl.rk4_samples(p, 0.01, nst))
        cs.append(wl.random_state(np.random.default_rng(q), h.nstates)[0])
    plans = [plan_of(h) for h in hs]
    out = Group(plans).propagate(fs, cs, 0.01)
    for h, f, c, o in zip(hs, fs, cs, out):
        ref = oracle.rk4(h.energies, h.dipole, 0.01, f[None], c[None], n=h.n)[0]
        assert rel_l2(o.cpu().numpy(), ref) <= TOL


def test_group_equals_single_instance_runs(monkeypatch):
    """Same kernels, same summation order: bitwise equal to propagating alone
    on the split path (a completion launch, then the patch products launch),
    which is what every group round runs."""
    from paper_1201_6062_amd.api import Group
    monkeypatch.setenv("TDSE_SPLIT", "1")
    specs = wl.uneven_specs(64)[:6]
    hs = [wl.hamiltonian(s.lmax, s.n, s.seed) for s in specs]
    fs = [wl.rk4_samples(s.pulse, 0.005, 60 + 13 * q) for q, s in enumerate(specs)]
    cs = [wl.ground_state(s.lmax, s.n)[0] for s in specs]
    plans = [plan_of(h) for h in hs]
    out = Group(plans).propagate(fs, cs, 0.005)
    for p, f, c, o in zip(plans, fs, cs, out):
        alone = p.propagate(f[None], c[None], 0.005, "rk4")
        assert torch.equal(alone.reshape(-1), o)


def test_group_members_on_other_tile_counts(monkeypatch):
    """Members built with forced tile counts above the default (up to 11, past
    the 8 a group streams with) join a group, which streams each at its
    default count: bitwise equal to the same group of default plans, and
    within the tolerance of the oracle."""
    from paper_1201_6062_amd.api import Group
    shapes = [(3, 300, 5), (2, 500, 7), (4, 257, 9), (1, 1000, 11), (2, 130, 0)]
    hs = [wl.hamiltonian(l, n, 300 + q) for q, (l, n, _) in enumerate(shapes)]
    fs = [wl.rk4_samples(wl.Pulse(0.08, 0.5, 2.0), 0.01, 40 + 7 * q) for q in range(len(shapes))]
    cs = [wl.random_state(np.random.default_rng(50 + q), h.nstates)[0] for q, h in enumerate(hs)]
    forced = []
    for h, (_, _, t) in zip(hs, shapes):
        if t:
            monkeypatch.setenv("TDSE_TILE", f"T={t}")
        else:
            monkeypatch.delenv("TDSE_TILE", raising=False)
        forced.append(plan_of(h))
    monkeypatch.delenv("TDSE_TILE", raising=False)
    default = [plan_of(h) for h in hs]
    out_f = Group(forced).propagate(fs, cs, 0.01)
    out_d = Group(default).propagate(fs, cs, 0.01)
    for q, (h, f, c) in enumerate(zip(hs, fs, cs)):
        assert torch.equal(out_f[q], out_d[q]), shapes[q]
        ref = oracle.rk4(h.energies, h.dipole, 0.01, f[None], c[None], n=h.n)[0]
        assert rel_l2(out_f[q].cpu().numpy(), ref) <= TOL, shapes[q]


def test_group_rejects_members_beyond_1024_states_per_block():
    """A group streams every member at ceil(n / 128) tiles per block
    dimension, at most 8: n = 1100 is refused, whatever the plan's own count."""
    from paper_1201_6062_amd.api import Group
    from paper_1201_6062_amd._capi import TDSE_E_UNSUPPORTED, TdseError
    h = wl.hamiltonian(1, 1100, 3)
    with pytest.raises(TdseError, match="n <= 1024") as err:
        Group([plan_of(wl.hamiltonian(1, 60, 2)), plan_of(h)])
    assert err.value.status == TDSE_E_UNSUPPORTED


def test_group_rejects_a_plan_given_twice():
    from paper_1201_6062_amd.api import Group
    h = wl.hamiltonian(2, 70, 1)
    p = plan_of(h)
    with pytest.raises(Exception, match="same plan"):
        Group([p, plan_of(h), p])


def test_group_full_length_sampled_instances():
    """Instances 16, 21, 39 of the 64-instance workload, whole pulses, vs stored oracle results."""
    from paper_1201_6062_amd.api import Group
    specs = wl.uneven_specs(64)
    ids = [16, 21, 39]
    hs = [wl.hamiltonian(specs[i].lmax, specs[i].n, specs[i].seed) for i in ids]
    fs = [wl.rk4_samples(specs[i].pulse, 0.005, specs[i].nsteps) for i in ids]
    cs = [wl.ground_state(specs[i].lmax, specs[i].n)[0] for i in ids]
    out = Group([plan_of(h) for h in hs]).propagate(fs, cs, 0.005)
    for i, o in zip(ids, out):
        gold = np.load(os.path.join(HERE, "golden", f"uneven_inst{i:02d}.npz"), allow_pickle=False)
        assert int(gold["nsteps"]) == specs[i].nsteps
        assert rel_l2(o.cpu().numpy(), gold["cT"]) <= TOL


@pytest.fixture(scope="module")
def uneven64():
    """The 64-instance uneven workload: specs, Hamiltonians' plans, full-length
    samples, c0. The plans are created on the split path, so that each one
    propagated alone runs the kernels a group round runs."""
    specs = wl.uneven_specs(64)
    plans, fs, cs = [], [], []
    old = os.environ.get("TDSE_SPLIT")
    os.environ["TDSE_SPLIT"] = "1"
    try:
        for s in specs:
            h = wl.hamiltonian(s.lmax, s.n, s.seed)
            plans.append(plan_of(h))
            fs.append(torch.as_tensor(wl.rk4_samples(s.pulse, 0.005, s.nsteps), device="cuda"))
            cs.append(torch.as_tensor(wl.ground_state(s.lmax, s.n)[0], device="cuda"))
    finally:
        if old is None:
            del os.environ["TDSE_SPLIT"]
        else:
            os.environ["TDSE_SPLIT"] = old
    yield specs, plans, fs, cs
    for p in plans:
        p.close()


def test_group_all64_bitwise_alone(uneven64):
    """All 64 instances in one group for 40 steps: every instance bitwise
    equal to propagating it alone (same kernels, same summation order)."""
    from paper_1201_6062_amd.api import Group
    specs, plans, fs, cs = uneven64
    steps = 40
    out = Group(plans).propagate([f[:steps] for f in fs], cs, 0.005)
    for i, (p, f, c, o) in enumerate(zip(plans, fs, cs, out)):
        alone = p.propagate(f[:steps][None], c[None], 0.005, "rk4")
        assert torch.equal(alone.reshape(-1), o), i


def test_group_all64_first_200_steps(uneven64):
    """All 64 instances in one group for the first 200 steps of their pulses
    (the schedule the benchmark times, every instance active): sampled
    entries (every block, both ends and 12 seeded positions each), |c|^2 and
    sum E|c|^2 against the stored oracle results."""
    from paper_1201_6062_amd.api import Group
    specs, plans, fs, cs = uneven64
    gold = np.load(os.path.join(HERE, "golden", "uneven_prefix200.npz"), allow_pickle=False)
    steps = int(gold["steps"])
    out = Group(plans).propagate([f[:steps] for f in fs], cs, 0.005)
    for i, (s, o) in enumerate(zip(specs, out)):
        z = o.cpu().numpy().reshape(-1, 2)
        idx, ref = gold[f"idx{i:02d}"], gold[f"val{i:02d}"]
        assert rel_l2(z[idx], ref) <= TOL, i
        assert abs((z * z).sum() - gold[f"norm2_{i:02d}"]) <= 1e-12, i
        en = wl.energies(s.lmax, s.n)
        e = ((z * z).sum(1) * en).sum()
        assert abs(e - gold[f"energy_{i:02d}"]) <= 1e-11 * max(1.0, abs(e)), i


@pytest.mark.timeout(600)
def test_group_all64_full_length(uneven64):
    """All 64 instances in one group, each over its whole pulse (13230 to
    60461 steps), as one call: the smallest instance (#28, N=210), the largest
    (#38, Lmax=31, N=923), #30 (N=986) and #16, #21, #39 against their stored
    full-length oracle results."""
    from paper_1201_6062_amd.api import Group
    specs, plans, fs, cs = uneven64
    out = Group(plans).propagate(fs, cs, 0.005)
    torch.cuda.synchronize()
    for i in (28, 38, 30, 16, 21, 39):
        gold = np.load(os.path.join(HERE, "golden", f"uneven_inst{i:02d}.npz"), allow_pickle=False)
        assert int(gold["nsteps"]) == specs[i].nsteps
        assert rel_l2(out[i].cpu().numpy(), gold["cT"]) <= TOL, i


def test_group_repeated_calls_reuse_graphs():
    """Two calls on one group with different step counts and dt (captured
    chunks are reused with the new descriptor) and a third after the work
    list grew (a new group over more instances)."""
    from paper_1201_6062_amd.api import Group
    shapes = [(2, 70, 0), (3, 140, 0), (1, 20, 0)]
    hs = [wl.hamiltonian(l, n, 200 + q) for q, (l, n, _) in enumerate(shapes)]
    plans = [plan_of(h) for h in hs]
    grp = Group(plans)
    for call, (dt, steps) in enumerate([(0.01, (80, 33, 50)), (0.02, (41, 90, 17))]):
        fs = [wl.rk4_samples(wl.Pulse(0.1, 0.4 + 0.1 * q, 2.0), dt, st) for q, st in enumerate(steps)]
        cs = [wl.random_state(np.random.default_rng(10 * call + q), h.nstates)[0] for q, h in enumerate(hs)]
        out = grp.propagate(fs, cs, dt)
        for h, f, c, o in zip(hs, fs, cs, out):
            ref = oracle.rk4(h.energies, h.dipole, dt, f[None], c[None], n=h.n)[0]
            assert rel_l2(o.cpu().numpy(), ref) <= TOL, (call, h.lmax, h.n)
