"""tdse_propagate_noalloc (the entry point that allocates nothing, its
scratch in the library's fixed device array) against tdse_propagate on the
same plans and inputs: two calls in a row on one device, the second on a
smaller problem, so the second runs on what the first left in the array.
Both entry points run the same kernels in the same order, so the results
agree to the parity bar (checked) and in fact bit for bit (also checked)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1201_6062_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rel_l2(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def _case(lmax, n, seed, nsteps, method, order, dt):
    from paper_1201_6062_amd.api import Plan
    h = wl.hamiltonian(lmax, n, seed)
    plan = Plan(h.energies, h.dipole)
    p = wl.Pulse(0.08, 0.6, 3.0)
    f = wl.rk4_samples(p, dt, nsteps) if method == "rk4" else wl.taylor_samples(p, dt, nsteps)
    f = torch.as_tensor(f[None], device="cuda")
    c0 = torch.as_tensor(wl.random_state(np.random.default_rng(seed), h.nstates), device="cuda")
    return plan, f, c0


@pytest.mark.parametrize("method,order,dt", [("rk4", 4, 0.005), ("taylor", 8, 0.02)])
def test_noalloc_matches_propagate_two_calls(method, order, dt):
    cases = [(15, 500, 0, 150), (5, 200, 1, 37)]  # the second call smaller than the first
    for lmax, n, seed, nsteps in cases:
        plan, f, c0 = _case(lmax, n, seed, nsteps, method, order, dt)
        ref = plan.propagate(f, c0, dt, method, order=order)
        out = torch.full_like(c0, float("nan"))
        got = plan.propagate_noalloc(f, c0, dt, method, order=order, out=out)
        torch.cuda.synchronize()
        assert rel_l2(got, ref) <= TOL, (lmax, n)
        assert torch.equal(got, ref), (lmax, n)
        plan.close()


def test_noalloc_checkpoints_and_split_path():
    """Checkpoint rows through the fixed array, and a plan on the split
    (separate completion and product launches) path."""
    from paper_1201_6062_amd.api import Plan
    for lmax, n, nsteps, K in [(7, 300, 70, 16), (40, 400, 9, 4)]:  # 63 tiles (fused); 640 tiles (split)
        h = wl.hamiltonian(lmax, n, 3)
        plan = Plan(h.energies, h.dipole)
        f = torch.as_tensor(wl.rk4_samples(wl.Pulse(0.1, 0.5, 2.0), 0.01, nsteps)[None], device="cuda")
        c0 = torch.as_tensor(wl.random_state(np.random.default_rng(4), h.nstates), device="cuda")
        ref, ck_ref = plan.propagate(f, c0, 0.01, "rk4", ckpt_every=K)
        ck = torch.full_like(ck_ref, float("nan"))
        got = plan.propagate_noalloc(f, c0, 0.01, "rk4", ckpt=ck, ckpt_every=K)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.equal(ck, ck_ref)
        plan.close()


def test_noalloc_rejects_what_it_does_not_cover():
    from paper_1201_6062_amd import _capi
    from paper_1201_6062_amd.api import Plan, TdseError
    # scratch beyond the fixed array: Lmax=31, N=1000 needs about 19 MB
    h = wl.hamiltonian(2, 20, 0)
    big_en = wl.energies(31, 1000)
    big = Plan(big_en, np.zeros((31, 1000, 1000)))
    c0 = torch.zeros(1, 2 * 32 * 1000, dtype=torch.float64, device="cuda")
    f = torch.zeros(1, 3, 3, dtype=torch.float64, device="cuda")
    with pytest.raises(TdseError) as ei:
        big.propagate_noalloc(f, c0, 0.01)
    assert ei.value.status == _capi.TDSE_E_UNSUPPORTED and "fixed array" in str(ei.value)
    big.close()
    batched = Plan(h.energies, h.dipole, batch=2)
    with pytest.raises(TdseError):
        batched.propagate_noalloc(torch.zeros(2, 3, 3, dtype=torch.float64, device="cuda"),
                                  torch.zeros(2, 120, dtype=torch.float64, device="cuda"), 0.01)
    small = Plan(h.energies, h.dipole)
    with pytest.raises(TdseError):
        small.propagate_noalloc(torch.zeros(1, 3, 1, dtype=torch.float64, device="cuda"),
                                torch.zeros(1, 120, dtype=torch.float64, device="cuda"), 0.01, "lanczos", order=4)
    lib = _capi.load()
    assert lib.tdse_propagate_noalloc(None, 0, 0, 0.01, 1, None, None, None, None, 0, None) == _capi.TDSE_E_INVAL
    assert "plan is NULL" in lib.tdse_last_error().decode()
    _ = ctypes  # (ctypes used through the binding)


def test_noalloc_under_graph_capture():
    """The entry point recorded into a HIP graph (torch.cuda.graph on a side
    stream): it only enqueues kernels, so the captured graph replays the whole
    propagation. Three replays with eager work between them, each bitwise
    equal to the eager call; the tile path over two 64-step chunks and the
    one-workgroup path."""
    for lmax, n, seed, nsteps in [(15, 500, 0, 70), (3, 40, 2, 70)]:
        plan, f, c0 = _case(lmax, n, seed, nsteps, "rk4", 4, 0.005)
        ref = plan.propagate_noalloc(f, c0, 0.005, "rk4", out=torch.empty_like(c0))
        out = torch.full_like(c0, float("nan"))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # one eager call on the capturing stream first
            plan.propagate_noalloc(f, c0, 0.005, "rk4", out=out)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            plan.propagate_noalloc(f, c0, 0.005, "rk4", out=out)
        for rep in range(3):
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (lmax, n, rep)
            plan.propagate(f, c0, 0.005, "rk4")  # eager work of the program between replays
            torch.cuda.synchronize()
        del graph
        plan.close()
