"""The tile autotuner (tdse_tune): it times the candidate tile shapes of a
problem on the device, records the fastest in a JSON cache keyed by shape and
GPU architecture (the library's own choice unless another shape is at least
3% faster), and plans created with $TDSE_TUNE_CACHE pointing at that
cache use the recorded shape. The tuned plans must still match the oracle
(relative L2 of c(T) <= 1e-10)."""
import json

import numpy as np
import pytest
import torch  # noqa: F401  (loads the HIP runtime before the library)

import oracle
from paper_1201_6062_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-10
# (tm, tn, kc, K groups): the LDS kernels with one and two K groups, and the
# small-batch kernel (K groups 8) for 2B <= 64
SHAPES_BATCHED = {(128, 128, 16, 1), (128, 64, 16, 1), (64, 128, 16, 1), (64, 64, 16, 1), (64, 32, 16, 1),
                  (32, 64, 16, 1), (32, 32, 16, 1), (128, 64, 32, 1), (64, 128, 32, 1), (64, 64, 32, 1),
                  (32, 64, 32, 1), (32, 64, 32, 2), (32, 32, 16, 2), (32, 32, 16, 8), (32, 64, 16, 8)}


def rel_l2(a, b):
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    return np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1))


@pytest.mark.parametrize("lmax,n,batch", [(3, 260, 1), (2, 70, 5)])
def test_tune_writes_cache_and_plans_use_it(lmax, n, batch, tmp_path, monkeypatch):
    from paper_1201_6062_amd.api import Plan, tune
    cache = tmp_path / "tune.json"
    msg = tune(lmax, n, batch, str(cache))
    assert "best" in msg, msg
    data = json.loads(cache.read_text())
    assert data["arch"].startswith("gfx")
    entry = data["entries"][f"L{lmax}_N{n}_B{batch}"]
    # the same choice under the shape's bucket (n rounded up to a multiple of 64)
    assert data["entries"][f"L{lmax}_N{(n + 63) // 64 * 64}b_B{batch}"] == entry
    # all zeros: the library's own choice, kept unless a candidate beats it by 3%
    if batch == 1:
        t0 = (n + 127) // 128
        assert entry["T"] == 0 or t0 <= entry["T"] <= min(t0 + 3, 16, (n + 15) // 16)
        assert entry["tm"] == 0
    else:
        shape = (entry["tm"], entry["tn"], entry["kc"], entry["ks"])
        assert (shape == (0, 0, 0, 0) or shape in SHAPES_BATCHED) and entry["T"] == 0
    assert entry["us_per_step"] > 0
    # a second shape is added to the same cache, the first one kept
    tune(1, 40, 2, str(cache))
    data2 = json.loads(cache.read_text())
    assert f"L{lmax}_N{n}_B{batch}" in data2["entries"] and "L1_N40_B2" in data2["entries"]

    monkeypatch.setenv("TDSE_TUNE_CACHE", str(cache))
    # the tuned shape itself, and an untuned one of the same bucket (served by the bucket entry)
    for nn in (n, n + 7):
        h = wl.hamiltonian(lmax, nn, 9)
        dt, nsteps = 0.01, 40
        ps = wl.random_pulses(np.random.default_rng(4), batch, ncyc=2.0)
        f = np.stack([wl.rk4_samples(wl.Pulse(p.e0 * 5, p.omega, p.ncyc), dt, nsteps) for p in ps])
        c0 = wl.random_state(np.random.default_rng(5), h.nstates, batch)
        got = Plan(h.energies, h.dipole, batch=batch).propagate(f, c0, dt, "rk4").cpu().numpy()
        ref = oracle.rk4(h.energies, h.dipole, dt, f, c0, n=nn)
        assert rel_l2(got, ref) <= TOL, nn


def test_tune_cache_of_another_architecture_is_ignored(tmp_path, monkeypatch):
    """A cache written for another GPU architecture does not select tiles."""
    from paper_1201_6062_amd.api import Plan
    cache = tmp_path / "other.json"
    cache.write_text('{"arch": "gfx000", "entries": {\n'
                     '"L2_N70_B5": {"T": 0, "tm": 999, "tn": 999, "kc": 16, "us_per_step": 1.000}\n}}\n')
    monkeypatch.setenv("TDSE_TUNE_CACHE", str(cache))
    h = wl.hamiltonian(2, 70, 9)
    c0 = wl.random_state(np.random.default_rng(5), h.nstates, 5)
    f = np.zeros((5, 10, 3))
    got = Plan(h.energies, h.dipole, batch=5).propagate(f, c0, 0.01, "rk4").cpu().numpy()
    ref = oracle.rk4(h.energies, h.dipole, 0.01, f, c0, n=70)
    assert rel_l2(got, ref) <= TOL
