"""Write the oracle's full-length results for the benchmark workloads.

Every stored value comes from the CPU oracle (package `oracle`) applied to the
seeded inputs of `paper_1201_6062_amd.workloads`; nothing here calls the HIP
library. Full-length runs take minutes to an hour each, so the GPU parity tests
read these files instead of re-running the oracle at full size.

    python tests/golden/make_golden.py single_small
    python tests/golden/make_golden.py single_large_rk4
    python tests/golden/make_golden.py single_large_taylor8
    python tests/golden/make_golden.py batched_col <b>       # one pulse of the 256-pulse batch
    python tests/golden/make_golden.py adjoint_pulse <b>     # one pulse of the 32-pulse adjoint batch
    python tests/golden/make_golden.py uneven_instance <i>   # one instance of the uneven batch
    python tests/golden/make_golden.py uneven_prefix <a> <b> # instances a..b-1, first 200 steps, sampled
    python tests/golden/make_golden.py uneven_prefix_merge   # join the parts into one file

Output: tests/golden/<name>.npz (plain arrays, loadable with allow_pickle=False).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1201_6062_amd import workloads as wl  # noqa: E402


def _save(name, **arrays):
    path = os.path.join(HERE, name + ".npz")
    np.savez(path + ".tmp.npz", **arrays)
    os.replace(path + ".tmp.npz", path)
    print("wrote", path, flush=True)


def _run_single(w):
    h = w.ham
    t = time.time()
    if w.method == "rk4":
        c = oracle.rk4(h.energies, h.dipole, w.dt, w.field, w.c0)
    else:
        c = oracle.taylor(h.energies, h.dipole, w.order, w.dt, w.field, w.c0)
    return c[0], time.time() - t


def single_small():
    w = wl.single_small()
    c, s = _run_single(w)
    _save("single_small_rk4", cT=c, nsteps=np.int64(w.nsteps), seconds=np.float64(s))


def single_large_rk4():
    w = wl.single_large("rk4")
    c, s = _run_single(w)
    _save("single_large_rk4", cT=c, nsteps=np.int64(w.nsteps), seconds=np.float64(s))


def single_large_taylor8():
    w = wl.single_large("taylor", 8)
    c, s = _run_single(w)
    _save("single_large_taylor8", cT=c, nsteps=np.int64(w.nsteps), seconds=np.float64(s))


def batched_col(b):
    w = wl.batched(256)
    h = w.ham
    t = time.time()
    c = oracle.rk4(h.energies, h.dipole, w.dt, w.field[b:b + 1], w.c0[b:b + 1])[0]
    _save(f"batched_col{b:03d}", cT=c, col=np.int64(b), nsteps=np.int64(w.nsteps),
          seconds=np.float64(time.time() - t))


def adjoint_pulse(b):
    h = wl.hamiltonian(15, 500, 0)
    p = wl.adjoint_pulses(32)[b]
    ek = wl.piecewise_samples(p)
    f = wl.expand_piecewise(ek[None], wl.ADJ_STEPS_PER_INTERVAL)[0]
    c0 = wl.ground_state(15, 500)[0]
    t = time.time()
    cT = oracle.rk4(h.energies, h.dipole, 0.01, f[None], c0[None])[0]
    lam_t = oracle.yield_seed(h.energies, cT)[0]
    lam0, g = oracle.rk4_adjoint(h.energies, h.dipole, 0.01, f, c0, lam_t)
    gk = wl.collapse_piecewise(g[None], wl.ADJ_STEPS_PER_INTERVAL)[0]
    _save(f"adjoint_pulse{b:02d}", cT=cT, lam0=lam0, grad_k=gk,
          yield_=np.float64(oracle.ionization_yield(h.energies, cT)[0]), pulse=np.int64(b),
          seconds=np.float64(time.time() - t))


def uneven_instance(i):
    spec = wl.uneven_specs(64)[i]
    h = wl.hamiltonian(spec.lmax, spec.n, spec.seed)
    f = wl.rk4_samples(spec.pulse, 0.005, spec.nsteps)
    t = time.time()
    c = oracle.rk4(h.energies, h.dipole, 0.005, f[None], wl.ground_state(spec.lmax, spec.n))[0]
    _save(f"uneven_inst{i:02d}", cT=c, inst=np.int64(i), nsteps=np.int64(spec.nsteps),
          seconds=np.float64(time.time() - t))


PREFIX_STEPS = 200


def prefix_sample_indices(i, lmax, n):
    """State indices kept from instance i's 200-step result: in every block the
    first two and last two states and 12 seeded random ones (up to 16 per block)."""
    rng = np.random.default_rng(7000 + i)
    out = []
    for l in range(lmax + 1):
        pick = set([0, min(1, n - 1), max(n - 2, 0), n - 1])
        pick.update(int(x) for x in rng.integers(0, n, 12))
        out.extend(l * n + a for a in sorted(pick))
    return np.array(out, dtype=np.int64)


def uneven_prefix(a, b):
    """Instances a..b-1 of the 64-instance workload, each over the first 200
    steps of its own pulse: sampled entries of c, plus |c|^2 and sum E|c|^2."""
    specs = wl.uneven_specs(64)
    out = {}
    t = time.time()
    for i in range(a, b):
        s = specs[i]
        h = wl.hamiltonian(s.lmax, s.n, s.seed)
        f = wl.rk4_samples(s.pulse, 0.005, PREFIX_STEPS)
        c = oracle.rk4(h.energies, h.dipole, 0.005, f[None], wl.ground_state(s.lmax, s.n))[0]
        idx = prefix_sample_indices(i, s.lmax, s.n)
        z = c.reshape(-1, 2)
        out[f"idx{i:02d}"] = idx
        out[f"val{i:02d}"] = np.ascontiguousarray(z[idx])
        out[f"norm2_{i:02d}"] = np.float64((z * z).sum())
        out[f"energy_{i:02d}"] = np.float64(((z * z).sum(1) * h.energies).sum())
        print("instance", i, "done", round(time.time() - t, 1), "s", flush=True)
    _save(f"uneven_prefix_{a:02d}_{b:02d}", steps=np.int64(PREFIX_STEPS), seconds=np.float64(time.time() - t), **out)


def uneven_prefix_merge():
    import glob
    merged = {}
    for path in sorted(glob.glob(os.path.join(HERE, "uneven_prefix_[0-9][0-9]_[0-9][0-9].npz"))):
        d = np.load(path, allow_pickle=False)
        merged.update({k: d[k] for k in d.files if k not in ("steps", "seconds")})
    have = sorted(k[3:] for k in merged if k.startswith("idx"))
    assert have == [f"{i:02d}" for i in range(64)], have
    _save("uneven_prefix200", steps=np.int64(PREFIX_STEPS), **merged)


if __name__ == "__main__":
    what = sys.argv[1]
    args = [int(a) for a in sys.argv[2:]]
    oracle.build(force=False)
    globals()[what](*args)
