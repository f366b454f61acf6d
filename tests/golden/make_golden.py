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


if __name__ == "__main__":
    what = sys.argv[1]
    args = [int(a) for a in sys.argv[2:]]
    oracle.build(force=False)
    globals()[what](*args)
