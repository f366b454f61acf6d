"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks one part of the oracle against a closed form, an independent
dense construction, a textbook routine (numpy eigh, scipy solve_ivp), an exact
identity, or a number the paper prints. Together they are chosen so that a
dropped term, a wrong sign, a wrong index or a transposed block in the oracle
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

from paper_1201_6062_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))


def cplx(v):
    v = np.asarray(v)
    return v[..., 0::2] + 1j * v[..., 1::2]


def interleave(z):
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty(z.shape[:-1] + (2 * z.shape[-1],))
    out[..., 0::2] = z.real
    out[..., 1::2] = z.imag
    return out


def random_system(rng, lmax, n, scale=1.0):
    """Energies and NON-symmetric random blocks: a transposed use shows up."""
    en = rng.uniform(-1.0, 1.0, (lmax + 1) * n)
    dip = scale * rng.standard_normal((lmax, n, n))
    return en, dip


def dense_h(en, dip, field):
    """Assemble the full real matrix of Sec. 3's block structure (Fig. Matrix)."""
    lmax, n = dip.shape[0], en.size // (dip.shape[0] + 1)
    ns = (lmax + 1) * n
    h = np.diag(en).astype(np.float64)
    for l in range(lmax):
        r, c = slice(l * n, (l + 1) * n), slice((l + 1) * n, (l + 2) * n)
        h[r, c] += field * dip[l]
        h[c, r] += field * dip[l].T
    assert h.shape == (ns, ns)
    return h


def poly_exp(z, order):
    """Truncated exponential series sum_{m<=order} z^m / m! (elementwise)."""
    out = np.zeros_like(z, dtype=np.complex128)
    term = np.ones_like(z, dtype=np.complex128)
    for m in range(order + 1):
        if m > 0:
            term = term * z / m
        out = out + term
    return out


def step_matrix(h, dt, order):
    """R_order(-i h dt) through the eigendecomposition of the symmetric h."""
    lam, v = np.linalg.eigh(h)
    return (v * poly_exp(-1j * lam * dt, order)[None, :]) @ v.T


# ---------------------------------------------------------------- matvec (O1)

@pytest.mark.parametrize("lmax,n", [(0, 4), (1, 1), (2, 3), (3, 5)])
def test_hmul_matches_dense_assembly(oracle_mod, lmax, n):
    rng = np.random.default_rng(10 + lmax * 7 + n)
    en, dip = random_system(rng, lmax, n)
    u = rng.standard_normal(2 * (lmax + 1) * n)
    for f in (0.0, 0.37, -1.3):
        y = oracle_mod.hmul(en, dip, f, u, n=n)
        ref = dense_h(en, dip, f) @ cplx(u)
        np.testing.assert_allclose(cplx(y), ref, rtol=0, atol=1e-14 * (1 + np.abs(ref).max()))


def test_dmul_is_field_part(oracle_mod):
    rng = np.random.default_rng(3)
    en, dip = random_system(rng, 3, 4)
    u = rng.standard_normal(2 * 16)
    z = oracle_mod.dmul(en, dip, u, n=4)
    h1 = dense_h(en, dip, 1.0) - np.diag(en)
    np.testing.assert_allclose(cplx(z), h1 @ cplx(u), atol=1e-14)


def test_hmul_symmetric(oracle_mod):
    """u^H (H v) = (H u)^H v for the symmetric H built from the generator."""
    h = wl.hamiltonian(3, 6, 5)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, 2 * h.nstates))
    hu = cplx(oracle_mod.hmul(h.energies, h.dipole, 0.8, u))
    hv = cplx(oracle_mod.hmul(h.energies, h.dipole, 0.8, v))
    a = np.vdot(cplx(u), hv)
    b = np.vdot(hu, cplx(v))
    assert abs(a - b) <= 1e-13 * abs(a)


# ------------------------------------------------------- field-free (O2, O3)

def test_rk4_field_free_closed_form(oracle_mod):
    h = wl.hamiltonian(2, 12, 0)
    rng = np.random.default_rng(2)
    c0 = wl.random_state(rng, h.nstates)
    dt, nst = 0.01, 400
    cT = oracle_mod.rk4(h.energies, h.dipole, dt, np.zeros((1, nst, 3)), c0)
    r = poly_exp(-1j * h.energies * dt, 4)
    ref = cplx(c0[0]) * r ** nst
    np.testing.assert_allclose(cplx(cT[0]), ref, rtol=0, atol=1e-13)
    # against the exact phase, within the RK4 local-error bound nsteps*|theta|^5/120
    theta = np.abs(h.energies * dt)
    exact = cplx(c0[0]) * np.exp(-1j * h.energies * dt * nst)
    bound = nst * theta ** 5 / 120 * np.abs(cplx(c0[0])) * 1.05 + 1e-14
    assert np.all(np.abs(cplx(cT[0]) - exact) <= bound)


@pytest.mark.parametrize("order", [1, 2, 5, 8, 10])
def test_taylor_field_free_closed_form(oracle_mod, order):
    h = wl.hamiltonian(1, 12, 0)
    rng = np.random.default_rng(order)
    c0 = wl.random_state(rng, h.nstates)
    dt, nst = 0.02, 150
    cT = oracle_mod.taylor(h.energies, h.dipole, order, dt, np.zeros((1, nst)), c0)
    ref = cplx(c0[0]) * poly_exp(-1j * h.energies * dt, order) ** nst
    np.testing.assert_allclose(cplx(cT[0]), ref, rtol=0, atol=1e-13)


def test_field_free_norm_drift_closed_form(oracle_mod):
    """|R4(i theta)|^2 = 1 - theta^6/72 + theta^8/576 per step (RK4 on a phase)."""
    en = np.array([0.0, 3.0, 9.0, 30.0])
    dip = np.zeros((3, 1, 1))
    dt, nst = 0.01, 50
    c0 = interleave(np.ones(4) / 2.0)[None]
    cT = oracle_mod.rk4(en, dip, dt, np.zeros((1, nst, 3)), c0, n=1)
    th = en * dt
    per_step = 1 - th ** 6 / 72 + th ** 8 / 576
    np.testing.assert_allclose(np.abs(cplx(cT[0])) ** 2, 0.25 * per_step ** nst, rtol=1e-13)


# -------------------------------------------------------- two-level Rabi

def rabi_exact(ea, eb, d, f, t):
    ebar, delta, v = (ea + eb) / 2, (eb - ea) / 2, f * d
    om = math.hypot(delta, v)
    ph = np.exp(-1j * ebar * t)
    ca = ph * (np.cos(om * t) + 1j * delta / om * np.sin(om * t))
    cb = -1j * ph * (v / om) * np.sin(om * t)
    return np.array([ca, cb])


def test_rabi_two_level(oracle_mod):
    ea, eb, d, f = -0.5, -0.125, 0.74, 0.2
    en, dip = np.array([ea, eb]), np.array([[[d]]])
    t_final = 30.0
    c0 = np.array([[1.0, 0.0, 0.0, 0.0]])
    errs = []
    for nst in (300, 600, 1200):
        dt = t_final / nst
        cT = oracle_mod.rk4(en, dip, dt, np.full((1, nst, 3), f), c0, n=1)
        exact = rabi_exact(ea, eb, d, f, t_final)
        errs.append(np.abs(cplx(cT[0]) - exact).max())
        # the discrete map itself, from the 2x2 eigendecomposition
        m = step_matrix(dense_h(en, dip, f), dt, 4)
        disc = np.linalg.matrix_power(m, nst) @ np.array([1.0, 0.0])
        # rounding of both sides grows at most linearly with the step count
        np.testing.assert_allclose(cplx(cT[0]), disc, rtol=0, atol=5e-16 * nst)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.0 < r1 < 18.0 and 14.0 < r2 < 18.0, (errs, r1, r2)


# ------------------------------------------- dense propagation, tiny systems

def stepwise_fields(nst, dt, seed=0):
    t = (np.arange(nst) + 0.5) * dt
    return 0.6 * np.sin(0.9 * t + seed) * np.exp(-((t - t[-1] / 2) / (t[-1] / 3)) ** 2)


def test_rk4_dense_step_product(oracle_mod):
    """Step-constant field: c(T) = prod_k R4(-i H_k dt) c0, each factor by eigh."""
    h = wl.hamiltonian(2, 3, 4)
    rng = np.random.default_rng(4)
    c0 = wl.random_state(rng, h.nstates)
    dt, nst = 0.05, 80
    fk = stepwise_fields(nst, dt)
    field = np.repeat(fk[:, None], 3, axis=1)[None]
    cT = oracle_mod.rk4(h.energies, h.dipole, dt, field, c0)
    v = cplx(c0[0])
    for k in range(nst):
        v = step_matrix(dense_h(h.energies, h.dipole, fk[k]), dt, 4) @ v
    np.testing.assert_allclose(cplx(cT[0]), v, rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [3, 6, 8])
def test_taylor_dense_step_product(oracle_mod, order):
    h = wl.hamiltonian(2, 3, 4)
    rng = np.random.default_rng(40 + order)
    c0 = wl.random_state(rng, h.nstates)
    dt, nst = 0.08, 60
    fk = stepwise_fields(nst, dt, 1.0)
    cT = oracle_mod.taylor(h.energies, h.dipole, order, dt, fk[None], c0)
    v = cplx(c0[0])
    for k in range(nst):
        v = step_matrix(dense_h(h.energies, h.dipole, fk[k]), dt, order) @ v
    np.testing.assert_allclose(cplx(cT[0]), v, rtol=0, atol=1e-13)


def expm_product(h_en, h_dip, fk, dt, c0):
    v = cplx(c0)
    for f in fk:
        hm = dense_h(h_en, h_dip, f)
        lam, vv = np.linalg.eigh(hm)
        v = (vv * np.exp(-1j * lam * dt)[None, :]) @ (vv.T @ v)
    return v


@pytest.mark.parametrize("method,order,expect", [("rk4", 4, 16.0), ("taylor", 3, 8.0), ("taylor", 5, 32.0)])
def test_convergence_to_exponential(oracle_mod, method, order, expect):
    """Against the exact exp(-i H_k dt) product: error ratio 2^order on halving dt."""
    h = wl.hamiltonian(1, 3, 9)
    c0 = wl.ground_state(1, 3)
    t_final, errs = 6.0, []
    for nst in (60, 120, 240):
        dt = t_final / nst
        # field constant over pairs of coarse steps so every resolution sees the same H(t)
        coarse = stepwise_fields(30, t_final / 30)
        fk = np.repeat(coarse, nst // 30)
        ref = expm_product(h.energies, h.dipole, fk, dt, c0[0])
        if method == "rk4":
            cT = oracle_mod.rk4(h.energies, h.dipole, dt, np.repeat(fk[:, None], 3, 1)[None], c0)
        else:
            cT = oracle_mod.taylor(h.energies, h.dipole, order, dt, fk[None], c0)
        errs.append(np.abs(cplx(cT[0]) - ref).max())
    r = errs[1] / errs[2]
    assert abs(r / expect - 1) < 0.15, errs


def test_rk4_time_dependent_order(oracle_mod):
    """Smooth field with distinct stage samples vs a tight DOP853 solve: 4th order.

    Using the samples in the wrong stage slots (planted below by permuting the
    sample columns) drops the order, so this pins the slot assignment.
    """
    from scipy.integrate import solve_ivp

    h = wl.hamiltonian(1, 3, 2)
    c0 = wl.ground_state(1, 3)
    pulse = wl.Pulse(0.8, 0.9, 2.0)
    t_final = pulse.duration
    h0, h1 = np.diag(h.energies), dense_h(h.energies, h.dipole, 1.0) - np.diag(h.energies)

    def rhs(t, y):
        return -1j * (h0 + float(pulse(t)) * h1) @ y

    sol = solve_ivp(rhs, (0, t_final), cplx(c0[0]).astype(complex), method="DOP853",
                    rtol=1e-13, atol=1e-15)
    ref = sol.y[:, -1]

    def err(nst, perm=(0, 1, 2)):
        dt = t_final / nst
        f = wl.rk4_samples(pulse, dt, nst)[:, list(perm)]
        cT = oracle_mod.rk4(h.energies, h.dipole, dt, f[None], c0)
        return np.abs(cplx(cT[0]) - ref).max()

    e = [err(m) for m in (100, 200, 400)]
    assert 13.0 < e[0] / e[1] < 19.0 and 13.0 < e[1] / e[2] < 19.0, e
    bad = [err(m, (2, 1, 0)) for m in (100, 200, 400)]
    assert bad[1] / bad[2] < 5.0, bad


def test_rk4_equals_taylor4_when_samples_equal(oracle_mod):
    h = wl.hamiltonian(3, 7, 1)
    rng = np.random.default_rng(8)
    c0 = wl.random_state(rng, h.nstates)
    dt, nst = 0.02, 120
    fk = stepwise_fields(nst, dt)
    a = oracle_mod.rk4(h.energies, h.dipole, dt, np.repeat(fk[:, None], 3, 1)[None], c0)
    b = oracle_mod.taylor(h.energies, h.dipole, 4, dt, fk[None], c0)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_norm_nonincreasing_when_stable(oracle_mod):
    """dt ||H_k|| <= 2 sqrt(2): the RK4 step matrix is a normal contraction."""
    h = wl.hamiltonian(2, 8, 3)
    rng = np.random.default_rng(5)
    c = wl.random_state(rng, h.nstates)
    fk = stepwise_fields(100, 0.05) * 2.0
    dt = 0.05
    for f in fk:
        hn = np.linalg.norm(dense_h(h.energies, h.dipole, f), 2)
        assert dt * hn <= 2 * math.sqrt(2)
        nxt = oracle_mod.rk4(h.energies, h.dipole, dt, np.full((1, 1, 3), f), c)
        assert np.linalg.norm(nxt) <= np.linalg.norm(c) * (1 + 1e-15)
        c = nxt


def test_linearity(oracle_mod):
    h = wl.hamiltonian(2, 10, 6)
    rng = np.random.default_rng(6)
    a, b = wl.random_state(rng, h.nstates, 2)
    f = wl.rk4_samples(wl.Pulse(0.3, 0.7, 2.0), 0.02, 300)[None]
    al, be = 0.3 - 1.1j, -0.7 + 0.2j
    mix = interleave(al * cplx(a) + be * cplx(b))[None]
    ra = oracle_mod.rk4(h.energies, h.dipole, 0.02, f, a[None])
    rb = oracle_mod.rk4(h.energies, h.dipole, 0.02, f, b[None])
    rm = oracle_mod.rk4(h.energies, h.dipole, 0.02, f, mix)
    np.testing.assert_allclose(cplx(rm[0]), al * cplx(ra[0]) + be * cplx(rb[0]), atol=1e-14)


# --------------------------------------------------------------- adjoint (O5, O6)

def _adj_case(seed=0, lmax=2, n=13, nst=40, dt=0.05):
    # n > 10: three continuum (E > 0) states per partial wave, so the yield is non-trivial
    h = wl.hamiltonian(lmax, n, seed)
    rng = np.random.default_rng(seed + 100)
    f = wl.rk4_samples(wl.Pulse(0.7, 0.8, 1.0), dt, nst) + 0.05 * rng.standard_normal((nst, 3))
    c0 = wl.ground_state(lmax, n)[0]
    return h, f, c0, dt


def test_adjoint_dot_product_identity(oracle_mod):
    """For the linear map c0 -> cT: Re<lambda_0, dc0> = Re<lambda_T, dcT>."""
    h, f, c0, dt = _adj_case()
    rng = np.random.default_rng(11)
    lam_t = rng.standard_normal(c0.size)
    dc0 = rng.standard_normal(c0.size)
    lam0, _ = oracle_mod.rk4_adjoint(h.energies, h.dipole, dt, f, c0, lam_t)
    dct = oracle_mod.rk4(h.energies, h.dipole, dt, f[None], dc0[None])[0]
    lhs = np.real(np.vdot(cplx(lam0), cplx(dc0)))
    rhs = np.real(np.vdot(cplx(lam_t), cplx(dct)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300) + 1e-15


def _yield_grad(oracle_mod, h, f, c0, dt):
    cT = oracle_mod.rk4(h.energies, h.dipole, dt, f[None], c0[None])[0]
    lam_t = oracle_mod.yield_seed(h.energies, cT)[0]
    return oracle_mod.rk4_adjoint(h.energies, h.dipole, dt, f, c0, lam_t)


def test_adjoint_matches_tangent_linear(oracle_mod):
    h, f, c0, dt = _adj_case(1)
    _, grad = _yield_grad(oracle_mod, h, f, c0, dt)
    assert np.abs(grad).max() > 1e-4
    mask = oracle_mod.positive_mask(h.energies)
    rng = np.random.default_rng(3)
    for trial in range(6):
        df = np.zeros_like(f)
        if trial < 3:
            df.flat[rng.integers(0, f.size)] = 1.0
        else:
            df = rng.standard_normal(f.shape)
        cT, dcT = oracle_mod.rk4_tangent(h.energies, h.dipole, dt, f, df, c0)
        dy = 2.0 * np.sum(np.real(np.conj(cplx(cT)) * cplx(dcT)) * mask)
        g = np.sum(grad * df)
        assert abs(g - dy) <= 1e-10 * max(abs(dy), np.abs(grad).max() * 1e-3), (g, dy)


def test_adjoint_matches_central_fd(oracle_mod):
    h, f, c0, dt = _adj_case(2)
    _, grad = _yield_grad(oracle_mod, h, f, c0, dt)
    assert np.abs(grad).max() > 1e-4

    def y_of(ff):
        cT = oracle_mod.rk4(h.energies, h.dipole, dt, ff[None], c0[None])
        return oracle_mod.ionization_yield(h.energies, cT)[0]

    hstep = 1e-5
    idx = np.argsort(-np.abs(grad).ravel())[:8]
    scale = np.abs(grad).max()
    for i in idx:
        fp, fm = f.copy(), f.copy()
        fp.flat[i] += hstep
        fm.flat[i] -= hstep
        fd = (y_of(fp) - y_of(fm)) / (2 * hstep)
        assert abs(fd - grad.flat[i]) <= 1e-6 * scale, (i, fd, grad.flat[i])


def test_adjoint_lambda0_matches_fd(oracle_mod):
    """lambda_0 = dY/dRe c0 + i dY/dIm c0, checked along a random direction."""
    h, f, c0, dt = _adj_case(3)
    lam0, _ = _yield_grad(oracle_mod, h, f, c0, dt)
    assert np.abs(lam0).max() > 1e-4
    rng = np.random.default_rng(12)
    d = rng.standard_normal(c0.size)

    def y_of(c):
        cT = oracle_mod.rk4(h.energies, h.dipole, dt, f[None], c[None])
        return oracle_mod.ionization_yield(h.energies, cT)[0]

    eps = 1e-6
    fd = (y_of(c0 + eps * d) - y_of(c0 - eps * d)) / (2 * eps)
    an = np.dot(lam0, d)   # Re(lambda^H d) in interleaved form
    assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-6)


# ------------------------------------------------------- generator and paper facts

# ---- Taylor-p adjoint (next to the RK4 adjoint: same convention dL = Re(lambda^H dc))

def _tay_case(seed=0, lmax=2, n=13, nst=30, dt=0.05):
    h = wl.hamiltonian(lmax, n, seed)
    rng = np.random.default_rng(seed + 200)
    f = wl.taylor_samples(wl.Pulse(0.7, 0.8, 1.0), dt, nst)[:, 0] + 0.05 * rng.standard_normal(nst)
    c0 = wl.ground_state(lmax, n)[0]
    return h, f, c0, dt


@pytest.mark.parametrize("order", [1, 4, 7])
def test_taylor_adjoint_dot_product_identity(oracle_mod, order):
    h, f, c0, dt = _tay_case(order)
    rng = np.random.default_rng(21 + order)
    lam_t = rng.standard_normal(c0.size)
    dc0 = rng.standard_normal(c0.size)
    lam0, _ = oracle_mod.taylor_adjoint(h.energies, h.dipole, order, dt, f, c0, lam_t)
    dct = oracle_mod.taylor(h.energies, h.dipole, order, dt, f[None], dc0[None])[0]
    lhs = np.real(np.vdot(cplx(lam0), cplx(dc0)))
    rhs = np.real(np.vdot(cplx(lam_t), cplx(dct)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300) + 1e-15


@pytest.mark.parametrize("order", [2, 5, 8])
def test_taylor_adjoint_matches_central_fd(oracle_mod, order):
    h, f, c0, dt = _tay_case(10 + order)

    def y_of(ff):
        cT = oracle_mod.taylor(h.energies, h.dipole, order, dt, ff[None], c0[None])
        return oracle_mod.ionization_yield(h.energies, cT)[0]

    cT = oracle_mod.taylor(h.energies, h.dipole, order, dt, f[None], c0[None])[0]
    lam_t = oracle_mod.yield_seed(h.energies, cT)[0]
    _, grad = oracle_mod.taylor_adjoint(h.energies, h.dipole, order, dt, f, c0, lam_t)
    assert np.abs(grad).max() > 1e-4
    scale = np.abs(grad).max()
    hstep = 1e-5
    for i in list(np.argsort(-np.abs(grad))[:6]) + [0, f.size - 1]:
        fp, fm = f.copy(), f.copy()
        fp[i] += hstep
        fm[i] -= hstep
        fd = (y_of(fp) - y_of(fm)) / (2 * hstep)
        assert abs(fd - grad[i]) <= 1e-6 * scale, (i, fd, grad[i])


def test_taylor4_adjoint_equals_rk4_adjoint_when_samples_equal(oracle_mod):
    """With the three RK4 stage samples of a step equal, RK4 and Taylor-4 are
    the same map (pinned above), so their adjoints agree: lambda_0 equal and
    the Taylor gradient of a step equal to the sum of its three RK4 slots."""
    h = wl.hamiltonian(2, 12, 4)
    rng = np.random.default_rng(31)
    dt, nst = 0.04, 35
    fk = stepwise_fields(nst, dt, seed=3) + 0.3
    c0 = wl.random_state(rng, h.nstates)[0]
    lam_t = rng.standard_normal(c0.size)
    l_rk, g_rk = oracle_mod.rk4_adjoint(h.energies, h.dipole, dt, np.repeat(fk[:, None], 3, 1), c0, lam_t)
    l_ty, g_ty = oracle_mod.taylor_adjoint(h.energies, h.dipole, 4, dt, fk, c0, lam_t)
    np.testing.assert_allclose(l_ty, l_rk, rtol=0, atol=1e-13 * np.abs(l_rk).max())
    np.testing.assert_allclose(g_ty, g_rk.sum(axis=1), rtol=0, atol=1e-12 * np.abs(g_rk).max())


def test_midpoint_taylor_second_order_in_field(oracle_mod):
    """Freezing H at the step's left end (appendix B) makes Taylor-p first
    order in dt once the field varies in time; sampling the field at the
    step's midpoint makes it second order (the exponential midpoint rule)."""
    from scipy.integrate import solve_ivp

    h = wl.hamiltonian(1, 4, 5)
    c0 = wl.ground_state(1, 4)
    pulse = wl.Pulse(0.9, 0.7, 1.0)
    t_final = pulse.duration
    h0, h1 = np.diag(h.energies), dense_h(h.energies, h.dipole, 1.0) - np.diag(h.energies)
    sol = solve_ivp(lambda t, y: -1j * (h0 + float(pulse(t)) * h1) @ y, (0, t_final),
                    cplx(c0[0]).astype(complex), method="DOP853", rtol=1e-13, atol=1e-15)
    ref = sol.y[:, -1]

    def err(nst, where):
        dt = t_final / nst
        f = wl.taylor_samples(pulse, dt, nst, where)
        cT = oracle_mod.taylor(h.energies, h.dipole, 10, dt, f[None], c0)
        return np.abs(cplx(cT[0]) - ref).max()

    left = [err(m, "left") for m in (200, 400, 800)]
    mid = [err(m, "mid") for m in (200, 400, 800)]
    assert 1.6 < left[0] / left[1] < 2.5 and 1.6 < left[1] / left[2] < 2.5, left
    assert 3.2 < mid[0] / mid[1] < 5.0 and 3.2 < mid[1] / mid[2] < 5.0, mid


# ---- velocity gauge (Sec. 5): H = E + A(t) P, P = -i Q Hermitian

def dense_h_velocity(en, q, a):
    """Full complex matrix: P_{l,l+1} = -i Q_l, P_{l+1,l} = +i Q_l^T."""
    lmax, n = q.shape[0], en.size // (q.shape[0] + 1)
    h = np.diag(en).astype(np.complex128)
    for l in range(lmax):
        r, c = slice(l * n, (l + 1) * n), slice((l + 1) * n, (l + 2) * n)
        h[r, c] += -1j * a * q[l]
        h[c, r] += 1j * a * q[l].T
    return h


@pytest.mark.parametrize("lmax,n", [(1, 1), (2, 3), (3, 5)])
def test_velocity_hmul_matches_dense_assembly(oracle_mod, lmax, n):
    rng = np.random.default_rng(40 + n)
    en, q = random_system(rng, lmax, n)      # non-symmetric blocks: a wrong transpose shows
    u = rng.standard_normal(2 * en.size)
    for a in (0.0, 0.37, -1.3):
        y = oracle_mod.hmul(en, q, a, u, n=n, gauge="velocity")
        ref = dense_h_velocity(en, q, a) @ cplx(u)
        np.testing.assert_allclose(cplx(y), ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()))
        assert np.allclose(dense_h_velocity(en, q, a), dense_h_velocity(en, q, a).conj().T)


def test_velocity_coupling_is_the_commutator():
    """P = -i Q built from the dipole equals i [H0, D] in the basis."""
    h = wl.hamiltonian(2, 6, 3)
    q = wl.velocity_coupling(h.energies, h.dipole)
    p_dense = dense_h_velocity(np.zeros_like(h.energies), q, 1.0)
    d_dense = dense_h(np.zeros_like(h.energies), h.dipole, 1.0)
    h0 = np.diag(h.energies)
    np.testing.assert_allclose(p_dense, 1j * (h0 @ d_dense - d_dense @ h0), rtol=0, atol=1e-14)


def test_velocity_rk4_dense_step_product(oracle_mod):
    h = wl.hamiltonian(2, 3, 5)
    q = wl.velocity_coupling(h.energies, h.dipole)
    rng = np.random.default_rng(6)
    c0 = wl.random_state(rng, h.nstates)
    dt, nst = 0.05, 60
    ak = stepwise_fields(nst, dt, seed=1)
    cT = oracle_mod.rk4(h.energies, q, dt, np.repeat(ak[:, None], 3, axis=1)[None], c0, gauge="velocity")
    v = cplx(c0[0])
    for k in range(nst):
        lam, w = np.linalg.eigh(dense_h_velocity(h.energies, q, ak[k]))
        v = (w * poly_exp(-1j * lam * dt, 4)[None, :]) @ (w.conj().T @ v)
    np.testing.assert_allclose(cplx(cT[0]), v, rtol=0, atol=1e-13)


@pytest.mark.parametrize("method", ["rk4", "taylor"])
def test_velocity_adjoint_dot_product_and_fd(oracle_mod, method):
    h = wl.hamiltonian(2, 13, 8)
    q = wl.velocity_coupling(h.energies, h.dipole)
    dt, nst, order = 0.05, 30, 6
    pulse = wl.Pulse(0.9, 0.8, 1.0)
    f = wl.vector_potential_samples(pulse, dt, nst, method)
    if method == "taylor":
        f = f[:, 0]
    c0 = wl.ground_state(2, 13)[0]
    rng = np.random.default_rng(9)

    def fwd(ff, c):
        if method == "rk4":
            return oracle_mod.rk4(h.energies, q, dt, ff[None], c[None], gauge="velocity")[0]
        return oracle_mod.taylor(h.energies, q, order, dt, ff[None], c[None], gauge="velocity")[0]

    def adj(lam):
        if method == "rk4":
            return oracle_mod.rk4_adjoint(h.energies, q, dt, f, c0, lam, gauge="velocity")
        return oracle_mod.taylor_adjoint(h.energies, q, order, dt, f, c0, lam, gauge="velocity")

    lam_t = rng.standard_normal(c0.size)
    dc0 = rng.standard_normal(c0.size)
    lam0, _ = adj(lam_t)
    lhs, rhs = np.dot(lam0, dc0), np.dot(lam_t, fwd(f, dc0))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    cT = fwd(f, c0)
    _, grad = adj(oracle_mod.yield_seed(h.energies, cT)[0])
    scale = np.abs(grad).max()
    assert scale > 1e-5
    hstep = 1e-5
    for i in np.argsort(-np.abs(grad).ravel())[:6]:
        fp, fm = f.copy(), f.copy()
        fp.flat[i] += hstep
        fm.flat[i] -= hstep
        fd = (oracle_mod.ionization_yield(h.energies, fwd(fp, c0))[0]
              - oracle_mod.ionization_yield(h.energies, fwd(fm, c0))[0]) / (2 * hstep)
        assert abs(fd - grad.flat[i]) <= 1e-6 * scale, (i, fd, grad.flat[i])


def test_vector_potential_quadrature_matches_closed_form():
    """Step-wise 5-point Gauss-Legendre accumulation of A = -int E vs the
    closed-form integral of the sin^2 cos pulse, at every stage time."""
    p = wl.Pulse(0.05, 0.5, 10.0)
    dt = 0.01
    nst = wl.nsteps_for(p.duration, dt)
    a = wl.vector_potential_samples(p, dt, nst, "rk4")
    t = np.arange(nst) * dt
    exact = np.stack([wl.vector_potential_exact(p, t + s * dt) for s in (0.0, 0.5, 1.0)], axis=1)
    assert np.abs(a - exact).max() <= 1e-12 * np.abs(exact).max()
    mid = wl.vector_potential_samples(p, dt, nst, "taylor", "mid")[:, 0]
    assert np.abs(mid - wl.vector_potential_exact(p, t + 0.5 * dt)).max() <= 1e-12 * np.abs(exact).max()


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "paper_values.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_paper_sizing_formula():
    rows = [r for r in _golden() if r[0] == "sizing_doubles"]
    assert rows
    for _, nl, nb, val in rows:
        assert wl.sizing_doubles(int(nl), int(nb)) == int(val)


def test_paper_smallest_vector():
    for _, nl, nb, val in [r for r in _golden() if r[0] == "smallest_vector_doubles"]:
        assert wl.ground_state(int(nb) - 1, int(nl)).shape[1] == int(val)


def test_paper_equal_matvec_counts():
    rows = [r for r in _golden() if r[0] == "equal_matvecs"]
    assert len(rows) == 3
    for _, _m, per_step, dt, per_unit in rows:
        assert round(int(per_step) / float(dt)) == int(per_unit)


def test_generator_shapes_and_determinism():
    h1 = wl.hamiltonian(3, 50, 0)
    h2 = wl.hamiltonian(3, 50, 0)
    assert h1.energies.shape == (200,) and h1.dipole.shape == (3, 50, 50)
    assert np.array_equal(h1.dipole, h2.dipole)
    e = h1.energies.reshape(4, 50)
    assert e[0, 0] == -0.5 and np.all(e[:, 10:] > 0) and np.all(e[:, :10] < 0)
    assert abs(e[0, 10] - 0.5 * (math.pi / 200) ** 2) < 1e-18
    assert not np.array_equal(wl.hamiltonian(3, 50, 1).dipole, h1.dipole)


def test_workload_step_counts():
    assert wl.single_small().nsteps == 12567
    assert wl.nsteps_for(wl.Pulse(0.05, 0.5, 20).duration, 0.005) == 50266
    assert wl.nsteps_for(wl.Pulse(0.05, 0.5, 20).duration, 0.02) == 12567
    f = wl.piecewise_samples(wl.Pulse(0.05, 0.5, 10.0))
    assert f.shape == (2048,)
    g = wl.expand_piecewise(f[None], 16)
    assert g.shape == (1, 32768, 3)
    assert np.allclose(wl.collapse_piecewise(np.ones_like(g), 16), 48.0)


# ---- short-iterative Lanczos (Krylov) propagator

def _expm_steps(h, fk, dt, c0, gauge="length", q=None):
    v = cplx(c0)
    for f in fk:
        hk = dense_h_velocity(h.energies, q, f) if gauge == "velocity" else dense_h(h.energies, h.dipole, f)
        lam, w = np.linalg.eigh(hk)
        v = (w * np.exp(-1j * lam * dt)[None, :]) @ (w.conj().T @ v)
    return v


@pytest.mark.parametrize("gauge", ["length", "velocity"])
def test_lanczos_full_krylov_space_is_exact(oracle_mod, gauge):
    """m = dimension of the space: the Krylov step is exp(-i dt H_k) exactly."""
    h = wl.hamiltonian(1, 3, 2)
    q = wl.velocity_coupling(h.energies, h.dipole)
    rng = np.random.default_rng(3)
    c0 = wl.random_state(rng, h.nstates)[0]
    dt, fk = 0.3, stepwise_fields(12, 0.3) + 0.2
    blocks = q if gauge == "velocity" else h.dipole
    got = oracle_mod.lanczos(h.energies, blocks, h.nstates, dt, fk[None], c0, gauge=gauge)[0]
    ref = _expm_steps(h, fk, dt, c0, gauge, q)
    np.testing.assert_allclose(cplx(got), ref, rtol=0, atol=1e-12)


def test_lanczos_eigenstate_breakdown_gives_exact_phase(oracle_mod):
    """Field-free and c an eigenstate: the basis breaks down after one vector
    and the step is the exact phase exp(-i E dt)."""
    h = wl.hamiltonian(2, 12, 1)
    c0 = np.zeros(2 * h.nstates)
    c0[2 * 13] = 1.0                     # state 13: block 1, a bound level
    dt, nst = 0.7, 25
    got = oracle_mod.lanczos(h.energies, h.dipole, 10, dt, np.zeros((1, nst)), c0)[0]
    e = h.energies[13]
    assert abs(cplx(got)[13] - np.exp(-1j * e * dt * nst)) <= 1e-13
    assert np.abs(np.delete(cplx(got), 13)).max() == 0.0


def test_lanczos_converges_rapidly_with_krylov_dimension(oracle_mod):
    h = wl.hamiltonian(2, 20, 4)
    rng = np.random.default_rng(5)
    c0 = wl.random_state(rng, h.nstates)[0]
    dt, fk = 0.2, stepwise_fields(10, 0.2) + 0.3
    ref = _expm_steps(h, fk, dt, c0)
    errs = [np.abs(cplx(oracle_mod.lanczos(h.energies, h.dipole, m, dt, fk[None], c0)[0]) - ref).max()
            for m in (4, 8, 12)]
    assert errs[1] < 1e-3 * errs[0] and errs[2] < 1e-3 * errs[1] and errs[2] < 1e-11, errs


def test_lanczos_preserves_the_norm(oracle_mod):
    h = wl.hamiltonian(3, 15, 6)
    rng = np.random.default_rng(7)
    c0 = wl.random_state(rng, h.nstates)[0]
    fk = stepwise_fields(60, 0.1) + 0.1
    got = oracle_mod.lanczos(h.energies, h.dipole, 8, 0.1, fk[None], c0)[0]
    assert abs(np.linalg.norm(got) - 1.0) <= 1e-12


# ---- Runge-Kutta-Fehlberg 4(5)

def _dop853_reference(h, c0, pulse, t_final, gauge="length", q=None):
    from scipy.integrate import solve_ivp
    h0 = np.diag(h.energies)
    h1 = (dense_h_velocity(h.energies, q, 1.0) - h0) if gauge == "velocity" else dense_h(h.energies, h.dipole, 1.0) - h0
    sol = solve_ivp(lambda t, y: -1j * (h0 + float(pulse(t)) * h1) @ y, (0, t_final), cplx(c0).astype(complex),
                    method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[:, -1]


def test_rkf45_fifth_order_solution(oracle_mod):
    """The propagated solution -- the pair's fifth-order one, which the paper
    uses (Sec. 5.1) -- converges at order 5 against a tight DOP853 solve;
    stage samples in the wrong slots (planted by reversing them) lose the
    order."""
    h = wl.hamiltonian(1, 3, 2)
    c0 = wl.ground_state(1, 3)[0]
    pulse = wl.Pulse(0.8, 0.9, 2.0)
    ref = _dop853_reference(h, c0, pulse, pulse.duration)

    def err(nst, rev=False):
        dt = pulse.duration / nst
        f = wl.rkf45_samples(pulse, dt, nst)
        if rev:
            f = f[:, ::-1].copy()
        cT, _ = oracle_mod.rkf45(h.energies, h.dipole, dt, f[None], c0[None])
        return np.abs(cplx(cT[0]) - ref).max()

    e = [err(m) for m in (60, 120, 240)]
    assert 24.0 < e[0] / e[1] < 40.0 and 24.0 < e[1] / e[2] < 40.0, e
    bad = [err(m, True) for m in (60, 120, 240)]
    assert bad[1] / bad[2] < 5.0, bad


def test_rkf45_error_estimate_and_local_error(oracle_mod):
    """Over one step the embedded estimate |dt sum (b5 - b4) k| scales as
    dt^5 (the local error of the pair's fourth-order member), while the step
    taken -- the fifth-order member -- errs by O(dt^6): a falling fraction of
    the estimate."""
    h = wl.hamiltonian(1, 4, 3)
    rng = np.random.default_rng(2)
    c0 = wl.random_state(rng, h.nstates)[0]
    pulse = wl.Pulse(1.2, 0.8, 1.0)
    t0 = 0.37 * pulse.duration
    shifted = lambda t: pulse(np.asarray(t) + t0)  # noqa: E731
    est, true = [], []
    for dt in (0.1, 0.05, 0.025):
        f = np.asarray(shifted(np.array(wl.RKF45_SLOTS) * dt))[None, None, :]
        cT, e = oracle_mod.rkf45(h.energies, h.dipole, dt, f, c0[None])
        ref = _dop853_reference(h, c0, shifted, dt)
        est.append(e[0, 0])
        true.append(np.linalg.norm(cplx(cT[0]) - ref))
    assert 24.0 < est[0] / est[1] < 40.0 and 24.0 < est[1] / est[2] < 40.0, est
    assert 48.0 < true[0] / true[1] < 80.0 and 48.0 < true[1] / true[2] < 80.0, true
    frac = [b / a for a, b in zip(est, true)]
    assert frac[0] > frac[1] > frac[2] and frac[2] < 0.1, (est, true)
