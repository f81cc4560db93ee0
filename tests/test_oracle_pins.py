"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula as its expectation: each
one compares the oracle with a closed form, an invariant, a brute-force
definition in exact rational arithmetic, or a value the paper prints.
Runs on the CPU only.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

C1 = dict(n_cells=1024, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=4.0,
          rho_kind=0, rho_amp=1.0, capacity=200000)


def _tube(oracle_mod, **kw):
    c = dict(C1)
    c.update(kw)
    return oracle_mod.OracleTube(c)


# --------------------------------------------------------------------------
# P1  eq. (1): a test particle in a uniform field follows hyperbolic motion
# --------------------------------------------------------------------------
def _hyperbolic_run(oracle_mod, dtdz, T):
    N, L = 1024, 10.0
    o = oracle_mod
    t = o.OracleTube(n_cells=N, length=L, radius=1.0, dt_over_dz=dtdz, q_over_m=-1.0, ppc=1.0,
                     flags=o.NO_AUTO_INJECT | o.FREEZE_FIELDS, capacity=4)
    E0 = -2.0
    dz = L / N
    dt = dtdz * dz
    K = -1.0 * dt * E0                      # (q/m) dt E0 > 0: electrons pushed to +z
    x0 = 2.0
    t.inject([x0], [-0.5 * K])              # at rest at t = 0: u(-dt/2) = -alpha dt/2
    t.ez[:] = E0
    n = int(round(T / dt))
    us = []
    for _ in range(n):
        t.step(1)
        us.append(t.u[0])
    alpha = 2.0
    z_exact = (math.sqrt(1.0 + (alpha * n * dt) ** 2) - 1.0) / alpha
    z_num = (t.x[0] - x0) * dz
    return np.array(us), K, z_num, z_exact, dt, n


def test_p1_momentum_sequence_exact(oracle_mod):
    us, K, _, _, _, n = _hyperbolic_run(oracle_mod, 0.5, 1.0)
    expect = (np.arange(n) + 0.5) * K       # dyadic K: every sum is exact
    assert np.array_equal(us, expect)


def test_p1_hyperbolic_trajectory_second_order(oracle_mod):
    _, _, zn1, ze1, dt1, _ = _hyperbolic_run(oracle_mod, 0.5, 2.0)
    _, _, zn2, ze2, dt2, _ = _hyperbolic_run(oracle_mod, 0.25, 2.0)
    e1, e2 = abs(zn1 - ze1), abs(zn2 - ze2)
    alpha = 2.0
    # gamma - 1 = alpha * dz_travelled (work-energy for uniform E): error bounded by alpha dt
    assert alpha * e1 <= alpha * dt1
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_gather_linear_field_exact(oracle_mod):
    """Linear interpolation of a linear E_z reproduces it; clamped beyond the end faces."""
    o = oracle_mod
    N, L = 64, 8.0
    t = o.OracleTube(n_cells=N, length=L, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=1.0,
                     flags=o.NO_AUTO_INJECT | o.FREEZE_FIELDS, capacity=64)
    xs = np.array([0.25, 0.5, 0.75, 3.0, 3.3, 17.625, 40.1, 62.9, 63.5, 63.75])
    t.inject(xs, np.zeros_like(xs))
    dz = L / N
    E0, E1 = -0.7, 0.3
    t.ez[:] = E0 + E1 * (np.arange(N) + 0.5) * dz
    t.step(1)
    qmdt = -1.0 * 0.5 * dz
    xc = np.clip(xs, 0.5, N - 0.5)
    expect = qmdt * (E0 + E1 * xc * dz)
    np.testing.assert_allclose(t.u, expect, rtol=1e-13, atol=1e-16)


# --------------------------------------------------------------------------
# P2  eq. (4) with its boundary conditions: closed form of the discrete problem
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,L,R,A", [(1024, 10.0, 1.0, 1.0), (512, 3.0, 0.7, 2.5),
                                     (2048, 40.0, 1.0, 0.3), (96, 5.0, 2.0, 1.0)])
def test_p2_poisson_closed_form(oracle_mod, N, L, R, A):
    t = _tube(oracle_mod, n_cells=N, length=L, radius=R, rho_amp=A)
    dz = L / N
    lam = 2.0 * math.asinh(dz / (2.0 * R))   # cosh(lam) = 1 + dz^2/(2R^2)
    i = np.arange(N + 1)
    rho = -A
    phi = -4.0 * math.pi * rho * R * R * (1.0 - np.cosh(lam * (N - i)) / math.cosh(lam * N))
    scale = np.abs(phi).max()
    # backward-stable solve of a system with condition number ~ (R/dz)^2
    tol = 10 * np.finfo(float).eps * (R / dz) ** 2
    assert np.abs(t.phi - phi).max() <= tol * scale
    np.testing.assert_allclose(t.er, phi / R, rtol=0, atol=tol * scale / R)
    ez = -(phi[1:] - phi[:-1]) / dz
    np.testing.assert_allclose(t.ez, ez, rtol=0, atol=1e-9 * np.abs(ez).max())
    # continuum limit of the surface field: E_z(0) = 4 pi rho_GJ R tanh(L/R)
    e0 = 4.0 * math.pi * rho * R * math.tanh(L / R)
    assert abs(t.ez[0] - e0) <= 2.0 * (dz / R) * abs(e0)


def test_poisson_mirror_images(oracle_mod):
    """phi'(L) = 0 is the symmetric half of a tube twice as long with the particles
    mirrored about x = N and phi = 0 at both ends.  Solve that doubled problem
    densely with explicit image particles and compare the left half."""
    rng = np.random.default_rng(11)
    N, L, R = 64, 4.0, 0.6
    t = _tube(oracle_mod, n_cells=N, length=L, radius=R, rho_kind=1, kappa=0.15, r_star=2.0,
              ppc=3.0)
    x = np.concatenate([rng.uniform(0, N, 150), rng.uniform(N - 1, N, 40)])
    t.inject(x, np.zeros_like(x))
    dz = L / N
    qm = t.rho_gj[0] * dz / 3.0
    M = 2 * N
    xa = np.concatenate([x, 2 * N - x])               # particles and their images
    w = np.zeros(M + 1)
    for i in range(M + 1):
        w[i] = np.clip(1 - np.abs(xa - i), 0, None).sum()
    rg = np.concatenate([t.rho_gj, t.rho_gj[-2::-1]])  # background, mirrored
    rho = qm * w / dz
    A = np.zeros((M - 1, M - 1))
    for r in range(M - 1):
        A[r, r] = -2.0 / dz ** 2 - 1.0 / R ** 2
        if r > 0:
            A[r, r - 1] = 1.0 / dz ** 2
        if r < M - 2:
            A[r, r + 1] = 1.0 / dz ** 2
    phi = np.zeros(M + 1)
    phi[1:M] = np.linalg.solve(A, -4 * np.pi * (rho[1:M] - rg[1:M]))
    assert np.abs(t.phi - phi[:N + 1]).max() <= 1e-11 * np.abs(phi).max()


# --------------------------------------------------------------------------
# Maxwell, eq. (3): vacuum dispersion of the leap-frog scheme on this grid
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [0, 3, 17])
def test_maxwell_vacuum_dispersion(oracle_mod, m):
    """For one standing mode (E_r ~ sin kz, B_phi and E_z ~ cos kz, k N dz = (m+1/2) pi,
    matching E_r = 0 at the star and the mirror at the top) the step is a 3x3 map.
    Its eigenvalues must be 1 (the static, Gauss-constrained mode) and exp(+-i theta)
    with sin^2(theta/2) = (dt/dz)^2 sin^2(k dz/2) + (dt/2R)^2, the discrete form of
    the wave-guide relation w^2 = k^2 + 1/R^2 that eq. (3) implies in vacuum."""
    o = oracle_mod
    N, L, R, dtdz = 128, 4.0, 0.8, 0.5
    dz = L / N
    dt = dtdz * dz
    k = (m + 0.5) * math.pi / (N * dz)
    sr = np.sin(k * np.arange(N + 1) * dz)
    cf = np.cos(k * (np.arange(N) + 0.5) * dz)
    cols = []
    for unit in range(3):
        t = o.OracleTube(n_cells=N, length=L, radius=R, dt_over_dz=dtdz, q_over_m=-1.0, ppc=1.0,
                         flags=o.NO_AUTO_INJECT, capacity=1)
        t.er[:] = sr if unit == 0 else 0.0
        t.b[:] = cf if unit == 1 else 0.0
        t.ez[:] = cf if unit == 2 else 0.0
        t.step(1)
        a = np.dot(t.er, sr) / np.dot(sr, sr)
        bb = np.dot(t.b, cf) / np.dot(cf, cf)
        zz = np.dot(t.ez, cf) / np.dot(cf, cf)
        # the mode shape must be preserved exactly (up to rounding)
        assert np.abs(t.er - a * sr).max() < 1e-13
        assert np.abs(t.b - bb * cf).max() < 1e-13
        assert np.abs(t.ez - zz * cf).max() < 1e-13
        cols.append([a, bb, zz])
    M = np.array(cols).T
    ev = np.linalg.eigvals(M)
    s2 = dtdz ** 2 * math.sin(k * dz / 2) ** 2 + (dt / (2 * R)) ** 2
    theta = 2 * math.asin(math.sqrt(s2))
    expect = np.array([1.0, np.exp(1j * theta), np.exp(-1j * theta)])
    got = sorted(ev, key=lambda z: (round(z.imag, 12), z.real))
    want = sorted(expect, key=lambda z: (round(z.imag, 12), z.real))
    np.testing.assert_allclose(got, want, atol=1e-12)
    assert abs(np.linalg.det(M) - 1.0) < 1e-12


# --------------------------------------------------------------------------
# P3  vacuum stationarity: the Poisson field is a fixed point of eq. (3)
# --------------------------------------------------------------------------
def test_p3_vacuum_stationary(oracle_mod):
    o = oracle_mod
    t = _tube(o, flags=o.NO_AUTO_INJECT)
    ez0, er0 = t.ez.copy(), t.er.copy()
    t.step(2000)
    emax = max(np.abs(ez0).max(), np.abs(er0).max())
    assert np.abs(t.b).max() <= 1e-12 * emax
    assert np.abs(t.ez - ez0).max() <= 1e-12 * emax
    assert np.abs(t.er - er0).max() <= 1e-12 * emax


# --------------------------------------------------------------------------
# P4  charge conservation of the deposit: exact integer continuity
# --------------------------------------------------------------------------
def _continuity_check(t, steps):
    N = t.N
    for _ in range(steps):
        w0 = t.weights()
        t.step(1)
        w1 = t.weights()
        j = t.j
        resid = (w1[1:N] - w0[1:N]) + (j[1:N] - j[0:N - 1])
        assert not resid.any()


def test_p4_continuity_c1(oracle_mod):
    t = _tube(oracle_mod)
    _continuity_check(t, 300)


def test_p4_continuity_warm_frame_drag(oracle_mod):
    rng = np.random.default_rng(3)
    N = 256
    t = _tube(oracle_mod, n_cells=N, rho_kind=1, kappa=0.15, r_star=10.0, q_over_m=-50.0,
              ppc=8.0)
    x = np.sort(rng.uniform(0, N, 8 * N))
    u = rng.uniform(-3, 40, 8 * N)
    t.inject(x, u)
    _continuity_check(t, 60)
    assert t.counters["n_exit"] > 0


# --------------------------------------------------------------------------
# P5  discrete Gauss law: small at t = 0, drift bounded by rounding
# --------------------------------------------------------------------------
def test_p5_gauss_initial_with_particles(oracle_mod):
    rng = np.random.default_rng(0)
    t = _tube(oracle_mod)
    N = t.N
    x = rng.uniform(0, N, 4 * N)
    t.inject(x, np.zeros_like(x))
    _, g = t.gauss()
    eps = np.finfo(float).eps
    assert g <= 10 * eps * (1.0 / t.dz) ** 2


def test_p5_gauss_drift_c1(oracle_mod):
    t = _tube(oracle_mod)
    G0, _ = t.gauss()
    eps = np.finfo(float).eps
    norm = 4 * math.pi * np.abs(t.rho_gj).max()
    for n in (500, 1000, 2000):
        t.step(n - t.counters["step"])
        G, _ = t.gauss()
        drift = np.abs(G - G0).max() / norm
        assert drift <= 10 * eps * (1.0 / t.dz) * math.sqrt(n), (n, drift)


# --------------------------------------------------------------------------
# P6  brute force on 8 cells in exact rational arithmetic
# --------------------------------------------------------------------------
def _q(x, P):
    """Fixed-point position: cell + round-half-even(2^P frac) / 2^P, exact."""
    f = Fraction(x)
    c = math.floor(f)
    return c + Fraction(round((f - c) * 2 ** P), 2 ** P)


def _hat(X, k):
    return max(Fraction(0), 1 - abs(X - k))


def test_p6_brute_force_8_cells(oracle_mod):
    o = oracle_mod
    P = 32
    N, L, R = 8, 1.0, 0.5
    t = o.OracleTube(n_cells=N, length=L, radius=R, dt_over_dz=0.5, q_over_m=-1.0, ppc=2.0,
                     capacity=64)
    xs = [0.25, 1.5, 2.0, 2.75, 3.125, 4.5, 5.0625, 6.5]
    us = [0.0, 0.5, -0.25, 2.0, -1.0, 0.75, 3.0, -0.5]
    t.inject(xs, us)
    # rho: hat functions (weights) of the initial particles
    W = t.weights()
    for i in range(N + 1):
        wi = sum(_hat(_q(x, P), i) for x in xs) * 2 ** P
        assert wi == W[i]
    ez0, er0, b0 = t.ez.copy(), t.er.copy(), t.b.copy()
    t.step(1)
    assert t.counters["n_exit"] == 0 and t.counters["n_absorb"] == 0
    new = list(t.x[:len(xs)])
    # J from the cumulative hat weight left of each face
    for i in range(N):
        Ji = 0
        for xo, xn in zip(xs, new):
            Co = sum(_hat(_q(xo, P), kk) for kk in range(0, i + 1))
            Cn = sum(_hat(_q(xn, P), kk) for kk in range(0, i + 1))
            Ji += (Co - Cn) * 2 ** P
        assert Ji == t.j[i], i
    # one leap-frog update of eq. (3) in exact arithmetic from the old fields
    dz = Fraction(L) / N
    dtdz = Fraction(1, 2)
    dt = dtdz * dz
    dtR = dt / Fraction(R)
    rho0 = Fraction(t.rho_gj[0])
    qm = rho0 * dz / 2
    pi = Fraction(math.pi)
    c4 = 4 * pi * qm / 2 ** P
    B = [Fraction(b0[i]) - (dtdz * (Fraction(er0[i + 1]) - Fraction(er0[i])) + dtR * Fraction(ez0[i]))
         for i in range(N)]
    Er = [Fraction(0)] + [Fraction(er0[i]) - dtdz * (B[i] - B[i - 1]) for i in range(1, N)] + \
         [Fraction(er0[N]) + 2 * dtdz * B[N - 1]]
    Ez = [Fraction(ez0[i]) + dtR * B[i] - c4 * int(t.j[i]) for i in range(N)]
    for i in range(N):
        assert math.isclose(float(B[i]), t.b[i], rel_tol=1e-14, abs_tol=1e-15)
        assert math.isclose(float(Ez[i]), t.ez[i], rel_tol=1e-14, abs_tol=1e-15)
    for i in range(N + 1):
        assert math.isclose(float(Er[i]), t.er[i], rel_tol=1e-14, abs_tol=1e-15)
    # surface field from the node-0 Gauss law over the half cell, and the SCLF count
    W0 = sum(_hat(_q(xn, P), 0) for xn in new) * 2 ** P
    assert W0 == t.counters["w0"]
    es = Fraction(t.ez[0]) - 4 * pi * (qm * W0 / 2 ** P - rho0 * dz / 2)
    assert math.isclose(float(es), t.counters["e_surf"], rel_tol=1e-13)
    ratio = es / (4 * pi * qm)
    ninj = math.floor(ratio) if ratio > 0 else 0
    assert ninj == t.counters["last_ninj"]
    assert t.n == len(xs) + ninj


def test_first_step_injection_from_closed_form(oracle_mod):
    """C1: the first injection count follows from the closed-form Poisson field."""
    t = _tube(oracle_mod)
    N, dz, R, rho = 1024, 10.0 / 1024, 1.0, -1.0
    lam = 2.0 * math.asinh(dz / (2.0 * R))   # cosh(lam) = 1 + dz^2/(2R^2)
    phi1 = -4.0 * math.pi * rho * R * R * (1.0 - math.cosh(lam * (N - 1)) / math.cosh(lam * N))
    ez_half = -phi1 / dz
    qm = rho * dz / 4.0
    es = ez_half + 4.0 * math.pi * rho * dz / 2.0
    t.step(1)
    assert math.isclose(t.counters["e_surf"], es, rel_tol=1e-11)
    assert t.counters["last_ninj"] == math.floor(es / (4 * math.pi * qm)) == 409


# --------------------------------------------------------------------------
# P7 / P8  SCLF physics (sec. 2-3): gamma behind the front and E(0) -> 0
# --------------------------------------------------------------------------
def test_p7_p8_sclf_long_tube(oracle_mod):
    """C1-long (L = 40R, same dz): once the front passes 30R the mean gamma over
    5R..25R is within 20% of the steady reduced-model value
    gamma* = (sqrt(9 + 8 a^2) - 1)/2, a^2 = 4 pi |rho_GJ| |q/m| R^2, whose large-a limit
    sqrt(2) a is the flat-space maximum of Tables 1-2.  The surface field vanishes
    (E(0) -> 0) and electrons pile up in a cloud at the base."""
    t = _tube(oracle_mod, n_cells=4096, length=40.0, capacity=400000)
    qm = t.macro_charge
    es_hist = []
    for s in range(7000):
        t.step(1)
        c = t.counters
        r = c["e_surf"] / (4 * math.pi * qm)
        if r > 0:
            assert 0.0 <= r - c["last_ninj"] < 1.0
        if s >= 6000:
            es_hist.append(c["e_surf"])
    x, u = t.x, t.u
    z = x * t.dz
    assert z.max() > 30.0
    gam = np.sqrt(1 + u * u)
    m = (z >= 5) & (z <= 25)
    a2 = 4 * math.pi
    gstar = (math.sqrt(9 + 8 * a2) - 1) / 2
    assert abs(gam[m].mean() / gstar - 1) < 0.2
    e0 = abs(oracle_mod.OracleTube(dict(t.cfg)).ez[0])
    assert abs(np.mean(es_hist)) < 0.05 * e0
    w = t.weights()
    rho = qm * w / 2.0 ** 32 / t.dz
    assert abs(rho[1]) > abs(t.rho_gj[1])


# --------------------------------------------------------------------------
# P10  the paper's printed gamma_max values (Tables 1 and 2)
# --------------------------------------------------------------------------
def _gstar(a):
    return (math.sqrt(9 + 8 * a * a) - 1) / 2


def test_p10_tables_gamma_max():
    rows = []
    with open(os.path.join(GOLDEN, "table1_table2_gamma_max.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                tab, R, wp, g = line.split()
                rows.append((tab, float(R), float(wp), float(g)))
    assert len(rows) == 8
    for tab, R, wp, g in rows:
        a = wp * R                       # a = omega_p R / c, c = 1
        gm = math.sqrt(2) * a
        # the printed values are loose ("~"): Table 2 prints ~7000 for 7778 and
        # ~15 for 15.56, so 12% for the large entries and 0.6 for the small ones
        tol = 0.12 * g if g >= 1000 else 0.6
        assert abs(gm - g) <= tol, (tab, R, wp, gm, g)
        # the reduced-model steady value tends to the printed law for large a
        if a > 100:
            assert abs(_gstar(a) - gm) / gm < 1e-3


# --------------------------------------------------------------------------
# background density, boundaries, diagnostics
# --------------------------------------------------------------------------
def test_rho_gj_frame_drag_eq7(oracle_mod):
    """eq. (7) with r_g/R_* = 0.4 gives omega/Omega = (2/5)(0.4)/eta^3 = 0.16/eta^3;
    replacing Omega by Omega - omega scales the flat density by 1 - omega/Omega."""
    N, L, Rs = 200, 10.0, 10.0
    t = _tube(oracle_mod, n_cells=N, length=L, rho_kind=1, kappa=0.4 * 2 / 5, r_star=Rs, rho_amp=1.7)
    z = np.arange(N + 1) * (L / N)
    omega = 2.0 / 5.0 * 0.4 * (Rs / (Rs + z)) ** 3
    np.testing.assert_allclose(t.rho_gj, -1.7 * (1 - omega), rtol=1e-14)


def test_rho_gj_knots(oracle_mod):
    rng = np.random.default_rng(1)
    K = 9
    th = rng.uniform(0.5, 1.5, K)
    N, L = 64, 10.0
    t = _tube(oracle_mod, n_cells=N, length=L, rho_kind=2, kappa=0.15, r_star=10.0, knots=th)
    z = np.arange(N + 1) * (L / N)
    fd = 1 - 0.15 / (1 + z / 10.0) ** 3
    theta = np.interp(z, np.linspace(0, L, K), th)
    np.testing.assert_allclose(t.rho_gj, -theta * fd, rtol=1e-13)


def test_rho_gj_gr_reduces_to_frame_drag(oracle_mod):
    """Eq. (6) with i = 0 and r_g = 0 (alpha = 1, no sin i term) is the
    frame-dragging density, bit for bit."""
    kw = dict(n_cells=128, length=10.0, kappa=0.15, r_star=7.0, rho_amp=1.3)
    a = _tube(oracle_mod, rho_kind=1, **kw)
    b = _tube(oracle_mod, rho_kind=3, incl=0.0, theta_star=0.0094, rg_over_rstar=0.0, **kw)
    assert np.array_equal(a.rho_gj, b.rho_gj)


def test_rho_gj_gr_redshift(oracle_mod):
    """alpha = (1 - r_g/r)^(1/2): with kappa = 0 and i = 0 the density is -A/alpha,
    so rho^2 (1 - g/eta) = A^2 at every node, and at the surface with
    r_g/R_* = 0.4 the magnitude is A/sqrt(0.6)."""
    N, L, Rs, g = 100, 20.0, 5.0, 0.4
    t = _tube(oracle_mod, n_cells=N, length=L, rho_kind=3, kappa=0.0, r_star=Rs, rho_amp=2.0,
              incl=0.0, rg_over_rstar=g)
    eta = 1 + np.arange(N + 1) * (L / N) / Rs
    np.testing.assert_allclose(t.rho_gj ** 2 * (1 - g / eta), 4.0, rtol=1e-14)
    assert abs(abs(t.rho_gj[0]) - 2.0 / np.sqrt(0.6)) < 1e-14 * 4
    assert np.all(np.diff(np.abs(t.rho_gj)) < 0)        # the redshift weakens with height


def test_rho_gj_gr_sin_i_term(oracle_mod):
    """The inclination term of eq. (6) grows as (r/R_*)^(1/2) and scales with
    theta_* tan(i) cos(varphi); near the star it is much smaller than the cos(i)
    term for the paper's standard pulsar (theta_p = 0.014, theta_* = 0.67 theta_p,
    i = 0.5 rad), as the paper states."""
    N, L, Rs = 64, 30.0, 10.0
    ts = 0.67 * 0.014
    kw = dict(n_cells=N, length=L, kappa=0.15, r_star=Rs, rho_amp=1.0, rg_over_rstar=0.0)
    base = _tube(oracle_mod, rho_kind=3, incl=0.0, theta_star=ts, **kw).rho_gj
    d5 = _tube(oracle_mod, rho_kind=3, incl=0.5, theta_star=ts, **kw).rho_gj - base
    d1 = _tube(oracle_mod, rho_kind=3, incl=0.1, theta_star=ts, **kw).rho_gj - base
    dphi = _tube(oracle_mod, rho_kind=3, incl=0.5, theta_star=ts, cos_phi=-0.5, **kw).rho_gj - base
    eta = 1 + np.arange(N + 1) * (L / N) / Rs
    prof = d5 / np.sqrt(eta)
    np.testing.assert_allclose(prof, prof[0], rtol=1e-9)           # proportional to eta^(1/2)
    np.testing.assert_allclose(d1 / d5, np.tan(0.1) / np.tan(0.5), rtol=1e-8)
    np.testing.assert_allclose(dphi / d5, -0.5, rtol=1e-8)
    assert abs(d5[0] / base[0]) < 0.01                           # sin(i) term << cos(i) term at the surface


def _uniform_beam(N, n_per_cell, u0):
    x = (np.arange(N * n_per_cell) + 0.5) / n_per_cell
    return x, np.full(len(x), u0)


def test_b_steady_init_equals_4pi_r_j(oracle_mod):
    """Steady start of eq. (3): dE_z/dt = B/R - 4 pi j = 0 gives B_phi = 4 pi R j.
    A uniform beam of n electrons per cell at u0 carries j = rho v with
    rho = q_m n / dz and v = u0 / sqrt(1 + u0^2)."""
    o = oracle_mod
    N, n, u0, R = 64, 8, 3.0, 0.7
    kw = dict(n_cells=N, length=N / 50.0, radius=R, q_over_m=-40.0, ppc=8.0, capacity=N * n + 16,
              flags=o.NO_AUTO_INJECT)
    t = _tube(oracle_mod, flags=o.NO_AUTO_INJECT | o.B_STEADY_INIT, **{k: v for k, v in kw.items() if k != "flags"})
    x, u = _uniform_beam(N, n, u0)
    t.inject(x, u)
    dz = kw["length"] / N
    qm = -1.0 * dz / kw["ppc"]                   # rho_GJ(0) dz / ppc with rho_GJ = -1
    v = u0 / np.sqrt(1 + u0 * u0)
    want = 4 * np.pi * R * (qm * n / dz) * v
    inner = t.b[2:N - 2]
    np.testing.assert_allclose(inner, want, rtol=1e-8)
    assert np.all(t.j == 0)


def test_b_steady_init_starts_steady(oracle_mod):
    """With the steady B the first step leaves E_z nearly unchanged in the
    interior; without it the beam's current drives E_z at once."""
    o = oracle_mod
    N, n = 128, 8
    x, u = _uniform_beam(N, n, 20.0)
    dez = []
    for flags in (o.NO_AUTO_INJECT, o.NO_AUTO_INJECT | o.B_STEADY_INIT):
        t = _tube(oracle_mod, n_cells=N, length=N / 50.0, q_over_m=-40.0, ppc=8.0, capacity=N * n + 16,
                  flags=flags)
        t.inject(x, u)
        e0 = t.ez.copy()
        t.step(1)
        dez.append(np.abs(t.ez - e0)[4:N - 4].max())
    assert dez[1] < 1e-3 * dez[0], dez


def test_exit_and_absorb(oracle_mod):
    o = oracle_mod
    N = 32
    t = o.OracleTube(n_cells=N, length=4.0, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=1.0,
                     flags=o.NO_AUTO_INJECT | o.FREEZE_FIELDS, capacity=8)
    t.inject([N - 0.1, 0.1, 10.0], [10.0, -10.0, 0.0])
    t.ez[:] = 0.0
    t.step(1)
    c = t.counters
    assert c["n_exit"] == 1 and c["n_absorb"] == 1 and t.n == 1
    assert t.exit_gamma_sum() == round(math.sqrt(101.0) * 2 ** 32) / 2 ** 32


def test_order_independence(oracle_mod):
    rng = np.random.default_rng(5)
    N = 128
    x = rng.uniform(0, N, 2000)
    u = rng.uniform(-2, 30, 2000)
    res = []
    for perm in (np.arange(2000), rng.permutation(2000)):
        t = _tube(oracle_mod, n_cells=N, q_over_m=-20.0, ppc=16.0, rho_kind=1, kappa=0.15)
        t.inject(x[perm], u[perm])
        t.step(40)
        res.append((t.ez.copy(), t.er.copy(), t.b.copy(), t.counters["exit_sum_lo"],
                    np.sort(t.x)))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_profile_brute_force(oracle_mod):
    t = _tube(oracle_mod)
    t.step(600)
    nb = 16
    cnt, lo, hi, mn, mx = t.profile(nb)
    x, u = t.x, t.u
    g = np.sqrt(1 + u * u) * np.where(u < 0, -1, 1)
    b = np.clip((x * nb / t.N).astype(int), 0, nb - 1)
    for k in range(nb):
        sel = g[b == k]
        assert cnt[k] == sel.size
        if sel.size:
            mean = oracle_mod.i128_to_float(lo[k], hi[k]) / 2 ** 32 / cnt[k]
            assert math.isclose(mean, sel.mean(), rel_tol=1e-9)
            assert mn[k] == sel.min() and mx[k] == sel.max()
