"""Pins of the oracle's full-GR step (the lapse alpha in Maxwell's equations and
the equation of motion, GR_ALPHA) against closed forms and invariants.

The paper names these corrections after eqs. (6)-(7) without writing them out;
the oracle header states the reading.  What pins it, on the CPU:
  * r_g = 0: every factor is 1 and the step is the flat one, bit for bit;
  * a test particle in a static uniform E_z keeps its redshifted energy
    alpha gamma - (q/m) E_0 z, to second order in dt;
  * free radial motion (E_z = 0) turns around where alpha(z) gamma = alpha_0 gamma_0
    (closed form) and falls back to the star with its launch speed;
  * the discrete Gauss law alpha_i dE_z/dz + E_r/R = 4 pi (alpha_i lambda_i - rho_GJ,i)
    holds at t = 0 and is kept to rounding while the beam runs;
  * the Poisson start in vacuum is a fixed point of the update (static fields);
  * the surface field of the SCLF rule is second-order accurate in dz;
  * a field pulse in vacuum converges at second order in dz, which needs the lapse
    where the staggered grid puts each field (faces for B and E_z, nodes for E_r).
"""
import math

import numpy as np
import pytest

G, RSTAR = 0.4, 10.0          # r_g / R_* of the paper's standard star, R_* = 10 R


def _alpha(z):
    return np.sqrt(1.0 - G / (1.0 + z / RSTAR))


def _gamma(u):
    return np.sqrt(1.0 + np.asarray(u) ** 2)


def _gr_tube(o, **kw):
    c = dict(n_cells=1024, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=4.0,
             rho_kind=o.RHO_GR, rho_amp=1.0, kappa=0.15, r_star=RSTAR, incl=0.1, theta_star=0.67 * 0.014,
             cos_phi=1.0, rg_over_rstar=G, flags=o.GR_ALPHA, capacity=200000)
    c.update(kw)
    return o.OracleTube(c)


def _state(t):
    return (t.x.copy(), t.u.copy(), t.ez.copy(), t.er.copy(), t.b.copy(), t.j.copy(),
            {k: v for k, v in t.counters.items()})


@pytest.mark.parametrize("warm", [False, True])
def test_gr_with_zero_rg_is_the_flat_step(oracle_mod, warm):
    """With r_g = 0, alpha = 1 and alpha' = 0: the GR step equals the flat step bit for bit
    (cold SCLF start, and a warm random load with the steady B start)."""
    o = oracle_mod
    runs = []
    for flags in (o.GR_ALPHA, 0):
        kw = dict(rho_kind=o.RHO_FRAME_DRAG, rg_over_rstar=0.0, flags=flags | (o.B_STEADY_INIT if warm else 0))
        t = _gr_tube(o, **kw)
        if warm:
            rng = np.random.default_rng(3)
            x = np.sort(rng.uniform(0.0, t.N, 20000))
            t.inject(x, rng.uniform(-2.0, 30.0, len(x)))
        t.step(300)
        runs.append(_state(t))
    for a, b in zip(*runs):
        if isinstance(a, dict):
            assert a == b
        else:
            assert np.array_equal(a, b)


def _energy_drift(o, dtdz, T=20.0):
    """max |eps_n - eps_1| / eps_1 of eps = alpha(z) gamma - (q/m) E0 z over the time T,
    gamma centred at the integer time from the two half-step momenta."""
    N, L, qm, E0 = 4000, 100.0, -1.0, -0.3
    t = o.OracleTube(n_cells=N, length=L, radius=1.0, dt_over_dz=dtdz, q_over_m=qm, ppc=1.0,
                     flags=o.NO_AUTO_INJECT | o.FREEZE_FIELDS | o.GR_ALPHA, capacity=4,
                     rg_over_rstar=G, r_star=RSTAR)
    dz = L / N
    t.inject([40.0], [2.0])
    t.ez[:] = E0
    steps = int(round(T / (dtdz * dz)))
    xs, us = [], []
    for _ in range(steps + 1):
        t.step(1)
        xs.append(t.x[0])
        us.append(t.u[0])
    xs, us = np.array(xs), np.array(us)
    z = xs[:-1] * dz                             # x^n, n = 1 .. steps
    gam = 0.5 * (_gamma(us[:-1]) + _gamma(us[1:]))
    eps = _alpha(z) * gam - qm * E0 * z
    return np.abs(eps - eps[0]).max() / eps[0], xs[-1] * dz


def test_gr_redshifted_energy_second_order(oracle_mod):
    """A test particle in a static uniform E_z = E_0 under gravity: du/dt = alpha (q/m) E_0
    - gamma alpha alpha', dz/dt = alpha^2 v keeps alpha gamma - (q/m) E_0 z; the leap-frog
    keeps it to O(dt^2) (halving dt quarters the drift)."""
    d1, z1 = _energy_drift(oracle_mod, 0.4)
    d2, z2 = _energy_drift(oracle_mod, 0.2)
    assert z1 > 10.0 and abs(z1 - z2) < 0.01 * z1        # the same path, far up the tube
    assert d2 < 1e-6
    assert 3.0 < d1 / d2 < 5.0, (d1, d2)


def test_gr_free_fall_turning_point(oracle_mod):
    """E_z = 0: a particle launched up from the surface with u_0 turns where
    alpha(z) = alpha_0 gamma_0, i.e. at eta = g / (1 - (alpha_0 gamma_0)^2), and is
    absorbed by the star with its launch speed."""
    o = oracle_mod
    N, L, u0 = 2000, 20.0, 0.3
    t = o.OracleTube(n_cells=N, length=L, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=1.0,
                     flags=o.NO_AUTO_INJECT | o.FREEZE_FIELDS | o.GR_ALPHA, capacity=4,
                     rg_over_rstar=G, r_star=RSTAR)
    dz = L / N
    t.inject([0.0], [u0])
    t.ez[:] = 0.0
    zmax, ulast = 0.0, u0
    for _ in range(20000):
        t.step(1)
        if t.counters["n_alive"] == 0:
            break
        zmax = max(zmax, t.x[0] * dz)
        ulast = t.u[0]
    assert t.counters["n_absorb"] == 1
    e0 = _alpha(0.0) * _gamma(u0)
    zt = (G / (1.0 - e0 ** 2) - 1.0) * RSTAR
    assert abs(zmax - zt) <= 2e-3 * zt, (zmax, zt)
    assert abs(abs(ulast) - u0) <= 2e-3 * u0, (ulast, u0)


def test_gr_gauss_law_initial_and_kept(oracle_mod):
    """The GR Poisson start satisfies the discrete GR Gauss law to rounding, and the
    alpha-weighted leap-frog with the charge-conserving deposit keeps it while the SCLF
    beam rises (the same bounds as in flat space)."""
    t = _gr_tube(oracle_mod)
    rng = np.random.default_rng(1)
    t.inject(rng.uniform(0.0, t.N, 4 * t.N), np.zeros(4 * t.N))
    G0, g0 = t.gauss()
    eps = np.finfo(float).eps
    assert g0 <= 10 * eps * (1.0 / t.dz) ** 2
    norm = 4 * math.pi * np.abs(t.rho_gj).max()
    for n in (300, 1000):
        t.step(n - t.counters["step"])
        G1, _ = t.gauss()
        drift = np.abs(G1 - G0).max() / norm
        assert drift <= 10 * eps * (1.0 / t.dz) * math.sqrt(n), (n, drift)
    assert t.counters["n_injected"] > 0 and np.abs(t.b).max() > 0


def test_gr_vacuum_start_is_static(oracle_mod):
    """No particles: E_z = -dPhi/dz and E_r = Phi/(alpha R) from the GR Poisson start are
    a fixed point of the alpha-weighted update (B stays 0 up to rounding)."""
    o = oracle_mod
    t = _gr_tube(o, flags=o.GR_ALPHA | o.NO_AUTO_INJECT)
    ez0, er0 = t.ez.copy(), t.er.copy()
    t.step(200)
    scale = np.abs(ez0).max()
    assert np.abs(t.b).max() <= 1e-12 * scale
    assert np.abs(t.ez - ez0).max() <= 1e-12 * scale
    assert np.abs(t.er - er0).max() <= 1e-12 * np.abs(er0).max()


def test_gr_surface_field_second_order(oracle_mod):
    """The SCLF rule's surface field (node-0 Gauss law over the half cell, with
    rho_GJ,0 / alpha_0) agrees with the extrapolation 3/2 E_z(dz/2) - 1/2 E_z(3dz/2) of
    the vacuum start to O(dz^2): halving dz quarters the difference."""
    o = oracle_mod
    errs = []
    for N in (256, 512):
        t = _gr_tube(o, n_cells=N, flags=o.GR_ALPHA | o.NO_AUTO_INJECT)
        ez0, ez1 = t.ez[0], t.ez[1]
        t.step(1)
        errs.append(abs(t.counters["e_surf"] - (1.5 * ez0 - 0.5 * ez1)) / abs(ez0))
    assert errs[1] < 1e-3
    assert errs[0] / errs[1] > 3.0, errs


def _pulse_response(o, N, rstar):
    """E_r raised by a Gaussian B pulse added at mid-tube to the vacuum start, after
    t = 2.5 (N/2 steps of dt = dz/2 on the 10 R tube): the pulse stays clear of both
    ends, and the static start is subtracted."""
    t = _gr_tube(o, n_cells=N, r_star=rstar, flags=o.GR_ALPHA | o.NO_AUTO_INJECT, capacity=16)
    er0 = t.er.copy()
    L = t.cfg["length"]
    zf = (np.arange(N) + 0.5) * (L / N)
    t.b[:] += 1e-2 * np.exp(-((zf - 0.5 * L) / (0.08 * L)) ** 2)
    t.step(N // 2)
    return t.er - er0


@pytest.mark.parametrize("rstar", [2.0, RSTAR])
def test_gr_field_update_second_order(oracle_mod, rstar):
    """The alpha-weighted leap-frog converges at second order in dz: the differences of
    the pulse response between successive grids (on the common nodes) fall by 4.  The
    lapse taken half a cell off its field's position (at the node for B, say) leaves a
    first-order error, and the differences fall by less than 3.3."""
    d = {N: _pulse_response(oracle_mod, N, rstar) for N in (128, 256, 512, 1024)}
    e = [np.abs(d[N] - d[2 * N][::2]).max() for N in (128, 256, 512)]
    assert e[2] < 1e-6 and e[0] > 1e-7, e
    assert e[0] / e[1] > 3.6 and e[1] / e[2] > 3.6, e
