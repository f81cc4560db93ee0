"""Pins of the oracle's reverse-mode gradient (the CPU reference gradient).

The loss is the mean Lorentz factor of the electrons that leave the tube during
the run; the parameters are the knot values of a piecewise-linear rho_GJ
amplitude, the frame-dragging kappa (eq. 7) and the charge factor of injected
electrons.  Discrete decisions are frozen: injection counts replay the
recorded run, the macro-particle charge is held fixed.  The adjoint must agree
with central finite differences of the forward oracle."""
import numpy as np
import pytest

from paper_1011_6330_amd import synth


def _setup(K=9, N=128, n=2000, seed=0):
    cfg = dict(n_cells=N, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=synth.q_over_m_for(0.9 * N / 10.0),
               ppc=n / N, rho_kind=2, rho_amp=1.0, kappa=0.15, r_star=10.0, knots=np.ones(K),
               capacity=int(n * 2) + 4096, warm=n)
    x, u = synth.warm_start(cfg, seed=seed)
    dz = cfg["length"] / N
    cfg["macro_charge"] = -(1.0 - cfg["kappa"]) * dz / cfg["ppc"]
    return cfg, x, u


def _tube(oracle_mod, cfg, x, u, **over):
    c = {k: v for k, v in cfg.items() if k != "warm"}
    c.update(over)
    t = oracle_mod.OracleTube(c)
    t.inject(x, u)
    return t


def _schedule(oracle_mod, cfg, x, u, T):
    t = _tube(oracle_mod, cfg, x, u)
    sched = []
    for _ in range(T):
        t.step(1)
        sched.append(t.counters["last_ninj"])
    return np.array(sched, np.int64)


def _loss(oracle_mod, cfg, x, u, T, sched, **over):
    t = _tube(oracle_mod, cfg, x, u, schedule=sched, **over)
    ex0 = t.counters["n_exit"]
    s0 = t.exit_gamma_sum()
    t.step(T)
    nex = t.counters["n_exit"] - ex0
    return (t.exit_gamma_sum() - s0) / nex, nex


def _knot_weights(cfg, K):
    N = cfg["n_cells"]
    z = np.arange(N + 1) * (cfg["length"] / N)
    kz = np.linspace(0, cfg["length"], K)
    W = np.stack([np.interp(z, kz, np.eye(K)[k]) for k in range(K)], axis=1)   # [N+1, K]
    eta = 1.0 + z / cfg["r_star"]
    return W, eta


@pytest.fixture(scope="module")
def run(oracle_mod):
    T = 160
    cfg, x, u = _setup()
    sched = _schedule(oracle_mod, cfg, x, u, T)
    t = _tube(oracle_mod, cfg, x, u, schedule=sched)
    L, nex, g_rho, g_rate = t.adjoint(T)
    return dict(cfg=cfg, x=x, u=u, T=T, sched=sched, L=L, nex=nex, g_rho=g_rho, g_rate=g_rate)


def test_adjoint_loss_matches_forward(oracle_mod, run):
    L, nex = _loss(oracle_mod, run["cfg"], run["x"], run["u"], run["T"], run["sched"])
    assert nex == run["nex"] > 100
    assert L == run["L"]


def test_adjoint_vs_finite_differences_knots_kappa(oracle_mod, run):
    cfg, T, sched = run["cfg"], run["T"], run["sched"]
    K = len(cfg["knots"])
    W, eta = _knot_weights(cfg, K)
    fd_fac = 1.0 - cfg["kappa"] / eta ** 3
    g_theta = -(W * fd_fac[:, None]).T @ run["g_rho"]
    theta_z = W @ cfg["knots"]
    g_kappa = float(run["g_rho"] @ (theta_z / eta ** 3))
    h = 1e-6
    checked = 0
    for k in (1, 4, K - 1):
        kp, km = cfg["knots"].copy(), cfg["knots"].copy()
        kp[k] += h
        km[k] -= h
        Lp, np_ = _loss(oracle_mod, cfg, run["x"], run["u"], T, sched, knots=kp)
        Lm, nm = _loss(oracle_mod, cfg, run["x"], run["u"], T, sched, knots=km)
        assert np_ == nm == run["nex"]           # no exit event flipped
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g_theta[k]) <= 2e-4 * abs(g_theta).max() + 1e-6 * abs(fd), (k, fd, g_theta[k])
        checked += 1
    Lp, _ = _loss(oracle_mod, cfg, run["x"], run["u"], T, sched, kappa=cfg["kappa"] + h)
    Lm, _ = _loss(oracle_mod, cfg, run["x"], run["u"], T, sched, kappa=cfg["kappa"] - h)
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - g_kappa) <= 2e-4 * abs(g_kappa) + 1e-9, (fd, g_kappa)
    assert checked == 3


@pytest.fixture(scope="module")
def cold(oracle_mod):
    """Cold start (empty tube, SCLF injection from step 1) in a short tube, long
    enough for the injected electrons to leave it: the loss then depends on the
    injected charge."""
    N, L, T = 256, 3.0, 700
    cfg = dict(n_cells=N, length=L, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=4.0, rho_kind=2,
               rho_amp=1.0, kappa=0.15, r_star=10.0, knots=np.ones(7), capacity=40000, warm=0)
    cfg["macro_charge"] = -(1.0 - cfg["kappa"]) * (L / N) / cfg["ppc"]
    x, u = np.zeros(0), np.zeros(0)
    sched = _schedule(oracle_mod, cfg, x, u, T)
    t = _tube(oracle_mod, cfg, x, u, schedule=sched)
    Lz, nex, g_rho, g_rate = t.adjoint(T)
    return dict(cfg=cfg, x=x, u=u, T=T, sched=sched, L=Lz, nex=nex, g_rho=g_rho, g_rate=g_rate)


def test_adjoint_vs_finite_differences_rate(oracle_mod, cold):
    cfg, T, sched = cold["cfg"], cold["T"], cold["sched"]
    assert cold["nex"] > 100 and sched.sum() > 500
    h = 1e-6
    Lp, np_ = _loss(oracle_mod, cfg, cold["x"], cold["u"], T, sched, inj_rate=1.0 + h)
    Lm, nm = _loss(oracle_mod, cfg, cold["x"], cold["u"], T, sched, inj_rate=1.0 - h)
    assert np_ == nm == cold["nex"]
    fd = (Lp - Lm) / (2 * h)
    assert abs(cold["g_rate"]) > 0.1
    assert abs(fd - cold["g_rate"]) <= 5e-4 * abs(cold["g_rate"]), (fd, cold["g_rate"])


def test_adjoint_cold_knots(oracle_mod, cold):
    cfg, T, sched = cold["cfg"], cold["T"], cold["sched"]
    K = len(cfg["knots"])
    W, eta = _knot_weights(cfg, K)
    g_theta = -(W * (1.0 - cfg["kappa"] / eta ** 3)[:, None]).T @ cold["g_rho"]
    h = 1e-6
    for k in (0, 3, K - 1):
        kp, km = cfg["knots"].copy(), cfg["knots"].copy()
        kp[k] += h
        km[k] -= h
        Lp, _ = _loss(oracle_mod, cfg, cold["x"], cold["u"], T, sched, knots=kp)
        Lm, _ = _loss(oracle_mod, cfg, cold["x"], cold["u"], T, sched, knots=km)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g_theta[k]) <= 5e-4 * abs(g_theta).max(), (k, fd, g_theta[k])


def test_gradient_is_linear_response_of_the_start(oracle_mod, run):
    """rho_GJ enters only through the Poisson start (eq. 4): the node gradient is
    zero at node 0 (phi = 0 there) and the knot gradient equals the node gradient
    mapped through the hat functions."""
    assert run["g_rho"][0] == 0.0
    assert np.abs(run["g_rho"][1:]).max() > 0


# ---- dot-product pins of the linearised kernels (P13) --------------------------
#
# Each kernel of one step, linearised with its discrete decisions frozen, as a
# tangent map d -> tl(d) and its transpose l -> ad(l) (the transpose is the code
# the reverse sweep runs): <ad(l), d> = <l, tl(d)> for random d and l, to the
# rounding of the sums.

def _dot_rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _lin_tube(oracle_mod, seed=0):
    N = 97
    cfg = dict(n_cells=N, length=5.0, radius=1.0, dt_over_dz=0.5, q_over_m=synth.q_over_m_for(15.0), ppc=20.0,
               rho_kind=synth.RHO_FRAME_DRAG, rho_amp=1.0, kappa=0.15, r_star=10.0, capacity=10000)
    rng = np.random.default_rng(seed)
    n = 3000
    x = np.concatenate([rng.uniform(0.0, N, n - 40), rng.uniform(N - 0.6, N, 20), rng.uniform(0.0, 0.4, 20)])
    x = np.minimum(x, np.nextafter(float(N), 0.0))
    u = np.concatenate([rng.uniform(-20.0, 60.0, n - 40), rng.uniform(10.0, 50.0, 20), rng.uniform(-40.0, -5.0, 20)])
    t = oracle_mod.OracleTube(cfg)
    t.inject(x, u)
    t.k[:] = rng.normal(0.0, 0.3, N)            # a kick array with structure on every face
    return t, rng


def test_dot_product_fields(oracle_mod):
    t, rng = _lin_tube(oracle_mod, 1)
    N = t.N
    for _ in range(5):
        d = [rng.normal(size=N), rng.normal(size=N + 1), rng.normal(size=N), rng.normal(size=N) * 2.0 ** 20]
        l = [rng.normal(size=N), rng.normal(size=N + 1), rng.normal(size=N)]
        tl = t.tl_fields(*d)
        ad = t.ad_fields(*l)
        lhs = sum(float(a @ b) for a, b in zip(l, tl))
        rhs = sum(float(a @ b) for a, b in zip(ad, d))
        assert _dot_rel(lhs, rhs) <= 1e-12, (lhs, rhs)


def test_dot_product_push(oracle_mod):
    t, rng = _lin_tube(oracle_mod, 2)
    N, n = t.N, t.n
    for _ in range(5):
        d = [rng.normal(size=n) * 1e-3, rng.normal(size=n), rng.normal(size=N)]
        l = [rng.normal(size=n), rng.normal(size=n), rng.normal(size=N) * 2.0 ** -20]
        tl = t.tl_push(*d)
        ad = t.ad_push(*l)
        lhs = sum(float(a @ b) for a, b in zip(l, tl))
        rhs = sum(float(a @ b) for a, b in zip(ad, d))
        assert _dot_rel(lhs, rhs) <= 1e-12, (lhs, rhs)


def test_push_tangent_matches_finite_differences(oracle_mod):
    """The push's tangent against central differences of the forward step in a
    frozen field: particles inside the tube (none leaves or returns in one
    step), perturbed in u; x1 and u1 are smooth in u (the current is not compared:
    a cell crossing may flip)."""
    from oracle.oracle import FREEZE_FIELDS, NO_AUTO_INJECT, OracleTube
    t, rng = _lin_tube(oracle_mod, 3)
    N = t.N
    n = 2000
    x0 = rng.uniform(2.0, N - 2.0, n)
    u0 = rng.uniform(-20.0, 60.0, n)
    k0 = t.k.copy()
    cfg = dict(t.cfg, flags=FREEZE_FIELDS | NO_AUTO_INJECT)

    def tube(uu):
        o = OracleTube(cfg)
        o.inject(x0, uu)
        o.ez[:] = k0 / (cfg["q_over_m"] * cfg["dt_over_dz"] * o.dz)   # the kick array is (q/m) dt E_z
        return o
    base = tube(u0)
    base.k[:] = base.cfg["q_over_m"] * (base.cfg["dt_over_dz"] * base.dz) * base.ez
    du = rng.normal(size=n)
    dx1, du1, _ = base.tl_push(np.zeros(n), du, np.zeros(N))
    h = 1e-7
    cp, cm = tube(u0 + h * du), tube(u0 - h * du)
    cp.step(1)
    cm.step(1)
    assert cp.n == cm.n == n
    # the differences lose about ulp(u) / h = 1e-7 to cancellation
    np.testing.assert_allclose((cp.u - cm.u) / (2 * h), du1, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose((cp.x - cm.x) / (2 * h), dx1, rtol=1e-5, atol=1e-6)


def test_dot_product_poisson(oracle_mod):
    t, rng = _lin_tube(oracle_mod, 4)
    N = t.N
    for _ in range(5):
        drho = rng.normal(size=N + 1)
        lez, ler = rng.normal(size=N), rng.normal(size=N + 1)
        dez, der = t.tl_poisson(drho)
        (lrho,) = t.ad_poisson(lez, ler)
        lhs = float(lez @ dez + ler @ der)
        rhs = float(lrho @ drho)
        assert _dot_rel(lhs, rhs) <= 1e-12, (lhs, rhs)
    # eq. (4) is linear in rho_GJ: the tangent is the change of the start fields of
    # an empty tube when the uniform amplitude moves by 1 (rho_GJ = -A)
    from oracle.oracle import OracleTube
    a1 = OracleTube(dict(t.cfg, rho_kind=synth.RHO_UNIFORM, rho_amp=1.0))
    a2 = OracleTube(dict(t.cfg, rho_kind=synth.RHO_UNIFORM, rho_amp=2.0))
    dez, der = t.tl_poisson(np.full(N + 1, -1.0))
    np.testing.assert_allclose(dez, a2.ez - a1.ez, rtol=1e-10, atol=1e-12 * np.abs(dez).max())
    np.testing.assert_allclose(der, a2.er - a1.er, rtol=1e-10, atol=1e-12 * np.abs(der).max())
