"""The hand-written GPU adjoint against the oracle's reverse-mode gradient
(itself pinned by finite differences in test_oracle_adjoint.py)."""
import numpy as np
import pytest

from gpu_common import assert_state_equal, make_pair, say
from paper_1011_6330_amd import synth

pytestmark = pytest.mark.gpu


def _warm_cfg(K=9, N=128, n=2000):
    cfg = dict(n_cells=N, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=synth.q_over_m_for(0.9 * N / 10.0),
               ppc=n / N, rho_kind=2, rho_amp=1.0, kappa=0.15, r_star=10.0, knots=np.ones(K),
               capacity=int(n * 2) + 4096, warm=n, sort_every=0)
    cfg["macro_charge"] = -(1.0 - cfg["kappa"]) * (cfg["length"] / N) / cfg["ppc"]
    x, u = synth.warm_start(cfg, seed=0)
    return cfg, x, u


def _cold_cfg():
    N, L = 256, 3.0
    cfg = dict(n_cells=N, length=L, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=4.0, rho_kind=2, rho_amp=1.0,
               kappa=0.15, r_star=10.0, knots=np.ones(7), capacity=40000, warm=0, sort_every=0)
    cfg["macro_charge"] = -(1.0 - cfg["kappa"]) * (L / N) / cfg["ppc"]
    return cfg, np.zeros(0), np.zeros(0)


def _compare(cfg, x, u, T, ckpt):
    g, o = make_pair(cfg, x, u)
    r = g.run_adjoint(T, ckpt)
    L, nex, g_rho, g_rate = o.adjoint(T)
    assert r["loss"] == L and r["n_exit"] == nex
    scale = np.abs(g_rho).max()
    assert scale > 0
    err = np.abs(r["g_rho"] - g_rho).max() / scale
    assert err <= 1e-8, err
    assert abs(r["g_rate"] - g_rate) <= 1e-8 * max(abs(g_rate), 1e-300) or g_rate == r["g_rate"] == 0.0
    # the tube is left where T plain steps leave it (bit-identical to the oracle)
    assert_state_equal(g, o, what="after adjoint")
    return r, g_rho, g_rate


@pytest.mark.parametrize("ckpt", [1, 7, 50, 160])
def test_adjoint_warm_matches_oracle(ckpt):
    cfg, x, u = _warm_cfg()
    say("adjoint warm ckpt", ckpt)
    r, g_rho, _ = _compare(cfg, x, u, 160, ckpt)
    # knot and kappa gradients from the node gradient (hat weights, eq. 7 factor)
    N, K = cfg["n_cells"], len(cfg["knots"])
    z = np.arange(N + 1) * (cfg["length"] / N)
    W = np.stack([np.interp(z, np.linspace(0, cfg["length"], K), np.eye(K)[k]) for k in range(K)], axis=1)
    eta = 1 + z / cfg["r_star"]
    g_theta = -(W * (1 - cfg["kappa"] / eta ** 3)[:, None]).T @ g_rho
    g_kappa = float(g_rho @ ((W @ cfg["knots"]) / eta ** 3))
    np.testing.assert_allclose(r["g_knots"], g_theta, rtol=1e-8, atol=1e-10 * np.abs(g_theta).max())
    assert abs(r["g_kappa"] - g_kappa) <= 1e-8 * abs(g_kappa)


def test_adjoint_odd_slot_count_matches_oracle():
    """An odd number of slots (the particle kernel takes two per thread, so the last
    thread holds one): the gradient still matches the oracle's."""
    cfg, x, u = _warm_cfg(n=2001)
    assert len(x) == 2001
    say("adjoint odd slot count")
    _compare(cfg, x, u, 120, 7)


def test_adjoint_cold_rate_matches_oracle():
    cfg, x, u = _cold_cfg()
    say("adjoint cold")
    r, _, g_rate = _compare(cfg, x, u, 700, 50)
    assert abs(g_rate) > 0.1


def test_adjoint_autograd_function():
    import torch

    from paper_1011_6330_amd.adjoint import exit_gamma_loss
    cfg, x, u = _warm_cfg()
    knots = torch.ones(9, dtype=torch.float64, requires_grad=True)
    kappa = torch.tensor(0.15, dtype=torch.float64, requires_grad=True)
    rate = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    loss = exit_gamma_loss(knots, kappa, rate, synth.tube_params(cfg), x, u, 160, 40)
    loss.backward()
    g, o = make_pair(cfg, x, u)
    L, nex, g_rho, g_rate = o.adjoint(160)
    assert float(loss.detach()) == L
    N, K = cfg["n_cells"], 9
    z = np.arange(N + 1) * (cfg["length"] / N)
    W = np.stack([np.interp(z, np.linspace(0, cfg["length"], K), np.eye(K)[k]) for k in range(K)], axis=1)
    eta = 1 + z / cfg["r_star"]
    g_theta = -(W * (1 - 0.15 / eta ** 3)[:, None]).T @ g_rho
    np.testing.assert_allclose(knots.grad.numpy(), g_theta, rtol=1e-8, atol=1e-10 * np.abs(g_theta).max())


def test_adjoint_rejects_sorting_tubes():
    from paper_1011_6330_amd import PicError, Tube
    cfg, x, u = _warm_cfg()
    t = Tube(dict(synth.tube_params(cfg), sort_every=16))
    with pytest.raises(PicError):
        t.run_adjoint(10, 5)


def _record_counts(cfg, x, u, T):
    """Injection counts of a plain run, step by step."""
    from paper_1011_6330_amd import Tube
    t = Tube(synth.tube_params(cfg))
    t.inject(x, u)
    counts = []
    for _ in range(T):
        t.step(1)
        counts.append(t.diagnostics(fields=False)["last_n_inj"])
    t.close()
    return np.array(counts, np.int64)


def test_injection_schedule_replay():
    """Replaying a run's own injection counts reproduces it bit for bit; a
    changed schedule injects exactly what it says."""
    from paper_1011_6330_amd import Tube
    cfg, x, u = _cold_cfg()
    T = 120
    counts = _record_counts(cfg, x, u, T)
    assert counts.sum() > 100
    ref = Tube(synth.tube_params(cfg))
    ref.step(T)
    rep = Tube(synth.tube_params(cfg))
    rep.set_injection_schedule(counts)
    rep.step(T)
    da, db = ref.diagnostics(j=True), rep.diagnostics(j=True)
    for k in ("ez", "er", "b_phi", "j_last"):
        assert np.array_equal(da[k], db[k]), k
    assert da["n_injected"] == db["n_injected"] == counts.sum()
    alt = counts.copy()
    alt[5:15] = 3
    t = Tube(synth.tube_params(cfg))
    t.set_injection_schedule(alt, first_step=0)
    for s in range(20):
        t.step(1)
        assert t.diagnostics(fields=False)["last_n_inj"] == alt[s]
    t.set_injection_schedule(None)
    for tt in (ref, rep, t):
        tt.close()


def _mean_exit_gamma(cfg, x, u, T, counts, **over):
    from paper_1011_6330_amd import Tube
    t = Tube(synth.tube_params(dict(cfg, **over)))
    t.inject(x, u)
    t.set_injection_schedule(counts)
    t.step(T)
    d = t.diagnostics(fields=False)
    t.close()
    return d["exit_gamma_sum"] / d["n_exit"], d["n_exit"]


def test_adjoint_c4_vs_finite_differences():
    """The 64-knot tube at full size (4096 cells, 1e6 particles, 1000 steps,
    checkpoint every 50): the hand-written gradient against central finite
    differences of the GPU forward (itself bit-identical to the oracle), with the
    injection counts frozen at the recorded run and h = 1e-6 (smaller if an exit
    event would flip)."""
    from paper_1011_6330_amd import Tube
    cfg = synth.preset("c4")
    x, u = synth.warm_start(cfg)
    T = 1000
    say("c4 adjoint: recording injection counts")
    counts = _record_counts(cfg, x, u, T)
    t = Tube(synth.tube_params(cfg))
    t.inject(x, u)
    r = t.run_adjoint(T, 50)
    t.close()
    g_knots, g_kappa = r["g_knots"], r["g_kappa"]
    L0, n0 = _mean_exit_gamma(cfg, x, u, T, counts)
    assert n0 == r["n_exit"] > 10000 and L0 == r["loss"]
    scale = np.abs(g_knots).max()
    say("c4 adjoint: loss", L0, "exits", n0, "max |dL/dknot|", scale, "dL/dkappa", g_kappa)
    checked = 0
    for name, k in (("kappa", None), ("knot", 0), ("knot", 21), ("knot", 42), ("knot", 63)):
        for h in (1e-6, 3e-7, 1e-7):
            if k is None:
                Lp, npl = _mean_exit_gamma(cfg, x, u, T, counts, kappa=cfg["kappa"] + h)
                Lm, nmi = _mean_exit_gamma(cfg, x, u, T, counts, kappa=cfg["kappa"] - h)
            else:
                kp, km = cfg["knots"].copy(), cfg["knots"].copy()
                kp[k] += h
                km[k] -= h
                Lp, npl = _mean_exit_gamma(cfg, x, u, T, counts, knots=kp)
                Lm, nmi = _mean_exit_gamma(cfg, x, u, T, counts, knots=km)
            if npl == nmi == n0:
                break
        assert npl == nmi == n0, f"{name} {k}: an exit event flips even at h = {h}"
        fd = (Lp - Lm) / (2 * h)
        g = g_kappa if k is None else g_knots[k]
        ref = abs(g_kappa) if k is None else scale
        say("c4 adjoint:", name, k, "fd", fd, "adjoint", g, "h", h)
        assert abs(fd - g) <= 2e-4 * ref, (name, k, fd, g)
        checked += 1
    assert checked == 5


def test_adjoint_gr_background_params():
    """The eq. (6) background: node gradient as the oracle's, and dL/dkappa, dL/dA
    mapped through rho = -A [(1 - kappa/eta^3) + s eta^(1/2)] / alpha."""
    cfg, x, u = _warm_cfg()
    cfg = dict(cfg, rho_kind=synth.RHO_GR, incl=0.5, theta_star=0.67 * 0.014, rg_over_rstar=0.4, knots=None)
    say("adjoint gr background")
    r, g_rho, _ = _compare(cfg, x, u, 160, 50)
    N = cfg["n_cells"]
    z = np.arange(N + 1) * (cfg["length"] / N)
    eta = 1 + z / cfg["r_star"]
    s = 1.5 * cfg["theta_star"] * np.tan(cfg["incl"])
    al = np.sqrt(1 - cfg["rg_over_rstar"] / eta)
    br = (1 - cfg["kappa"] / eta ** 3) + s * np.sqrt(eta)
    g_amp = float(g_rho @ (-br / al))
    g_kappa = float(g_rho @ (cfg["rho_amp"] / (eta ** 3 * al)))
    assert abs(r["g_amp"] - g_amp) <= 1e-8 * abs(g_amp)
    assert abs(r["g_kappa"] - g_kappa) <= 1e-8 * abs(g_kappa)


def test_adjoint_reproducible_lazy_and_scaled():
    """The reverse sweep shares every sum between waves as an integer sum, so
    the gradient is the same bits on every run: two reverse sweeps of one
    recorded forward, and a second tube's whole adjoint, agree bit for bit.
    pic_backward scales by the incoming gradient, and refuses once the tube has
    moved on from its recorded forward."""
    from paper_1011_6330_amd import PicError, Tube
    cfg, x, u = _cold_cfg()
    T = 700
    say("adjoint reproducible")
    t = Tube(synth.tube_params(cfg))
    f = t.adjoint_forward(T, 50)
    a = t.backward()
    b = t.backward()
    c = t.backward(2.5)
    assert f["loss"] == a["loss"] and f["n_exit"] == a["n_exit"] > 0
    for k in ("g_rate", "g_kappa", "g_amp"):
        assert a[k] == b[k], k
        assert c[k] == 2.5 * a[k], k
    assert np.array_equal(a["g_rho"], b["g_rho"]) and np.array_equal(a["g_knots"], b["g_knots"])
    assert np.array_equal(c["g_rho"], 2.5 * a["g_rho"])
    assert abs(a["g_rate"]) > 0.1
    t2 = Tube(synth.tube_params(cfg))
    r2 = t2.run_adjoint(T, 50)
    for k in ("g_rate", "g_kappa", "g_amp", "loss"):
        assert r2[k] == a[k], k
    assert np.array_equal(r2["g_rho"], a["g_rho"]) and np.array_equal(r2["g_knots"], a["g_knots"])
    # the tube ends where the forward left it, so the sweep can run again; once
    # it steps on, the recorded forward is gone
    t.step(1)
    with pytest.raises(PicError) as e:
        t.backward()
    assert e.value.code == -7
    fresh = Tube(synth.tube_params(cfg))
    with pytest.raises(PicError) as e:
        fresh.backward()
    assert e.value.code == -7
    for tt in (t, t2, fresh):
        tt.close()


@pytest.mark.parametrize("T", [1, 2, 5])
def test_adjoint_few_steps_tight(T):
    """A few reverse steps against the oracle's at 1e-12: one step exercises each
    transposed kernel once (field update, particle push and deposit, Poisson).
    Particles start next to the top of the tube so that some leave in the first
    step and seed the loss."""
    N = 128
    cfg = dict(n_cells=N, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=synth.q_over_m_for(12.0),
               ppc=30.0, rho_kind=2, rho_amp=1.0, kappa=0.15, r_star=10.0, knots=np.ones(9),
               capacity=20000, warm=0, sort_every=0)
    cfg["macro_charge"] = -(1.0 - cfg["kappa"]) * (cfg["length"] / N) / cfg["ppc"]
    rng = np.random.default_rng(T)
    x = np.concatenate([N - rng.uniform(0.0, 1.4, 400), rng.uniform(0.0, N, 3000)])
    u = np.concatenate([rng.uniform(2.0, 30.0, 400), rng.uniform(-5.0, 30.0, 3000)])
    x = np.minimum(x, np.nextafter(float(N), 0.0))
    g, o = make_pair(cfg, x, u)
    r = g.run_adjoint(T, 1)
    L, nex, g_rho, g_rate = o.adjoint(T)
    assert r["loss"] == L and r["n_exit"] == nex > 0
    err = np.abs(r["g_rho"] - g_rho).max() / np.abs(g_rho).max()
    say("adjoint", T, "steps: g_rho max rel", err, "g_rate", r["g_rate"], g_rate)
    assert err <= 1e-12
    assert abs(r["g_rate"] - g_rate) <= 1e-12 * max(abs(g_rate), 1e-300) or g_rate == r["g_rate"] == 0.0
