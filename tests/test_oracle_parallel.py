"""The threaded oracle step (orc_step_par, used to time the oracle on every host
core) against the serial oracle, CPU only: the state after every step must be
identical bit for bit -- fields, current, counters, the particles in their order
and the injected-class bookkeeping -- whatever the thread count."""
import numpy as np
import pytest

from paper_1011_6330_amd import synth


def _tube(cfg, x=None, u=None):
    from oracle.oracle import OracleTube
    p = {k: v for k, v in synth.tube_params(cfg).items() if k not in ("sort_every", "max_bins", "precision",
                                                                       "gamma_fp64")}
    o = OracleTube(p)
    if x is not None and len(x):
        o.inject(x, u)
    return o


def _same(a, b, what):
    assert a.counters == b.counters, f"{what}: counters {a.counters} vs {b.counters}"
    for k in ("x", "u", "ez", "er", "b", "j", "cls", "j_inj"):
        va, vb = getattr(a, k), getattr(b, k)
        assert np.array_equal(va, vb), f"{what}: {k} differs"


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_cold_start_c1(threads, oracle_mod):
    cfg = synth.preset("c1")
    a, b = _tube(cfg), _tube(cfg)
    for s in range(4):
        a.step(100)
        b.step_par(100, threads)
        _same(a, b, f"c1 step {100 * (s + 1)} threads {threads}")
    assert a.counters["n_injected"] > 409


@pytest.mark.parametrize("threads", [2, 5, 16])
def test_random_particles_ragged_grid(threads, oracle_mod):
    """Unsorted particles, returns to the star and exits every step, N = 777."""
    N = 777
    cfg = dict(synth.preset("c1"), n_cells=N, length=N / 100.0, q_over_m=-40.0, ppc=6.0,
               rho_kind=synth.RHO_FRAME_DRAG, kappa=0.15, r_star=3.0, capacity=200000)
    x, u = synth.random_particles(N, 30011, seed=4)
    a, b = _tube(cfg, x, u), _tube(cfg, x, u)
    for s in range(30):
        a.step(1)
        b.step_par(1, threads)
        _same(a, b, f"random step {s + 1} threads {threads}")
    assert a.counters["n_exit"] > 0 and a.counters["n_absorb"] > 0


def test_warm_beam_injection_rate_and_schedule(oracle_mod):
    """The injected-class current (injection-rate factor) and a replayed
    injection schedule take the same paths in both."""
    N = 1024
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(120.0), ppc=30.0, warm=30 * N,
               capacity=int(30 * N * 1.5), inj_rate=1.7)
    x, u = synth.warm_start(cfg)
    a, b = _tube(cfg, x, u), _tube(cfg, x, u)
    a.step(40)
    b.step_par(40, 6)
    _same(a, b, "injection rate")
    assert a.counters["n_injected"] > 0 and a.j_inj.any()
    sched = np.array([3, 0, 5, 1] * 10, np.int64)
    cfg2 = dict(cfg, inj_rate=0.0, schedule=sched)
    a, b = _tube(cfg2, x, u), _tube(cfg2, x, u)
    a.step(40)
    b.step_par(40, 7)
    _same(a, b, "schedule")
    assert a.counters["n_injected"] == sched.sum()


def test_fewer_particles_than_threads(oracle_mod):
    cfg = dict(synth.preset("c1"), flags=1)
    x, u = np.array([3.25, 700.5]), np.array([0.5, -2.0])
    a, b = _tube(cfg, x, u), _tube(cfg, x, u)
    a.step(20)
    b.step_par(20, 8)
    _same(a, b, "two particles, eight threads")
