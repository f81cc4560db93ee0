"""GPU FP64 path vs the CPU oracle, through the C ABI: bit-identical results.

The FP64 kernels evaluate every formula of the step with the oracle's operand
order (no FMA contraction, IEEE division and square root), deposit the current
in exact fixed point, and reduce only integers, so the two must agree to the
last bit; the 1e-10 relative gate of the FP64 path is never needed.
"""
import math

import numpy as np
import pytest

from gpu_common import assert_state_equal, make_pair, say
from paper_1011_6330_amd import synth

pytestmark = pytest.mark.gpu


def test_c1_full_run_bit_identical():
    """C1: flat-space SCLF from an empty tube, 2000 steps (cold start)."""
    cfg = synth.preset("c1")
    say("c1 full run", cfg["n_cells"], "cells, 2000 steps")
    g, o = make_pair(cfg)
    for s in range(8):
        g.step(250)
        o.step(250)
        assert_state_equal(g, o, what=f"c1 step {250 * (s + 1)}")
    d = g.diagnostics()
    assert d["n_injected"] > 409 and d["n_absorb"] > 0
    g.close()


def test_vacuum_stays_fixed():
    """No particles, no injection: the Poisson field is stationary (P3), identically."""
    cfg = synth.preset("c1", flags=1)   # PIC_NO_AUTO_INJECT
    say("vacuum 2000 steps")
    g, o = make_pair(cfg)
    g.step(2000)
    o.step(2000)
    assert_state_equal(g, o, what="vacuum")


@pytest.mark.parametrize("N,n", [(777, 3 * 1024 + 123), (1000, 1), (256, 0), (2048, 20000), (257, 900), (511, 1700),
                                 (255, 800)])
def test_ragged_grid_and_tail_stepwise(N, n):
    """Grids that are not a multiple of the 256 faces a wave of the field update takes
    (a whole last span, one face past it, a span short by one, a grid shorter than
    one span), particle counts with a ragged last tile; J of every step bit-exact,
    frame-drag background."""
    cfg = dict(synth.preset("c1"), n_cells=N, length=N / 100.0, q_over_m=-40.0, ppc=6.0,
               rho_kind=synth.RHO_FRAME_DRAG, kappa=0.15, r_star=3.0, capacity=200000)
    x, u = synth.random_particles(N, n, seed=7)
    say("ragged", N, n)
    g, o = make_pair(cfg, x, u)
    for s in range(60):
        g.step(1)
        o.step(1)
        d = g.diagnostics(fields=False, j=True)
        assert np.array_equal(d["j_last"], o.j), f"J differs at step {s + 1}"
        assert d["last_n_inj"] == o.counters["last_ninj"]
    assert_state_equal(g, o, what=f"ragged N={N} n={n}")


def test_sorted_warm_tube():
    """Warm frame-drag beam with the cell sort every 16 steps: the sort only
    reorders, so fields and counters stay bit-identical and the particle multiset
    is the oracle's."""
    N = 4096
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(430.0), ppc=40.0,
               warm=40 * N, capacity=int(40 * N * 1.2), sort_every=16)
    x, u = synth.warm_start(cfg)
    say("sorted warm", N, len(x))
    g, o = make_pair(cfg, x, u)
    for s in range(5):
        g.step(40)
        o.step(40)
        assert_state_equal(g, o, ordered=False, what=f"sorted warm step {40 * (s + 1)}")
    d = g.diagnostics(fields=False)
    assert d["n_slots"] >= d["n_alive"]


@pytest.mark.parametrize("ppc,sub", [(520.0, 4), (250.0, 3)])
def test_sort_width_bit_identical(ppc, sub):
    """The cell sort at the sub-cell key widths of the full-size tubes: 2^4 bins
    per cell from ppc 257 on (C2), 2^3 for ppc 129..256 (C4, C5).  A warm
    frame-drag beam loaded in a shuffled order (so that the first sort has to
    reorder everything), sorted every 16 steps for 40 steps: right after each
    sort the slots are in key order (key = floor(x 2^sub)) with no removed slot
    left, and fields, current, counters and the particle multiset are
    bit-identical to the oracle's after steps 16, 32 and 40."""
    N = 4096
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(430.0), ppc=ppc,
               warm=int(ppc * N), capacity=int(ppc * N * 1.2), sort_every=16)
    x, u = synth.warm_start(cfg)
    perm = np.random.default_rng(9).permutation(len(x))
    x, u = x[perm], u[perm]
    say("sort width 2^%d:" % sub, len(x), "particles")
    g, o = make_pair(cfg, x, u)
    del x, u
    done = 0
    for h in (16, 32, 40):
        g.step(h - done)
        o.step(h - done)
        done = h
        d = assert_state_equal(g, o, ordered=False, what=f"sort width 2^{sub} step {h}")
        if h % 16 == 0:
            assert d["n_slots"] == d["n_alive"]
            px, _ = g.read_particles()
            assert np.all(np.diff(np.floor(px * 2 ** sub)) >= 0), "slots not in key order after the sort"
    g.close()


@pytest.mark.parametrize("shape", [(64, 4), (128, 4), (256, 2), (256, 4), (512, 2), (128, 2, True),
                                   (256, 2, True), (64, 4, True), (64, 8, True), (128, 8)])
def test_push_launch_shapes_identical(shape):
    """Every push launch shape the tuner may pick gives the oracle's state."""
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0,
               warm=30 * N, capacity=int(30 * N * 1.3), sort_every=16)
    x, u = synth.warm_start(cfg)
    say("push shape", shape)
    g, o = make_pair(cfg, x, u)
    g.set_push_config(*shape)
    g.step(50)
    o.step(50)
    assert_state_equal(g, o, ordered=False, what=f"shape {shape}")


def test_shuffled_load_and_rerun_identical():
    N = 512
    cfg = dict(synth.preset("c1"), n_cells=N, q_over_m=-25.0, ppc=10.0, rho_kind=synth.RHO_FRAME_DRAG,
               kappa=0.15, r_star=5.0, capacity=100000, sort_every=8)
    x, u = synth.random_particles(N, 6000, seed=3)
    perm = np.random.default_rng(0).permutation(len(x))
    from paper_1011_6330_amd import Tube
    outs = []
    for xx, uu in ((x, u), (x[perm], u[perm]), (x, u)):
        t = Tube(synth.tube_params(cfg))
        t.inject(xx, uu)
        t.step(100)
        d = t.diagnostics(fields=True, j=True)
        px, pu = t.read_particles()
        k = np.lexsort((pu, px))
        outs.append((d["ez"], d["er"], d["b_phi"], d["j_last"], px[k], pu[k], d["exit_sum_lo"]))
        t.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0], outs[2]):
        assert np.array_equal(a, b)


def test_diagnostics_match_oracle():
    cfg = synth.preset("c1")
    g, o = make_pair(cfg)
    g.step(700)
    o.step(700)
    nb = 37
    d = g.diagnostics(n_bins=nb, gauss=True, weights=True, rho=True)
    cnt, lo, hi, mn, mx = o.profile(nb)
    assert np.array_equal(d["prof_count"], cnt)
    assert np.array_equal(d["prof_sum_lo"], lo) and np.array_equal(d["prof_sum_hi"], hi)
    sel = cnt > 0
    assert np.array_equal(d["prof_min"][sel], mn[sel]) and np.array_equal(d["prof_max"][sel], mx[sel])
    assert np.array_equal(d["weights"], o.weights())
    assert np.array_equal(d["rho_gj"], o.rho_gj)
    G, gmax = o.gauss()
    assert np.array_equal(d["gauss"], G)
    assert d["gauss_max"] == gmax
    assert d["gauss_max"] < 1e-10
    # L2 norm of the residual over the interior nodes, same normalisation as the maximum
    l2 = np.sqrt(np.mean(G[1:-1] ** 2)) / (4 * np.pi * np.abs(o.rho_gj).max())
    assert d["gauss_l2"] == pytest.approx(l2, rel=1e-12, abs=0.0)
    assert 0.0 < d["gauss_l2"] <= d["gauss_max"]
    # the norm alone, without the residual array
    d2 = g.diagnostics(gauss=False, fields=False)
    assert d2["gauss_l2"] == 0.0
    from paper_1011_6330_amd._binding import PicDiag, PicDiagReq
    import ctypes
    req, out = PicDiagReq(0, 1, 0.0), PicDiag()
    assert g.lib.pic_diagnostics(g._h, ctypes.byref(req), ctypes.byref(out)) == 0
    assert out.gauss_l2 == d["gauss_l2"] and out.gauss_max == d["gauss_max"]


def test_uniform_field_test_particle():
    """P1 on the GPU: frozen uniform field, u_n = (n + 1/2) K exactly, positions
    identical to the oracle."""
    cfg = dict(synth.preset("c1"), flags=1 | 2, capacity=8)
    g, o = make_pair(cfg, np.array([2.0]), np.array([-0.5 * 10.0 / 1024]))
    ez = np.full(1024, -2.0)
    g.write_fields(ez=ez)
    o.ez[:] = ez
    for n in range(1, 400):
        g.step(1)
        o.step(1)
    x, u = g.read_particles()
    assert u[0] == o.u[0] and x[0] == o.x[0]
    assert u[0] == 398.5 * 10.0 / 1024     # u_n = u_0 + n K, K = (q/m) dt E0 = 10/1024


def _near_midpoint_momenta(n_keep, n_cand=20_000_000, seed=21):
    """Momenta u whose velocity u / sqrt(1 + u^2) lies closest to a rounding
    midpoint of the double grid (the hard cases of a correctly rounded
    quotient): the exact remainder u - g q of the rounded quotient q = u / g,
    g = sqrt(1 + u^2), from Dekker's exact product, gives the distance of u / g
    from q in ulps; the n_keep candidates nearest to half an ulp are kept."""
    rng = np.random.default_rng(seed)
    u = 10.0 ** rng.uniform(-8.0, 9.0, n_cand)
    g = np.sqrt(1.0 + u * u)
    q = u / g
    split = 134217729.0                         # 2^27 + 1

    def halves(a):
        t = split * a
        hi = t - (t - a)
        return hi, a - hi
    gh, gl = halves(g)
    qh, ql = halves(q)
    p = g * q
    e = ((gh * qh - p) + gh * ql + gl * qh) + gl * ql   # g q = p + e exactly
    rem = (u - p) - e                                  # u - p is exact (p is within an ulp of u)
    frac = np.abs(rem / g) / np.spacing(q)
    keep = np.argsort(-frac)[:n_keep]
    return u[keep], float(frac[keep].min())


def test_gamma_velocity_bits():
    """The push's gamma = sqrt(1 + u^2) and v = u / gamma against the oracle's C
    library square root and division, bit for bit.  Particles start at x = 0 in
    a zero field, so after one step x = v / 2 exactly (dt/dz = 1/2) and each
    stored position holds the bits of v.  10^7 momenta: log-uniform over
    2^-1074 .. 1e153, the edges of the range [2^-400, 2^400] where the push skips
    the library's range scaling, the powers of two in between, and the 2e5
    momenta (of 2e7 candidates) whose quotient lies nearest to a rounding
    midpoint: the nearest within 1e-8 ulp of it, all within 6e-3 ulp."""
    rng = np.random.default_rng(5)
    edges = [2.0 ** -400, 2.0 ** 400, 2.0 ** -1022]
    special = [5e-324, 1.0, 0.5, 3.0] + edges + [np.nextafter(e, 0.0) for e in edges] + \
              [np.nextafter(e, np.inf) for e in edges] + [2.0 ** k for k in range(-80, 80)]
    mid, mid_frac = _near_midpoint_momenta(200_000)
    say("gamma/v bits: near-midpoint quotients within", f"{0.5 - mid_frac:.2e}", "ulp of a midpoint")
    assert mid_frac > 0.494
    u = np.concatenate([10.0 ** rng.uniform(-323.5, 153.0, 9_800_000), mid, np.array(special)])
    x = np.zeros_like(u)
    cfg = dict(synth.preset("c1"), flags=1 | 2, capacity=len(u) + 8)
    g, o = make_pair(cfg, x, u)
    ez = np.zeros(1024)
    g.write_fields(ez=ez)
    o.ez[:] = ez
    g.step(1)
    o.step(1)
    gx, gu = g.read_particles()
    assert len(gx) == len(u) == o.n
    assert np.array_equal(gu, o.u[:o.n]) and np.array_equal(gu, u)
    bad = np.flatnonzero(gx != o.x[:o.n])
    assert bad.size == 0, f"{bad.size} positions differ, first u = {u[bad[:5]]}"
    # the oracle's quotient is the correctly rounded one: v = 2 x agrees with numpy's division
    nrm = u >= 2.0 ** -1000                   # v / 2 is not subnormal: x holds v exactly
    v = 2.0 * o.x[:o.n][nrm]
    assert np.array_equal(v, u[nrm] / np.sqrt(1.0 + u[nrm] * u[nrm]))
    g.close()


def test_exit_absorb_and_gamma_sum():
    N = 64
    cfg = dict(synth.preset("c1"), n_cells=N, length=1.0, flags=1 | 2, capacity=16)
    x = np.array([N - 0.1, 0.1, 10.0, N - 0.3])
    u = np.array([10.0, -10.0, 0.0, 1e7])
    g, o = make_pair(cfg, x, u)
    z = np.zeros(N)
    g.write_fields(ez=z)
    o.ez[:] = z
    g.step(1)
    o.step(1)
    d = assert_state_equal(g, o, what="exits")
    assert d["n_exit"] == 2 and d["n_absorb"] == 1
    expect = (round(math.sqrt(101.0) * 2 ** 32) + round(math.sqrt(1.0 + 1e14) * 2 ** 32)) / 2 ** 32
    assert d["exit_gamma_sum"] == expect


def test_capacity_clip_latches_status():
    from paper_1011_6330_amd import PicError
    cfg = dict(synth.preset("c1"), capacity=300)
    g, o = make_pair(cfg)
    g.step(1)
    o.step(1)
    d = g.diagnostics(raise_on_status=False)
    assert d["status"] & 1 and d["n_alive"] == 300 == o.n
    assert o.counters["status"] & 1
    with pytest.raises(PicError) as e:
        g.sync()
    assert e.value.code == -9


def test_inject_rejects_bad_particles():
    from paper_1011_6330_amd import PicError, Tube
    t = Tube(synth.tube_params(dict(synth.preset("c1"), capacity=10)))
    for x, u, code in (([1.0, 2000.0], [0.0, 0.0], -1), ([1.0], [np.nan], -4),
                       (np.ones(11), np.zeros(11), -3), ([-0.5], [0.0], -1)):
        with pytest.raises(PicError) as e:
            t.inject(np.array(x, float), np.array(u, float))
        assert e.value.code == code
    import torch
    xd = torch.tensor([1.0, 5000.0], device="cuda", dtype=torch.float64)
    ud = torch.zeros(2, device="cuda", dtype=torch.float64)
    with pytest.raises(PicError):
        t.inject(xd, ud)
    assert t.diagnostics(fields=False)["n_alive"] == 0
    t.close()


def test_c2_full_size_first_steps():
    """The frame-dragging tube at full size (65,536 cells, ~4e7 particles, gamma up
    to ~6e6), in the benchmark's launch configuration: every result after 3 steps
    bit-identical to the oracle."""
    import bench
    cfg = synth.preset("c2")
    x, u = synth.warm_start(cfg)
    say("c2 full size", len(x), "particles, push shape", bench.DEFAULT_PUSH)
    g, o = make_pair(cfg, x, u)
    g.set_push_config(*bench.shape_of(bench.DEFAULT_PUSH))
    del x, u
    g.step(3)
    o.step(3)
    d = assert_state_equal(g, o, what="c2 full size")
    assert d["n_alive"] > 3.9e7
    # diagnostics at full size: each wave walks long runs of one profile bin and
    # one cell, so the per-wave partial sums carry almost every particle
    nb = 64
    d = g.diagnostics(n_bins=nb, gauss=True, weights=True, fields=False)
    cnt, lo, hi, mn, mx = o.profile(nb)
    assert np.array_equal(d["prof_count"], cnt)
    assert np.array_equal(d["prof_sum_lo"], lo) and np.array_equal(d["prof_sum_hi"], hi)
    assert np.array_equal(d["prof_min"], mn) and np.array_equal(d["prof_max"], mx)
    assert np.array_equal(d["weights"], o.weights())
    G, gmax = o.gauss()
    assert np.array_equal(d["gauss"], G) and d["gauss_max"] == gmax


@pytest.mark.parametrize("precision", [0, 1])
def test_save_load_resumes_bit_for_bit(precision):
    """P11: a tube restored from pic_save continues exactly as the saved one
    (fields, last-step current, counters, particle slots), across sorts."""
    from paper_1011_6330_amd import PicError, Tube
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0,
               warm=30 * N, capacity=int(30 * N * 1.3), sort_every=16, precision=precision, gamma_fp64=2000.0)
    x, u = synth.warm_start(cfg)
    say("save/load precision", precision)
    a = Tube(synth.tube_params(cfg))
    a.inject(x, u)
    a.step(37)
    state = a.save()
    a.step(100)
    b = Tube(synth.tube_params(dict(cfg, capacity=int(30 * N * 1.5))))   # more room: the slots still fit
    b.load(state)
    b.step(100)
    da, db = a.diagnostics(fields=True, j=True), b.diagnostics(fields=True, j=True)
    for k in ("ez", "er", "b_phi", "j_last"):
        assert np.array_equal(da[k], db[k]), k
    for k in ("step", "n_alive", "n_slots", "n_injected", "n_exit", "n_absorb", "exit_sum_lo", "exit_sum_hi",
              "e_surf", "w0", "n_slots_high"):
        assert da[k] == db[k], k
    xa, ua = a.read_particles()
    xb, ub = b.read_particles()
    ka, kb = np.lexsort((ua, xa)), np.lexsort((ub, xb))   # the sort may order equal keys differently
    assert np.array_equal(xa[ka], xb[kb]) and np.array_equal(ua[ka], ub[kb])
    # another tube's parameters are refused
    c = Tube(synth.tube_params(dict(cfg, kappa=0.1)))
    with pytest.raises(PicError):
        c.load(state)
    for t in (a, b, c):
        t.close()


def test_c5_full_size_first_steps():
    """The large tube at full size (2^20 cells, L = 100R, 2.5e8 particles): two
    steps bit-identical to the oracle, sorted like the benchmark runs it."""
    import bench
    cfg = synth.preset("c5")
    say("c5: warm start of", cfg["warm"], "particles")
    x, u = synth.warm_start(cfg)
    g, o = make_pair(cfg, x, u)
    g.set_push_config(*bench.shape_of(bench.DEFAULT_PUSH))
    del x, u
    say("c5: stepping")
    g.step(2)
    o.step(2)
    d = assert_state_equal(g, o, what="c5 full size")
    assert d["n_alive"] > 2.4e8
    g.close()


def _first_fixed_c_prime(N, bd):
    """First row i < N at which the forward elimination's c'_i = 1/(bd - c'_{i-1})
    repeats c'_{i-1} exactly (Python floats: IEEE double, correctly rounded), or None."""
    c = 1.0 / bd
    for i in range(2, N):
        cn = 1.0 / (bd - c)
        if cn == c:
            return i
        c = cn
    return None


POISSON_CASES = {
    # c' reaches a fixed point early (dz/R = 0.01): most rows take the d'-only runs
    "fixed_c": dict(n_cells=5000, length=50.0),
    # rho_GJ = 0 over the first knots: zero numerators, so those runs fall back to plain divisions
    "zero_rhs": dict(n_cells=4096, length=40.96, rho_kind=synth.RHO_KNOTS, kappa=0.0,
                     knots=np.array([0.0, 0.0, 0.0, 1.0, 1.5, 1.0, 0.5, 1.0]), macro_charge=0.01),
    # numerators beyond 2^400 and below 2^-600: plain divisions throughout
    "huge_rhs": dict(n_cells=3000, length=30.0, rho_amp=1e125),
    "tiny_rhs": dict(n_cells=3000, length=30.0, rho_amp=1e-185),
    # fewer rows than a run, and one run plus a tail
    "small_5": dict(n_cells=5, length=0.05),
    "small_17": dict(n_cells=17, length=0.17),
    # several chunks with a ragged last one, a warm random load and the frame-drag background
    "chunks_ragged": dict(n_cells=2 * 2048 + 37, length=41.33, rho_kind=synth.RHO_FRAME_DRAG, kappa=0.15,
                          r_star=3.0, capacity=200000),
}


@pytest.mark.parametrize("case", sorted(POISSON_CASES))
def test_poisson_start_bit_identical(case):
    """The Poisson start (eq. 4) on tubes that take each path of the solver: runs
    whose c' has stopped changing, runs that fall back to plain divisions, fewer
    rows than a run, several chunks; E_z and E_r bit-identical to the oracle."""
    over = POISSON_CASES[case]
    cfg = dict(synth.preset("c1"), flags=1, **over)     # PIC_NO_AUTO_INJECT
    N = int(cfg["n_cells"])
    if case == "fixed_c":
        h2 = (cfg["length"] / N / cfg["radius"]) ** 2
        row = _first_fixed_c_prime(N, -(2.0 + h2))
        assert row is not None and row < N - 64, row
    x = u = None
    if case == "chunks_ragged":
        x, u = synth.random_particles(N, 30000, seed=11)
    say("poisson start", case, N)
    g, o = make_pair(cfg, x, u)
    d = g.diagnostics()
    assert np.array_equal(d["ez"], o.ez), f"E_z differs ({case})"
    assert np.array_equal(d["er"], o.er), f"E_r differs ({case})"
    assert np.all(np.isfinite(d["ez"]))
    g.close()


def test_gr_background_bit_identical():
    """Eq. (6) background with the redshift and the inclination term
    (i = 0.5 rad, theta_* = 0.67 theta_p, r_g/R_* = 0.4): background, start and
    100 sorted steps of a warm beam bit-identical to the oracle."""
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0,
               warm=30 * N, capacity=int(30 * N * 1.3), sort_every=16, rho_kind=synth.RHO_GR, incl=0.5,
               theta_star=0.67 * 0.014, rg_over_rstar=0.4)
    x, u = synth.warm_start(cfg)
    say("gr background", N, len(x))
    g, o = make_pair(cfg, x, u)
    d = g.diagnostics(rho=True)
    assert np.array_equal(d["rho_gj"], o.rho_gj)
    assert np.array_equal(d["ez"], o.ez)
    g.step(100)
    o.step(100)
    assert_state_equal(g, o, ordered=False, what="gr background")
    g.close()


def test_b_steady_init_bit_identical():
    """Warm start with B_phi = 4 pi R j of the loaded beam (PIC_B_STEADY_INIT):
    the starting fields and 60 sorted steps bit-identical to the oracle."""
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0,
               warm=30 * N, capacity=int(30 * N * 1.3), sort_every=16, flags=4)
    x, u = synth.warm_start(cfg)
    say("b steady init", N, len(x))
    g, o = make_pair(cfg, x, u)
    d = g.diagnostics()
    assert np.array_equal(d["b_phi"], o.b) and np.abs(o.b).max() > 0
    assert np.array_equal(d["ez"], o.ez) and np.array_equal(d["er"], o.er)
    g.step(60)
    o.step(60)
    assert_state_equal(g, o, ordered=False, what="b steady init")
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_rounds_equal_direct_steps(precision):
    """pic_step replays whole sort_every rounds from captured graphs; stepping
    one step per call launches every kernel directly.  Both give the same state,
    bit for bit (also across a launch-shape change, which drops the graphs)."""
    from paper_1011_6330_amd import Tube
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0,
               warm=30 * N, capacity=int(30 * N * 1.3), sort_every=16)
    x, u = synth.warm_start(cfg)
    p = dict(synth.tube_params(cfg), precision=precision)
    a, b = Tube(p), Tube(p)
    a.inject(x, u)
    b.inject(x, u)
    say("graph rounds, precision", precision)
    a.step(64)
    for _ in range(64):
        b.step(1)
    a.set_push_config(64, 4 if precision else 2, True)
    b.set_push_config(64, 4 if precision else 2, True)
    a.step(40)
    for _ in range(40):
        b.step(1)
    da = a.diagnostics(n_bins=16, fields=True, j=True)
    db = b.diagnostics(n_bins=16, fields=True, j=True)
    for k in ("ez", "er", "b_phi", "j_last", "prof_count", "prof_sum_lo", "prof_sum_hi"):
        assert np.array_equal(da[k], db[k]), k
    for k in ("step", "n_alive", "n_injected", "n_exit", "n_absorb", "exit_sum_lo", "exit_sum_hi", "w0"):
        assert da[k] == db[k], k
    xa, ua = a.read_particles()
    xb, ub = b.read_particles()
    ka, kb = np.lexsort((ua, xa)), np.lexsort((ub, xb))
    assert np.array_equal(xa[ka], xb[kb]) and np.array_equal(ua[ka], ub[kb])
    a.close()
    b.close()


def test_stream_copy_exact():
    """The benchmark's reference copy moves every byte, including a ragged tail
    of 16-byte vectors past the last full block."""
    import ctypes

    import torch

    from paper_1011_6330_amd import _binding
    lib = _binding.load()
    n = 64 * 1000 + 37                       # vectors of 16 bytes
    src = torch.randint(-2 ** 62, 2 ** 62, (2 * n + 2,), dtype=torch.int64, device="cuda:0")
    dst = torch.zeros_like(src)
    rc = lib.pic_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), 16 * n,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.pic_last_error().decode()
    torch.cuda.synchronize()
    assert torch.equal(dst[:2 * n], src[:2 * n])
    assert int(dst[2 * n:].abs().sum()) == 0  # nothing written past the end


def test_gauss_residual_status_bit():
    """A diagnostics call with a Gauss tolerance latches PIC_ST_GAUSS when the
    residual of eq. (2) exceeds it, and only then."""
    from paper_1011_6330_amd import PicError, Tube
    t = Tube(synth.tube_params(synth.preset("c1")))
    t.step(300)
    d = t.diagnostics(gauss=True, fields=False, gauss_tol=1e-6)      # C1 keeps it near 1e-11
    assert d["status"] == 0 and 0.0 < d["gauss_max"] < 1e-6
    d = t.diagnostics(gauss=True, fields=False, gauss_tol=d["gauss_max"] / 2, raise_on_status=False)
    assert d["status"] & 4
    with pytest.raises(PicError) as e:
        t.sync()                                                       # latched
    assert e.value.code == -9
    t.close()
