"""GPU full-GR step (PIC_GR_ALPHA: the lapse alpha in Maxwell's equations and the
equation of motion) against the CPU oracle, through the C ABI: bit-identical.

The reading is stated in pcpic.h and pinned on the CPU (test_oracle_gr.py); the
GPU evaluates the same expressions in the same order, so the two must agree to
the last bit, as the flat FP64 path does.
"""
import numpy as np
import pytest

from gpu_common import assert_state_equal, make_pair, say
from paper_1011_6330_amd import synth

pytestmark = pytest.mark.gpu

GR_ALPHA = 8
GR = dict(rho_kind=synth.RHO_GR, incl=0.5, theta_star=0.67 * 0.014, rg_over_rstar=0.4)


def test_gr_alpha_cold_start_bit_identical():
    """Cold SCLF start of the eq. (6) tube with the lapse, 1500 steps: the GR Poisson
    start, the alpha-weighted leap-frog, the GR push and the surface-field rule."""
    cfg = dict(synth.preset("c1"), kappa=0.15, r_star=10.0, flags=GR_ALPHA, **GR)
    say("gr alpha cold start", cfg["n_cells"], "cells")
    g, o = make_pair(cfg)
    for s in range(3):
        g.step(500)
        o.step(500)
        assert_state_equal(g, o, what=f"gr alpha cold start step {500 * (s + 1)}")
    d = g.diagnostics(gauss=True)
    G, gmax = o.gauss()
    assert np.array_equal(d["gauss"], G) and d["gauss_max"] == gmax
    assert d["n_injected"] > 0 and np.abs(d["b_phi"]).max() > 0
    g.close()


@pytest.mark.parametrize("steady", [False, True])
def test_gr_alpha_warm_beam_sorted_bit_identical(steady):
    """A warm beam in the eq. (6) tube with the lapse, sorted every 16 steps (with and
    without the steady B start): 120 steps, every result bit-identical."""
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0, warm=30 * N,
               capacity=int(30 * N * 1.3), sort_every=16, flags=GR_ALPHA | (4 if steady else 0), **GR)
    x, u = synth.warm_start(cfg)
    say("gr alpha warm beam", N, len(x), "steady", steady)
    g, o = make_pair(cfg, x, u)
    d = g.diagnostics()
    assert np.array_equal(d["ez"], o.ez) and np.array_equal(d["er"], o.er) and np.array_equal(d["b_phi"], o.b)
    g.step(120)
    o.step(120)
    assert_state_equal(g, o, ordered=False, what=f"gr alpha warm beam steady={steady}")
    g.close()


def test_gr_alpha_c2_full_size_first_steps():
    """The frame-dragging tube at full size (65,536 cells, ~4e7 particles) with the
    lapse: every result after 3 steps bit-identical to the oracle."""
    cfg = dict(synth.preset("c2"), flags=GR_ALPHA, rg_over_rstar=0.4)
    x, u = synth.warm_start(cfg)
    say("gr alpha c2 full size", len(x))
    g, o = make_pair(cfg, x, u)
    del x, u
    g.step(3)
    o.step(3)
    d = assert_state_equal(g, o, what="gr alpha c2 full size")
    assert d["n_alive"] > 3.9e7
    g.close()


@pytest.mark.parametrize("rg", [0.05, 0.95])
def test_gr_alpha_strong_and_weak_lapse_bit_identical(rg):
    """The lapse at r_g/R_* = 0.05 and 0.95 (alpha^2 down to 0.05 at the surface): a
    sorted warm beam, 80 steps, every result bit-identical to the oracle."""
    N = 2048
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(300.0), ppc=30.0, warm=30 * N,
               capacity=int(30 * N * 1.3), sort_every=16, flags=GR_ALPHA, rg_over_rstar=rg)
    x, u = synth.warm_start(cfg)
    say("gr alpha lapse", rg, N, len(x))
    g, o = make_pair(cfg, x, u)
    g.step(80)
    o.step(80)
    assert_state_equal(g, o, ordered=False, what=f"gr alpha r_g/R_* = {rg}")
    g.close()


def test_gr_alpha_zero_rg_equals_flat_on_gpu():
    """r_g = 0: the GR kernels give the flat step's bits (200 steps of the C1 tube)."""
    cfg = dict(synth.preset("c1"), rho_kind=synth.RHO_FRAME_DRAG, kappa=0.15, r_star=10.0)
    from paper_1011_6330_amd import Tube
    a = Tube(synth.tube_params(dict(cfg, flags=GR_ALPHA, rg_over_rstar=0.0)))
    b = Tube(synth.tube_params(cfg))
    a.step(200)
    b.step(200)
    da, db = a.diagnostics(j=True), b.diagnostics(j=True)
    for k in ("ez", "er", "b_phi", "j_last"):
        assert np.array_equal(da[k], db[k]), k
    xa, ua = a.read_particles()
    xb, ub = b.read_particles()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
    a.close()
    b.close()


def test_gr_alpha_rejected_where_not_built():
    """PIC_GR_ALPHA with FP32-bulk, in a batch, or for the adjoint: PIC_EINVAL."""
    from paper_1011_6330_amd import Batch, PicError, Tube
    cfg = dict(synth.preset("c1"), flags=GR_ALPHA, **GR)
    with pytest.raises(PicError) as e:
        Tube(dict(synth.tube_params(cfg), precision=1))
    assert e.value.code == -1
    with pytest.raises(PicError) as e:
        Batch([synth.tube_params(cfg), synth.tube_params(cfg)])
    assert e.value.code == -1
    t = Tube(synth.tube_params(dict(cfg, sort_every=0)))
    with pytest.raises(PicError) as e:
        t.adjoint_forward(10, 5)
    assert e.value.code == -1
    t.close()
