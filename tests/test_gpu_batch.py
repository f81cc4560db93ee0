"""Batched tubes (one graph launch per round) vs the oracle
and vs the same tubes stepped alone."""
import numpy as np
import pytest

from gpu_common import assert_state_equal, say
from paper_1011_6330_amd import synth

pytestmark = pytest.mark.gpu


def _mixed_tubes(precision, sort_every=8):
    """Six tubes of uneven size and load: warm beams, random particles, an empty tube."""
    specs = [(500, 0, "empty"), (1024, 3000, "random"), (3000, 40000, "warm"), (2048, 20000, "random"),
             (777, 5000, "warm"), (4096, 60000, "warm")]
    cfgs, loads = [], []
    for k, (N, n, kind) in enumerate(specs):
        c = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(0.9 * N / 10.0), ppc=max(n, 1) / N,
                 warm=n, capacity=int(n * 1.5) + 4096, sort_every=sort_every, kappa=0.05 + 0.03 * k,
                 rho_amp=0.5 + 0.4 * k, precision=precision)
        if kind == "empty":
            c["ppc"] = 4.0
            x, u = np.zeros(0), np.zeros(0)
        elif kind == "random":
            x, u = synth.random_particles(N, n, seed=k)
        else:
            x, u = synth.warm_start(c, seed=k)
        cfgs.append(c)
        loads.append((x, u))
    return cfgs, loads


def _oracle(c):
    from oracle.oracle import OracleTube
    p = synth.tube_params(c)
    return OracleTube({k: v for k, v in p.items() if k not in ("sort_every", "max_bins", "precision", "gamma_fp64")})


def test_batch_fp64_matches_oracle_per_tube():
    from paper_1011_6330_amd import Batch
    cfgs, loads = _mixed_tubes(precision=0)
    say("batch fp64", len(cfgs), "tubes")
    b = Batch([synth.tube_params(c) for c in cfgs])
    oracles = [_oracle(c) for c in cfgs]
    for t, (x, u) in enumerate(loads):
        if len(x):
            b.tubes[t].inject(x, u)
            oracles[t].inject(x, u)
    for r in range(5):               # five rounds of 8 steps: graph capture, then replays
        b.step(8)
        for o in oracles:
            o.step(8)
        b.sync()
        for t in range(len(cfgs)):
            assert_state_equal(b.tubes[t], oracles[t], ordered=False, what=f"tube {t} round {r}")
    b.close()


@pytest.mark.parametrize("shape", [(64, 2, True), (256, 4, True), (512, 2, False), (128, 2, False)])
def test_batch_shapes_and_graph_identical(shape):
    from paper_1011_6330_amd import Batch
    cfgs, loads = _mixed_tubes(precision=0)
    outs = []
    for cfg_shape in ((256, 2, True), shape):
        b = Batch([synth.tube_params(c) for c in cfgs])
        b.set_config(cfg_shape[0], cfg_shape[1], graph=cfg_shape[2])
        for t, (x, u) in enumerate(loads):
            if len(x):
                b.tubes[t].inject(x, u)
        b.step(37)                   # not a multiple of the sort period: rounds + remainder
        res = []
        for t in range(len(cfgs)):
            d = b.tubes[t].diagnostics(fields=True, j=True)
            px, pu = b.tubes[t].read_particles()
            k = np.lexsort((pu, px))
            res.append((d["ez"], d["er"], d["b_phi"], d["j_last"], px[k], pu[k], d["n_injected"]))
        outs.append(res)
        b.close()
    for ta, tb in zip(outs[0], outs[1]):
        for a, c in zip(ta, tb):
            assert np.array_equal(a, c)


def test_batch_fp32_tube_equals_single_tube():
    """FP32-bulk: every tube of the batch computes what it computes alone.  The
    single tubes step on their own streams while the batch runs, so the batched
    kernel shares the GPU with other kernels."""
    from paper_1011_6330_amd import Batch, Tube
    cfgs = synth.ensemble(n_tubes=5, seed=3, sort_every=16)   # three sorts in 48 steps
    for c in cfgs:                   # keep the test small: 2e4 particles per tube at most
        c["warm"] = min(c["warm"], 20000)
        c["ppc"] = c["warm"] / c["n_cells"]
        c["capacity"] = int(c["warm"] * 1.4) + 4096
    loads = [synth.warm_start(c, seed=t) for t, c in enumerate(cfgs)]
    say("batch fp32", len(cfgs), "tubes")
    b = Batch([synth.tube_params(c) for c in cfgs])
    singles = []
    for t, (x, u) in enumerate(loads):
        b.tubes[t].inject(x, u)
        s = Tube(synth.tube_params(cfgs[t]))
        s.inject(x, u)
        singles.append(s)
    b.step(48)
    for s in singles:
        s.step(48)
    b.sync()
    for t, s in enumerate(singles):
        db = b.tubes[t].diagnostics(fields=True, j=True)
        ds = s.diagnostics(fields=True, j=True)
        for k in ("ez", "er", "b_phi", "j_last"):
            assert np.array_equal(db[k], ds[k]), (t, k)
        for k in ("n_alive", "n_injected", "n_exit", "n_absorb", "exit_sum_lo", "e_surf"):
            assert db[k] == ds[k], (t, k)
        bx, bu = b.tubes[t].read_particles()
        sx, su = s.read_particles()
        kb, ks = np.lexsort((bu, bx)), np.lexsort((su, sx))
        assert np.array_equal(bx[kb], sx[ks]) and np.array_equal(bu[kb], su[ks])
        s.close()
    b.close()


def test_batch_rejects_mixed_precision():
    from paper_1011_6330_amd import Batch, PicError
    a = synth.tube_params(dict(synth.preset("c1"), precision=0))
    c = synth.tube_params(dict(synth.preset("c1"), precision=1))
    with pytest.raises(PicError):
        Batch([a, c])


def test_c3_full_size_sampled_tubes():
    """The whole C3 ensemble (256 tubes, 5.5e7 particles) in FP64 as the bench
    runs it, one 64-step round from its graph plus 16 more steps: the smallest
    tube against the oracle and the largest against the same tube stepped
    alone, bit for bit."""
    from paper_1011_6330_amd import Batch, Tube, autotune
    cfgs = synth.ensemble(n_tubes=256, seed=0, precision=0)
    loads = [synth.warm_start(c, seed=t) for t, c in enumerate(cfgs)]
    say("c3 full size:", sum(len(x) for x, _ in loads), "particles")
    b = Batch([synth.tube_params(c) for c in cfgs])
    for t, (x, u) in enumerate(loads):
        b.tubes[t].inject(x, u)
    autotune.tune_batch(b, steps=8, use_cache=False)      # the bench's shape choice (8-step trials)
    small = min(range(256), key=lambda t: len(loads[t][0]))
    large = max(range(256), key=lambda t: len(loads[t][0]) * cfgs[t]["n_cells"])
    o = _oracle(cfgs[small])
    o.inject(*loads[small])
    s = Tube(synth.tube_params(cfgs[large]))
    s.inject(*loads[large])
    done = b.tubes[0].diagnostics(fields=False)["step"]   # the tuning trials stepped the batch
    b.step((64 - done % 64) % 64 + 64 + 16)                # to the next round boundary, a round, 16 more
    total = b.tubes[0].diagnostics(fields=False)["step"]
    o.step(total)
    s.step(total)
    b.sync()
    say("c3 full size: steps", total, "small tube", small, "large tube", large)
    assert_state_equal(b.tubes[small], o, ordered=False, what=f"tube {small} vs oracle")
    db = b.tubes[large].diagnostics(fields=True, j=True)
    ds = s.diagnostics(fields=True, j=True)
    for k in ("ez", "er", "b_phi", "j_last"):
        assert np.array_equal(db[k], ds[k]), k
    for k in ("n_alive", "n_injected", "n_exit", "exit_sum_lo", "exit_sum_hi", "w0"):
        assert db[k] == ds[k], k
    xb, ub = b.tubes[large].read_particles()
    xs, us = s.read_particles()
    kb, ks = np.lexsort((ub, xb)), np.lexsort((us, xs))
    assert np.array_equal(xb[kb], xs[ks]) and np.array_equal(ub[kb], us[ks])
    s.close()
    b.close()


def test_c3_full_size_fp32_bulk():
    """The whole C3 ensemble as the bench runs it: 256 tubes, 5.5e7 particles,
    FP32-bulk, autotuned launch shape, one 64-step round from its graph plus 16
    more steps.  The smallest tube against the oracle per result (gamma(z), E_z,
    exit gamma, counts, Gauss residual); the largest against the same tube
    stepped alone, bit for bit."""
    from gpu_common import gate_errors, oracle_errors
    from paper_1011_6330_amd import Batch, Tube, autotune
    cfgs = synth.ensemble(n_tubes=256, seed=0, precision=1)
    loads = [synth.warm_start(c, seed=t) for t, c in enumerate(cfgs)]
    say("c3 fp32 full size:", sum(len(x) for x, _ in loads), "particles")
    b = Batch([synth.tube_params(c) for c in cfgs])
    for t, (x, u) in enumerate(loads):
        b.tubes[t].inject(x, u)
    shape = autotune.tune_batch(b, use_cache=False)         # the bench's shape choice
    say("c3 fp32: tuned shape", shape, b.get_config())
    small = min(range(256), key=lambda t: len(loads[t][0]))
    large = max(range(256), key=lambda t: len(loads[t][0]) * cfgs[t]["n_cells"])
    o = _oracle(cfgs[small])
    o.inject(*loads[small])
    s = Tube(synth.tube_params(cfgs[large]))
    s.inject(*loads[large])
    done = b.tubes[0].diagnostics(fields=False)["step"]   # the tuning trials stepped the batch
    b.step((64 - done % 64) % 64 + 64 + 16)                # to the next round boundary, a round, 16 more
    total = b.tubes[0].diagnostics(fields=False)["step"]
    o.step(total)
    s.step(total)
    b.sync()
    say("c3 fp32: steps", total, "small tube", small, "large tube", large)
    err = oracle_errors(b.tubes[small], o)
    gate_errors(err, f"c3 fp32 tube {small} vs oracle")
    db = b.tubes[large].diagnostics(fields=True, j=True)
    ds = s.diagnostics(fields=True, j=True)
    for k in ("ez", "er", "b_phi", "j_last"):
        assert np.array_equal(db[k], ds[k]), k
    for k in ("n_alive", "n_slots_high", "n_injected", "n_exit", "exit_sum_lo", "exit_sum_hi", "w0", "e_surf"):
        assert db[k] == ds[k], k
    xb, ub = b.tubes[large].read_particles()
    xs, us = s.read_particles()
    kb, ks = np.lexsort((ub, xb)), np.lexsort((us, xs))
    assert np.array_equal(xb[kb], xs[ks]) and np.array_equal(ub[kb], us[ks])
    s.close()
    b.close()
