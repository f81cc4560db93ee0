"""Helpers shared by the GPU tests: build a GPU tube and an oracle tube from the
same config and the same seeded particle load, and compare their states."""
import numpy as np

from paper_1011_6330_amd import synth


def say(*a):
    print("[gpu-test]", *a, flush=True)


def make_pair(cfg, x=None, u=None):
    from oracle.oracle import OracleTube
    from paper_1011_6330_amd import Tube
    p = synth.tube_params(cfg)
    g = Tube(p)
    o = OracleTube({k: v for k, v in p.items() if k not in ("sort_every", "max_bins", "precision", "gamma_fp64")})
    # (macro_charge passes through: the oracle takes the same override)
    if x is not None and len(x):
        g.inject(x, u)
        o.inject(x, u)
    return g, o


def counters_equal(d, o):
    c = o.counters
    mism = {}
    for gk, ok in (("step", "step"), ("n_alive", "n_alive"), ("n_injected", "n_injected"),
                   ("n_exit", "n_exit"), ("n_absorb", "n_absorb"), ("last_n_inj", "last_ninj"),
                   ("w0", "w0"), ("status", "status"), ("exit_sum_lo", "exit_sum_lo"),
                   ("exit_sum_hi", "exit_sum_hi")):
        if d[gk] != c[ok]:
            mism[gk] = (d[gk], c[ok])
    if d["e_surf"] != c["e_surf"]:
        mism["e_surf"] = (d["e_surf"], c["e_surf"])
    return mism


def max_ulp(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.size == 0:
        return 0
    ia = a.view(np.int64).astype(np.int64)
    ib = b.view(np.int64).astype(np.int64)
    ia = np.where(ia < 0, np.int64(-0x8000000000000000) - ia, ia)
    ib = np.where(ib < 0, np.int64(-0x8000000000000000) - ib, ib)
    return int(np.abs(ia - ib).max())


def assert_state_equal(g, o, ordered=True, what=""):
    """Bit-identical state: counters, fields, last-step current, particles."""
    d = g.diagnostics(fields=True, j=True)
    mism = counters_equal(d, o)
    assert not mism, f"{what} counters differ: {mism}"
    for k, ok in (("ez", o.ez), ("er", o.er), ("b_phi", o.b)):
        if not np.array_equal(d[k], ok):
            raise AssertionError(f"{what} {k} differs: max ulp {max_ulp(d[k], ok)}, "
                                 f"max abs {np.abs(d[k] - ok).max():.3e}")
    assert np.array_equal(d["j_last"], o.j), f"{what} J differs"
    x, u = g.read_particles()
    ox, ou = o.x.copy(), o.u.copy()
    assert len(x) == len(ox), f"{what} particle count {len(x)} vs {len(ox)}"
    if not ordered:
        kg = np.lexsort((u, x))
        ko = np.lexsort((ou, ox))
        x, u, ox, ou = x[kg], u[kg], ox[ko], ou[ko]
    if not (np.array_equal(x, ox) and np.array_equal(u, ou)):
        raise AssertionError(f"{what} particles differ: x max ulp {max_ulp(x, ox)}, u max ulp {max_ulp(u, ou)}")
    return d
