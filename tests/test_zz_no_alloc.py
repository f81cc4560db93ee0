"""pic_profile_noalloc -- the entry point for callers that cannot allocate --
against pic_diagnostics' profile, through the C ABI: bit for bit, on two calls
in a row (the second with a smaller tube and fewer bins, so that it must clear
what the first left in the fixed scratch), in FP64 and FP32-bulk, and the size
limit of the scratch."""
import ctypes

import numpy as np
import pytest

from gpu_common import say
from paper_1011_6330_amd import synth

pytestmark = pytest.mark.gpu


def _noalloc(t, nb):
    """Call the C ABI with torch device outputs allocated here (the caller's)."""
    import torch
    dev = t.device
    outs = dict(prof_count=torch.zeros(nb, dtype=torch.int64, device=dev),
                prof_sum_lo=torch.zeros(nb, dtype=torch.int64, device=dev),      # uint64 bits
                prof_sum_hi=torch.zeros(nb, dtype=torch.int64, device=dev),
                prof_min=torch.zeros(nb, dtype=torch.float64, device=dev),
                prof_max=torch.zeros(nb, dtype=torch.float64, device=dev))
    torch.cuda.synchronize(dev)
    ptrs = [ctypes.c_void_p(outs[k].data_ptr()) for k in ("prof_count", "prof_sum_lo", "prof_sum_hi",
                                                          "prof_min", "prof_max")]
    rc = t.lib.pic_profile_noalloc(t.handle, nb, *ptrs)
    assert rc == 0, t.lib.pic_last_error().decode()
    t.stream.synchronize()
    res = {k: v.cpu().numpy() for k, v in outs.items()}
    res["prof_sum_lo"] = res["prof_sum_lo"].view(np.uint64)
    return res


def _tube(precision, N, n, a, seed):
    from paper_1011_6330_amd import Tube
    cfg = dict(synth.preset("c2"), n_cells=N, q_over_m=synth.q_over_m_for(a), ppc=max(n / N, 1.0), warm=n,
               capacity=int(n * 1.3) + 4096, sort_every=16, precision=precision, gamma_fp64=1000.0,
               max_bins=4096)
    t = Tube(synth.tube_params(cfg))
    x, u = synth.warm_start(cfg, seed=seed)
    xr, ur = synth.random_particles(N, n // 10, seed=seed)          # some returning (u < 0) particles too
    t.inject(np.concatenate([x, xr]), np.concatenate([u, ur]))
    t.step(20)
    return t


def _same(d, r, what):
    for k in ("prof_count", "prof_sum_lo", "prof_sum_hi", "prof_min", "prof_max"):
        assert np.array_equal(d[k], r[k]), f"{what}: {k} differs"


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_profile_matches_diagnostics_twice(precision):
    big = _tube(precision, 8192, 600_000, 800.0, 1)
    small = _tube(precision, 1000, 20_000, 120.0, 2)
    say("noalloc profile, precision", precision)
    for t, nb, what in ((big, 2000, "first call, 2000 bins"), (small, 37, "second call, smaller tube, 37 bins")):
        r = _noalloc(t, nb)
        d = t.diagnostics(n_bins=nb, fields=False)
        _same(d, r, what)
        assert r["prof_count"].sum() == d["n_alive"]
        assert np.isinf(r["prof_min"][r["prof_count"] == 0]).all()
    big.close()
    small.close()


def test_noalloc_profile_limits():
    from paper_1011_6330_amd import Tube
    t = Tube(synth.tube_params(synth.preset("c1")))
    rc = t.lib.pic_profile_noalloc(t.handle, 65537, None, None, None, None, None)
    assert rc == -1 and b"65536" in t.lib.pic_last_error()
    assert t.lib.pic_profile_noalloc(t.handle, 0, None, None, None, None, None) == -1
    assert t.lib.pic_profile_noalloc(t.handle, 65536, None, None, None, None, None) == 0   # outputs skipped
    t.sync()
    t.close()
