"""FP32 path against the FP64 path (itself matched to the reference spin by
spin): the same observables within |dm| <= 1e-3 and within 3 combined
batch-means standard errors (chi within 4).  FP32 parity is statistical
only: the chain is chaotic, so FP32 rounding decorrelates the trajectories."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_2103_03517_amd import protocols
    assert torch.cuda.is_available()
    return protocols


@pytest.mark.parametrize("T", [0.3, 0.8, 1.2])
def test_fp32_matches_fp64_statistically(P, T):
    kw = dict(size=64, equil=1000, samples=24000, block=600, init="aligned", Ku=0.005)
    r32 = P.mt_sweep([T], precision=32, seed=11, **kw)[0]
    r64 = P.mt_sweep([T], precision=64, seed=12, **kw)[0]
    print(f"T={T}: m32={r32['m'][0]:.6f}+-{r32['se_m'][0]:.1e} m64={r64['m'][0]:.6f}+-"
          f"{r64['se_m'][0]:.1e} E32={r32['E']:.6f} E64={r64['E']:.6f}", file=sys.stderr, flush=True)
    for a in (0, 3):   # |m| and m_z
        d = abs(r32["m"][a] - r64["m"][a])
        se = math.hypot(r32["se_m"][a], r64["se_m"][a])
        assert d <= 1e-3, (a, d)
        assert d <= 3 * se + 1e-12, (a, d, se)
    d = abs(r32["E"] - r64["E"])
    assert d <= 3 * math.hypot(r32["se_E"], r64["se_E"]) + 1e-12
    d = abs(r32["chi"][0] - r64["chi"][0])
    assert d <= 4 * math.hypot(r32["se_chi"][0], r64["se_chi"][0]), (r32["chi"][0], r64["chi"][0])


def test_block_statistics_match_the_accumulators(P):
    """The block combination reproduces the whole-window mean and variance
    that the device accumulators give for the same sweeps."""
    from paper_2103_03517_amd import Lattice
    g = Lattice(16, 16, 16, precision=64, Ku=0.01, seed=3)
    g.sweep(0.9, 100)
    state = g.get_state()
    blocks = []
    for _ in range(5):
        g.reset_stats()
        g.sweep(0.9, 40, sample=True)
        blocks.append(g.observables())
    r = P._block_stats(blocks, g.n, 0.9)
    g.set_state(state)
    g.reset_stats()
    g.sweep(0.9, 200, sample=True)
    whole = g.observables()
    assert np.allclose(r["m"], whole["mean_m"], rtol=1e-12, atol=1e-14)
    assert np.allclose(r["chi"], whole["chi"], rtol=1e-9, atol=1e-12)
    assert abs(r["E"] - whole["mean_E"]) < 1e-12
