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
    # 40 blocks of 2400 sweeps: blocks much longer than the autocorrelation
    # time of m at these temperatures, so the batch-means errors are honest
    kw = dict(size=64, equil=2000, samples=96000, block=2400, init="aligned", Ku=0.005)
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


def test_batched_fp32_jobs_match_fp64(P):
    """The batched FP32 jobs against the same jobs run as an FP64 batch with
    independent random keys (so the two standard errors add in quadrature):
    every job's m(T) = <|m|> and <E>/N within 3 combined blocking errors, and
    |dm| <= 1e-3 wherever the resolution allows it (3 SE < 1e-3); <m_z> and
    chi_l are printed.  The results are deterministic (keyed random numbers),
    so a pass is a fixed fact of this build, not a draw; with honest errors a
    3 SE gate on 16 comparisons fails by chance for about one key in twenty."""
    jobs = [(32, 0.3), (48, 0.5), (32, 0.6), (48, 0.9), (32, 1.2), (48, 1.3), (32, 1.6), (48, 0.1)]
    kw = dict(equil=1000, samples=24000, block=600)
    r32, _ = P.batched_mt(jobs, 32, tune=False, seed=4, **kw)
    r64, _ = P.batched_mt(jobs, 64, tune=False, seed=5, **kw)
    for c in P.compare_precisions(r32, r64):
        print(c, file=sys.stderr, flush=True)
        assert c["dm_over_se"] <= 3.0, c
        assert c["dE_over_se"] <= 3.0, c
        assert c["pass"], c
