"""Host-side logic of the measurement protocols (no GPU)."""
import numpy as np

from paper_2103_03517_amd import protocols as P


def test_block_stats_from_cumulative_reads_equal_reset_blocks():
    """Blocks recovered from running sums read at the block ends equal the
    blocks of accumulators reset at each block start."""
    rng = np.random.default_rng(0)
    x = rng.normal(0.5, 0.1, (600, 4))
    e = rng.normal(-3.0, 0.1, 600)
    reads, blocks = [], []
    for b in range(6):
        ns = (b + 1) * 100
        reads.append({"samples": ns, "mean_m": x[:ns].mean(0).tolist(),
                      "var_m": x[:ns].var(0).tolist(), "mean_E": float(e[:ns].mean())})
        xb, eb = x[b * 100:ns], e[b * 100:ns]
        blocks.append({"mean_m": xb.mean(0), "var_m": xb.var(0), "mean_E": float(eb.mean())})
    r1 = P.block_stats_from_reads(reads, 1000, 0.7)
    r2 = P._block_stats(blocks, 1000, 0.7)
    assert np.allclose(r1["m"], r2["m"], rtol=1e-12)
    assert np.allclose(r1["se_m"], r2["se_m"], rtol=1e-8)
    assert np.allclose(r1["chi"], r2["chi"], rtol=1e-8)
    assert abs(r1["E"] - r2["E"]) < 1e-12
    # whole-window variance = mean within-block variance + variance of block means
    assert np.allclose(np.asarray(r1["chi"]) * 0.7 / 1000, x.var(0), rtol=1e-9)


def test_batched_workload_recipe():
    jobs = P.c4_jobs()
    assert len(jobs) == 64 and jobs == P.c4_jobs()
    edges = {e for e, _ in jobs}
    assert edges <= {48, 64, 80, 96, 128} and len(edges) == 5
    assert all(0.05 <= t < 1.7 for _, t in jobs)
    assert P.c4_jobs(seed=5) != jobs


def test_compare_precisions_units():
    a = [{"edge": 8, "T": 1.0, "m": [0.5, 0, 0, 0.5], "se_m": [3e-4, 0, 0, 4e-4], "E": -2.0, "se_E": 1e-4}]
    b = [{"edge": 8, "T": 1.0, "m": [0.5005, 0, 0, 0.5], "se_m": [4e-4, 0, 0, 3e-4], "E": -2.0001,
          "se_E": 1e-4}]
    r = P.compare_precisions(a, b)[0]
    assert abs(r["dm"] - 5e-4) < 1e-12
    assert abs(r["dm_over_se"] - 1.0) < 1e-9
    assert abs(r["dE_over_se"] - 1e-4 / np.hypot(1e-4, 1e-4)) < 1e-9


def test_serving_job_schedule_and_stream():
    from paper_2103_03517_amd import serving as S
    j = S.Job(16, 1.0, equil=30, samples=100, block=25)
    assert j.total == 130 and not j.sampling() and j.next_event() == 30
    j.done = 30
    assert j.sampling() and j.next_event() == 25
    j.done = 42
    assert j.next_event() == 13
    import pytest
    with pytest.raises(ValueError):
        S.Job(16, 1.0, samples=90, block=25)
    a = S.poisson_jobs(rate=20, seconds=10)
    b = S.poisson_jobs(rate=20, seconds=10)
    assert [(x.edge, x.T, x.arrival) for x in a] == [(x.edge, x.T, x.arrival) for x in b]
    assert 150 < len(a) < 250
    gaps = np.diff([0.0] + [x.arrival for x in a])
    assert abs(gaps.mean() - 1 / 20) < 0.015
    assert {x.instance for x in a} == set(range(len(a)))
