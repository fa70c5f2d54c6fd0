"""The continuous-batching loop (serving.py) on the device.

Each job's result must be the same alone and in a mix (bit for bit: its
chain depends only on its own key, temperature, sweep schedule and launch
shape), admission must respect the HBM budget, and a Poisson stream must
complete with latencies recorded.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    from paper_2103_03517_amd import serving
    assert torch.cuda.is_available()
    return serving


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _mix(S, seed=5):
    kw = dict(equil=60, samples=120, block=40, seed=seed)
    return [S.Job(16, 0.9, instance=0, arrival=0.00, **kw),
            S.Job(24, 0.4, instance=1, arrival=0.00, **kw),
            S.Job(32, 1.3, instance=2, arrival=0.02, **kw),
            S.Job(16, 1.6, instance=3, arrival=0.03, **kw),
            S.Job(24, 0.2, instance=4, arrival=0.05, **dict(kw, equil=20, samples=200)),
            S.Job(0, 0.3, instance=5, arrival=0.01, kind="wall", shape=(8, 8, 64), Ku=0.05, seed=seed,
                  equil=100, samples=160, block=40),
            S.Job(12, 0.6, instance=6, arrival=0.01, kind="aniso", Kc=0.05, theta=30.0, phi=45.0, **kw),
            S.Job(0, 0.8, instance=7, arrival=0.02, kind="film", shape=(24, 16, 3), diameter=5.0, **kw)]


def test_lattice_on_another_stream_takes_that_streams_memory(S):
    """A lattice on a stream other than torch's current one allocates its
    workspace from that stream's pool: a block just freed on the current
    stream (whose queued work may still use it) is not handed to it.  Its
    spins then equal those of the same lattice made on the current stream."""
    import torch
    import paper_2103_03517_amd as H
    kw = dict(precision=64, J=1.0, Ku=0.02, seed=3, init="random")
    nbytes = H.workspace_bytes(H.make_params(24, 16, 12, **kw))
    ref = H.Lattice(24, 16, 12, **kw)
    ref.sweep(0.7, 5)
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    x.fill_(0xAB)                        # work queued on the current stream
    freed = x.data_ptr()
    del x
    side = torch.cuda.Stream()
    g = H.Lattice(24, 16, 12, stream=side, **kw)
    assert g.workspace.data_ptr() != freed
    g.sweep(0.7, 5)
    torch.cuda.synchronize()
    assert np.array_equal(g.spins(), ref.spins())
    g.close()
    ref.close()


@pytest.mark.parametrize("precision", [32, 64])
def test_result_same_alone_and_in_mix(S, precision):
    shapes = {(16,) * 3: (1, 4), (24,) * 3: (2, 8), (32,) * 3: (1, 16)}
    mixed = S.Server(precision=precision, quantum=30, shapes=shapes).run(_mix(S))
    assert len(mixed) == 8
    assert {j.kind for j in mixed} == {"mt", "wall", "aniso", "film"}
    for j in mixed:
        alone_job = [x for x in _mix(S) if x.instance == j.instance][0]
        alone = S.Server(precision=precision, quantum=7, shapes=shapes).run([alone_job])[0]
        assert alone.result == j.result, (j.name, alone.result, j.result)
        assert j.result["sweeps"] == j.total
    _say("alone == in mix for", [j.name for j in mixed])


def test_admission_respects_the_hbm_budget(S):
    srv0 = S.Server(precision=32)
    one = srv0.need_bytes(S.Job(24, 1.0))
    jobs = [S.Job(24, 0.5 + 0.2 * i, equil=20, samples=40, block=20, instance=i) for i in range(3)]
    srv = S.Server(precision=32, hbm_budget=one + one // 2, quantum=10)
    done = srv.run(jobs, realtime=False)
    assert len(done) == 3 and srv.stats["max_active"] == 1
    assert srv.stats["max_bytes"] <= one + one // 2
    ref = S.Server(precision=32, quantum=10).run(
        [S.Job(24, 0.5 + 0.2 * i, equil=20, samples=40, block=20, instance=i) for i in range(3)])
    for a, b in zip(sorted(done, key=lambda j: j.instance), sorted(ref, key=lambda j: j.instance)):
        assert a.result == b.result
    with pytest.raises(ValueError):
        S.Server(precision=32, hbm_budget=one // 2).run([S.Job(24, 1.0)])


def test_poisson_stream_completes_with_latencies(S):
    jobs = S.poisson_jobs(rate=40.0, seconds=0.5, edges=(16, 24, 32), equil=40, samples=80, block=40)
    srv = S.Server(precision=32, quantum=20)
    done = srv.run(jobs)
    assert len(done) == len(jobs) > 5
    summ = S.latency_summary(done)
    _say(summ, srv.stats)
    assert 0 < summ["p50_s"] <= summ["p99_s"] <= summ["max_s"]
    for j in done:
        assert j.arrival <= j.admitted <= j.finished
        assert j.result["sweeps"] == j.total
    assert srv.stats["max_active"] >= 2       # requests overlapped on the device


def test_wall_job_width_at_low_temperature(S):
    """A wall job at T = 0.05 (Ku = 0.05, 16x16x128 anti-periodic along z)
    reports the width pi sqrt(J/(2 Ku)) of the continuum wall within 6%."""
    from paper_2103_03517_amd import walls as W
    job = S.Job(0, 0.05, kind="wall", shape=(16, 16, 128), Ku=0.05, equil=1500, samples=1000, block=100)
    done = S.Server(precision=32, quantum=100).run([job])
    r = done[0].result
    d0 = W.zero_temperature_width(1.0, 0.05)
    _say("wall width", r["delta"], "continuum", d0, "fits", r["wall_fits"])
    assert r["wall_fits"] == 10
    assert abs(r["delta"] / d0 - 1) < 0.06
    assert r["m_wall"] > 0.95


def test_fp64_served_jobs_match_reference(S):
    """FP64 jobs of three kinds served together (an m(T) job in the batch, a
    constrained anisotropy job and a granular film swept alone) end where the
    CPU reference ends after the same sweep schedule: the accumulators of the
    last snapshot equal the reference's averages."""
    from oracle import oracle as O
    from paper_2103_03517_amd import films as F
    kw = dict(equil=30, samples=60, block=20, seed=13)
    jobs = [S.Job(8, 0.7, instance=0, **kw),
            S.Job(8, 0.5, instance=1, kind="aniso", Kc=0.05, theta=40.0, phi=45.0, **kw),
            S.Job(0, 0.9, instance=2, kind="film", shape=(12, 10, 3), diameter=4.0, **kw)]
    done = S.Server(precision=64, quantum=7).run(jobs)
    assert len(done) == 3
    for j in sorted(done, key=lambda j: j.instance):
        last = j.reads[-1]
        if j.kind == "mt":
            o = O.OracleLattice(*j.shape, J=1.0, Ku=j.Ku, eu=(0, 0, 1), seed=j.seed, instance=j.instance,
                                init="aligned")
            o.sweep(j.T, j.equil)
            o.sweep(j.T, j.samples, sample=True)
        elif j.kind == "aniso":
            o = O.OracleLattice(*j.shape, J=1.0, Kc=j.Kc, seed=j.seed, instance=j.instance, init="aligned",
                                init_dir=j.e_c())
            o.constrained_sweep(j.T, j.e_c(), j.equil)
            o.constrained_sweep(j.T, j.e_c(), j.samples, sample=True)
        else:
            o = O.OracleLattice(*j.shape, J=1.0, Ku=j.Ku, eu=(0, 0, 1), seed=j.seed, instance=j.instance,
                                init="aligned", boundary_z="open")
            g, _ = F.voronoi_grains(j.shape[0], j.shape[1], j.diameter, j.grain_seed)
            o.set_bond_masks(F.grain_bond_masks(g, j.shape[2]))
            o.sweep(j.T, j.equil)
            o.sweep(j.T, j.samples, sample=True)
        ref = o.observables(j.T)
        _say(j.kind, "served <|m|>", last["mean_m"][0], "reference", ref["mean_m"][0])
        assert last["sweeps_done"] == j.total and last["samples"] == j.samples
        assert last["theta_deg"] == o.counters()[0]
        assert np.allclose(last["mean_m"], ref["mean_m"], rtol=1e-11, atol=1e-13), j.kind
        assert abs(last["mean_E"] - ref["mean_E"]) < 1e-11 * max(1.0, abs(ref["mean_E"])), j.kind
        assert abs(last["mean_Eanis"] - ref["mean_Eanis"]) < 1e-12, j.kind
        if j.kind == "aniso":
            assert np.allclose(last["mean_torque"], ref["mean_torque"], rtol=1e-9, atol=1e-12)
            assert j.result["se_g"] >= 0 and abs(j.result["g"] + np.dot(ref["mean_torque"],
                                                                        [-np.sin(np.pi / 4), np.cos(np.pi / 4), 0])) < 1e-9
