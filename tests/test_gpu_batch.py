"""Batches of lattices (hmc_batch_*) through the C interface.

A lattice advanced inside a batch must end bit for bit where the same
lattice ends when swept alone with the same launch shape: spins, cone
angle, sweep counter, acceptance count and FP64 accumulators (the state
image compares all of them).  FP64 lattices of a batch are also matched to
the CPU reference spin by spin.  Graph replays must equal eager launches,
and the autotuner must leave the chains where they were.
"""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12

# (shape, sites per thread, z chunk): uneven sizes, several kernel variants
# (1, 2 and 4 sites per thread; one and two halo slots) and ragged tiles
MIX = [((8, 8, 8), 1, 4), ((6, 10, 4), 2, 3), ((16, 16, 16), 4, 8), ((34, 6, 4), 1, 16),
       ((12, 2, 2), 2, 1), ((40, 18, 6), 2, 4), ((2, 2, 2), 1, 1), ((600, 2, 2), 1, 2)]


@pytest.fixture(scope="module")
def H():
    import paper_2103_03517_amd as H
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    H.lib()
    return H


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _make(H, precision, mix=MIX, seed0=50):
    out = []
    for i, (shape, spt, zc) in enumerate(mix):
        kw = dict(inputs.random_params(seed0 + i), seed=seed0 + 7 * i, instance=i, theta0_deg=20 + i)
        g = H.Lattice(*shape, precision=precision, init="random", **kw)
        g.set_launch(spt, zc)
        out.append(g)
    return out


def _temps(n, seed=3):
    return np.random.default_rng(seed).uniform(0.3, 1.6, n)


def _schedule():
    # (n_sweeps, sample): unsampled, sampled, unsampled again
    return [(3, False), (5, True), (2, False), (4, True)]


@pytest.mark.parametrize("precision", [64, 32])
def test_batch_equals_single_runs(H, precision):
    _say("batch vs single", precision)
    T = _temps(len(MIX))
    alone = _make(H, precision)
    inb = _make(H, precision)
    B = H.Batch(inb)
    for n, smp in _schedule():
        B.sweep(T, n, sample=smp)
        for g, t in zip(alone, T):
            g.sweep(t, n, sample=smp)
    for i, (a, b) in enumerate(zip(alone, inb)):
        assert a.get_state() == b.get_state(), (precision, MIX[i])
    # batch observables equal the per-lattice ones
    obs = B.observables()
    for a, ob in zip(alone, obs):
        oa = a.observables()
        oa.pop("status")
        assert oa == ob
        assert ob["sweeps_done"] == 14 and ob["samples"] == 9
    # the batch reset equals the per-lattice reset
    B.reset_stats()
    B.sweep(T, 3, sample=True)
    for g, t in zip(alone, T):
        g.reset_stats()
        g.sweep(t, 3, sample=True)
    for i, (a, b) in enumerate(zip(alone, inb)):
        assert a.get_state() == b.get_state(), ("after reset", MIX[i])
        assert b.observables()["samples"] == 3
    B.close()


def test_batch_many_record_groups_equals_single(H):
    """Lattices whose passes write more than 1024 work-group records end bit
    for bit the same in a batch, whose finalize forms the group sums one
    after the other, as alone, where fold_groups_kernel forms them in
    parallel: 96^3 with 256-site tiles and one-plane chunks writes 1728
    records (two groups) and, in FP32, 256^3 likewise 32768 (32 groups)."""
    _say("batch vs single, several record groups")
    for precision in (64, 32):
        shapes = [((96, 96, 96), 1, 1), ((16, 16, 16), 2, 4)]
        if precision == 32:
            shapes.append(((256, 256, 256), 1, 1))
        T = [0.8, 1.1, 1.3][:len(shapes)]
        alone = _make(H, precision, mix=shapes, seed0=90)
        inb = _make(H, precision, mix=shapes, seed0=90)
        B = H.Batch(inb)
        for n, smp in [(2, False), (3, True), (1, False), (2, True)]:
            B.sweep(T, n, sample=smp)
            for g, t in zip(alone, T):
                g.sweep(t, n, sample=smp)
        for i, (a, b) in enumerate(zip(alone, inb)):
            assert a.get_state() == b.get_state(), (precision, shapes[i])
        for a, ob in zip(alone, B.observables()):
            oa = a.observables()
            oa.pop("status")
            assert oa == ob, precision
        B.close()
        for g in alone + inb:
            g.close()


def test_per_lattice_sample_flags(H):
    """Lattices in different phases (some sampling, some not) in one batch
    equal the same lattices swept alone with their own flags."""
    T = _temps(len(MIX), seed=4)
    alone = _make(H, 32, seed0=60)
    inb = _make(H, 32, seed0=60)
    B = H.Batch(inb)
    flags = [[i % 2 == 0 for i in range(len(MIX))], [i % 3 == 0 for i in range(len(MIX))],
             [False] * len(MIX), [True] * len(MIX)]
    for k, f in enumerate(flags):
        B.sweep_each(T, f, 3 + k)
        for g, t, smp in zip(alone, T, f):
            g.sweep(t, 3 + k, sample=smp)
    for i, (a, b) in enumerate(zip(alone, inb)):
        assert a.get_state() == b.get_state(), MIX[i]
    B.close()


def test_batch_fp64_matches_reference(H):
    from oracle import oracle as O
    O.lib()
    mix = [((8, 8, 8), 2, 4), ((6, 10, 4), 1, 2), ((12, 2, 2), 4, 1), ((34, 6, 4), 1, 3)]
    T = _temps(len(mix), seed=9)
    gs, os_ = [], []
    for i, (shape, spt, zc) in enumerate(mix):
        kw = dict(inputs.random_params(70 + i), seed=900 + i, instance=11 + i, theta0_deg=30)
        n = shape[0] * shape[1] * shape[2]
        S = inputs.random_unit_spins(n, 400 + i)
        g = H.Lattice(*shape, precision=64, **kw)
        g.set_spins(S)
        g.set_launch(spt, zc)
        o = O.OracleLattice(*shape, **kw)
        o.set_spins(S)
        gs.append(g)
        os_.append(o)
    B = H.Batch(gs)
    worst = 0.0
    for s in range(12):
        B.sweep(T, 1)
        for g, o, t in zip(gs, os_, T):
            acc = o.sweep(t)
            ob = g.observables()
            theta, sweeps = o.counters()
            d = float(np.abs(g.spins() - o.spins()).max())
            worst = max(worst, d)
            assert ob["theta_deg"] == theta and ob["sweeps_done"] == sweeps
            assert ob["accepted_last"] == acc
            assert d <= TOL, (s, d)
    _say("batch fp64 vs reference: worst", worst)


@pytest.mark.parametrize("chunk", [0, 20000])
def test_graph_replay_equals_eager(H, chunk):
    """Graph replay of every call gives the eager states, also when the batch
    is swept in chunks (one graph per chunk and sample flag), as the bench's
    batch leg runs it."""
    T = _temps(len(MIX), seed=5)
    eager = _make(H, 32, seed0=80)
    graph = _make(H, 32, seed0=80)
    Be, Bg = H.Batch(eager), H.Batch(graph)
    Be.set_chunk_bytes(chunk)
    Bg.set_chunk_bytes(chunk)
    Bg.set_graph(3)
    for rep, (n, smp) in enumerate([(7, False), (6, True), (3, True), (5, False)]):
        Be.sweep(T, n, sample=smp)
        Bg.sweep(T, n, sample=smp)
        # eager work of the program between replays (a measurement refreshes
        # the instantaneous M and E kept in the state, so both sides do it)
        for g in graph + eager:
            g.observables()
        for i, (a, b) in enumerate(zip(eager, graph)):
            assert a.get_state() == b.get_state(), (rep, MIX[i])
    Be.close()
    Bg.close()


def test_tune_restores_chains_and_results_do_not_move(H):
    T = _temps(len(MIX), seed=6)
    gs = _make(H, 32, seed0=120)
    B = H.Batch(gs)
    B.sweep(T, 4, sample=True)
    before = [g.get_state() for g in gs]
    shapes = B.tune(T, trial_sweeps=2)
    _say("tuned shapes", shapes)
    assert [g.get_state() for g in gs] == before
    for (spt, zc), g in zip(shapes, gs):
        assert spt in (1, 2, 4) and 1 <= zc <= 64
    # continuing in the batch with the tuned shapes equals continuing alone
    alone = _make(H, 32, seed0=120)
    for a, g, (spt, zc) in zip(alone, gs, shapes):
        a.set_state(g.get_state())
        a.set_launch(spt, zc)
    B.sweep(T, 5, sample=True)
    for a, t in zip(alone, T):
        a.sweep(t, 5, sample=True)
    for a, g in zip(alone, gs):
        assert a.get_state() == g.get_state()


def test_launch_change_and_mixed_use(H):
    """A launch shape changed after the batch was built is picked up, and a
    lattice swept alone between batch sweeps stays consistent."""
    T = _temps(len(MIX), seed=8)
    alone = _make(H, 64, seed0=160)
    inb = _make(H, 64, seed0=160)
    B = H.Batch(inb)
    B.sweep(T, 2)
    inb[2].set_launch(1, 2)
    alone[2].set_launch(1, 2)
    B.sweep(T, 3, sample=True)
    inb[0].sweep(0.9, 2)
    B.sweep(T, 1, sample=True)
    for g, t in zip(alone, T):
        g.sweep(t, 2)
        g.sweep(t, 3, sample=True)
    alone[0].sweep(0.9, 2)
    for g, t in zip(alone, T):
        g.sweep(t, 1, sample=True)
    for a, b in zip(alone, inb):
        assert a.get_state() == b.get_state()


def test_set_lattices_reuses_the_batch(H):
    """Swapping lattices in and out of one batch (up to its capacity) gives
    the results of sweeping them alone."""
    T = _temps(len(MIX), seed=12)
    alone = _make(H, 32, seed0=200)
    inb = _make(H, 32, seed0=200)
    B = H.Batch(inb[:2], capacity=5)
    B.sweep(T[:2], 3)
    B.set_lattices([inb[2], inb[0], inb[5], inb[6]])
    B.sweep([T[2], T[0], T[5], T[6]], 4, sample=True)
    B.set_lattices([inb[1]])
    B.sweep([T[1]], 2)
    for i, n, smp in [(0, 3, False), (1, 3, False), (2, 4, True), (0, 4, True), (5, 4, True), (6, 4, True),
                      (1, 2, False)]:
        alone[i].sweep(T[i], n, sample=smp)
    for i in (0, 1, 2, 5, 6):
        assert alone[i].get_state() == inb[i].get_state(), MIX[i]
    with pytest.raises(H.HmcError) as e:
        B.set_lattices(inb[:6])
    assert e.value.status == H.ENOMEM
    B.close()


@pytest.mark.parametrize("chunk", [0, 1, 20000])
def test_chunking_does_not_change_results(H, chunk):
    """Chunk sizes from one lattice per chunk to a few: every lattice ends
    bit for bit where it ends alone; graph replays per chunk as well."""
    T = _temps(len(MIX), seed=13)
    alone = _make(H, 32, seed0=240)
    inb = _make(H, 32, seed0=240)
    B = H.Batch(inb)
    B.set_chunk_bytes(chunk)
    B.sweep(T, 5)
    B.set_graph(2)
    B.sweep(T, 5, sample=True)
    for g, t in zip(alone, T):
        g.sweep(t, 5)
        g.sweep(t, 5, sample=True)
    for i, (a, b) in enumerate(zip(alone, inb)):
        assert a.get_state() == b.get_state(), (chunk, MIX[i])
    B.close()


def test_wall_initial_state(H):
    """init = "wall" writes the T = 0 profile on the device."""
    from paper_2103_03517_amd import walls as W
    shape, w = (4, 6, 40), 9.5
    g = H.Lattice(*shape, precision=64, init="wall", init_width=w, boundary_z="antiperiodic")
    assert np.allclose(g.spins(), W.initial_wall(*shape, width=w), rtol=0, atol=1e-14)


def test_batch_argument_errors(H):
    import ctypes
    g32 = H.Lattice(4, 4, 4, precision=32)
    g64 = H.Lattice(4, 4, 4, precision=64)
    h32 = H.Lattice(6, 4, 4, precision=32)
    with pytest.raises(H.HmcError) as e:
        H.Batch([g32, g64])
    assert e.value.status == H.EINVAL
    with pytest.raises(H.HmcError) as e:
        H.Batch([g32, h32, g32])
    assert e.value.status == H.EINVAL
    with pytest.raises(H.HmcError) as e:
        H.Batch([g32, H.Lattice(4, 4, 4, precision=32, bond_masks=True)])
    assert e.value.status == H.EINVAL
    B = H.Batch([g32, h32])
    for bad in ([1.0, 0.0], [1.0, float("nan")], [-1.0, 1.0], [1.0, float("inf")]):
        with pytest.raises(H.HmcError) as e:
            B.sweep(bad, 1)
        assert e.value.status == H.EINVAL
    with pytest.raises(H.HmcError):
        B.sweep([1.0, 1.0], -1)
    with pytest.raises(H.HmcError):
        B.set_graph(-1)
    with pytest.raises(H.HmcError):
        B.tune([1.0, 1.0], trial_sweeps=0)
    B.sweep([1.0, 1.0], 0)
    # workspace too small or misaligned
    L = H.lib()
    import torch
    n = int(L.hmc_batch_workspace_bytes(2))
    ws = torch.empty(n + 512, dtype=torch.uint8, device="cuda")
    hs = (ctypes.c_void_p * 2)(g32._h, h32._h)
    out = ctypes.c_void_p()
    assert L.hmc_batch_create(hs, 2, ctypes.c_void_p(ws.data_ptr()), n - 1, ctypes.byref(out)) == H.ENOMEM
    assert L.hmc_batch_create(hs, 2, ctypes.c_void_p(ws.data_ptr() + 8), n, ctypes.byref(out)) == H.ENOMEM
    assert L.hmc_batch_create(hs, 0, ctypes.c_void_p(ws.data_ptr()), n, ctypes.byref(out)) == H.EINVAL
    B.close()
