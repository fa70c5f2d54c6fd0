"""Parity of the HIP library (through its C interface) with the CPU reference.

FP64 lattices must match the reference spin by spin within 1e-12 after every
sweep, with identical cone angles and acceptance counts (an accept decision
that differs moves a spin by O(theta), so any divergence is counted).
"""
import sys

import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def H():
    import paper_2103_03517_amd as H
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    H.lib()
    return H


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.lib()
    return O


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(H, O, shape, kw, init="aligned", init_dir=(0, 0, 1), spins=None, precision=64):
    g = H.Lattice(*shape, precision=precision, init=init, init_dir=init_dir, **kw)
    o = O.OracleLattice(*shape, init=init, init_dir=init_dir, **kw)
    if spins is not None:
        g.set_spins(spins)
        o.set_spins(spins)
    return g, o


def _compare_every_sweep(g, o, n, step, what):
    worst = 0.0
    diverged = 0
    for s in range(n):
        acc_o = step(s)
        ob = g.observables()
        theta_o, sweeps_o = o.counters()
        d = np.abs(g.spins() - o.spins())
        worst = max(worst, float(d.max()))
        diverged += int(np.sum(d.max(axis=1) > 1e-9))
        assert ob["sweeps_done"] == sweeps_o, (what, s)
        assert ob["accepted_last"] == acc_o, (what, s, ob["accepted_last"], acc_o)
        assert ob["theta_deg"] == theta_o, (what, s)
        assert diverged == 0, (what, s, diverged)
        assert worst <= TOL, (what, s, worst)
    return worst


SHAPES = [(2, 2, 2), (4, 4, 4), (8, 8, 8), (16, 16, 16), (6, 10, 4), (2, 6, 12),
          (34, 6, 4), (12, 2, 2), (600, 2, 2), (40, 18, 6)]


@pytest.mark.parametrize("prefetch", [1, 2])
@pytest.mark.parametrize("shape", SHAPES)
def test_standard_sweep_fp64_matches_reference(H, O, shape, prefetch):
    """Both marches over z (one or two planes of look-ahead) against the
    reference, spin by spin, every sweep."""
    _say("standard fp64", shape, "prefetch", prefetch)
    kw = dict(inputs.random_params(sum(shape)), seed=1234 + shape[0], instance=3, theta0_deg=25)
    n = shape[0] * shape[1] * shape[2]
    S = inputs.random_unit_spins(n, 99)
    g, o = _pair(H, O, shape, kw, spins=S)
    g.set_prefetch(prefetch)
    assert g.get_prefetch() == prefetch
    T = 0.7

    def step(s):
        g.sweep(T)
        return o.sweep(T)

    _compare_every_sweep(g, o, 100 if n <= 4096 else 30, step, shape)


def test_random_initial_spins_match_reference(H, O):
    _say("random init")
    kw = dict(J=1.0, Ku=0.1, seed=77, instance=5)
    g, o = _pair(H, O, (8, 6, 4), kw, init="random")
    assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    assert np.allclose(np.linalg.norm(g.spins(), axis=1), 1.0, atol=1e-15)


def test_plain_method_16cubed_observables(H, O):
    """16^3 FP64, Ku = 0.01 along z, T = 0.5, aligned start, seed 1: 1000 adaptive
    sweeps, the last 800 sampled; <|m|> and <E>/N equal the reference's."""
    _say("16^3 observables")
    kw = dict(J=1.0, Ku=0.01, eu=(0, 0, 1), seed=1)
    g, o = _pair(H, O, (16, 16, 16), kw)
    T = 0.5
    g.sweep(T, 200)
    o.sweep(T, 200)
    g.sweep(T, 800, sample=True)
    o.sweep(T, 800, sample=True)
    a, b = g.observables(), o.observables(T)
    assert a["samples"] == b["samples"] == 800
    assert a["theta_deg"] == b["theta_deg"]
    assert np.max(np.abs(g.spins() - o.spins())) < 1e-10
    for k in ("mean_m", "mean_E"):
        assert np.allclose(a[k], b[k], rtol=1e-11, atol=1e-13), (k, a[k], b[k])
    for k in ("var_m", "var_E", "chi"):
        assert np.allclose(a[k], b[k], rtol=1e-7, atol=1e-14), (k, a[k], b[k])
    for k in ("E", "E_exch", "E_uni", "E_cub", "E_zee"):
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), k
    assert np.allclose(a["M"], b["M"], rtol=0, atol=1e-9)
    _say("16^3: <|m|> =", a["mean_m"][0], " <E>/N =", a["mean_E"])


def test_many_record_groups_fp64_observables(H, O):
    """More than 1024 work-group records per pass: 96^3 FP64 with 256-site
    tiles and one-plane chunks writes 1728 records, two groups of the
    finalize's fold, whose sums fold_groups_kernel forms in parallel (the
    on-demand measurement also writes 1728).  Spins within 1e-12 after every sweep;
    the sampled means and the measured energies equal the reference's."""
    _say("96^3 fp64, two record groups")
    shape = (96, 96, 96)
    kw = dict(inputs.random_params(7), seed=4321, instance=2, theta0_deg=30)
    S = inputs.random_unit_spins(96 ** 3, 5)
    g, o = _pair(H, O, shape, kw, spins=S)
    g.set_launch(1, 1)
    T = 0.9

    def step(s):
        g.sweep(T, sample=True)
        return o.sweep(T, sample=True)

    _compare_every_sweep(g, o, 4, step, shape)
    a, b = g.observables(), o.observables(T)
    assert a["samples"] == b["samples"] == 4
    for k in ("mean_m", "mean_E"):
        assert np.allclose(a[k], b[k], rtol=1e-11, atol=1e-13), (k, a[k], b[k])
    for k in ("E", "E_exch", "E_uni", "E_cub", "E_zee"):
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), k
    assert np.allclose(a["M"], b["M"], rtol=0, atol=1e-9)


CSHAPES = [(4, 4, 4), (8, 8, 8), (6, 10, 4), (16, 16, 16), (2, 2, 2), (12, 6, 2)]


@pytest.mark.parametrize("shape", CSHAPES)
def test_constrained_sweep_fp64_matches_reference(H, O, shape):
    _say("constrained fp64", shape)
    rng = np.random.default_rng(sum(shape))
    eC = rng.normal(size=3)
    eC /= np.linalg.norm(eC)
    kw = dict(inputs.random_params(sum(shape) + 1), seed=4321 + shape[1], instance=1)
    n = shape[0] * shape[1] * shape[2]
    S = inputs.tilted_spins(n, 5, spread=0.4, axis=eC)
    g, o = _pair(H, O, shape, kw, spins=S)
    T = 0.6

    def step(s):
        g.constrained_sweep(T, eC, sample=(s % 2 == 0))
        return o.constrained_sweep(T, eC, sample=(s % 2 == 0))

    _compare_every_sweep(g, o, 60 if n <= 4096 else 25, step, shape)
    a, b = g.observables(), o.observables(T)
    assert np.allclose(a["mean_torque"], b["mean_torque"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["mean_E"], b["mean_E"], rtol=1e-11, atol=1e-13)
    assert abs(a["mean_Eanis"] - b["mean_Eanis"]) < 1e-12


# (shape, sites per thread, z chunk): z chunks that put a tile start on the
# last plane (rC across the boundary), end a tile's march on it (the z+2 load
# across the boundary) and start on plane 0 (the z-1 plane across it)
APSHAPES = [((4, 4, 4), 2, 16), ((6, 10, 4), 1, 3), ((8, 8, 2), 1, 1), ((4, 4, 12), 4, 2),
            ((34, 6, 4), 2, 1), ((8, 6, 10), 1, 4)]


@pytest.mark.parametrize("prefetch", [1, 2])
@pytest.mark.parametrize("shape,spt,zc", APSHAPES)
def test_antiperiodic_z_fp64_matches_reference(H, O, shape, spt, zc, prefetch):
    _say("antiperiodic fp64", shape, spt, zc, "prefetch", prefetch)
    kw = dict(inputs.random_params(5 * sum(shape)), seed=99 + shape[2], instance=4, theta0_deg=35,
              boundary_z="antiperiodic")
    n = shape[0] * shape[1] * shape[2]
    S = inputs.random_unit_spins(n, 321)
    g, o = _pair(H, O, shape, kw, spins=S)
    g.set_launch(spt, zc)
    g.set_prefetch(prefetch)
    T = 0.8

    def step(s):
        g.sweep(T, sample=(s % 3 == 0))
        return o.sweep(T, sample=(s % 3 == 0))

    _compare_every_sweep(g, o, 60, step, shape)
    a, b = g.observables(), o.observables(T)
    for k in ("E", "E_exch"):
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), k
    assert np.allclose(a["mean_E"], b["mean_E"], rtol=1e-11, atol=1e-13)
    # constrained sweeps on the same lattice
    eC = np.array([0.3, -0.4, 0.866])
    eC /= np.linalg.norm(eC)
    for _ in range(10):
        g.constrained_sweep(T, eC, sample=True)
        o.constrained_sweep(T, eC, sample=True)
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    assert g.observables()["theta_deg"] == o.counters()[0]


# (shape, boundary, sites per thread, z chunk, cut probability): open films of
# odd and even thickness (nz = 1 is a monolayer) and bond masks
MASKED = [((8, 6, 5), "open", 1, 2, 0.3), ((4, 4, 1), "open", 2, 1, 0.0), ((10, 6, 3), "open", 1, 16, 0.25),
          ((6, 10, 4), "periodic", 2, 3, 0.3), ((8, 8, 6), "antiperiodic", 4, 4, 0.2), ((34, 6, 4), "open", 1, 1, 0.4)]


@pytest.mark.parametrize("shape,boundary,spt,zc,pcut", MASKED)
def test_open_z_and_bond_masks_fp64_match_reference(H, O, shape, boundary, spt, zc, pcut):
    _say("masked fp64", shape, boundary, spt, zc, pcut)
    kw = dict(inputs.random_params(7 * sum(shape)), seed=55 + shape[2], instance=6, theta0_deg=40,
              boundary_z=boundary)
    n = shape[0] * shape[1] * shape[2]
    S = inputs.random_unit_spins(n, 77)
    mask = inputs.random_bond_masks(shape, pcut, sum(shape))
    g = H.Lattice(*shape, precision=64, bond_masks=True, **kw)
    o = O.OracleLattice(*shape, init=None, **kw)
    g.set_bond_masks(mask)
    o.set_bond_masks(mask)
    g.set_spins(S)
    o.set_spins(S)
    g.set_launch(spt, zc)
    T = 0.7

    def step(s):
        g.sweep(T, sample=(s % 2 == 1))
        return o.sweep(T, sample=(s % 2 == 1))

    _compare_every_sweep(g, o, 50, step, shape)
    a, b = g.observables(), o.observables(T)
    for k in ("E", "E_exch"):
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), k
    assert np.allclose(a["mean_E"], b["mean_E"], rtol=1e-11, atol=1e-13)
    eC = np.array([0.5, 0.5, 0.7071])
    eC /= np.linalg.norm(eC)
    for _ in range(8):
        g.constrained_sweep(T, eC, sample=True)
        o.constrained_sweep(T, eC, sample=True)
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    assert g.observables()["theta_deg"] == o.counters()[0]


# open films without bond masks: odd, unit and even thickness, tiles that
# start on the top or bottom plane, under both marches
OPENSHAPES = [((8, 6, 3), 1, 2), ((4, 4, 1), 2, 1), ((10, 6, 5), 1, 16), ((6, 4, 7), 2, 3), ((8, 8, 6), 4, 4)]


@pytest.mark.parametrize("prefetch", [1, 2])
@pytest.mark.parametrize("shape,spt,zc", OPENSHAPES)
def test_open_z_fp64_matches_reference(H, O, shape, spt, zc, prefetch):
    _say("open fp64", shape, spt, zc, "prefetch", prefetch)
    kw = dict(inputs.random_params(11 * sum(shape)), seed=71 + shape[2], instance=2, theta0_deg=30,
              boundary_z="open")
    n = shape[0] * shape[1] * shape[2]
    S = inputs.random_unit_spins(n, 5 + shape[2])
    g, o = _pair(H, O, shape, kw, spins=S)
    g.set_launch(spt, zc)
    g.set_prefetch(prefetch)
    T = 0.9

    def step(s):
        g.sweep(T, sample=(s % 2 == 0))
        return o.sweep(T, sample=(s % 2 == 0))

    _compare_every_sweep(g, o, 40, step, shape)
    a, b = g.observables(), o.observables(T)
    for k in ("E", "E_exch"):
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), k
    assert np.allclose(a["mean_E"], b["mean_E"], rtol=1e-11, atol=1e-13)


def test_bond_mask_errors(H):
    g = H.Lattice(4, 4, 4, precision=32)
    with pytest.raises(H.HmcError):
        g.set_bond_masks(np.full(64, 0x3F, dtype=np.uint8))      # created without masks
    h = H.Lattice(4, 4, 4, precision=32, bond_masks=True)
    bad = np.full(64, 0x3F, dtype=np.uint8)
    bad[5] &= 0xFD                                               # x+ cut on one end only
    with pytest.raises(H.HmcError):
        h.set_bond_masks(bad)
    bad = np.full(64, 0x7F, dtype=np.uint8)
    with pytest.raises(H.HmcError):
        h.set_bond_masks(bad)
    h.set_bond_masks(np.full(64, 0x3F, dtype=np.uint8))


def test_prefetch_depth_rule_and_errors(H):
    """Automatic depth: one plane of look-ahead while the spins fit the
    256 MiB last-level cache, two above; masks keep depth one."""
    small = H.Lattice(8, 8, 8, precision=64)
    assert small.get_prefetch() == 1
    small.set_prefetch(2)
    assert small.get_prefetch() == 2
    small.set_prefetch(0)
    assert small.get_prefetch() == 1
    for bad in (-1, 3):
        with pytest.raises(H.HmcError):
            small.set_prefetch(bad)
    big = H.Lattice(256, 256, 256, precision=64)            # 384 MiB of spins
    assert big.get_prefetch() == 2
    big.close()
    fits = H.Lattice(256, 256, 256, precision=32)           # 192 MiB
    assert fits.get_prefetch() == 1
    fits.close()
    m = H.Lattice(4, 4, 4, precision=32, bond_masks=True)
    assert m.get_prefetch() == 1
    with pytest.raises(H.HmcError):
        m.set_prefetch(2)


def test_plane_means(H):
    """Mean spin per z plane equals the average of the spins of that plane."""
    shape = (10, 6, 8)
    g = H.Lattice(*shape, precision=64, init="random", seed=3, boundary_z="antiperiodic")
    g.sweep(0.7, 5)
    S = g.spins().reshape(shape[2], shape[1], shape[0], 3)
    assert np.allclose(g.plane_means(), S.mean(axis=(1, 2)), rtol=0, atol=1e-14)
    h = H.Lattice(*shape, precision=32, init="random", seed=3)
    S = h.spins().reshape(shape[2], shape[1], shape[0], 3)
    assert np.allclose(h.plane_means(), S.mean(axis=(1, 2)), rtol=0, atol=1e-12)


def test_constrained_fp64_grid_stride_size(H, O):
    """Above 2^20 spins the constrained pair kernels loop over their pairs
    (a grid-stride loop): 128 x 128 x 68 FP64 against the reference for two
    sampled sweeps."""
    _say("constrained grid-stride 128x128x68")
    shape = (128, 128, 68)
    eC = np.array([0.2, -0.3, 0.9])
    eC /= np.linalg.norm(eC)
    kw = dict(J=1.0, Ku=0.02, Kc=0.03, eu=(0, 0, 1), seed=17, instance=2)
    n = shape[0] * shape[1] * shape[2]
    S = inputs.tilted_spins(n, 9, spread=0.3, axis=eC)
    g, o = _pair(H, O, shape, kw, spins=S)
    for _ in range(2):
        acc_g = g.constrained_sweep(0.8, eC, sample=True)
        acc_o = o.constrained_sweep(0.8, eC, sample=True)
        assert g.observables()["accepted_last"] == acc_o
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    a, b = g.observables(), o.observables(0.8)
    assert np.allclose(a["mean_torque"], b["mean_torque"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["mean_E"], b["mean_E"], rtol=1e-11, atol=1e-13)


def test_mixed_standard_and_constrained(H, O):
    """Standard and constrained sweeps share the sweep counter and cone angle;
    the constrained pass takes M_L from the current spins after a standard one."""
    _say("mixed")
    kw = dict(J=1.0, Ku=0.05, Kc=0.1, seed=8, instance=2)
    g, o = _pair(H, O, (8, 8, 4), kw, init_dir=(1, 1, 1))
    eC = np.array([1.0, 1.0, 1.0]) / np.sqrt(3)
    for it in range(6):
        g.sweep(0.5, 3)
        o.sweep(0.5, 3)
        g.constrained_sweep(0.5, eC, 2)
        o.constrained_sweep(0.5, eC, 2)
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL
        assert g.observables()["theta_deg"] == o.counters()[0]


@pytest.mark.parametrize("shape", [(8, 8, 4), (96, 96, 64)])
def test_mixed_sampled_sweeps_fp64_observables(H, O, shape):
    """Sampled standard and constrained sweeps on one lattice: constrained
    passes reduce the torque as well, standard passes only M and the
    energies, and neither reads what the other left in the work-group
    records.  Spins every round and all accumulated observables against the
    reference (the larger lattice's standard passes write two groups of
    records, folded in parallel)."""
    _say("mixed sampled", shape)
    kw = dict(J=1.0, Ku=0.04, Kc=0.06, h=(0.0, 0.01, 0.0), seed=21, instance=3)
    g, o = _pair(H, O, shape, kw, init_dir=(1, 1, 1))
    if shape[0] > 8:
        g.set_launch(1, 1)      # 1152 records per standard pass: two groups, folded in parallel
    eC = np.array([0.3, 0.5, 0.8]) / np.linalg.norm([0.3, 0.5, 0.8])
    for it in range(3):
        g.constrained_sweep(0.7, eC, 2, sample=True)
        o.constrained_sweep(0.7, eC, 2, sample=True)
        g.sweep(0.7, 2, sample=True)
        o.sweep(0.7, 2, sample=True)
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    a, b = g.observables(), o.observables(0.7)
    assert a["samples"] == b["samples"] == 12 and a["torque_samples"] == 6
    assert np.allclose(a["mean_m"], b["mean_m"], rtol=1e-11, atol=1e-13)
    assert np.allclose(a["mean_E"], b["mean_E"], rtol=1e-11, atol=1e-13)
    assert abs(a["mean_Eanis"] - b["mean_Eanis"]) < 1e-12
    assert np.allclose(a["mean_torque"], b["mean_torque"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["M"], b["M"], rtol=1e-11, atol=1e-9)
    assert np.allclose(a["E"], b["E"], rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("precision", [64, 32])
def test_launch_shape_does_not_change_spins(H, precision):
    _say("launch shapes", precision)
    shape = (64, 32, 24)
    kw = dict(J=1.0, Ku=0.02, Kc=-0.03, h=(0.01, 0.0, 0.02), seed=11, init="random",
              precision=precision)
    ref = None
    for spt, zc, pf in [(2, 16, 1), (1, 1, 1), (1, 5, 1), (4, 3, 1), (4, 64, 1), (2, 24, 1), (1, 1024, 1),
                        (2, 16, 2), (1, 1, 2), (1, 5, 2), (4, 3, 2), (2, 2, 2), (1, 1024, 2)]:
        g = H.Lattice(*shape, **kw)
        g.set_launch(spt, zc)
        g.set_prefetch(pf)
        g.sweep(0.9, 12)
        S = g.spins()
        ob = g.observables()
        if ref is None:
            ref = (S, ob["theta_deg"], ob["accepted_last"])
        else:
            assert np.array_equal(S, ref[0]), (spt, zc, pf)
            assert ob["theta_deg"] == ref[1] and ob["accepted_last"] == ref[2]
        g.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_checkpoint_resume_is_bit_exact(H, precision):
    _say("checkpoint", precision)
    kw = dict(J=1.0, Ku=0.01, seed=5, init="random", precision=precision)
    g = H.Lattice(16, 8, 12, **kw)
    g.sweep(0.8, 20, sample=True)
    blob = g.get_state()
    g.sweep(0.8, 30, sample=True)
    g.constrained_sweep(0.8, (0, 0, 1), 5)
    A, oa = g.spins(), g.observables()
    g.set_state(blob)
    g.sweep(0.8, 30, sample=True)
    g.constrained_sweep(0.8, (0, 0, 1), 5)
    B, ob = g.spins(), g.observables()
    assert np.array_equal(A, B)
    for k in ("sweeps_done", "theta_deg", "samples", "mean_m", "var_m", "mean_E"):
        assert oa[k] == ob[k], k
    other = H.Lattice(16, 8, 14, **kw)
    with pytest.raises(H.HmcError):
        other.set_state(blob)


@pytest.mark.parametrize("field,value", [("theta", 0), ("theta", 181), ("theta", -7), ("sweep", -1),
                                         ("samples", -3), ("torque_samples", -1)])
def test_corrupted_state_image_is_refused(H, field, value):
    """A state image whose chain state is out of range (a cone angle outside
    [1, 180] degrees, negative counters) is refused with ESTATE before
    anything reaches the device, and the lattice keeps its chain."""
    import struct
    g = H.Lattice(8, 6, 4, precision=64, init="random", seed=2)
    g.sweep(0.7, 3, sample=True)
    blob = bytearray(g.get_state())
    before = g.spins()
    # the image is a 112-byte header (magic, precision, nx, ny, nz, boundary,
    # seed, instance, mask flag, J, Ku, eu, Kc, h), then the device state:
    # int32 theta, int32 flag, then int64 sweep, accepted_last, samples,
    # torque_samples, ...
    off = 112
    assert struct.unpack_from("<i", blob, off)[0] == g.observables()["theta_deg"]
    where = {"theta": (off, "<i"), "sweep": (off + 8, "<q"), "samples": (off + 24, "<q"),
             "torque_samples": (off + 32, "<q")}[field]
    struct.pack_into(where[1], blob, where[0], value)
    with pytest.raises(H.HmcError) as e:
        g.set_state(bytes(blob))
    assert e.value.status == H.ESTATE
    assert np.array_equal(g.spins(), before)
    ob = g.observables()
    assert ob["sweeps_done"] == 3 and 1 <= ob["theta_deg"] <= 180


def test_cone_angle_clamps_at_180_fp64(H, O):
    """With no interactions (J = K = h = 0) every proposal has dE = 0 and is
    accepted, so the cone angle rises by one degree per sweep from 170 and
    then stays at 180 (Table A1's upper guard); spins, counts and angles equal
    the reference's every sweep."""
    _say("theta clamp at 180")
    kw = dict(J=0.0, Ku=0.0, Kc=0.0, seed=21, instance=1, theta0_deg=170)
    g, o = _pair(H, O, (6, 4, 8), kw, init="random")
    thetas = []

    def step(s):
        g.sweep(0.5, sample=(s % 2 == 0))
        acc = o.sweep(0.5, sample=(s % 2 == 0))
        thetas.append(o.counters()[0])
        return acc

    _compare_every_sweep(g, o, 16, step, "clamp 180")
    assert thetas == [171, 172, 173, 174, 175, 176, 177, 178, 179, 180, 180, 180, 180, 180, 180, 180]
    assert g.observables()["accepted_last"] == 6 * 4 * 8
    # constrained sweeps from the whole-sphere cone: pair moves can still be
    # rejected (no real compensating spin, or the ratio of Table A2), so the
    # angle may move either way; it and the spins equal the reference's
    eC = (0.0, 0.6, 0.8)
    for _ in range(3):
        g.constrained_sweep(0.5, eC, sample=True)
        acc = o.constrained_sweep(0.5, eC, sample=True)
        ob = g.observables()
        assert ob["theta_deg"] == o.counters()[0] and ob["accepted_last"] == acc
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL


def test_cone_angle_clamps_at_1_fp64(H, O):
    """In the aligned ground state at T = 1e-12 a proposal is accepted only
    if it raises the energy by less than about T (a cone step of order
    1e-12 degrees: almost never), so the cone angle falls by one degree per
    sweep from 6 and then stays at 1 (Table A1's lower guard), in the
    standard and the constrained sweep; spins, counts and angles equal the
    reference's."""
    _say("theta clamp at 1")
    kw = dict(J=1.0, Ku=0.01, Kc=0.02, eu=(0, 0, 1), seed=22, instance=2, theta0_deg=6)
    g, o = _pair(H, O, (8, 6, 4), kw, init="aligned", init_dir=(0, 0, 1))
    T = 1e-12
    thetas = []

    def step(s):
        g.sweep(T, sample=True)
        acc = o.sweep(T, sample=True)
        thetas.append(o.counters()[0])
        return acc

    _compare_every_sweep(g, o, 9, step, "clamp 1")
    assert thetas == [5, 4, 3, 2, 1, 1, 1, 1, 1]
    for _ in range(3):
        g.constrained_sweep(T, (0, 0, 1), sample=True)
        acc = o.constrained_sweep(T, (0, 0, 1), sample=True)
        ob = g.observables()
        assert ob["theta_deg"] == o.counters()[0] == 1
        assert ob["accepted_last"] == acc
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    assert np.max(np.abs(g.spins() - np.array([0.0, 0.0, 1.0]))) <= 1e-6


def test_argument_errors(H):
    g = H.Lattice(4, 4, 4)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(H.HmcError) as e:
            g.sweep(bad)
        assert e.value.status == H.EINVAL
    with pytest.raises(H.HmcError):
        g.sweep(1.0, -1)
    with pytest.raises(H.HmcError):
        g.constrained_sweep(1.0, (0, 0, 0))
    with pytest.raises(H.HmcError):
        g.set_launch(3, 4)
    with pytest.raises(H.HmcError):
        g.set_launch(2, 0)
    g.sweep(1.0, 0)   # zero sweeps is a no-op
    assert g.observables()["sweeps_done"] == 0


def test_non_finite_spin_is_reported(H):
    g = H.Lattice(4, 4, 4)
    S = g.spins()
    S[5] = np.nan
    g.set_spins(S)
    ob = g.observables(check=False)
    assert ob["status"] == H.ENUMERIC


def test_unit_length_preserved_fp32(H):
    g = H.Lattice(32, 32, 32, precision=32, Kc=0.05, Ku=0.01, init="random", seed=3)
    g.sweep(0.4, 200)
    g.constrained_sweep(0.4, (0.3, 0.2, 0.9), 50)
    assert np.max(np.abs(np.linalg.norm(g.spins(), axis=1) - 1.0)) < 1e-5


# ---------------------------------------------------------------------------
# Full size: 256^3, in the launch configuration the benchmark uses
# ---------------------------------------------------------------------------

def test_full_size_fp64_one_sweep_matches_reference(H, O):
    """256^3 FP64 from a random start: one sweep, every spin within 1e-12."""
    _say("256^3 fp64 one sweep")
    kw = dict(J=1.0, Ku=0.005, eu=(0, 0, 1), seed=7)
    g = H.Lattice(256, 256, 256, precision=64, init="random", **kw)
    o = O.OracleLattice(256, 256, 256, init="random", **kw)
    # the starts differ by rounding only (fused vs separate multiply-add in
    # sqrt(1 - z^2)); every spin within the parity bound
    assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    g.sweep(0.8)
    acc = o.sweep(0.8)
    ob = g.observables()
    assert ob["accepted_last"] == acc
    assert ob["theta_deg"] == o.counters()[0]
    assert np.max(np.abs(g.spins() - o.spins())) <= TOL
    # the measurement writes 32768 work-group records: 32 groups, whose sums
    # fold_groups_kernel forms in parallel before the finalize adds them
    b = o.observables(0.8)
    for k in ("E", "E_exch", "E_uni"):
        assert abs(ob[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), (k, ob[k], b[k])
    assert np.allclose(ob["M"], b["M"], rtol=0, atol=1e-7), (ob["M"], b["M"])


def test_full_size_film_fp64_matches_reference(H, O):
    """The film workload at its largest size: 1024 x 1024 x 15 (15.7 M spins),
    open z, columnar Voronoi grains of mean diameter 16 with every intergrain
    bond cut, Ku = 0.01 along z, FP64, from the same random spins: two
    sampled sweeps match the reference spin by spin within 1e-12, with the
    same acceptance counts and cone angle, and the same energies."""
    shape = (1024, 1024, 15)
    mask, ng = inputs.grain_bond_masks(shape, 16.0, 11)
    _say("film 1024x1024x15 fp64,", ng, "grains")
    kw = dict(J=1.0, Ku=0.01, eu=(0, 0, 1), seed=21, instance=1, boundary_z="open")
    S = inputs.random_unit_spins(shape[0] * shape[1] * shape[2], 13)
    g = H.Lattice(*shape, precision=64, bond_masks=True, **kw)
    o = O.OracleLattice(*shape, init=None, **kw)
    g.set_bond_masks(mask)
    o.set_bond_masks(mask)
    g.set_spins(S)
    o.set_spins(S)
    T = 0.9
    for s in range(2):
        g.sweep(T, sample=True)
        acc = o.sweep(T, sample=True)
        ob = g.observables()
        assert ob["accepted_last"] == acc, s
        assert ob["theta_deg"] == o.counters()[0], s
        assert np.max(np.abs(g.spins() - o.spins())) <= TOL, s
    a, b = g.observables(), o.observables(T)
    for k in ("E", "E_exch", "E_uni"):
        assert abs(a[k] - b[k]) <= 1e-11 * max(1.0, abs(b[k])), (k, a[k], b[k])
    g.close()


def test_full_size_wall_fp64_matches_reference(H, O):
    """The wall workload at its size: 64 x 64 x 512, anti-periodic along z,
    from the same noisy wall across z, Ku = 0.01, FP64: three sampled sweeps
    match the reference spin by spin within 1e-12."""
    _say("wall 64x64x512 fp64")
    shape = (64, 64, 512)
    kw = dict(J=1.0, Ku=0.01, eu=(0, 0, 1), seed=6, instance=4, boundary_z="antiperiodic")
    S = inputs.wall_spins(shape, 22.2, 17)
    g, o = _pair(H, O, shape, kw, spins=S)
    T = 0.5

    def step(s):
        g.sweep(T, sample=True)
        return o.sweep(T, sample=True)

    _compare_every_sweep(g, o, 3, step, shape)
    g.close()


def test_paper_size_fp32_marches_agree(H):
    """464^3 FP32 (99.9 M spins, the lattice size of the paper's timing and of
    the bench leg, which runs the two-plane march): two sampled sweeps give
    the same spins and the same observables with one and two planes of
    look-ahead."""
    _say("464^3 fp32 both marches")
    kw = dict(J=1.0, Ku=0.005, eu=(0, 0, 1), seed=7, init="random", precision=32)
    out = []
    for pf in (1, 2):
        g = H.Lattice(464, 464, 464, **kw)
        g.set_launch(2, 16)
        g.set_prefetch(pf)
        g.sweep(1.0, 2, sample=True)
        out.append((g.spins(), g.observables()))
        g.close()
    assert np.array_equal(out[0][0], out[1][0])
    for k in ("E", "E_exch", "m", "theta_deg", "accepted_last"):
        assert out[0][1][k] == out[1][1][k], k


def test_full_size_fp32_one_sweep_tracks_reference(H, O):
    """256^3 FP32 (the benchmark's lattice and launch shape): from the same
    start, one sweep agrees with the FP64 reference site by site except where
    an FP32 rounding flips a near-threshold decision."""
    _say("256^3 fp32 one sweep")
    kw = dict(J=1.0, Ku=0.005, eu=(0, 0, 1), seed=7)
    g = H.Lattice(256, 256, 256, precision=32, init="random", **kw)
    o = O.OracleLattice(256, 256, 256, init=None, **kw)
    o.set_spins(g.spins())
    g.sweep(0.8)
    acc = o.sweep(0.8)
    ob = g.observables()
    d = np.max(np.abs(g.spins() - o.spins()), axis=1)
    assert np.mean(d < 1e-4) > 0.9995, np.mean(d < 1e-4)
    assert abs(ob["accepted_last"] - acc) < 1e-4 * acc
    assert ob["theta_deg"] == o.counters()[0]


def test_constrained_fp32_128cubed_one_sweep_tracks_reference(H, O):
    """The constrained workload at its full size and precision (128^3 FP32,
    J = 1, Kc = 0.05, e_C = (0.6, 0, 0.8), spins along e_C, T = 0.6, the
    benchmark's leg): from the same spins, one constrained sweep agrees with
    the FP64 reference pair by pair except where an FP32 rounding flips a
    near-threshold decision (the pairing and the random numbers are the
    same); the acceptance counts agree to 1e-4 and the cone angles exactly.
    A second sweep starts again from the GPU's spins on both sides."""
    _say("128^3 fp32 constrained one sweep")
    kw = dict(J=1.0, Ku=0.0, Kc=0.05, eu=(0, 0, 1), seed=7)
    eC = (0.6, 0.0, 0.8)
    g = H.Lattice(128, 128, 128, precision=32, init="aligned", init_dir=eC, **kw)
    o = O.OracleLattice(128, 128, 128, init=None, **kw)
    o.set_spins(g.spins())
    M = np.asarray(g.observables()["M"])
    Mp0 = M - (M @ np.asarray(eC)) * np.asarray(eC)
    for s in range(2):
        g.constrained_sweep(0.6, eC, sample=True)
        acc = o.constrained_sweep(0.6, eC, sample=True)
        ob = g.observables()
        d = np.max(np.abs(g.spins() - o.spins()), axis=1)
        _say("  sweep", s, "accepted", ob["accepted_last"], acc, "fraction within 1e-4:", np.mean(d < 1e-4))
        assert np.mean(d < 1e-4) > 0.9995, (s, np.mean(d < 1e-4))
        assert abs(ob["accepted_last"] - acc) < 1e-4 * acc, (s, ob["accepted_last"], acc)
        assert ob["theta_deg"] == o.counters()[0]
        # the pair moves keep the moment perpendicular to e_C: unchanged up to
        # FP32 rounding
        M = np.asarray(ob["M"])
        e = np.asarray(eC)
        Mp = M - (M @ e) * e
        assert np.linalg.norm(Mp - Mp0) < 1e-8 * g.n, (s, Mp, Mp0)
        Mp0 = Mp
        o.set_spins(g.spins())
