"""hmc_measure_static (the measurement without a workspace, its reduction
scratch in the library's static device array) against hmc_observables on the
same spins: the same kernels with the same grid, so the same bits.  Four
calls in a row, each on a smaller lattice than the last (the first two with
more than 1024 work-group records), then a call
on spins holding a non-finite value (reported) followed by a clean call (the
sticky flag is cleared between calls)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("M", "m", "E", "E_exch", "E_uni", "E_cub", "E_zee", "torque")


@pytest.fixture(scope="module")
def H():
    import torch
    import paper_2103_03517_amd as H
    assert torch.cuda.is_available(), "this test needs the GPU"
    H.lib()
    return H


def _model(seed):
    return dict(J=1.0, Ku=0.03, eu=(0.2, -0.4, 0.9), Kc=-0.02, h=(0.01, 0.02, -0.015), seed=seed,
                init="random")


def test_measure_static_matches_observables(H):
    import sys
    # 256^3: 32768 measurement records, 32 groups of the finalize's fold,
    # 96^3: 1728 records, two groups; their sums are formed in parallel into
    # the static array; each call smaller than the last
    cases = [((256, 256, 256), 32, "periodic"), ((96, 96, 96), 32, "periodic"), ((64, 48, 40), 64, "periodic"),
             ((16, 12, 10), 32, "antiperiodic")]
    for shape, precision, bz in cases:
        print("measure_static", shape, precision, bz, file=sys.stderr, flush=True)
        g = H.Lattice(*shape, precision=precision, boundary_z=bz, **_model(sum(shape)))
        g.sweep(0.7, 4, sample=True)
        ref = g.observables()
        got = H.measure_static(g.params, g.workspace.data_ptr(), g.workspace.numel())
        assert got["status"] == H.OK
        assert got["n"] == g.n and got["precision"] == precision
        for k in FIELDS:
            assert got[k] == ref[k], (shape, k, got[k], ref[k])
        assert got["sweeps_done"] == 0 and got["samples"] == 0
        g.close()


def test_measure_static_non_finite_then_clean(H):
    g = H.Lattice(8, 8, 8, precision=64, **_model(3))
    S = g.spins()
    S[17] = np.nan
    g.set_spins(S)
    bad = H.measure_static(g.params, g.workspace.data_ptr(), g.workspace.numel(), check=False)
    assert bad["status"] == H.ENUMERIC
    h = H.Lattice(6, 4, 8, precision=32, **_model(4))
    ok = H.measure_static(h.params, h.workspace.data_ptr(), h.workspace.numel())
    assert ok["status"] == H.OK
    ref = h.observables()
    for k in FIELDS:
        assert ok[k] == ref[k], k


def test_measure_static_argument_checks(H):
    import ctypes
    g = H.Lattice(8, 8, 8, precision=32, **_model(5))
    base = g.workspace.data_ptr()
    pitch = 8 * 8 * 8 // 2 * 4
    pitch = (pitch + 255) // 256 * 256
    with pytest.raises(H.HmcError) as e:           # above the 2^25-spin maximum
        H.measure_static(H.make_params(514, 256, 256, precision=32), base, 1 << 40)
    assert e.value.status == H.EDIM
    with pytest.raises(H.HmcError) as e:           # too few bytes of spins
        H.measure_static(g.params, base, 6 * pitch - 1)
    assert e.value.status == H.ENOMEM
    with pytest.raises(H.HmcError) as e:           # misaligned
        H.measure_static(g.params, base + 8, 6 * pitch)
    assert e.value.status == H.ENOMEM
    with pytest.raises(H.HmcError) as e:           # bond masks are not read
        H.measure_static(H.make_params(8, 8, 8, precision=32, bond_masks=True), base, 6 * pitch)
    assert e.value.status == H.EINVAL
    assert H.lib().hmc_measure_static(None, ctypes.c_void_p(base), 6 * pitch, None, None) == H.EINVAL
    assert H.measure_static(g.params, base, 6 * pitch)["status"] == H.OK
