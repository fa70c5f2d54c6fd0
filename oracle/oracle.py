"""ctypes wrapper of the serial CPU reference (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark use it to produce expected values.  The GPU library
never imports this module.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of the same source (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleObs(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("sweeps_done", ctypes.c_int64),
        ("samples", ctypes.c_int64),
        ("accepted_last", ctypes.c_int64),
        ("theta_deg", ctypes.c_int32),
        ("M", ctypes.c_double * 3),
        ("m", ctypes.c_double),
        ("E", ctypes.c_double),
        ("E_exch", ctypes.c_double),
        ("E_uni", ctypes.c_double),
        ("E_cub", ctypes.c_double),
        ("E_zee", ctypes.c_double),
        ("torque", ctypes.c_double * 3),
        ("mean_m", ctypes.c_double * 4),
        ("var_m", ctypes.c_double * 4),
        ("mean_E", ctypes.c_double),
        ("var_E", ctypes.c_double),
        ("mean_Eanis", ctypes.c_double),
        ("mean_torque", ctypes.c_double * 3),
        ("chi", ctypes.c_double * 4),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    D3 = ctypes.POINTER(ctypes.c_double)
    U32P = ctypes.POINTER(ctypes.c_uint32)
    vp = ctypes.c_void_p
    lib.oracle_create.restype = vp
    lib.oracle_create.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.c_double, D3,
                                                         ctypes.c_double, D3, ctypes.c_uint64,
                                                         ctypes.c_uint32, ctypes.c_int32]
    lib.oracle_destroy.argtypes = [vp]
    lib.oracle_init_aligned.argtypes = [vp, D3]
    lib.oracle_set_boundary_z.argtypes = [vp, ctypes.c_int32]
    lib.oracle_set_bond_masks.argtypes = [vp, ctypes.c_void_p]
    lib.oracle_set_bond_masks.restype = ctypes.c_int
    lib.oracle_init_random.argtypes = [vp]
    lib.oracle_set_spins.argtypes = [vp, D3]
    lib.oracle_get_spins.argtypes = [vp, D3]
    lib.oracle_get_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_set_counters.argtypes = [vp, ctypes.c_int32, ctypes.c_int64]
    lib.oracle_sweep.restype = ctypes.c_int64
    lib.oracle_sweep.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_constrained_sweep.restype = ctypes.c_int64
    lib.oracle_constrained_sweep.argtypes = [vp, ctypes.c_double, D3, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32]
    lib.oracle_serial_random_sweep.restype = ctypes.c_int64
    lib.oracle_serial_random_sweep.argtypes = [vp, ctypes.c_double, ctypes.c_int32,
                                               ctypes.c_int32]
    lib.oracle_heatbath_sweep.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_reset_stats.argtypes = [vp]
    lib.oracle_observables.argtypes = [vp, ctypes.c_double, ctypes.POINTER(OracleObs)]
    lib.oracle_samples.restype = ctypes.c_int64
    lib.oracle_samples.argtypes = [vp, D3, ctypes.c_int64]
    lib.oracle_philox4x32_10.argtypes = [U32P, U32P, U32P]
    lib.oracle_fmix32.restype = ctypes.c_uint32
    lib.oracle_fmix32.argtypes = [ctypes.c_uint32]
    lib.oracle_feistel.restype = ctypes.c_uint32
    lib.oracle_feistel.argtypes = [ctypes.c_uint32, ctypes.c_uint32, U32P]
    lib.oracle_onb.argtypes = [D3, D3, D3]
    lib.oracle_cone_move.argtypes = [D3, ctypes.c_double, ctypes.c_double, ctypes.c_int32, D3]
    lib.oracle_local_energy.restype = ctypes.c_double
    lib.oracle_local_energy.argtypes = [vp, ctypes.c_int64, D3]
    lib.oracle_total_energy.restype = ctypes.c_double
    lib.oracle_total_energy.argtypes = [vp]
    lib.oracle_site_of.restype = ctypes.c_int64
    lib.oracle_site_of.argtypes = [vp, ctypes.c_int32, ctypes.c_int64]
    _lib = lib
    return lib


def lib():
    return _load()


def _d3(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox(ctr, key):
    L = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = (ctypes.c_uint32 * 4)()
    L.oracle_philox4x32_10(c, k, out)
    return [int(out[i]) for i in range(4)]


def fmix32(h):
    return int(_load().oracle_fmix32(h & 0xFFFFFFFF))


def feistel(x, n, key):
    k = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in key])
    return int(_load().oracle_feistel(x, n, k))


def onb(n):
    _, pn = _d3(n)
    b1 = np.zeros(3)
    b2 = np.zeros(3)
    _load().oracle_onb(pn, _dptr(b1), _dptr(b2))
    return b1, b2


def cone_move(S, u0, u1, theta_deg):
    _, ps = _d3(S)
    out = np.zeros(3)
    _load().oracle_cone_move(ps, float(u0), float(u1), int(theta_deg), _dptr(out))
    return out


def _obs_dict(o):
    d = {}
    for name, _ in OracleObs._fields_:
        v = getattr(o, name)
        if hasattr(v, "__len__"):
            v = [float(x) for x in v]
        d[name] = v
    return d


class OracleLattice:
    """A lattice held by the serial reference (lexicographic AoS spins)."""

    def __init__(self, nx, ny, nz, J=1.0, Ku=0.0, eu=(0.0, 0.0, 1.0), Kc=0.0,
                 h=(0.0, 0.0, 0.0), seed=1, instance=0, theta0_deg=30,
                 init="aligned", init_dir=(0.0, 0.0, 1.0), boundary_z="periodic"):
        L = _load()
        self._eu, peu = _d3(eu)
        self._h, ph = _d3(h)
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        self.h_ = L.oracle_create(nx, ny, nz, float(J), float(Ku), peu, float(Kc), ph,
                                  int(seed), int(instance), int(theta0_deg))
        if not self.h_:
            raise ValueError("invalid oracle lattice parameters")
        apz = ({"periodic": 0, "antiperiodic": 1, "open": 2}[boundary_z] if isinstance(boundary_z, str)
               else int(boundary_z))
        L.oracle_set_boundary_z(self.h_, apz)
        if init == "aligned":
            _, pd = _d3(init_dir)
            L.oracle_init_aligned(self.h_, pd)
        elif init == "random":
            L.oracle_init_random(self.h_)
        elif init is not None:
            raise ValueError(init)

    def __del__(self):
        if getattr(self, "h_", None):
            _load().oracle_destroy(self.h_)
            self.h_ = None

    def set_bond_masks(self, mask):
        """mask: N uint8 in site order (bit k = bond x-, x+, y-, y+, z-, z+ active), or None."""
        if mask is None:
            _load().oracle_set_bond_masks(self.h_, None)
            return
        self._mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(self.n))
        if _load().oracle_set_bond_masks(self.h_, self._mask.ctypes.data) != 0:
            raise MemoryError("bond masks")

    def spins(self):
        out = np.zeros((self.n, 3))
        _load().oracle_get_spins(self.h_, _dptr(out))
        return out

    def set_spins(self, S):
        a = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(self.n, 3))
        _load().oracle_set_spins(self.h_, _dptr(a))

    def counters(self):
        t = ctypes.c_int32()
        s = ctypes.c_int64()
        _load().oracle_get_counters(self.h_, ctypes.byref(t), ctypes.byref(s))
        return int(t.value), int(s.value)

    def set_counters(self, theta_deg, sweeps_done):
        _load().oracle_set_counters(self.h_, int(theta_deg), int(sweeps_done))

    def sweep(self, T, n=1, sample=False):
        return int(_load().oracle_sweep(self.h_, float(T), int(n), int(bool(sample))))

    def constrained_sweep(self, T, eC, n=1, sample=False, exact_serial=False):
        _, pe = _d3(eC)
        return int(_load().oracle_constrained_sweep(self.h_, float(T), pe, int(n),
                                                    int(bool(sample)), int(bool(exact_serial))))

    def serial_random_sweep(self, T, n=1, sample=False):
        return int(_load().oracle_serial_random_sweep(self.h_, float(T), int(n),
                                                      int(bool(sample))))

    def heatbath_sweep(self, T, n=1, sample=False):
        _load().oracle_heatbath_sweep(self.h_, float(T), int(n), int(bool(sample)))

    def reset_stats(self):
        _load().oracle_reset_stats(self.h_)

    def observables(self, T):
        o = OracleObs()
        _load().oracle_observables(self.h_, float(T), ctypes.byref(o))
        return _obs_dict(o)

    def samples(self):
        """Per-sample rows (m_l, m_x, m_y, m_z, E/N, Eanis/N, tau/N)."""
        cap = 1 << 20
        buf = np.zeros((cap, 9))
        rows = int(_load().oracle_samples(self.h_, _dptr(buf), cap))
        return buf[:rows].copy()

    def local_energy(self, site, S):
        _, ps = _d3(S)
        return float(_load().oracle_local_energy(self.h_, int(site), ps))

    def total_energy(self):
        return float(_load().oracle_total_energy(self.h_))

    def site_of(self, colour, idx):
        return int(_load().oracle_site_of(self.h_, int(colour), int(idx)))
