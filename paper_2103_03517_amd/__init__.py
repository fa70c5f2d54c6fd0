"""Python binding of the MI355X library for the parallel Metropolis sweeps of a
classical Heisenberg spin lattice (Lepadatu et al., arXiv:2103.03517).

Argument marshalling only: every step of the sweeps runs in the HIP kernels of
libhmc.so (built from csrc/ for gfx950).  PyTorch supplies the device
workspace and the stream.  The library must be built (``__graft_entry__.build``)
before use; there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

__all__ = ["Lattice", "Batch", "Snapshot", "HmcError", "lib", "measure_static", "LIB_PATH", "SYMBOLS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmc.so")

# status codes of include/hmc.h
OK, EINVAL, EDIM, ENOMEM, EHIP, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5, -6


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("J", ctypes.c_double), ("Ku", ctypes.c_double), ("eu", ctypes.c_double * 3),
        ("Kc", ctypes.c_double), ("h", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32),
        ("init", ctypes.c_int32), ("init_dir", ctypes.c_double * 3),
        ("theta0_deg", ctypes.c_int32), ("boundary_z", ctypes.c_int32), ("bond_masks", ctypes.c_int32),
        ("init_width", ctypes.c_double),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("sweeps_done", ctypes.c_int64), ("samples", ctypes.c_int64),
        ("torque_samples", ctypes.c_int64), ("accepted_last", ctypes.c_int64),
        ("theta_deg", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("M", ctypes.c_double * 3), ("m", ctypes.c_double), ("E", ctypes.c_double),
        ("E_exch", ctypes.c_double), ("E_uni", ctypes.c_double), ("E_cub", ctypes.c_double),
        ("E_zee", ctypes.c_double), ("torque", ctypes.c_double * 3),
        ("mean_m", ctypes.c_double * 4), ("var_m", ctypes.c_double * 4),
        ("mean_E", ctypes.c_double), ("var_E", ctypes.c_double), ("mean_Eanis", ctypes.c_double),
        ("mean_torque", ctypes.c_double * 3), ("chi", ctypes.c_double * 4),
        ("T_sample", ctypes.c_double),
    ]


class Timing(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64 * 4), ("total_ms", ctypes.c_double * 4)]


TIMING_KINDS = ("pass", "constrained", "reduce", "other")

# every function declared in include/hmc.h
SYMBOLS = ("hmc_workspace_bytes", "hmc_init_lattice", "hmc_sweep", "hmc_constrained_sweep",
           "hmc_observables", "hmc_reset_stats", "hmc_set_bond_masks", "hmc_plane_means", "hmc_copy_spins",
           "hmc_state_bytes",
           "hmc_get_state", "hmc_set_state", "hmc_set_launch", "hmc_get_launch", "hmc_set_prefetch", "hmc_get_prefetch",
           "hmc_set_timing", "hmc_read_timing", "hmc_destroy", "hmc_strerror",
           "hmc_last_error", "hmc_batch_workspace_bytes", "hmc_batch_create", "hmc_batch_sweep",
           "hmc_batch_tune", "hmc_batch_set_graph", "hmc_batch_set_timing",
           "hmc_batch_read_timing", "hmc_batch_destroy", "hmc_batch_last_error",
           "hmc_batch_observables", "hmc_batch_reset_stats", "hmc_batch_sweep_each",
           "hmc_batch_set_lattices", "hmc_batch_set_chunk_bytes", "hmc_batch_get_chunk_bytes",
           "hmc_measure_static", "hmc_snapshot_bytes", "hmc_snapshot_enqueue", "hmc_snapshot_observables",
           "hmc_plane_means_async", "hmc_set_bond_masks_async")

_lib = None


def lib():
    """Load libhmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    L.hmc_workspace_bytes.restype = ctypes.c_size_t
    L.hmc_workspace_bytes.argtypes = [P(Params)]
    L.hmc_init_lattice.restype = i32
    L.hmc_init_lattice.argtypes = [P(Params), vp, ctypes.c_size_t, vp, P(vp)]
    L.hmc_sweep.restype = i32
    L.hmc_sweep.argtypes = [vp, dbl, i32, i32]
    L.hmc_constrained_sweep.restype = i32
    L.hmc_constrained_sweep.argtypes = [vp, dbl, P(dbl), i32, i32]
    L.hmc_observables.restype = i32
    L.hmc_observables.argtypes = [vp, P(Obs)]
    L.hmc_reset_stats.restype = i32
    L.hmc_reset_stats.argtypes = [vp]
    L.hmc_set_bond_masks.restype = i32
    L.hmc_set_bond_masks.argtypes = [vp, ctypes.c_void_p]
    L.hmc_plane_means.restype = i32
    L.hmc_plane_means.argtypes = [vp, P(dbl)]
    L.hmc_copy_spins.restype = i32
    L.hmc_copy_spins.argtypes = [vp, P(dbl), i32]
    L.hmc_state_bytes.restype = ctypes.c_size_t
    L.hmc_state_bytes.argtypes = [vp]
    L.hmc_get_state.restype = i32
    L.hmc_get_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.hmc_set_state.restype = i32
    L.hmc_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.hmc_set_launch.restype = i32
    L.hmc_set_launch.argtypes = [vp, i32, i32]
    L.hmc_get_launch.restype = i32
    L.hmc_get_launch.argtypes = [vp, P(i32), P(i32)]
    L.hmc_set_prefetch.restype = i32
    L.hmc_set_prefetch.argtypes = [vp, i32]
    L.hmc_get_prefetch.restype = i32
    L.hmc_get_prefetch.argtypes = [vp, P(i32)]
    L.hmc_set_timing.restype = i32
    L.hmc_set_timing.argtypes = [vp, i32]
    L.hmc_read_timing.restype = i32
    L.hmc_read_timing.argtypes = [vp, P(Timing)]
    L.hmc_destroy.restype = None
    L.hmc_destroy.argtypes = [vp]
    L.hmc_strerror.restype = ctypes.c_char_p
    L.hmc_strerror.argtypes = [i32]
    L.hmc_last_error.restype = ctypes.c_char_p
    L.hmc_last_error.argtypes = [vp]
    L.hmc_batch_workspace_bytes.restype = ctypes.c_size_t
    L.hmc_batch_workspace_bytes.argtypes = [i32]
    L.hmc_batch_create.restype = i32
    L.hmc_batch_create.argtypes = [P(vp), i32, vp, ctypes.c_size_t, P(vp)]
    L.hmc_batch_sweep.restype = i32
    L.hmc_batch_sweep.argtypes = [vp, P(dbl), i32, i32]
    L.hmc_batch_tune.restype = i32
    L.hmc_batch_tune.argtypes = [vp, P(dbl), i32]
    L.hmc_batch_set_graph.restype = i32
    L.hmc_batch_set_graph.argtypes = [vp, i32]
    L.hmc_batch_set_timing.restype = i32
    L.hmc_batch_set_timing.argtypes = [vp, i32]
    L.hmc_batch_read_timing.restype = i32
    L.hmc_batch_read_timing.argtypes = [vp, P(Timing)]
    L.hmc_batch_destroy.restype = None
    L.hmc_batch_destroy.argtypes = [vp]
    L.hmc_batch_last_error.restype = ctypes.c_char_p
    L.hmc_batch_last_error.argtypes = [vp]
    L.hmc_batch_observables.restype = i32
    L.hmc_batch_observables.argtypes = [vp, P(Obs)]
    L.hmc_batch_reset_stats.restype = i32
    L.hmc_batch_reset_stats.argtypes = [vp]
    L.hmc_batch_sweep_each.restype = i32
    L.hmc_batch_sweep_each.argtypes = [vp, P(dbl), P(i32), i32]
    L.hmc_batch_set_lattices.restype = i32
    L.hmc_batch_set_lattices.argtypes = [vp, P(vp), i32]
    L.hmc_batch_set_chunk_bytes.restype = i32
    L.hmc_batch_set_chunk_bytes.argtypes = [vp, ctypes.c_int64]
    L.hmc_batch_get_chunk_bytes.restype = i32
    L.hmc_batch_get_chunk_bytes.argtypes = [vp, P(ctypes.c_int64)]
    L.hmc_measure_static.restype = i32
    L.hmc_measure_static.argtypes = [P(Params), vp, ctypes.c_size_t, vp, P(Obs)]
    L.hmc_snapshot_bytes.restype = ctypes.c_size_t
    L.hmc_snapshot_bytes.argtypes = []
    L.hmc_snapshot_enqueue.restype = i32
    L.hmc_snapshot_enqueue.argtypes = [P(vp), i32, vp]
    L.hmc_snapshot_observables.restype = i32
    L.hmc_snapshot_observables.argtypes = [vp, ctypes.c_int64, i32, P(Obs)]
    L.hmc_set_bond_masks_async.restype = i32
    L.hmc_set_bond_masks_async.argtypes = [vp, vp, i32]
    L.hmc_plane_means_async.restype = i32
    L.hmc_plane_means_async.argtypes = [vp, vp]
    _lib = L
    return L


class HmcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"hmc status {status}: {message}")
        self.status = status


def make_params(nx, ny, nz, precision=64, J=1.0, Ku=0.0, eu=(0.0, 0.0, 1.0), Kc=0.0,
                h=(0.0, 0.0, 0.0), seed=1, instance=0, init="aligned", init_dir=(0.0, 0.0, 1.0),
                theta0_deg=30, boundary_z="periodic", bond_masks=False, init_width=0.0):
    p = Params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.precision = int(precision)
    p.J, p.Ku, p.Kc = float(J), float(Ku), float(Kc)
    p.eu[:] = [float(v) for v in eu]
    p.h[:] = [float(v) for v in h]
    p.seed = int(seed)
    p.instance = int(instance)
    p.init = {"aligned": 0, "random": 1, "wall": 2}[init] if isinstance(init, str) else int(init)
    p.init_width = float(init_width)
    p.init_dir[:] = [float(v) for v in init_dir]
    p.theta0_deg = int(theta0_deg)
    p.boundary_z = ({"periodic": 0, "antiperiodic": 1, "open": 2}[boundary_z] if isinstance(boundary_z, str)
                    else int(boundary_z))
    p.bond_masks = int(bool(bond_masks))
    return p


def workspace_bytes(params):
    return int(lib().hmc_workspace_bytes(ctypes.byref(params)))


def _obs_dict(o):
    d = {}
    for name, _ in Obs._fields_:
        v = getattr(o, name)
        d[name] = [float(x) for x in v] if hasattr(v, "__len__") else v
    return d


class Lattice:
    """One spin lattice resident in a torch-owned device workspace."""

    def __init__(self, nx, ny, nz, device="cuda", stream=None, **kw):
        self._lib = lib()
        self.params = make_params(nx, ny, nz, **kw)
        self.shape = (int(nx), int(ny), int(nz))
        self.n = int(nx) * int(ny) * int(nz)
        nbytes = workspace_bytes(self.params)
        if nbytes == 0:
            h = ctypes.c_void_p()
            st = self._lib.hmc_init_lattice(ctypes.byref(self.params), None, 0, None, ctypes.byref(h))
            raise HmcError(st, self._lib.hmc_strerror(st).decode())
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the workspace comes from the pool of the stream the lattice runs on:
        # a block last used on another stream could still be in use by work
        # pending there, and the caching allocator orders reuse per stream
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        st = self._lib.hmc_init_lattice(ctypes.byref(self.params),
                                        ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise HmcError(st, self._lib.hmc_strerror(st).decode())
        self._h = h

    # -- helpers -----------------------------------------------------------
    def _check(self, st):
        if st != OK:
            raise HmcError(st, self._lib.hmc_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method --------------------------------------------------------
    def sweep(self, T, n=1, sample=False):
        self._check(self._lib.hmc_sweep(self._h, float(T), int(n), int(bool(sample))))

    def constrained_sweep(self, T, eC, n=1, sample=False):
        e = (ctypes.c_double * 3)(*[float(v) for v in eC])
        self._check(self._lib.hmc_constrained_sweep(self._h, float(T), e, int(n), int(bool(sample))))

    def observables(self, check=True):
        o = Obs()
        st = self._lib.hmc_observables(self._h, ctypes.byref(o))
        if check:
            self._check(st)
        d = _obs_dict(o)
        d["status"] = st
        return d

    def reset_stats(self):
        self._check(self._lib.hmc_reset_stats(self._h))

    def set_bond_masks(self, mask):
        """mask: one uint8 per site in site order (bits x-, x+, y-, y+, z-, z+ = bond active)."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(self.n))
        self._check(self._lib.hmc_set_bond_masks(self._h, m.ctypes.data))

    def set_bond_masks_async(self, mask, check=True):
        """Enqueue the bond masks from a pinned uint8 torch tensor of one byte
        per site (kept alive by the lattice until replaced), without waiting."""
        assert mask.dtype == torch.uint8 and not mask.is_cuda and mask.numel() == self.n
        self._mask_host = mask
        self._check(self._lib.hmc_set_bond_masks_async(self._h, ctypes.c_void_p(mask.data_ptr()), int(bool(check))))

    def plane_means_async(self, dev_out):
        """Enqueue the plane means into a device float64 tensor of nz x 3
        (or 3 nz) elements, without waiting."""
        assert dev_out.dtype == torch.float64 and dev_out.is_cuda and dev_out.numel() >= 3 * self.shape[2]
        self._check(self._lib.hmc_plane_means_async(self._h, ctypes.c_void_p(dev_out.data_ptr())))

    def plane_means(self):
        """Mean spin of every z plane of the current spins, shape (nz, 3)."""
        out = np.empty((self.shape[2], 3), dtype=np.float64)
        self._check(self._lib.hmc_plane_means(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    # -- data movement -----------------------------------------------------
    def spins(self):
        out = np.empty((self.n, 3), dtype=np.float64)
        self._check(self._lib.hmc_copy_spins(
            self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1))
        return out

    def set_spins(self, S):
        a = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(self.n, 3))
        self._check(self._lib.hmc_copy_spins(
            self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0))

    def get_state(self):
        n = int(self._lib.hmc_state_bytes(self._h))
        buf = (ctypes.c_char * n)()
        self._check(self._lib.hmc_get_state(self._h, buf, n))
        return bytes(buf)

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(self._lib.hmc_set_state(self._h, buf, len(blob)))

    # -- launch shape and timing ------------------------------------------
    def set_launch(self, sites_per_thread, z_chunk):
        self._check(self._lib.hmc_set_launch(self._h, int(sites_per_thread), int(z_chunk)))

    def get_launch(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.hmc_get_launch(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def set_prefetch(self, depth):
        """Look-ahead of the pass's march: 1 or 2 planes, 0 automatic."""
        self._check(self._lib.hmc_set_prefetch(self._h, int(depth)))

    def get_prefetch(self):
        d = ctypes.c_int32()
        self._check(self._lib.hmc_get_prefetch(self._h, ctypes.byref(d)))
        return int(d.value)

    def set_timing(self, enable=True):
        self._check(self._lib.hmc_set_timing(self._h, int(bool(enable))))

    def read_timing(self):
        t = Timing()
        self._check(self._lib.hmc_read_timing(self._h, ctypes.byref(t)))
        return {k: {"count": int(t.count[i]), "total_ms": float(t.total_ms[i])}
                for i, k in enumerate(TIMING_KINDS)}


def measure_static(params, dev_spins, nbytes, stream=None, check=True):
    """hmc_measure_static: M, the energy terms and the torque of spins in the
    lattice layout at device address dev_spins (nbytes long), with the
    library's static scratch instead of a workspace.  Returns the observables
    dict (instantaneous fields only) with its status."""
    L = lib()
    s = stream if stream is not None else torch.cuda.current_stream()
    o = Obs()
    st = L.hmc_measure_static(ctypes.byref(params), ctypes.c_void_p(int(dev_spins)), int(nbytes),
                              ctypes.c_void_p(s.cuda_stream), ctypes.byref(o))
    if check and st != OK:
        raise HmcError(st, L.hmc_strerror(st).decode())
    d = _obs_dict(o)
    d["status"] = st
    return d


class Snapshot:
    """An asynchronous read of the chain states of some lattices (one
    stream): copies into a pinned host buffer are enqueued at construction,
    followed by an event.  ready() polls the event without blocking;
    observables() waits for it if needed and converts each record as
    hmc_observables would (accumulators; no fresh measurement)."""

    def __init__(self, lattices, stream=None):
        L = lib()
        self.lattices = list(lattices)
        self.rec = int(L.hmc_snapshot_bytes())
        self.meta = [(l.n, l.params.precision) for l in self.lattices]
        self.host = torch.empty(max(1, len(self.lattices)) * self.rec, dtype=torch.uint8, pin_memory=True)
        hs = (ctypes.c_void_p * max(1, len(self.lattices)))(*[l._h for l in self.lattices])
        st = L.hmc_snapshot_enqueue(hs, len(self.lattices), ctypes.c_void_p(self.host.data_ptr()))
        if st != OK:
            raise HmcError(st, L.hmc_strerror(st).decode())
        self.event = torch.cuda.Event()
        self.event.record(stream if stream is not None else self.lattices[0].stream)

    def ready(self):
        return self.event.query()

    def observables(self):
        self.event.synchronize()
        L = lib()
        out = []
        base = self.host.data_ptr()
        for i, (n, prec) in enumerate(self.meta):
            o = Obs()
            st = L.hmc_snapshot_observables(ctypes.c_void_p(base + i * self.rec), n, prec, ctypes.byref(o))
            d = _obs_dict(o)
            d["status"] = st
            out.append(d)
        return out


def _timing_dict(t):
    return {k: {"count": int(t.count[i]), "total_ms": float(t.total_ms[i])}
            for i, k in enumerate(TIMING_KINDS)}


class Batch:
    """Independent lattices (one precision, one stream) swept together: one
    launch per colour pass and kernel variant, one finalize launch.  The
    lattices stay usable on their own (observables, checkpoints, single
    sweeps) and must outlive the batch."""

    def __init__(self, lattices, capacity=None):
        self._lib = lib()
        self.lattices = list(lattices)
        n = len(self.lattices)
        nbytes = int(self._lib.hmc_batch_workspace_bytes(max(n, int(capacity or 0))))
        handles = (ctypes.c_void_p * max(n, 1))(*[l._h for l in self.lattices])
        dev = self.lattices[0].device if n else torch.device("cuda")
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        st = self._lib.hmc_batch_create(handles, n, ctypes.c_void_p(self.workspace.data_ptr()),
                                        nbytes, ctypes.byref(h))
        if st != OK:
            raise HmcError(st, self._lib.hmc_strerror(st).decode())
        self._h = h

    def _check(self, st):
        if st != OK:
            raise HmcError(st, self._lib.hmc_batch_last_error(self._h).decode())

    def _temps(self, T):
        T = np.broadcast_to(np.asarray(T, dtype=np.float64), (len(self.lattices),))
        return (ctypes.c_double * len(T))(*[float(v) for v in T])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hmc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_lattices(self, lattices):
        """Swap in another list of lattices (up to the capacity given at creation)."""
        new = list(lattices)
        handles = (ctypes.c_void_p * max(len(new), 1))(*[l._h for l in new])
        self._check(self._lib.hmc_batch_set_lattices(self._h, handles, len(new)))
        self.lattices = new

    def sweep(self, T, n=1, sample=False):
        """n standard sweeps of every lattice; T is one value or one per lattice."""
        self._check(self._lib.hmc_batch_sweep(self._h, self._temps(T), int(n), int(bool(sample))))

    def sweep_each(self, T, sample, n=1):
        """n standard sweeps; sample[i] says whether lattice i accumulates."""
        flags = (ctypes.c_int32 * len(self.lattices))(*[int(bool(v)) for v in sample])
        self._check(self._lib.hmc_batch_sweep_each(self._h, self._temps(T), flags, int(n)))

    def tune(self, T, trial_sweeps=4):
        """Pick the launch shape of each lattice size by timing batch sweeps;
        the chains are restored afterwards.  Returns the shapes per lattice."""
        self._check(self._lib.hmc_batch_tune(self._h, self._temps(T), int(trial_sweeps)))
        return [l.get_launch() for l in self.lattices]

    def observables(self, check=True):
        """Observables of every lattice (one synchronisation)."""
        n = len(self.lattices)
        o = (Obs * n)()
        st = self._lib.hmc_batch_observables(self._h, o)
        if check:
            self._check(st)
        return [_obs_dict(x) for x in o]

    def reset_stats(self):
        """Clear every lattice's accumulators (enqueued, no synchronisation)."""
        self._check(self._lib.hmc_batch_reset_stats(self._h))

    def set_chunk_bytes(self, nbytes):
        """Sweep consecutive lattices in chunks of at most nbytes of spins (0: one chunk)."""
        self._check(self._lib.hmc_batch_set_chunk_bytes(self._h, int(nbytes)))

    def chunk_bytes(self):
        v = ctypes.c_int64()
        self._check(self._lib.hmc_batch_get_chunk_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def set_graph(self, sweeps_per_graph):
        self._check(self._lib.hmc_batch_set_graph(self._h, int(sweeps_per_graph)))

    def set_timing(self, enable=True):
        self._check(self._lib.hmc_batch_set_timing(self._h, int(bool(enable))))

    def read_timing(self):
        t = Timing()
        self._check(self._lib.hmc_batch_read_timing(self._h, ctypes.byref(t)))
        return _timing_dict(t)
