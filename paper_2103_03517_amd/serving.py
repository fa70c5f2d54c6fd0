"""Continuous batching of mixed jobs on one device.

Requests (one lattice, one temperature, a sweep budget each) arrive over
time.  Four kinds of job, after the paper's uses of the method:

* "mt": m(T) of a periodic cube started along z (Sec. 3), reporting <|m|>,
  chi and E with batch-means errors;
* "wall": a lattice anti-periodic along z started from the T = 0 wall
  profile, reporting the fitted wall width (Sec. 3, Eq. 5);
* "aniso": a constrained run (Table A2) of a periodic cube with cubic
  anisotropy, the moment held along e_C(theta, phi), reporting the mean
  torque, its component -<tau>.e_phi and the anisotropy energy (Sec. 3);
* "film": a granular film, open along z with Voronoi grains whose
  intergrain exchange is cut (Sec. 4), reporting m(T).

The loop admits waiting requests in arrival order whenever a slot is free and
their workspace fits in the HBM budget.  m(T) and wall jobs advance together
through the batch interface (one launch per colour pass for all of them,
each with its own temperature and sample flag); constrained and film jobs,
which the batch kernels do not cover, are swept one by one on the same
stream in the same tick.  The host never waits for a read: at a job's block
end it enqueues an asynchronous snapshot of the chain states (and, for a
wall, of its plane profile) followed by an event, and consumes the snapshot
when the event has passed; it runs at most a few ticks ahead of the device,
waiting on the oldest tick's event only when it gets further ahead.  A job
finishes when its last snapshot has reached the host; it is then retired and
its memory released for the next admissions.

A job's chain depends only on its own key (seed, instance), its temperature,
its sweep schedule and its launch shape, so its result is the same alone and
in any mix (tests check this bit for bit).

    python -m paper_2103_03517_amd.serving --rate 20 --seconds 10
"""
import argparse
import collections
import json
import math
import sys
import time

import numpy as np
import torch

from . import Batch, Lattice, Snapshot, workspace_bytes, make_params
from .protocols import block_stats_from_reads, ec_of, blocking_se
from . import films as F
from . import walls as W

KINDS = ("mt", "wall", "aniso", "film")


class Job:
    """One request: `equil` unsampled sweeps, then `samples` sampled sweeps
    read every `block` sweeps.  kind "mt": an edge^3 periodic cube started
    along z; "wall": a shape = (nx, ny, nz) lattice anti-periodic along z,
    started from the T = 0 wall, whose m_z plane profile is kept at every
    block end and fitted when the job retires; "aniso": an edge^3 periodic
    cube with cubic anisotropy Kc, started and held along e_C(theta, phi)
    (constrained sweeps); "film": a shape = (nx, ny, nz) film open along z
    with Voronoi grains of mean diameter `diameter` (grain seed `grain_seed`),
    started along z."""

    def __init__(self, edge, T, equil=200, samples=800, block=100, seed=5, instance=0, Ku=0.01,
                 J=1.0, arrival=0.0, name=None, kind="mt", shape=None, Kc=0.0, theta=0.0, phi=0.0,
                 diameter=16.0, grain_seed=9):
        if samples % block or equil < 0 or samples <= 0 or block <= 0:
            raise ValueError("samples must be a positive multiple of block")
        if kind not in KINDS:
            raise ValueError(f"unknown job kind {kind}")
        self.kind = kind
        self.shape = tuple(int(v) for v in shape) if shape is not None else (int(edge),) * 3
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.profiles = []
        self.edge, self.T = int(edge), float(T)
        self.equil, self.samples, self.block = int(equil), int(samples), int(block)
        self.seed, self.instance, self.Ku, self.J = int(seed), int(instance), float(Ku), float(J)
        self.Kc, self.theta, self.phi = float(Kc), float(theta), float(phi)
        self.diameter, self.grain_seed = float(diameter), int(grain_seed)
        self.arrival = float(arrival)
        self.name = name if name is not None else f"job{instance}"
        self.done = 0
        self.reads = []
        self.expected_reads = self.samples // self.block
        self.lattice = None
        self.prof_dev = None
        self.prof_enqueued = 0
        self.admitted = self.finished = None
        self.result = None

    @property
    def total(self):
        return self.equil + self.samples

    @property
    def batched(self):
        """m(T) and wall jobs run in the batch; constrained and film jobs alone."""
        return self.kind in ("mt", "wall")

    def e_c(self):
        return ec_of(self.theta, self.phi)

    def lattice_kw(self, precision):
        kw = dict(precision=precision, J=self.J, seed=self.seed, instance=self.instance)
        if self.kind == "aniso":
            kw.update(Kc=self.Kc, Ku=0.0, init="aligned", init_dir=self.e_c())
        elif self.kind == "film":
            kw.update(Ku=self.Ku, eu=(0.0, 0.0, 1.0), init="aligned", boundary_z="open", bond_masks=True)
        elif self.kind == "wall":
            kw.update(Ku=self.Ku, eu=(0.0, 0.0, 1.0), init="wall", init_width=W.zero_temperature_width(self.J, self.Ku),
                      boundary_z="antiperiodic")
        else:
            kw.update(Ku=self.Ku, eu=(0.0, 0.0, 1.0), init="aligned")
        return kw

    def params(self, precision):
        return make_params(*self.shape, **self.lattice_kw(precision))

    def sampling(self):
        return self.done >= self.equil

    def next_event(self):
        """Sweeps until this job's next phase change, block end or end."""
        if self.done < self.equil:
            return self.equil - self.done
        k = (self.done - self.equil) % self.block
        return self.block - k


def poisson_jobs(rate=20.0, seconds=10.0, seed=5, edges=(32, 48, 64, 96, 128, 160, 192),
                 t_lo=0.05, t_hi=1.7, wall_fraction=0.0, wall_shape=(64, 64, 512), wall_t_hi=1.2,
                 wall_sweeps=(1000, 1000, 100), aniso_fraction=0.0, aniso_edges=(32, 48, 64), aniso_Kc=0.05,
                 aniso_t=(0.2, 1.4), aniso_sweeps=(500, 500, 100), film_fraction=0.0, film_n=1024,
                 film_nz=(5, 10, 15), film_diameters=(8.0, 16.0, 24.0), film_t_hi=1.4, film_sweeps=(200, 800, 100),
                 **job_kw):
    """Poisson arrivals: exponential gaps of mean 1/rate.  Each job is a wall
    job with probability wall_fraction (wall_shape, T ~ U(t_lo, wall_t_hi)),
    a constrained anisotropy job with probability aniso_fraction (edge from
    aniso_edges, Kc = aniso_Kc, theta uniform in 0..90 degrees by 10, phi 0 or
    45, T ~ U(aniso_t)), a film job with probability film_fraction
    (film_n^2 x nz, nz from film_nz, grain diameter from film_diameters, T ~
    U(t_lo, film_t_hi)), else an m(T) job with the edge uniform over `edges`
    and T ~ U(t_lo, t_hi).  (equil, samples, block) per kind as given."""
    rng = np.random.default_rng(seed)
    jobs, t, i = [], 0.0, 0
    base = {k: v for k, v in job_kw.items() if k not in ("equil", "samples", "block")}
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        edge = int(rng.choice(edges))
        T = float(rng.uniform(t_lo, t_hi))
        u = rng.uniform()
        if u < wall_fraction:
            eq, smp, blk = wall_sweeps
            T = t_lo + (T - t_lo) * (wall_t_hi - t_lo) / (t_hi - t_lo)
            jobs.append(Job(edge, T, equil=eq, samples=smp, block=blk, seed=seed, instance=i, arrival=t,
                            kind="wall", shape=wall_shape, **base))
        elif u < wall_fraction + aniso_fraction:
            eq, smp, blk = aniso_sweeps
            e = int(rng.choice(aniso_edges))
            th = 10.0 * int(rng.integers(0, 10))
            ph = 45.0 * int(rng.integers(0, 2))
            Ta = float(rng.uniform(*aniso_t))
            jobs.append(Job(e, Ta, equil=eq, samples=smp, block=blk, seed=seed, instance=i, arrival=t,
                            kind="aniso", Kc=aniso_Kc, theta=th, phi=ph,
                            **{k: v for k, v in base.items() if k not in ("Ku",)}))
        elif u < wall_fraction + aniso_fraction + film_fraction:
            eq, smp, blk = film_sweeps
            nz = int(rng.choice(film_nz))
            d = float(rng.choice(film_diameters))
            Tf = t_lo + (T - t_lo) * (film_t_hi - t_lo) / (t_hi - t_lo)
            jobs.append(Job(film_n, Tf, equil=eq, samples=smp, block=blk, seed=seed, instance=i, arrival=t,
                            kind="film", shape=(film_n, film_n, nz), diameter=d, **base))
        else:
            jobs.append(Job(edge, T, seed=seed, instance=i, arrival=t, **job_kw))
        i += 1
    return jobs


class Server:
    """The continuous-batching loop.  `shapes` maps a lattice shape to the
    launch shape (sites per thread, z chunk) its lattices use; `quantum` is
    the largest number of sweeps enqueued per tick; the host runs at most
    `ahead` ticks ahead of the device."""

    def __init__(self, precision=32, hbm_budget=32 << 30, max_slots=64, quantum=50, shapes=None,
                 graph=0, ahead=3, solo_streams=4, log=None):
        self.precision = int(precision)
        # jobs that run alone (constrained and film jobs) go round-robin onto
        # this many streams of their own (default priority), so that their
        # small launches overlap the batch's instead of queueing behind them
        self.solo_streams = int(solo_streams)
        self._streams = []
        self._next_stream = 0
        self.hbm_budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.quantum = int(quantum)
        self.shapes = dict(shapes or {})
        self.graph = int(graph)
        self.ahead = int(ahead)
        self.log = log
        self._grains = {}
        self.stats = {"ticks": 0, "rebuilds": 0, "max_active": 0, "max_bytes": 0, "sweep_launches": 0,
                      "snapshots": 0}
        # host seconds per phase of the loop; "wait" is the time spent
        # blocked on the device when the host got `ahead` ticks ahead
        self.phase_s = {"admit": 0.0, "rebuild": 0.0, "enqueue": 0.0, "read": 0.0, "retire": 0.0, "wait": 0.0}

    def need_bytes(self, job):
        return workspace_bytes(job.params(self.precision))

    def tune_shapes(self, shapes, T=1.0, trial_sweeps=3):
        """One lattice per shape (nx, ny, nz), tuned together in one batch;
        the launch shapes are kept per lattice shape."""
        shapes = [tuple(s) for s in shapes]
        lats = [Lattice(*s, precision=self.precision, Ku=0.01, seed=1, instance=i) for i, s in enumerate(shapes)]
        B = Batch(lats)
        launch = B.tune([T] * len(lats), trial_sweeps)
        B.close()
        for l in lats:
            l.close()
        self.shapes.update({s: tuple(ln) for s, ln in zip(shapes, launch)})
        return dict(self.shapes)

    def _film_masks(self, job):
        """Bond masks of a film as a pinned tensor, built once per film
        configuration (the grain map does not change with the thickness);
        returns (masks, first use)."""
        key = (job.shape, job.diameter, job.grain_seed)
        first = key not in self._grains
        if first:
            g, _ = F.voronoi_grains(job.shape[0], job.shape[1], job.diameter, job.grain_seed)
            m = torch.from_numpy(F.grain_bond_masks(g, job.shape[2])).pin_memory()
            self._grains[key] = m
        return self._grains[key], first

    def _solo_stream(self):
        if not self._streams:
            return None
        s = self._streams[self._next_stream % len(self._streams)]
        self._next_stream += 1
        return s

    def _admit(self, job, now):
        stream = None if job.batched else self._solo_stream()
        job.lattice = Lattice(*job.shape, stream=stream, **job.lattice_kw(self.precision))
        if job.kind == "film":
            # enqueued without waiting; checked on the host the first time
            masks, first = self._film_masks(job)
            job.lattice.set_bond_masks_async(masks, check=first)
        if job.kind == "wall":
            job.prof_dev = torch.empty((job.expected_reads, job.shape[2], 3), dtype=torch.float64, device="cuda")
        if job.shape in self.shapes and job.kind != "film":
            job.lattice.set_launch(*self.shapes[job.shape])
        job.admitted = now
        job.bytes = self.need_bytes(job)

    @staticmethod
    def _fit_walls(job, profiles):
        fits = []
        for prof in profiles:
            try:
                fits.append(W.fit_wall(prof, delta_guess=W.zero_temperature_width(job.J, job.Ku)))
            except RuntimeError:
                pass
        if fits:
            f = np.array(fits)
            job.result.update(delta=float(f[:, 2].mean()), m_wall=float(f[:, 0].mean()), wall_fits=len(f))

    @staticmethod
    def _aniso_result(job):
        """Mean torque, its component -<tau>.e_phi with its blocking error,
        and the anisotropy energy, from the cumulative constrained samples."""
        ephi = np.array([-math.sin(math.radians(job.phi)), math.cos(math.radians(job.phi)), 0.0])
        g, prev = [], (0, np.zeros(3))
        for r in job.reads:
            ns = r["torque_samples"]
            tsum = ns * np.asarray(r["mean_torque"])
            g.append(-float((tsum - prev[1]) @ ephi) / (ns - prev[0]))
            prev = (ns, tsum)
        last = job.reads[-1]
        return {"theta": job.theta, "phi": job.phi, "torque": last["mean_torque"], "g": float(np.mean(g)),
                "se_g": float(blocking_se(np.array(g)[:, None])[0]), "E_anis": last["mean_Eanis"]}

    def _retire(self, job, now):
        job.result = block_stats_from_reads(job.reads, job.n, job.T)
        job.result.update(edge=job.edge, shape=list(job.shape), kind=job.kind,
                          sweeps=job.reads[-1]["sweeps_done"], theta_deg=job.reads[-1]["theta_deg"])
        if job.kind == "aniso":
            job.result.update(self._aniso_result(job))
        if job.kind == "film":
            job.result.update(diameter=job.diameter)
        job.lattice.close()
        job.lattice = None
        job.finished = now

    def run(self, jobs, realtime=True):
        """Serves `jobs` (arrival times in seconds from the start).  With
        realtime=False every job counts as arrived at time 0 (a saturation
        run).  Returns the finished jobs with results and admission and
        finish times (seconds from the start) filled in."""
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        for j in pending:
            if self.need_bytes(j) > self.hbm_budget:
                raise ValueError(f"{j.name} needs {self.need_bytes(j)} bytes, above the HBM budget")
        waiting = collections.deque()
        active = []          # admitted, still sweeping
        draining = []        # all sweeps enqueued, reads still in flight
        inflight = collections.deque()   # (Snapshot, jobs, wall profile copies)
        ticks = collections.deque()      # events of the ticks the device may still be running
        used = 0
        batch = None
        changed = True
        if not realtime:
            for j in pending:
                j.arrival = 0.0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        done = []
        stream = torch.cuda.current_stream()
        if self.solo_streams > 0 and not self._streams:
            self._streams = [torch.cuda.Stream() for _ in range(self.solo_streams)]

        def consume(block):
            """Takes every snapshot that has reached the host (all of them,
            waiting if needed, when block) and retires the jobs whose last
            read it was."""
            nonlocal used
            t_ph = time.perf_counter()
            # snapshots of different streams finish out of order; a job's own
            # snapshots share its stream, so they are taken in order
            keep = collections.deque()
            while inflight:
                item = inflight.popleft()
                if not (block or item[0].ready()):
                    keep.append(item)
                    continue
                snap, js, walls = item
                obs = snap.observables()
                for j, o in zip(js, obs):
                    j.reads.append(o)
                for j, prof in walls:
                    j.profiles.append(prof)
                now = clock()
                for j in js:
                    if len(j.reads) == j.expected_reads:
                        self._retire(j, now)
                        if j.kind == "wall":
                            self._fit_walls(j, j.profiles)
                        used -= j.bytes
                        done.append(j)
                        draining.remove(j)
            inflight.extend(keep)
            self.phase_s["read"] += time.perf_counter() - t_ph

        while pending or waiting or active or draining or inflight:
            now = clock()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            t_ph = time.perf_counter()
            while (waiting and len(active) + len(draining) < self.max_slots
                   and used + self.need_bytes(waiting[0]) <= self.hbm_budget):
                j = waiting.popleft()
                self._admit(j, clock())
                used += j.bytes
                active.append(j)
                if j.batched:
                    changed = True
            self.phase_s["admit"] += time.perf_counter() - t_ph
            self.stats["max_active"] = max(self.stats["max_active"], len(active) + len(draining))
            self.stats["max_bytes"] = max(self.stats["max_bytes"], used)
            if not active:
                if inflight:
                    consume(block=True)
                elif pending:
                    time.sleep(max(0.0, pending[0].arrival - clock()))
                continue
            batched = [j for j in active if j.batched]
            solo = [j for j in active if not j.batched]
            if changed:
                t_ph = time.perf_counter()
                if batched:
                    if batch is None:
                        # one batch for the whole run, sized for max_slots lattices
                        batch = Batch([j.lattice for j in batched], capacity=self.max_slots)
                        if self.graph:
                            batch.set_graph(self.graph)
                    else:
                        batch.set_lattices([j.lattice for j in batched])
                    self.stats["rebuilds"] += 1
                changed = False
                self.phase_s["rebuild"] += time.perf_counter() - t_ph
            q = min(self.quantum, min(j.next_event() for j in active))
            t_ph = time.perf_counter()
            if batched:
                batch.sweep_each([j.T for j in batched], [j.sampling() for j in batched], q)
            for j in solo:
                if j.kind == "aniso":
                    j.lattice.constrained_sweep(j.T, j.e_c(), q, sample=j.sampling())
                else:
                    j.lattice.sweep(j.T, q, sample=j.sampling())
            self.stats["ticks"] += 1
            self.stats["sweep_launches"] += q
            for j in active:
                j.done += q
            hit = [j for j in active if j.sampling() and j.done > j.equil and (j.done - j.equil) % j.block == 0]
            if hit:
                # the wall profiles (plane means into the job's device rows,
                # m_z copied to pinned host memory), then the snapshot of
                # every job at a block end, then one event behind them all
                copies = []
                for j in hit:
                    if j.kind == "wall":
                        row = j.prof_dev[j.prof_enqueued]
                        j.lattice.plane_means_async(row)
                        host = torch.empty(j.shape[2], dtype=torch.float64, pin_memory=True)
                        host.copy_(row[:, 2], non_blocking=True)
                        copies.append((j, host))
                        j.prof_enqueued += 1
                # one snapshot per stream: the batch's and each solo stream's
                groups = collections.OrderedDict()
                for j in hit:
                    groups.setdefault(j.lattice.stream, []).append(j)
                for st_, js in groups.items():
                    snap = Snapshot([j.lattice for j in js], st_)
                    inflight.append((snap, js, [(j, h.numpy()) for j, h in copies if j in js]))
                    self.stats["snapshots"] += 1
            self.phase_s["enqueue"] += time.perf_counter() - t_ph
            # jobs whose sweeps are all enqueued leave the batch; they finish
            # when their last snapshot arrives
            finished = [j for j in active if j.done >= j.total]
            if finished:
                active = [j for j in active if j.done < j.total]
                draining.extend(finished)
                if any(j.batched for j in finished):
                    changed = True
            evs = []
            for st_ in [stream] + self._streams:
                ev = torch.cuda.Event()
                ev.record(st_)
                evs.append(ev)
            ticks.append(evs)
            t_ph = time.perf_counter()
            while len(ticks) > self.ahead:
                for ev in ticks.popleft():
                    ev.synchronize()
            self.phase_s["wait"] += time.perf_counter() - t_ph
            consume(block=False)
            if finished and self.log:
                self.log(f"t={clock():.3f}s draining {len(draining)}, active {len(active)}, "
                         f"waiting {len(waiting)}, pending {len(pending)}")
        if batch is not None:
            batch.close()
        torch.cuda.synchronize()
        return done


def latency_summary(done, window=None):
    lat = np.array([j.finished - j.arrival for j in done])
    span = window if window is not None else max(j.finished for j in done)
    updates = sum(j.n * j.total for j in done)
    out = {"jobs": len(done), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "mean_s": float(lat.mean()), "max_s": float(lat.max()), "span_s": float(span),
           "jobs_per_s": len(done) / span, "updates_per_s": updates / span, "by_kind": {}}
    for k in KINDS:
        lk = np.array([j.finished - j.arrival for j in done if j.kind == k])
        if len(lk):
            out["by_kind"][k] = {"jobs": int(len(lk)), "p50_s": float(np.percentile(lk, 50)),
                                 "p99_s": float(np.percentile(lk, 99))}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--quantum", type=int, default=50)
    ap.add_argument("--no-tune", action="store_true")
    args = ap.parse_args(argv)

    def log(s):
        print(s, file=sys.stderr, flush=True)

    jobs = poisson_jobs(args.rate, args.seconds, wall_fraction=0.15, aniso_fraction=0.15, film_fraction=0.1)
    srv = Server(precision=args.precision, hbm_budget=int(args.budget_gib * (1 << 30)), quantum=args.quantum,
                 log=log)
    if not args.no_tune:
        log(f"tuned shapes: {srv.tune_shapes(sorted({j.shape for j in jobs if j.batched}))}")
    done = srv.run(jobs)
    out = latency_summary(done)
    out.update(offered_jobs=len(jobs), rate=args.rate, stats=srv.stats)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
