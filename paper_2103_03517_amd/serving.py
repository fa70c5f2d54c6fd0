"""Continuous batching of m(T) and domain-wall jobs on one device.

Requests (one lattice, one temperature, a sweep budget each) arrive over
time.  An m(T) job runs a periodic cube and reports <|m|>, chi and E with
batch-means errors; a wall job runs a lattice that is anti-periodic along z
from a sharp wall and reports the fitted wall width (Sec. 3, Eq. 5).  The loop admits waiting requests in arrival order whenever a slot is
free and their workspace fits in the HBM budget, advances every admitted job
together through the batch interface (one launch per colour pass for all of
them, each job with its own temperature and its own sample flag), reads the
observables at the jobs' block ends, and retires finished jobs, releasing
their memory for the next admissions.  Jobs that arrive while others run join
the batch at the next tick, so their work overlaps on the device.

A job's chain depends only on its own key (seed, instance), its temperature,
its sweep schedule and its launch shape, so its result is the same alone and
in any mix (tests check this bit for bit).

    python -m paper_2103_03517_amd.serving --rate 20 --seconds 10
"""
import argparse
import collections
import json
import sys
import time

import numpy as np
import torch

from . import Batch, Lattice, workspace_bytes, make_params
from .protocols import block_stats_from_reads
from . import walls as W


class Job:
    """One request: `equil` unsampled sweeps, then `samples` sampled sweeps
    read every `block` sweeps.  kind "mt": an edge^3 periodic cube started
    along z; kind "wall": a shape = (nx, ny, nz) lattice anti-periodic along
    z, started from a sharp wall, whose m_z plane profile is kept at every
    block end and fitted when the job retires."""

    def __init__(self, edge, T, equil=200, samples=800, block=100, seed=5, instance=0, Ku=0.01,
                 J=1.0, arrival=0.0, name=None, kind="mt", shape=None):
        if samples % block or equil < 0 or samples <= 0 or block <= 0:
            raise ValueError("samples must be a positive multiple of block")
        if kind not in ("mt", "wall"):
            raise ValueError(f"unknown job kind {kind}")
        self.kind = kind
        self.shape = tuple(int(v) for v in shape) if shape is not None else (int(edge),) * 3
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.profiles = []
        self.edge, self.T = int(edge), float(T)
        self.equil, self.samples, self.block = int(equil), int(samples), int(block)
        self.seed, self.instance, self.Ku, self.J = int(seed), int(instance), float(Ku), float(J)
        self.arrival = float(arrival)
        self.name = name if name is not None else f"job{instance}"
        self.done = 0
        self.reads = []
        self.lattice = None
        self.admitted = self.finished = None
        self.result = None

    @property
    def total(self):
        return self.equil + self.samples

    def params(self, precision):
        return make_params(*self.shape, precision=precision, J=self.J, Ku=self.Ku, eu=(0.0, 0.0, 1.0),
                           seed=self.seed, instance=self.instance, init="aligned",
                           boundary_z="antiperiodic" if self.kind == "wall" else "periodic")

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
                 wall_sweeps=(1000, 1000, 100), **job_kw):
    """Poisson arrivals: exponential gaps of mean 1/rate.  With probability
    wall_fraction a job is a wall job on wall_shape at T ~ U(t_lo,
    wall_t_hi) with (equil, samples, block) = wall_sweeps; otherwise an m(T)
    job with the edge uniform over `edges` and T ~ U(t_lo, t_hi)."""
    rng = np.random.default_rng(seed)
    jobs, t, i = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        edge = int(rng.choice(edges))
        T = float(rng.uniform(t_lo, t_hi))
        if rng.uniform() < wall_fraction:
            eq, smp, blk = wall_sweeps
            T = t_lo + (T - t_lo) * (wall_t_hi - t_lo) / (t_hi - t_lo)
            jobs.append(Job(edge, T, equil=eq, samples=smp, block=blk, seed=seed, instance=i, arrival=t,
                            kind="wall", shape=wall_shape,
                            **{k: v for k, v in job_kw.items() if k not in ("equil", "samples", "block")}))
        else:
            jobs.append(Job(edge, T, seed=seed, instance=i, arrival=t, **job_kw))
        i += 1
    return jobs


class Server:
    """The continuous-batching loop.  `shapes` maps an edge to the launch
    shape (sites per thread, z chunk) its lattices use; `quantum` is the
    largest number of sweeps enqueued per tick."""

    def __init__(self, precision=32, hbm_budget=32 << 30, max_slots=64, quantum=50, shapes=None,
                 graph=0, log=None):
        self.precision = int(precision)
        self.hbm_budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.quantum = int(quantum)
        self.shapes = dict(shapes or {})
        self.graph = int(graph)
        self.log = log
        self.stats = {"ticks": 0, "rebuilds": 0, "max_active": 0, "max_bytes": 0, "sweep_launches": 0}
        # host seconds per phase of the loop (the device waits during admit,
        # rebuild and retire, which follow a synchronising read)
        self.phase_s = {"admit": 0.0, "rebuild": 0.0, "enqueue": 0.0, "read": 0.0, "retire": 0.0}

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

    def _admit(self, job, now):
        if job.kind == "wall":
            # the T = 0 wall profile, written on the device
            job.lattice = Lattice(*job.shape, precision=self.precision, J=job.J, Ku=job.Ku, eu=(0.0, 0.0, 1.0),
                                  seed=job.seed, instance=job.instance, init="wall",
                                  init_width=W.zero_temperature_width(job.J, job.Ku), boundary_z="antiperiodic")
        else:
            job.lattice = Lattice(*job.shape, precision=self.precision, J=job.J, Ku=job.Ku, eu=(0.0, 0.0, 1.0),
                                  seed=job.seed, instance=job.instance, init="aligned")
        if job.shape in self.shapes:
            job.lattice.set_launch(*self.shapes[job.shape])
        job.admitted = now
        job.bytes = self.need_bytes(job)

    @staticmethod
    def _fit_walls(job):
        fits = []
        for prof in job.profiles:
            try:
                fits.append(W.fit_wall(prof, delta_guess=W.zero_temperature_width(job.J, job.Ku)))
            except RuntimeError:
                pass
        if fits:
            f = np.array(fits)
            job.result.update(delta=float(f[:, 2].mean()), m_wall=float(f[:, 0].mean()), wall_fits=len(f))

    def _retire(self, job, now, pool, clock):
        job.result = block_stats_from_reads(job.reads, job.lattice.n, job.T)
        job.result.update(edge=job.edge, shape=list(job.shape), kind=job.kind,
                          sweeps=job.reads[-1]["sweeps_done"], theta_deg=job.reads[-1]["theta_deg"])
        job.lattice.close()
        job.lattice = None
        if job.kind == "wall":
            # the profile fits run beside the loop (the main thread mostly
            # waits on the device); the job finishes when its fits are done
            def work(j=job):
                self._fit_walls(j)
                j.finished = clock()
            return pool.submit(work)
        job.finished = now
        return None

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
        active = []
        used = 0
        batch = None
        changed = True
        if not realtime:
            for j in pending:
                j.arrival = 0.0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=2)
        futures = []
        done = []
        while pending or waiting or active:
            now = clock()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            t_ph = time.perf_counter()
            while waiting and len(active) < self.max_slots and used + self.need_bytes(waiting[0]) <= self.hbm_budget:
                j = waiting.popleft()
                self._admit(j, clock())
                used += j.bytes
                active.append(j)
                changed = True
            self.phase_s["admit"] += time.perf_counter() - t_ph
            self.stats["max_active"] = max(self.stats["max_active"], len(active))
            self.stats["max_bytes"] = max(self.stats["max_bytes"], used)
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - clock()))
                continue
            if changed:
                t_ph = time.perf_counter()
                if batch is None:
                    # one batch for the whole run, sized for max_slots lattices
                    batch = Batch([j.lattice for j in active], capacity=self.max_slots)
                    if self.graph:
                        batch.set_graph(self.graph)
                else:
                    batch.set_lattices([j.lattice for j in active])
                self.stats["rebuilds"] += 1
                changed = False
                self.phase_s["rebuild"] += time.perf_counter() - t_ph
            q = min(self.quantum, min(j.next_event() for j in active))
            t_ph = time.perf_counter()
            batch.sweep_each([j.T for j in active], [j.sampling() for j in active], q)
            self.phase_s["enqueue"] += time.perf_counter() - t_ph
            self.stats["ticks"] += 1
            self.stats["sweep_launches"] += q
            for j in active:
                j.done += q
            at_block_end = [j.sampling() and j.done > j.equil and (j.done - j.equil) % j.block == 0
                            for j in active]
            t_ph = time.perf_counter()
            if any(at_block_end):
                obs = batch.observables()
                for j, o, hit in zip(active, obs, at_block_end):
                    if hit:
                        j.reads.append(o)
                        if j.kind == "wall":
                            j.profiles.append(j.lattice.plane_means()[:, 2])
            self.phase_s["read"] += time.perf_counter() - t_ph
            finished = [j for j in active if j.done >= j.total]
            t_ph = time.perf_counter()
            if finished:
                now = clock()
                for j in finished:
                    f = self._retire(j, now, pool, clock)
                    if f is not None:
                        futures.append(f)
                    used -= j.bytes
                    done.append(j)
                active = [j for j in active if j.done < j.total]
                changed = True
                if self.log:
                    self.log(f"t={now:.3f}s retired {len(finished)}, active {len(active)}, "
                             f"waiting {len(waiting)}, pending {len(pending)}")
            self.phase_s["retire"] += time.perf_counter() - t_ph
        if batch is not None:
            batch.close()
        for f in futures:
            f.result()
        pool.shutdown()
        torch.cuda.synchronize()
        return done


def latency_summary(done, window=None):
    lat = np.array([j.finished - j.arrival for j in done])
    span = window if window is not None else max(j.finished for j in done)
    updates = sum(j.n * j.total for j in done)
    return {"jobs": len(done), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "span_s": float(span),
            "jobs_per_s": len(done) / span, "updates_per_s": updates / span}


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

    jobs = poisson_jobs(args.rate, args.seconds)
    srv = Server(precision=args.precision, hbm_budget=int(args.budget_gib * (1 << 30)), quantum=args.quantum,
                 log=log)
    if not args.no_tune:
        log(f"tuned shapes: {srv.tune_shapes(sorted({j.shape for j in jobs}))}")
    done = srv.run(jobs)
    out = latency_summary(done)
    out.update(offered_jobs=len(jobs), rate=args.rate, stats=srv.stats)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
