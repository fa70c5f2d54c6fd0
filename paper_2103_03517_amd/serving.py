"""Continuous batching of m(T) jobs on one device.

Requests (one lattice size, one temperature, a sweep budget each) arrive over
time.  The loop admits waiting requests in arrival order whenever a slot is
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


class Job:
    """One m(T) request: `equil` unsampled sweeps, then `samples` sampled
    sweeps read every `block` sweeps."""

    def __init__(self, edge, T, equil=200, samples=800, block=100, seed=5, instance=0, Ku=0.01,
                 J=1.0, arrival=0.0, name=None):
        if samples % block or equil < 0 or samples <= 0 or block <= 0:
            raise ValueError("samples must be a positive multiple of block")
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
        return make_params(self.edge, self.edge, self.edge, precision=precision, J=self.J, Ku=self.Ku,
                           eu=(0.0, 0.0, 1.0), seed=self.seed, instance=self.instance, init="aligned")

    def sampling(self):
        return self.done >= self.equil

    def next_event(self):
        """Sweeps until this job's next phase change, block end or end."""
        if self.done < self.equil:
            return self.equil - self.done
        k = (self.done - self.equil) % self.block
        return self.block - k


def poisson_jobs(rate=20.0, seconds=10.0, seed=5, edges=(32, 48, 64, 96, 128, 160, 192),
                 t_lo=0.05, t_hi=1.7, **job_kw):
    """Poisson arrivals of m(T) jobs: exponential gaps of mean 1/rate, edges
    uniform over `edges`, temperatures uniform in [t_lo, t_hi)."""
    rng = np.random.default_rng(seed)
    jobs, t, i = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        jobs.append(Job(int(rng.choice(edges)), float(rng.uniform(t_lo, t_hi)), seed=seed, instance=i,
                        arrival=t, **job_kw))
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

    def need_bytes(self, job):
        return workspace_bytes(job.params(self.precision))

    def tune_shapes(self, edges, T=1.0, trial_sweeps=3):
        """One lattice per edge, tuned together in one batch."""
        lats = [Lattice(e, e, e, precision=self.precision, Ku=0.01, seed=1, instance=i)
                for i, e in enumerate(edges)]
        B = Batch(lats)
        shapes = B.tune([T] * len(lats), trial_sweeps)
        B.close()
        for l in lats:
            l.close()
        self.shapes.update({int(e): tuple(s) for e, s in zip(edges, shapes)})
        return dict(self.shapes)

    def _admit(self, job, now):
        p = job.params(self.precision)
        job.lattice = Lattice(job.edge, job.edge, job.edge, precision=self.precision, J=job.J, Ku=job.Ku,
                              eu=(0.0, 0.0, 1.0), seed=job.seed, instance=job.instance, init="aligned")
        assert job.lattice.params.seed == p.seed
        if job.edge in self.shapes:
            job.lattice.set_launch(*self.shapes[job.edge])
        job.admitted = now
        job.bytes = self.need_bytes(job)

    def _retire(self, job, now):
        job.result = block_stats_from_reads(job.reads, job.lattice.n, job.T)
        job.result.update(edge=job.edge, sweeps=job.reads[-1]["sweeps_done"],
                          theta_deg=job.reads[-1]["theta_deg"])
        job.finished = now
        job.lattice.close()
        job.lattice = None

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

        done = []
        while pending or waiting or active:
            now = clock()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting and len(active) < self.max_slots and used + self.need_bytes(waiting[0]) <= self.hbm_budget:
                j = waiting.popleft()
                self._admit(j, clock())
                used += j.bytes
                active.append(j)
                changed = True
            self.stats["max_active"] = max(self.stats["max_active"], len(active))
            self.stats["max_bytes"] = max(self.stats["max_bytes"], used)
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - clock()))
                continue
            if changed:
                if batch is not None:
                    batch.close()
                batch = Batch([j.lattice for j in active])
                if self.graph:
                    batch.set_graph(self.graph)
                self.stats["rebuilds"] += 1
                changed = False
            q = min(self.quantum, min(j.next_event() for j in active))
            batch.sweep_each([j.T for j in active], [j.sampling() for j in active], q)
            self.stats["ticks"] += 1
            self.stats["sweep_launches"] += q
            for j in active:
                j.done += q
            at_block_end = [j.sampling() and j.done > j.equil and (j.done - j.equil) % j.block == 0
                            for j in active]
            if any(at_block_end):
                obs = batch.observables()
                for j, o, hit in zip(active, obs, at_block_end):
                    if hit:
                        j.reads.append(o)
            finished = [j for j in active if j.done >= j.total]
            if finished:
                now = clock()
                for j in finished:
                    self._retire(j, now)
                    used -= j.bytes
                    done.append(j)
                active = [j for j in active if j.done < j.total]
                changed = True
                if self.log:
                    self.log(f"t={now:.3f}s retired {len(finished)}, active {len(active)}, "
                             f"waiting {len(waiting)}, pending {len(pending)}")
        if batch is not None:
            batch.close()
        torch.cuda.synchronize()
        return done


def latency_summary(done, window=None):
    lat = np.array([j.finished - j.arrival for j in done])
    span = window if window is not None else max(j.finished for j in done)
    updates = sum(j.edge ** 3 * j.total for j in done)
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
        log(f"tuned shapes: {srv.tune_shapes(sorted({j.edge for j in jobs}))}")
    done = srv.run(jobs)
    out = latency_summary(done)
    out.update(offered_jobs=len(jobs), rate=args.rate, stats=srv.stats)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
