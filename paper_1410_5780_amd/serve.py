"""Serving driver: a seeded Poisson stream of shading jobs through the serving
loop (pv3d_submit / pv3d_poll / pv3d_wait), with p50 / p99 latency
(completion minus arrival) reported beside throughput.

Requests follow the serving workload of the workloads module: Poisson
arrivals, scenes drawn with Zipf popularity from a pool of synthetic sites
(10k to 1M triangles), each job a run of 1 to 4,379 consecutive suns of the
year and a row plant of 60 to 24,000 cells. Scenes stay resident once loaded
(least recently used ones are released when the budget runs short);
generators are cached by size. Arrivals are paced in real time.
"""
from __future__ import annotations

import collections
import threading
import time
from typing import Dict, List, Optional

import numpy as np

from . import pv3d
from . import workloads as W


class Pool:
    """Device-resident scenes and generators of the stream, least recently used released first."""

    def __init__(self, ctx: pv3d.Context, seed: int):
        self.ctx, self.seed = ctx, seed
        self.scenes: "collections.OrderedDict[int, int]" = collections.OrderedDict()
        self.gens: Dict[int, tuple] = {}
        self.loads = 0

    def scene(self, sid: int) -> int:
        if sid in self.scenes:
            self.scenes.move_to_end(sid)
            return self.scenes[sid]
        sc = W.serving_scene(self.seed, sid)
        while True:
            try:
                h = self.ctx.load_scene(sc)
                break
            except pv3d.Pv3dError as e:
                if e.code != pv3d.ENOMEM or not self._evict():
                    raise
        self.scenes[sid] = h
        self.loads += 1
        return h

    def _evict(self) -> bool:
        for sid in list(self.scenes):
            try:
                self.ctx.release_scene(self.scenes[sid])
            except pv3d.Pv3dError:
                continue                       # still used by a running job
            del self.scenes[sid]
            return True
        return False

    def generator(self, n_cells: int):
        if n_cells not in self.gens:
            g = W.site_generator(n_cells)
            self.gens[n_cells] = (self.ctx.define_generator(g), g)
        return self.gens[n_cells]


def run_stream(ctx: pv3d.Context, reqs: List[W.Request], seed: int = 5, k: int = 8,
               year: Optional[W.Sweep] = None, poll_s: float = 0.0005, log=None) -> dict:
    """Submit every request at its arrival time; returns latency percentiles and throughput."""
    yr = year if year is not None else W.year_sweep()
    pool = Pool(ctx, seed)
    for r in reqs:                              # scenes and generators before the clock starts
        pool.scene(r.scene_id)
        pool.generator(r.n_cells)
    done: Dict[int, float] = {}
    failed: Dict[int, str] = {}
    outstanding: Dict[int, int] = {}
    lock = threading.Lock()
    stop = threading.Event()

    def watcher():
        # a job that fails is recorded, never raised here: an exception would end this thread
        # and leave the stream waiting for it forever
        last = time.perf_counter()
        while not stop.is_set() or outstanding:
            with lock:
                items = list(outstanding.items())
            for t, i in items:
                try:
                    if not ctx.poll(t):
                        continue
                    now = time.perf_counter()
                    ctx.wait(t)
                except pv3d.Pv3dError as e:
                    now = time.perf_counter()
                    failed[i] = str(e)
                with lock:
                    done[i] = now
                    del outstanding[t]
            if log and time.perf_counter() - last > 2.0:
                last = time.perf_counter()
                st = ctx.serve_stats()
                log(f"[serve] {len(done)} of {len(reqs)} done, {len(outstanding)} running or waiting; loop: "
                    f"{st['jobs_done']} jobs done, {st['launches']} launches, {st['items']} items, "
                    f"{st['pending']} pending admission")
            time.sleep(poll_s)

    th = threading.Thread(target=watcher, daemon=True)
    arrival = {}
    samples = 0
    t0 = time.perf_counter()
    th.start()
    try:
        for i, r in enumerate(reqs):
            target = t0 + r.arrival_s
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                time.sleep(min(target - now, 0.001))
            gh, g = pool.generator(r.n_cells)
            spec = dict(scene=pool.scene(r.scene_id), gen=gh, generator=g, sweep=yr.subset(r.sun_idx),
                        map_n=r.map_n, k=k, counts=False)
            arrival[i] = time.perf_counter()
            t = ctx.submit(spec, device=True)
            samples += g.n_cells * k * k * len(r.sun_idx)
            with lock:
                outstanding[t] = i
    finally:
        stop.set()
        th.join()
    if failed:
        raise RuntimeError(f"{len(failed)} of {len(reqs)} serving jobs failed, first: {next(iter(failed.values()))}")
    t1 = time.perf_counter()
    lat = np.array([done[i] - arrival[i] for i in range(len(reqs))])
    st = ctx.serve_stats()
    out = {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
           "wall_s": t1 - t0, "offered_s": reqs[-1].arrival_s if reqs else 0.0,
           "tests_per_s": samples / (t1 - t0), "tests": samples, "suns": int(sum(len(r.sun_idx) for r in reqs)),
           "launches": st["launches"], "scene_loads": pool.loads}
    if log:
        log(f"[serve] {out}")
    return out
