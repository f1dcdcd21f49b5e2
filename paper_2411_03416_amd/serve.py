"""Continuous-batching request loop over the C ABI.

Requests (planning problems of uneven horizon N and state dimension n)
arrive over time.  Each state dimension has one resident context (its own
arena and stream) driven by its own host thread:

  * admission: a request waits in its queue until `pgvimp_add_plan` finds a
    free slot, states and map memory in the context (the context's arena is
    the HBM budget); it then joins the batch between two iteration chunks;
  * iteration: every chunk runs `chunk` proximal iterations for all live
    plans of the context in one graph replay; plans leave when their budget
    is spent (nonlinear plans first take their remaining rounds of
    statistical linearisation and prior rebuild, Alg. 2);
  * completion: the plan's mean and marginal covariances are read back and
    its slot, states and memory are freed.

Contexts of different state dimensions run concurrently on their own
streams (the ctypes calls release the interpreter lock).  Latency of a
request = completion time - arrival time.
"""
from __future__ import annotations

import collections
import threading
import time

import numpy as np

from . import (FP64, PgvimpError, ipgvimp_begin, ipgvimp_next_round, pgvimp_add_plan, pgvimp_arena_bytes,
               pgvimp_create, pgvimp_destroy, pgvimp_get_state, pgvimp_marginals, pgvimp_prox_step,
               pgvimp_remove_plan, EBUSY, ENOMEM)


def _heap_for(prob):
    sdf = int(np.asarray(prob["sdf"]).size) * 4 + 256 if prob.get("coll_kind", "none") != "none" else 0
    n, m, N = prob["n"], prob["m"], prob["N"]
    return sdf + 8 * (4 * n * n + 2 * n + m * m + max(N - 1, 1) * (n * n + n + n * m) + 100) + 512


class _Lane:
    """One context (state dimension n) and the thread that drives it."""

    def __init__(self, n, precision, max_plans, max_states, heap_bytes, chunk, trial_width, use_graph):
        self.n = n
        self.chunk = chunk
        self.queue = collections.deque()
        self.live = {}  # plan id -> request record
        self.lock = threading.Lock()
        self.ctx = pgvimp_create([], n=n, precision=precision, max_plans=max_plans, max_states=max_states,
                                 heap_bytes=heap_bytes, use_graph=use_graph, trial_width=trial_width)
        self.done = []
        self.batch_sizes = []

    def admit(self, now):
        """Admit queued requests that have arrived and fit."""
        admitted = 0
        while self.queue and self.queue[0]["arrival"] <= now:
            req = self.queue[0]
            try:
                pid = pgvimp_add_plan(self.ctx, req["prob"], mu_init=req.get("mu_init"))
            except PgvimpError as e:
                if e.code in (EBUSY, ENOMEM):
                    break  # wait for a plan to leave
                raise
            self.queue.popleft()
            req["admitted"] = time.perf_counter()
            req["rounds_left"] = 0
            if "quad" in req["prob"]:
                ipgvimp_begin(self.ctx, pid, req["prob"])
                req["rounds_left"] = req["prob"].get("n_rounds", 1) - 1
            self.live[pid] = req
            admitted += 1
        return admitted

    def step(self):
        stats = pgvimp_prox_step(self.ctx, self.chunk)
        self.batch_sizes.append(len(self.live))
        finished = []
        for pid, req in list(self.live.items()):
            st = stats[pid]
            if st["iters_left"] > 0:
                continue
            if req["rounds_left"] > 0:
                ipgvimp_next_round(self.ctx, pid, req["prob"])
                req["rounds_left"] -= 1
                continue
            mu, _, _ = pgvimp_get_state(self.ctx, pid)
            S, _, _ = pgvimp_marginals(self.ctx, pid)
            req["result"] = {"mu": mu, "cov_diag": S, "stats": st}
            req["done"] = time.perf_counter()
            finished.append(pid)
        for pid in finished:
            pgvimp_remove_plan(self.ctx, pid)
            self.done.append(self.live.pop(pid))
        return len(finished)

    def run(self, t0, deadline):
        while True:
            now = time.perf_counter() - t0
            self.admit(now)
            if self.live:
                self.step()
            elif self.queue:
                wait = self.queue[0]["arrival"] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            else:
                return
            if time.perf_counter() > deadline:
                return

    def close(self):
        pgvimp_destroy(self.ctx)


class ServingEngine:
    """Continuous batching of planning requests on one GPU."""

    def __init__(self, precision=FP64, hbm_budget=16 << 30, max_plans=256, chunk=2, trial_width=8,
                 dims=(4, 6, 14), max_N=1000, use_graph=2, serial=False):
        self.precision = precision
        self.serial = serial
        self.lanes = {}
        share = hbm_budget // len(dims)
        for n in dims:
            plans = 1 if serial else max_plans
            # states and heap sized so that the arena fits the budget share
            heap = plans * (_heap_for({"coll_kind": "x", "sdf": np.zeros(128 ** 3 if n == 14 else 500 * 500),
                                       "n": n, "m": n // 2, "N": max_N}))
            states = plans * max_N
            while states > max_N and pgvimp_arena_bytes(n, plans, states, heap, trial_width) > share:
                states = int(states * 0.8)
                heap = int(heap * 0.8)
            self.lanes[n] = _Lane(n, precision, plans, max(states, max_N), heap, chunk, trial_width,
                                  use_graph)

    def run(self, requests, timeout_s=600.0):
        """requests: list of (arrival_s, problem).  Returns metrics and the
        completed request records."""
        recs = []
        for k, (t, prob) in enumerate(requests):
            rec = {"id": k, "arrival": float(t), "prob": prob}
            recs.append(rec)
            self.lanes[prob["n"]].queue.append(rec)
        t0 = time.perf_counter()
        for rec in recs:
            rec["arrival_abs"] = t0 + rec["arrival"]
        deadline = t0 + timeout_s
        if self.serial:
            self._run_serial(recs, t0, deadline)
        else:
            threads = [threading.Thread(target=lane.run, args=(t0, deadline)) for lane in self.lanes.values()]
            for th in threads:
                th.start()
            for th in threads:
                th.join()
        wall = time.perf_counter() - t0
        done = [r for r in recs if "done" in r]
        lat = np.array([r["done"] - r["arrival_abs"] for r in done]) if done else np.zeros(0)
        bs = [b for lane in self.lanes.values() for b in lane.batch_sizes]
        return {
            "requests": len(recs), "completed": len(done), "wall_s": wall,
            "plans_per_s": len(done) / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_batch": float(np.mean(bs)) if bs else 0.0,
        }, recs

    def _run_serial(self, recs, t0, deadline):
        """Baseline: one plan at a time in arrival order."""
        for rec in sorted(recs, key=lambda r: r["arrival"]):
            lane = self.lanes[rec["prob"]["n"]]
            now = time.perf_counter() - t0
            if rec["arrival"] > now:
                time.sleep(rec["arrival"] - now)
            lane.queue.clear()
            lane.queue.append(rec)
            lane.admit(time.perf_counter() - t0)
            while lane.live and time.perf_counter() < deadline:
                lane.step()
            if time.perf_counter() > deadline:
                return

    def close(self):
        for lane in self.lanes.values():
            lane.close()
