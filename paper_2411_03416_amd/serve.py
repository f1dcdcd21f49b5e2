"""Continuous-batching request loop over the C ABI.

Requests (planning problems of uneven horizon N and state dimension n)
arrive over time.  Each state dimension has one resident context (its own
arena and stream) driven by its own host thread, and all of them share one
admission controller:

  * admission: a request waits in its queue until the engine has room for
    it: fewer than `max_concurrent` live plans in all contexts together, and
    the device bytes of the live plans plus its own within the HBM budget
    (each plan's bytes are what a context needs for exactly that plan, from
    the library's own sizing).  A request larger than the whole budget is
    admitted only when the engine is empty, so every request is served.
    Admitted plans join their context's batch between two iteration chunks;
  * iteration: every chunk runs `chunk` proximal iterations for all live
    plans of the context in one graph replay; a plan leaves when its budget
    is spent, nonlinear plans first taking their remaining rounds of
    statistical linearisation and prior rebuild (Alg. 2), all plans of a
    context that finish a round in the same chunk in one call;
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

from . import (EBUSY, ENOMEM, FP64, OK, PgvimpError, _heap_need, ipgvimp_begin, ipgvimp_next_round_many,
               pgvimp_add_plan, pgvimp_arena_bytes, pgvimp_create, pgvimp_destroy, pgvimp_get_state,
               pgvimp_marginals, pgvimp_prox_step, pgvimp_remove_plan, pgvimp_set_budget)


def plan_bytes(prob, trial_width, trial_slots):
    """Device bytes one plan of prob takes in a context: what a context for
    exactly this plan needs beyond an empty one."""
    n, N = int(prob["n"]), int(prob["N"])
    heap = _heap_need([prob])
    full = pgvimp_arena_bytes(n, 1, N, heap, trial_width, trial_slots)
    empty = pgvimp_arena_bytes(n, 1, 1, 0, trial_width, trial_slots)
    return max(full - empty, 1)


class Admission:
    """Shared budget of live plans and their device bytes."""

    def __init__(self, budget_bytes, max_concurrent):
        self.budget = int(budget_bytes)
        self.max_concurrent = int(max_concurrent)
        self.used = 0
        self.live = 0
        self.peak_used = 0
        self.peak_live = 0
        self.lock = threading.Lock()

    def try_take(self, nbytes):
        with self.lock:
            if self.live >= self.max_concurrent:
                return False
            if self.used + nbytes > self.budget and self.live > 0:
                return False
            self.used += nbytes
            self.live += 1
            self.peak_used = max(self.peak_used, self.used)
            self.peak_live = max(self.peak_live, self.live)
            return True

    def give(self, nbytes):
        with self.lock:
            self.used -= nbytes
            self.live -= 1


class _Lane:
    """One context (state dimension n) and the thread that drives it."""

    def __init__(self, n, precision, max_plans, max_states, heap_bytes, chunk, trial_width, trial_slots, use_graph,
                 admission):
        self.n = n
        self.chunk = chunk
        self.trial_width, self.trial_slots = trial_width, trial_slots
        self.queue = collections.deque()
        self.live = {}  # plan id -> request record
        self.adm = admission
        self.ctx = pgvimp_create([], n=n, precision=precision, max_plans=max_plans, max_states=max_states,
                                 heap_bytes=heap_bytes, use_graph=use_graph, trial_width=trial_width,
                                 trial_slots=trial_slots)
        self.done = []
        self.batch_sizes = []

    def admit(self, now):
        """Admit queued requests that have arrived and fit."""
        admitted = 0
        while self.queue and self.queue[0]["arrival"] <= now:
            req = self.queue[0]
            if "bytes" not in req:
                req["bytes"] = plan_bytes(req["prob"], self.trial_width, self.trial_slots)
            if not self.adm.try_take(req["bytes"]):
                break  # wait for plans to leave
            try:
                pid = pgvimp_add_plan(self.ctx, req["prob"], mu_init=req.get("mu_init"))
            except PgvimpError as e:
                self.adm.give(req["bytes"])
                if e.code in (EBUSY, ENOMEM) and self.live:
                    break  # this context is full: wait for one of its plans to leave
                # a problem the library rejects (for instance a prior that is
                # not positive definite, or one larger than an empty context)
                # is answered with its error
                self.queue.popleft()
                req["error"] = str(e)
                req["done"] = time.perf_counter()
                self.done.append(req)
                continue
            self.queue.popleft()
            req["admitted"] = time.perf_counter()
            req["rounds_left"] = 0
            self.live[pid] = req
            if "quad" in req["prob"]:
                try:
                    ipgvimp_begin(self.ctx, pid, req["prob"])
                    req["rounds_left"] = req["prob"].get("n_rounds", 1) - 1
                except PgvimpError as e:
                    req["error"] = str(e)
                    pgvimp_set_budget(self.ctx, pid, 0)
            admitted += 1
        return admitted

    def step(self):
        stats = pgvimp_prox_step(self.ctx, self.chunk)
        self.batch_sizes.append(len(self.live))
        finished, next_round = [], []
        for pid, req in list(self.live.items()):
            st = stats[pid]
            if st["iters_left"] > 0:
                continue
            if req["rounds_left"] > 0 and "error" not in req:
                next_round.append(pid)
                continue
            finished.append(pid)
        if next_round:
            prob = self.live[next_round[0]]["prob"]
            codes = ipgvimp_next_round_many(self.ctx, next_round, prob)
            for pid, code in zip(next_round, codes):
                req = self.live[pid]
                req["rounds_left"] -= 1
                if code != OK:
                    req["error"] = "linearised prior not positive definite"
                    finished.append(pid)
        for pid in finished:
            req = self.live.pop(pid)
            mu, _, _ = pgvimp_get_state(self.ctx, pid)
            S, _, _ = pgvimp_marginals(self.ctx, pid) if "error" not in req else (None, None, None)
            req["result"] = {"mu": mu, "cov_diag": S, "stats": stats[pid]}
            req["done"] = time.perf_counter()
            pgvimp_remove_plan(self.ctx, pid)
            self.adm.give(req["bytes"])
            self.done.append(req)
        return len(finished)

    def run(self, t0, deadline):
        while True:
            now = time.perf_counter() - t0
            self.admit(now)
            if self.live:
                self.step()
            elif self.queue:
                wait = self.queue[0]["arrival"] - (time.perf_counter() - t0)
                time.sleep(min(max(wait, 0.0), 0.002) if wait > 0 else 0.0005)
            else:
                return
            if time.perf_counter() > deadline:
                return

    def close(self):
        pgvimp_destroy(self.ctx)


class ServingEngine:
    """Continuous batching of planning requests on one GPU.

    hbm_budget: device bytes the live plans may take together (admission);
    each context's arena is sized to hold that much of its own kind of plans
    (at least one plan of max_N states).  max_concurrent: live plans in all
    contexts together."""

    def __init__(self, precision=FP64, hbm_budget=16 << 30, max_concurrent=256, chunk=2, trial_width=None,
                 trial_slots=None, dims=(4, 6, 14), max_N=1000, use_graph=2, serial=False, max_map_bytes=None):
        self.precision = precision
        self.serial = serial
        self.adm = Admission(hbm_budget, 1 if serial else max_concurrent)
        self.lanes = {}
        for n in dims:
            # trial windows (None: 8 step sizes for n <= 4; 24 for n >= 6, whose
            # trials are long latency-bound chains, so one wide window beats
            # several narrow ones in a row)
            tw = trial_width if trial_width is not None else (8 if n <= 4 else 24)
            ts = trial_slots if trial_slots is not None else tw
            # arena: states and heap for the budget's worth of this lane's plans
            # the largest map a plan brings, with its table of cell corners (16
            # bytes a cell): a 128^3 grid for the arm, else a 500 x 500 grid
            m = max_map_bytes if max_map_bytes is not None else (
                128 ** 3 * 4 + 127 * 127 * 128 * 16 if n == 14 else 500 * 500 * 4 + 499 * 499 * 16)
            per_state = (pgvimp_arena_bytes(n, 1, 1001, 0, tw, ts) - pgvimp_arena_bytes(n, 1, 1, 0, tw, ts)) / 1000.0
            plans = 1 if serial else max_concurrent
            states = int(min(plans * max_N, max(max_N, hbm_budget / per_state)))
            # heap per plan: its map and FP64 model (per interval A, a, B,
            # plus fixed blocks), with slack for alignment
            one = m + 8 * (max_N * (n * n + n + n * (n // 2)) + 8 * n * n) + (64 << 10)
            heap = int(min(plans * one, max(one, hbm_budget)))
            self.lanes[n] = _Lane(n, precision, plans, states, heap, chunk, tw, ts, use_graph, self.adm)

    def run(self, requests, timeout_s=600.0, measured_from=0):
        """requests: list of (arrival_s, problem).  Metrics cover the
        requests from index measured_from on (the earlier ones warm up):
        plans/s = measured completions / (last measured completion - first
        measured arrival).  Returns metrics and the request records."""
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
        meas = [r for r in recs[measured_from:]]
        done = [r for r in meas if "done" in r and "error" not in r]
        lat = np.array([r["done"] - r["arrival_abs"] for r in done]) if done else np.zeros(0)
        wait = np.array([r["admitted"] - r["arrival_abs"] for r in done if "admitted" in r])
        span = (max(r["done"] for r in done) - min(r["arrival_abs"] for r in meas)) if done else 0.0
        bs = [b for lane in self.lanes.values() for b in lane.batch_sizes]
        return {
            "requests": len(meas), "completed": len(done),
            "errors": sum(1 for r in meas if "error" in r), "wall_s": wall,
            "plans_per_s": len(done) / span if span > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "admission_wait_p99_ms": float(np.percentile(wait, 99) * 1e3) if wait.size else None,
            "mean_batch": float(np.mean(bs)) if bs else 0.0,
            "peak_live": self.adm.peak_live, "peak_bytes": self.adm.peak_used,
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
