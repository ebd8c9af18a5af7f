"""Continuous-batching service of stationary-vector solves.

Requests (independent block generators) arrive over time.  The service
admits them in arrival order while the HBM footprint of the admitted chains
stays under a budget and a batch slot is free, keeps every admitted chain's
factored blocks and iterate resident on the device, and sweeps all admitted
chains together with the batched (multi-chain) launch.  A
chain in its FP32 stage that meets the switch tolerance, or whose FP32
change has stopped falling (its rounding floor lies above the switch
tolerance), is promoted to FP64 (stc_promote); a chain whose FP64 change
meets the tolerance is retired: its
vector is copied out, its memory freed, and waiting requests are admitted.
A chain that reaches the per-request sweep cap is retired the same way with
status STC_EMAXIT (its last iterate is returned).  A request whose setup
fails (not a generator, a singular diagonal block, a bad shape) or whose
sweeps lose all mass is rejected on its own; the service goes on.
Setup of new chains overlaps the work already on the GPU, and only the
serving thread calls into the HIP runtime:

- the host half of each admitted request's setup (validation, and packing
  of its blocks in the sweep's layout: stc_prepare) runs on a prepare
  thread, which makes no HIP call (prepare_thread=True, the default);
- the device half (upload, inverse of the diagonal blocks, state:
  stc_setup_prepared) runs on the serving thread, on a side stream, right
  after it has enqueued a round of sweeps and before it waits for them.

The requests set up join the next round.  prepare_thread=False does both
halves on the serving thread.  setup_thread=True runs the whole setup on a
host thread of its own instead.  That form is off by default: twice it
ended in a segmentation fault of the process inside the batch's graph
capture and launch (stc_batch_sweeps) on the serving thread while the
setup thread was inside stc_setup, in runs of the 512-request stream with
Poisson arrivals.

The batch's sweeps are plain launches by default (use_graph=False).  With
graph replay (use_graph=True), three runs of the 512-request stream with
Poisson arrivals ended in a segmentation fault of the process inside
stc_batch_sweeps on the serving thread, the third with no other thread in
the runtime.  Those runs capture the batch's graph again whenever the block
sizes or precision stages present change, thousands of times; runs with
all requests at t = 0 (few captures) never did.

Every step of the method runs in libstc.so; this module schedules calls.
"""
from __future__ import annotations

import queue
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import stc


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    blocks: np.ndarray        # [L][2b+1][m][m] generator blocks
    sizes: np.ndarray | None
    b: int = 1


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    pi: np.ndarray
    sweeps: int
    sweeps_fp32: int
    footprint: int
    status: int = stc.STC_OK    # STC_OK, or STC_EMAXIT at the sweep cap

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    results: list = field(default_factory=list)
    wall: float = 0.0
    peak_chains: int = 0
    peak_bytes: int = 0
    rounds: int = 0
    rejected: list = field(default_factory=list)
    errors: dict = field(default_factory=dict)    # rid -> why it was rejected

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        first = min((r.arrival for r in self.results), default=0.0)
        last = max((r.done for r in self.results), default=0.0)
        return {
            "completed": len(self.results),
            "maxit": sum(1 for r in self.results if r.status != stc.STC_OK),
            "rejected": len(self.rejected),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "solves_per_s": len(self.results) / max(last - first, 1e-9),
            "wall_s": self.wall,
            "peak_chains": self.peak_chains,
            "peak_bytes": self.peak_bytes,
            "batch_rounds": self.rounds,
        }


class _Floor32:
    """The FP32 stage's rounding floor, per request: the change read after
    each round either makes a new low or not; `rounds` readings in a row with
    no new low mean the FP32 sweeps have stopped converging (a converging
    stage makes a new low at every reading), whatever switch_tol asks."""

    def __init__(self, rounds: int):
        self.rounds = rounds
        self.state = {}

    def reached(self, rid, diff: float) -> bool:
        low, stale = self.state.get(rid, (float("inf"), 0))
        if diff < low:
            self.state[rid] = (diff, 0)
            return False
        self.state[rid] = (low, stale + 1)
        return stale + 1 >= self.rounds


class Server:
    """Admission by footprint, continuous batching, FP32 -> FP64 promotion.

    nontemporal: stream the blocks with non-temporal loads (the admitted
    chains together exceed the last-level cache under any useful budget).
    max_sweeps: sweeps (both stages) after which a request that has not met
    its tolerance is retired with STC_EMAXIT.
    prepare_thread: the host half of setup on a thread of its own (see the
    module notes).
    setup_thread: the whole setup on a thread of its own (off: see the
    module notes).
    use_graph: replay the batch's sweeps as a captured hipGraph (off: see
    the module notes)."""

    def __init__(self, budget_bytes: int, *, max_chains: int = 64, max_items: int = 1 << 17,
                 sweeps_per_round: int = 20, tol: float = 1e-13, switch_tol: float = 1e-6,
                 precision: str = "mixed", nontemporal: bool = True, device=None,
                 b: int = 1, use_graph: bool = False, max_sweeps: int = 1_000_000,
                 prepare_thread: bool = True, setup_thread: bool = False):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_chains = int(max_chains)
        self.K = int(sweeps_per_round)
        self.tol = float(tol)
        self.switch_tol = float(switch_tol)
        self.precision = precision
        self.nontemporal = bool(nontemporal)
        self.use_graph = use_graph
        self.max_sweeps = int(max_sweeps)
        self.setup_thread = bool(setup_thread)
        self.prepare_thread = bool(prepare_thread)
        self.device = torch.device(device if device is not None else "cuda")
        self.setup_stream = torch.cuda.Stream(device=self.device)
        self.batch = stc.Batch(self.max_chains, max_items, b=b, device=self.device)

    def footprint(self, req: Request) -> int:
        gen, _keep = stc.make_generator(req.blocks, req.sizes, req.b)
        opt = stc.make_options(self.precision, 1, "diff", 1, self.switch_tol)
        return stc.stc_footprint_bytes(gen, opt)

    def autotune(self, probes, trial_sweeps: int = 10) -> float:
        """Tune the batch's launch shapes (stc_batch_autotune) before serving,
        on probe chains (Requests) standing in for the stream.  Under mixed
        precision each probe is set up twice, sweeping in FP32 and in FP64,
        so that both stages are tuned; probes beyond the batch's slots are
        left out.  The probes are released afterwards; the shapes stay with
        the batch and apply to every chain admitted later.  Returns the
        probes' batched sweep time in ms."""
        precs = ("fp32", "fp64") if self.precision == "mixed" else (self.precision,)
        probes = list(probes)[: max(1, self.max_chains // len(precs))]
        solvers = []
        try:
            for req in probes:
                for prec in precs:
                    s = stc.Solver(req.blocks, req.sizes, req.b, precision=prec,
                                   device=self.device, stream=self.setup_stream)
                    s.load(None)
                    solvers.append(s)
            self.setup_stream.synchronize()
            self.batch.set(solvers, self.tol, self.nontemporal)
            ms = self.batch.autotune(trial_sweeps)
            self.batch.set([], self.tol, self.nontemporal)
        finally:
            for s in solvers:
                s.close()
        return ms

    def _admit(self, req: Request) -> stc.Solver:
        # the batch gives the chain its launch variants when it joins
        s = stc.Solver(req.blocks, req.sizes, req.b, precision=self.precision,
                       switch_tol=self.switch_tol, device=self.device,
                       stream=self.setup_stream)
        s.load(None)
        return s

    def _prepare_worker(self, todo: "queue.Queue", done: "queue.Queue"):
        """The host half of the setup of admitted requests, in order: no HIP
        call and no torch device state.  Each stc.Prepared (or the error its
        validation raised) goes to `done`."""
        while True:
            job = todo.get()
            if job is None:
                return
            req, fp = job
            try:
                p = stc.Prepared(req.blocks, req.sizes, req.b, precision=self.precision,
                                 switch_tol=self.switch_tol)
                done.put((req, p, fp, None))
            except Exception as e:          # reported by the serving loop
                done.put((req, None, fp, e))

    def _finish(self, prep: "stc.Prepared") -> stc.Solver:
        # the device half, on the serving thread; the batch gives the chain
        # its launch variants when it joins
        s = stc.Solver.from_prepared(prep, device=self.device, stream=self.setup_stream)
        s.load(None)
        return s

    def _setup_worker(self, todo: "queue.Queue", ready: "queue.Queue"):
        """Set up admitted requests in order; each ready solver (or the error
        its setup raised) goes to `ready`."""
        import torch
        with torch.cuda.device(self.device):
            while True:
                job = todo.get()
                if job is None:
                    return
                req, fp = job
                try:
                    s = self._admit(req)
                    self.setup_stream.synchronize()
                    ready.put((req, s, fp, None))
                except Exception as e:          # reported by the serving loop
                    ready.put((req, None, fp, e))

    def run(self, requests, clock=time.perf_counter) -> ServeStats:
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = deque(reqs)
        waiting: deque = deque()
        active = []          # [request, solver, footprint, admitted_at, stage(, fp32 sweeps)]
        fps = {}
        used = 0
        in_setup = 0         # admitted, not yet set up or not yet active
        to_setup = []        # inline setup: admitted requests to set up this round
        stats = ServeStats()
        # readings spanning at least 4 rounds and 128 sweeps, as stc_solve's
        floor32 = _Floor32(max(4, -(-128 // self.K)))
        todo: queue.Queue = queue.Queue()
        ready: queue.Queue = queue.Queue()     # solvers set up (or errors)
        done: queue.Queue = queue.Queue()      # prepared host halves (or errors)
        mode = ("thread" if self.setup_thread else
                "prepare" if self.prepare_thread else "inline")
        worker = None
        if mode == "thread":
            worker = threading.Thread(target=self._setup_worker, args=(todo, ready), daemon=True)
        elif mode == "prepare":
            worker = threading.Thread(target=self._prepare_worker, args=(todo, done), daemon=True)
        if worker is not None:
            worker.start()
        t0 = clock()
        dirty = False

        def join(item):
            """A chain whose setup finished joins the batch; a failed setup
            rejects its request alone."""
            nonlocal in_setup, used, dirty
            req, s, fp, err = item
            in_setup -= 1
            if err is not None:
                stats.rejected.append(req.rid)
                stats.errors[req.rid] = str(err)
                used -= fp
                return
            active.append([req, s, fp, clock() - t0, 32 if self.precision != "fp64" else 64])
            dirty = True

        def finish(item):
            """The device half of a prepared request; its solver (or the
            error) goes to `ready`."""
            req, prep, fp, err = item
            if err is None:
                try:
                    s = self._finish(prep)
                    self.setup_stream.synchronize()
                    ready.put((req, s, fp, None))
                except Exception as e:          # reported by the serving loop
                    ready.put((req, None, fp, e))
                finally:
                    prep.close()
            else:
                ready.put((req, None, fp, err))

        def setup_inline():
            """The setup work of the serving thread (solvers, or the errors
            their setup raised, go to `ready`): whole setups of the requests
            admitted inline, or the device halves of those prepared so far."""
            for req, fp in to_setup:
                try:
                    s = self._admit(req)
                    self.setup_stream.synchronize()
                    ready.put((req, s, fp, None))
                except Exception as e:          # reported by the serving loop
                    ready.put((req, None, fp, e))
            to_setup.clear()
            while mode == "prepare":
                try:
                    item = done.get_nowait()
                except queue.Empty:
                    break
                finish(item)

        try:
            while pending or waiting or active or in_setup:
                now = clock() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                # admission in arrival order (budget and free slots); the setup
                # starts on the worker thread, or inline while this round sweeps
                while waiting and len(active) + in_setup < self.max_chains:
                    req = waiting[0]
                    fp = fps.get(req.rid)
                    if fp is None:
                        fp = fps[req.rid] = self.footprint(req)
                    if fp == 0 or fp > self.budget:
                        # an unsupported shape, or larger than the whole budget
                        waiting.popleft()
                        stats.rejected.append(req.rid)
                        stats.errors[req.rid] = ("unsupported generator shape" if fp == 0
                                                 else f"footprint {fp} B above the budget")
                        continue
                    if used + fp > self.budget:
                        break
                    waiting.popleft()
                    used += fp
                    in_setup += 1
                    if worker is not None:
                        todo.put((req, fp))
                    else:
                        to_setup.append((req, fp))
                # chains whose setup finished join this round
                while True:
                    try:
                        item = ready.get_nowait()
                    except queue.Empty:
                        break
                    join(item)
                stats.peak_chains = max(stats.peak_chains, len(active))
                stats.peak_bytes = max(stats.peak_bytes, used)
                if not active:
                    if to_setup:
                        # nothing to sweep: set the admitted requests up now
                        setup_inline()
                    elif in_setup and mode == "prepare":
                        # nothing to sweep: wait for a host half, finish it
                        finish(done.get())
                    elif in_setup:
                        # nothing to sweep: wait for the setup thread
                        join(ready.get())
                    elif pending:
                        delay = pending[0].arrival - (clock() - t0)
                        if delay > 0:
                            time.sleep(min(delay, 0.05))
                    continue
                if dirty:
                    self.batch.set([a[1] for a in active], self.tol, self.nontemporal)
                    dirty = False
                self.batch.sweeps(self.K, self.use_graph)     # asynchronous
                # the requests admitted this round are set up while the batch
                # sweeps (same host thread; the GPU runs both); they join the
                # next round
                setup_inline()
                # one device-to-host copy for every chain's stopping state
                sweeps, stopped, diffs, status = self.batch.query()
                stats.rounds += 1
                keep = []
                for k, entry in enumerate(active):
                    req, s, fp, t_adm, stage = entry[:5]
                    if status[k] != stc.STC_OK:
                        # a sweep produced no positive mass: drop the request
                        stats.rejected.append(req.rid)
                        stats.errors[req.rid] = "e^T z <= 0 after a sweep"
                        s.close()
                        used -= fp
                        dirty = True
                        continue
                    capped = not stopped[k] and int(sweeps[k]) >= self.max_sweeps
                    if not stopped[k] and not capped:
                        if (stage == 32 and self.precision == "mixed"
                                and floor32.reached(req.rid, float(diffs[k]))):
                            # the FP32 stage's rounding floor lies above
                            # switch_tol: continue in FP64
                            s.promote()
                            entry[4] = 64
                            entry.append(int(sweeps[k]))
                            dirty = True
                        keep.append(entry)
                        continue
                    if stage == 32 and self.precision == "mixed" and not capped:
                        s.promote()
                        entry[4] = 64
                        entry.append(int(sweeps[k]))          # sweeps in FP32
                        keep.append(entry)
                        dirty = True
                        continue
                    pi = s.store()
                    it = int(sweeps[k])
                    it32 = (entry[5] if len(entry) > 5
                            else (it if self.precision == "fp32" or stage == 32 else 0))
                    stats.results.append(Result(req.rid, req.arrival, t_adm, clock() - t0, pi, it,
                                                it32, fp,
                                                stc.STC_EMAXIT if capped else stc.STC_OK))
                    s.close()
                    used -= fp
                    dirty = True
                active = keep
        finally:
            if worker is not None:
                todo.put(None)
                worker.join()
            # on an early exit, release every chain still held
            to_setup.clear()
            for entry in active:
                entry[1].close()
            while True:
                try:
                    _req, s, _fp, _err = ready.get_nowait()
                except queue.Empty:
                    break
                if s is not None:
                    s.close()
            while True:
                try:
                    _req, prep, _fp, _err = done.get_nowait()
                except queue.Empty:
                    break
                if prep is not None:
                    prep.close()
        stats.wall = clock() - t0
        return stats

    def close(self):
        self.batch.close()
