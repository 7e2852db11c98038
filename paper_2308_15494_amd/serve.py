"""Serving: refinement requests admitted by HBM footprint and refined with
continuous batching.

Every request is one graph with its k, eps and number of rounds; it starts
from a seeded random balanced partition and runs its own tau schedule. The
server keeps the admitted requests' state (partition, gain table, block
weights) on the device. Requests with the same (k, eps) share a batch (the
disjoint union of their graphs, refined by the same launches); at every step
each batch runs one round of all its requests, finished requests leave, and
requests that have arrived are admitted as long as their footprint fits the
budget; a running batch takes newcomers at most every `admit_every` steps,
since each change of membership rebuilds it. When a batch's membership
changes, a new union is built and the surviving requests' partitions, gain
tables and block weights are carried into it on the device
(upr_batch_carry), so their state stays resident; only when newcomers join
does the next step rebuild the tables (a table is a function of the
partition, so the result is the same either way).

Because no kernel lets two graphs of a batch interact, each request's result
is exactly what it gets when refined alone. With `concurrent`, every group
has a context and stream of its own and the groups' rounds of a step run
from host threads of their own at the same time (their launches and the host
waits of their rebalancing overlap); each group still goes through its own
rebuilds and rounds in the same order, so the results are the same. With
`uploads_ahead`, a thread uploads and validates every arrived request's graph
while the steps run, so that admission no longer waits for the copies.

The refinement arithmetic runs in libupr (upr_batch_*); this module only
schedules, moves partitions between batches and measures latency.
"""
from __future__ import annotations

import dataclasses
import queue
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import graphgen as gg
from . import upr


@dataclasses.dataclass
class Request:
    rid: int
    graph: gg.Graph
    k: int
    eps: tuple = (3, 100)
    rounds: int = 10
    arrival: float = 0.0      # seconds after the start of the stream
    part_seed: int = 0

    def footprint(self) -> int:
        """HBM bytes held while admitted: the graph (as uploaded and in the
        batch union), the n x k gain table, block weights and per-node
        workspace of the round."""
        g = self.graph
        csr = 8 * (g.n + 1) + 4 * g.nnz * (2 if g.adjwgt is not None else 1)
        csr += 4 * g.n if g.vwgt is not None else 0
        return 2 * csr + 4 * g.n * self.k + 8 * self.k + 96 * g.n


@dataclasses.dataclass
class Result:
    rid: int
    part: np.ndarray          # final partition (local block ids)
    stats: list               # per-round statistics dicts
    arrival: float
    admitted: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Job:
    def __init__(self, req: Request, dg, admitted: float):
        self.req = req
        self.dg = dg
        self.round = 0
        self.part = gg.random_partition(req.graph.n, req.k, req.part_seed)  # local ids, host
        self.stats = []
        self.admitted = admitted


class _Group:
    """The batch of the admitted requests with one (k, eps)."""

    def __init__(self, ctx, k, eps, stream=None):
        self.ctx, self.k, self.eps, self.stream = ctx, k, eps, stream
        self.jobs: list[_Job] = []
        self.members: list[_Job] = []
        self.batch = None
        self.dirty = True
        self.fresh = True
        self.waiting: list[_Job] = []   # admitted, joining at the next rebuild
        self.since_rebuild = 0

    def rebuild(self):
        """New union of the current jobs. Jobs that were in the old union
        keep their partition, table rows and block weights, carried on the
        device; returns True if newcomers joined (their tables must be
        built, so the next step rebuilds every table)."""
        old, old_members = self.batch, self.members
        self.batch = None
        self.members = list(self.jobs)
        where = {id(j): i for i, j in enumerate(old_members)} if old is not None else {}
        src = [where.get(id(j), -1) for j in self.members]
        if self.members:
            # admitted graphs were validated on admission
            self.batch = upr.Batch(self.ctx, [j.dg for j in self.members], self.k, self.eps,
                                   trusted=True)
            # newcomers start from their own partition (uploaded); carried
            # slices are filled on the device
            self.batch.set_partitions([j.part if s < 0 else None
                                       for j, s in zip(self.members, src)])
            if old is not None and any(s >= 0 for s in src):
                self.batch.carry_from(old, src)
        if old is not None:
            old.close()  # waits for the carry
        self.dirty = False
        return any(s < 0 for s in src)

    def launch(self):
        """Enqueue one round of every member (on the group's stream)."""
        b = self.batch
        rebuild = 1 if self.fresh else 0
        taus = [gg.tau_schedule(j.round + 1, j.req.rounds) for j in self.members]
        b.round(upr.params(self.k, self.eps, tau=(1, 1), rebuild_table=rebuild), taus=taus,
                stream=self.stream)
        self.fresh = False

    def step(self):
        """One round of every member; returns the members that finished."""
        self.launch()
        return self.finish()

    def finish(self):
        """After the round has completed (the group's stream synchronised):
        count it for every member; returns the members that finished."""
        b = self.batch
        st = b.stats.cpu().numpy().reshape(b.ng, upr.STATS_LEN)
        finished = []
        for i, j in enumerate(self.members):
            j.round += 1
            j.stats.append(upr.stats_dict(st[i]))
            if j.round >= j.req.rounds:
                finished.append((i, j))
        return finished


class Server:
    """Admission by footprint, continuous batching, latency bookkeeping."""

    def __init__(self, ctx: upr.Context, budget_bytes: int, admit_every: int = 3,
                 concurrent: bool = False, uploads_ahead: int = 0):
        """concurrent: every (k, eps) group on a context, stream and thread of
        its own. uploads_ahead > 0: a thread uploads and validates the graphs
        of arrived requests (on a stream and context of its own), at most that
        many ahead of admission, while the steps run; those graphs are held
        on the device beyond the footprint budget until admitted."""
        self.ctx = ctx
        self.budget = budget_bytes
        self.admit_every = max(int(admit_every), 1)
        self.concurrent = bool(concurrent)
        self.uploads_ahead = max(int(uploads_ahead), 0)
        self.timings = {}
        self._upload = None  # (context, stream) of the upload thread
        # concurrent: a context and stream per (k, eps), kept across runs so
        # that their workspaces are allocated once
        self._group_ctx = {}
        self._pool, self._pool_size = None, 0  # the threads that run the groups' rounds

    def _context_for(self, key):
        import torch
        if key not in self._group_ctx:
            self._group_ctx[key] = (upr.Context(self.ctx.device), torch.cuda.Stream())
        return self._group_ctx[key]

    def close(self):
        """Release the contexts of the groups and of the upload thread."""
        if self._pool is not None:
            self._pool.shutdown()
            self._pool, self._pool_size = None, 0
        for c, _ in self._group_ctx.values():
            c.close()
        self._group_ctx = {}
        if self._upload is not None:
            self._upload[0].close()
            self._upload = None

    def _uploader(self, pending, t0, clock, out, stop):
        """Upload and validate the graphs of `pending` in order, each once it
        has arrived; hand (request, graph) or (None, error) to `out`."""
        import torch
        uctx, ustream = self._upload
        dev = torch.device("cuda", self.ctx.device)

        def put(item):
            while not stop.is_set():
                try:
                    out.put(item, timeout=0.01)
                    return True
                except queue.Full:
                    pass
            return False

        try:
            for req in pending:
                while not stop.is_set():
                    wait = req.arrival - (clock() - t0)
                    if wait <= 0:
                        break
                    time.sleep(min(wait, 0.002))
                if stop.is_set():
                    return
                with torch.cuda.stream(ustream):
                    dg = upr.DeviceGraph(req.graph, dev)
                    upr.validate_graph(uctx, dg, stream=ustream)
                ustream.synchronize()
                if not put((req, dg)):
                    return
        except Exception as e:  # re-raised by the admission loop
            put((None, e))

    def _tick(self, name, t):
        self.timings[name] = self.timings.get(name, 0.0) + t

    def run(self, requests, clock=time.perf_counter, on_done=None):
        import torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        groups: dict = {}
        used = 0
        results = []
        t0 = clock()
        pi = 0
        active = 0

        def settle(grp, finished):
            # results of the requests that finished this step; the batch
            # is rebuilt without them at the next step
            nonlocal used, active
            grp.since_rebuild += 1
            if not finished:
                return
            parts = grp.batch.local_partitions([i for i, _ in finished])
            done = clock() - t0
            for (i, j), part in zip(finished, parts):
                res = Result(j.req.rid, part, j.stats, j.req.arrival, j.admitted, done)
                results.append(res)
                if on_done:
                    on_done(res)
                grp.jobs.remove(j)
                used -= j.req.footprint()
                active -= 1
            grp.dirty = True

        uploads = stop = uploader = None
        if self.uploads_ahead:
            if self._upload is None:
                self._upload = (upr.Context(self.ctx.device), torch.cuda.Stream())
            uploads = queue.Queue(maxsize=self.uploads_ahead)
            stop = threading.Event()
            uploader = threading.Thread(target=self._uploader,
                                        args=(pending, t0, clock, uploads, stop), daemon=True)
            uploader.start()
        try:
            while pi < len(pending) or active:
                now = clock() - t0
                # admission: arrived requests in arrival order while they fit
                while pi < len(pending) and pending[pi].arrival <= now:
                    req = pending[pi]
                    need = req.footprint()
                    if active and used + need > self.budget:
                        break  # wait for memory to free up (arrival order is kept)
                    key = (req.k, tuple(req.eps))
                    grp = groups.get(key)
                    if grp is not None and (len(grp.jobs) + len(grp.waiting) + 1) * req.k > upr.MAX_BATCH_BLOCKS:
                        break  # the batch has as many graphs as its block ids allow
                    t1 = clock()
                    if uploads is not None:
                        # uploaded and validated by the upload thread, in order
                        got, dg = uploads.get()
                        if got is None:
                            raise dg
                        assert got is req
                    else:
                        dg = upr.DeviceGraph(req.graph, torch.device("cuda", self.ctx.device))
                        upr.validate_graph(self.ctx, dg)
                    self._tick("admit_s", clock() - t1)
                    if grp is None:
                        if self.concurrent:
                            gctx, gstream = self._context_for(key)
                            grp = _Group(gctx, req.k, req.eps, gstream)
                        else:
                            grp = _Group(self.ctx, req.k, req.eps)
                        groups[key] = grp
                    grp.waiting.append(_Job(req, dg, clock() - t0))
                    used += need
                    active += 1
                    pi += 1
                    now = clock() - t0
                if not active:
                    # idle until the next arrival
                    wait = pending[pi].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                    continue
                self._step_groups(groups, clock, settle)
        finally:
            if uploader is not None:
                stop.set()
                uploader.join()
            for grp in groups.values():
                if grp.batch is not None:
                    grp.batch.close()
        return sorted(results, key=lambda r: r.rid)

    def _step_groups(self, groups, clock, settle):
        """Rebuild the groups whose membership changes, then one round of
        every group with members (concurrently with `concurrent`)."""
        import torch
        stepping = []
        for grp in groups.values():
            # newcomers join an idle batch at once, a running one every
            # admit_every steps or whenever it is rebuilt anyway (each
            # change of membership rebuilds the batch)
            if grp.waiting and (not grp.members or grp.dirty
                                or grp.since_rebuild >= self.admit_every):
                grp.jobs.extend(grp.waiting)
                grp.waiting = []
                grp.dirty = True
            if grp.dirty:
                t1 = clock()
                # resident state carried over unless newcomers joined
                grp.fresh = grp.rebuild()
                grp.since_rebuild = 0
                self._tick("rebuild_s", clock() - t1)
                self._tick("rebuilds", 1)
            if not grp.members:
                continue
            if self.concurrent:
                stepping.append(grp)
                continue
            t1 = clock()
            finished = grp.step()
            self._tick("step_s", clock() - t1)
            self._tick("steps", 1)
            settle(grp, finished)
        if not stepping:
            return
        # every group's round from a thread of its own, on its own context
        # and stream; the uploads, rebuilds and carries made on the current
        # stream complete first
        t1 = clock()
        torch.cuda.synchronize()
        if self._pool_size < len(stepping):
            if self._pool is not None:
                self._pool.shutdown()
            self._pool_size = max(len(stepping), 8)
            self._pool = ThreadPoolExecutor(max_workers=self._pool_size)
        futures = [self._pool.submit(grp.launch) for grp in stepping]
        errors = [f.exception() for f in futures]  # waits for every round to be enqueued
        torch.cuda.synchronize()
        for e in errors:
            if e is not None:
                raise e
        finished_by = [(grp, grp.finish()) for grp in stepping]
        self._tick("step_s", clock() - t1)
        self._tick("steps", len(stepping))
        for grp, finished in finished_by:
            settle(grp, finished)


def refine_alone(ctx, req: Request):
    """The same request refined by itself (plain per-graph calls)."""
    r = upr.Refiner(req.graph, req.k, ctx=ctx)
    r.set_partition(gg.random_partition(req.graph.n, req.k, req.part_seed))
    stats = []
    for i in range(1, req.rounds + 1):
        r.round(upr.params(req.k, req.eps, tau=gg.tau_schedule(i, req.rounds)))
        stats.append(upr.stats_dict(r.stats))
    return r.part.cpu().numpy(), stats


def poisson_arrivals(count, rate, seed):
    """Arrival times of a Poisson process with `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def percentile(xs, q):
    xs = np.sort(np.asarray(xs, dtype=np.float64))
    if xs.size == 0:
        return float("nan")
    return float(np.percentile(xs, q))
