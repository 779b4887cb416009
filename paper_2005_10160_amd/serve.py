"""Serving loop for the fast gravity operator: continuous batching over HIP
streams with a geometry-keyed cache of resident kernel spectra.

Requests carry a geometry (nx, ny, nz, dx, dy, dz, h, components, and
optionally the layer edges of a layered mesh or a number of observation
levels), an operation (forward d = G rho or adjoint g = G^T r) and 1..B
models.  The
kernel spectra of a geometry are built once (the geometry/density split of
section 2.2: the kernel does not change between calls) and stay resident
while memory allows.

``Scheduler`` is the policy, free of any device code so that it can run on a
virtual clock in tests:
  * pending requests are grouped by (geometry, operation); a launch takes
    the group of the oldest pending request, in arrival order, up to
    ``max_models`` models;
  * a group is admitted when a stream slot is free and its bytes (workspace,
    inputs and outputs) fit in the memory budget; idle cached spectra are
    evicted, least recently used first, to make room;
  * a group whose spectra are not resident first reserves their bytes and
    has them built in the background (``prepare``); it takes no slot and
    holds nobody up while they are built, and is admitted like any other
    once they are ready;
  * younger groups may pass an older one that does not fit yet, until the
    older one has waited ``backfill_limit`` seconds: then admission stops
    until memory drains for it;
  * a request that can never fit is rejected at once; one that cannot be
    admitted within ``admit_timeout`` is rejected; pending requests can be
    cancelled.
Requests that arrive while others run are admitted as soon as a slot and
memory free up, and run concurrently on separate streams.

``GpuExecutor`` launches groups through the HIP library, ``Server`` runs the
scheduler in real time, and ``bench_served`` replays a seeded Poisson trace.
"""

import collections
import math
import itertools
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Optional, Tuple

import numpy as np

@dataclass(frozen=True)
class GeometryKey:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    h: float
    components: int
    zedges: Optional[Tuple[float, ...]] = None   # layered mesh: nz + 1 layer-edge depths (dz unused)
    levels: int = 1                               # observation planes dz apart (equal-dimension survey)

    @property
    def n_out(self):
        return bin(self.components & 0x1FF).count("1")

    @property
    def data_shape(self):
        """One model's data: [levels][C][ny][nx] (levels dropped for one plane)."""
        return ((self.levels,) if self.levels > 1 else ()) + (self.n_out, self.ny, self.nx)

    @property
    def n_spec(self):
        spec = self.components & 0x1BF        # every component but gzz has a spectrum
        if self.components & 0x40:
            spec |= 0x12                       # gzz = -(gxx + gyy)
        return bin(spec).count("1")


@dataclass
class Request:
    rid: int
    key: GeometryKey
    op: str                       # "forward" | "adjoint"
    batch: int
    t_arrival: Optional[float] = None   # scheduler clock; stamped on submit when None
    data: Any = None              # [B][nz][ny][nx] (forward) or [B][C][ny][nx] (adjoint)
    result: Any = None
    status: str = "pending"       # pending | running | done | rejected | cancelled
    error: Optional[str] = None
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    cache: Optional[str] = None   # "hit": spectra resident on arrival; "miss": they had to be built
    keep_result: bool = True      # False: the output buffer is recycled once done (load replay)
    device_ms: Optional[float] = None   # its group's time on the device: input copies, operator, output copies
    compute_ms: Optional[float] = None  # its group's operator time on the device
    event: threading.Event = field(default_factory=threading.Event, repr=False)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival

    def wait(self, timeout=None):
        self.event.wait(timeout)
        return self


def _circulant(n):
    p = 16
    while p < 2 * n - 1:
        p *= 2
    return p


def spectra_bytes(key: GeometryKey, elem: int) -> int:
    """Resident spectra of a plan: one real per frequency of the quarter plane
    for each stored component and layer."""
    layers = key.nz + key.levels - 1
    return key.n_spec * layers * (_circulant(key.nx) // 2 + 1) * (_circulant(key.ny) // 2 + 1) * elem


def io_bytes(key: GeometryKey, op: str, batch: int, elem: int) -> int:
    plane = key.nx * key.ny
    model = key.nz * plane
    data = key.levels * key.n_out * plane
    return batch * (model + data) * elem


class Scheduler:
    """Admission and batching policy.  ``executor`` must provide
    ``elem`` (bytes per value), ``workspace_bytes(key, op, batch)``,
    ``prepare(key)`` (start building the key's spectra without waiting),
    ``ready(key) -> bool`` (True once built; raises if the build failed),
    ``evict(key)``, ``launch(slot, requests)`` and ``poll(slot) -> bool``
    (True when the slot's launch has completed)."""

    def __init__(self, executor, budget_bytes, n_slots=4, max_models=32, admit_timeout=30.0,
                 backfill_limit=0.25, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.n_slots = int(n_slots)
        self.max_models = int(max_models)
        self.admit_timeout = admit_timeout
        self.backfill_limit = backfill_limit
        self.clock = clock
        self.pending = collections.OrderedDict()      # (key, op) -> deque of requests
        self.slots = [None] * self.n_slots            # slot -> (requests, bytes, key)
        self.in_use = 0                               # bytes of running groups
        self.resident = collections.OrderedDict()     # key -> bytes (LRU order), built or being built
        self.building = set()                         # keys whose spectra are being built
        self.busy_keys = collections.Counter()        # key -> running groups using it
        self.completed = []
        self.stats = collections.Counter()
        self._seq = itertools.count()

    # -- bookkeeping ---------------------------------------------------------
    def resident_bytes(self):
        return sum(self.resident.values())

    def free_bytes(self):
        return self.budget - self.in_use - self.resident_bytes()

    def group_bytes(self, key, op, batch):
        return self.ex.workspace_bytes(key, op, batch) + io_bytes(key, op, batch, self.ex.elem)

    def submit(self, req: Request):
        if req.t_arrival is None:
            req.t_arrival = self.clock()
        need = self.group_bytes(req.key, req.op, req.batch) + spectra_bytes(req.key, self.ex.elem)
        if req.batch < 1 or req.batch > self.max_models or need > self.budget:
            self._finish(req, "rejected", "request needs %d bytes / %d models; budget %d bytes / %d models"
                         % (need, req.batch, self.budget, self.max_models))
            return False
        req.cache = "hit" if req.key in self.resident and req.key not in self.building else "miss"
        self.pending.setdefault((req.key, req.op), collections.deque()).append(req)
        self.stats["submitted"] += 1
        return True

    def cancel(self, req: Request):
        q = self.pending.get((req.key, req.op))
        if q is not None and req in q and req.status == "pending":
            q.remove(req)
            if not q:
                del self.pending[(req.key, req.op)]
            self._finish(req, "cancelled", "cancelled by client")
            return True
        return False

    def _finish(self, req, status, error=None):
        req.status = status
        req.error = error
        req.t_done = self.clock()
        self.stats[status] += 1
        self.completed.append(req)
        req.event.set()

    # -- one scheduling step -------------------------------------------------
    def step(self):
        """Retire finished launches, expire waiters, admit what fits.
        Returns the number of launches started."""
        now = self.clock()
        for s, entry in enumerate(self.slots):
            if entry is not None and self.ex.poll(s):
                reqs, nbytes, key = entry
                self.slots[s] = None
                self.in_use -= nbytes
                self.busy_keys[key] -= 1
                for r in reqs:
                    if r.status == "running":
                        self._finish(r, "done")
        for k in list(self.pending):
            q = self.pending[k]
            while q and self.admit_timeout is not None and now - q[0].t_arrival > self.admit_timeout:
                self._finish(q.popleft(), "rejected", "not admitted within %.3g s" % self.admit_timeout)
            if not q:
                del self.pending[k]
        for key in list(self.building):
            try:
                done = self.ex.ready(key)
            except Exception as e:  # a failed build fails the key's requests, not the loop
                self.building.discard(key)
                self.resident.pop(key, None)
                for k in [k for k in self.pending if k[0] == key]:
                    for r in self.pending.pop(k):
                        self._finish(r, "rejected", "spectra build failed: %s" % e)
                continue
            if done:
                self.building.discard(key)
        launched = 0
        while self.pending and None in self.slots:
            # groups waiting for their spectra to be built are not in line
            heads = sorted(((k, q) for k, q in self.pending.items() if k[0] not in self.building),
                           key=lambda kv: kv[1][0].t_arrival)
            if not heads:
                break
            oldest_wait = now - heads[0][1][0].t_arrival
            chosen = None
            for i, ((key, op), q) in enumerate(heads):
                if i > 0 and oldest_wait > self.backfill_limit:
                    break
                if key not in self.resident:
                    # reserve the spectra and have them built off this loop;
                    # the group is admitted once they are ready
                    need = spectra_bytes(key, self.ex.elem)
                    if not self._make_room(need, key):
                        continue
                    self.resident[key] = need
                    self.building.add(key)
                    self.stats["spectra_miss"] += 1
                    for k2, q2 in self.pending.items():
                        if k2[0] == key:
                            for r in q2:
                                r.cache = "miss"
                    self.ex.prepare(key)
                    try:
                        if not self.ex.ready(key):
                            continue
                    except Exception:
                        continue                # reported at the next step
                    self.building.discard(key)
                group, models = [], 0
                for r in q:
                    if models + r.batch > self.max_models:
                        break
                    group.append(r)
                    models += r.batch
                nbytes = self.group_bytes(key, op, models)
                if self._make_room(nbytes, key):
                    chosen = (key, op, group, nbytes)
                    break
            if chosen is None:
                break
            key, op, group, nbytes = chosen
            q = self.pending[(key, op)]
            for r in group:
                q.popleft()
                r.status = "running"
                r.t_admit = now
            if not q:
                del self.pending[(key, op)]
            self.stats["spectra_hit" if all(r.cache == "hit" for r in group) else "launch_after_build"] += 1
            self.resident.move_to_end(key)
            slot = self.slots.index(None)
            self.slots[slot] = (group, nbytes, key)
            self.in_use += nbytes
            self.busy_keys[key] += 1
            self.stats["launches"] += 1
            self.stats["batched_requests"] += len(group)
            try:
                self.ex.launch(slot, group)
            except Exception as e:  # a failed launch fails its requests, not the loop
                self.slots[slot] = None
                self.in_use -= nbytes
                self.busy_keys[key] -= 1
                for r in group:
                    self._finish(r, "rejected", "launch failed: %s" % e)
                # the key's spectra are not trusted after a failure: they are
                # dropped and built again for the next request
                if self.busy_keys[key] == 0 and key in self.resident:
                    del self.resident[key]
                    self.ex.evict(key)
                continue
            launched += 1
        return launched

    def _make_room(self, need, key):
        if need <= self.free_bytes():
            return True
        for k in list(self.resident):
            if need <= self.free_bytes():
                break
            if k == key or self.busy_keys[k] > 0 or k in self.building:
                continue
            del self.resident[k]
            self.ex.evict(k)
            self.stats["evictions"] += 1
        return need <= self.free_bytes()

    def idle(self):
        return not self.pending and all(s is None for s in self.slots)


# ---------------------------------------------------------------------------
# GPU executor and real-time server
# ---------------------------------------------------------------------------
class GpuExecutor:
    """Launches a group on one of ``n_slots`` HIP streams: host inputs are
    copied into one batched device tensor, the operator runs once for the
    whole group, and each request's slice is copied back to its host
    buffer.  Plans (resident spectra) are built on a worker thread, one at
    a time, on a stream of their own (``prepare``/``ready``), so that the
    scheduler keeps retiring and launching other groups meanwhile."""

    def __init__(self, precision="f32", n_slots=4, device="cuda:0"):
        import torch
        from . import operator as op_mod
        self.torch = torch
        self.op_mod = op_mod
        self.device = torch.device(device)
        self.precision = precision
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        self.elem = 4 if precision == "f32" else 8
        # all streams at the default priority
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_slots)]
        self.plan_stream = torch.cuda.Stream(device=self.device)
        self.plans = {}
        self.build_errors = {}
        self.build_queue = collections.deque()
        self.build_cv = threading.Condition()
        self.building = None
        self.builder_running = True
        self.builder = threading.Thread(target=self._build_loop, daemon=True)
        self.builder.start()
        self.events = [None] * n_slots
        self.keep = [None] * n_slots
        self.lock = threading.Lock()
        # pinned output buffers of requests that do not keep their result,
        # by shape, for reuse
        self.out_pool = collections.defaultdict(list)

    def _build_loop(self):
        self.torch.cuda.set_device(self.device)
        while True:
            with self.build_cv:
                while not self.build_queue and self.builder_running:
                    self.build_cv.wait()
                if not self.build_queue:
                    return
                key = self.build_queue.popleft()
                if isinstance(key, GeometryKey):
                    self.building = key
            if not isinstance(key, GeometryKey):
                key[1].close()              # ("close", plan) from evict
                continue
            try:
                p = self._make_plan(key)
                err = None
            except Exception as e:
                p, err = None, e
            with self.build_cv:
                if err is None:
                    self.plans[key] = p
                else:
                    self.build_errors[key] = err
                self.building = None
                self.build_cv.notify_all()

    def prepare(self, key):
        """Start building the key's plan on the worker thread (no wait)."""
        with self.build_cv:
            if key in self.plans or key == self.building or key in self._queued_keys():
                return
            self.build_errors.pop(key, None)
            self.build_queue.append(key)
            self.build_cv.notify_all()

    def _queued_keys(self):
        return [k for k in self.build_queue if isinstance(k, GeometryKey)]

    def ready(self, key):
        """True once the key's plan is built; raises the build's error."""
        with self.build_cv:
            if key in self.build_errors:
                raise self.build_errors[key]
            return key in self.plans

    def _make_plan(self, key):
        if key.levels > 1:
            return self.op_mod.plan_levels(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, key.levels,
                                           key.components, self.precision, device=self.device,
                                           stream=self.plan_stream)
        if key.zedges is None:
            return self.op_mod.plan(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, key.components,
                                    self.precision, device=self.device, stream=self.plan_stream)
        return self.op_mod.plan_layered(key.nx, key.ny, key.dx, key.dy, key.zedges, key.h, key.components,
                                        self.precision, device=self.device, stream=self.plan_stream)

    def plan_for(self, key):
        """The key's plan, waiting for (or making) it if it is not built."""
        with self.build_cv:
            p = self.plans.get(key)
            if p is not None:
                return p
            queued = key == self.building or key in self._queued_keys()
        if queued:
            with self.build_cv:
                while key not in self.plans and key not in self.build_errors:
                    self.build_cv.wait()
            self.ready(key)              # raises the build's error
            return self.plans[key]
        p = self._make_plan(key)
        with self.build_cv:
            self.plans[key] = p
        return p

    def workspace_bytes(self, key, op, batch):
        # the plan's own figure when it exists; otherwise an upper bound of the
        # same layout (complex intermediates of the model and data sizes)
        with self.build_cv:
            p = self.plans.get(key)
        if p is not None:
            return p.workspace_bytes(op, batch)
        # forward: row-transformed model, up to 32 layer splits of partial
        # data and up to 32 Nyquist chunks; adjoint: the residual's spectra
        # and one model-sized slab per group of six spectra
        # with several levels a column pass may carry up to six output slots
        # and the adjoint keeps up to four passes' slabs
        ux = _circulant(key.nx) // 2 + 1
        nspec = key.n_spec
        groups = (nspec + 5) // 6
        slots = max(nspec, 6) if key.levels > 1 else nspec
        chunk = min(key.levels, 4)
        splits = 32
        per = 2 * self.elem * ux * (key.ny + 1)
        fwd = per * batch * (key.nz + splits * slots) + self.elem * splits * batch * slots * (key.ny + 1)
        adj = per * batch * chunk * (slots + groups * key.nz)
        # levels as a Toeplitz product in depth: column slabs and two-row
        # spectrum slabs for the layers and for every level's components
        toep = 0
        if key.levels > 1:
            py = _circulant(key.ny)
            toep = batch * (key.nz + key.levels * nspec) * 2 * self.elem * ux * ((key.ny + 1) + (py + 8))
        return max(fwd, adj, toep)

    def is_resident(self, key):
        with self.build_cv:
            return key in self.plans

    def evict(self, key):
        with self.build_cv:
            p = self.plans.pop(key, None)
            self.build_errors.pop(key, None)
        if p is not None:
            # the scheduler evicts only keys with no running group, so the
            # plan's launches are done; it is freed on the worker thread
            # (freeing device memory waits for the device)
            with self.build_cv:
                self.build_queue.append(("close", p))
                self.build_cv.notify_all()

    def launch(self, slot, reqs):
        torch = self.torch
        key, op = reqs[0].key, reqs[0].op
        p = self.plan_for(key)
        st = self.streams[slot]
        B = sum(r.batch for r in reqs)
        if op == "forward":
            shape_in = (B, key.nz, key.ny, key.nx)
            shape_out = (B,) + key.data_shape
        else:
            shape_in = (B,) + key.data_shape
            shape_out = (B, key.nz, key.ny, key.nx)
        # device-side timing of the group: its input copies, the operator,
        # its output copies
        tev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        with torch.cuda.stream(st):
            x = torch.empty(shape_in, dtype=self.dtype, device=self.device)
            y = torch.empty(shape_out, dtype=self.dtype, device=self.device)
            ws = torch.empty(p.workspace_bytes(op, B), dtype=torch.uint8, device=self.device)
            tev[0].record(st)
            o = 0
            for r in reqs:
                x[o:o + r.batch].copy_(r.data, non_blocking=True)
                o += r.batch
            tev[1].record(st)
            if op == "forward":
                p.forward(x, y, ws, stream=st)
            else:
                p.adjoint(x, y, ws, stream=st)
            tev[2].record(st)
            o = 0
            for r in reqs:
                if r.result is None:
                    shp = (r.batch,) + shape_out[1:]
                    free = self.out_pool.get(shp)
                    r.result = free.pop() if free else torch.empty(shp, dtype=self.dtype, pin_memory=True)
                r.result.copy_(y[o:o + r.batch], non_blocking=True)
                o += r.batch
            tev[3].record(st)
        self.events[slot] = tev[3]
        self.keep[slot] = (x, y, ws, reqs, tev)

    def poll(self, slot):
        ev = self.events[slot]
        if ev is None or ev.query():
            kept = self.keep[slot]
            if kept is not None:
                tev = kept[4]
                dev_ms, comp_ms = tev[0].elapsed_time(tev[3]), tev[1].elapsed_time(tev[2])
                for r in kept[3]:
                    r.device_ms, r.compute_ms = dev_ms, comp_ms
                    if not r.keep_result and r.result is not None:
                        self.out_pool[tuple(r.result.shape)].append(r.result)
                        r.result = None
            self.events[slot] = None
            self.keep[slot] = None
            return True
        return False

    def close(self):
        with self.build_cv:
            self.builder_running = False
            self.build_queue = collections.deque(k for k in self.build_queue if not isinstance(k, GeometryKey))
            self.build_cv.notify_all()
        self.builder.join()
        self.torch.cuda.synchronize(self.device)
        for p in self.plans.values():
            p.close()
        self.plans.clear()


class Server:
    """Real-time loop around a Scheduler: ``submit`` from any thread, a
    background thread steps the scheduler."""

    def __init__(self, executor, budget_bytes, n_slots=4, max_models=32, admit_timeout=30.0,
                 backfill_limit=0.25):
        self.sched = Scheduler(executor, budget_bytes, n_slots, max_models, admit_timeout, backfill_limit)
        self.inbox = collections.deque()
        self.cv = threading.Condition()
        self.running = True
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def submit(self, req: Request):
        with self.cv:
            self.inbox.append(req)
            self.cv.notify()
        return req

    def cancel(self, req):
        with self.cv:
            self.inbox.append(("cancel", req))
            self.cv.notify()

    def _loop(self):
        while True:
            with self.cv:
                while self.inbox:
                    item = self.inbox.popleft()
                    if isinstance(item, tuple):
                        self.sched.cancel(item[1])
                    else:
                        self.sched.submit(item)
                if not self.running and self.sched.idle():
                    return
            self.sched.step()
            if self.sched.idle():
                with self.cv:
                    if not self.inbox and self.running:
                        self.cv.wait(0.01)
            else:
                time.sleep(2e-5)

    def close(self):
        with self.cv:
            self.running = False
            self.cv.notify()
        self.thread.join()


def _percentiles(vals):
    if not vals:
        return None, None
    a = np.asarray(vals)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def latency_summary(records):
    """p50 / p99 latency (ms) of completed requests, overall and split by
    whether their spectra were resident on arrival (hit) or had to be built
    (miss); overall also the device-only figures where the records carry
    them: the request's time on the device (its group's input copies,
    operator and output copies) and its group's operator time."""
    out = {}
    for name, sel in (("all", lambda r: True), ("hit", lambda r: r["cache"] == "hit"),
                      ("miss", lambda r: r["cache"] == "miss")):
        lat = [r["latency_ms"] for r in records if r["status"] == "done" and sel(r)]
        p50, p99 = _percentiles(lat)
        out[name] = {"n": len(lat), "p50_ms": p50, "p99_ms": p99}
    for key in ("device_ms", "compute_ms"):
        vals = [r[key] for r in records if r["status"] == "done" and r.get(key) is not None]
        if vals:
            p50, p99 = _percentiles(vals)
            out["all"][key.replace("_ms", "_p50_ms")] = p50
            out["all"][key.replace("_ms", "_p99_ms")] = p99
    return out


def request_shape(tr):
    """Host input of a trace request: [B][nz][n][n] densities for a forward,
    [B][C][n][n] residuals for an adjoint."""
    C = 6 if tr.full_tensor else 1
    return (tr.batch, tr.nz, tr.n, tr.n) if tr.op == "forward" else (tr.batch, C, tr.n, tr.n)


class InputBank:
    """Seeded host inputs for a request trace within a bounded buffer.

    One flat buffer of uniform(-500, 500) values (seed 500) is drawn once,
    its length the trace's largest request plus ``slack`` values; request r
    takes the window starting at an offset drawn from a generator seeded by
    the request's own seed, so every request carries its own models (the
    same ones on every replay) while the pinned host memory stays bounded by
    that one buffer."""

    def __init__(self, trace, precision, pin=True, slack=1 << 24, seed=500):
        import torch
        dt = torch.float32 if precision == "f32" else torch.float64
        self.largest = max(math.prod(request_shape(tr)) for tr in trace)
        self.n = self.largest + int(slack)
        self.buf = torch.empty(self.n, dtype=dt, pin_memory=pin)
        gen = torch.Generator().manual_seed(seed)
        chunk = 1 << 24
        for o in range(0, self.n, chunk):
            m = min(chunk, self.n - o)
            self.buf[o:o + m].copy_(torch.rand(m, generator=gen, dtype=torch.float64).sub_(0.5).mul_(1000.0))

    @property
    def nbytes(self):
        return self.buf.numel() * self.buf.element_size()

    def offset(self, tr):
        size = math.prod(request_shape(tr))
        rng = np.random.default_rng(tr.seed)
        return int(rng.integers(0, self.n - size + 1))

    def get(self, tr):
        shape = request_shape(tr)
        o = self.offset(tr)
        return self.buf[o:o + math.prod(shape)].view(shape)


def make_inputs(trace, precision, pin=True):
    """The inputs of every request of a trace, as views of one InputBank."""
    bank = InputBank(trace, precision, pin=pin)
    return [bank.get(tr) for tr in trace]


def replay(trace, inputs, executor_factory, budget_bytes, batched=True, n_slots=4, max_models=32,
           time_limit=None):
    """Replay arrivals in real time.  batched=False gives the plain baseline:
    one stream, FIFO, one model per call.  Returns the summary and one record
    per request: arrival, admission and completion times (seconds from the
    start of the replay, admission of its first model for the baseline), its
    latency, and whether its spectra were resident on arrival."""
    ex = executor_factory(n_slots if batched else 1)
    if batched:
        srv = Server(ex, budget_bytes, n_slots=n_slots, max_models=max_models, admit_timeout=None)
    else:
        srv = Server(ex, budget_bytes, n_slots=1, max_models=1, admit_timeout=None, backfill_limit=0.0)
    reqs = []
    t0 = time.perf_counter()
    for tr, x in zip(trace, inputs):
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        key = GeometryKey(tr.n, tr.n, tr.nz, 20.0, 20.0, 20.0, 10.0, 0x3F if tr.full_tensor else 0x1)
        delay = t0 + tr.t_arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        if batched:
            r = Request(tr.rid, key, tr.op, tr.batch, time.perf_counter(), x, keep_result=False)
            srv.submit(r)
            reqs.append((tr, [r]))
        else:
            # the plain operator: one model per call, in arrival order
            t_arr = time.perf_counter()
            parts = []
            for b in range(tr.batch):
                r = Request(tr.rid * 100 + b, key, tr.op, 1, t_arr, x[b:b + 1], keep_result=False)
                srv.submit(r)
                parts.append(r)
            reqs.append((tr, parts))
    for _, parts in reqs:
        for r in parts:
            r.wait()
    wall = time.perf_counter() - t0
    srv.close()
    stats = dict(srv.sched.stats)
    ex.close()
    records = []
    evals = 0.0
    for tr, parts in reqs:
        done = all(r.status == "done" for r in parts)
        t_done = max(r.t_done for r in parts) if done else None
        admits = [r.t_admit for r in parts if r.t_admit is not None]
        records.append({
            "rid": tr.rid, "n": tr.n, "nz": tr.nz, "batch": tr.batch, "op": tr.op,
            "components": 6 if tr.full_tensor else 1,
            "status": "done" if done else parts[0].status,
            "cache": "hit" if all(r.cache == "hit" for r in parts) else "miss",
            "t_arrival": parts[0].t_arrival - t0,
            "t_admit": (min(admits) - t0) if admits else None,
            "t_done": (t_done - t0) if done else None,
            "latency_ms": (t_done - parts[0].t_arrival) * 1e3 if done else None,
            # the plain baseline runs a request's models one call after another
            "device_ms": sum(r.device_ms for r in parts) if done and all(r.device_ms is not None for r in parts)
            else None,
            "compute_ms": sum(r.compute_ms for r in parts) if done and all(r.compute_ms is not None for r in parts)
            else None,
        })
        if done:
            k = parts[0].key
            evals += tr.batch * k.n_out * (k.nx * k.ny) ** 2 * k.nz
    lat = latency_summary(records)
    completed = lat["all"]["n"]
    return {"requests": len(reqs), "completed": completed, "wall_s": wall,
            "p50_ms": lat["all"]["p50_ms"], "p99_ms": lat["all"]["p99_ms"],
            "device_p50_ms": lat["all"].get("device_p50_ms"), "device_p99_ms": lat["all"].get("device_p99_ms"),
            "compute_p50_ms": lat["all"].get("compute_p50_ms"), "compute_p99_ms": lat["all"].get("compute_p99_ms"),
            "hit": lat["hit"], "miss": lat["miss"],
            "requests_per_s": completed / wall, "effective_evals_per_s": evals / wall, "stats": stats,
            "records": records}


def bench_served(seconds=20.0, rate=200.0, budget_gb=64.0, baseline_seconds=3.0, records_path=None):
    """Seeded Poisson trace (rate req/s, `seconds` long: 4000 requests by
    default) of mixed grids, replayed through the FP32 continuous-batching
    server; the plain FP64 operator (FIFO, one model per call) replays the
    first `baseline_seconds` of the same trace (it falls behind the arrival
    rate, so a longer replay only grows its queue), and the served figures
    over that same prefix are reported beside it.  Both keep the spectra
    cache.  The per-request records go to `records_path` (CSV) when given;
    the summary names the ten slowest served requests."""
    from synth import poisson_trace
    n = max(1, int(seconds * rate))
    trace = poisson_trace(n_requests=n, rate=rate, seed=500)
    budget = int(budget_gb * (1 << 30))
    out = {"trace": "poisson %.0f req/s, %d requests (%.1f s), seed 500" % (rate, n, trace[-1].t_arrival)}
    bank = InputBank(trace, "f32")
    out["input_bank_bytes"] = bank.nbytes
    served = replay(trace, [bank.get(tr) for tr in trace], lambda k: GpuExecutor("f32", k), budget, batched=True)
    del bank
    recs = served.pop("records")
    nb = max(1, int(baseline_seconds * rate))
    served["first_%d" % nb] = latency_summary(recs[:nb])
    served["slowest"] = sorted((r for r in recs if r["latency_ms"] is not None),
                               key=lambda r: -r["latency_ms"])[:10]
    out["served_f32"] = served
    if records_path:
        import csv
        with open(records_path, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=list(recs[0].keys()))
            w.writeheader()
            w.writerows(recs)
    # the served run's pinned buffer goes back to the system before the
    # baseline's (torch keeps freed pinned blocks cached otherwise)
    import gc
    import torch
    gc.collect()
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()
    sub = trace[:nb]
    bank = InputBank(sub, "f64")
    plain = replay(sub, [bank.get(tr) for tr in sub], lambda k: GpuExecutor("f64", k), budget, batched=False)
    del bank
    plain.pop("records")
    out["plain_f64"] = plain
    return out
