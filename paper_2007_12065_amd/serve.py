"""Serving loop: organized point clouds arrive over time and are smoothed with
continuous batching on one GPU.

* Admission.  Every frame size class owns resident slots (device buffers for
  one frame's input and all its outputs and scratch).  `SlotPool` hands out a
  free slot of the request's class, grows the class while the total stays
  within the device-memory budget, makes the request wait when neither is
  possible, and rejects requests that could never fit.
* Execution.  One batch plan (pl_batch_*) spans all slots; each step writes a
  device activity mask selecting the slots admitted since the previous step
  and replays a HIP graph of the whole pipeline captured with that mask.  A
  step of a single frame (a lightly loaded stream) instead runs the fused
  single-frame entry (pl_smooth_frame) on that slot's buffers: three
  launches sized for one frame, and the same output bits (the batched and
  single-frame paths agree bit for bit).
* Continuous batching.  The next step is enqueued as soon as requests are
  waiting, while earlier steps may still be on the GPU: frames that arrive
  during a step join the next one instead of waiting for the queue to drain.
* Input copies.  A frame's points are copied into its slot on a copy stream
  of their own, so the copies of the next step overlap the running step;
  the step waits for its copies by event.  Frames may come from pinned host
  memory (the copy crosses PCIe) or already sit in device memory.
* Latency.  Arrival (host clock) to the completion of the frame's step,
  taken from a GPU event's timestamp on the same clock.

The plain per-frame path (`PlainServer`) serves the same stream one frame at
a time through the four single-frame calls, for comparison.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

ADMITTED, WAITING, REJECTED = "admitted", "waiting", "rejected"


@dataclass(frozen=True)
class FrameClass:
    """A frame size and its filter settings (one slot class)."""
    name: str
    M: int
    N: int
    kernel_lap: int
    lam: float
    iters_lap: int
    kernel_bil: int
    sigma_length: float
    sigma_angle: float
    iters_bil: int


def frame_sources(torch, frames: dict) -> dict:
    """Per class, the frames requests copy from: device tensors are used as
    they are, host arrays are pinned (so copies are asynchronous)."""
    out = {}
    for k, v in frames.items():
        out[k] = [f if isinstance(f, torch.Tensor) and f.is_cuda else
                  (f if isinstance(f, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(f))).pin_memory()
                  for f in v]
    return out


def slot_bytes(c: FrameClass, normal_bytes: int = 2, lap_fuse: int = 4, bil_fuse: int = 1) -> int:
    """Device bytes one resident slot of class `c` holds: input, outputs and
    the batch workspace's per-frame scratch (the same sizes the library lays
    out), rounded to 256 B per buffer."""
    def a(x):
        return (x + 255) // 256 * 256
    P = c.M * c.N
    Q = (c.M - 1) * (c.N - 1)
    T = 2 * Q
    lap_passes = 1 if c.iters_lap == 0 else -(-c.iters_lap // max(lap_fuse, 1))
    bil_passes = 1 if c.iters_bil == 0 else -(-c.iters_bil // max(bil_fuse, 1))
    total = a(12 * P)                         # input points
    total += a(12 * P)                        # smoothed points
    total += a(3 * T * normal_bytes) * 2      # filtered normals, normals of T
    total += a(12 * T)                        # centroids
    total += a(T) + a(4 * T) + a(12 * T) + a(12 * T) + a(4)   # tri_valid, T_map, T, HE, n_tri
    total += a(Q) + a(4 * (c.M - 1))          # validity codes, row counts
    total += a(12 * P) if lap_passes > 1 else 0
    total += a(3 * T * normal_bytes) * (2 if bil_passes > 1 else 1)
    return total


@dataclass
class Slot:
    cls: str
    index: int                 # position in the pool's slot list (= batch frame index)
    busy: bool = False


@dataclass
class SlotPool:
    """Resident slots per class under a byte budget (pure host logic).

    `allocate(cls_name)` is called to create a slot's device buffers when the
    pool grows; it must return nothing or raise.  Growth is only permitted
    while `growth_open` is true (the server closes it once the batch plan
    that spans the slots has been built for the measured window)."""
    budget: int
    bytes_per_slot: dict
    allocate: object = None
    growth_open: bool = True
    used: int = 0
    slots: list = field(default_factory=list)
    free: dict = field(default_factory=lambda: collections.defaultdict(list))

    def acquire(self, cls: str):
        """(status, slot): a free slot of the class, a new one if the budget
        allows, WAITING if neither, REJECTED if the class can never fit."""
        need = self.bytes_per_slot[cls]
        if need > self.budget:
            return REJECTED, None
        if self.free[cls]:
            s = self.free[cls].pop()
            s.busy = True
            return ADMITTED, s
        if self.growth_open and self.used + need <= self.budget:
            if self.allocate is not None:
                self.allocate(cls)
            s = Slot(cls, len(self.slots), busy=True)
            self.slots.append(s)
            self.used += need
            return ADMITTED, s
        return WAITING, None

    def release(self, s: Slot) -> None:
        assert s.busy, "slot released twice"
        s.busy = False
        self.free[s.cls].append(s)

    def count(self, cls: str) -> int:
        return sum(1 for s in self.slots if s.cls == cls)


@dataclass
class Request:
    rid: int
    cls: str
    arrival: float             # seconds since the start of the stream
    frame: int                 # index into the host frame pool of its class
    admitted: float = -1.0
    done: float = -1.0
    status: str = ""


def arrival_wait(dt: float) -> None:
    """Wait toward an event `dt` seconds ahead without oversleeping it: the
    OS sleep overshoots by tens of microseconds, so a long gap (over 200 us)
    is only half slept, for the caller to wait again, and a short one is
    spun out on the clock.  The spin touches no GPU state: querying events
    in a tight loop slowed the stream's own copies and launches.  Both
    servers wait for arrivals this way."""
    if dt > 2e-4:
        time.sleep(dt * 0.5)
        return
    end = time.perf_counter() + dt
    while time.perf_counter() < end:
        pass


def run_stream(reqs: list, pool: SlotPool, executor, clock, sleep, max_inflight: int = 2,
               on_done=None) -> dict:
    """Continuous batching over an arrival-ordered request list.

    `executor` provides: n (frames the current plan spans),
    launch(members) -> handle (enqueue one step over [(slot, request)]),
    ready(handle) -> bool, wait(handle) -> completion time (same clock as
    arrivals), and rebuild() (re-plan after the pool grew; called with no
    step in flight).  `clock()` gives seconds since the stream started and
    `sleep(dt)` waits at most `dt` (returning early only costs another
    poll).  `on_done(request, slot)`, if given, runs when a request's step
    has completed and before its slot is released (its outputs are still in
    the slot).  Every request ends ADMITTED with a
    completion time or REJECTED; the loop always terminates."""
    waiting = collections.OrderedDict()       # class -> FIFO of waiting requests
    nwait = 0
    inflight = collections.deque()            # (handle, [(slot, request)])
    nxt = 0
    stats = {"steps": 0, "plan_rebuilds": 0, "max_step": 0}

    def retire(block_one: bool) -> None:
        while inflight and (block_one or executor.ready(inflight[0][0])):
            h, members = inflight.popleft()
            done = executor.wait(h)
            for s, r in members:
                r.done = done
                if on_done is not None:
                    on_done(r, s)
                pool.release(s)
            block_one = False

    while nxt < len(reqs) or nwait or inflight:
        now = clock()
        while nxt < len(reqs) and reqs[nxt].arrival <= now:
            waiting.setdefault(reqs[nxt].cls, collections.deque()).append(reqs[nxt])
            nwait += 1
            nxt += 1
        retire(False)
        if nwait and len(inflight) >= max_inflight:
            retire(True)                      # a step slot frees when the oldest ends
            continue
        # admission: per class, in arrival order, while the class gets slots
        # (a slot depends only on the class, so the first refusal ends the class)
        admitted, grew = [], False
        for cls, q in waiting.items():
            while q:
                st, s = pool.acquire(cls)
                if st == ADMITTED:
                    r = q.popleft()
                    grew |= s.index >= executor.n
                    admitted.append((s, r))
                elif st == REJECTED:      # the class can never fit
                    for r in q:
                        r.status = REJECTED
                    nwait -= len(q)
                    q.clear()
                else:
                    break
        nwait -= len(admitted)
        if grew:
            while inflight:                   # let the GPU drain, then re-plan
                retire(True)
            executor.rebuild()
            stats["plan_rebuilds"] += 1
        if admitted:
            admitted.sort(key=lambda sr: sr[1].rid)
            for _, r in admitted:
                r.admitted = now
                r.status = ADMITTED
            inflight.append((executor.launch(admitted), admitted))
            stats["steps"] += 1
            stats["max_step"] = max(stats["max_step"], len(admitted))
        elif nwait and inflight:
            retire(True)                      # waiting for slots: they free when a step ends
        elif nwait:
            # nothing in flight and nothing admissible: every slot is free and
            # the budget is spent on other classes, so these can never run
            for q in waiting.values():
                for r in q:
                    r.status = REJECTED
                q.clear()
            nwait = 0
        else:
            # idle: until the next arrival, polling in-flight steps meanwhile
            gap = reqs[nxt].arrival - clock() if nxt < len(reqs) else float("inf")
            if inflight:
                gap = min(gap, 5e-5)
            if gap != float("inf"):
                sleep(max(gap, 1e-6))
    return stats


class GpuBatchExecutor:
    """Runs steps of `run_stream` on the GPU: one batch plan over all slots,
    a device activity mask, and a captured HIP graph replayed per step."""

    def __init__(self, classes: dict, host_frames: dict, normal_dtype, max_inflight: int, device):
        import torch

        import paper_2007_12065_amd as pl
        self.torch, self.pl = torch, pl
        self.dev = device
        self.classes = classes
        self.ndtype = normal_dtype
        self.host = frame_sources(torch, host_frames)
        self.inputs = []                      # device input tensor per slot
        self.slot_cls = []
        self.batch = None
        self.n = 0
        self.ring = 0
        self.max_inflight = max_inflight
        self.stream = torch.cuda.current_stream(device)
        self.copy_stream = torch.cuda.Stream(device)      # default priority
        self.ref = None
        self.single = {}                      # per class: scratch of the single-frame calls

    @staticmethod
    def single_bytes(pl, c, normal_bytes: int) -> int:
        """Device bytes of one class's scratch for single-frame steps: the
        fused entry's workspace."""
        return GpuBatchExecutor._frame_ws_bytes(pl, c, normal_bytes) + 256

    @staticmethod
    def _frame_ws_bytes(pl, c, normal_bytes: int) -> int:
        f = pl.PLFrame()
        f.M, f.N = c.M, c.N
        f.kernel_lap, f.iters_lap, f.lambda_ = c.kernel_lap, c.iters_lap, c.lam
        f.kernel_bil, f.iters_bil = c.kernel_bil, c.iters_bil
        f.sigma_length, f.sigma_angle = c.sigma_length, c.sigma_angle
        # the size query reads no buffer: distinct, aligned, non-overlapping
        # stand-in addresses are enough
        for i, name in enumerate(("pts", "pts_out", "normals", "centroids", "tri_map",
                                  "triangles", "n_tri", "normals_T")):
            setattr(f, name, (i + 1) << 36)
        ndt = pl.PL_F32 if normal_bytes == 4 else pl.PL_F16
        n = pl._lib.pl_smooth_frame_workspace(pl.ctypes.byref(f), ndt)
        if n == 0:
            raise pl.PLError(-1, "pl_smooth_frame_workspace")
        return int(n)

    def _single_scratch(self, cls: str):
        torch, pl = self.torch, self.pl
        if cls not in self.single:
            c = self.classes[cls]
            nb = 2 if self.ndtype == torch.float16 else 4
            n = self._frame_ws_bytes(pl, c, nb)
            self.single[cls] = (torch.empty(n, dtype=torch.uint8, device=self.dev), n)
        return self.single[cls]

    def _slot_frame(self, index: int):
        """The fused entry's frame descriptor for slot `index` (its input
        and the plan's outputs for it), built once per plan."""
        pl = self.pl
        c = self.classes[self.slot_cls[index]]
        o = self.batch.outputs[index]
        f = pl.PLFrame()
        f.M, f.N = c.M, c.N
        f.kernel_lap, f.iters_lap, f.lambda_ = c.kernel_lap, c.iters_lap, c.lam
        f.kernel_bil, f.iters_bil = c.kernel_bil, c.iters_bil
        f.sigma_length, f.sigma_angle = c.sigma_length, c.sigma_angle
        f.pts = self.inputs[index].data_ptr()
        for key, field in (("points", "pts_out"), ("normals", "normals"),
                           ("centroids", "centroids"), ("tri_valid", "tri_valid"),
                           ("tri_map", "tri_map"), ("triangles", "triangles"),
                           ("halfedges", "halfedges"), ("n_tri", "n_tri"),
                           ("normals_T", "normals_T")):
            setattr(f, field, o[key].data_ptr() if o[key] is not None else None)
        return f

    def run_single(self, index: int) -> None:
        """Slot `index` alone through the fused single-frame entry
        (pl_smooth_frame, a few launches), into its outputs: the same bits
        as a batched step."""
        pl = self.pl
        ws, n = self._single_scratch(self.slot_cls[index])
        pl._check(pl._lib.pl_smooth_frame(pl.ctypes.byref(self.frames[index]), pl._ndt(self.ndtype),
                                          pl._ptr(ws), n, pl._stream(self.dev)), "pl_smooth_frame")

    def alloc(self, cls: str) -> None:
        c = self.classes[cls]
        self.inputs.append(self.torch.zeros((c.M, c.N, 3), dtype=self.torch.float32, device=self.dev))
        self.slot_cls.append(cls)

    def rebuild(self) -> None:
        torch = self.torch
        if self.batch is not None:
            self.batch.close()
        specs = []
        for cls, x in zip(self.slot_cls, self.inputs):
            c = self.classes[cls]
            specs.append(dict(pts=x, kernel_lap=c.kernel_lap, lam=c.lam, iters_lap=c.iters_lap,
                              kernel_bil=c.kernel_bil, sigma_length=c.sigma_length,
                              sigma_angle=c.sigma_angle, iters_bil=c.iters_bil))
        self.batch = self.pl.Batch(specs, self.ndtype)
        self.n = len(specs)
        for cls in set(self.slot_cls):        # scratch for one-frame steps, allocated up front
            self._single_scratch(cls)
        self.frames = [self._slot_frame(i) for i in range(self.n)]
        self.mask_dev = torch.zeros(self.n, dtype=torch.uint8, device=self.dev)
        # the pinned mask of a step is reused max_inflight + 1 steps later,
        # when that step has been retired
        self.mask_host = [torch.zeros(self.n, dtype=torch.uint8).pin_memory()
                          for _ in range(self.max_inflight + 1)]
        self.mask_np = [m.numpy() for m in self.mask_host]   # host views of the pinned masks
        # one graph per bound on the step size (1, 2, 4, ..., all slots): a
        # step replays the smallest covering graph, whose launches are sized
        # for that many frames
        b = 1
        while True:
            self.batch.capture(self.mask_dev, max_active=min(b, self.n))
            if b >= self.n:
                break
            b *= 2

    def start_clock(self) -> None:
        self.stream.synchronize()
        self.ref = self.torch.cuda.Event(enable_timing=True)
        self.ref.record(self.stream)
        self.ref.synchronize()

    def launch(self, members):
        buf, view = self.mask_host[self.ring], self.mask_np[self.ring]
        self.ring = (self.ring + 1) % len(self.mask_host)
        view[:] = 0
        view[[s.index for s, _ in members]] = 1
        # a slot is refilled only after the step that last used it retired,
        # so these copies may overlap the steps still on the GPU; device-side
        # sources go in one fused copy, host sources one DMA each
        if len(members) == 1:
            # a lone frame: its copy and its calls back to back on the compute
            # stream (no cross-stream wait), as the plain path does
            s, r = members[0]
            self.inputs[s.index].copy_(self.host[r.cls][r.frame], non_blocking=True)
            self.run_single(s.index)
        else:
            dsts, srcs = [], []
            with self.torch.cuda.stream(self.copy_stream):
                for s, r in members:
                    src = self.host[r.cls][r.frame]
                    if src.is_cuda:
                        dsts.append(self.inputs[s.index])
                        srcs.append(src)
                    else:
                        self.inputs[s.index].copy_(src, non_blocking=True)
                if dsts:
                    self.torch._foreach_copy_(dsts, srcs, non_blocking=True)
                copied = self.torch.cuda.Event()
                copied.record(self.copy_stream)
            self.stream.wait_event(copied)
            self.mask_dev.copy_(buf, non_blocking=True)
            self.batch.replay(n_active=len(members))
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def ready(self, ev) -> bool:
        return ev.query()

    def wait(self, ev) -> float:
        ev.synchronize()
        return self.ref.elapsed_time(ev) / 1e3


class Server:
    """Continuous-batching server over one GPU (see module docstring)."""

    def __init__(self, classes: dict, host_frames: dict, budget_bytes: int,
                 normal_dtype=None, max_inflight: int = 2, device=None):
        import torch

        import paper_2007_12065_amd as pl
        dev = torch.device("cuda:0") if device is None else torch.device(device)
        self.classes = classes
        ndtype = torch.float16 if normal_dtype is None else normal_dtype
        nb = 2 if ndtype == torch.float16 else 4
        per = {k: slot_bytes(c, nb, pl.pl_tune_get(pl.PL_STAGE_LAPLACIAN, c.kernel_lap)[2],
                             pl.pl_tune_get(pl.PL_STAGE_BILATERAL, c.kernel_bil)[2])
               for k, c in classes.items()}
        self.exe = GpuBatchExecutor(classes, host_frames, ndtype, max_inflight, dev)
        # the single-frame steps' scratch (one set per class) comes out of the budget
        reserve = sum(GpuBatchExecutor.single_bytes(pl, c, nb) for c in classes.values())
        self.pool = SlotPool(max(budget_bytes - reserve, 0), per, allocate=self.exe.alloc)
        self.max_inflight = max_inflight

    def presize(self, counts: dict, freeze: bool = False) -> None:
        """Create `counts[cls]` slots of each class up front (within the
        budget) and build the plan; the pool may still grow later, unless
        `freeze` (then the budget shrinks to the slots just made: no plan
        rebuild can interrupt serving)."""
        for cls, k in counts.items():
            got = []
            for _ in range(k):
                st, s = self.pool.acquire(cls)
                if st != ADMITTED:
                    break
                got.append(s)
            for s in got:
                self.pool.release(s)
        if freeze:
            self.pool.budget = self.pool.used
        self.exe.rebuild()

    def serve(self, times, kinds, warmup_s: float = 1.0, pool_index=None, on_done=None) -> dict:
        """Serve arrivals at `times` (s) of classes `kinds`; requests arriving
        before `warmup_s` are served but not measured.  `on_done(request,
        outputs)` receives each completed request with the dict of its
        slot's device outputs (valid until the call returns)."""
        reqs = [Request(i, k, float(t), (i if pool_index is None else pool_index[i]) % len(self.exe.host[k]))
                for i, (t, k) in enumerate(zip(times, kinds))]
        self.exe.start_clock()
        t0 = time.perf_counter()
        cb = None
        if on_done is not None:
            cb = lambda r, s: on_done(r, self.exe.batch.outputs[s.index])
        stats = run_stream(reqs, self.pool, self.exe, lambda: time.perf_counter() - t0,
                           arrival_wait, self.max_inflight, cb)
        stats.update(slots=len(self.pool.slots), slot_bytes=self.pool.used)
        return summarize(reqs, warmup_s, self.classes, extra=stats)


class PlainServer:
    """The same arrival stream through the plain per-frame float32 path:
    frames are processed one at a time in arrival order (one resident
    buffer set per class, four ABI calls per frame).  Each frame's input is
    copied on the compute stream ahead of its calls: a per-frame copy stream
    (as the batched server uses per step) measured slower here, the loop
    being bound by its per-frame host work."""

    def __init__(self, classes: dict, host_frames: dict, device=None):
        import torch

        import paper_2007_12065_amd as pl
        self.torch, self.pl = torch, pl
        self.dev = torch.device("cuda:0") if device is None else torch.device(device)
        self.classes = classes
        self.host = frame_sources(torch, host_frames)
        self.inp = {k: torch.zeros((c.M, c.N, 3), dtype=torch.float32, device=self.dev)
                    for k, c in classes.items()}
        self.plan = {k: pl.FramePlan(c.M, c.N, c.kernel_lap, c.lam, c.iters_lap, c.kernel_bil,
                                     c.sigma_length, c.sigma_angle, c.iters_bil, torch.float32,
                                     self.dev) for k, c in classes.items()}
        self.stream = torch.cuda.current_stream(self.dev)

    def serve(self, times, kinds, warmup_s: float = 1.0, pool_index=None, max_inflight: int = 64) -> dict:
        torch = self.torch
        reqs = [Request(i, k, float(t), (i if pool_index is None else pool_index[i]) % len(self.host[k]))
                for i, (t, k) in enumerate(zip(times, kinds))]
        self.stream.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.stream)
        ref.synchronize()
        t0 = time.perf_counter()
        inflight = collections.deque()
        for r in reqs:
            while True:
                now = time.perf_counter() - t0
                if now >= r.arrival:
                    break
                arrival_wait(r.arrival - now)
            while len(inflight) >= max_inflight:
                ev, rr = inflight.popleft()
                ev.synchronize()
                rr.done = ref.elapsed_time(ev) / 1e3
            r.admitted = time.perf_counter() - t0
            r.status = ADMITTED
            self.inp[r.cls].copy_(self.host[r.cls][r.frame], non_blocking=True)
            self.plan[r.cls].run(self.inp[r.cls])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.stream)
            inflight.append((ev, r))
        while inflight:
            ev, rr = inflight.popleft()
            ev.synchronize()
            rr.done = ref.elapsed_time(ev) / 1e3
        return summarize(reqs, warmup_s, self.classes)


def summarize(reqs, warmup_s: float, classes: dict, extra: dict | None = None) -> dict:
    meas = [r for r in reqs if r.arrival >= warmup_s and r.status == ADMITTED and r.done >= 0]
    rejected = sum(1 for r in reqs if r.status == REJECTED)
    if not meas:
        return {"frames": 0, "rejected": rejected, **(extra or {})}
    lat = np.array([r.done - r.arrival for r in meas])
    t_first = min(r.arrival for r in meas)
    t_last = max(r.done for r in meas)
    tris = sum(2 * (classes[r.cls].M - 1) * (classes[r.cls].N - 1) for r in meas)
    out = {
        "frames": len(meas),
        "rejected": rejected,
        "triangles_per_s": tris / max(t_last - t_first, 1e-9),
        "frames_per_s": len(meas) / max(t_last - t_first, 1e-9),
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "latency_ms_max": float(lat.max() * 1e3),
    }
    out.update(extra or {})
    return out
