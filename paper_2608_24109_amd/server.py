"""Relighting service over exported assets: continuous batching of single-view renders.

A request names an asset (mesh-UV carrier with its material maps), one of the service's env
maps, a view, and direct-only or direct + one-bounce indirect shading (Eq. 17-20; relighting
is the forward pass under a new environment map). Requests arrive on a host clock and are
admitted while render slots and device memory are free, so work of requests that arrive
while others are on the GPU overlaps with theirs: every slot owns a HIP stream, and a request
runs on its slot's stream from map upload to the copy of its image into host memory.

Device memory is admitted by footprint against a budget:
  fixed     every asset's geometry (positions, indices, UVs, FP64 normals, tangents) and its
            BVH, and every env map with its sampling tables: resident for the service's life;
  maps      an asset's packed material map, uploaded from pinned host memory when a request
            needs it and evicted least-recently-used when no admitted request uses it;
  requests  G-buffer, outputs, visibility bits and secondary records of an admitted request,
            and its ray workspace (capped; the passes run in pixel chunks beyond the cap).
Admission is first-come first-served: a request that does not fit after evicting every idle
map waits for in-flight requests to finish; one larger than the whole budget is rejected.
A launch that raises (a library error) fails its request, or every request of its batch: they
retire with status "failed" and the error, their slot and memory are returned, and the service
goes on with the others.

The scheduler holds no device code and runs against any backend with the DeviceBackend
interface (the tests drive it with a simulated one on the CPU).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    asset: int
    env: int
    res: int
    azimuth: float
    indirect: bool
    arrival: float                 # scheduled arrival (seconds on the service clock)
    t_admit: float = math.nan
    t_done: float = math.nan
    status: str = "queued"         # queued | running | done | rejected | failed
    result: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Scheduler:
    """FIFO admission into `slots` render slots under an HBM budget (bytes).

    With batch_max > 1 and a backend that has `launch_batch`, a slot takes a batch: the admitted
    head of the queue plus the requests right behind it while they are direct-only and at most
    batch_res^2 pixels (up to batch_max of them, each admitted by footprint as usual); the batch
    renders in one launch sequence of the direct pass and its requests retire together."""

    def __init__(self, backend, budget: int, slots: int, batch_max: int = 1, batch_res: int = 512):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.b = backend
        self.budget = int(budget)
        self.free = list(range(slots - 1, -1, -1))
        self.queue: collections.deque[Request] = collections.deque()
        self.inflight: dict[int, tuple[list[Request], object, int]] = {}
        self.resident: collections.OrderedDict[int, int] = collections.OrderedDict()  # LRU first
        self.pins: collections.Counter = collections.Counter()
        self.fixed = int(backend.fixed_bytes())
        self.used = self.fixed
        self.peak = self.used
        self.loads = 0
        self.evictions = 0
        self.batch_max = max(1, int(batch_max)) if hasattr(backend, "launch_batch") else 1
        self.batch_res = int(batch_res)
        self.batches = 0
        self.failures = 0
        if self.fixed > self.budget:
            raise ValueError(f"resident geometry and env tables ({self.fixed} B) exceed the budget")

    def submit(self, req: Request) -> None:
        req.status = "queued"
        self.queue.append(req)

    def idle(self) -> bool:
        return not self.queue and not self.inflight

    def batchable(self, req: Request) -> bool:
        return self.batch_max > 1 and not req.indirect and req.res <= self.batch_res

    def poll(self, clock) -> list[Request]:
        """Retire finished requests (completion time read from `clock`)."""
        out = []
        for slot in list(self.inflight):
            reqs, tok, nb = self.inflight[slot]
            if self.b.done(tok):
                res = self.b.result(tok)
                res = res if isinstance(res, list) else [res]
                t = clock()
                for req, r in zip(reqs, res):
                    req.t_done = t
                    req.result = r
                    req.status = "done"
                    self.pins[req.asset] -= 1
                    out.append(req)
                del self.inflight[slot]
                self.free.append(slot)
                self.used -= nb
        return out

    def _fits(self, req: Request, slot: int):
        """Reserve the footprint of `req` (evicting idle maps as needed) and load its map into
        `slot`'s stream; returns the request bytes, None if it must wait, -1 if it never fits."""
        need = int(self.b.request_bytes(req))
        mb = 0 if req.asset in self.resident else int(self.b.map_bytes(req.asset))
        if self.fixed + need + mb > self.budget:
            return -1
        while self.used + need + mb > self.budget:
            victim = next((a for a in self.resident if self.pins[a] == 0 and a != req.asset), None)
            if victim is None:
                break
            self.used -= self.resident.pop(victim)
            self.b.evict_map(victim)
            self.evictions += 1
        if self.used + need + mb > self.budget:
            return None
        if mb:
            self.b.load_map(req.asset, slot)
            self.resident[req.asset] = mb
            self.used += mb
            self.loads += 1
        else:
            self.resident.move_to_end(req.asset)
        self.pins[req.asset] += 1
        self.used += need
        self.peak = max(self.peak, self.used)
        return need

    def admit(self, clock) -> list[Request]:
        """Admit queued requests in order while a slot is free and their footprint fits; returns
        the requests started, rejected or failed at launch."""
        started, rejected = [], []
        while self.queue and self.free:
            req = self.queue[0]
            slot = self.free[-1]
            need = self._fits(req, slot)
            if need == -1:
                self.queue.popleft()
                req.status = "rejected"
                req.t_done = clock()
                rejected.append(req)
                continue
            if need is None:
                break  # wait for in-flight requests to release memory
            self.queue.popleft()
            self.free.pop()
            batch, total = [req], need
            if self.batchable(req):
                while self.queue and len(batch) < self.batch_max and self.batchable(self.queue[0]):
                    nxt = self._fits(self.queue[0], slot)
                    if nxt is None or nxt == -1:
                        break
                    batch.append(self.queue.popleft())
                    total += nxt
            t = clock()
            for r in batch:
                r.t_admit = t
                r.status = "running"
            try:
                if len(batch) > 1:
                    tok = self.b.launch_batch(batch, slot)
                    self.batches += 1
                else:
                    tok = self.b.launch(req, slot)
            except RuntimeError as e:  # the library's errors (ExmError) and the backend's own
                t = clock()
                for r in batch:
                    r.status = "failed"
                    r.t_done = t
                    r.result = e
                    self.pins[r.asset] -= 1
                self.failures += len(batch)
                self.free.append(slot)
                self.used -= total
                rejected.extend(batch)
                continue
            self.inflight[slot] = (batch, tok, total)
            started.extend(batch)
        return started + rejected


def serve(sched: Scheduler, requests: list[Request], clock=time.monotonic, idle_sleep: float = 2e-4,
          realtime: bool = True, keep_results: bool = True) -> float:
    """Feed `requests` (arrival times relative to the start) into the scheduler on `clock` and
    run until all are retired. With realtime=False every request is submitted at once (used
    to measure saturation throughput). Completion and arrival times are stored on the
    requests relative to the start; with keep_results=False each image is dropped as soon as
    its request is retired. Returns the start time."""
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = clock()
    rel = lambda: clock() - t0  # noqa: E731
    i, left = 0, len(order)
    while left:
        now = rel()
        while i < len(order) and (not realtime or order[i].arrival <= now):
            if not realtime:
                order[i].arrival = now
            sched.submit(order[i])
            i += 1
        done = sched.poll(rel)
        out = sched.admit(rel)
        finished = done + [r for r in out if r.status in ("rejected", "failed")]
        left -= len(finished)
        if not keep_results:
            for r in finished:
                r.result = None
        if not finished and not any(r.status == "running" for r in out):
            nxt = order[i].arrival - rel() if i < len(order) else idle_sleep
            time.sleep(max(0.0, min(idle_sleep, nxt)))
    return t0


def latency_stats(reqs: list[Request], window: float | None = None) -> dict:
    """p50/p99/mean latency (ms) of completed requests, and throughput over the window from the
    stream's start to the last completion (or `window` seconds)."""
    ok = [r for r in reqs if r.status == "done"]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = window if window is not None else max((r.t_done for r in ok), default=float("nan"))
    px = float(sum(r.res * r.res for r in ok))
    return {"requests": len(reqs), "completed": len(ok), "rejected": sum(r.status == "rejected" for r in reqs),
            "failed": sum(r.status == "failed" for r in reqs),
            "p50_ms": float(np.percentile(lat, 50)) if len(ok) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(ok) else None,
            "mean_ms": float(lat.mean()) if len(ok) else None,
            "req_per_s": len(ok) / span if span and span > 0 else None,
            "mpx_per_s": px / span / 1e6 if span and span > 0 else None}


# ------------------------------------------------------------------------------------------
# device backend (torch memory and streams, every step of the render in libexm)
# ------------------------------------------------------------------------------------------

@dataclass
class HostAsset:
    """An exported asset in host memory: mesh-UV carrier and packed maps (pinned)."""
    pos: np.ndarray
    tri: np.ndarray
    uv: np.ndarray
    tri_uv: np.ndarray
    tex: object                     # torch.Tensor [Ht,Wt,8] float32, pinned host memory
    tmin: float = 0.0


@dataclass
class _Token:
    event: object
    out: object
    keep: list = field(default_factory=list)


class DeviceBackend:
    """Renders requests with the C ABI on per-slot HIP streams."""

    def __init__(self, assets: list[HostAsset], envs: list[np.ndarray], slots: int, N_d: int = 8, N_b: int = 4,
                 N_s: int = 4, seed: int = 3, ws_cap: int = 512 << 20, device="cuda"):
        import torch

        from .scene import DeviceEnv, DeviceMesh
        self.torch = torch
        self.device = device
        self.assets = assets
        self.N_d, self.N_b, self.N_s, self.seed = N_d, N_b, N_s, seed
        self.ws_cap = int(ws_cap)
        self.meshes = [DeviceMesh(a.pos, a.tri, a.uv, a.tri_uv, device=device) for a in assets]
        self.envs = [DeviceEnv(e, device=device) for e in envs]
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.maps: dict[int, tuple[object, object]] = {}
        torch.cuda.synchronize()

    def fixed_bytes(self) -> int:
        return sum(m.device_bytes() for m in self.meshes) + sum(e.device_bytes() for e in self.envs)

    def map_bytes(self, asset: int) -> int:
        t = self.assets[asset].tex
        return t.numel() * t.element_size()

    def _params(self, req: Request):
        from .render import PassParams
        return PassParams(N_d=self.N_d, N_b=self.N_b if req.indirect else 0, N_s=self.N_s, seed=self.seed,
                          tmin=self.assets[req.asset].tmin)

    def request_bytes(self, req: Request) -> int:
        from .render import shade_fwd_ws_bytes, trace_indirect_ws_bytes
        p = self._params(req)
        px = req.res * req.res
        per_px = 12 + 12 + 8                       # G-buffer, L_dir, vis
        ws = shade_fwd_ws_bytes(1, req.res, req.res, p)
        if p.N_b > 0:
            per_px += 12 + 12 * p.N_b + 8          # L_ind, secondary records, secondary vis
            ws = max(ws, trace_indirect_ws_bytes(1, req.res, req.res, p))
        return px * per_px + min(ws, self.ws_cap)

    def load_map(self, asset: int, slot: int) -> None:
        from .scene import DeviceMaterial
        torch = self.torch
        s = self.streams[slot]
        host = self.assets[asset].tex
        with torch.cuda.stream(s):
            t = torch.empty(host.shape, dtype=host.dtype, device=self.device)
            t.copy_(host, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.maps[asset] = (DeviceMaterial(t, device=self.device), ev)

    def evict_map(self, asset: int) -> None:
        del self.maps[asset]

    def launch(self, req: Request, slot: int) -> _Token:
        from . import _lib as L
        from . import inputs as I
        from .render import PassBuffers, render_forward
        torch = self.torch
        s = self.streams[slot]
        mat, ready = self.maps[req.asset]
        a = self.assets[req.asset]
        p = self._params(req)
        cam = I.relight_camera(a.pos, req.res, req.azimuth)
        with torch.cuda.stream(s):
            s.wait_event(ready)
            mat.tex.record_stream(s)
            bufs = PassBuffers(1, req.res, req.res, p.N_b, device=self.device, ws_cap=self.ws_cap)
            render_forward(self.meshes[req.asset], mat, self.envs[req.env], L.cameras([cam], [req.rid]), p, bufs,
                           rebuild_tables=False)
            if p.N_b > 0:
                bufs.L_dir.add_(bufs.L_ind)
            out = torch.empty((req.res, req.res, 3), dtype=torch.float32, pin_memory=True)
            out.copy_(bufs.L_dir[0], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return _Token(ev, out, [bufs, mat])

    def launch_batch(self, reqs: list[Request], slot: int) -> _Token:
        """Direct-only requests rendered together: a G-buffer per request, then one batched
        direct pass (exm_shade_fwd_batch) over all of them, on the slot's stream."""
        from . import _lib as L
        from . import inputs as I
        from .render import PassBuffers, raster
        torch = self.torch
        s = self.streams[slot]
        keep, bufs_all, creqs, outs = [], [], [], []
        with torch.cuda.stream(s):
            for req in reqs:
                mat, ready = self.maps[req.asset]
                s.wait_event(ready)
                mat.tex.record_stream(s)
                a = self.assets[req.asset]
                cam = L.cameras([I.relight_camera(a.pos, req.res, req.azimuth)], [req.rid])
                bufs = PassBuffers(1, req.res, req.res, 0, device=self.device)
                raster(self.meshes[req.asset], cam, bufs)
                creqs.append(L.request(self.meshes[req.asset], mat, self.envs[req.env], cam[0], a.tmin, bufs.tri_id,
                                       bufs.bary, bufs.L_dir, bufs.vis))
                bufs_all.append(bufs)
                keep.append(mat)
            p = self._params(reqs[0]).c()  # N_d and flags are shared; each request carries its tmin
            ws = L.workspace(L.exm_shade_fwd_batch_workspace_size(creqs, p.N_d), self.device)
            L.exm_shade_fwd_batch(creqs, p, ws)
            keep += bufs_all + [ws]
            for req, bufs in zip(reqs, bufs_all):
                out = torch.empty((req.res, req.res, 3), dtype=torch.float32, pin_memory=True)
                out.copy_(bufs.L_dir[0], non_blocking=True)
                outs.append(out)
            ev = torch.cuda.Event()
            ev.record(s)
        return _Token(ev, outs, keep)

    def done(self, tok: _Token) -> bool:
        return tok.event.query()

    def result(self, tok: _Token):
        tok.keep.clear()
        return tok.out


def build_host_assets(specs, device="cuda", workers: int = 8) -> list[HostAsset]:
    """Meshes on host threads; maps drawn on the device and copied into pinned host memory."""
    import torch
    from concurrent.futures import ThreadPoolExecutor

    from . import inputs as I
    with ThreadPoolExecutor(max(1, workers)) as ex:
        meshes = list(ex.map(I.relight_asset_mesh, specs))
    out = []
    for sp, (pos, tri, uv, tri_uv) in zip(specs, meshes):
        dev = I.pbr_maps_device(sp.tex_res, sp.tex_res, sp.seed, device=device)
        host = torch.empty(dev.shape, dtype=torch.float32, pin_memory=True)
        host.copy_(dev)
        del dev
        out.append(HostAsset(pos, tri, uv, tri_uv, host, tmin=1e-4 * I.aabb_diagonal(pos)))
    torch.cuda.synchronize()
    return out


def requests_from_specs(specs) -> list[Request]:
    return [Request(s.rid, s.asset, s.env, s.res, s.azimuth, s.indirect, s.arrival) for s in specs]
