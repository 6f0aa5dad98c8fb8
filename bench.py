"""Benchmark of the Stage-II UV-PBR render pass on one MI355X.

One step = one pass of the whole hot path over the workload's views: env sampling tables,
G-buffer raster, direct shading and one-bounce indirect light, then the adjoint of both into
the UV maps and the env map. Inputs are resident in HBM before timing starts.

The headline workload (the default) is the differentiation form at its full size: the tori
mesh (1M triangles), 32 views of 1024^2, 4096^2 maps, a 512x1024 env map with gradients,
N_d 64 + N_b 4 x N_s 4, through the autograd.Function with the G-buffer rasterised again in
backward. The sphere (8 views, direct), tori (8 views, indirect), small, serving and paper-shape
rows run beside it as extras.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tori32|sphere|tori|small]

Prints one JSON line. The metric is forward+backward Mpixels/s at 1024^2 (all pixels of the
step counted, background included); per-kernel times come from HIP events recorded on the
stream the kernels are launched on.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP32_LANE_PEAK_T = 39.32    # 256 CU x 64 lanes x 2.4 GHz, non-packed FP32 instructions per second (1e12)

METRIC = "fwd+bwd Mpixels/s and indirect Mrays/s at 1024²; relight p50/p99 ms"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tori32", choices=["tori32", "sphere", "tori", "small"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-views", type=int, default=8, help="views of the workload the oracle baseline samples")
    ap.add_argument("--cpu-pixels", type=int, default=393216, help="pixels per view the oracle baseline renders")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB once (HBM counter calibration)")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the extra workloads (sphere, tori, small, serving, paper shape, Stage I/II)")
    ap.add_argument("--relight-seconds", type=float, default=60.0, help="length of the relight request stream")
    ap.add_argument("--relight-rate", type=float, default=200.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--relight-budget-gib", type=float, default=8.0, help="HBM budget of the relight service")
    ap.add_argument("--relight-slots", type=int, default=8, help="concurrent render slots (streams)")
    return ap.parse_args()


class Timer:
    """Per-ABI-call HIP event pairs on the current (launch) stream."""

    def __init__(self, torch):
        self.torch = torch
        self.ev = {}

    def __call__(self, name, fn):
        t = self.torch.cuda
        a, b = t.Event(enable_timing=True), t.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.ev.setdefault(name, []).append((a, b))

    def mean_ms(self):
        return {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in self.ev.items()}


def run_gpu(workload: str, steps: int, warmup: int):
    import torch

    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd import inputs as I
    from paper_2608_24109_amd.render import PassBuffers, PassParams, raster
    from paper_2608_24109_amd.scene import DeviceEnv, DeviceMaterial, DeviceMesh

    sc = I.config(workload)
    mesh = DeviceMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    mat = DeviceMaterial(sc.tex)
    env = DeviceEnv(sc.env)
    V, H, W = len(sc.cams), sc.cams[0].H, sc.cams[0].W
    p = PassParams(N_d=sc.N_d, N_b=sc.N_b, N_s=sc.N_s, seed=sc.seed, tmin=sc.tmin)
    pc = p.c()
    cc = L.cameras(sc.cams, list(range(V)))
    bufs = PassBuffers(V, H, W, p.N_b)
    dI = torch.from_numpy(I.upstream_grad(V, H, W)).cuda()
    dtex = torch.zeros_like(mat.tex)
    denv = torch.zeros(env.env.shape, dtype=torch.float64, device="cuda")
    lam = 1.0
    He, We = sc.env.shape[:2]
    ws_fwd = bufs.workspace(max(L.exm_shade_fwd_workspace_size(V, H, W, p.N_d),
                                L.exm_trace_indirect_workspace_size(V, H, W, p.N_b, p.N_s) if p.N_b else 0,
                                L.exm_shade_bwd_workspace_size(V, H, W, p.N_d, He, We),
                                L.exm_trace_bwd_workspace_size(V, H, W, p.N_b, p.N_s, He, We) if p.N_b else 0))
    torch.cuda.synchronize()

    def step(tm):
        tm("build_env_sampler", lambda: env.update())
        tm("raster_gbuffer", lambda: raster(mesh, cc, bufs))
        tm("shade_fwd", lambda: L.exm_shade_fwd(mesh.s, mesh.bvh, mat.s, env.s, cc, bufs.tri_id, bufs.bary, pc,
                                                bufs.L_dir, bufs.vis, ws_fwd))
        if p.N_b > 0:
            tm("trace_indirect", lambda: L.exm_trace_indirect(mesh.s, mesh.bvh, mat.s, env.s, cc, bufs.tri_id,
                                                              bufs.bary, pc, bufs.L_ind, bufs.sec_rec, bufs.sec_vis,
                                                              ws_fwd))
            tm("compose", lambda: torch.add(bufs.L_dir, bufs.L_ind, alpha=lam))
        tm("zero_grads", lambda: (dtex.zero_(), denv.zero_()))
        tm("shade_bwd", lambda: L.exm_shade_bwd(mesh.s, mat.s, env.s, cc, bufs.tri_id, bufs.bary, pc, dI, bufs.vis,
                                                dtex, denv, ws_fwd))
        if p.N_b > 0:
            tm("trace_bwd", lambda: L.exm_trace_bwd(mesh.s, mat.s, env.s, cc, bufs.tri_id, bufs.bary, pc, lam, dI,
                                                    bufs.sec_rec, bufs.sec_vis, dtex, denv, ws_fwd))

    warm = Timer(torch)
    for _ in range(warmup):
        step(warm)
    torch.cuda.synchronize()
    tm = Timer(torch)
    L.exm_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(tm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = tm.mean_ms()
    gk = L.exm_timing_collect()
    L.exm_timing_enable(False)
    gpu_kern = {k: {"avg_ms": ms / n, "launches_per_step": n / steps, "ms_per_step": ms / steps}
                for k, (ms, n) in gk.items()}

    stats = count_work(sc, mesh, mat, env, p)
    stats["gpu_kernels"] = gpu_kern
    return sc, p, wall, kern, stats, (mesh, mat, env, bufs)


def count_work(sc, mesh, mat, env, p, chunk: int = 8) -> dict:
    """Work counts of one step of the workload, from the library's counting variants of the
    direct and indirect passes (run outside the timed region, `chunk` views at a time): rays
    traced, BVH nodes visited, triangles tested, env samples drawn, covered pixels, unoccluded
    samples and secondary hits."""
    import torch

    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd.render import PassBuffers, raster
    V, H, W = len(sc.cams), sc.cams[0].H, sc.cams[0].W
    pc = p.c()
    n = min(chunk, V)
    bufs = PassBuffers(n, H, W, p.N_b)
    ws = bufs.workspace(max(L.exm_shade_fwd_workspace_size(n, H, W, p.N_d),
                            L.exm_trace_indirect_workspace_size(n, H, W, p.N_b, p.N_s) if p.N_b else 0))
    c_dir = torch.zeros(4, dtype=torch.uint64, device="cuda")
    c_ind = torch.zeros(6, dtype=torch.uint64, device="cuda")
    covered = set_bits = sec_hits = sec_set = 0
    env.update()
    for v0 in range(0, V, n):
        cc = L.cameras(sc.cams[v0:v0 + n], list(range(v0, v0 + n)))
        raster(mesh, cc, bufs)
        L.exm_shade_fwd_counted(mesh.s, mesh.bvh, mat.s, env.s, cc, bufs.tri_id, bufs.bary, pc, bufs.L_dir,
                                bufs.vis, ws, c_dir)
        if p.N_b > 0:
            L.exm_trace_indirect_counted(mesh.s, mesh.bvh, mat.s, env.s, cc, bufs.tri_id, bufs.bary, pc, bufs.L_ind,
                                         bufs.sec_rec, bufs.sec_vis, ws, c_ind)
            sec_hits += int((bufs.sec_rec[..., 0] >= 0).sum())
            sec_set += int(np.unpackbits(bufs.sec_vis.cpu().numpy().reshape(-1).view(np.uint8)).sum())
        covered += int((bufs.tri_id >= 0).sum())
        set_bits += int(np.unpackbits(bufs.vis.cpu().numpy().reshape(-1).view(np.uint8)).sum())
    torch.cuda.synchronize()
    cd = [int(x) for x in c_dir.cpu().numpy()]
    ci = [int(x) for x in c_ind.cpu().numpy()]
    stats = dict(views=V, H=H, W=W, pixels=V * H * W, covered=covered, tris=int(sc.nF),
                 texels=int(sc.tex.shape[0] * sc.tex.shape[1]), He=int(sc.env.shape[0]), We=int(sc.env.shape[1]),
                 samples=cd[3], shadow_rays=cd[0], shadow_nodes=cd[1], shadow_tris=cd[2], unoccluded=set_bits)
    if p.N_b > 0:
        stats.update(sec_rays=ci[0], sec_nodes=ci[1], sec_tris=ci[2], sec_shadow_rays=ci[3], sec_shadow_nodes=ci[4],
                     sec_shadow_tris=ci[5], sec_hits=sec_hits, sec_unoccluded=sec_set)
    return stats


def run_tori32(steps: int, warmup: int):
    """The headline: the differentiation form at full size. RenderPBR (the autograd.Function)
    over the 32 views of the tori mesh with 4096^2 maps and env gradients, 8 views per chunk,
    each chunk's G-buffer freed after the forward and rasterised again in backward. One step =
    env tables, forward, backward (gradient buffers allocated and cleared inside)."""
    import torch

    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd import inputs as I
    from paper_2608_24109_amd.render import PassParams, RenderPBR
    from paper_2608_24109_amd.scene import DeviceEnv, DeviceMaterial, DeviceMesh
    sc = I.config("tori32")
    mesh = DeviceMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    mat = DeviceMaterial(sc.tex)
    env = DeviceEnv(sc.env)
    p = PassParams(N_d=sc.N_d, N_b=sc.N_b, N_s=sc.N_s, seed=sc.seed, tmin=sc.tmin)
    V, H, W = len(sc.cams), sc.cams[0].H, sc.cams[0].W
    g = torch.from_numpy(I.upstream_grad(V, H, W)).cuda()
    tex = mat.tex.requires_grad_(True)
    emap = env.env.requires_grad_(True)

    def step():
        out = RenderPBR.apply(tex, emap, mesh, mat, env, sc.cams, p, 1.0, True)
        out.backward(g)
        tex.grad = None
        emap.grad = None

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    L.exm_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gk = L.exm_timing_collect()
    L.exm_timing_enable(False)
    tex.requires_grad_(False)
    emap.requires_grad_(False)
    stats = count_work(sc, mesh, mat, env, p)
    stats["gpu_kernels"] = {k: {"avg_ms": ms / n, "launches_per_step": n / steps, "ms_per_step": ms / steps}
                            for k, (ms, n) in gk.items()}
    return sc, p, wall, stats


def run_relight(seconds: float, rate: float, budget_gib: float, slots: int, batch_max: int = 8,
                per_stream_seconds: float = 20.0):
    """The relighting service: 64 seeded assets (spheres and tori of 10k-2M triangles, maps of
    512^2-4096^2), 16 env maps of 256x512, Poisson arrivals; p50/p99 latency (arrival to image
    in host memory, host monotonic clock) and throughput; then the saturation throughput with
    every request of a 5 s stream queued at once. Direct-only requests of at most 512^2 that stand
    together at the head of the queue render in one batched direct pass (up to batch_max of
    them); the same service without batching runs beside it on a shorter stream."""
    from paper_2608_24109_amd import inputs as I
    from paper_2608_24109_amd.server import (DeviceBackend, Scheduler, build_host_assets, latency_stats,
                                             requests_from_specs, serve)
    specs = I.relight_asset_specs()
    assets = build_host_assets(specs, workers=min(16, len(os.sched_getaffinity(0))))
    be = DeviceBackend(assets, I.relight_envs(), slots=slots)
    budget = int(budget_gib * (1 << 30))
    r = lambda x: None if x is None else round(x, 3)  # noqa: E731

    def one(secs, bmax):
        reqs = requests_from_specs(I.relight_stream(rate=rate, seconds=secs))
        sched = Scheduler(be, budget, slots=slots, batch_max=bmax, batch_res=512)
        serve(sched, reqs, keep_results=False)
        st = latency_stats(reqs)
        sat_reqs = requests_from_specs(I.relight_stream(rate=rate, seconds=min(5.0, secs)))
        sat = Scheduler(be, budget, slots=slots, batch_max=bmax, batch_res=512)
        serve(sat, sat_reqs, realtime=False, keep_results=False)
        ss = latency_stats(sat_reqs)
        return {"p50_ms": r(st["p50_ms"]), "p99_ms": r(st["p99_ms"]), "mean_ms": r(st["mean_ms"]),
                "completed": st["completed"], "rejected": st["rejected"], "req_per_s": r(st["req_per_s"]),
                "Mpixels_s": r(st["mpx_per_s"]), "batches": sched.batches, "map_loads": sched.loads,
                "map_evictions": sched.evictions, "resident_fixed_GiB": round(sched.fixed / 2**30, 3),
                "peak_GiB": round(sched.peak / 2**30, 3), "saturation_req_per_s": r(ss["req_per_s"]),
                "saturation_Mpixels_s": r(ss["mpx_per_s"])}

    out = {"workload": f"{len(specs)} assets ({sum(s.n_tris for s in specs) / 1e6:.1f}M tris, "
                       f"{sum(be.map_bytes(a) for a in range(len(specs))) / 2**30:.1f} GiB of maps), 16 envs "
                       f"256x512, views 256^2-2048^2, direct (N_d=8) or + indirect (N_b=4, N_s=4), "
                       f"Poisson {rate:g} req/s for {seconds:g} s, HBM budget {budget_gib:g} GiB, {slots} slots, "
                       f"batches of up to {batch_max} direct-only requests of at most 512^2"}
    out.update(one(seconds, batch_max))
    row = one(per_stream_seconds, 1)
    row["workload"] = f"the same service without batching (one request per slot), {per_stream_seconds:g} s stream"
    out["per_stream"] = row
    return out


def run_paper_shape(frames: int = 20):
    """Relighting at the paper's timing shape (forward only): per frame a new env map is copied
    from pinned host memory and its tables rebuilt, then the G-buffer, the direct pass and, for
    the full setting, the half-resolution indirect pass and its upsampling; timed over `frames`
    frames after one warm-up frame, cycling through 4 env maps."""
    import torch

    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd import inputs as I
    from paper_2608_24109_amd.render import PassBuffers, PassParams, render_forward
    from paper_2608_24109_amd.scene import DeviceEnv, DeviceMaterial, DeviceMesh
    sc = I.config("paper_shape")
    mesh = DeviceMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    mat = DeviceMaterial(sc.tex)
    env = DeviceEnv(sc.env)
    envs = [torch.from_numpy(I.env_map(256, 512, 1.0, seed=200 + k)).pin_memory() for k in range(4)]
    cam = sc.cams[0]
    cc = L.cameras([cam], [0])
    out = {"workload": f"paper_shape: {sc.nF} tris ({sc.nV} vertices), 1 view {cam.H}x{cam.W}, "
                       f"{sc.tex.shape[0]}^2 maps, 256x512 env (new map each frame: copy from host + tables), "
                       f"N_d={sc.N_d}; full adds N_b={sc.N_b} at half resolution (upsampled), N_s={sc.N_s}",
           "paper_context_fps": {"direct": 40.47, "full": 15.09, "hardware": "RTX A6000 (RT cores), its own scenes"}}
    for mode in ("direct", "full"):
        p = PassParams(N_d=sc.N_d, N_b=sc.N_b if mode == "full" else 0, N_s=sc.N_s, seed=sc.seed, tmin=sc.tmin,
                       half_res_indirect=mode == "full")
        bufs = PassBuffers(1, cam.H, cam.W, p.N_b, half=p.half_res_indirect)

        def frame(k):
            env.env.copy_(envs[k % 4], non_blocking=True)
            render_forward(mesh, mat, env, cc, p, bufs)
            if p.N_b > 0:
                bufs.L_dir.add_(bufs.L_ind)

        frame(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, frames + 1):
            frame(k)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / frames
        out[f"{mode}_fps"] = round(1.0 / dt, 2)
        out[f"{mode}_ms"] = round(dt * 1e3, 3)
    return out


def run_stage2(iters: int = 20):
    """Stage-II optimisation iterations at the paper's sampling (N_d 8; full adds N_b 16 at half
    resolution, upsampled, N_s 4) on the paper-shape asset: per iteration one 1600^2 training
    view rendered, the objective (log-L1 + D-SSIM, material TV of the projected maps, env TV and
    chroma) and its gradient, the render adjoint, and the Adam steps of the maps and the env map;
    timed over `iters` iterations after 3 warm-up iterations. Targets are renders of the asset's
    own maps; the loop starts from the Stage-II initialisation."""
    import torch

    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd import inputs as I
    from paper_2608_24109_amd.optimize import Stage2, Stage2Config, initial_maps
    from paper_2608_24109_amd.render import PassBuffers, PassParams, render_forward
    from paper_2608_24109_amd.scene import DeviceEnv, DeviceMaterial, DeviceMesh
    sc = I.config("paper_shape")
    mesh = DeviceMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    H = W = sc.cams[0].H
    cams = I.ring_cameras(4, 3.0, H, W)
    mat_gt, env_gt = DeviceMaterial(sc.tex), DeviceEnv(sc.env)
    pt = PassParams(N_d=sc.N_d, N_b=sc.N_b, N_s=sc.N_s, seed=sc.seed, tmin=sc.tmin, flags=L.EXM_METALLIC_OFF,
                    half_res_indirect=True)
    tg = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device="cuda")
    b = PassBuffers(1, H, W, pt.N_b, half=True)
    for k, c in enumerate(cams):
        render_forward(mesh, mat_gt, env_gt, L.cameras([c], [k]), pt, b)
        tg[k] = (b.L_dir + b.L_ind)[0]
    del b, mat_gt
    Ht, Wt = sc.tex.shape[:2]
    out = {"workload": f"paper_shape: {sc.nF} tris, {Ht}^2 maps, 256x512 env, 1 training view {H}x{W} per "
                       f"iteration (of 4), N_d={sc.N_d}; full adds N_b={sc.N_b} at half resolution, N_s={sc.N_s}",
           "paper_context_ms_per_iteration": {"full": 102, "direct": 60,
                                              "hardware": "RTX A6000 (RT cores), 10K iterations in 17 / 10 min"}}
    for mode in ("full", "direct"):
        tex0, env0 = initial_maps(np.clip(sc.tex[..., :3], 0, 1), Ht, Wt, 256, 512)
        cfg = Stage2Config(iters=10_000, N_d=sc.N_d, N_b=sc.N_b, N_s=sc.N_s, half_res_indirect=True,
                           tmin=sc.tmin, ramp_iters=1, indirect="train" if mode == "full" else "off")
        opt = Stage2(mesh, DeviceMaterial(tex0), DeviceEnv(env0), cams, tg, cfg)
        for _ in range(3):
            opt.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            opt.step()
        torch.cuda.synchronize()
        out[f"{mode}_ms_per_iteration"] = round((time.perf_counter() - t0) / iters * 1e3, 3)
        del opt
    return out


def run_topology(rounds: int = 5):
    """Stage-I topology rounds at the paper's scale: the paper-shape mesh (99,372 faces) with 500
    planted slivers, random vertex EMAs and 2% of the faces unrendered; per round the criteria,
    5% of the faces selected for splitting, the merge candidates, the conflict resolution, the
    operations with their UV updates and the compaction. Each timed round starts from the same
    mesh (copied in, untimed)."""
    import torch

    from paper_2608_24109_amd import inputs as I
    from paper_2608_24109_amd.topology import DeviceTopoMesh, TopoConfig
    sc = I.config("paper_shape")
    rng = np.random.default_rng(7)
    pos = sc.pos.copy()
    keys = np.unique(np.sort(np.stack([sc.tri, np.roll(sc.tri, -1, 1)], -1).reshape(-1, 2), 1), axis=0)
    for a, b in keys[rng.choice(len(keys), 500, replace=False)]:
        pos[a] = pos[a] + 0.9 * (pos[b] - pos[a])
    G = rng.random(pos.shape[0]).astype(np.float32)
    c = np.ones(sc.tri.shape[0], np.int32)
    c[rng.choice(sc.tri.shape[0], 2000, replace=False)] = 0
    c_dev = torch.from_numpy(c).cuda()
    times, st = [], None
    for k in range(rounds + 1):
        dm = DeviceTopoMesh(pos, sc.tri, sc.uv, sc.tri_uv, G, TopoConfig())
        dm._workspace()  # allocated outside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = dm.round(c_dev)
        torch.cuda.synchronize()
        if k > 0:
            times.append((time.perf_counter() - t0) * 1e3)
    return {"workload": f"paper_shape mesh: {sc.tri.shape[0]} faces, 500 slivers, 2% unrendered faces, "
                        f"split fraction 0.05, face budget 200K; one round (criteria, ranking, conflict "
                        f"resolution, operations, UV updates, compaction)",
            "ms_per_round": round(float(np.median(times)), 3), "faces_out": int(dm.nF),
            "splits": st["splits"], "merges": st["merges"], "conflict_passes": st["mis_iterations"]}


def cpu_baseline(sc, p, n_views: int, n_pix: int):
    """The FP64 oracle as it stands on a bounded sample of the workload: `n_pix` pixels drawn
    uniformly (seeded, background included in proportion) from each of `n_views` views spread
    over the workload's views; its forward pass and one forward-mode derivative pass (the
    gradient along one direction) per view, timed on the host cores."""
    import oracle as O
    om = O.OracleMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    tab = O.EnvTables(sc.env)
    cores = len(os.sched_getaffinity(0))
    tex_dot = np.zeros_like(sc.tex, dtype=np.float64)
    tex_dot[..., 0] = 1.0
    rng = np.random.default_rng(12)
    views = np.linspace(0, len(sc.cams) - 1, n_views).round().astype(int)
    px = 0
    t0 = time.perf_counter()
    for v in views:
        cam = sc.cams[v]
        pix = np.sort(rng.choice(cam.H * cam.W, min(n_pix, cam.H * cam.W), replace=False))
        kw = dict(N_d=p.N_d, N_b=p.N_b, N_s=p.N_s, seed=p.seed, tmin=p.tmin, view_id=int(v), pix=pix,
                  n_threads=cores)
        O.render(om, cam, tab, sc.tex, sc.env, **kw)
        O.render(om, cam, tab, sc.tex, sc.env, tex_dot=tex_dot, **kw)
        px += pix.size
    t = time.perf_counter() - t0
    return {"value": round(px / t / 1e6, 5), "unit": "Mpixels/s", "cores": cores, "kind": "oracle",
            "sample": f"{px} pixels of the {sc.name} workload ({n_pix} drawn uniformly from each of {len(views)} of "
                      f"its {len(sc.cams)} views, background included), FP64 forward + one forward-mode derivative "
                      f"pass (the fwd+bwd work of those pixels; each pass also rasterises its view), {t:.1f} s on "
                      f"{cores} host threads"}


# Algorithmic bytes: what the method itself must read or write per unit, times the units of one
# launch. Per covered pixel the attribute query reads 3 vertices (12 B position + 24 B FP64
# normal), the triangle's vertex and UV indices (12 + 12 B), 3 UVs (24 B), the face tangent
# (16 B) and 4 bilinear taps of 8 floats (128 B): 300 B. Each env sample reads the two
# cutpoint entries of its column bucket (8 B), the CDF entry that decides the pick (8 B) and the
# texel's record (E and 1/pdf, 16 B): 32 B (the row tables are block-shared). Each traced ray
# reads the 4-wide nodes it visits (NODE_BYTES) and the triangles it tests (48 B). An adjoint
# env sample adds three FP64 read-modify-writes (48 B); a pixel's map adjoint 4 taps x 8 FP32
# (256 B).
SURF_BYTES = 3 * (12 + 24) + 12 + 12 + 24 + 16 + 4 * 32
SAMPLE_BYTES = 8 + 8 + 16
NODE_BYTES = 128.0  # four child boxes (96 B) and four child references (16 B), one cache line


def algorithmic_bytes(kernel: str, st: dict, p) -> float:
    P, C = st["pixels"], st["covered"]
    if kernel == "raster_gbuffer":  # G-buffer out, 8 B depth key in/out, mesh per view
        return (12.0 + 16.0) * P + st["views"] * 24.0 * st["tris"]
    if kernel == "build_env_sampler":
        return st["He"] * st["We"] * (12 + 8 + 4 + 16 + 4) + 8.0 * st["He"]
    if kernel == "shade_fwd":
        return (32.0 * P + SURF_BYTES * C + SAMPLE_BYTES * st["samples"]
                + NODE_BYTES * st["shadow_nodes"] + 48.0 * st["shadow_tris"])
    if kernel == "shade_bwd":
        return 32.0 * P + (SURF_BYTES + 256.0) * C + (SAMPLE_BYTES + 48) * st["unoccluded"]
    if kernel == "trace_indirect":
        return (12.0 * P + 20.0 * C + st["sec_rays"] * 12.0 + st["sec_hits"] * SURF_BYTES
                + SAMPLE_BYTES * st["sec_shadow_rays"]
                + NODE_BYTES * (st["sec_nodes"] + st["sec_shadow_nodes"]) + 48.0 * (st["sec_tris"] + st["sec_shadow_tris"]))
    if kernel == "trace_bwd":
        return (44.0 * P + (SURF_BYTES + 224.0) * C + st["sec_hits"] * (SURF_BYTES + 224.0)
                + (SAMPLE_BYTES + 48) * st["sec_unoccluded"])
    return float("nan")


def kernel_bytes_per_step(kernel: str, st: dict, p) -> float:
    """Algorithmic bytes of one GPU kernel over one step (same per-unit figures as above; the
    ray workspace that links the wavefront kernels is this design's own traffic, not counted)."""
    P, C = st["pixels"], st["covered"]
    if kernel == "trace_any":  # direct shadow rays, and the secondary ones where the workload has them:
        # a 16 B ray record in and 1 B out per ray, a 16 B origin record per covered pixel or secondary point
        return (17.0 * (st["shadow_rays"] + st.get("sec_shadow_rays", 0)) + 16.0 * (C + st.get("sec_hits", 0))
                + NODE_BYTES * (st["shadow_nodes"] + st.get("sec_shadow_nodes", 0))
                + 48.0 * (st["shadow_tris"] + st.get("sec_shadow_tris", 0)))
    if kernel == "trace_closest":  # 16 B ray record in, 16 B hit out, a 16 B origin per covered pixel
        return 32.0 * st["sec_rays"] + 16.0 * C + NODE_BYTES * st["sec_nodes"] + 48.0 * st["sec_tris"]
    if kernel == "dir_gen":
        return 12.0 * P + SURF_BYTES * C + SAMPLE_BYTES * st["samples"]
    if kernel == "dir_finalize":
        return 20.0 * P + 13.0 * st["shadow_rays"]
    if kernel == "shade_bwd":
        return 32.0 * P + (SURF_BYTES + 256.0) * C + (SAMPLE_BYTES + 16) * st["unoccluded"]
    if kernel == "raster":
        return st["views"] * 24.0 * st["tris"] + 8.0 * C
    return float("nan")


# Algorithmic VALU work per unit, one lane operation each (add, mul, fma, min, max, compare,
# select): a 4-wide node visit tests four child boxes, per child and axis 2 subtractions, 2
# multiplications by the inverse direction, a min and a max (18), entry and exit as the max /
# min of three axes and the ray interval (6) and their comparison (1): 4 x 25; then orders the
# hit children by entry distance, a compare-exchange of (distance, reference) being a min, a max
# and two selects (4): the nearest first for an any-hit query (3 exchanges, NODE_OPS = 112), all
# four sorted for a closest-hit one (5 exchanges, NODE_OPS_CLOSEST = 120). A watertight
# ray/triangle test (Woop, Benthin and Wald 2013): vertices relative to the origin (9), shear
# (6), edge functions U, V, W (9), sign tests (6), determinant (2), scaled distance (8), its
# reciprocal and product (2), range test (2): 44. The env-map pick and the
# shading of one sample (dir_gen, every sample drawn) and the adjoint of one unoccluded sample
# (shade_bwd; samples that are occluded or face away contribute nothing and are skipped) take
# about 150 and 350 lane operations (estimates from the instruction mix of the BRDF and its
# derivatives). Every count stays below the lane operations the SQ counters show executed.
NODE_OPS, NODE_OPS_CLOSEST, TRI_OPS, GEN_SAMPLE_OPS, BWD_SAMPLE_OPS = 112.0, 120.0, 44.0, 150.0, 350.0
# plain (non-packed) FP32 vector issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def kernel_lane_ops_per_step(kernel: str, st: dict) -> float:
    if kernel == "trace_any":
        return (NODE_OPS * (st["shadow_nodes"] + st.get("sec_shadow_nodes", 0))
                + TRI_OPS * (st["shadow_tris"] + st.get("sec_shadow_tris", 0)))
    if kernel == "trace_closest":
        return NODE_OPS_CLOSEST * st["sec_nodes"] + TRI_OPS * st["sec_tris"]
    if kernel == "dir_gen":
        return GEN_SAMPLE_OPS * st["samples"]
    if kernel == "shade_bwd":
        return BWD_SAMPLE_OPS * st["unoccluded"]
    return float("nan")


def pmc_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc summary, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        from paper_2608_24109_amd.profiling import source_digest
        d = json.load(open(path))
        k = d["kernels"].get(kernel)
        if k is None or d.get("source_sha") != source_digest():
            return None
        return k["fetch_bytes"] + k["write_bytes"]
    except Exception:
        return None


def sq_lane_ops(kernel: str, workload: str):
    """VALU lane operations executed per launch of `kernel` (SQ_THREAD_CYCLES_VALU) from the
    committed SQ counter summary of the workload, if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", f"sq_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        from paper_2608_24109_amd.profiling import source_digest
        d = json.load(open(path))
        if d.get("source_sha") != source_digest():
            return None
        return d["kernels"][kernel]["SQ_THREAD_CYCLES_VALU"]
    except Exception:
        return None


def roofline_objects(workload: str, stats: dict, p) -> dict:
    """The roofline object of the dominant kernel and the per-kernel views beside it."""
    gk = stats["gpu_kernels"]
    dom = max(gk, key=lambda k: gk[k]["ms_per_step"])

    def rate(x, k):
        return x / gk[k]["launches_per_step"] / (gk[k]["avg_ms"] * 1e-3)

    ops_launch = kernel_lane_ops_per_step(dom, stats) / gk[dom]["launches_per_step"]
    ops_rate = rate(kernel_lane_ops_per_step(dom, stats), dom) / 1e12
    traffic = pmc_traffic(dom, workload)
    executed = sq_lane_ops(dom, workload)
    bytes_launch = kernel_bytes_per_step(dom, stats, p) / gk[dom]["launches_per_step"]
    ok = not math.isnan(ops_rate)
    out = {
        # the traversal is bound by VALU issue (its node and triangle bytes come from L2 and the
        # MALL), so the roofline is the ALU one: algorithmic lane operations per launch over the
        # launch time, against the non-packed FP32 vector issue rate of the chip
        "roofline": {"bound": "alu", "kernel": dom, "achieved": round(ops_rate, 3) if ok else None,
                     "peak": round(VALU_PEAK_T, 2), "unit": "T lane-ops/s",
                     "frac": round(ops_rate / VALU_PEAK_T, 4) if ok else None,
                     "traffic": None if traffic is None else round(traffic),
                     "algorithmic_lane_ops_per_launch": round(ops_launch) if ok else None,
                     "executed_lane_ops_per_launch": None if executed is None else round(executed),
                     "avg_launch_ms": round(gk[dom]["avg_ms"], 4)},
        # the same launches counted in the method's bytes (128 B per node visit, 48 B per triangle
        # test, the ray in and the answer out): served from L2 and the 256 MB MALL, so no HBM
        # peak applies to this rate
        "cache_bytes": {"kernel": dom, "bytes_per_launch": None if math.isnan(bytes_launch) else round(bytes_launch),
                        "GBps": None if math.isnan(bytes_launch) else
                        round(bytes_launch / (gk[dom]["avg_ms"] * 1e-3) / 1e9, 1)},
    }
    alu = {}
    for k in ("trace_any", "trace_closest", "dir_gen", "shade_bwd"):
        if k not in gk:
            continue
        o = rate(kernel_lane_ops_per_step(k, stats), k) / 1e12
        e = sq_lane_ops(k, workload)
        alu[k] = {"achieved": round(o, 3), "frac": round(o / VALU_PEAK_T, 4),
                  "algorithmic_lane_ops_per_launch": round(kernel_lane_ops_per_step(k, stats) / gk[k]["launches_per_step"]),
                  "executed_lane_ops_per_launch": None if e is None else round(e)}
    out["alu_rooflines"] = alu
    hbm = {}
    for k in gk:
        t = pmc_traffic(k, workload)
        if t is not None:
            g = t / (gk[k]["avg_ms"] * 1e-3) / 1e9
            hbm[k] = {"bytes_per_launch": round(t), "GBps": round(g, 1), "frac": round(g / HBM_PEAK_GBS, 4)}
    # HBM bytes measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE, calibrated on a copy) over each
    # kernel's launch time, against 8 TB/s; empty when the counters predate the kernel sources
    out["hbm_measured"] = hbm
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: the render pass would shard views across GPUs "
                                   "with one all-reduce of the gradient maps, which is not built; run --gpus 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if a.calib_copy_mb:
        src = torch.ones(a.calib_copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"{a.workload}: {a.warmup} warmup + {a.steps} timed steps")
    kern = None
    if a.workload == "tori32":
        sc, p, wall, stats = run_tori32(a.steps, a.warmup)
        desc = (f"tori32: {stats['tris']} tris, {stats['views']} views {stats['H']}x{stats['W']}, "
                f"{sc.tex.shape[0]}^2 maps, {sc.env.shape[0]}x{sc.env.shape[1]} env with gradients, N_d={p.N_d}, "
                f"N_b={p.N_b}, N_s={p.N_s}, G-buffer rasterised again in backward (autograd.Function), fwd+bwd")
    else:
        sc, p, wall, kern, stats, _ = run_gpu(a.workload, a.steps, a.warmup)
        desc = (f"{sc.name}: {stats['tris']} tris, {stats['views']} views {stats['H']}x{stats['W']}, "
                f"{sc.tex.shape[0]}^2 maps, {sc.env.shape[0]}x{sc.env.shape[1]} env, N_d={p.N_d}"
                + (f", N_b={p.N_b}, N_s={p.N_s}" if p.N_b else "") + ", fwd+bwd")
    ms_step = wall / a.steps * 1e3
    value = stats["pixels"] / (ms_step * 1e-3) / 1e6
    gk = stats["gpu_kernels"]
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpixels/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "global_batch": stats["views"], "seq_len": stats["H"] * stats["W"],
                   "parallelism": "none"},
        "covered_fraction": round(stats["covered"] / stats["pixels"], 4),
    }
    traced = "trace_any" in gk
    if traced:
        # shadow rays (direct, and the secondary light samples where the workload has them) per
        # second of the any-hit traversal kernel; indirect rays per second of the indirect pass's kernels
        n_any = stats["shadow_rays"] + stats.get("sec_shadow_rays", 0)
        out["shadow_Mrays_s_in_traversal"] = round(n_any / (gk["trace_any"]["ms_per_step"] * 1e-3) / 1e6, 1)
        out["nodes_per_shadow_ray"] = round(stats["shadow_nodes"] / max(stats["shadow_rays"], 1), 2)
        out["tris_per_shadow_ray"] = round(stats["shadow_tris"] / max(stats["shadow_rays"], 1), 2)
    if p.N_b > 0:
        ind = [k for k in gk if k in ("ind_gen1", "trace_closest", "ind_gen2", "ind_finalize")]
        t_ind = sum(gk[k]["ms_per_step"] for k in ind)
        # the secondary shadow rays' share of the any-hit traversal time, by their node visits
        nodes_all = stats["shadow_nodes"] + stats["sec_shadow_nodes"]
        t_ind += gk["trace_any"]["ms_per_step"] * stats["sec_shadow_nodes"] / max(nodes_all, 1)
        rays = stats["sec_rays"] + stats["sec_shadow_rays"]
        out["indirect_Mrays_s"] = round(rays / (t_ind * 1e-3) / 1e6, 1)
    if kern is not None:
        out["kernels_ms"] = {k: round(v, 4) for k, v in kern.items()}
    out.update(roofline_objects(a.workload, stats, p))
    out["gpu_kernels_ms"] = {k: round(v["avg_ms"], 4) for k, v in sorted(gk.items(), key=lambda kv: -kv[1]["ms_per_step"])}
    out["gpu_kernel_launches_per_step"] = {k: v["launches_per_step"] for k, v in gk.items()}
    out["gpu_kernels_ms_per_step"] = {k: round(v["ms_per_step"], 4) for k, v in gk.items()}
    if kern is not None:
        out["algorithmic_GBps"] = {k: round(algorithmic_bytes(k, stats, p) / (kern[k] * 1e-3) / 1e9, 1)
                                   for k in kern if not math.isnan(algorithmic_bytes(k, stats, p))}
    if a.extras:
        for name, steps in (("sphere", max(3, a.steps // 2)), ("tori", max(2, a.steps // 3)), ("small", 20)):
            if name == a.workload:
                continue
            log(f"{name}")
            sc2, p2, wall2, kern2, st2, _ = run_gpu(name, steps, 1 if name != "small" else 3)
            g2 = st2.pop("gpu_kernels")
            row = {"workload": f"{sc2.name}: {st2['tris']} tris, {st2['views']} views {st2['H']}x{st2['W']}, "
                               f"{sc2.tex.shape[0]}^2 maps, {sc2.env.shape[0]}x{sc2.env.shape[1]} env, N_d={p2.N_d}"
                               + (f", N_b={p2.N_b}, N_s={p2.N_s}" if p2.N_b else "") + ", fwd+bwd",
                   "fwd_bwd_Mpixels_s": round(st2["pixels"] / (wall2 / steps) / 1e6, 3),
                   "ms_per_step": round(wall2 / steps * 1e3, 3),
                   "kernels_ms": {k: round(v, 4) for k, v in kern2.items()},
                   "gpu_kernels_ms": {k: round(v["avg_ms"], 4) for k, v in
                                      sorted(g2.items(), key=lambda kv: -kv[1]["ms_per_step"])}}
            if "trace_any" in g2:
                row["direct_shadow_Mrays_s"] = round(st2["shadow_rays"] / (kern2["shade_fwd"] * 1e-3) / 1e6, 1)
            if p2.N_b > 0:
                row["indirect_Mrays_s"] = round((st2["sec_rays"] + st2["sec_shadow_rays"]) /
                                                (kern2["trace_indirect"] * 1e-3) / 1e6, 1)
            st2["gpu_kernels"] = g2
            row.update(roofline_objects(name, st2, p2))
            out[name] = row
        log("paper-shape relighting (1600^2, half-resolution indirect)")
        out["paper_shape_relight"] = run_paper_shape()
        log("Stage-II iterations (paper shape, 1600^2 training view)")
        out["stage2_iteration"] = run_stage2()
        log("Stage-I topology round (paper-size mesh)")
        out["topology_round"] = run_topology()
        log(f"relight service, {a.relight_seconds:g} s stream")
        out["relight"] = run_relight(a.relight_seconds, a.relight_rate, a.relight_budget_gib, a.relight_slots)
    if not a.no_cpu:
        log(f"oracle CPU baseline on {a.cpu_pixels} pixels of each of {a.cpu_views} views")
        out["cpu_baseline"] = cpu_baseline(sc, p, a.cpu_views, a.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
