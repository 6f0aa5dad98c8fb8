"""The Stage-II render pass over the C ABI, and its autograd form.

render_forward:  env tables -> G-buffer -> direct (Eq. 17) -> indirect (Eq. 18-19)
render_backward: adjoints of the direct and indirect passes into the maps and the env map
RenderPBR:       torch.autograd.Function; I = L_dir + lambda_ind * L_ind (Eq. 20); with
                 checkpoint=True the G-buffer is not kept between forward and backward but
                 rasterised again in backward (only the visibility bits and secondary-hit
                 records are stored).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _lib as L
from .scene import DeviceEnv, DeviceMaterial, DeviceMesh


@dataclass
class PassParams:
    N_d: int = 8          # direct env samples (hyperparameter table default)
    N_b: int = 0          # secondary rays (0: direct only)
    N_s: int = 4          # light samples per secondary hit
    seed: int = 3
    iteration: int = 0
    tmin: float = 0.0
    flags: int = 0
    f_diel: float = 0.04  # F_dielectric of Eq. 16
    eps: float = 1e-6     # epsilon of Eq. 15
    half_res_indirect: bool = False  # indirect pass at half resolution, upsampled (Implementation Details)

    def c(self) -> L.exm_params:
        return L.params(self.N_d, self.N_b, self.N_s if self.N_b > 0 else 0, self.seed, self.iteration,
                        self.f_diel, self.eps, self.tmin, self.flags)


# Upper bound of the ray workspace a pass allocates; larger passes run in pixel chunks. 24 GiB
# holds the direct pass of 8 views of 1024^2 at N_d = 64 in one chunk (one traversal launch per
# pass, so one tail), a small share of the 288 GB of HBM.
WORKSPACE_CAP = 24 << 30


class PassBuffers:
    """Per-view outputs of one forward pass (device tensors) and its ray workspace."""

    def __init__(self, n: int, H: int, W: int, N_b: int, device="cuda", gbuffer: bool = True,
                 ws_cap: int = WORKSPACE_CAP, half: bool = False):
        self.n, self.H, self.W, self.N_b = n, H, W, N_b
        self.device = device
        self.ws = None
        self.ws_cap = ws_cap
        self.tri_id = torch.empty((n, H, W), dtype=torch.int32, device=device) if gbuffer else None
        self.bary = torch.empty((n, H, W, 2), dtype=torch.float32, device=device) if gbuffer else None
        self.L_dir = torch.empty((n, H, W, 3), dtype=torch.float32, device=device)
        self.vis = torch.empty((n, H, W), dtype=torch.uint64, device=device)
        self.L_ind = torch.empty((n, H, W, 3), dtype=torch.float32, device=device) if N_b > 0 else None
        self.sec_rec = None
        self.sec_vis = None
        self.half = None  # buffers of a half-resolution indirect pass
        if N_b > 0 and half:
            self.half = PassBuffers(n, (H + 1) // 2, (W + 1) // 2, N_b, device=device, ws_cap=ws_cap)
        elif N_b > 0:
            self.sec_rec = torch.empty((n, H, W, max(N_b, 1), 3), dtype=torch.int32, device=device)
            self.sec_vis = torch.empty((n, H, W), dtype=torch.uint64, device=device)

    def workspace(self, nbytes: int):
        """The pass's ray workspace, grown to `nbytes` (capped at ws_cap) when needed."""
        nbytes = min(int(nbytes), self.ws_cap)
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            self.ws = L.workspace(nbytes, self.device)
        return self.ws

    def ensure_gbuffer(self, device="cuda"):
        if self.tri_id is None:
            self.tri_id = torch.empty((self.n, self.H, self.W), dtype=torch.int32, device=device)
            self.bary = torch.empty((self.n, self.H, self.W, 2), dtype=torch.float32, device=device)

    def drop_gbuffer(self):
        self.tri_id = None
        self.bary = None
        if self.half is not None:
            self.half.drop_gbuffer()


def half_cameras(cams_c):
    """The same cameras at half resolution in both image dimensions (rounded up)."""
    out = (L.exm_camera * len(cams_c))()
    for i, c in enumerate(cams_c):
        out[i] = c
        out[i].H, out[i].W = (c.H + 1) // 2, (c.W + 1) // 2
    return out


def shade_fwd_ws_bytes(n: int, H: int, W: int, p: PassParams) -> int:
    """Workspace the direct pass asks for: whole views at once, or its minimum."""
    return max(L.exm_shade_fwd_workspace_size(n, H, W, p.N_d), L.exm_shade_fwd_workspace_min(p.N_d))


def trace_indirect_ws_bytes(n: int, H: int, W: int, p: PassParams) -> int:
    return max(L.exm_trace_indirect_workspace_size(n, H, W, p.N_b, p.N_s),
               L.exm_trace_indirect_workspace_min(p.N_b, p.N_s))


def raster(mesh: DeviceMesh, cams_c, bufs: PassBuffers, stream=None) -> None:
    bufs.ensure_gbuffer()
    L.exm_raster_gbuffer(mesh.s, cams_c, bufs.tri_id, bufs.bary, stream)


def render_forward(mesh: DeviceMesh, mat: DeviceMaterial, env: DeviceEnv, cams_c, p: PassParams,
                   bufs: PassBuffers, stream=None, rebuild_tables: bool = True, do_raster: bool = True) -> None:
    pc = p.c()
    if rebuild_tables:
        env.update(stream=stream)
    if do_raster:
        raster(mesh, cams_c, bufs, stream)
    ws = bufs.workspace(shade_fwd_ws_bytes(len(cams_c), bufs.H, bufs.W, p))
    L.exm_shade_fwd(mesh.s, mesh.bvh, mat.s, env.s, cams_c, bufs.tri_id, bufs.bary, pc, bufs.L_dir, bufs.vis, ws,
                    stream)
    if p.N_b > 0 and bufs.half is not None:  # half-resolution indirect, upsampled
        hb = bufs.half
        ch = half_cameras(cams_c)
        raster(mesh, ch, hb, stream)
        ws = bufs.workspace(trace_indirect_ws_bytes(len(cams_c), hb.H, hb.W, p))
        L.exm_trace_indirect(mesh.s, mesh.bvh, mat.s, env.s, ch, hb.tri_id, hb.bary, pc, hb.L_ind, hb.sec_rec,
                             hb.sec_vis, ws, stream)
        L.exm_upsample_indirect(hb.tri_id, hb.L_ind, bufs.tri_id, bufs.L_ind, stream)
    elif p.N_b > 0:
        ws = bufs.workspace(trace_indirect_ws_bytes(len(cams_c), bufs.H, bufs.W, p))
        L.exm_trace_indirect(mesh.s, mesh.bvh, mat.s, env.s, cams_c, bufs.tri_id, bufs.bary, pc, bufs.L_ind,
                             bufs.sec_rec, bufs.sec_vis, ws, stream)


def shade_bwd_ws_bytes(n: int, H: int, W: int, p: PassParams, He: int, We: int) -> int:
    return max(L.exm_shade_bwd_workspace_size(n, H, W, p.N_d, He, We), L.exm_shade_bwd_workspace_min(p.N_d, He, We))


def trace_bwd_ws_bytes(n: int, H: int, W: int, p: PassParams, He: int, We: int) -> int:
    return max(L.exm_trace_bwd_workspace_size(n, H, W, p.N_b, p.N_s, He, We),
               L.exm_trace_bwd_workspace_min(p.N_b, p.N_s, He, We))


def render_backward(mesh: DeviceMesh, mat: DeviceMaterial, env: DeviceEnv, cams_c, p: PassParams,
                    bufs: PassBuffers, dI: torch.Tensor, lambda_ind: float, dtex: torch.Tensor,
                    denv: torch.Tensor, stream=None, dquery: torch.Tensor | None = None) -> None:
    """Adjoints of the direct and indirect passes into dtex and denv (+=). dquery [n,H,W,8], if
    given, is a gradient with respect to the queried map values at the visible pixels, scattered
    with the direct pass's map adjoint."""
    pc = p.c()
    He, We = env.env.shape[:2]
    ws = bufs.workspace(shade_bwd_ws_bytes(len(cams_c), bufs.H, bufs.W, p, He, We))
    L.exm_shade_bwd(mesh.s, mat.s, env.s, cams_c, bufs.tri_id, bufs.bary, pc, dI, bufs.vis, dtex, denv, ws, stream,
                    dquery=dquery)
    if p.N_b > 0 and lambda_ind != 0.0 and bufs.half is not None:
        hb = bufs.half
        ch = half_cameras(cams_c)
        if hb.tri_id is None:
            raster(mesh, ch, hb, stream)
        dLh = torch.empty((hb.n, hb.H, hb.W, 3), dtype=torch.float32, device=dI.device)
        L.exm_upsample_indirect_bwd(hb.tri_id, bufs.tri_id, lambda_ind, dI, dLh, stream)
        ws = bufs.workspace(trace_bwd_ws_bytes(len(cams_c), hb.H, hb.W, p, He, We))
        L.exm_trace_bwd(mesh.s, mat.s, env.s, ch, hb.tri_id, hb.bary, pc, 1.0, dLh, hb.sec_rec, hb.sec_vis, dtex,
                        denv, ws, stream)
    elif p.N_b > 0 and lambda_ind != 0.0:
        ws = bufs.workspace(trace_bwd_ws_bytes(len(cams_c), bufs.H, bufs.W, p, He, We))
        L.exm_trace_bwd(mesh.s, mat.s, env.s, cams_c, bufs.tri_id, bufs.bary, pc, lambda_ind, dI, bufs.sec_rec,
                        bufs.sec_vis, dtex, denv, ws, stream)


def _forward_chunks(tex_device, mesh, mat, env_dev, cams, p: PassParams, lambda_ind: float, chunk: int,
                    keep: bool, checkpoint: bool):
    """Renders `cams` in chunks of `chunk` views into one [V,H,W,3] image. With keep=True the
    per-chunk records the adjoint needs are returned (G-buffer dropped if checkpoint)."""
    H, W = cams[0].H, cams[0].W
    out = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device=tex_device)
    chunks = []
    for v0 in range(0, len(cams), chunk):
        cs = cams[v0:v0 + chunk]
        cc = L.cameras(cs, [getattr(c, "view_id", v0 + i) for i, c in enumerate(cs)])
        bufs = PassBuffers(len(cs), H, W, p.N_b, device=tex_device, half=p.half_res_indirect)
        render_forward(mesh, mat, env_dev, cc, p, bufs, rebuild_tables=False)
        o = out[v0:v0 + len(cs)]
        if p.N_b > 0:
            torch.add(bufs.L_dir, bufs.L_ind, alpha=lambda_ind, out=o)
        else:
            o.copy_(bufs.L_dir)
        if keep:
            bufs.L_dir = bufs.L_ind = None
            bufs.ws = None
            if bufs.half is not None:
                bufs.half.L_dir = bufs.half.L_ind = bufs.half.vis = None
            if checkpoint:
                bufs.drop_gbuffer()
            chunks.append((cc, bufs))
    return out, chunks


def render_image(mesh: DeviceMesh, mat: DeviceMaterial, env_dev: DeviceEnv, cams, p: PassParams,
                 lambda_ind: float = 1.0, chunk: int = 8, rebuild_tables: bool = True) -> torch.Tensor:
    """I = L_dir + lambda_ind L_ind (Eq. 20) for `cams`, keeping nothing for a backward pass."""
    if rebuild_tables:
        env_dev.update()
    out, _ = _forward_chunks(mat.tex.device, mesh, mat, env_dev, cams, p, lambda_ind, chunk, False, False)
    return out


class RenderPBR(torch.autograd.Function):
    """I = L_dir + lambda_ind L_ind for the views `cams`, differentiable w.r.t. the packed
    material map `tex` [Ht,Wt,8] and the env map `env` [He,We,3].

    The maps passed in must be the tensors that `mat` and `env_dev` point to (the kernels read
    them through the device structs). Views are processed in chunks of `chunk` views; with
    checkpoint=True each chunk's G-buffer is freed after the forward and rasterised again in
    backward. The env gradient is accumulated in FP64 and returned in FP32 (the FP64 sum stays
    on ctx.denv64).
    """

    @staticmethod
    def forward(ctx, tex, env, mesh, mat, env_dev, cams, p: PassParams, lambda_ind: float = 1.0,
                checkpoint: bool = False, chunk: int = 8, rebuild_tables: bool = True):
        if tex.data_ptr() != mat.tex.data_ptr() or env.data_ptr() != env_dev.env.data_ptr():
            raise ValueError("tex/env must be the tensors bound to the device material/env")
        if rebuild_tables:
            env_dev.update()
        out, chunks = _forward_chunks(tex.device, mesh, mat, env_dev, cams, p, lambda_ind, chunk, True, checkpoint)
        ctx.state = (mesh, mat, env_dev, chunks, p, lambda_ind, chunk)
        return out

    @staticmethod
    def backward(ctx, dI):
        mesh, mat, env_dev, chunks, p, lambda_ind, chunk = ctx.state
        dI = dI.contiguous().float()
        dtex = torch.zeros_like(mat.tex)
        denv = torch.zeros(env_dev.env.shape, dtype=torch.float64, device=dI.device)
        for k, (cc, bufs) in enumerate(chunks):
            if bufs.tri_id is None:
                raster(mesh, cc, bufs)
            g = dI[k * chunk:k * chunk + bufs.n]
            render_backward(mesh, mat, env_dev, cc, p, bufs, g, lambda_ind, dtex, denv)
            bufs.drop_gbuffer()
            bufs.ws = None
        ctx.state = None
        ctx.denv64 = denv
        return dtex, denv.to(torch.float32), None, None, None, None, None, None, None, None, None
