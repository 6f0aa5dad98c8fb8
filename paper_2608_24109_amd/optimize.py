"""Stage-II optimisation around the render pass (Stage-II Optimization; Implementation Details).

Each iteration renders one training view with the current maps and env map
(I = L_dir + lambda_ind(t) L_ind, Eq. 20, lambda_ind ramped linearly from 0 to its target over
the first `ramp_iters` iterations), evaluates the objective of Eq. 21-24 on the device
(L_img, lambda_mat TV of the screen-projected maps, lambda_env TV(E), lambda_chroma(t) chroma
with lambda_chroma(t) = lambda_0 (1 - t / T)), pulls its gradient back through the hand-written
adjoints into the packed map and the env map, and takes one Adam step per parameter at the
learning rates of the hyperparameter table. The optimiser step clamps the maps to their ranges
and E to [0, inf) (the non-negative parameterisation of the env map, read as a projection).
Every step is a call of libexm; torch only holds the buffers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .render import PassBuffers, PassParams, render_backward, render_forward
from .scene import DeviceEnv, DeviceMaterial, DeviceMesh

# channel ranges of the packed map (a.rgb, r, m, n.xyz); the normal map is left free (the
# shading normalises it)
TEX_LO = (0.0, 0.0, 0.0, 0.02, 0.0, -math.inf, -math.inf, -math.inf)
TEX_HI = (1.0, 1.0, 1.0, 1.0, 1.0, math.inf, math.inf, math.inf)


@dataclass
class Stage2Config:
    iters: int = 10_000
    lr_tex: float = 2.5e-3         # texture/material learning rate
    lr_env: float = 1.5e-2         # environment learning rate
    lambda_mat: float = 0.1
    lambda_env: float = 0.1
    lambda_chroma0: float = 0.1
    lambda_ind_max: float = 1.0
    ramp_iters: int = 1_000
    metallic: bool = False         # optimise the metallic map (else m = 0, dielectric)
    N_d: int = 8
    N_b: int = 16
    N_s: int = 4
    half_res_indirect: bool = True
    seed: int = 3
    tmin: float = 0.0
    flags: int = 0
    view_seed: int = 0

    def lambda_ind(self, t: int) -> float:
        return self.lambda_ind_max * min(1.0, t / max(1, self.ramp_iters))

    def lambda_chroma(self, t: int) -> float:
        return self.lambda_chroma0 * (1.0 - t / max(1, self.iters))


class Stage2:
    """Optimises `mat.tex` and `env.env` in place to reproduce `targets` [V,H,W,3] seen by
    `cams` (a list of camera objects with .mvp, .eye, .H, .W)."""

    def __init__(self, mesh: DeviceMesh, mat: DeviceMaterial, env: DeviceEnv, cams, targets: torch.Tensor,
                 cfg: Stage2Config):
        self.mesh, self.mat, self.env, self.cams, self.cfg = mesh, mat, env, cams, cfg
        self.targets = targets.contiguous()
        H, W = cams[0].H, cams[0].W
        dev = mat.tex.device
        self.m_tex = torch.zeros_like(mat.tex)
        self.v_tex = torch.zeros_like(mat.tex)
        self.m_env = torch.zeros_like(env.env)
        self.v_env = torch.zeros_like(env.env)
        self.dtex = torch.zeros_like(mat.tex)
        self.denv = torch.zeros(env.env.shape, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.acc3 = torch.zeros(3, dtype=torch.float64, device=dev)
        self.dI = torch.empty((1, H, W, 3), dtype=torch.float32, device=dev)
        self.P = torch.empty((1, H, W, 8), dtype=torch.float32, device=dev)
        self.dP = torch.empty_like(self.P)
        self.ws_img = L.workspace(L.exm_image_loss_workspace_size(H, W), dev)
        self.bufs = PassBuffers(1, H, W, cfg.N_b, device=dev, half=cfg.half_res_indirect and cfg.N_b > 0)
        self.rng = np.random.default_rng(cfg.view_seed)
        self.t = 0
        flags = cfg.flags | (0 if cfg.metallic else L.EXM_METALLIC_OFF)
        self.p = PassParams(N_d=cfg.N_d, N_b=cfg.N_b, N_s=cfg.N_s, seed=cfg.seed, tmin=cfg.tmin, flags=flags,
                            half_res_indirect=cfg.half_res_indirect)
        self.env_lo = (0.0, 0.0, 0.0)
        self.env_hi = (math.inf, math.inf, math.inf)

    def render(self, view: int, lam: float, iteration: int = 0) -> torch.Tensor:
        """I = L_dir + lam * L_ind of one view (the buffers stay for the adjoint)."""
        self.p.iteration = iteration
        cc = L.cameras([self.cams[view]], [view])
        render_forward(self.mesh, self.mat, self.env, cc, self.p, self.bufs)
        img = self.bufs.L_dir
        if self.p.N_b > 0 and lam != 0.0:
            img = img + lam * self.bufs.L_ind
        return img, cc

    def step(self) -> int:
        """One iteration; returns the view it used. The loss accumulates in self.loss."""
        cfg, t = self.cfg, self.t
        view = int(self.rng.integers(len(self.cams)))
        lam = cfg.lambda_ind(t)
        img, cc = self.render(view, lam, iteration=t)
        self.dtex.zero_()
        self.denv.zero_()
        L.exm_image_loss(img.contiguous(), self.targets[view:view + 1], 1.0, self.loss, self.dI, self.ws_img)
        # material TV on the screen projection of the maps
        L.exm_project_maps(self.mesh.s, self.mat.s, self.bufs.tri_id, self.bufs.bary, self.P)
        L.exm_tv_screen(self.P, self.bufs.tri_id, cfg.metallic, cfg.lambda_mat, self.loss, self.dP)
        L.exm_project_maps_bwd(self.mesh.s, self.mat.s, self.bufs.tri_id, self.bufs.bary, self.dP, self.dtex)
        # adjoint of the render pass
        render_backward(self.mesh, self.mat, self.env, cc, self.p, self.bufs, self.dI, lam, self.dtex, self.denv)
        # env regularisers
        L.exm_env_regularizers(self.env.env, cfg.lambda_env, cfg.lambda_chroma(t), self.loss, self.denv, self.acc3)
        # optimiser
        L.exm_adam_step(self.mat.tex, self.dtex, self.m_tex, self.v_tex, TEX_LO, TEX_HI, cfg.lr_tex, t + 1)
        L.exm_adam_step(self.env.env, self.denv, self.m_env, self.v_env, self.env_lo, self.env_hi, cfg.lr_env, t + 1)
        self.t += 1
        return view

    def run(self, iters: int) -> list[float]:
        """`iters` iterations; returns the mean objective of each block of 10 iterations."""
        out = []
        for k in range(iters):
            if k % 10 == 0:
                self.loss.zero_()
            self.step()
            if k % 10 == 9:
                out.append(float(self.loss.item()) / 10.0)
        return out
