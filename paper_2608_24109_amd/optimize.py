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

The indirect-lighting variants of the ablation study are modes of the loop: "train" (the full
method), "eval_only" (trained direct only, the one-bounce term added when evaluating) and "off"
(direct only throughout); the No Secondary Material variant is the pass flag of that name.
initial_maps gives the Stage-II initialisation (base colour from the Stage-I RGB texture taken
from sRGB to linear, or grey for the grey-init variant; neutral roughness, normals and env map;
metallic zero). state_dict / load_state_dict save and resume the loop.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

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
    indirect: str = "train"        # "train" | "eval_only" | "off"

    def lambda_ind(self, t: int) -> float:
        return self.lambda_ind_max * min(1.0, t / max(1, self.ramp_iters))

    def lambda_chroma(self, t: int) -> float:
        return self.lambda_chroma0 * (1.0 - t / max(1, self.iters))


NEUTRAL_ROUGHNESS = 0.5
NEUTRAL_ENV = 0.5


def srgb_to_linear(c: np.ndarray) -> np.ndarray:
    """The inverse sRGB transfer curve (IEC 61966-2-1), on values in [0, 1]."""
    c = np.clip(np.asarray(c, np.float64), 0.0, 1.0)
    return np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)


def initial_maps(t_rgb: np.ndarray | None, Ht: int, Wt: int, He: int, We: int,
                 grey_base: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Stage-II initial parameters: the packed map [Ht,Wt,8] and the env map [He,We,3].
    Base colour = the Stage-I RGB texture [Ht,Wt,3] (sRGB) in linear RGB, or 0.5 grey when
    grey_base (or no texture) is given; roughness NEUTRAL_ROUGHNESS; metallic 0; tangent-space
    normal (0, 0, 1); env map constant NEUTRAL_ENV."""
    tex = np.zeros((Ht, Wt, 8), np.float32)
    if t_rgb is None or grey_base:
        tex[..., 0:3] = 0.5
    else:
        if tuple(t_rgb.shape) != (Ht, Wt, 3):
            raise ValueError(f"RGB texture must be [{Ht},{Wt},3], got {tuple(t_rgb.shape)}")
        tex[..., 0:3] = srgb_to_linear(t_rgb)
    tex[..., 3] = NEUTRAL_ROUGHNESS
    tex[..., 7] = 1.0
    return tex, np.full((He, We, 3), NEUTRAL_ENV, np.float32)


class Stage2:
    """Optimises `mat.tex` and `env.env` in place to reproduce `targets` [V,H,W,3] seen by
    `cams` (a list of camera objects with .mvp, .eye, .H, .W)."""

    def __init__(self, mesh: DeviceMesh, mat: DeviceMaterial, env: DeviceEnv, cams, targets: torch.Tensor,
                 cfg: Stage2Config):
        if cfg.indirect not in ("train", "eval_only", "off"):
            raise ValueError(f"indirect must be train, eval_only or off, got {cfg.indirect!r}")
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
        N_b_train = cfg.N_b if cfg.indirect == "train" else 0
        self.bufs = PassBuffers(1, H, W, N_b_train, device=dev, half=cfg.half_res_indirect and N_b_train > 0)
        self.eval_bufs = None
        self.rng = np.random.default_rng(cfg.view_seed)
        self.t = 0
        flags = cfg.flags | (0 if cfg.metallic else L.EXM_METALLIC_OFF)
        self.p = PassParams(N_d=cfg.N_d, N_b=N_b_train, N_s=cfg.N_s, seed=cfg.seed, tmin=cfg.tmin, flags=flags,
                            half_res_indirect=cfg.half_res_indirect)
        self.p_eval = PassParams(N_d=cfg.N_d, N_b=cfg.N_b if cfg.indirect != "off" else 0, N_s=cfg.N_s,
                                 seed=cfg.seed, tmin=cfg.tmin, flags=flags, half_res_indirect=cfg.half_res_indirect)
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

    def evaluate(self, view: int, iteration: int = 0) -> torch.Tensor:
        """The image of one view as the ablation variant evaluates it: L_dir + L_ind for "train"
        and "eval_only", L_dir for "off" (a fresh tensor [1,H,W,3])."""
        H, W = self.cams[0].H, self.cams[0].W
        if self.eval_bufs is None:
            pe = self.p_eval
            self.eval_bufs = PassBuffers(1, H, W, pe.N_b, device=self.mat.tex.device,
                                         half=pe.half_res_indirect and pe.N_b > 0)
        self.p_eval.iteration = iteration
        cc = L.cameras([self.cams[view]], [view])
        render_forward(self.mesh, self.mat, self.env, cc, self.p_eval, self.eval_bufs)
        img = self.eval_bufs.L_dir.clone()
        if self.p_eval.N_b > 0:
            img += self.eval_bufs.L_ind
        return img

    def state_dict(self) -> dict:
        """Everything the loop needs to resume: parameters, Adam moments, step count and the
        view sampler's state (host copies)."""
        return {"tex": self.mat.tex.cpu(), "env": self.env.env.cpu(), "m_tex": self.m_tex.cpu(),
                "v_tex": self.v_tex.cpu(), "m_env": self.m_env.cpu(), "v_env": self.v_env.cpu(), "t": self.t,
                "rng": self.rng.bit_generator.state}

    def load_state_dict(self, st: dict) -> None:
        for name, dst in (("tex", self.mat.tex), ("env", self.env.env), ("m_tex", self.m_tex), ("v_tex", self.v_tex),
                          ("m_env", self.m_env), ("v_env", self.v_env)):
            if tuple(st[name].shape) != tuple(dst.shape):
                raise ValueError(f"{name}: shape {tuple(st[name].shape)} != {tuple(dst.shape)}")
            dst.copy_(st[name])
        self.t = int(st["t"])
        self.rng.bit_generator.state = st["rng"]
        self.env.update()

    def step(self) -> int:
        """One iteration; returns the view it used. The loss accumulates in self.loss."""
        cfg, t = self.cfg, self.t
        view = int(self.rng.integers(len(self.cams)))
        lam = cfg.lambda_ind(t)
        img, cc = self.render(view, lam, iteration=t)
        self.dtex.zero_()
        self.denv.zero_()
        L.exm_image_loss(img.contiguous(), self.targets[view:view + 1], 1.0, self.loss, self.dI, self.ws_img)
        # material TV on the screen projection of the maps; its gradient joins the direct pass's
        # map adjoint (one scatter into the maps)
        L.exm_project_maps(self.mesh.s, self.mat.s, self.bufs.tri_id, self.bufs.bary, self.P)
        L.exm_tv_screen(self.P, self.bufs.tri_id, cfg.metallic, cfg.lambda_mat, self.loss, self.dP)
        # adjoint of the render pass
        render_backward(self.mesh, self.mat, self.env, cc, self.p, self.bufs, self.dI, lam, self.dtex, self.denv,
                        dquery=self.dP)
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
