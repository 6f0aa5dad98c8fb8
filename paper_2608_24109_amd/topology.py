"""Stage-I topology refinement over the C ABI (Vertex Splitting, Vertex Merging, UV Maintenance;
Eq. 1-6).

DeviceTopoMesh keeps a mesh being refined in device arrays with room for a round's growth:
`grad_ema` folds a position gradient into the per-vertex EMA of Eq. 1, `render_counts` counts the
pixels each face covers over a set of views (C_rend of the merging criterion, through the
library's rasteriser), and `round` runs one round of splits and merges with the UV updates, in
place. Every step is a call of libexm; torch only holds the buffers.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


@dataclass
class TopoConfig:
    beta_g: float = 0.95           # gradient EMA coefficient (hyperparameter table)
    w_g: float = 0.6               # split-score weights
    w_k: float = 0.4
    tau_degen: float = 0.05        # degeneracy threshold
    tau_uv: float = 0.5 / 2048.0   # seam threshold: half a texel of a 2048^2 map
    split_fraction: float = 0.05   # share of the faces selected per splitting round
    max_faces: int = 200_000
    split: bool = True
    merge: bool = True

    def c(self) -> L.exm_topo_params:
        flags = (0 if self.split else L.EXM_TOPO_NO_SPLIT) | (0 if self.merge else L.EXM_TOPO_NO_MERGE)
        return L.exm_topo_params(self.beta_g, self.w_g, self.w_k, self.tau_degen, self.tau_uv, self.split_fraction,
                                 self.max_faces, flags)

    def split_count(self, nF: int) -> int:
        if not self.split:
            return 0
        return max(0, min(int(np.floor(self.split_fraction * nF)), (self.max_faces - nF) // 2))


class DeviceTopoMesh:
    def __init__(self, pos, tri, uv, tri_uv, G=None, cfg: TopoConfig | None = None, device="cuda"):
        self.cfg = cfg or TopoConfig()
        self.device = device
        pos = np.ascontiguousarray(pos, np.float32)
        tri = np.ascontiguousarray(tri, np.int32)
        uv = np.ascontiguousarray(uv, np.float32)
        tri_uv = np.ascontiguousarray(tri_uv, np.int32)
        G = np.zeros(pos.shape[0], np.float32) if G is None else np.ascontiguousarray(G, np.float32)
        self.nV, self.nF, self.nUV = pos.shape[0], tri.shape[0], uv.shape[0]
        self._alloc(self.nV, self.nF, self.nUV)
        self.pos[:self.nV] = torch.from_numpy(pos).to(device)
        self.G[:self.nV] = torch.from_numpy(G).to(device)
        self.uv[:self.nUV] = torch.from_numpy(uv).to(device)
        self.tri[:self.nF] = torch.from_numpy(tri).to(device)
        self.tri_uv[:self.nF] = torch.from_numpy(tri_uv).to(device)
        self.ws = None

    def _alloc(self, nV: int, nF: int, nUV: int) -> None:
        K = self.cfg.split_count(nF)
        self.capV, self.capF, self.capUV = nV + K, nF + 2 * K, nUV + 2 * K
        d = self.device
        self.pos = torch.zeros((max(self.capV, 1), 3), dtype=torch.float32, device=d)
        self.G = torch.zeros(max(self.capV, 1), dtype=torch.float32, device=d)
        self.uv = torch.zeros((max(self.capUV, 1), 2), dtype=torch.float32, device=d)
        self.tri = torch.zeros((max(self.capF, 1), 3), dtype=torch.int32, device=d)
        self.tri_uv = torch.zeros((max(self.capF, 1), 3), dtype=torch.int32, device=d)

    def _grow(self) -> None:
        """Room for the next round's splits (the arrays are reallocated when they lack it)."""
        K = self.cfg.split_count(self.nF)
        if self.nV + K <= self.capV and self.nF + 2 * K <= self.capF and self.nUV + 2 * K <= self.capUV:
            return
        old = (self.pos, self.G, self.uv, self.tri, self.tri_uv)
        self._alloc(self.nV, self.nF, self.nUV)
        for dst, src, n in zip((self.pos, self.G, self.uv, self.tri, self.tri_uv), old,
                               (self.nV, self.nV, self.nUV, self.nF, self.nF)):
            dst[:n] = src[:n]

    def c(self) -> L.exm_topo_mesh:
        return L.exm_topo_mesh(self.nV, self.nF, self.nUV, self.capV, self.capF, self.capUV, self.pos.data_ptr(),
                               self.G.data_ptr(), self.uv.data_ptr(), self.tri.data_ptr(), self.tri_uv.data_ptr())

    def _workspace(self):
        n = L.exm_topology_workspace_size(self.nV, self.nF, self.nUV, self.cfg.c())
        if self.ws is None or self.ws.numel() < n:
            self.ws = None
            self.ws = L.workspace(n, self.device)
        return self.ws

    def grad_ema(self, grad: torch.Tensor, stream=None) -> None:
        """Eq. 1 with the position gradient grad [nV,3]."""
        L.exm_vertex_grad_ema(self.G[:self.nV], grad.contiguous(), self.cfg.beta_g, stream)

    def render_counts(self, cams, view_ids=None, stream=None) -> torch.Tensor:
        """C_rend: per face, the number of pixels where it is visible over `cams`."""
        vnrm = torch.empty((self.nV, 3), dtype=torch.float64, device=self.device)
        ftan = torch.empty((self.nF, 4), dtype=torch.float32, device=self.device)
        m = L.exm_mesh(self.nV, self.nF, self.nUV, self.pos.data_ptr(), self.tri.data_ptr(), self.uv.data_ptr(),
                       self.tri_uv.data_ptr(), vnrm.data_ptr(), ftan.data_ptr())
        L.exm_mesh_prepare(m, stream)
        counts = torch.zeros(self.nF, dtype=torch.int32, device=self.device)
        for k, cam in enumerate(cams):
            tri_id = torch.empty((1, cam.H, cam.W), dtype=torch.int32, device=self.device)
            bary = torch.empty((1, cam.H, cam.W, 2), dtype=torch.float32, device=self.device)
            L.exm_raster_gbuffer(m, L.cameras([cam], [k if view_ids is None else view_ids[k]]), tri_id, bary, stream)
            L.exm_face_render_counts(tri_id, self.nF, counts, stream)
        return counts

    def scores(self, stream=None) -> dict:
        """Per-face S_f, K_f, D_f and area (FP64 device tensors)."""
        out = {k: torch.empty(self.nF, dtype=torch.float64, device=self.device) for k in ("S", "K", "D", "area")}
        L.exm_topology_scores(self.c(), self.cfg.c(), out["S"], out["K"], out["D"], out["area"], self._workspace(),
                              stream)
        return out

    def round(self, c_rend: torch.Tensor | None = None, stream=None) -> dict:
        """One round of splitting then merging; returns its counts."""
        self._grow()
        m = self.c()
        st = L.exm_topology_round(m, c_rend, self.cfg.c(), self._workspace(), stream)
        self.nV, self.nF, self.nUV = int(m.nV), int(m.nF), int(m.nUV)
        return st

    def to_numpy(self):
        """(pos, G, uv, tri, tri_uv) of the current mesh on the host."""
        return (self.pos[:self.nV].cpu().numpy(), self.G[:self.nV].cpu().numpy(), self.uv[:self.nUV].cpu().numpy(),
                self.tri[:self.nF].cpu().numpy(), self.tri_uv[:self.nF].cpu().numpy())
