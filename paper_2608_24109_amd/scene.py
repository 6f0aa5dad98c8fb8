"""Device-resident asset: the fixed mesh-UV carrier, its BVH, the packed material maps and the
environment map with its sampling tables, kept alive behind the C-ABI structs.

All arithmetic happens in libexm.so; this module only allocates device tensors and fills
the structs the ABI takes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


class DeviceMesh:
    """Mesh arrays on the device plus prepared vertex normals and face tangents."""

    def __init__(self, pos: np.ndarray, tri: np.ndarray, uv: np.ndarray, tri_uv: np.ndarray, device="cuda",
                 stream=None, with_bvh: bool = True):
        self.pos_host = np.ascontiguousarray(pos, dtype=np.float32)
        self.tri_host = np.ascontiguousarray(tri, dtype=np.int32)
        self.pos = torch.from_numpy(self.pos_host).to(device)
        self.tri = torch.from_numpy(self.tri_host).to(device)
        self.uv = torch.from_numpy(np.ascontiguousarray(uv, dtype=np.float32)).to(device)
        self.tri_uv = torch.from_numpy(np.ascontiguousarray(tri_uv, dtype=np.int32)).to(device)
        self.vnrm = torch.empty((self.pos.shape[0], 3), dtype=torch.float64, device=device)
        self.ftan = torch.empty((self.tri.shape[0], 4), dtype=torch.float32, device=device)
        self.s = L.exm_mesh(self.pos.shape[0], self.tri.shape[0], self.uv.shape[0], self.pos.data_ptr(),
                            self.tri.data_ptr(), self.uv.data_ptr(), self.tri_uv.data_ptr(), self.vnrm.data_ptr(),
                            self.ftan.data_ptr())
        L.exm_mesh_prepare(self.s, stream)
        self.bvh = L.exm_build_bvh(self.pos_host, self.tri_host, stream) if with_bvh else None

    @property
    def nF(self) -> int:
        return int(self.tri.shape[0])

    def device_bytes(self) -> int:
        t = sum(x.numel() * x.element_size() for x in (self.pos, self.tri, self.uv, self.tri_uv, self.vnrm, self.ftan))
        return t + (self.bvh.device_bytes if self.bvh else 0)


class DeviceMaterial:
    def __init__(self, tex, device="cuda"):
        self.tex = tex if isinstance(tex, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(tex, np.float32))
        self.tex = self.tex.to(device).contiguous()
        self.s = L.exm_material(self.tex.shape[0], self.tex.shape[1], self.tex.data_ptr())

    def device_bytes(self) -> int:
        return self.tex.numel() * 4


class DeviceEnv:
    """Environment map with its importance-sampling tables (rebuilt by `update`)."""

    def __init__(self, env, device="cuda", stream=None):
        env = env if isinstance(env, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(env, np.float32))
        self.env = env.to(device).contiguous()
        He, We = self.env.shape[:2]
        self.cdf_row = torch.empty(He, dtype=torch.uint64, device=device)
        self.cdf_col = torch.empty((He, We), dtype=torch.uint64, device=device)
        self.pdf = torch.empty((He, We), dtype=torch.float32, device=device)
        self.guide = torch.empty(L.exm_env_guide_len(He, We), dtype=torch.int32, device=device)
        self.rec = torch.empty((He, We, 4), dtype=torch.float32, device=device)
        self.s = L.exm_env(He, We, self.env.data_ptr(), self.cdf_row.data_ptr(), self.cdf_col.data_ptr(),
                           self.pdf.data_ptr(), self.guide.data_ptr(), self.rec.data_ptr())
        self.update(stream=stream)

    def update(self, env: torch.Tensor | None = None, stream=None) -> None:
        """Copy in a new map (same shape) if given, then rebuild the tables."""
        if env is not None:
            self.env.copy_(env)
        L.exm_build_env_sampler(self.env, self.cdf_row, self.cdf_col, self.pdf, self.guide, self.rec, stream)

    def device_bytes(self) -> int:
        return sum(x.numel() * x.element_size()
                   for x in (self.env, self.cdf_row, self.cdf_col, self.pdf, self.guide, self.rec))
