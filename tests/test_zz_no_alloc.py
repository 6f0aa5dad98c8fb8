"""exm_shade_fwd_noalloc (the direct pass in the library's own 64 MiB device scratch, for callers
that cannot allocate) against exm_shade_fwd with a caller workspace: the same L_dir and visibility
bits, bit for bit, on two calls in a row, the second smaller than the first (the scratch keeps the
first call's contents)."""
import sys

import numpy as np
import pytest
import torch

from paper_2608_24109_amd import inputs as I

pytestmark = pytest.mark.gpu


def _direct_both_ways(sc, nviews):
    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd.render import PassBuffers, PassParams, raster, shade_fwd_ws_bytes
    from paper_2608_24109_amd.scene import DeviceEnv, DeviceMaterial, DeviceMesh
    mesh = DeviceMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    mat = DeviceMaterial(sc.tex)
    env = DeviceEnv(sc.env)
    p = PassParams(N_d=sc.N_d, seed=sc.seed, tmin=sc.tmin)
    cams = sc.cams[:nviews]
    cc = L.cameras(cams, list(range(nviews)))
    H, W = cams[0].H, cams[0].W
    b = PassBuffers(nviews, H, W, 0)
    raster(mesh, cc, b)
    ws = L.workspace(shade_fwd_ws_bytes(nviews, H, W, p))
    L.exm_shade_fwd(mesh.s, mesh.bvh, mat.s, env.s, cc, b.tri_id, b.bary, p.c(), b.L_dir, b.vis, ws)
    L_na = torch.full_like(b.L_dir, float("nan"))
    vis_na = torch.zeros_like(b.vis)
    L.exm_shade_fwd_noalloc(mesh.s, mesh.bvh, mat.s, env.s, cc, b.tri_id, b.bary, p.c(), L_na, vis_na)
    torch.cuda.synchronize()
    return b, L_na, vis_na


def test_shade_fwd_noalloc_equals_workspace_call():
    # 1) the displaced sphere, 2 views of 512^2 at N_d 64: 524,288 pixels in about 15 chunks of the scratch
    sc = I.config("sphere", views=2, res=512)
    print("[noalloc] sphere 2 x 512^2, N_d 64", flush=True)
    b, L_na, vis_na = _direct_both_ways(sc, 2)
    assert torch.equal(b.vis, vis_na) and torch.equal(b.L_dir, L_na)
    assert int((b.tri_id >= 0).sum()) > 100_000 and float(b.L_dir.abs().max()) > 0
    # 2) smaller: the icosphere, one 128^2 view at N_d 16 (one chunk; the scratch holds leftovers of 1)
    sc = I.config("small")
    print("[noalloc] icosphere 1 x 128^2, N_d 16", flush=True)
    b, L_na, vis_na = _direct_both_ways(sc, 1)
    assert torch.equal(b.vis, vis_na) and torch.equal(b.L_dir, L_na)
    assert int((b.tri_id >= 0).sum()) > 1000
