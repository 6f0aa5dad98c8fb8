"""Half-resolution indirect light (Implementation Details: secondary rays at half resolution in
both image dimensions, indirect component upsampled), against the oracle:

- the upsampling map and its transpose on random inputs and coverage, even and ragged sizes,
  within FP32 rounding of the FP64 definition in oracle/;
- the half-resolution indirect pass on the concave small-tori scene under the same bars as the
  full-resolution one, and the full-resolution L_ind equal to the oracle's upsampling of it;
- the gradient through the upsampled indirect term (adjoint of the upsampling, then the
  indirect adjoint on the half-resolution buffers) against the oracle's forward-mode
  derivative composed with the upsampling, along random directions over all texels and env
  texels, with the upstream gradient zeroed on pixels fed by a flipped decision."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2608_24109_amd import inputs as I

from test_gpu_parity import Dev, _compare_view, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tori():
    log("[setup] small tori 2 x 96^2 (indirect at 48^2)")
    pos, tri = I.interlocking_tori(48, 20)
    cams = I.ring_cameras(2, 4.5, 96, 96)
    return Dev(I.make_scene("small_tori", pos, tri, 128, 128, 32, 64, 1.0, cams, N_d=16, N_b=4, N_s=4))


@pytest.mark.parametrize("H,W,Hh,Wh", [(64, 96, 32, 48), (37, 53, 19, 27)])
def test_upsample_and_transpose_match_oracle(H, W, Hh, Wh):
    from paper_2608_24109_amd import _lib as L
    rng = np.random.default_rng(H)
    n = 2
    th = np.where(rng.random((n, Hh, Wh)) < 0.8, 1, -1).astype(np.int32)
    tf = np.where(rng.random((n, H, W)) < 0.9, 1, -1).astype(np.int32)
    Lh = rng.random((n, Hh, Wh, 3)).astype(np.float32)
    G = rng.normal(size=(n, H, W, 3)).astype(np.float32)
    d_th, d_tf = torch.from_numpy(th).cuda(), torch.from_numpy(tf).cuda()
    out = torch.empty((n, H, W, 3), dtype=torch.float32, device="cuda")
    L.exm_upsample_indirect(d_th, torch.from_numpy(Lh).cuda(), d_tf, out)
    dLh = torch.empty((n, Hh, Wh, 3), dtype=torch.float32, device="cuda")
    L.exm_upsample_indirect_bwd(d_th, d_tf, 0.7, torch.from_numpy(G).cuda(), dLh)
    torch.cuda.synchronize()
    for v in range(n):
        ref = O.upsample_indirect(Lh[v], th[v], tf[v])
        assert np.allclose(out[v].cpu().numpy(), ref, rtol=1e-6, atol=1e-7)
        refT = O.upsample_indirect_T(0.7 * G[v].astype(np.float64), th[v], tf[v])
        assert np.allclose(dLh[v].cpu().numpy(), refT, rtol=1e-5, atol=1e-6 * np.abs(refT).max())


def _forward_half(dev, p):
    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd.render import PassBuffers, render_forward
    cams = dev.sc.cams
    cc = L.cameras(cams, list(range(len(cams))))
    b = PassBuffers(len(cams), cams[0].H, cams[0].W, p.N_b, half=True)
    render_forward(dev.mesh, dev.mat, dev.env, cc, p, b)
    torch.cuda.synchronize()
    return cc, b


def _half_cam(cam):
    return I.Camera(mvp=cam.mvp, eye=cam.eye, H=(cam.H + 1) // 2, W=(cam.W + 1) // 2)


def test_half_res_indirect_parity(tori):
    """The half-resolution indirect pass is the indirect pass of the same cameras at half
    resolution (bitwise), that pass meets the oracle bars, and the full-resolution L_ind is the
    oracle's upsampling of it."""
    p = tori.params()
    p.half_res_indirect = True
    _, b = _forward_half(tori, p)
    hb = b.half
    assert (hb.L_ind.cpu().numpy() > 0).mean() > 0.05
    hcams = [_half_cam(c) for c in tori.sc.cams]
    p0 = tori.params()
    _, ref = tori.forward(hcams, p0)
    for k in ("tri_id", "bary", "L_ind", "sec_rec", "sec_vis"):
        assert torch.equal(getattr(ref, k), getattr(hb, k)), k
    for v in range(len(hcams)):
        log(f"[half] view {v}: 48^2 pass vs the oracle")
        _compare_view(tori, hcams[v], p0, ref, v, v)
        up = O.upsample_indirect(hb.L_ind[v].cpu().numpy(), hb.tri_id[v].cpu().numpy(), b.tri_id[v].cpu().numpy())
        got = b.L_ind[v].cpu().numpy()
        assert np.allclose(got, up, rtol=1e-6, atol=1e-7 * max(1.0, np.abs(up).max()))


def test_half_res_indirect_gradient(tori):
    from paper_2608_24109_amd import _lib as L
    from paper_2608_24109_amd.render import render_backward
    sc = tori.sc
    p = tori.params()
    p.half_res_indirect = True
    lam = 0.8
    cc, b = _forward_half(tori, p)
    hb = b.half
    V, H, W = len(sc.cams), sc.cams[0].H, sc.cams[0].W
    g = I.upstream_grad(V, H, W, seed=9).astype(np.float64)
    # zero the upstream gradient on pixels fed by a flipped decision: a full-resolution direct
    # decision, or a half-resolution indirect decision among the pixel's taps
    pd = dataclasses.replace(p, N_b=0, half_res_indirect=False)  # the full-resolution direct pass
    for v, cam in enumerate(sc.cams):
        rf = tori.oracle(cam, pd, view_id=v)
        bad = b.vis[v].cpu().numpy().reshape(-1) != rf.vis
        rh = tori.oracle(_half_cam(cam), p, view_id=v)
        st = hb.sec_rec[v].cpu().numpy().reshape(-1, p.N_b, 3)[..., 0]
        badh = (st != rh.sec_tri).any(1) | (hb.sec_vis[v].cpu().numpy().reshape(-1) != rh.sec_vis)
        if badh.any():
            idx, wts = O._up_taps(hb.tri_id[v].cpu().numpy(), b.tri_id[v].cpu().numpy())
            bad |= (badh[idx.reshape(-1, 4)] & (wts.reshape(-1, 4) > 0)).any(1)
        log(f"  view {v}: {int(bad.sum())} pixels zeroed")
        assert bad.mean() < 0.01
        g[v].reshape(-1, 3)[bad] = 0.0
    dtex = torch.zeros_like(tori.mat.tex)
    denv = torch.zeros(tori.env.env.shape, dtype=torch.float64, device="cuda")
    render_backward(tori.mesh, tori.mat, tori.env, cc, p, b, torch.from_numpy(g.astype(np.float32)).cuda(), lam,
                    dtex, denv)
    torch.cuda.synchronize()
    dtex = dtex.cpu().numpy().astype(np.float64)
    denv = denv.cpu().numpy()
    rng = np.random.default_rng(3)
    for _ in range(3):
        vt = rng.normal(size=sc.tex.shape)
        ve = rng.normal(size=sc.env.shape)
        for kind, dot_kw, got, grad in (("tex", "tex_dot", float(np.sum(dtex * vt)), dtex),
                                        ("env", "env_dot", float(np.sum(denv * ve)), denv)):
            ref = 0.0
            for v, cam in enumerate(sc.cams):
                kw = {dot_kw: vt if kind == "tex" else ve}
                rf = tori.oracle(cam, pd, view_id=v, **kw)
                rh = tori.oracle(_half_cam(cam), p, view_id=v, **kw)
                up = O.upsample_indirect(rh.dL_ind.reshape(_half_cam(cam).H, _half_cam(cam).W, 3),
                                         hb.tri_id[v].cpu().numpy(), b.tri_id[v].cpu().numpy())
                gv = g[v].reshape(-1, 3)
                ref += float(np.sum(gv * rf.dL_dir)) + lam * float(np.sum(gv * up.reshape(-1, 3)))
            log(f"  {kind}: adjoint {got:.6e} oracle {ref:.6e}")
            assert abs(got - ref) <= 1e-3 * abs(ref) + 1e-6 * np.abs(grad).max() * np.sqrt(grad.size)
