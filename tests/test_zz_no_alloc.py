"""The no-allocation resolve, hm_resolve_shade_noalloc, against the resolve
with a caller workspace, hm_resolve_shade, called through the C ABI on the same
device buffers: two frames in a row, the second smaller than the first (so the
library's scratch still holds the first frame's records when the second call
starts), each compared element by element within 1e-4 (the kernels are shared,
so the results are in fact identical bit for bit); every resolve mode; and a
filtered frame beyond the scratch's maximum is rejected before anything is
enqueued, while modes that need no scratch accept it."""
import ctypes

import numpy as np
import pytest

from paper_2607_04230_amd import hm, scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _rendered(sc, torch):
    from paper_2607_04230_amd.render import DeviceScene
    ds = DeviceScene(sc)
    ds.render()
    torch.cuda.synchronize()
    return ds


def _noalloc(st, vis, cams, fr, sp, out, torch):
    L = hm.load()
    return L.hm_resolve_shade_noalloc(ctypes.byref(st), vis.data_ptr(), cams.data_ptr(),
                                      ctypes.byref(fr), ctypes.byref(sp), out.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)


def _both(ds, mode, torch):
    sp = hm.shade_params(ds.resolve_params, mode, ds.sc.bg)
    ref = torch.full_like(ds.out, float("nan"))
    hm.resolve_shade(ds.st, ds.vis, ds.cams, ds.fr, sp, ref, ds.ws_resolve)
    got = torch.full_like(ds.out, float("nan"))
    rc = _noalloc(ds.st, ds.vis, ds.cams, ds.fr, sp, got, torch)
    assert rc == hm.HM_OK, hm.load().hm_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_filter_two_frames_second_smaller(torch):
    big = scenes.config_head(width=640, height=360, strands_per_quad=16)
    small = scenes.config_tiny()
    for sc in (big, small):
        print(f"[noalloc] filter resolve {sc.width}x{sc.height}", flush=True)
        ds = _rendered(sc, torch)
        ref, got = _both(ds, hm.RESOLVE_FILTER, torch)
        assert np.isfinite(got).all()
        assert np.abs(got.astype(np.float64) - ref).max() <= TOL
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        assert (got[..., 3] > 0).sum() > 1000          # hair was resolved
        del ds


@pytest.mark.parametrize("mode", [hm.RESOLVE_CENTER, hm.RESOLVE_SOFT])
def test_noalloc_other_modes(torch, mode):
    ds = _rendered(scenes.config_tiny(), torch)
    ref, got = _both(ds, mode, torch)
    assert np.abs(got.astype(np.float64) - ref).max() <= TOL
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_noalloc_rejects_frames_beyond_its_scratch(torch):
    sc = scenes.config_tiny()
    ds = _rendered(sc, torch)
    W, H = 2049, 2048                       # 4,196,352 pixels > HM_NOALLOC_MAX_PIXELS
    assert W * H > 4194304
    fr = hm.frame(1, W, H)
    cams = torch.from_numpy(np.repeat(sc.cams[:1], 1, 0)).cuda()
    vis = torch.full((1, 2, H, W), -1, dtype=torch.int64, device="cuda")   # no hair
    out = torch.zeros((1, H, W, 4), dtype=torch.float32, device="cuda")
    sp = hm.shade_params(ds.resolve_params, hm.RESOLVE_FILTER, sc.bg)
    assert _noalloc(ds.st, vis, cams, fr, sp, out, torch) == 3      # HM_ERR_WORKSPACE
    assert b"no-allocation" in hm.load().hm_last_error()
    # the centre resolve needs no scratch: the same frame is accepted
    sp = hm.shade_params(ds.resolve_params, hm.RESOLVE_CENTER, (0.25, 0.5, 0.75))
    assert _noalloc(ds.st, vis, cams, fr, sp, out, torch) == hm.HM_OK
    torch.cuda.synchronize()
    o = out[0, ::97, ::89].cpu().numpy()
    assert np.array_equal(o[..., :3], np.broadcast_to(np.float32([0.25, 0.5, 0.75]), o[..., :3].shape))
    assert (o[..., 3] == 0).all()
