"""GPU gradients of the soft-coverage resolve (hand-written backward through the
C ABI) against the oracle's binary64 autograd gradient, visibility fixed."""
import numpy as np
import pytest

from paper_2607_04230_amd import scenes
from paper_2607_04230_amd.scenes import ResolveParams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _setup(O, torch, sc):
    from paper_2607_04230_amd.diff import SoftContext
    ref = O.render(sc, want=("vis",))
    pos = torch.from_numpy(ref["pos_w"].copy()).cuda()
    rgb = torch.from_numpy(ref["rgb"].copy()).cuda()
    flags = torch.from_numpy(ref["flags"].copy()).cuda()
    soff = torch.from_numpy(ref["scene_off"].view(np.int32).copy()).cuda()
    cams = torch.from_numpy(sc.cams.copy()).cuda()
    ctx = SoftContext(flags, soff, cams, sc.width, sc.height, r_min=sc.r_min)
    return ref, pos, rgb, ctx


def _oracle_target(O, torch, sc, ref, rp):
    """The differentiable workload's target: the oracle's soft render (its own
    visibility) of the parameters perturbed by N(0, 0.01) on positions,
    multiplicatively on widths, and on colours."""
    tp, tc = scenes.perturb_stream(ref["pos_w"], ref["rgb"], seed=sc.seed + 1)
    with O.threads(O.host_threads()):
        tvis = O.raster(tp, ref["flags"], ref["scene_off"], sc.cams, sc.width, sc.height,
                        sc.r_min, sc.scene_z)
    t = O.soft_forward(torch.as_tensor(tp.astype(np.float64)),
                       torch.as_tensor(tc.astype(np.float64)), ref["flags"], tvis, sc.cams,
                       sc.width, sc.height, rp).numpy()
    assert not np.array_equal(tvis, ref["vis"])       # the perturbation moves strands
    return t.astype(np.float32)


def _rel(g, r):
    return float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30))


@pytest.mark.parametrize("name", ["micro", "diff"])
def test_soft_gradient_matches_oracle(O, torch, name):
    from paper_2607_04230_amd.diff import soft_render
    if name == "micro":
        sc = scenes.micro_scene(3, res=48, width=0.03)
        sc.r_min = 1.0
    else:
        sc = scenes.config_diff()
    ref, pos, rgb, ctx = _setup(O, torch, sc)
    rp = ResolveParams()
    target = _oracle_target(O, torch, sc, ref, rp)
    p = pos.clone().requires_grad_(True)
    c = rgb.clone().requires_grad_(True)
    out = soft_render(p, c, ctx)
    vis_gpu = ctx.vis.cpu().numpy().view(np.uint64)
    assert np.array_equal(vis_gpu, ref["vis"])
    o_ref = O.soft_forward(torch.as_tensor(ref["pos_w"].astype(np.float64)),
                           torch.as_tensor(ref["rgb"].astype(np.float64)), ref["flags"],
                           ref["vis"], sc.cams, sc.width, sc.height, rp).numpy()
    assert np.abs(out.detach().cpu().numpy() - o_ref).max() <= 1e-4
    loss = ((out - torch.from_numpy(target).cuda()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    gp_ref, gc_ref = O.soft_grad(ref["pos_w"].astype(np.float64), ref["rgb"].astype(np.float64),
                                 ref["flags"], ref["vis"], sc.cams, sc.width, sc.height, rp,
                                 2.0 * (o_ref - target))
    gp = p.grad.cpu().numpy().astype(np.float64)
    gc = c.grad.cpu().numpy().astype(np.float64)
    for g, r, label in ((gp[:, :3], gp_ref[:, :3], "pos"), (gp[:, 3], gp_ref[:, 3], "width"),
                        (gc[:, :3], gc_ref[:, :3], "rgb")):
        rel = _rel(g, r)
        mx = float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-30))
        print(f"{name} {label}: rel L2 {rel:.2e}, max rel {mx:.2e}")
        assert rel <= 1e-4 and mx <= 1e-4, (label, rel, mx)
    assert np.abs(gc[:, 3]).max() == 0.0


def test_soft_gradient_descent_reduces_loss(O, torch):
    """Fit to a target rendered from perturbed parameters: the loss falls."""
    from paper_2607_04230_amd.diff import soft_render
    sc = scenes.config_diff(res=256, strands_per_quad=4)
    ref, pos, rgb, ctx = _setup(O, torch, sc)
    tp, tc = scenes.perturb_stream(ref["pos_w"], ref["rgb"], seed=5)
    with torch.no_grad():
        target = soft_render(torch.from_numpy(tp).cuda(), torch.from_numpy(tc).cuda(), ctx).clone()
    c = rgb.clone().requires_grad_(True)
    losses = []
    for _ in range(5):
        out = soft_render(pos, c, ctx)
        loss = ((out - target) ** 2).sum()
        losses.append(float(loss))
        g, = torch.autograd.grad(loss, [c])
        with torch.no_grad():
            c -= 0.02 * g
    assert losses[-1] < losses[0]
