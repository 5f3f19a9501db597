"""GPU parity of DeepFlow (Sec. 4.3) against the FP64 oracle: the same images
and the same matches in, the flow fields compared pixel by pixel.

Tolerance: the GPU computes in FP32.  Each fixed-point step solves a
well-conditioned system (SOR is a contraction), so rounding differences do
not grow from level to level; the flows of the two paths stay within
FLOW_ATOL pixels everywhere (measured: a few 1e-5 px on these pairs)."""
import numpy as np
import pytest
import torch

import paper_1506_07656_amd as dm
import synth
from oracle import deepflow_oracle as F
from oracle import dm_oracle as O
from tests.test_deepflow_oracle import smooth_texture

pytestmark = pytest.mark.gpu

FLOW_ATOL = 2e-3


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def gpu_flow(I1, I2, matches=None, **kw):
    m = None if matches is None or len(matches) == 0 else cuda(np.asarray(matches, np.int32), torch.int32)
    f = dm.deepflow(cuda(I1), cuda(I2), m, prm=dm.flow_params(**kw))
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64)


def compare(name, g, o):
    d = np.abs(g - o)
    print(f"{name}: max |flow_gpu - flow_oracle| {d.max():.2e} px (mean {d.mean():.2e}); "
          f"oracle flow range u [{o[..., 0].min():.2f}, {o[..., 0].max():.2f}]", flush=True)
    assert np.isfinite(g).all()
    assert d.max() <= FLOW_ATOL


@pytest.mark.parametrize("delta", [0.0, 1.0])
def test_translation_pair_equals_oracle(delta):
    t = (1.6, -0.9)
    I1, I2 = smooth_texture(64, 56), smooth_texture(64, 56, t=t)
    o = F.deepflow(I1, I2, np.zeros((0, 4)), F.FlowParams(delta=delta))
    g = gpu_flow(I1, I2, delta=delta)
    compare(f"translation, delta {delta}", g, o)


@pytest.mark.parametrize("W,H", [(37, 23), (64, 64), (101, 77)])
def test_ground_truth_matches_equal_oracle(W, H):
    """A warped pair with matches on a 4-pixel grid read off its ground-truth
    field (rounded to whole pixels, as DeepMatching's are), odd sizes."""
    p = synth.make_warp_pair(900 + W, W, H, 6.0)
    ys, xs = np.mgrid[2:H:4, 2:W:4]
    qx, qy = p["flow"](xs, ys)   # target positions of the grid points
    m = np.stack([xs.ravel(), ys.ravel(), np.rint(qx).ravel(), np.rint(qy).ravel(),
                  np.zeros(xs.size)], axis=1).astype(np.int64)
    o = F.deepflow(p["img1"], p["img2"], m[:, :4].astype(np.float64), F.FlowParams())
    g = gpu_flow(p["img1"], p["img2"], m)
    compare(f"{W}x{H} warped pair, {len(m)} matches", g, o)
    # the flow follows the field: at the grid points it is within a pixel of the matches
    gx = g[m[:, 1], m[:, 0]]
    err = np.hypot(gx[:, 0] - (m[:, 2] - m[:, 0]), gx[:, 1] - (m[:, 3] - m[:, 1]))
    print(f"{W}x{H}: flow at the match points within {np.median(err):.3f} px (median) of the matches")
    assert np.median(err) < 0.75


@pytest.mark.parametrize("kw", [dict(n_sor=7), dict(n_sor=0), dict(n_fixed=0), dict(n_sor=3, n_fixed=2, omega=1.2)])
def test_sweep_counts_equal_oracle(kw):
    """Other SOR schedules on a warped pair whose fine levels take the tiled
    SOR on 64 x 64 tiles: 7 sweeps (one launch of 14 half-sweeps per fixed
    point, on the tiles with a rim of 17), 3 sweeps with 2 fixed points, no
    sweeps or no fixed points (each level keeps the flow it receives, and
    the level's add runs instead of the last SOR launch)."""
    W, H = 96, 72
    p = synth.make_warp_pair(505, W, H, 5.0)
    ys, xs = np.mgrid[2:H:4, 2:W:4]
    qx, qy = p["flow"](xs, ys)
    m = np.stack([xs.ravel(), ys.ravel(), np.rint(qx).ravel(), np.rint(qy).ravel(),
                  np.zeros(xs.size)], axis=1).astype(np.int64)
    o = F.deepflow(p["img1"], p["img2"], m[:, :4].astype(np.float64), F.FlowParams(**kw))
    g = gpu_flow(p["img1"], p["img2"], m, **kw)
    compare(f"{W}x{H} pair, {kw}", g, o)


def grid_matches(p, W, H, step):
    ys, xs = np.mgrid[2:H:step, 2:W:step]
    qx, qy = p["flow"](xs, ys)
    return np.stack([xs.ravel(), ys.ravel(), np.rint(qx).ravel(), np.rint(qy).ravel(),
                     np.zeros(xs.size)], axis=1).astype(np.int64)


@pytest.mark.parametrize("W,H,kw", [(240, 240, {}), (520, 460, dict(n_fixed=1, n_sor=5))])
def test_every_tile_shape_equals_oracle(W, H, kw):
    """On a 256-CU device: the 240 x 240 pair's two finest levels take the
    64 x 64 tiles with a rim of 17 (three launches per fixed point: the
    tiles with a rim of 25 would be more than the compute units), the levels
    below those with a rim of 25 (two launches), the last ones of at most
    4096 pixels one workgroup; the 520 x 460 pair's finest level needs more
    64 x 64 tiles than compute units even with a rim of 17 and takes the
    64 x 32 tiles with a rim of 10 (one fixed point of 5 sweeps keeps the
    oracle quick)."""
    p = synth.make_warp_pair(515 + W, W, H, 5.0)
    m = grid_matches(p, W, H, 4 if W < 400 else 8)
    o = F.deepflow(p["img1"], p["img2"], m[:, :4].astype(np.float64), F.FlowParams(**kw))
    g = gpu_flow(p["img1"], p["img2"], m, **kw)
    compare(f"{W}x{H} pair, {len(m)} matches, {kw}", g, o)


def test_deepmatching_matches_of_the_oracle():
    """DeepFlow on the 64 x 64 pair with the oracle's own DeepMatching matches
    (no input comes from the GPU path)."""
    pr = synth.make_pair("c1")
    out = O.match(pr["img1"], pr["img2"], O.Params(max_patch=32))[0]
    m = np.asarray(out)[:, :4]
    assert len(m) > 50
    o = F.deepflow(pr["img1"], pr["img2"], m.astype(np.float64), F.FlowParams())
    g = gpu_flow(pr["img1"], pr["img2"], np.concatenate([m, np.zeros((len(m), 1))], axis=1))
    compare(f"c1 pair, {len(m)} oracle matches", g, o)
    inner = g[12:-12, 12:-12]
    print(f"c1: median flow ({np.median(inner[..., 0]):.2f}, {np.median(inner[..., 1]):.2f}), true (5, -3)")
    assert abs(np.median(inner[..., 0]) - 5) < 0.5 and abs(np.median(inner[..., 1]) + 3) < 0.5


def test_device_count_limits_the_matches_and_runs_repeat():
    """Only the first n_matches rows count (the rest are garbage here); two
    runs give the same flow bit for bit."""
    p = synth.make_warp_pair(77, 48, 40, 4.0)
    ys, xs = np.mgrid[2:40:4, 2:48:4]
    m = np.stack([xs.ravel(), ys.ravel(), xs.ravel() + 2, ys.ravel() - 1, np.zeros(xs.size)], axis=1)
    k = len(m) // 2
    junk = m.copy()
    junk[k:, 2:4] += 17
    a = dm.deepflow(cuda(p["img1"]), cuda(p["img2"]), cuda(junk.astype(np.int32), torch.int32),
                    n_matches=torch.tensor([k], dtype=torch.int32, device="cuda"))
    b = dm.deepflow(cuda(p["img1"]), cuda(p["img2"]), cuda(m[:k].astype(np.int32), torch.int32))
    c = dm.deepflow(cuda(p["img1"]), cuda(p["img2"]), cuda(m[:k].astype(np.int32), torch.int32))
    assert torch.equal(a, b) and torch.equal(b, c)


def test_graph_replays_equal_eager():
    """The captured graph (DM_FLOW_GRAPH) replayed several times, with eager
    work and synchronisations in between and new inputs copied in, gives the
    eager call's flow bit for bit each time."""
    pairs = [synth.make_warp_pair(300 + k, 96, 72, 5.0) for k in range(2)]
    ys, xs = np.mgrid[2:72:4, 2:96:4]
    m = cuda(np.stack([xs.ravel(), ys.ravel(), xs.ravel() + 1, ys.ravel(), np.zeros(xs.size)], axis=1)
             .astype(np.int32), torch.int32)
    runner = dm.DeepFlow(96, 72, m.shape[0], graph=True)
    try:
        for rep in range(4):
            p = pairs[rep % 2]
            i1, i2 = cuda(p["img1"]), cuda(p["img2"])
            ref = dm.deepflow(i1, i2, m)
            torch.cuda.synchronize()
            runner.set(i1, i2, m)
            got = runner.run().clone()
            _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work and a sync in between
            assert torch.equal(got, ref), rep
    finally:
        runner.release()
