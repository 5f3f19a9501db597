"""Batches of uneven pairs (dm_match_batch): every pair's matches and
gradients equal those of the single-pair entry points bit for bit (same
kernels, same arithmetic, grouped into one launch per stage); HIP graph
replays equal the eager run, replay after replay, with unrelated eager work
and synchronisations in between; the autotuner changes launch shapes only."""
import functools

import numpy as np
import pytest
import torch

import paper_1506_07656_amd as dm
import synth
from oracle import dm_oracle as O
from tests.helpers import compare_matches, within_px

pytestmark = pytest.mark.gpu

# (W1, H1, W2, H2) crops of the uneven batch recipe: mixed sizes, I != I'
# sizes, widths that are and are not multiples of 4, pyramids of 4 to 7 levels.
SIZES = [(128, 96, 128, 96), (203, 117, 190, 121), (64, 64, 72, 60), (310, 150, 300, 156), (157, 99, 157, 99),
         (96, 130, 101, 128)]


@functools.lru_cache(maxsize=None)
def batch_arrays():
    pairs = synth.make_batch(len(SIZES), base_seed=7100, max_disp=20.0)
    out = []
    for (W1, H1, W2, H2), p in zip(SIZES, pairs):
        a = np.zeros((H1, W1), np.float32)
        b = np.zeros((H2, W2), np.float32)
        h, w = min(H1, p["img1"].shape[0]), min(W1, p["img1"].shape[1])
        a[:h, :w] = p["img1"][:h, :w]
        h, w = min(H2, p["img2"].shape[0]), min(W2, p["img2"].shape[1])
        b[:h, :w] = p["img2"][:h, :w]
        out.append((a, b))
    return out


def batch_images():
    i1 = [torch.from_numpy(a).cuda() for a, _ in batch_arrays()]
    i2 = [torch.from_numpy(b).cuda() for _, b in batch_arrays()]
    return i1, i2


@functools.lru_cache(maxsize=None)
def textured_arrays():
    """The SIZES pairs with warped blurred-noise content over their whole
    area (no zero padding: flat padding makes FP64 scores tie exactly along
    different paths, which FP32 may resolve either way)."""
    out = []
    for k, (W1, H1, W2, H2) in enumerate(SIZES):
        p = synth.make_warp_pair(7200 + k, max(W1, W2), max(H1, H2), 20.0)
        out.append((np.ascontiguousarray(p["img1"][:H1, :W1]), np.ascontiguousarray(p["img2"][:H2, :W2])))
    return out


@functools.lru_cache(maxsize=None)
def batch_oracle():
    """The FP64 oracle's matches and decision margins of every textured pair."""
    res = []
    for a, b in textured_arrays():
        out, margin, _, _ = O.match(a, b, O.Params())
        res.append((out, margin))
    return res


def single(i1, i2, prec):
    return [dm.match_images(a, b, dm.params(precision=prec)) for a, b in zip(i1, i2)]


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batch_equals_single_pairs(prec):
    i1, i2 = batch_images()
    B = dm.Batch(SIZES, dm.params(precision=prec), graph=False)
    B.set_images(i1, i2)
    B.run()
    got = B.matches()
    ref = single(i1, i2, prec)
    for k, (g, r) in enumerate(zip(got, ref)):
        print(f"pair {k} {SIZES[k]}: lmax {B.info.lmax[k]}, {len(g)} matches", flush=True)
        assert len(g) > 0
        assert torch.equal(g, r), k
    B.release()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_matches_oracle(prec):
    """Every pair of a graph-replayed batch (the SIZES shapes, textured over
    their whole area) against the FP64 oracle on the same images: FP32 loses
    or moves no match away from the oracle's near-ties and keeps scores
    within 1e-5; BF16 keeps >= 99 % of the oracle's matches within 1 px."""
    i1 = [torch.from_numpy(a).cuda() for a, _ in textured_arrays()]
    i2 = [torch.from_numpy(b).cuda() for _, b in textured_arrays()]
    B = dm.Batch(SIZES, dm.params(precision=prec), graph=True)
    B.set_images(i1, i2)
    B.run()
    got = B.matches()
    for k, (g, (ref, margin)) in enumerate(zip(got, batch_oracle())):
        g = g.cpu().numpy()
        if prec == "fp32":
            r = compare_matches(g, ref, margin, tie=1e-4)
            print(f"pair {k} {SIZES[k]}: ref {r['n_ref']} gpu {r['n_gpu']} near-ties {r['near_ties']} "
                  f"missing {len(r['missing'])} moved {len(r['moved'])} bad-score {len(r['bad_score'])} "
                  f"extra {len(r['extra'])} worst rel {r['worst_rel']:.2e}", flush=True)
            assert not r["missing"] and not r["moved"] and not r["bad_score"], k
            assert len(r["extra"]) <= r["near_ties"], k
        else:
            frac = within_px(g, ref, 1.0)
            print(f"pair {k} {SIZES[k]}: {len(g)} matches vs {len(ref)}; within 1 px {frac:.4f}", flush=True)
            assert frac >= 0.99, k
    B.release()


def test_wide_pair_in_a_batch_equals_single_pair():
    """A pair of the batch recipe's largest width (621 x 188, I' 600 x 180)
    beside a small one: the batch gives the single-pair results bit for bit,
    matches and gradients."""
    sizes = [(621, 188, 600, 180), (140, 100, 132, 96)]
    i1, i2 = [], []
    for k, (W1, H1, W2, H2) in enumerate(sizes):
        p = synth.make_warp_pair(7300 + k, W1, H1, 30.0)
        i1.append(torch.from_numpy(np.ascontiguousarray(p["img1"])).cuda())
        i2.append(torch.from_numpy(np.ascontiguousarray(p["img2"][:H2, :W2])).cuda())
    prm = dm.params(precision="bf16")
    B = dm.Batch(sizes, prm, bwd=True, graph=True)
    B.set_images(i1, i2)
    B.run()
    torch.cuda.synchronize()
    ref = single(i1, i2, "bf16")
    for k, g in enumerate(B.matches()):
        print(f"pair {k} {sizes[k]}: lmax {B.info.lmax[k]}, {len(g)} matches", flush=True)
        assert len(g) > 0 and torch.equal(g, ref[k]), k
    for k, (a, b) in enumerate(zip(i1, i2)):
        d1, d2 = dm.descriptors(a, prm), dm.descriptors(b, prm)
        pyr = dm.Pyramid(d1, d2, prm, False)
        top = pyr.forward()
        flat = top.reshape(top.shape[0] * top.shape[1], -1)
        dtop = torch.zeros_like(flat)
        dtop.scatter_(1, flat.argmax(1, keepdim=True), 1.0)
        g1, g2 = pyr.backward(dtop.view_as(top))
        torch.cuda.synchronize()
        assert torch.equal(B.dd1[k], g1) and torch.equal(B.dd2[k], g2), k
    B.release()


def test_graph_replays_equal_eager():
    i1, i2 = batch_images()
    E = dm.Batch(SIZES, dm.params(precision="bf16"), graph=False)
    E.set_images(i1, i2)
    E.run()
    want = E.matches()
    G = dm.Batch(SIZES, dm.params(precision="bf16"), graph=True)
    G.set_images(i1, i2)
    other = dm.Matcher(96, 80, 96, 80, dm.params(precision="fp32"))
    x = torch.rand(96 * 80, device="cuda").reshape(80, 96)
    for rep in range(4):
        G.n_out.zero_()
        G.out.fill_(-1)
        G.run()
        got = G.matches()
        for k in range(len(SIZES)):
            assert torch.equal(got[k], want[k]), (rep, k)
        # unrelated eager work and a synchronisation between replays
        other.run_images(x, x.flip(1).contiguous())
        _ = (x @ x.t()).sum().item()
        torch.cuda.synchronize()
    E.release()
    G.release()


def test_batch_backward_equals_single_pyramid():
    i1, i2 = batch_images()
    prm = dm.params(precision="bf16")
    B = dm.Batch(SIZES, prm, bwd=True, graph=True)
    B.set_images(i1, i2)
    B.run()
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(i1, i2)):
        d1, d2 = dm.descriptors(a, prm), dm.descriptors(b, prm)
        pyr = dm.Pyramid(d1, d2, prm, False)
        top = pyr.forward()
        flat = top.reshape(top.shape[0] * top.shape[1], -1)
        dtop = torch.zeros_like(flat)
        dtop.scatter_(1, flat.argmax(1, keepdim=True), 1.0)     # first maximum of each top map
        g1, g2 = pyr.backward(dtop.view_as(top))
        torch.cuda.synchronize()
        e1 = (B.dd1[k] - g1).abs().max().item()
        e2 = (B.dd2[k] - g2).abs().max().item()
        print(f"pair {k}: |dd1| max {g1.abs().max().item():.3e} diff {e1:.1e}; |dd2| max {g2.abs().max().item():.3e} "
              f"diff {e2:.1e}", flush=True)
        assert g1.abs().max().item() > 0 and g2.abs().max().item() > 0
        assert torch.equal(B.dd1[k], g1) and torch.equal(B.dd2[k], g2), k
    # the forward of the same batch call is unchanged by the backward
    ref = single(i1, i2, "bf16")
    for k, g in enumerate(B.matches()):
        assert torch.equal(g, ref[k]), k
    B.release()


def test_autotuner_keeps_results(tmp_path, monkeypatch):
    """The tuner changes launch shapes only; its tiles persist in the tile
    cache (DM_TILE_CACHE), from which a second batch of the same size bucket
    takes them untimed, with the same matches."""
    import json
    cache = tmp_path / "tiles.json"
    monkeypatch.setenv("DM_TILE_CACHE", str(cache))
    i1, i2 = batch_images()
    T = dm.Batch(SIZES, dm.params(precision="bf16"), graph=True, autotune=True)
    T.set_images(i1, i2)
    T.run()
    t = T.tiles()
    print(f"tuned: level rows {t.level_rows}, backtrack rows {t.bt_rows}, forward {t.tuned_ms:.3f} ms", flush=True)
    assert t.tuned == 1 and t.level_rows in (8, 16, 32, 64) and t.bt_rows in (8, 16, 32, 64) and t.tuned_ms > 0
    ref = single(i1, i2, "bf16")
    for k, g in enumerate(T.matches()):
        assert torch.equal(g, ref[k]), k
    T.release()
    entries = json.loads(cache.read_text())["entries"]
    assert len(entries) == 1 and entries[0]["level_rows"] == t.level_rows and entries[0]["bt_rows"] == t.bt_rows
    assert entries[0]["key"].startswith("bf16/fwd/n8/")
    # a second batch of the same bucket reads the tiles from the cache
    T2 = dm.Batch(SIZES, dm.params(precision="bf16"), graph=True, autotune=True)
    T2.set_images(i1, i2)
    T2.run()
    t2 = T2.tiles()
    assert t2.tuned == 2 and (t2.level_rows, t2.bt_rows) == (t.level_rows, t.bt_rows)
    assert list(t2.blocks_per_cu) == list(t.blocks_per_cu)
    for k, g in enumerate(T2.matches()):
        assert torch.equal(g, ref[k]), k
    T2.release()
    # a foreign or damaged file is ignored and rewritten
    cache.write_text("not json\n")
    T3 = dm.Batch(SIZES, dm.params(precision="bf16"), graph=False, autotune=True)
    T3.set_images(i1, i2)
    T3.run()
    assert T3.tiles().tuned == 1
    for k, g in enumerate(T3.matches()):
        assert torch.equal(g, ref[k]), k
    T3.release()
    assert len(json.loads(cache.read_text())["entries"]) == 1
