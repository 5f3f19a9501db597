"""Approximate DeepMatching (Sec. 4.1) on the GPU against the FP64 oracle.

The k-means decisions of the library are those of an FP64 evaluation, so on
the same (float32) descriptors the assignments must equal the oracle's
exactly and the prototypes agree to FP64 rounding; the pyramid and matches
built on them follow the exact method's FP32 tolerances."""
import functools

import numpy as np
import pytest
import torch

import paper_1506_07656_amd as dm
import synth
from oracle import dm_oracle as O
from tests.helpers import FP32_TIE, compare_matches, oracle_pair, within_px

pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return a.astype(np.float32).astype(np.float64)


@functools.lru_cache(maxsize=None)
def approx_oracle(name: str, D: int, iters: int = 10):
    """Oracle run of approximate DM on the float32-rounded descriptors the
    GPU receives."""
    o = oracle_pair(name)
    D1, D2 = f32(o["D1"]), f32(o["D2"])
    prm = O.Params(max_patch=synth.CONFIG_NMAX[name], prototypes=D, kmeans_iters=iters)
    out, margin, pyr, M = O.match_descriptors(D1, D2, prm)
    return dict(D1=D1, D2=D2, out=out, margin=margin, pyr=pyr, prm=prm)


def run_gpu(D1, D2, **kw):
    m, ws, pl = dm.match_descriptors(cuda(D1), cuda(D2), dm.params(**kw), return_state=True)
    torch.cuda.synchronize()
    return m.cpu().numpy(), dm.workspace_views(ws, pl), pl


def check_kmeans(views, pyr, label):
    assign = views["assign"].cpu().numpy().ravel()
    protos = views["protos"].cpu().numpy()
    ks = views["kstat"].cpu().numpy()
    diff = int((assign != pyr.assign).sum())
    print(f"{label}: {len(assign)} patches, D={len(protos)}, assignments differing {diff}, "
          f"settled in FP64: {ks[0]} (two candidates) {ks[1]} (all centroids), "
          f"max |proto diff| {np.abs(protos - pyr.protos).max():.2e}", flush=True)
    assert diff == 0
    np.testing.assert_allclose(protos, pyr.protos, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(protos, axis=1), 4.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,D,iters", [("c1", 16, 10), ("c1", 256, 3), ("c2", 64, 10), ("c2", 512, 6),
                                          ("c2", 1, 2), ("c2", 700, 0), ("c2", 3072, 1)])
def test_kmeans_equals_oracle(name, D, iters):
    o = oracle_pair(name)
    D1 = f32(o["D1"])
    C, asg = O.spherical_kmeans(O.atomic_patch_vectors(D1), D, iters)
    _, views, pl = run_gpu(D1, f32(o["D2"]), max_patch=synth.CONFIG_NMAX[name], prototypes=D, kmeans_iters=iters)
    assert pl.prototypes == D
    check_kmeans(views, type("KM", (), dict(assign=asg, protos=C)), f"{name} D={D} iters={iters}")


@pytest.mark.parametrize("name,D", [("c1", 16), ("c2", 64), ("c2", 512)])
def test_approx_pyramid_and_matches_equal_oracle(name, D):
    o = approx_oracle(name, D)
    pyr = o["pyr"]
    gpu, views, pl = run_gpu(o["D1"], o["D2"], max_patch=synth.CONFIG_NMAX[name], prototypes=D)
    check_kmeans(views, pyr, f"{name} D={D}")
    # Level 0: the D prototype maps (each compared through a patch that uses it).
    cp0 = views["levels"][0]["cp"].cpu().numpy()[0]
    code0 = views["levels"][0]["code"].cpu().numpy()[0]
    ny, nx = pyr.G[0].shape
    used, first = np.unique(pyr.assign, return_index=True)
    ref = pyr.Cp[0].reshape(ny * nx, *pyr.Cp[0].shape[2:])[first]
    np.testing.assert_allclose(cp0[used], ref, rtol=1e-5, atol=1e-7)
    gap = pyr.gap[0].reshape(ny * nx, *pyr.gap[0].shape[2:])[first]
    cref = pyr.code[0].reshape(ny * nx, *pyr.code[0].shape[2:])[first]
    clear = gap > FP32_TIE * (1 + ref)
    assert ((code0[used] != cref) & clear).sum() == 0
    for lv in range(1, pyr.lmax):
        G = pyr.G[lv]
        cp = views["levels"][lv]["cp"].cpu().numpy()[G]
        np.testing.assert_allclose(cp, pyr.Cp[lv][G], rtol=1e-5, atol=1e-7, err_msg=f"level {lv}")
    G = pyr.G[pyr.lmax]
    np.testing.assert_allclose(views["top"].cpu().numpy()[G], pyr.top[G], rtol=1e-5, atol=1e-7)
    r = compare_matches(gpu, o["out"], o["margin"])
    print(f"{name} D={D}: ref {r['n_ref']} gpu {r['n_gpu']} near-ties {r['near_ties']} missing {len(r['missing'])} "
          f"moved {len(r['moved'])} bad-score {len(r['bad_score'])} extra {len(r['extra'])}", flush=True)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]


def test_every_patch_a_prototype_is_the_exact_method():
    o = oracle_pair("c1")
    gpu, views, _ = run_gpu(f32(o["D1"]), f32(o["D2"]), max_patch=32, prototypes=256, kmeans_iters=2)
    assert (views["assign"].cpu().numpy().ravel() == np.arange(256)).all()
    r = compare_matches(gpu, o["out"], o["margin"])
    assert not r["missing"] and not r["moved"] and not r["bad_score"]


def test_approx_bf16():
    o = approx_oracle("c2", 512)
    gpu, views, _ = run_gpu(o["D1"], o["D2"], max_patch=64, prototypes=512, precision="bf16")
    check_kmeans(views, o["pyr"], "c2 D=512 bf16")   # k-means runs in FP32/FP64 in every precision
    frac = within_px(gpu, o["out"], 1.0)
    print(f"c2 D=512 bf16: {len(gpu)} matches, {frac:.4f} of oracle matches within 1 px", flush=True)
    assert frac >= 0.99


def test_approx_deterministic_and_images_entry():
    o = oracle_pair("c2")
    a, va, _ = run_gpu(o["D1"], o["D2"], max_patch=64, prototypes=300)
    b, vb, _ = run_gpu(o["D1"], o["D2"], max_patch=64, prototypes=300)
    np.testing.assert_array_equal(a, b)
    assert torch.equal(va["assign"], vb["assign"]) and torch.equal(va["protos"], vb["protos"])
    assert torch.equal(va["levels"][0]["cp"], vb["levels"][0]["cp"])
    # The images entry computes its descriptors, then runs the same path as
    # the descriptors entry on them.
    p = o["pair"]
    prm = dm.params(max_patch=64, prototypes=300)
    i1, i2 = cuda(p["img1"]), cuda(p["img2"])
    m, ws, pl = dm.match_images(i1, i2, prm, return_state=True)
    v = dm.workspace_views(ws, pl)
    m2, ws2, pl2 = dm.match_descriptors(dm.descriptors(i1), dm.descriptors(i2), prm, return_state=True)
    v2 = dm.workspace_views(ws2, pl2)
    assert torch.equal(m, m2) and torch.equal(v["assign"], v2["assign"]) and torch.equal(v["protos"], v2["protos"])


def test_approx_512x256_bench_configuration():
    """The benchmark's approximate workload: 512x256 images, D = 1024 and 64.
    The k-means result equals the oracle's; the matches keep the structure of
    Eq. (16) and, for D = 1024, most of the exact method's matches."""
    from tests.test_gpu_parity import load_golden
    p = synth.make_pair("c3")
    od1, od2 = f32(O.descriptors(p["img1"])), f32(O.descriptors(p["img2"]))
    X = O.atomic_patch_vectors(od1)
    for D in (1024, 64):
        m, views, pl = run_gpu(od1, od2, prototypes=D)
        C, asg = O.spherical_kmeans(X, D, 10)
        check_kmeans(views, type("KM", (), dict(assign=asg, protos=C)), f"c3 D={D}")
        assert len(np.unique(m[:, :2], axis=0)) == len(m)
        assert len(np.unique(m[:, 2:4] // 4, axis=0)) == len(m)
        keys = m[:, 1] * 1e6 + m[:, 0]
        assert (np.diff(keys) > 0).all()
        if D == 1024:
            _, ref, _, _ = load_golden("c3")
            print(f"c3 D=1024: {len(m)} matches; {within_px(m, ref, 1.0):.4f} of the exact method's within 1 px",
                  flush=True)


def test_approx_uneven_crops():
    """I 310x150, I' 300x156 (crops of the 512x256 pair): level maps 150, 75,
    38, ... wide, 2849 atomic patches, D = 333 (not a multiple of the
    64-centroid chunks)."""
    from tests.test_gpu_parity import odd_case
    o = odd_case()
    D1, D2 = f32(o["D1"]), f32(o["D2"])
    prm = O.Params(prototypes=333, kmeans_iters=6)
    out, margin, pyr, _ = O.match_descriptors(D1, D2, prm)
    gpu, views, pl = run_gpu(D1, D2, prototypes=333, kmeans_iters=6)
    assert pl.lmax == pyr.lmax and pl.n_atomic == 77 * 37
    check_kmeans(views, pyr, "odd D=333")
    r = compare_matches(gpu, out, margin)
    print(f"odd D=333: ref {r['n_ref']} gpu {r['n_gpu']} near-ties {r['near_ties']} missing {len(r['missing'])} "
          f"moved {len(r['moved'])} bad-score {len(r['bad_score'])} extra {len(r['extra'])}", flush=True)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]
