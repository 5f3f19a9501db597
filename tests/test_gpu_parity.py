"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import functools

import numpy as np
import pytest
import torch

import paper_1506_07656_amd as dm
import synth
from oracle import dm_oracle as O
from tests.helpers import FP32_TIE, compare_matches, oracle_from_desc, oracle_pair, within_px

pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run_desc(D1, D2, **kw):
    m, ws, pl = dm.match_descriptors(cuda(D1), cuda(D2), dm.params(**kw), return_state=True)
    torch.cuda.synchronize()
    return m.cpu().numpy(), dm.workspace_views(ws, pl), pl


def report(name, r):
    print(f"{name}: ref {r['n_ref']} gpu {r['n_gpu']} near-ties {r['near_ties']} missing {len(r['missing'])} "
          f"moved {len(r['moved'])} bad-score {len(r['bad_score'])} extra {len(r['extra'])} "
          f"worst rel {r['worst_rel']:.2e}", flush=True)


def explain_code_mismatch(pyr, lv, views, where):
    """Print the oracle's 9 pooling candidates next to the GPU's choice, and
    the candidates recomputed in FP64 from the GPU's own level below."""
    A = O.aggregate(pyr.Cp[lv - 1], lv, pyr) if lv else None
    Ag = None
    if lv:
        g = dict(pyr.__dict__)
        gp = O.Pyramid(**{k: g[k] for k in ("W", "H", "W2", "H2", "lmax", "lam", "G", "h", "w")})
        Ag = O.aggregate(views["levels"][lv - 1]["cp"].cpu().numpy().astype(np.float64), lv, gp)
    cpg = views["levels"][lv]["cp"].cpu().numpy()
    cdg = views["levels"][lv]["code"].cpu().numpy()

    def cands(M, b, a, ry, rx):
        out = []
        for my in (-1, 0, 1):
            for mx in (-1, 0, 1):
                y, x = 2 * ry + my, 2 * rx + mx
                ok = M is not None and 0 <= y < M.shape[2] and 0 <= x < M.shape[3]
                out.append(round(float(M[b, a, y, x]), 8) if ok else None)
        return out

    for b, a, ry, rx in where:
        print(f"level {lv} patch ({b},{a}) r=({ry},{rx}): oracle code {pyr.code[lv][b, a, ry, rx]} "
              f"value {pyr.Cp[lv][b, a, ry, rx]!r} gap {pyr.gap[lv][b, a, ry, rx]!r}; gpu code {cdg[b, a, ry, rx]} "
              f"value {cpg[b, a, ry, rx]!r}\n  oracle A {cands(A, b, a, ry, rx)}\n  from gpu {cands(Ag, b, a, ry, rx)}",
              flush=True)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_descriptors_match_oracle(name):
    o = oracle_pair(name)
    p = synth.make_pair(name)
    for img, ref in ((p["img1"], o["D1"]), (p["img2"], o["D2"])):
        d = dm.descriptors(cuda(img)).cpu().numpy()
        np.testing.assert_allclose(d, ref, rtol=0, atol=3e-6)


@functools.lru_cache(maxsize=None)
def odd_case():
    """Uneven crops of the 512x256 pair, I 310x150 and I' 300x156: the level
    maps are 150, 75, 38, ... wide, so the streaming kernels run on widths
    that are not multiples of 4 (scalar loads) and on odd widths."""
    p = synth.make_pair("c3")
    i1 = np.ascontiguousarray(p["img1"][40:190, 60:370])
    i2 = np.ascontiguousarray(p["img2"][37:193, 66:366])
    o = oracle_from_desc(O.descriptors(i1), O.descriptors(i2))
    o["img1"], o["img2"] = i1, i2
    return o


@functools.lru_cache(maxsize=None)
def narrow_case():
    """Crops I 168x120 and I' 200x148: level 1 maps are 100 wide (a multiple
    of 4) and pool to 50 x 37, the narrow streaming form whose two lane
    groups walk bands of 10 rows, the last one ragged (7 rows)."""
    p = synth.make_pair("c3")
    i1 = np.ascontiguousarray(p["img1"][60:180, 100:268])
    i2 = np.ascontiguousarray(p["img2"][50:198, 90:290])
    o = oracle_from_desc(O.descriptors(i1), O.descriptors(i2))
    o["img1"], o["img2"] = i1, i2
    return o


@functools.lru_cache(maxsize=None)
def wide_case(w2):
    """I 96x72 against I' w2 x 72, I a window of I' before a smooth warp of up
    to 10 px: level 1 maps are w2 / 2 wide and pool to w2 / 4 columns, so the
    streaming level form runs a second column tile; at w2 = 540 (maps 270
    wide, not a multiple of 4) that is the coalesced form, also at level 2
    (135 wide), and at w2 = 544 the 4-columns-per-lane form."""
    rng = np.random.default_rng(707)
    big = synth.blurred_noise(rng, 72, w2)
    field = synth.smooth_field(rng, 72, w2, 10.0)
    i2 = np.ascontiguousarray(synth.warp_bilinear(big, field))
    i1 = np.ascontiguousarray(big[:, 200:296])
    o = oracle_from_desc(O.descriptors(i1), O.descriptors(i2))
    o["img1"], o["img2"] = i1, i2
    return o


def case(name):
    if name == "odd":
        return odd_case(), 0
    if name == "narrow":
        return narrow_case(), 0
    if name.startswith("wide"):
        return wide_case(int(name[4:])), 0
    if name.startswith("random"):
        return random_shape_case(int(name[6:])), 0
    return oracle_pair(name), synth.CONFIG_NMAX[name]


@pytest.mark.parametrize("name", ["c1", "c2", "odd", "narrow", "wide540", "wide544"])
def test_pyramid_levels_match_oracle(name):
    o, mp = case(name)
    pyr = o["pyr"]
    gpu, views, pl = run_desc(o["D1"], o["D2"], max_patch=mp)
    assert pl.lmax == pyr.lmax
    for lv in range(pyr.lmax):
        G = pyr.G[lv]
        cp = views["levels"][lv]["cp"].cpu().numpy()[G]
        code = views["levels"][lv]["code"].cpu().numpy()[G]
        ref = pyr.Cp[lv][G]
        print(f"level {lv}: max rel err {np.max(np.abs(cp - ref) / np.maximum(ref, 1e-30)):.3e}", flush=True)
        np.testing.assert_allclose(cp, ref, rtol=1e-5, atol=1e-7, err_msg=f"level {lv}")
        # Codes are compared where the oracle's decision has a clear margin.
        # Exact FP64 ties (one value shared by overlapping windows) are left
        # out: an FP32 near-tie one level down can make the two shared inputs
        # differ by an ulp and break the tie the other way.
        raw = pyr.gap[lv][G]
        clear = raw > FP32_TIE * (1 + ref)
        ties = (raw == 0) & (code != pyr.code[lv][G])
        print(f"level {lv}: exact oracle ties resolved differently: {int(ties.sum())} / {int((raw == 0).sum())}",
              flush=True)
        mism = (code != pyr.code[lv][G]) & clear
        if mism.sum():
            pidx, mry, mrx = np.nonzero(mism)
            bas = np.argwhere(G)[pidx]
            explain_code_mismatch(pyr, lv, views, [(int(p[0]), int(p[1]), int(y), int(x))
                                                   for p, y, x in zip(bas[:5], mry[:5], mrx[:5])])
        assert mism.sum() == 0, f"level {lv}: {mism.sum()} codes differ away from near-ties"
        print(f"level {lv}: codes compared {clear.sum()} / {clear.size}", flush=True)
    G = pyr.G[pyr.lmax]
    np.testing.assert_allclose(views["top"].cpu().numpy()[G], pyr.top[G], rtol=1e-5, atol=1e-7)


def random_shape_case(seed):
    """Seeded sizes, I in [40, 140] x [32, 96], I' in [60, 300] x [40, 160]:
    crops of one blurred-noise image, I' warped by up to 6 px, so that level
    maps of every width class occur (not a multiple of 4, narrow, tiled)."""
    rng = np.random.default_rng(9000 + seed)
    W1, H1 = int(rng.integers(40, 141)), int(rng.integers(32, 97))
    W2, H2 = int(rng.integers(60, 301)), int(rng.integers(40, 161))
    Wb, Hb = max(W1, W2) + 16, max(H1, H2) + 16
    base = synth.blurred_noise(rng, Hb, Wb)
    warped = synth.warp_bilinear(base, synth.smooth_field(rng, Hb, Wb, 6.0))
    i1 = np.ascontiguousarray(base[4:4 + H1, 6:6 + W1])
    i2 = np.ascontiguousarray(warped[7:7 + H2, 3:3 + W2])
    return oracle_from_desc(O.descriptors(i1), O.descriptors(i2))


@pytest.mark.parametrize("seed", range(10))
def test_random_shapes_match_oracle(seed):
    o = random_shape_case(seed)
    pyr = o["pyr"]
    gpu, views, pl = run_desc(o["D1"], o["D2"])
    assert pl.lmax == pyr.lmax
    for lv in range(pyr.lmax):
        G = pyr.G[lv]
        cp = views["levels"][lv]["cp"].cpu().numpy()[G]
        code = views["levels"][lv]["code"].cpu().numpy()[G]
        ref = pyr.Cp[lv][G]
        np.testing.assert_allclose(cp, ref, rtol=1e-5, atol=1e-7, err_msg=f"seed {seed} level {lv}")
        clear = pyr.gap[lv][G] > FP32_TIE * (1 + ref)
        assert ((code != pyr.code[lv][G]) & clear).sum() == 0, f"seed {seed} level {lv}: codes differ"
    G = pyr.G[pyr.lmax]
    np.testing.assert_allclose(views["top"].cpu().numpy()[G], pyr.top[G], rtol=1e-5, atol=1e-7)
    r = compare_matches(gpu, o["out"], o["margin"])
    report(f"random shape {seed} {o['D1'].shape[:2]} {o['D2'].shape[:2]}", r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]


@pytest.mark.parametrize("name", ["c1", "c2", "odd", "narrow", "wide540", "wide544"])
def test_matches_fp32_match_oracle(name):
    o, mp = case(name)
    gpu, _, _ = run_desc(o["D1"], o["D2"], max_patch=mp)
    r = compare_matches(gpu, o["out"], o["margin"])
    report(name, r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]
    # order (y1, x1) and at most one match per atomic patch / target cell
    keys = gpu[:, 1] * 1e6 + gpu[:, 0]
    assert (np.diff(keys) > 0).all()
    assert len(np.unique(gpu[:, 2:4] // 4, axis=0)) == len(gpu)


def test_match_images_end_to_end_c1():
    o = oracle_pair("c1")
    p = o["pair"]
    m = dm.match_images(cuda(p["img1"]), cuda(p["img2"]), dm.params(max_patch=32)).cpu().numpy()
    r = compare_matches(m, o["out"], o["margin"], tie=1e-4)
    report("c1 images", r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    x1, y1 = m[:, 0], m[:, 1]
    inner = (x1 >= 8) & (x1 < 64 - 13) & (y1 >= 11) & (y1 < 56)
    assert ((m[inner, 2] - x1[inner] == 5) & (m[inner, 3] - y1[inner] == -3)).all()


@pytest.mark.parametrize("W1,H1,W2,H2,mp", [(4, 4, 4, 4, 0), (8, 8, 5, 3, 0), (9, 5, 3, 2, 0), (37, 23, 19, 41, 0),
                                             (41, 19, 37, 23, 16), (64, 40, 50, 70, 0), (30, 30, 30, 30, 8)])
def test_ragged_and_tiny_shapes(W1, H1, W2, H2, mp):
    rng = np.random.default_rng(W1 * 1000 + H1 * 10 + W2)
    i1 = synth.blurred_noise(rng, H1, W1)
    i2 = synth.blurred_noise(rng, H2, W2)
    D1 = O.descriptors(i1)
    D2 = O.descriptors(i2)
    o = oracle_from_desc(D1, D2, mp)
    gpu, _, pl = run_desc(D1, D2, max_patch=mp)
    assert pl.lmax == o["pyr"].lmax
    r = compare_matches(gpu, o["out"], o["margin"])
    report(f"{W1}x{H1}/{W2}x{H2}", r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]


def test_identity_pair_matches_itself():
    img = synth.make_pair("c1")["img1"]
    D = O.descriptors(img)
    gpu, _, _ = run_desc(D, D, max_patch=32)
    assert len(gpu) == 256
    np.testing.assert_array_equal(gpu[:, 0:2], gpu[:, 2:4])


@pytest.mark.parametrize("W1,H1,W2,H2", [(64, 64, 64, 64), (100, 76, 90, 70), (256, 192, 256, 192)])
def test_images_entry_equals_descriptors_entry_bf16(W1, H1, W2, H2):
    """With the library's own descriptors (mu > 0) every bottom correlation
    inside I' is positive, and the images entry point runs the bottom kernel
    without its clamp at 0; matching the same descriptors through the
    descriptors entry point (clamp kept) gives the same pooled maps, codes
    and matches bit for bit.  Widths whose pooled maps are and are not
    multiples of 16 (staged and direct code stores)."""
    rng = np.random.default_rng(W1 + H2)
    i1 = synth.blurred_noise(rng, H1, W1)
    i2 = synth.blurred_noise(rng, H2, W2)
    prm = dm.params(precision="bf16")
    mi, wsi, pli = dm.match_images(cuda(i1), cuda(i2), prm, return_state=True)
    d1, d2 = dm.descriptors(cuda(i1)), dm.descriptors(cuda(i2))
    md, wsd, pld = dm.match_descriptors(d1, d2, prm, return_state=True)
    torch.cuda.synchronize()
    vi, vd = dm.workspace_views(wsi, pli), dm.workspace_views(wsd, pld)
    for lv in range(pli.lmax):
        assert torch.equal(vi["levels"][lv]["cp"], vd["levels"][lv]["cp"]), lv
        assert torch.equal(vi["levels"][lv]["code"], vd["levels"][lv]["code"]), lv
    assert torch.equal(mi, md)


def test_deterministic():
    o = oracle_pair("c1")
    a, va, _ = run_desc(o["D1"], o["D2"], max_patch=32)
    b, vb, _ = run_desc(o["D1"], o["D2"], max_patch=32)
    np.testing.assert_array_equal(a, b)
    for la, lb in zip(va["levels"], vb["levels"]):
        assert torch.equal(la["cp"], lb["cp"]) and torch.equal(la["code"], lb["code"])


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_bf16_agreement(name):
    o = oracle_pair(name)
    gpu, _, _ = run_desc(o["D1"], o["D2"], max_patch=synth.CONFIG_NMAX[name], precision="bf16")
    frac = within_px(gpu, o["out"], 1.0)
    print(f"{name} bf16: {len(gpu)} matches, {frac:.4f} of oracle matches within 1 px", flush=True)
    assert frac >= 0.99


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_warped_pair_recovers_the_ground_truth_field(prec):
    """Images in, matches out on the 256x192 warped pair c2: the GPU's
    matches follow the true displacement field as closely as the oracle's
    (bounds set from the oracle's run; the oracle test holds it to them)."""
    from tests.helpers import GT_WITHIN_1PX_ALL, GT_WITHIN_1PX_CLEAR, ground_truth_agreement
    o = oracle_pair("c2")
    p = o["pair"]
    m = dm.match_images(cuda(p["img1"]), cuda(p["img2"]), dm.params(precision=prec, max_patch=64)).cpu().numpy()
    fa, fc, n = ground_truth_agreement(m, p)
    ra, rc, _ = ground_truth_agreement(o["out"], p)
    print(f"c2 {prec}: {len(m)} matches, {fa:.4f} within 1 px of the true field ({fc:.4f} of {n} clear); "
          f"oracle {ra:.4f} ({rc:.4f})", flush=True)
    assert fc >= GT_WITHIN_1PX_CLEAR and fa >= GT_WITHIN_1PX_ALL
    assert fc >= rc - 0.01 and fa >= ra - 0.01


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), kept as float64: the
    values a BF16 operand holds exactly."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@functools.lru_cache(maxsize=None)
def bf16_operand_case(name):
    o, mp = case(name)
    return oracle_from_desc(bf16_round(o["D1"]), bf16_round(o["D2"]), mp), mp


@pytest.mark.parametrize("name", ["c1", "c2", "odd", "narrow", "wide540"] + [f"random{k}" for k in range(5)])
def test_bf16_pyramid_equals_oracle_on_bf16_operands(name):
    """The BF16 path on descriptors that BF16 holds exactly against the FP64
    oracle on the same values, element by element.  Products of BF16 values
    are exact in FP32 and the descriptors are non-negative, so the level-0
    correlation differs from the oracle's only by FP32 accumulation over
    K = 160 (about 1e-5 relative at worst) and the 4 mantissa bits the
    pooling keys drop (2^-19), raised to lambda; the upper levels add FP32
    rounding.  Codes are compared where the oracle's margin exceeds that.
    The odd and narrow crops pool to 150 x 78 and 100 x 74 entries, so the
    bottom kernel's last 16-column step and last 8-row band are partial."""
    o, mp = bf16_operand_case(name)
    pyr = o["pyr"]
    gpu, views, pl = run_desc(o["D1"], o["D2"], max_patch=mp, precision="bf16")
    assert pl.lmax == pyr.lmax
    tie = 5e-5
    for lv in range(pyr.lmax):
        G = pyr.G[lv]
        cp = views["levels"][lv]["cp"].cpu().numpy()[G]
        code = views["levels"][lv]["code"].cpu().numpy()[G]
        ref = pyr.Cp[lv][G]
        print(f"{name} bf16 level {lv}: max rel err {np.max(np.abs(cp - ref) / np.maximum(ref, 1e-30)):.3e}",
              flush=True)
        np.testing.assert_allclose(cp, ref, rtol=3e-5, atol=1e-7, err_msg=f"level {lv}")
        clear = pyr.gap[lv][G] > tie * (1 + ref)
        mism = (code != pyr.code[lv][G]) & clear
        assert mism.sum() == 0, f"level {lv}: {mism.sum()} codes differ away from near-ties"
    G = pyr.G[pyr.lmax]
    np.testing.assert_allclose(views["top"].cpu().numpy()[G], pyr.top[G], rtol=3e-5, atol=1e-7)
    r = compare_matches(gpu, o["out"], o["margin"], tie=tie, score_rtol=3e-5)
    report(f"{name} bf16 operands", r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]


def load_golden(name):
    import os
    from tests.golden.make_golden import image_hash, path_of
    path = path_of(name)
    if not os.path.exists(path):
        pytest.skip(f"{path} missing (tests/golden/make_golden.py {name} writes it)")
    z = np.load(path)
    p = synth.make_pair(name)
    assert image_hash(p["img1"], p["img2"]) == str(z["sha256"]), "regenerated inputs differ from the stored ones"
    return p, z["matches"], z["margin"], int(z["lmax"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_512x256_against_stored_oracle(prec):
    """Images in, matches out at 512x256 (the benchmark workload and launch
    configuration) against the oracle's matches stored by make_golden.py."""
    p, ref, margin, lmax = load_golden("c3")
    m, ws, pl = dm.match_images(cuda(p["img1"]), cuda(p["img2"]), dm.params(precision=prec), return_state=True)
    m = m.cpu().numpy()
    assert pl.lmax == lmax
    if prec == "fp32":
        r = compare_matches(m, ref, margin, tie=1e-4)
        report("c3 fp32", r)
        assert not r["missing"] and not r["moved"] and not r["bad_score"]
        assert len(r["extra"]) <= r["near_ties"]
    else:
        frac = within_px(m, ref, 1.0)
        exact = within_px(m, ref, 0.0)
        print(f"c3 bf16: {len(m)} matches vs {len(ref)}; within 1 px {frac:.4f}, exact {exact:.4f}", flush=True)
        assert frac >= 0.99
