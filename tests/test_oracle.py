"""Pins of the FP64 oracle against what the paper and the mathematics fix:
closed forms, library routines, brute force on tiny inputs, invariants and the
paper's one worked example (Sec. 3.2, "Boundary effects").  CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import dm_oracle as O
from tests import torch_ref as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_desc(rng, h, w):
    d = rng.random((h, w, 9)) + 0.05
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


# ---------------------------------------------------------------- descriptor

def test_gaussian_taps_closed_form():
    g = O.gaussian_taps(1.0)
    t = np.arange(-3, 4)
    ref = np.exp(-t * t / 2.0)
    np.testing.assert_allclose(g, ref / ref.sum(), rtol=1e-15)
    assert len(O.gaussian_taps(1.5)) == 2 * 5 + 1


def test_smooth_constant_and_impulse():
    c = np.full((20, 17), 3.25)
    np.testing.assert_allclose(O.smooth(c, 1.0), c, rtol=1e-14)
    img = np.zeros((21, 21))
    img[10, 10] = 1.0
    g = O.gaussian_taps(1.0)
    out = O.smooth(img, 1.0)
    np.testing.assert_allclose(out[7:14, 7:14], np.outer(g, g), atol=1e-16)
    assert abs(out.sum() - 1.0) < 1e-14


def test_descriptor_unit_norm_nonnegative():
    img = synth.make_pair("c1")["img1"]
    d = O.descriptors(img)
    assert d.shape == (64, 64, 9)
    np.testing.assert_allclose(np.linalg.norm(d, axis=-1), 1.0, rtol=1e-14)
    assert (d >= 0).all()


def test_descriptor_flat_region_is_mu_axis():
    """No gradient -> (0,...,0,1): flat areas still correlate (value 1)."""
    d = O.descriptors(np.full((16, 16), 0.4))
    ref = np.zeros(9)
    ref[8] = 1.0
    np.testing.assert_array_equal(d.reshape(-1, 9), np.tile(ref, (256, 1)))


def test_descriptor_ramp_closed_form():
    """Horizontal ramp, no smoothing: interior gradient (255*alpha, 0)."""
    alpha = 0.01
    img = alpha * np.tile(np.arange(24, dtype=np.float64), (10, 1))
    prm = O.Params(nu1=0, nu2=0, nu3=0, slope=0.2, mu=0.1)
    d = O.descriptors(img, prm)
    g = 255.0 * alpha
    proj = np.array([max(0.0, g * math.cos(k * math.pi / 4)) for k in range(1, 9)])
    sig = 2.0 / (1.0 + np.exp(-0.2 * proj)) - 1.0
    v = np.append(sig, 0.1)
    v /= np.linalg.norm(v)
    np.testing.assert_allclose(d[5, 12], v, atol=1e-15)
    # orientation bins 1, 7 (at 45 deg) share, bin 8 (0 deg) is the largest
    assert d[5, 12, 7] > d[5, 12, 0] > 0 and abs(d[5, 12, 0] - d[5, 12, 6]) < 1e-15


def test_descriptor_rotation_permutes_bins():
    """Rotating the image by 90 deg rotates the gradient by -90 deg (y down),
    which maps orientation bin k to bin k+2."""
    img = synth.make_pair("c1")["img1"][:40, :32].astype(np.float64)
    d = O.descriptors(img)
    dr = O.descriptors(np.rot90(img))
    rot = np.rot90(d)
    for c in range(8):
        np.testing.assert_allclose(dr[..., c], rot[..., (c + 2) % 8], atol=1e-13)
    np.testing.assert_allclose(dr[..., 8], rot[..., 8], atol=1e-13)


# ---------------------------------------------------------------- bottom level

def test_bottom_equals_conv2d():
    rng = np.random.default_rng(1)
    D1 = rand_desc(rng, 13, 18)
    D2 = rand_desc(rng, 11, 15)
    A = O.bottom_scores(D1, D2)
    ref = T.bottom(torch.from_numpy(D1), torch.from_numpy(D2)).numpy()
    assert A.shape == ref.shape == (3, 4, 11, 15)
    np.testing.assert_allclose(A, ref, rtol=1e-13, atol=1e-15)


def test_bottom_bruteforce_tiny():
    rng = np.random.default_rng(2)
    D1 = rng.standard_normal((8, 9, 9))
    D2 = rng.standard_normal((6, 5, 9))
    A = O.bottom_scores(D1, D2)
    for b, a in itertools.product(range(2), range(2)):
        py, px = 2 + 4 * b, 2 + 4 * a
        for y in range(6):
            for x in range(5):
                acc = 0.0
                for i in range(4):
                    for j in range(4):
                        yy, xx = y - 2 + i, x - 2 + j
                        if 0 <= yy < 6 and 0 <= xx < 5:
                            acc += D1[py - 2 + i, px - 2 + j] @ D2[yy, xx]
                assert abs(A[b, a, y, x] - acc / 16) < 1e-13


def test_bottom_bounds_and_identity():
    img = synth.make_pair("c1")["img1"]
    D = O.descriptors(img)
    A = O.bottom_scores(D, D)
    assert A.max() <= 1 + 1e-12                      # Cauchy-Schwarz on unit vectors
    ny, nx = A.shape[:2]
    for b in range(ny):
        for a in range(nx):
            assert abs(A[b, a, 2 + 4 * b, 2 + 4 * a] - 1.0) < 1e-14


# ---------------------------------------------------------------- pooling

def test_pool_equals_max_pool2d():
    rng = np.random.default_rng(3)
    C = rng.random((5, 13, 18))
    v, code, _ = O.pool_subsample(C)
    tv, tcode = T.pool(torch.from_numpy(C))
    np.testing.assert_array_equal(v, tv.numpy())
    np.testing.assert_array_equal(code, tcode.numpy())


def test_pool_ties_first_in_order():
    rng = np.random.default_rng(4)
    C = rng.integers(0, 3, size=(4, 7, 9)).astype(float)
    v, code, gap = O.pool_subsample(C)
    for i in range(4):
        for ry in range(4):
            for rx in range(5):
                cands = [(C[i, 2 * ry + my, 2 * rx + mx], 3 * (my + 1) + mx + 1)
                         for my in (-1, 0, 1) for mx in (-1, 0, 1)
                         if 0 <= 2 * ry + my < 7 and 0 <= 2 * rx + mx < 9]
                m = max(c[0] for c in cands)
                assert v[i, ry, rx] == m
                assert code[i, ry, rx] == min(k for val, k in cands if val == m)
                srt = sorted((c[0] for c in cands), reverse=True)
                assert gap[i, ry, rx] == srt[0] - srt[1]


# ---------------------------------------------------------------- grids

@pytest.mark.parametrize("W,H", [(64, 64), (256, 192), (621, 188), (37, 23), (8, 8)])
def test_grids_match_centre_sets(W, H):
    lmax = int(math.log2(1024 // 4))
    G = O.grids(W, H, lmax)
    S = T.centre_sets(W, H, lmax)
    for lv in range(lmax + 1):
        cy, cx = O.lattice_centres(lv, W, H)
        got = {(int(cx[a]), int(cy[b])) for b, a in zip(*np.nonzero(G[lv]))}
        assert got == S[lv], lv


def test_grid_holes_and_cap_for_driving_half_frame():
    """621x188: the loop bound gives N=1024, whose grid is empty; N=512 has
    row holes; the top is capped at N=512 (R7)."""
    G = O.grids(621, 188, 8)
    assert not G[8].any()
    rows = np.nonzero(G[7].any(1))[0] * 4
    assert rows.min() == 0 and rows.max() == 184 and len(rows) < 47
    assert O.pyramid_top(621, 188) == 7
    assert O.pyramid_top(512, 256) == 7 and O.pyramid_top(256, 192) == 6
    assert O.pyramid_top(64, 64, 32) == 3


def test_boundary_worked_example():
    """Sec. 3.2, "Boundary effects": the patch centred at (0,0) has the single
    child i=3 and its average carries that child with weight 1."""
    with open(os.path.join(GOLDEN, "boundary_example.json")) as f:
        ex = json.load(f)
    rng = np.random.default_rng(5)
    D1, D2 = rand_desc(rng, 40, 40), rand_desc(rng, 24, 28)
    prm = O.Params(max_patch=32)
    pyr = O.pyramid(D1, D2, prm, keep_full=True)
    for lv in range(1, pyr.lmax + 1):
        assert pyr.G[lv][0, 0]
        ox, oy = O.OFFSETS[ex["valid_child"]]
        children = []
        for i, (cx_, cy_) in enumerate(O.OFFSETS):
            b, a, ok = O.lattice_index(lv - 1, 40, 40, (2 ** lv) * cy_, (2 ** lv) * cx_)
            if ok and pyr.G[lv - 1][b, a]:
                children.append(i)
        assert children == [ex["valid_child"]]
        b, a, _ = O.lattice_index(lv - 1, 40, 40, (2 ** lv) * oy, (2 ** lv) * ox)
        child = pyr.Cp[lv - 1][b, a]
        h, w = child.shape
        expect = np.zeros((h, w))
        expect[:h - 1, :w - 1] = ex["weight"] * child[1:, 1:]
        np.testing.assert_array_equal(pyr.A[lv][0, 0], expect)


# ---------------------------------------------------------------- pyramid

def test_pyramid_matches_torch_reexpression():
    rng = np.random.default_rng(6)
    D1, D2 = rand_desc(rng, 26, 21), rand_desc(rng, 23, 18)
    prm = O.Params(max_patch=32)
    pyr = O.pyramid(D1, D2, prm)
    levels, top, _ = T.forward(torch.from_numpy(D1), torch.from_numpy(D2), 1.4, pyr.lmax)
    for lv in range(pyr.lmax):
        pooled, codes = levels[lv]
        cy, cx = O.lattice_centres(lv, 21, 26)
        for (x, y), v in pooled.items():
            b, a = np.nonzero(cy == y)[0][0], np.nonzero(cx == x)[0][0]
            np.testing.assert_allclose(pyr.Cp[lv][b, a], v.numpy(), rtol=1e-13, atol=1e-15)
            np.testing.assert_array_equal(pyr.code[lv][b, a], codes[(x, y)].numpy())
    cy, cx = O.lattice_centres(pyr.lmax, 21, 26)
    assert len(top) == pyr.G[pyr.lmax].sum()
    for (x, y), v in top.items():
        b, a = np.nonzero(cy == y)[0][0], np.nonzero(cx == x)[0][0]
        np.testing.assert_allclose(pyr.top[b, a], v.numpy(), rtol=1e-13, atol=1e-15)


def test_joint_quadrant_max_at_N8():
    """Eq. (1): the joint maximum over all 9^|V| child placements of the mean
    child score equals the factorised recursion (Eq. (2)/(12)) at N=8."""
    rng = np.random.default_rng(7)
    D1, D2 = rand_desc(rng, 16, 16), rand_desc(rng, 14, 13)
    pyr = O.pyramid(D1, D2, O.Params(max_patch=8), keep_full=True)
    C0 = O.rectify(pyr.A[0], 1.4)
    h1, w1 = pyr.h[1], pyr.w[1]
    cy, cx = O.lattice_centres(1, 16, 16)
    for b, a in [(0, 0), (1, 2), (3, 3), (2, 1)]:
        for qy, qx in [(0, 0), (3, 4), (6, 6), (5, 0)]:
            kids = []
            for ox, oy in O.OFFSETS:
                cb, ca, ok = O.lattice_index(0, 16, 16, cy[b] + 2 * oy, cx[a] + 2 * ox)
                if ok:
                    kids.append((cb, ca, qy + oy, qx + ox))
            best = -np.inf
            for ms in itertools.product(itertools.product((-1, 0, 1), repeat=2), repeat=len(kids)):
                tot, okall = 0.0, True
                for (cb, ca, ry, rx), (my, mx) in zip(kids, ms):
                    if not (0 <= ry < h1 and 0 <= rx < w1):
                        continue                     # child read outside the map: 0 (R5)
                    y, x = 2 * ry + my, 2 * rx + mx
                    if not (0 <= y < 14 and 0 <= x < 13):
                        okall = False
                        break
                    tot += C0[cb, ca, y, x]
                if okall:
                    best = max(best, tot / len(kids))
            assert abs(pyr.A[1][b, a, qy, qx] - best) < 1e-13


def test_recursion_in_image_coordinates():
    """Eq. (6) evaluated top-down in pixel coordinates: child i of a patch
    matched at pixel x is searched in the window of radius N/8 centred at
    x + (N/4) o_i, on the subsampled lattice of its level."""
    rng = np.random.default_rng(8)
    W = H = 24
    D1, D2 = rand_desc(rng, H, W), rand_desc(rng, 22, 20)
    pyr = O.pyramid(D1, D2, O.Params(max_patch=32), keep_full=True)
    C0 = O.rectify(pyr.A[0], 1.4)
    memo = {}

    def F(lv, cxy, X):       # C_{N,p}(X), X a pixel position (multiple of 2^lv)
        key = (lv, cxy, X)
        if key in memo:
            return memo[key]
        if lv == 0:
            b, a, _ = O.lattice_index(0, W, H, cxy[1], cxy[0])
            v = C0[b, a, X[1], X[0]]
        else:
            step = 2 ** (lv - 1)
            N = 4 * 2 ** lv
            terms = []
            for ox, oy in O.OFFSETS:
                c = (cxy[0] + (N // 4) * ox, cxy[1] + (N // 4) * oy)
                b, a, ok = O.lattice_index(lv - 1, W, H, c[1], c[0])
                if not (ok and pyr.G[lv - 1][b, a]):
                    continue
                centre = (X[0] + (N // 4) * ox, X[1] + (N // 4) * oy)
                if not (0 <= centre[0] < 2 ** lv * pyr.w[lv] and 0 <= centre[1] < 2 ** lv * pyr.h[lv]):
                    terms.append(0.0)
                    continue
                best = -np.inf
                for my in (-1, 0, 1):
                    for mx in (-1, 0, 1):
                        Y = (centre[0] + mx * step, centre[1] + my * step)
                        if 0 <= Y[0] < step * pyr.w[lv - 1] and 0 <= Y[1] < step * pyr.h[lv - 1]:
                            best = max(best, F(lv - 1, c, Y))
                terms.append(best)
            v = max(sum(terms) / len(terms), 0.0) ** 1.4
        memo[key] = v
        return v

    for lv in (1, 2, 3):
        cy, cx = O.lattice_centres(lv, W, H)
        for b, a in [(0, 0), (2, 3), (5, 5), (3, 1)]:
            if not pyr.G[lv][b, a]:
                continue
            C = O.rectify(pyr.A[lv], 1.4)
            for qy in range(0, pyr.h[lv], 2):
                for qx in range(0, pyr.w[lv], 3):
                    v = F(lv, (int(cx[a]), int(cy[b])), (qx * 2 ** lv, qy * 2 ** lv))
                    assert abs(C[b, a, qy, qx] - v) < 1e-13


def test_identity_pair_top_is_one():
    img = synth.make_pair("c1")["img1"]
    D = O.descriptors(img)
    pyr = O.pyramid(D, D, O.Params(max_patch=32))
    G = pyr.G[pyr.lmax]
    cy, cx = O.lattice_centres(pyr.lmax, 64, 64)
    for b, a in zip(*np.nonzero(G)):
        m = pyr.top[b, a]
        assert abs(m.max() - 1.0) < 1e-12
        qy, qx = np.unravel_index(np.argmax(m), m.shape)
        assert abs(qy * 2 ** pyr.lmax - cy[b]) <= 2 ** pyr.lmax
        assert abs(qx * 2 ** pyr.lmax - cx[a]) <= 2 ** pyr.lmax


@pytest.mark.parametrize("noise", [False, True])
def test_translation_recovered(noise):
    p = synth.make_pair("c1")
    i1 = p["img1"].astype(np.float64)
    i2 = synth.shift_reflect(i1, 5, -3) if not noise else p["img2"].astype(np.float64)
    out, margin, pyr, M = O.match(i1, i2, O.Params(max_patch=32))
    x1, y1 = out[:, 0], out[:, 1]
    inner = (x1 >= 8) & (x1 < 64 - 8 - 5) & (y1 >= 8 + 3) & (y1 < 64 - 8)
    assert inner.sum() > 100
    assert (out[inner, 2] == x1[inner] + 5).all() and (out[inner, 3] == y1[inner] - 3).all()
    # at most one match per atomic patch and per 4x4 target cell (Eq. (16))
    assert len(np.unique(out[:, :2], axis=0)) == len(out)
    assert len(np.unique(out[:, 2:4] // 4, axis=0)) == len(out)


def test_warped_pair_recovers_the_ground_truth_field():
    """End to end on the 256x192 warped pair c2: the oracle's matches follow
    the true displacement field (the inverse of the smooth warp that made
    I') to within 1 px, except in the periodic rectangle, where the texture
    repeats every 8 px, and near the borders."""
    from tests.helpers import GT_WITHIN_1PX_ALL, GT_WITHIN_1PX_CLEAR, ground_truth_agreement, oracle_pair
    o = oracle_pair("c2")
    frac_all, frac_clear, n_clear = ground_truth_agreement(o["out"], o["pair"])
    print(f"c2 oracle: {len(o['out'])} matches, {frac_all:.4f} within 1 px of the true field, "
          f"{frac_clear:.4f} of the {n_clear} away from the periodic rectangle and the borders")
    assert n_clear > 1000
    assert frac_clear >= GT_WITHIN_1PX_CLEAR and frac_all >= GT_WITHIN_1PX_ALL


# ---------------------------------------------------------------- backtracking

def _enumerate(pyr, lv, b, a, qy, qx, s, path, out):
    """B applied recursively without merging (Eq. (14))."""
    W, H = pyr.W, pyr.H
    if lv == 0:
        out.append((b, a, qy, qx, s, path))
        return
    cy, cx = O.lattice_centres(lv, W, H)
    for ox, oy in O.OFFSETS:
        cb, ca, ok = O.lattice_index(lv - 1, W, H, cy[b] + (2 ** lv) * oy, cx[a] + (2 ** lv) * ox)
        cb, ca = int(cb), int(ca)
        if not (ok and pyr.G[lv - 1][cb, ca]):
            continue
        ry, rx = qy + oy, qx + ox
        if not (0 <= ry < pyr.h[lv] and 0 <= rx < pyr.w[lv]):
            continue
        k = int(pyr.code[lv - 1][cb, ca, ry, rx])
        ny, nx = 2 * ry + k // 3 - 1, 2 * rx + k % 3 - 1
        assert (ny - 2 * (qy + oy), nx - 2 * (qx + ox)) in {(m, n) for m in (-1, 0, 1) for n in (-1, 0, 1)}
        _enumerate(pyr, lv - 1, cb, ca, ny, nx, s + pyr.Cp[lv - 1][cb, ca, ry, rx],
                   path + [(lv, b, a, qy, qx)], out)


def test_backtracking_equals_unmerged_enumeration():
    rng = np.random.default_rng(9)
    img1 = synth.blurred_noise(rng, 24, 24)
    img2 = synth.shift_reflect(img1, 1, 2) + rng.normal(0, 0.05, (24, 24))
    prm = O.Params(max_patch=16)
    D1, D2 = O.descriptors(img1, prm), O.descriptors(img2, prm)
    pyr = O.pyramid(D1, D2, prm)
    assert pyr.lmax == 2
    leaves = []
    nfull = 0
    cy, cx = O.lattice_centres(2, 24, 24)
    for b, a in zip(*np.nonzero(pyr.G[2])):
        b, a = int(b), int(a)
        for qy in range(pyr.h[2]):
            for qx in range(pyr.w[2]):
                before = len(leaves)
                _enumerate(pyr, 2, b, a, qy, qx, pyr.top[b, a, qy, qx], [], leaves)
                # all 16 descendants exist and stay inside the maps
                if cx[a] in (8, 12) and cy[b] in (8, 12) and qy in (2, 3) and qx in (2, 3):
                    assert len(leaves) - before == 4 ** 2         # 4^(log2(N/4)) atomic tuples
                    nfull += 1
                # rigid position of each leaf within 2^l - 1 px (deformation bound)
                for lb, la, ly, lx, _, _ in leaves[before:]:
                    ry = ly - (2 + 4 * lb - cy[b] + qy * 4)
                    rx = lx - (2 + 4 * la - cx[a] + qx * 4)
                    assert max(abs(ry), abs(rx)) <= 2 ** 2 - 1
    assert nfull > 0
    best = {}
    for lb, la, ly, lx, s, _ in leaves:
        k = (lb, la, ly, lx)
        best[k] = max(best.get(k, -np.inf), s)
    M = O.backtrack(pyr)
    got = {(b, a, y, x): s for b, a, y, x, s in zip(M["b"], M["a"], M["qy"], M["qx"], M["s"])}
    assert set(got) == set(best)
    for k in best:
        assert abs(got[k] - best[k]) < 1e-13


def test_scores_are_path_sums():
    """Each merged score equals the top value plus the pooled values along the
    path recovered by re-running the argmax undo (R11)."""
    p = synth.make_pair("c1")
    prm = O.Params(max_patch=32)
    D1, D2 = O.descriptors(p["img1"], prm), O.descriptors(p["img2"], prm)
    pyr = O.pyramid(D1, D2, prm)
    M = O.backtrack(pyr)
    rng = np.random.default_rng(10)
    top_b, top_a = np.nonzero(pyr.G[pyr.lmax])
    for j in rng.choice(len(top_b), 5, replace=False):
        b, a = top_b[j], top_a[j]
        leaves = []
        _enumerate(pyr, pyr.lmax, b, a, 1, 1, pyr.top[b, a, 1, 1], [], leaves)
        got = {(lb, la, ly, lx): s for lb, la, ly, lx, s in zip(M["b"], M["a"], M["qy"], M["qx"], M["s"])}
        for lb, la, ly, lx, s, _ in leaves:
            assert got[(lb, la, ly, lx)] >= s - 1e-13     # merged value is the max over paths


# ---------------------------------------------------------------- DM* entry points (R24)

def test_local_maxima_bruteforce_with_plateaus():
    """Small integer maps (many equal values): the tie-broken 3 x 3 maxima
    against a literal scan of each position's neighbours; the first global
    maximum is always one, and no two of them touch."""
    rng = np.random.default_rng(31)
    for h, w in ((1, 1), (1, 5), (4, 1), (5, 6), (7, 9)):
        M = rng.integers(0, 4, size=(3, h, w)).astype(np.float64)
        mask, margin = O.local_maxima(M)
        for k in range(3):
            for y in range(h):
                for x in range(w):
                    ok = M[k, y, x] > 0
                    nb = -np.inf
                    for yy in range(y - 1, y + 2):
                        for xx in range(x - 1, x + 2):
                            if (yy, xx) == (y, x) or not (0 <= yy < h and 0 <= xx < w):
                                continue
                            nb = max(nb, M[k, yy, xx])
                            ok &= M[k, y, x] > M[k, yy, xx] if (yy, xx) < (y, x) else M[k, y, x] >= M[k, yy, xx]
                    assert bool(mask[k, y, x]) == ok, (h, w, k, y, x)
            if M[k].max() > 0:
                assert mask[k].reshape(-1)[np.argmax(M[k].reshape(-1))]
            ys, xs = np.nonzero(mask[k])
            for i in range(len(ys)):
                for j in range(i + 1, len(ys)):
                    assert max(abs(ys[i] - ys[j]), abs(xs[i] - xs[j])) >= 2
    # margins: a perturbation of every value by less than half a decision's
    # margin keeps the decision, and some decisions change under larger ones
    M = rng.random((400, 5, 6))
    mask, margin = O.local_maxima(M)
    changed = 0
    for t in range(20):
        noise = rng.uniform(-1, 1, M.shape) * 1e-2
        m2, _ = O.local_maxima(M + noise)
        keep = margin > 2e-2
        assert (m2[keep] == mask[keep]).all()
        changed += int((m2 != mask).sum())
    assert changed > 0


def test_backtracking_from_every_top_position_is_the_current_method():
    """The level-entry form of backtrack with every top position as an entry
    and no lower entries reduces to the plain backtracking exactly."""
    p = synth.make_pair("c1")
    prm = O.Params(max_patch=32)
    pyr = O.pyramid(O.descriptors(p["img1"]), O.descriptors(p["img2"]), prm)
    L = pyr.lmax
    bb, aa = np.nonzero(pyr.G[L])
    ht, wt = pyr.h[L], pyr.w[L]
    qy, qx = np.meshgrid(np.arange(ht), np.arange(wt), indexing="ij")
    b, a = np.repeat(bb, ht * wt), np.repeat(aa, ht * wt)
    qy, qx = np.tile(qy.ravel(), len(bb)), np.tile(qx.ravel(), len(bb))
    empty = tuple(np.zeros(0, dtype=t) for t in (np.int64, np.int64, np.int64, np.int64, np.float64, np.float64))
    lev = {lv: empty for lv in range(L)}
    lev[L] = (b, a, qy, qx, pyr.top[b, a, qy, qx], np.full(len(b), np.inf))
    M1, M0 = O.backtrack(pyr, level_entries=lev), O.backtrack(pyr)
    k1 = np.lexsort((M1["qx"], M1["qy"], M1["a"], M1["b"]))
    k0 = np.lexsort((M0["qx"], M0["qy"], M0["a"], M0["b"]))
    for f in ("b", "a", "qy", "qx", "s"):
        np.testing.assert_array_equal(M1[f][k1], M0[f][k0])


def test_dmstar_equals_unmerged_enumeration():
    """Every entry of every level expanded by B down to the atomic patches
    without merging (Eq. (14)), reduced by max per (p, p'): the merged DM*
    backtracking gives exactly that set and those scores."""
    rng = np.random.default_rng(9)
    img1 = synth.blurred_noise(rng, 24, 24)
    img2 = synth.shift_reflect(img1, 1, 2) + rng.normal(0, 0.05, (24, 24))
    prm = O.Params(max_patch=16)
    D1, D2 = O.descriptors(img1, prm), O.descriptors(img2, prm)
    pyr = O.pyramid(D1, D2, prm, keep_full=True)
    E = O.dmstar_entries(pyr)
    assert all(len(E[lv][0]) > 0 for lv in range(pyr.lmax + 1))
    # an entry's node is the position its pooled value came from: the
    # unpooled map holds that value there
    for lv in range(pyr.lmax):
        b, a, qy, qx, s_ = E[lv][:5]
        np.testing.assert_array_equal(O.rectify(pyr.A[lv][b, a, qy, qx], pyr.lam), s_)
    leaves = []
    for lv in range(pyr.lmax + 1):
        for b, a, qy, qx, s in zip(*E[lv][:5]):
            _enumerate(pyr, lv, int(b), int(a), int(qy), int(qx), float(s), [], leaves)
    best = {}
    for lb, la, ly, lx, s, _ in leaves:
        k = (lb, la, ly, lx)
        best[k] = max(best.get(k, -np.inf), s)
    M = O.backtrack(pyr, level_entries=E)
    got = {(b, a, y, x): s for b, a, y, x, s in zip(M["b"], M["a"], M["qy"], M["qx"], M["s"])}
    assert set(got) == set(best)
    for k in best:
        assert abs(got[k] - best[k]) < 1e-13
    # an entry below the top joins only where its own node is reached: the
    # plain method's tuples that DM* keeps carry the same or a lower score
    M0 = O.backtrack(pyr)
    plain = {(b, a, y, x): s for b, a, y, x, s in zip(M0["b"], M0["a"], M0["qy"], M0["qx"], M0["s"])}
    assert all(got[k] <= plain[k] + 1e-13 for k in got if k in plain)


def test_start_end_scoring_equals_unmerged_enumeration():
    """R26: every entry of every level expanded without merging; an atomic
    correspondence scores its entry's value plus the value of C_0 (read in the
    unpooled map) at the node its path ends on, once for a one-node path; the
    max per (p, p') is the merged start/end backtracking, tuple for tuple."""
    rng = np.random.default_rng(9)
    img1 = synth.blurred_noise(rng, 24, 24)
    img2 = synth.shift_reflect(img1, 1, 2) + rng.normal(0, 0.05, (24, 24))
    prm = O.Params(max_patch=16)
    pyr = O.pyramid(O.descriptors(img1, prm), O.descriptors(img2, prm), prm, keep_full=True)
    E = O.dmstar_entries(pyr)
    best = {}
    for lv in range(pyr.lmax + 1):
        for b, a, qy, qx, s in zip(*E[lv][:5]):
            leaves = []
            _enumerate(pyr, lv, int(b), int(a), int(qy), int(qx), 0.0, [], leaves)
            for lb, la, ly, lx, _, path in leaves:
                end = float(O.rectify(pyr.A[0][lb, la, ly, lx], pyr.lam)) if path else 0.0
                k = (lb, la, ly, lx)
                best[k] = max(best.get(k, -np.inf), float(s) + end)
    M = O.backtrack(pyr, level_entries=E, start_end=True)
    got = {(b, a, y, x): s for b, a, y, x, s in zip(M["b"], M["a"], M["qy"], M["qx"], M["s"])}
    assert set(got) == set(best)
    for k in best:
        assert abs(got[k] - best[k]) < 1e-13
    # path sums add the non-negative values in between: never below, equal
    # for paths of at most two nodes (entries at levels 0 and 1), and above
    # for many of those from higher entries
    P = O.backtrack(pyr, level_entries=E)
    ps = {(b, a, y, x): s for b, a, y, x, s in zip(P["b"], P["a"], P["qy"], P["qx"], P["s"])}
    assert set(ps) == set(got)
    assert all(ps[k] >= got[k] - 1e-13 for k in got)
    assert sum(ps[k] > got[k] + 1e-9 for k in got) > len(got) // 4


def test_start_end_scoring_recovers_translation():
    p = synth.make_pair("c1")
    i1 = p["img1"].astype(np.float64)
    i2 = synth.shift_reflect(i1, 5, -3)
    out, margin, pyr, M = O.match(i1, i2, O.Params(max_patch=32, entry_points=1, scoring=1))
    x1, y1 = out[:, 0], out[:, 1]
    inner = (x1 >= 8) & (x1 < 64 - 8 - 5) & (y1 >= 8 + 3) & (y1 < 64 - 8)
    assert inner.sum() > 100
    assert (out[inner, 2] == x1[inner] + 5).all() and (out[inner, 3] == y1[inner] - 3).all()


def test_dmstar_recovers_translation():
    p = synth.make_pair("c1")
    i1 = p["img1"].astype(np.float64)
    i2 = synth.shift_reflect(i1, 5, -3)
    out, margin, pyr, M = O.match(i1, i2, O.Params(max_patch=32, entry_points=1))
    x1, y1 = out[:, 0], out[:, 1]
    inner = (x1 >= 8) & (x1 < 64 - 8 - 5) & (y1 >= 8 + 3) & (y1 < 64 - 8)
    assert inner.sum() > 100
    assert (out[inner, 2] == x1[inner] + 5).all() and (out[inner, 3] == y1[inner] - 3).all()


# ---------------------------------------------------------------- reciprocal

def test_reciprocal_bruteforce():
    rng = np.random.default_rng(11)
    n = 400
    M = dict(b=rng.integers(0, 4, n), a=rng.integers(0, 5, n), qy=rng.integers(0, 12, n),
             qx=rng.integers(0, 14, n), s=rng.integers(0, 6, n).astype(float), margin=np.full(n, np.inf))
    key = M["b"] * 10 ** 6 + M["a"] * 10 ** 4 + M["qy"] * 100 + M["qx"]
    _, first = np.unique(key, return_index=True)           # one tuple per (p, p')
    M = {k: v[first] for k, v in M.items()}
    out, _ = O.reciprocal(M, 20, 16, 14, 12)
    tuples = list(zip(M["b"], M["a"], M["qy"], M["qx"], M["s"]))

    def best_at(b, a):
        cands = [t for t in tuples if t[0] == b and t[1] == a]
        return min(cands, key=lambda t: (-t[4], t[2], t[3]))

    def best_at2(cy, cx):
        cands = [t for t in tuples if t[2] // 4 == cy and t[3] // 4 == cx]
        return min(cands, key=lambda t: (-t[4], t[0], t[1], t[2], t[3]))

    ref = sorted({t for t in tuples if best_at(t[0], t[1]) == t == best_at2(t[2] // 4, t[3] // 4)},
                 key=lambda t: (t[0], t[1]))
    exp = np.array([[2 + 4 * t[1], 2 + 4 * t[0], t[3], t[2], t[4]] for t in ref], dtype=float)
    np.testing.assert_array_equal(out, exp)


# ---------------------------------------------------------------- gradient

def _loss(D1, D2, prm):
    return O.top_loss(O.pyramid(D1, D2, prm))


def test_gradient_central_differences():
    rng = np.random.default_rng(12)
    D1, D2 = rand_desc(rng, 12, 12), rand_desc(rng, 10, 11)
    prm = O.Params(max_patch=16)
    pyr = O.pyramid(D1, D2, prm, keep_full=True)
    g1, g2 = O.pyramid_backward(D1, D2, pyr)
    eps = 1e-6
    for D, g in ((D1, g1), (D2, g2)):
        fd = np.zeros_like(D)
        for idx in np.ndindex(D.shape):
            old = D[idx]
            D[idx] = old + eps
            lp = _loss(D1, D2, prm)
            D[idx] = old - eps
            lm = _loss(D1, D2, prm)
            D[idx] = old
            fd[idx] = (lp - lm) / (2 * eps)
        assert np.linalg.norm(fd - g) / np.linalg.norm(g) < 1e-6
        assert np.abs(fd - g).max() < 1e-6


def test_gradient_matches_autograd_reexpression():
    rng = np.random.default_rng(13)
    D1, D2 = rand_desc(rng, 28, 24), rand_desc(rng, 22, 26)
    prm = O.Params(max_patch=32)
    pyr = O.pyramid(D1, D2, prm, keep_full=True)
    g1, g2 = O.pyramid_backward(D1, D2, pyr)
    t1 = torch.from_numpy(D1).requires_grad_()
    t2 = torch.from_numpy(D2).requires_grad_()
    _, top, _ = T.forward(t1, t2, 1.4, pyr.lmax)
    L = T.loss(top)
    assert abs(L.item() - O.top_loss(pyr)) < 1e-12
    L.backward()
    np.testing.assert_allclose(g1, t1.grad.numpy(), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(g2, t2.grad.numpy(), rtol=1e-10, atol=1e-13)


def _c4_sub_pair():
    p = synth.make_pair("c4")
    D1, D2 = O.descriptors(p["img1"]), O.descriptors(p["img2"])
    return np.ascontiguousarray(D1[72:120, 104:152]), np.ascontiguousarray(D2[72:120, 104:152])


def test_gradient_risk_bounds_every_alternative_route():
    """The near-tie risk of pyramid_backward (R14): forcing any risky
    decision (a pooling argmax, or the top map's maximum) to any other
    candidate within the tie moves each coordinate's gradient by at most its
    risk R, and coordinates with R = 0 not at all.  A generous tie makes
    decisions at every level risky."""
    D1, D2 = _c4_sub_pair()
    tie = 1e-3
    pyr = O.pyramid(D1, D2, O.Params(max_patch=64), keep_full=True)
    g1, g2, R1, R2, dec = O.pyramid_backward(D1, D2, pyr, tie=tie)
    ref1, ref2 = O.pyramid_backward(D1, D2, pyr)
    np.testing.assert_array_equal(g1, ref1)
    np.testing.assert_array_equal(g2, ref2)
    levels = {d[0] for d in dec}
    assert levels == set(range(pyr.lmax + 1)), levels
    assert (R1 > 0).mean() < 0.95 and (R2 > 0).mean() < 0.95
    gmax = max(np.abs(g1).max(), np.abs(g2).max())
    flips = changed = 0
    worst = 0.0

    def check():
        nonlocal flips, changed, worst
        h1, h2 = O.pyramid_backward(D1, D2, pyr)
        for g, h, R in ((g1, h1, R1), (g2, h2, R2)):
            moved = np.abs(h - g)
            changed += int((moved > 1e-12 * gmax).any())
            assert (moved <= R * (1 + 1e-9) + 1e-12 * gmax).all(), "a route moves a coordinate beyond its risk"
            if (R > 0).any():
                worst = max(worst, float((moved[R > 0] / R[R > 0]).max()))
        flips += 1

    for lv, b, a, y, x in dec:
        if lv == pyr.lmax:
            top = pyr.top[b, a]
            m = top[y, x]
            for k in np.flatnonzero(top.reshape(-1) >= m - tie * (1 + m)):
                qy, qx = divmod(int(k), top.shape[1])
                if (qy, qx) == (y, x):
                    continue
                old = top[qy, qx]
                top[qy, qx] = np.nextafter(m, np.inf) if (qy, qx) > (y, x) else m
                check()
                top[qy, qx] = old
            continue
        code = pyr.code[lv]
        k0, best = int(code[b, a, y, x]), pyr.Cp[lv][b, a, y, x]
        A = pyr.A[lv][b, a] if lv else O.bottom_scores(D1, D2, np.array([b]))[0, a]
        C = O.rectify(A, pyr.lam)
        for k in range(9):
            yy, xx = 2 * y + k // 3 - 1, 2 * x + k % 3 - 1
            if k == k0 or not (0 <= yy < C.shape[0] and 0 <= xx < C.shape[1]) or C[yy, xx] < best - tie * (1 + best):
                continue
            code[b, a, y, x] = k
            check()
            code[b, a, y, x] = k0
    print(f"{flips} forced alternatives, {changed} changed fields, largest change / risk {worst:.3f}")
    assert flips >= 50 and changed >= 50, (flips, changed)
    assert worst > 0.5   # the bound is reached by some alternative, not loose everywhere


def test_pooling_stability_bruteforce_provenance():
    """pooling_stability against a brute force: every value of every map is
    given the explicit tree of the child values it averages (a stable pooled
    cell passes on its source's tree, an unstable one a leaf of its own), and
    equal trees are interned to one id by an exact dictionary.  A decision is
    unstable iff a runner-up lies within the tie with a lower value, or
    equals the winner with a different tree (level 0: any equal value)."""
    D1, D2 = _c4_sub_pair()
    pyr = O.pyramid(D1, D2, O.Params(max_patch=64), keep_full=True)
    W, H = pyr.W, pyr.H
    for tie in (2e-5, 1e-3):
        unstable, top_vid, _ = O.pooling_stability(pyr, tie)
        intern = {}
        pid = {}          # (lv, b, a, y, x) of a pooled cell -> tree id of its value
        for lv in range(pyr.lmax + 1):
            ny, nx = O.lattice_shape(lv, W, H)
            h, w = pyr.h[lv], pyr.w[lv]
            vid = {}
            if lv >= 1:
                for b in range(ny):
                    for a in range(nx):
                        if not pyr.G[lv][b, a]:
                            continue
                        kids = []
                        for ox, oy in O.OFFSETS:
                            cb, ca, ok = O.lattice_index(lv - 1, W, H, 4 * b + (2 ** lv) * oy, 4 * a + (2 ** lv) * ox)
                            kids.append((bool(ok and pyr.G[lv - 1][cb, ca]), int(cb), int(ca), ox, oy))
                        for y in range(h):
                            for x in range(w):
                                t = tuple(("out",) if not (0 <= y + oy < h and 0 <= x + ox < w)
                                          else pid[(lv - 1, cb, ca, y + oy, x + ox)]
                                          for ok, cb, ca, ox, oy in kids if ok)
                                vid[(b, a, y, x)] = intern.setdefault(t, len(intern))
            if lv == pyr.lmax:
                # the vectorised ids induce the same partition of every top map
                for b in range(ny):
                    for a in range(nx):
                        if pyr.G[lv][b, a]:
                            mine = np.array([[vid[(b, a, y, x)] for x in range(w)] for y in range(h)])
                            _, inv1 = np.unique(mine, return_inverse=True)
                            _, inv2 = np.unique(top_vid[b, a], return_inverse=True)
                            assert len(set(zip(inv1.ravel(), inv2.ravel()))) == len(set(inv1.ravel()))
                            assert len(set(inv1.ravel())) == len(set(inv2.ravel()))
                break
            C = O.rectify(pyr.A[lv] if lv else O.bottom_scores(D1, D2), pyr.lam)
            hp, wp = pyr.h[lv + 1], pyr.w[lv + 1]
            n_unstable = 0
            for b in range(ny):
                for a in range(nx):
                    if not pyr.G[lv][b, a]:
                        continue
                    for y in range(hp):
                        for x in range(wp):
                            k0 = int(pyr.code[lv][b, a, y, x])
                            sy, sx = 2 * y + k0 // 3 - 1, 2 * x + k0 % 3 - 1
                            best = C[b, a, sy, sx]
                            bad = False
                            for k in range(9):
                                yy, xx = 2 * y + k // 3 - 1, 2 * x + k % 3 - 1
                                if k == k0 or not (0 <= yy < h and 0 <= xx < w) or best <= 0:
                                    continue
                                v = C[b, a, yy, xx]
                                if best - tie * (1 + best) <= v < best:
                                    bad = True
                                elif v == best and (lv == 0 or vid[(b, a, yy, xx)] != vid[(b, a, sy, sx)]):
                                    bad = True
                            assert bad == bool(unstable[lv][b, a, y, x]), (tie, lv, b, a, y, x)
                            n_unstable += bad
                            pid[(lv, b, a, y, x)] = (("u", lv, b, a, y, x) if bad else
                                                     (("c0", b, a, sy, sx) if lv == 0 else vid[(b, a, sy, sx)]))
            assert n_unstable > 0 or tie < 1e-4


# ---------------------------------------------------------------- approximate DeepMatching (Sec. 4.1)

def _sphere_patches(rng, n):
    """n atomic-patch vectors: 16 unit pixel descriptors each (norm 4)."""
    P = rng.random((n, 16, 9)) + 0.05
    P /= np.linalg.norm(P, axis=-1, keepdims=True)
    return P.reshape(n, 144)


def test_kmeans_init_evenly_spread():
    assert O.kmeans_init(10, 10).tolist() == list(range(10))
    assert O.kmeans_init(10, 3).tolist() == [1, 5, 8]
    assert O.kmeans_init(7, 1).tolist() == [3]
    for n, D in ((1000, 999), (1000, 7), (8192, 1024), (6912, 4096)):
        idx = O.kmeans_init(n, D)
        assert len(np.unique(idx)) == D and idx.min() >= 0 and idx.max() < n
    for D in (0, 11):
        with pytest.raises(ValueError):
            O.kmeans_init(10, D)


def test_kmeans_single_prototype_is_mean_direction():
    # Cauchy-Schwarz: over the sphere of radius 4, sum_p <x_p, c> peaks at
    # c = 4 s / |s| with s = sum_p x_p.
    X = _sphere_patches(np.random.default_rng(30), 50)
    for iters in (0, 1, 5):
        C, a = O.spherical_kmeans(X, 1, iters)
        s = X.sum(0)
        if iters:
            np.testing.assert_allclose(C[0], 4 * s / np.linalg.norm(s), rtol=0, atol=1e-13)
        assert (a == 0).all()


def test_kmeans_objective_monotone_and_on_sphere():
    X = _sphere_patches(np.random.default_rng(31), 300)
    prev = -np.inf
    for iters in range(8):
        C, a = O.spherical_kmeans(X, 12, iters)
        np.testing.assert_allclose(np.linalg.norm(C, axis=1), 4.0, rtol=0, atol=1e-12)
        J = O.kmeans_objective(X, C, a)
        assert J >= prev - 1e-9, (iters, J, prev)
        # every vector sits with a nearest centroid
        S = X @ C.T
        assert (S[np.arange(len(X)), a] >= S.max(1) - 1e-12).all()
        prev = J


def test_kmeans_reaches_bruteforce_optimum_on_separated_data():
    # Two well-separated groups of 3 vectors: the best partition over all
    # 2^6 splits, scored by sum_k 4 |sum of group k| (the objective with each
    # centroid at its optimum), is what k-means converges to.
    rng = np.random.default_rng(32)
    base = _sphere_patches(rng, 2)
    X = []
    for g in (0, 1, 0, 1, 1, 0):
        v = base[g].reshape(16, 9) + 0.01 * rng.random((16, 9))
        X.append((v / np.linalg.norm(v, axis=-1, keepdims=True)).ravel())
    X = np.array(X)
    best = max(sum(4 * np.linalg.norm(X[[i for i in range(6) if (m >> i) & 1 == k]].sum(0)) for k in (0, 1))
               for m in range(1, 63))
    C, a = O.spherical_kmeans(X, 2, 10)
    assert abs(O.kmeans_objective(X, C, a) - best) < 1e-10
    assert len(set(a[[0, 2, 5]])) == 1 and len(set(a[[1, 3, 4]])) == 1 and a[0] != a[1]


def test_kmeans_ties_go_to_lowest_index():
    X = _sphere_patches(np.random.default_rng(33), 4)
    C = np.stack([X[1], X[0], X[0], X[1]])
    assert O.nearest_prototype(X[:2], C).tolist() == [1, 0]


def _substituted(D1, pyr):
    """D1 with every atomic patch replaced by its prototype (Sec. 4.1)."""
    H, W, _ = D1.shape
    ny, nx = O.lattice_shape(0, W, H)
    S = D1.copy()
    P = pyr.protos[pyr.assign].reshape(ny, nx, 4, 4, 9)
    for b in range(ny):
        for a in range(nx):
            S[4 * b:4 * b + 4, 4 * a:4 * a + 4] = P[b, a]
    return S


@pytest.mark.parametrize("D", [1, 5, 37])
def test_approx_equals_exact_method_on_substituted_patches(D):
    # Each patch replaced by its closest prototype, then the exact method:
    # the same pyramid and matches as the approximate path.
    rng = np.random.default_rng(34)
    D1, D2 = rand_desc(rng, 30, 27), rand_desc(rng, 26, 29)
    prm = O.Params(max_patch=16, prototypes=D, kmeans_iters=4)
    out, margin, pyr, _ = O.match_descriptors(D1, D2, prm)
    assert pyr.protos.shape == (D, 144) and pyr.assign.shape == (7 * 6,)
    ex_prm = O.Params(max_patch=16)
    out_e, _, pyr_e, _ = O.match_descriptors(_substituted(D1, pyr), D2, ex_prm)
    for lv in range(pyr.lmax):
        np.testing.assert_allclose(pyr.Cp[lv], pyr_e.Cp[lv], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(pyr.top, pyr_e.top, rtol=1e-12, atol=1e-14)
    assert out.shape == out_e.shape
    np.testing.assert_array_equal(out[:, :4], out_e[:, :4])
    np.testing.assert_allclose(out[:, 4], out_e[:, 4], rtol=1e-12)


def test_approx_with_every_patch_a_prototype_is_the_exact_method():
    rng = np.random.default_rng(35)
    D1, D2 = rand_desc(rng, 24, 28), rand_desc(rng, 25, 22)
    n = 6 * 7
    out, _, pyr, _ = O.match_descriptors(D1, D2, O.Params(max_patch=16, prototypes=n, kmeans_iters=3))
    assert pyr.assign.tolist() == list(range(n))
    out_e, _, pyr_e, _ = O.match_descriptors(D1, D2, O.Params(max_patch=16))
    np.testing.assert_allclose(pyr.Cp[0], pyr_e.Cp[0], rtol=1e-12)
    np.testing.assert_array_equal(out[:, :4], out_e[:, :4])


def test_gradient_rejects_prototypes():
    rng = np.random.default_rng(36)
    D1, D2 = rand_desc(rng, 16, 16), rand_desc(rng, 16, 16)
    with pytest.raises(ValueError):
        O.pyramid(D1, D2, O.Params(max_patch=16, prototypes=4), keep_full=True)


# ---------------------------------------------------------------- scale and rotation invariance (Sec. 4.2)

def test_scale_and_rotation_tables():
    assert [O.scale_factor(k) for k in range(5)] == [1.0, math.sqrt(2.0), 2.0, 2 * math.sqrt(2.0), 4.0]
    assert O.scale_pair(3) == (O.scale_factor(3), 1.0) and O.scale_pair(-2) == (1.0, 2.0) and O.scale_pair(0) == (1.0, 1.0)
    for r, (c, s) in enumerate(O.ROTATIONS):
        assert abs(c - math.cos(r * math.pi / 4)) < 1e-15 and abs(s - math.sin(r * math.pi / 4)) < 1e-15


def test_resample_identity_quarter_turns_and_halving():
    rng = np.random.default_rng(40)
    img = rng.random((23, 30))
    np.testing.assert_array_equal(O.resample(img, 1.0, 0), img)
    for r, k in ((2, 1), (4, 2), (6, 3)):
        np.testing.assert_allclose(O.resample(img, 1.0, r), np.rot90(img, k), rtol=0, atol=1e-15)
    box = img[:22, :30].reshape(11, 2, 15, 2).mean(axis=(1, 3))
    np.testing.assert_allclose(O.resample(img, 2.0, 0), box, rtol=0, atol=1e-15)


def test_resample_eighth_turn_of_a_ramp():
    # Bilinear sampling reproduces a linear function exactly: inside the
    # source, the rotated canvas holds the x coordinate of the mapped point.
    H, W = 20, 26
    img = np.tile(np.arange(W, dtype=np.float64), (H, 1))
    out = O.resample(img, 1.0, 1)
    Ws, Hs, Wr, Hr, cin, cout = O.resampled_geometry(W, H, 1.0, 1)
    assert (Wr, Hr) == (math.ceil(46 * O.SQRT_HALF), math.ceil(46 * O.SQRT_HALF))
    v, u = np.meshgrid(np.arange(Hr, dtype=float), np.arange(Wr, dtype=float), indexing="ij")
    x, y = O.canvas_to_source(u, v, 1.0, 1, cin, cout)
    inside = (x >= 0) & (x <= W - 1) & (y >= 0) & (y <= H - 1)
    assert inside.sum() > 300
    np.testing.assert_allclose(out[inside], x[inside], rtol=0, atol=1e-12)
    assert (out[(x < -1) | (x > W) | (y < -1) | (y > H)] == 0).all()


def test_invariant_single_run_is_the_exact_method():
    p = synth.make_pair("c1")
    prm = O.Params(max_patch=32)
    out, margin = O.invariant_match(p["img1"], p["img2"], prm, scales=[0], rotations=[0])
    ref, rmargin, _, _ = O.match(p["img1"], p["img2"], prm)
    np.testing.assert_array_equal(out, ref)
    np.testing.assert_array_equal(margin, rmargin)


def test_invariant_recovers_a_quarter_turn():
    img1 = synth.make_pair("c1")["img1"].astype(np.float64)
    img2 = np.rot90(img1, -1).copy()            # I' = I turned a quarter: the r = 2 run sees I against I
    prm = O.Params(max_patch=32)
    out, _ = O.invariant_match(img1, img2, prm, scales=[0], rotations=[0, 2])
    H, W = img1.shape
    x1, y1, x2, y2 = (out[:, i].astype(int) for i in range(4))
    # pixel (x, y) of I sits at (H - 1 - y, x) in I'
    ok = (x2 == H - 1 - y1) & (y2 == x1)
    assert len(out) > 150 and ok.mean() > 0.95
    assert len(np.unique(out[:, 2:4] // 4, axis=0)) == len(out)
    out0, _ = O.invariant_match(img1, img2, prm, scales=[0], rotations=[0])
    assert ((out0[:, 2] == H - 1 - out0[:, 1]) & (out0[:, 3] == out0[:, 0])).mean() < 0.2


def test_invariant_recovers_a_halving():
    img1 = synth.make_pair("c1")["img1"].astype(np.float64)
    img2 = O.resample(img1, 2.0, 0)              # I' = I at half size: the sigma = 1 run sees I' against I'
    out, _ = O.invariant_match(img1, img2, O.Params(max_patch=16), scales=[0, 2], rotations=[0])
    x1, y1, x2, y2 = (out[:, i].astype(int) for i in range(4))
    ok = (x1 == 2 * x2 + 1) & (y1 == 2 * y2 + 1)   # P = 2 (p + 0.5) - 0.5 rounded, T = p
    assert len(out) > 40 and ok.mean() > 0.9
