"""Host-side model of the pixel mapping of DeepFlow's one-workgroup level
kernel (k_deepflow.hip, k_df_level_small): thread t of 1024 owns the pixel
pairs (2 p, 2 p + 1), p = t + 1024 k, k < 2, and keeps the pair's pixel of
colour c ((x + y) mod 2) in slot c, so that each red-black half-sweep of
Sec. 4.3's SOR updates slot c of every pair.  On every level size the
pyramid gives to that kernel (levels of at most 4096 pixels) and on odd
shapes, the model shows that the slots cover each pixel once, that slot c
holds colour c, and that every neighbour read stays inside the level.
"""
import math

import pytest

THREADS = 1024
SMALL_PIXELS = 4096
PAIRS = SMALL_PIXELS // 2 // THREADS


def flow_levels(W, H, eta=0.95, min_size=16):
    out = [(W, H)]
    for k in range(1, 200):
        w = math.floor(W * eta ** k + 0.5)
        h = math.floor(H * eta ** k + 0.5)
        if w < min_size or h < min_size:
            break
        out.append((w, h))
    return out


def small_shapes():
    shapes = set()
    for W, H in [(512, 256), (96, 72), (101, 77), (64, 64), (37, 23), (64, 56), (48, 40), (621, 188)]:
        shapes.update((w, h) for w, h in flow_levels(W, H) if w * h <= SMALL_PIXELS)
    shapes.update([(1, 1), (1, 7), (7, 1), (2, 3), (63, 65), (64, 64), (4096, 1), (1, 4096), (45, 91)])
    return sorted(s for s in shapes if s[0] * s[1] <= SMALL_PIXELS)


@pytest.mark.parametrize("W,H", small_shapes())
def test_slots_cover_each_pixel_once_with_their_colour(W, H):
    """Also the colour-split LDS layout: pixel j of colour c sits at
    uv[c][j >> 1]; the neighbour entries a slot reads (the pair partner from
    registers, the other horizontal neighbour and the vertical ones from
    uv[1 - c]) are exactly the neighbours of Sec. 4.3's 4-neighbourhood, and
    a missing neighbour reads an initialised entry (a pair below (n + 1) / 2)."""
    n = W * H
    npairs = (n + 1) // 2
    seen = [0] * n
    where = {}
    for j in range(n):
        where[(((j % W) + j // W) & 1, j >> 1)] = j
    for t in range(THREADS):
        for k in range(PAIRS):
            p = t + k * THREADS
            i0 = 2 * p
            y0 = i0 // W
            c0 = (i0 - y0 * W + y0) & 1
            for c in range(2):
                i = i0 + (c0 ^ c)
                if i >= n:
                    continue
                y, x = divmod(i, W)
                assert (x + y) & 1 == c, (W, H, t, k, c)
                seen[i] += 1
                e = (x > 0, x + 1 < W, y > 0, y + 1 < H)
                sd = i & 1
                nx = (p + 1 if e[1] else p) if sd else (p - 1 if e[0] else p)
                nu = (i - W) >> 1 if e[2] else p
                nd = (i + W) >> 1 if e[3] else p
                partner = i0 + (c0 ^ (1 - c))
                got = [partner if sd else where.get((1 - c, nx)), where.get((1 - c, nx)) if sd else partner,
                       where.get((1 - c, nu)), where.get((1 - c, nd))]
                want = [i - 1, i + 1, i - W, i + W]
                for g, w, ok in zip(got, want, e):
                    if ok:
                        assert g == w, (W, H, i, got, want)
                        assert ((w % W) + w // W) & 1 != c   # a neighbour has the other colour
                for q in (nx, nu, nd):
                    assert 0 <= q < npairs
    assert seen == [1] * n


def test_pyramid_levels_that_take_the_one_workgroup_kernel():
    """On the 512 x 256 pair, 21 of the 55 levels (every level from 90 x 45
    down) run in one workgroup; the other 34 take the tiled SOR."""
    lv = flow_levels(512, 256)
    assert len(lv) == 55
    small = [s for s in lv if s[0] * s[1] <= SMALL_PIXELS]
    assert len(small) == 21 and small[0] == (90, 45)
    assert all(w * h > SMALL_PIXELS for w, h in lv[:34])
