"""An independent FP64 re-expression of the correlation pyramid with torch
library routines (conv2d, max_pool2d, pad), used only to pin the oracle.

It shares nothing with the oracle: the atomic correlation is a convolution
with the source patches as filters, the joint max-pool/subsample is
``max_pool2d(kernel 3, stride 2, padding 1)``, grids are built from Python sets
of centres, and the gradient comes from autograd.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

OFFS = [(-1, -1), (-1, 1), (1, -1), (1, 1)]  # (x, y)


def centre_sets(W: int, H: int, lmax: int):
    """G_l as sets of (x, y) centres (existence of at least one child)."""
    g0 = {(2 + 4 * a, 2 + 4 * b) for a in range(W // 4) for b in range(H // 4)}
    sets = [g0]
    for lv in range(1, lmax + 1):
        prev = sets[-1]
        cur = set()
        for x in range(0, W, 4):
            for y in range(0, H, 4):
                if any((x + (2 ** lv) * ox, y + (2 ** lv) * oy) in prev for ox, oy in OFFS):
                    cur.add((x, y))
        sets.append(cur)
    return sets


def bottom(D1: torch.Tensor, D2: torch.Tensor) -> torch.Tensor:
    """A_0 as conv2d of I' descriptors with the 4x4 source patches / 16.
    Returns (ny0, nx0, H', W')."""
    H, W, C = D1.shape
    ny0, nx0 = H // 4, W // 4
    w = D1[:4 * ny0, :4 * nx0].reshape(ny0, 4, nx0, 4, C).permute(0, 2, 4, 1, 3)
    w = w.reshape(ny0 * nx0, C, 4, 4) / 16.0
    x = F.pad(D2.permute(2, 0, 1)[None], (2, 1, 2, 1))
    out = F.conv2d(x, w)[0]
    return out.reshape(ny0, nx0, D2.shape[0], D2.shape[1])


def pool(C: torch.Tensor):
    """Values and argmax codes of max_pool2d(3, 2, 1) on (..., h, w) maps."""
    lead = C.shape[:-2]
    h, w = C.shape[-2:]
    v, idx = F.max_pool2d(C.reshape(-1, 1, h, w), 3, 2, 1, return_indices=True)
    h2, w2 = v.shape[-2:]
    ry = torch.arange(h2).view(-1, 1)
    rx = torch.arange(w2).view(1, -1)
    my = idx // w - 2 * ry
    mx = idx % w - 2 * rx
    code = 3 * (my + 1) + (mx + 1)
    return v.reshape(*lead, h2, w2), code.reshape(*lead, h2, w2)


def forward(D1: torch.Tensor, D2: torch.Tensor, lam: float, lmax: int):
    """Returns (levels, top, sets): levels[l] = (pooled C'_l dict, codes dict)
    for l < lmax, keyed by centre; top = dict centre -> C_lmax map."""
    H, W, _ = D1.shape
    sets = centre_sets(W, H, lmax)
    A0 = bottom(D1, D2)
    C0 = torch.clamp(A0, min=0.0) ** lam
    cur = {(2 + 4 * a, 2 + 4 * b): C0[b, a] for a in range(W // 4) for b in range(H // 4)}
    levels = []
    for lv in range(1, lmax + 1):
        pooled, codes = {}, {}
        for c, m in cur.items():
            v, k = pool(m)
            pooled[c], codes[c] = v, k
        levels.append((pooled, codes))
        nxt = {}
        for (x, y) in sets[lv]:
            terms = []
            for ox, oy in OFFS:
                c = (x + (2 ** lv) * ox, y + (2 ** lv) * oy)
                if c in pooled:
                    m = pooled[c]
                    h, w = m.shape
                    mp = F.pad(m, (1, 1, 1, 1))
                    terms.append(mp[1 + oy:1 + oy + h, 1 + ox:1 + ox + w])
            A = torch.stack(terms).sum(0) / len(terms)
            nxt[(x, y)] = torch.clamp(A, min=0.0) ** lam
        cur = nxt
    return levels, cur, sets


def loss(top: dict) -> torch.Tensor:
    """Sum of map maxima; the gradient goes to the returned (first) index."""
    return torch.stack([m.reshape(-1).max(0).values for m in top.values()]).sum()
