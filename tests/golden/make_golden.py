"""Writes the oracle's results for the full-size synthetic pairs.

Calls only oracle/ and synth/.  For each pair it stores the reciprocal matches
[x1, y1, x2, y2, score], their decision margins, and the SHA-256 of the two
input images, so a test can check that it regenerated the same inputs before
comparing against the stored matches.  With a name ending in "grad" (c3grad)
it stores a sample of the oracle's gradient of the top loss instead, with the
oracle's near-tie risk of the sampled coordinates (how far their gradient can
move when decisions within FP32_TIE go another way).  Usage:
    python tests/golden/make_golden.py c3 [c2 ...] [c3grad]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dm_oracle as O  # noqa: E402
from tests.helpers import FP32_TIE  # noqa: E402


def image_hash(img1: np.ndarray, img2: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in (img1, img2):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    return h.hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}_oracle.npz")


def grad_path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}_grad_oracle.npz")


def make_grad(name: str, n_sample: int = 4096, n_top: int = 256):
    """The FP64 oracle gradient of L = sum of the top-map maxima with respect
    to both descriptor fields, from the oracle's own descriptors of the pair,
    at a seeded sample of coordinates plus the largest entries (the full
    fields are too large to store)."""
    p = synth.make_pair(name)
    D1, D2 = O.descriptors(p["img1"]), O.descriptors(p["img2"])
    lam32 = float(np.float32(1.4))   # the library's lambda is a float32 parameter
    prm = O.Params(max_patch=synth.CONFIG_NMAX[name], lam=lam32)
    t0 = time.time()
    pyr = O.pyramid(D1, D2, prm, keep_full=True, keep_bottom=False)
    g1, g2, R1, R2, decisions = O.pyramid_backward(D1, D2, pyr, tie=FP32_TIE)
    dt = time.time() - t0
    rng = np.random.default_rng(20261)
    out = dict(sha256=image_hash(p["img1"], p["img2"]), lmax=pyr.lmax, loss=O.top_loss(pyr), oracle_seconds=dt,
               tie=FP32_TIE, n_risky_decisions=len(decisions),
               risky_by_level=np.bincount([d[0] for d in decisions], minlength=pyr.lmax + 1))
    for k, g, R in (("1", g1, R1), ("2", g2, R2)):
        flat = g.reshape(-1)
        idx = np.union1d(rng.choice(flat.size, n_sample, replace=False), np.argsort(-np.abs(flat))[:n_top])
        out["idx" + k] = idx.astype(np.int64)
        out["val" + k] = flat[idx]
        out["norm" + k] = float(np.linalg.norm(flat))
        # how far each coordinate's gradient can move when decisions that FP32
        # may take the other way (FP32_TIE) go another way
        out["risk" + k] = R.reshape(-1)[idx]
        out["risk_norm" + k] = float(np.linalg.norm(R))
    np.savez_compressed(grad_path_of(name), **out)
    print(f"{name} gradient: lmax {pyr.lmax}, loss {out['loss']:.6f}, |g1| {out['norm1']:.4e}, "
          f"|g2| {out['norm2']:.4e}, {len(decisions)} risky decisions {out['risky_by_level'].tolist()}, "
          f"|R1| {out['risk_norm1']:.3e}, |R2| {out['risk_norm2']:.3e}, {dt:.1f} s", flush=True)


def main(names):
    for name in names:
        if name.endswith("grad"):
            make_grad(name[:-4])
            continue
        p = synth.make_pair(name)
        prm = O.Params(max_patch=synth.CONFIG_NMAX[name])
        t0 = time.time()
        out, margin, pyr, M = O.match(p["img1"], p["img2"], prm)
        dt = time.time() - t0
        np.savez_compressed(path_of(name), matches=out, margin=margin, lmax=pyr.lmax,
                            sha256=image_hash(p["img1"], p["img2"]), n_atomic_tuples=len(M["s"]),
                            oracle_seconds=dt)
        print(f"{name}: {len(out)} matches, lmax {pyr.lmax}, |M'| {len(M['s'])}, {dt:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3"])
