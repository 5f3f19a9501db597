"""Writes the oracle's results for the full-size synthetic pairs.

Calls only oracle/ and synth/.  For each pair it stores the reciprocal matches
[x1, y1, x2, y2, score], their decision margins, and the SHA-256 of the two
input images, so a test can check that it regenerated the same inputs before
comparing against the stored matches.  Usage:
    python tests/golden/make_golden.py c3 [c2 ...]
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


def image_hash(img1: np.ndarray, img2: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in (img1, img2):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    return h.hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}_oracle.npz")


def main(names):
    for name in names:
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
