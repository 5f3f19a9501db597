"""GPU parity of the DM* entry points (local maxima of every level, scored by
path sums, Table 1's middle configuration, or by the values at the start and
end of each path, its first; Sec. 3.3 and Sec. 5) against the FP64 oracle:
the entry marks of every pooled level, and the reciprocal matches."""
import functools

import numpy as np
import pytest
import torch

import paper_1506_07656_amd as dm
import synth
from oracle import dm_oracle as O
from tests.helpers import FP32_TIE, compare_matches, within_px
from tests.test_gpu_parity import case, cuda, report

pytestmark = pytest.mark.gpu

CASES = ["c1", "c2", "odd", "narrow"] + [f"random{k}" for k in range(4)]


@functools.lru_cache(maxsize=None)
def dmstar_case(name, scoring=0):
    """The oracle's DM* run on the descriptors of a named test case."""
    o, mp = case(name)
    prm = O.Params(max_patch=mp, entry_points=1, scoring=scoring)
    out, margin, pyr, M = O.match_descriptors(o["D1"], o["D2"], prm)
    return dict(D1=o["D1"], D2=o["D2"], out=out, margin=margin, pyr=pyr, M=M), mp


def run(o, mp, prec, scoring=0):
    m, ws, pl = dm.match_descriptors(cuda(o["D1"]), cuda(o["D2"]),
                                     dm.params(max_patch=mp, precision=prec, entry_points="local_maxima",
                                               scoring=scoring),
                                     return_state=True)
    torch.cuda.synchronize()
    return m.cpu().numpy(), dm.workspace_views(ws, pl), pl


@pytest.mark.parametrize("name", CASES)
def test_dmstar_entries_and_matches_equal_oracle(name):
    o, mp = dmstar_case(name)
    pyr = o["pyr"]
    gpu, views, pl = run(o, mp, "fp32")
    assert pl.lmax == pyr.lmax
    _, _, pids = O.pooling_stability(pyr, FP32_TIE)
    # entry marks of every pooled level, wherever the oracle's decision is clear
    for lv in range(pyr.lmax):
        G = pyr.G[lv]
        mask, margin = O.local_maxima(np.nan_to_num(pyr.Cp[lv], nan=-np.inf), pids[lv])
        got = (views["levels"][lv]["code"].cpu().numpy() & 0x10) != 0
        clear = margin > FP32_TIE * (1 + np.abs(np.nan_to_num(pyr.Cp[lv])))
        diff = (got != mask) & clear & G[..., None, None]
        print(f"{name} level {lv}: {int(mask[G].sum())} oracle entries, {int(got[G].sum())} marked, "
              f"{int(diff.sum())} differ where the decision is clear", flush=True)
        assert diff.sum() == 0
    r = compare_matches(gpu, o["out"], o["margin"])
    report(f"{name} dm*", r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]


@pytest.mark.parametrize("name", CASES)
def test_start_end_scoring_matches_equal_oracle(name):
    """Start/end-point scores (R26): both backtracking forms (the tiled one on
    the small maps, the streaming one on the wide levels of c2 and the random
    shapes) against the oracle's matches and scores."""
    o, mp = dmstar_case(name, 1)
    gpu, _, _ = run(o, mp, "fp32", 1)
    r = compare_matches(gpu, o["out"], o["margin"])
    report(f"{name} dm* start/end", r)
    assert not r["missing"] and not r["moved"] and not r["bad_score"]
    assert len(r["extra"]) <= r["near_ties"]
    # the scores are not the path sums: the two schemes differ somewhere
    ps, _ = dmstar_case(name, 0)
    assert len(o["out"]) != len(ps["out"]) or not np.array_equal(o["out"], ps["out"])


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_start_end_scoring_bf16_agreement(name):
    o, mp = dmstar_case(name, 1)
    gpu, _, _ = run(o, mp, "bf16", 1)
    frac = within_px(gpu, o["out"], 1.0)
    print(f"{name} dm* start/end bf16: {len(gpu)} matches, {frac:.4f} of the oracle's within 1 px", flush=True)
    assert frac >= 0.99


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_dmstar_bf16_agreement(name):
    o, mp = dmstar_case(name)
    gpu, _, _ = run(o, mp, "bf16")
    frac = within_px(gpu, o["out"], 1.0)
    print(f"{name} dm* bf16: {len(gpu)} matches, {frac:.4f} of the oracle's within 1 px", flush=True)
    assert frac >= 0.99


def test_dmstar_images_entry_recovers_translation():
    p = synth.make_pair("c1")
    m = dm.match_images(cuda(p["img1"]), cuda(p["img2"]),
                        dm.params(max_patch=32, entry_points="local_maxima")).cpu().numpy()
    x1, y1 = m[:, 0], m[:, 1]
    inner = (x1 >= 8) & (x1 < 64 - 13) & (y1 >= 11) & (y1 < 56)
    assert inner.sum() > 100
    assert ((m[inner, 2] - x1[inner] == 5) & (m[inner, 3] - y1[inner] == -3)).all()
