"""Host-side tests of the C ABI (no GPU): the library loads and exports every
symbol include/dm.h declares; dm_plan's geometry equals the oracle's; every
validation error is raised before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1506_07656_amd as dm
from paper_1506_07656_amd import binding as B
from oracle import dm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = dm.lib()
    syms = declared_symbols()
    assert "dm_match_images" in syms and "dm_plan" in syms
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) <= set(B.SIGNATURES), set(syms) - set(B.SIGNATURES)


def test_status_strings_and_version():
    L = dm.lib()
    for code in B.STATUS:
        assert L.dm_status_string(code)
    assert dm.version().startswith("dm-mi355x")


def test_default_params():
    p = dm.params()
    assert abs(p.nu1) < 1e-9 and p.nu2 == 1 and p.nu3 == 1 and abs(p.sigmoid_slope - 0.2) < 1e-7
    assert abs(p.mu - 0.1) < 1e-7 and p.intensity_scale == 255 and abs(p.lam - 1.4) < 1e-7
    assert p.max_patch == 0 and p.precision == 0
    assert p.prototypes == 0 and p.kmeans_iters == 10


@pytest.mark.parametrize("W,H,W2,H2,mp", [(64, 64, 64, 64, 32), (256, 192, 256, 192, 64), (512, 256, 512, 256, 0),
                                           (621, 188, 621, 188, 0), (256, 192, 256, 192, 0), (37, 23, 19, 41, 0),
                                           (4, 4, 4, 4, 0), (9, 5, 3, 2, 0), (128, 96, 300, 150, 0)])
def test_plan_matches_oracle_geometry(W, H, W2, H2, mp):
    pl = dm.plan(W, H, W2, H2, dm.params(max_patch=mp))
    lmax = O.pyramid_top(W, H, mp)
    assert pl.lmax == lmax and pl.N_max == 4 << lmax
    G = O.grids(W, H, lmax)
    h, w = O.map_dims(H2, W2, lmax)
    assert pl.n_atomic == G[0].size == pl.max_matches
    for lv in range(lmax + 1):
        assert (pl.gy[lv], pl.gx[lv]) == G[lv].shape
        assert pl.n_valid[lv] == G[lv].sum()
    for lv in range(lmax + 2):
        assert (pl.h[lv], pl.w[lv]) == (h[lv], w[lv])
    offs = [pl.off_top, pl.off_best, pl.off_cell, pl.off_valid] + [pl.off_cp[i] for i in range(lmax)]
    assert all(o % 256 == 0 for o in offs)
    assert pl.workspace_bytes >= pl.off_cell + ((H2 + 3) // 4) * ((W2 + 3) // 4) * 8


@pytest.mark.parametrize("kw", [dict(max_patch=12), dict(max_patch=2), dict(lam=0.5), dict(mu=-1.0),
                                dict(nu2=3.0), dict(sigmoid_slope=0.0), dict(precision=7), dict(nu1=float("nan"))])
def test_plan_rejects_bad_params(kw):
    with pytest.raises(dm.DMError) as e:
        dm.plan(64, 64, 64, 64, dm.params(**kw))
    assert e.value.status == -1


def test_plan_rejects_bad_shapes():
    for args in [(3, 64, 64, 64), (64, 2, 64, 64), (64, 64, 0, 64), (9000, 64, 64, 64)]:
        with pytest.raises(dm.DMError) as e:
            dm.plan(*args, dm.params())
        assert e.value.status == -2
    p = dm.params()
    p.reserved[2] = 1
    with pytest.raises(dm.DMError):
        dm.plan(64, 64, 64, 64, p)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_plan_approximate_layout(prec):
    ex = dm.plan(512, 256, 512, 256, dm.params(precision=prec))
    pl = dm.plan(512, 256, 512, 256, dm.params(precision=prec, prototypes=1024))
    assert pl.prototypes == 1024 and pl.kmeans_chunks == 16 and ex.prototypes == 0
    assert pl.lmax == ex.lmax and pl.n_atomic == ex.n_atomic == 128 * 64
    # C'_0 holds D maps instead of one per atomic patch
    assert pl.off_code[0] - pl.off_cp[0] == 1024 * pl.h[1] * pl.w[1] * 4
    assert ex.off_code[0] - ex.off_cp[0] == 8192 * ex.h[1] * ex.w[1] * 4
    assert pl.workspace_bytes < ex.workspace_bytes
    offs = [pl.off_protos, pl.off_assign, pl.off_kstat, pl.off_proto_img, pl.off_kpart]
    assert all(o % 256 == 0 and o < pl.workspace_bytes for o in offs)
    assert (pl.off_proto_bf != 0) == (prec == "bf16")
    assert pl.workspace_bytes >= pl.off_kpart + 16 * 8192 * 20


def test_plan_approximate_errors():
    with pytest.raises(dm.DMError) as e:                          # more prototypes than patches
        dm.plan(64, 64, 64, 64, dm.params(prototypes=257))
    assert e.value.status == -1
    dm.plan(64, 64, 64, 64, dm.params(prototypes=256))
    for kw in (dict(prototypes=-1), dict(prototypes=4097), dict(prototypes=8, kmeans_iters=-1)):
        with pytest.raises(dm.DMError) as e:
            dm.plan(64, 64, 64, 64, dm.params(**kw))
        assert e.value.status == -1
    for args, kw in (((64, 64, 64, 64), dict(prototypes=8, precision="fp64")),      # FP64
                     ((4, 4, 4, 4), dict(prototypes=1))):                           # no pooled level
        with pytest.raises(dm.DMError) as e:
            dm.plan(*args, dm.params(**kw))
        assert e.value.status == -5
    with pytest.raises(dm.DMError) as e:                          # the gradient is the exact method's
        dm.plan_grad(64, 64, 64, 64, dm.params(prototypes=8))
    assert e.value.status == -5


def _call_match(ws_bytes, capacity, ws=0x10000, out=0x20000, n_out=0x30000, d1=0x40000, d2=0x50000, prm=None):
    prm = prm or dm.params()
    return dm.lib().dm_match_descriptors(ctypes.c_void_p(d1), 64, 64, ctypes.c_void_p(d2), 64, 64,
                                         ctypes.byref(prm), ctypes.c_void_p(ws), ws_bytes, ctypes.c_void_p(out),
                                         capacity, ctypes.c_void_p(n_out), None)


def test_match_validation_before_any_launch():
    """Fake device addresses are fine: every call below fails validation on
    the host, so nothing dereferences them."""
    pl = dm.plan(64, 64, 64, 64)
    need = pl.workspace_bytes
    assert _call_match(need - 1, pl.max_matches) == -3                 # workspace too small
    assert b"workspace" in dm.lib().dm_last_error()
    assert _call_match(need, pl.max_matches - 1) == -4                 # capacity too small
    assert _call_match(need, pl.max_matches, ws=0) == -1               # null workspace
    assert _call_match(need, pl.max_matches, ws=0x10010) == -1         # misaligned workspace
    assert _call_match(need, pl.max_matches, d1=0) == -1               # null descriptors
    assert _call_match(need, pl.max_matches, n_out=0) == -1
    assert _call_match(need, pl.max_matches, prm=dm.params(precision="fp64")) in (-5, -3)
    L = dm.lib()
    assert L.dm_match_descriptors(None, 64, 64, None, 64, 64, None, None, 0, None, 0, None, None) == -1
    assert L.dm_descriptors(ctypes.c_void_p(0x1000), 0, 5, 0, ctypes.byref(dm.params()),
                            ctypes.c_void_p(0x2000), None) == -2
    assert L.dm_descriptors(ctypes.c_void_p(0x1000), 8, 5, 4, ctypes.byref(dm.params()),
                            ctypes.c_void_p(0x2000), None) == -2


def test_grad_plan_layout_and_errors():
    gp = dm.plan_grad(256, 192, 256, 192, dm.params(), recompute=False)
    assert gp.geom.lmax == 6 and gp.nsplit >= 1
    assert all(gp.cp_in_saved[i] == 1 for i in range(gp.geom.lmax))
    gr = dm.plan_grad(256, 192, 256, 192, dm.params(), recompute=True)
    assert gr.cp_in_saved[0] == 1 and all(gr.cp_in_saved[i] == 0 for i in range(1, gr.geom.lmax))
    assert gr.saved_bytes < gp.saved_bytes
    g64 = dm.plan_grad(48, 48, 48, 48, dm.params(precision="fp64", max_patch=64))
    assert g64.nsplit == 1 and g64.geom.lmax == 4
    with pytest.raises(dm.DMError) as e:
        dm.plan_grad(4, 4, 4, 4, dm.params())
    assert e.value.status == -5
    L = dm.lib()
    prm = dm.params()
    # validation happens before anything is enqueued (fake device addresses)
    st = L.dm_pyramid_forward(ctypes.c_void_p(0x1000), 256, 192, ctypes.c_void_p(0x2000), 256, 192,
                              ctypes.byref(prm), 0, ctypes.c_void_p(0x10000), gp.saved_bytes - 1,
                              ctypes.c_void_p(0x20000), gp.scratch_bytes, None)
    assert st == -3
    st = L.dm_pyramid_backward(ctypes.c_void_p(0x1000), 256, 192, ctypes.c_void_p(0x2000), 256, 192,
                               ctypes.byref(prm), 0, ctypes.c_void_p(0x10000), gp.saved_bytes, None,
                               ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), ctypes.c_void_p(0x20000),
                               gp.scratch_bytes, None)
    assert st == -1


@pytest.mark.parametrize("W1,H1,W2,H2", [(9, 401, 1, 1), (401, 9, 1, 1), (13, 13, 2, 2), (256, 192, 256, 192),
                                         (37, 23, 19, 41)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grad_plan_holds_every_level_gradient(W1, H1, W2, H2, prec):
    """The two level-gradient buffers alternate over the pooled maps C'_l,
    l < lmax, so each must hold the largest, which need not be level 0's: the
    lattice above level 0 has ceil(W/4) x ceil(H/4) points, level 0
    floor(W/4) x floor(H/4)."""
    gp = dm.plan_grad(W1, H1, W2, H2, dm.params(precision=prec))
    g = gp.geom
    es = 8 if prec == "fp64" else 4
    need = max(g.gx[l] * g.gy[l] * g.h[l + 1] * g.w[l + 1] for l in range(g.lmax)) * es
    # scratch layout: ..., g[0], g[1], part, ...
    assert gp.off_g[0] < gp.off_g[1] < gp.off_part
    assert gp.off_g[1] - gp.off_g[0] >= need and gp.off_part - gp.off_g[1] >= need


def test_entry_points_validation():
    """DM* entry points: accepted by the matching plan, rejected with
    prototypes, without a pooled level, and by the gradient, batch and
    invariant plans; values other than the two schemes are invalid."""
    L = dm.lib()
    pl = dm.plan(64, 64, 64, 64, dm.params(entry_points="local_maxima"))
    assert pl.lmax == 4
    pl = dm.plan(64, 64, 64, 64, dm.params(entry_points="local_maxima", scoring="start_end"))
    assert pl.lmax == 4
    for kw, want in ((dict(entry_points=2), -1), (dict(entry_points=-1), -1),
                     (dict(entry_points=1, prototypes=8), -5), (dict(entry_points=1, max_patch=4), -5),
                     (dict(scoring=2), -1), (dict(scoring=-1), -1), (dict(entry_points=1, scoring=2), -1),
                     (dict(scoring=1), -5), (dict(entry_points=1, scoring=1, prototypes=8), -5)):
        with pytest.raises(dm.DMError) as e:
            dm.plan(64, 64, 64, 64, dm.params(**kw))
        assert e.value.status == want, kw
    with pytest.raises(dm.DMError) as e:
        dm.plan_grad(64, 64, 64, 64, dm.params(entry_points=1))
    assert e.value.status == -5
    info = B.BatchInfo()
    assert L.dm_plan_batch(1, _pairs([(64, 64, 64, 64)]), ctypes.byref(dm.params(entry_points=1)), 0,
                           ctypes.byref(info)) == -5
    inv = dm.InvariantInfo()
    assert L.dm_plan_invariant(ctypes.byref(dm.params(entry_points=1)), 64, 64, 64, 64, 0x10, 1,
                               ctypes.byref(inv)) == -5


def test_match_images_noalloc_validation_before_any_launch():
    """The allocation-free entry point checks its arguments and the size of
    the pair's workspace against its static array on the host, before it
    touches the device (fake addresses)."""
    L = dm.lib()
    prm = dm.params()
    out, n = ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000)
    assert L.dm_match_images_noalloc(ctypes.c_void_p(0x1000), 512, 256, 512, ctypes.c_void_p(0x2000), 512, 256,
                                     512, ctypes.byref(prm), out, 32768, n, None) == -3
    assert "static array" in L.dm_last_error().decode()
    assert dm.plan(512, 256, 512, 256, prm).workspace_bytes > dm.NOALLOC_MAX_BYTES
    assert dm.plan(160, 120, 160, 120, prm).workspace_bytes <= dm.NOALLOC_MAX_BYTES
    assert L.dm_match_images_noalloc(ctypes.c_void_p(0x1000), 2, 2, 2, ctypes.c_void_p(0x2000), 8, 8, 8,
                                     ctypes.byref(prm), out, 16, n, None) == -2
    assert L.dm_match_images_noalloc(ctypes.c_void_p(0x1000), 64, 64, 64, ctypes.c_void_p(0x2000), 64, 64, 64,
                                     None, out, 256, n, None) == -1


def _pairs(sizes, img=0x1000, dd=None):
    P = (dm.Pair * len(sizes))()
    for k, (a, b, c, d) in enumerate(sizes):
        P[k] = dm.Pair(img, a, b, a, img, c, d, c, dd, dd)
    return P


def test_plan_batch_layout_and_errors():
    L = dm.lib()
    sizes = [(64, 64, 64, 64), (203, 117, 190, 121), (621, 188, 621, 188)]
    prm = dm.params(precision="bf16")
    info, info_b = B.BatchInfo(), B.BatchInfo()
    assert L.dm_plan_batch(3, _pairs(sizes), ctypes.byref(prm), 0, ctypes.byref(info)) == 0
    assert L.dm_plan_batch(3, _pairs(sizes), ctypes.byref(prm), B.DM_BATCH_BWD, ctypes.byref(info_b)) == 0
    ws_sum = grad_sum = 0
    for k, sz in enumerate(sizes):
        pl = dm.plan(*sz, prm)
        assert info.max_matches[k] == pl.max_matches and info.lmax[k] == pl.lmax
        ws_sum += pl.workspace_bytes
        grad_sum += dm.plan_grad(*sz, prm).scratch_bytes
    assert info.n_pairs == 3 and info.workspace_bytes >= ws_sum
    assert info_b.workspace_bytes >= ws_sum + grad_sum and info_b.n_launches > info.n_launches
    bad = [(0, sizes, prm, -1), (257, sizes * 86, prm, -1), (3, sizes, dm.params(precision="fp64"), -5),
           (1, [(4, 4, 4, 4)], prm, -5), (1, [(3, 64, 64, 64)], prm, -2),
           (1, sizes, dm.params(prototypes=16), -5)]
    for n, sz, p, want in bad:
        P = _pairs(sz[:max(n, 1)])
        assert L.dm_plan_batch(n, P, ctypes.byref(p), 0, ctypes.byref(info)) == want, (n, want)
    assert L.dm_plan_batch(1, None, ctypes.byref(prm), 0, ctypes.byref(info)) == -1


def test_match_batch_validation_before_any_launch():
    """Fake device addresses: every call below fails on the host."""
    L = dm.lib()
    sizes = [(64, 64, 64, 64), (128, 96, 120, 100)]
    prm = dm.params(precision="bf16")
    info = B.BatchInfo()
    assert L.dm_plan_batch(2, _pairs(sizes), ctypes.byref(prm), 0, ctypes.byref(info)) == 0
    need = info.workspace_bytes
    offs_ok = (ctypes.c_int32 * 2)(0, info.max_matches[0])
    offs_bad = (ctypes.c_int32 * 2)(0, info.max_matches[0] - 1)

    def call(P=None, flags=0, ws=0x100000, nbytes=need, out=0x200000, offs=offs_ok, n_out=0x300000, stream=None):
        return L.dm_match_batch(2, P if P is not None else _pairs(sizes), ctypes.byref(prm), flags,
                                ctypes.c_void_p(ws), nbytes, ctypes.c_void_p(out), offs, ctypes.c_void_p(n_out),
                                stream)

    assert call(nbytes=need - 1) == -3
    assert call(ws=0x100010) == -1
    assert call(ws=0) == -1
    assert call(offs=offs_bad) == -4
    assert b"overlap" in L.dm_last_error()
    assert call(n_out=0) == -1
    assert call(flags=B.DM_BATCH_GRAPH) == -1              # graph capture needs a stream of its own
    assert call(flags=B.DM_BATCH_BWD, nbytes=1 << 40) == -1   # no gradient buffers
    assert call(P=_pairs(sizes, img=0)) == -1
    t = B.BatchTiles()
    assert L.dm_batch_tiles_get(ctypes.c_void_p(0x100000), ctypes.byref(t)) == -1
    assert L.dm_batch_release(ctypes.c_void_p(0x100000)) == 0


def test_plan_invariant_runs_and_errors():
    info = dm.plan_invariant(64, 48, 64, 48, dm.params())
    assert info.n_runs == 72 and info.max_matches == 16 * 12
    k = [info.run_k[i] for i in range(72)]
    r = [info.run_r[i] for i in range(72)]
    assert k == [kk for kk in range(-4, 5) for _ in range(8)] and r == list(range(8)) * 9
    for i in range(72):
        s1, s2 = O.scale_pair(k[i])
        Ws, Hs, _, _, _, _ = O.resampled_geometry(64, 48, s1, 0)
        _, _, Wr, Hr, _, _ = O.resampled_geometry(64, 48, s2, r[i])
        assert (info.run_W1[i], info.run_H1[i], info.run_W2[i], info.run_H2[i]) == (Ws, Hs, Wr, Hr)
    offs = [info.off_best, info.off_cell, info.off_img1, info.off_img2, info.off_run]
    assert all(o % 256 == 0 for o in offs) and info.workspace_bytes > info.off_run
    one = dm.plan_invariant(64, 48, 64, 48, dm.params(), 0x10, 0x1)
    assert one.n_runs == 1 and (one.run_W1[0], one.run_W2[0]) == (64, 64)
    # image 1 too small once downsized: those runs are left out
    small = dm.plan_invariant(12, 12, 64, 48, dm.params(), 0x1FF, 0x1)
    assert small.n_runs == 8          # k = 4 leaves a 3x3 image 1
    for kw, args, want in ((dict(), (0, 0xFF), -1), (dict(), (0x200, 0xFF), -1), (dict(), (0x1FF, 0x100), -1),
                           (dict(precision="fp64"), (0x1FF, 0xFF), -5), (dict(prototypes=8), (0x1FF, 0xFF), -5)):
        with pytest.raises(dm.DMError) as e:
            dm.plan_invariant(64, 48, 64, 48, dm.params(**kw), *args)
        assert e.value.status == want


def test_match_invariant_validation_before_any_launch():
    """Fake device addresses: every call below fails on the host."""
    L = dm.lib()
    info = dm.plan_invariant(64, 48, 64, 48, dm.params(), 0x1FF, 0xFF)
    need, cap = info.workspace_bytes, info.max_matches

    def call(prm=None, smask=0x1FF, rmask=0xFF, ws=0x100000, nbytes=need, out=0x200000, capacity=cap,
             n_out=0x300000, img1=0x1000, img2=0x2000, ld1=64, ld2=64):
        prm = prm or dm.params()
        return L.dm_match_invariant(ctypes.c_void_p(img1), 64, 48, ld1, ctypes.c_void_p(img2), 64, 48, ld2,
                                    ctypes.byref(prm), smask, rmask, ctypes.c_void_p(ws), nbytes,
                                    ctypes.c_void_p(out), capacity, ctypes.c_void_p(n_out), None)

    assert call(nbytes=need - 1) == -3
    assert call(capacity=cap - 1) == -4
    assert call(ws=0x100010) == -1 and call(ws=0) == -1
    assert call(img1=0) == -1 and call(out=0) == -1 and call(n_out=0) == -1
    assert call(ld1=63) == -2
    assert call(smask=0) == -1 and call(rmask=0x100) == -1
    assert call(prm=dm.params(precision="fp64")) == -5
    assert call(prm=dm.params(prototypes=4)) == -5
    assert b"prototypes" in L.dm_last_error()


def test_flow_params_and_plan_against_the_oracle():
    """dm_flow_default_params holds the paper's values (Sec. 4.3 and its
    parameter study) and dm_flow_plan the oracle's level sizes."""
    from oracle import deepflow_oracle as F
    p, q = dm.flow_params(), F.FlowParams()
    for name in ("sigma", "eta", "min_size", "n_fixed", "n_sor", "omega", "kappa", "beta", "b", "gamma", "delta",
                 "eps", "zeta", "sigma_m", "lam_scale"):
        assert abs(getattr(p, name) - getattr(q, name)) <= 1e-6 * max(1.0, abs(getattr(q, name))), name
    for W, H in ((64, 56), (512, 256), (128, 96), (17, 40), (16, 16)):
        info = dm.flow_plan(W, H, 100)
        sizes = F.level_sizes(W, H, q)
        assert info.n_levels == len(sizes)
        assert [(info.W[k], info.H[k]) for k in range(info.n_levels)] == sizes
        assert info.workspace_bytes > 8 * W * H * 4


def test_deepflow_validation_before_any_launch():
    L = dm.lib()
    p = dm.flow_params()
    info = dm.FlowInfo()
    img, ws, fl = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000), ctypes.c_void_p(0x2000)
    big = ctypes.c_size_t(1 << 40)
    # parameters out of range
    for k, v in (("sigma", 0.0), ("sigma", 3.0), ("eta", 1.0), ("omega", 2.0), ("min_size", 1), ("eps", 0.0),
                 ("n_sor", -1), ("beta", -1.0)):
        q = dm.flow_params(**{k: v})
        assert L.dm_flow_plan(64, 64, 0, ctypes.byref(q), ctypes.byref(info)) == -1, k
    assert L.dm_flow_plan(0, 64, 0, ctypes.byref(p), ctypes.byref(info)) == -2
    assert L.dm_flow_plan(64, 64, -1, ctypes.byref(p), ctypes.byref(info)) == -1
    assert L.dm_flow_plan(64, 64, 0, ctypes.byref(p), None) == -1
    # a level count past the limit
    assert L.dm_flow_plan(1 << 12, 1 << 12, 0, ctypes.byref(dm.flow_params(eta=0.999)), ctypes.byref(info)) == -2
    # null pointers, leading dimension, workspace size and alignment
    assert L.dm_deepflow(None, img, 64, 64, 64, None, None, 0, ctypes.byref(p), 0, fl, ws, big, None) == -1
    assert L.dm_deepflow(img, img, 64, 64, 63, None, None, 0, ctypes.byref(p), 0, fl, ws, big, None) == -2
    assert L.dm_deepflow(img, img, 64, 64, 64, None, None, 10, ctypes.byref(p), 0, fl, ws, big, None) == -1
    assert L.dm_deepflow(img, img, 64, 64, 64, None, None, 0, ctypes.byref(p), 0, fl, ctypes.c_void_p(0x100010), big,
                         None) == -1
    assert L.dm_deepflow(img, img, 64, 64, 64, None, None, 0, ctypes.byref(p), 0, fl, ws, ctypes.c_size_t(1024),
                         None) == -3
    # unknown flags; a graph needs a stream of its own
    assert L.dm_deepflow(img, img, 64, 64, 64, None, None, 0, ctypes.byref(p), 4, fl, ws, big, None) == -1
    assert L.dm_deepflow(img, img, 64, 64, 64, None, None, 0, ctypes.byref(p), 1, fl, ws, big, None) == -1
    assert L.dm_flow_release(ws) == 0
