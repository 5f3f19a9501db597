#!/usr/bin/env python3
"""Throughput of the DeepMatching hot path on one MI355X.

One step = one 512x256 image pair (the half-resolution movie-frame workload,
synthetic pair "c3") through the whole path: descriptors, bottom correlation,
pyramid levels, backtracking, reciprocal verification.  Inputs are resident
in device memory before timing starts.  The headline value is the BF16
correlation path (FP32 pyramid); the plain FP32 path is timed beside it.

Prints one JSON line.  Stage times come from HIP events the library records
on the launch stream around each kernel (dm_timing_*), in a second pass of
the same steps right after the timed one.

The "approx" entry is approximate DeepMatching (Sec. 4.1) on the same pair
with D = 1024 and 64 prototypes: throughput, k-means time, workspace size and
agreement with the exact path's matches.

The "invariant" entry is scale and rotation invariant DeepMatching (Sec. 4.2,
Algorithm 2) on the same pair: the paper's grid of 9 scales x 8 rotations (72
runs of the pipeline on resampled pairs, one reciprocal check over their
union), BF16 correlation.

The "dmstar" entry is the earlier entry-point scheme (DM*, Sec. 3.3 and
Table 1): local maxima of every level start the backtracking, scored by the
current path sums; entry counts and agreement with the plain method; and
the same entry points with the earlier start/end-point scores (Table 1's
first configuration), time and agreement beside it; for all three, the
fraction of matches within 1 px of the pair's ground-truth field (Table 1's
accuracy measure, on the synthetic pair).

The "batch" entry is the uneven-batch workload: 32 pairs with W ~ U{128..621},
H ~ U{96..188} (half of a 1242x375 driving-frame shape), BF16 correlation,
FP32 pyramid, forward plus backward of the top loss, every stage one
persistent grouped launch over all pairs, the whole sequence one HIP graph
replay with autotuned tiles; beside it the same pairs one by one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
PEAKS_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_512x256.md")

# Algorithmic bytes per entry: a correlation value is 4 bytes; an argmax code
# (one of 9 window positions) needs 4 bits.  The library stores codes as one
# byte, so the stored traffic is also reported (stored_* fields).
CODE_BYTES = 0.5
CODE_BYTES_STORED = 1.0


def stage_work(pl, name: str, level: int, precision: str, code_bytes: float = CODE_BYTES):
    """Algorithmic work of one launch: (bound, amount, unit).  FLOPs for the
    correlation on the matrix cores when it is the bound, HBM bytes otherwise."""
    gx, gy, h, w = list(pl.gx), list(pl.gy), list(pl.h), list(pl.w)
    L = pl.lmax
    cb = code_bytes
    # maps stored at level 0: one per atomic patch, or one per prototype
    npat = lambda l: (pl.prototypes or gx[0] * gy[0]) if l == 0 else gx[l] * gy[l]
    if name == "kmeans_assign":   # FP32 MFMA dot products of every patch with every centroid
        return "mfma", 2.0 * pl.n_atomic * pl.prototypes * 144, "FLOP"
    if name.startswith("corr_pool"):
        flops = 2.0 * npat(0) * pl.H2 * pl.W2 * 144
        out_bytes = npat(0) * h[1] * w[1] * (4.0 + cb)
        if precision == "fp32":
            return "mfma", flops, "FLOP"
        return "hbm", out_bytes, "B"
    if name == "level":
        rd = npat(level - 1) * h[level] * w[level] * 4.0
        wr = npat(level) * (h[level] * w[level] * 4.0 if level == L else h[level + 1] * w[level + 1] * (4.0 + cb))
        return "hbm", rd + wr, "B"
    if name == "backtrack":
        rd = npat(level - 1) * h[level] * w[level] * (4.0 + cb if level == 1 else 4.0)
        rd += npat(level) * (h[level] * w[level] * 4.0 if level == L else h[level + 1] * w[level + 1] * (4.0 + cb))
        wr = 0.0 if level == 1 else npat(level - 1) * h[level] * w[level] * 4.0
        return "hbm", rd + wr, "B"
    if name == "descriptor":   # one launch for both images: 4 B in, 36 B out (+ 20 B BF16 copy) per pixel
        return "hbm", (pl.W1 * pl.H1 + pl.W2 * pl.H2) * (40.0 + (20.0 if precision == "bf16" else 0.0)), "B"
    return "hbm", 0.0, "B"


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of a kernel at 512x256 from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE profile (its JSON block), scaled by the plain-copy
    calibration recorded there; None when the profile lacks the kernel or the
    kernel's source file has changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        prof = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    k = prof.get("kernels", {}).get(kernel)
    if not k:
        return None
    src = os.path.join(ROOT, "paper_1506_07656_amd", "csrc", k["source"])
    if not os.path.exists(src) or _sha256(src) != k["source_sha256"]:
        return None
    cal = prof["calibration"]
    return k["fetch_kib"] * 1024.0 * cal["read_factor"] + k["write_kib"] * 1024.0 * cal["write_factor"]


def roofline_of(stages, pl, precision):
    """Roofline entry of the kernel (stage name + level) with the largest time."""
    rows = []
    for name, level, count, total in stages:
        bound, amount, unit = stage_work(pl, name, level, precision)
        avg_ms = total / count
        if unit == "FLOP":
            ach = amount / (avg_ms * 1e-3) / 1e12
            peak = PEAKS_TFLOPS["fp32" if name == "kmeans_assign" else precision]
            u = "TFLOP/s"
        else:
            ach = amount / (avg_ms * 1e-3) / 1e9
            peak = HBM_PEAK_GBS
            u = "GB/s"
        row = dict(kernel=f"{name}{'' if level < 0 else '_l%d' % level}", bound=bound, avg_ms=avg_ms,
                   launches=count, achieved=ach, peak=peak, unit=u, frac=ach / peak if peak else None, work=amount)
        if unit == "B":
            stored = stage_work(pl, name, level, precision, CODE_BYTES_STORED)[1]
            row["stored_achieved"] = stored / (avg_ms * 1e-3) / 1e9
            row["stored_frac"] = row["stored_achieved"] / peak if peak else None
        rows.append(row)
    rows.sort(key=lambda r: -r["avg_ms"] * r["launches"])
    return rows


def time_path(dm, torch, img1, img2, precision, steps, warmup, **kw):
    W1, H1 = img1.shape[1], img1.shape[0]
    W2, H2 = img2.shape[1], img2.shape[0]
    m = dm.Matcher(W1, H1, W2, H2, dm.params(precision=precision, **kw))
    for _ in range(warmup):
        m.run_images(img1, img2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.run_images(img1, img2)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    matches = m.result().cpu().numpy()
    dm.timing_enable(True)
    for _ in range(steps):
        m.run_images(img1, img2)
    torch.cuda.synchronize()
    stages = dm.timing_read()
    dm.timing_enable(False)
    return dt, matches, stages, m.plan


def time_fwd_bwd(dm, torch, d1, d2, precision, recompute, steps, warmup):
    """Leaf descriptors -> pyramid -> L = sum of top-map maxima -> dL/dD1, dL/dD2."""
    pyr = dm.Pyramid(d1, d2, dm.params(precision=precision), recompute)
    P = pyr.top_shape()[0] * pyr.top_shape()[1]

    def step():
        top = pyr.forward()
        flat = top.reshape(P, -1)
        dtop = torch.zeros_like(flat)
        dtop.scatter_(1, flat.argmax(1, keepdim=True), 1.0)
        return pyr.backward(dtop.view_as(top))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    dm.timing_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    stages = dm.timing_read()
    dm.timing_enable(False)
    return dt, stages


def within_1px(a, b):
    """Fraction of b's matches whose source patch has a match in a within 1 px."""
    ga = {(int(r[0]), int(r[1])): r for r in a}
    ok = 0
    for r in b:
        q = ga.get((int(r[0]), int(r[1])))
        ok += q is not None and max(abs(q[2] - r[2]), abs(q[3] - r[3])) <= 1
    return ok / max(1, len(b))


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def cpu_baseline(pair, cw=128, ch=128):
    """The FP64 oracle from images to matches on the full pair (the
    benchmark's workload), with every BLAS thread of the host; beside it the
    central cw x ch crop with every thread and with one (the paper's CPU
    timings are for one core), the thread count checked inside the limit."""
    import numpy as np
    from oracle import dm_oracle as O
    cores = _blas_threads()
    H, W = pair["img1"].shape
    t0 = time.perf_counter()
    O.match(pair["img1"], pair["img2"], O.Params())
    t = time.perf_counter() - t0
    y0, x0 = (H - ch) // 2, (W - cw) // 2
    c1 = np.ascontiguousarray(pair["img1"][y0:y0 + ch, x0:x0 + cw])
    c2 = np.ascontiguousarray(pair["img2"][y0:y0 + ch, x0:x0 + cw])
    t1 = time.perf_counter()
    O.match(c1, c2, O.Params())
    t_crop = time.perf_counter() - t1
    t_crop_1, threads_1 = None, None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            threads_1 = _blas_threads()
            t1 = time.perf_counter()
            O.match(c1, c2, O.Params())
            t_crop_1 = round(time.perf_counter() - t1, 3)
    except Exception:
        pass
    return dict(value=1.0 / t, unit="pairs/s", cores=int(cores), kind="oracle",
                sample=f"oracle (FP64 NumPy) from images to reciprocal matches on the whole {W}x{H} pair, "
                       f"{t:.1f} s with {cores} BLAS threads",
                crop=f"central {cw}x{ch} crop of the pair", crop_s=round(t_crop, 3), crop_s_one_thread=t_crop_1,
                one_thread_blas_threads=threads_1, host=host_info())


def host_info():
    """CPU model, logical CPUs and memory of the host the oracle ran on."""
    model, mem_gb = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return dict(cpu_model=model, cpu_count=os.cpu_count(), mem_gb=mem_gb)


def small_pairs(dm, torch, steps):
    """GPU throughput on the 64x64 and 256x192 pairs (BF16 correlation)."""
    import synth
    res = {}
    for name, mp in (("c1", 32), ("c2", 64)):
        p = synth.make_pair(name)
        i1, i2 = torch.from_numpy(p["img1"]).cuda(), torch.from_numpy(p["img2"]).cuda()
        dt, _, _, _ = time_path(dm, torch, i1, i2, "bf16", steps, 3, max_patch=mp)
        res[name] = dict(size=f"{p['img1'].shape[1]}x{p['img1'].shape[0]}", pairs_s=round(1.0 / dt, 1),
                         ms_per_step=round(dt * 1e3, 4))
    return res


def pair_work(pl):
    """Algorithmic (HBM bytes, MFMA FLOPs) of one pair's forward and of its
    backward, from its plan: every stage's compulsory reads and writes."""
    gx, gy, h, w, L = list(pl.gx), list(pl.gy), list(pl.h), list(pl.w), pl.lmax
    npat = lambda l: gx[l] * gy[l]
    by = (pl.W1 * pl.H1 + pl.W2 * pl.H2) * (4 + 36 + 20)                 # descriptors: image in, FP32 + BF16 out
    by += pl.n_atomic * h[1] * w[1] * (4.0 + CODE_BYTES)                    # C'_0 + codes out of the correlation
    for l in range(1, L + 1):
        by += stage_work(pl, "level", l, "bf16")[1] + stage_work(pl, "backtrack", l, "bf16")[1]
    fl = 2.0 * pl.n_atomic * pl.H2 * pl.W2 * 144
    cb = CODE_BYTES
    # backward: the top and its gradient; per level adjoint, the pooled child
    # values (for the rectification factor) read and their gradient written,
    # the parent gradient and codes read; the bottom reads the pooled
    # gradient and codes of level 0 once and both descriptor fields, and
    # writes both gradients.
    bb = npat(L) * h[L] * w[L] * 8.0
    for l in range(1, L + 1):
        bb += npat(l - 1) * h[l] * w[l] * (4 + 4) + (npat(l) * h[l + 1] * w[l + 1] * (4.0 + cb) if l < L else 0)
    bb += pl.n_atomic * h[1] * w[1] * (4.0 + cb) + (pl.W1 * pl.H1 + pl.W2 * pl.H2) * 9 * 4 * 2
    return by, fl, bb, 2 * fl


def batch_bench(dm, torch, steps):
    import synth
    prm = dm.params(precision="bf16")
    pairs = synth.make_batch(32)
    sizes = [(p["img1"].shape[1], p["img1"].shape[0], p["img2"].shape[1], p["img2"].shape[0]) for p in pairs]
    i1 = [torch.from_numpy(p["img1"]).cuda() for p in pairs]
    i2 = [torch.from_numpy(p["img2"]).cuda() for p in pairs]
    plans = [dm.plan(*sz, prm) for sz in sizes]
    work = [pair_work(pl) for pl in plans]
    fwd_bytes = sum(x[0] for x in work)
    fwd_flops = sum(x[1] for x in work)
    all_bytes = fwd_bytes + sum(x[2] for x in work)
    all_flops = fwd_flops + sum(x[3] for x in work)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    res = {}
    B = dm.Batch(sizes, prm, bwd=True, graph=True, autotune=True)
    B.set_images(i1, i2)
    B.run()
    torch.cuda.synchronize()
    tiles = B.tiles()
    t = timed(B.run, steps)
    res["batch_fwd_bwd"] = dict(pairs_s=round(32 / t, 2), ms=round(t * 1e3, 3),
                                hbm_gbs=round(all_bytes / t / 1e9, 1),
                                mfma_util=round(all_flops / t / 1e12 / PEAKS_TFLOPS["bf16"], 4))
    n_launch = B.info.n_launches
    B.release()
    del B
    # the same pairs one by one: one-pair schedules of the same kernels, replayed in turn
    singles = []
    for k in range(32):
        S = dm.Batch([sizes[k]], prm, bwd=True, graph=True)
        S.set_images([i1[k]], [i2[k]])
        singles.append(S)
    t1 = timed(lambda: [S.run() for S in singles], max(1, steps // 2))
    res["one_by_one_fwd_bwd"] = dict(pairs_s=round(32 / t1, 2), ms=round(t1 * 1e3, 3),
                                     hbm_gbs=round(all_bytes / t1 / 1e9, 1),
                                     mfma_util=round(all_flops / t1 / 1e12 / PEAKS_TFLOPS["bf16"], 4))
    for S in singles:
        S.release()
    del singles
    F = dm.Batch(sizes, prm, bwd=False, graph=True, autotune=True)
    F.set_images(i1, i2)
    F.run()
    t2 = timed(F.run, steps)
    res["batch_fwd"] = dict(pairs_s=round(32 / t2, 2), ms=round(t2 * 1e3, 3), hbm_gbs=round(fwd_bytes / t2 / 1e9, 1),
                            mfma_util=round(fwd_flops / t2 / 1e12 / PEAKS_TFLOPS["bf16"], 4))
    F.release()
    del F
    ms = [dm.Matcher(*sz, prm) for sz in sizes]
    t3 = timed(lambda: [m.run_images(a, b) for m, a, b in zip(ms, i1, i2)], max(1, steps // 2))
    res["one_by_one_fwd"] = dict(pairs_s=round(32 / t3, 2), ms=round(t3 * 1e3, 3),
                                 hbm_gbs=round(fwd_bytes / t3 / 1e9, 1),
                                 mfma_util=round(fwd_flops / t3 / 1e12 / PEAKS_TFLOPS["bf16"], 4))
    del ms
    res["workload"] = ("32 uneven pairs, W ~ U{128..621}, H ~ U{96..188}, warped blurred noise (max 30 px); "
                       "BF16 correlation, FP32 pyramid; fwd_bwd = matches + gradient of the top loss")
    res["grouped_launches"] = n_launch
    res["tiles"] = dict(level_rows=tiles.level_rows, bt_rows=tiles.bt_rows, tuned_fwd_ms=round(tiles.tuned_ms, 3))
    res["algorithmic_gb_fwd_bwd"] = round(all_bytes / 1e9, 2)
    res["gflop_fwd_bwd"] = round(all_flops / 1e9, 1)
    return res


def approx_bench(dm, torch, img1, img2, exact_matches, exact_plan, steps, warmup):
    """Approximate DeepMatching (Sec. 4.1) on the same pair: D prototypes from
    10 rounds of spherical k-means, BF16 correlation of the D prototype maps."""
    import numpy as np
    res = {}
    for D in (1024, 64):
        dt, matches, stages, pl = time_path(dm, torch, img1, img2, "bf16", steps, warmup, prototypes=D)
        m = dm.Matcher(img1.shape[1], img1.shape[0], img2.shape[1], img2.shape[0],
                       dm.params(precision="bf16", prototypes=D))
        m.run_images(img1, img2)
        kstat = dm.workspace_views(m.ws, m.plan)["kstat"].cpu().numpy()
        km = [(n, l, c, t) for n, l, c, t in stages if n.startswith("kmeans")]
        km_ms = sum(t for _, _, _, t in km) / steps
        rows = roofline_of(stages, pl, "bf16")
        res[f"D{D}"] = dict(
            pairs_s=round(1.0 / dt, 3), ms_per_step=round(dt * 1e3, 4), matches=int(len(matches)),
            exact_matches_within_1px=round(within_1px(matches, exact_matches), 5),
            kmeans_ms=round(km_ms, 4),
            kmeans_assign=next(({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items() if k != "work"}
                                for r in rows if r["kernel"] == "kmeans_assign_l0"), None),
            settled_in_fp64=[int(kstat[0]), int(kstat[1])],
            workspace_mb=round(pl.workspace_bytes / 2**20, 1),
            top_kernels=[(r["kernel"], round(r["avg_ms"] * r["launches"] / steps, 4)) for r in rows[:6]])
        del m
    res["exact_workspace_mb"] = round(exact_plan.workspace_bytes / 2**20, 1)
    res["workload"] = ("the same 512x256 pair; 10 k-means rounds over its 8192 atomic patches; "
                       "BF16 correlation of the D prototype maps, FP32 pyramid")
    return res


def truth_within_1px(pair, matches):
    """Fraction of matches whose target lies within 1 px of where the pair's
    ground-truth field sends the source pixel (Table 1's accuracy measure on
    a synthetic pair)."""
    import numpy as np
    m = np.asarray(matches, dtype=np.float64)
    if len(m) == 0:
        return 0.0
    qx, qy = pair["flow"](m[:, 0], m[:, 1])
    return round(float((np.hypot(m[:, 2] - qx, m[:, 3] - qy) <= 1.0).mean()), 5)


def dmstar_bench(dm, torch, pair, img1, img2, plain_matches, plain_ms, steps, warmup):
    """DM* entry points (Sec. 3.3, Table 1's middle configuration) on the same
    pair: local maxima of every level start the backtracking, path-sum
    scores; BF16 correlation.  Entry counts of the pooled levels come from
    the marks the library leaves in the codes."""
    dt, matches, stages, pl = time_path(dm, torch, img1, img2, "bf16", steps, warmup, entry_points="local_maxima")
    m = dm.Matcher(img1.shape[1], img1.shape[0], img2.shape[1], img2.shape[0],
                   dm.params(precision="bf16", entry_points="local_maxima"))
    m.run_images(img1, img2)
    torch.cuda.synchronize()
    views = dm.workspace_views(m.ws, m.plan)
    entries = [int(((lv["code"] & 0x10) != 0).sum().item()) for lv in views["levels"]]
    del m
    rows = roofline_of(stages, pl, "bf16")
    dt_se, m_se, _, _ = time_path(dm, torch, img1, img2, "bf16", steps, warmup, entry_points="local_maxima",
                                  scoring="start_end")
    return dict(pairs_s=round(1.0 / dt, 3), ms_per_step=round(dt * 1e3, 4), vs_plain_ms=round(plain_ms, 4),
                matches=int(len(matches)), plain_matches=int(len(plain_matches)),
                plain_matches_within_1px=round(within_1px(matches, plain_matches), 5),
                truth_within_1px={"plain": truth_within_1px(pair, plain_matches),
                                  "dmstar": truth_within_1px(pair, matches),
                                  "dmstar_start_end": truth_within_1px(pair, m_se)},
                entries_per_pooled_level=entries,
                top_kernels=[(r["kernel"], round(r["avg_ms"] * r["launches"] / steps, 4)) for r in rows[:6]],
                start_end=dict(pairs_s=round(1.0 / dt_se, 3), ms_per_step=round(dt_se * 1e3, 4),
                               matches=int(len(m_se)),
                               plain_matches_within_1px=round(within_1px(m_se, plain_matches), 5)),
                workload="the same 512x256 pair; entry points at the local maxima of every level, path-sum "
                         "scores (start_end: start/end-point scores); BF16 correlation, FP32 pyramid")


def deepflow_bench(dm, torch, pair, img1, img2, matches, steps, warmup):
    """DeepFlow (Sec. 4.3) on the pair with the BF16 matches: time per pair
    (eager launches; with the launch graph beside it), the stage breakdown,
    the roofline of the SOR half-sweeps, and the end-point error against the
    pair's ground-truth field next to that of the matches themselves."""
    import numpy as np
    H, W = img1.shape
    f = dm.deepflow(img1, img2, matches)
    for _ in range(max(0, warmup - 1)):
        f = dm.deepflow(img1, img2, matches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f = dm.deepflow(img1, img2, matches)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    R = dm.DeepFlow(W, H, int(matches.shape[0]), graph=True)
    R.set(img1, img2, matches)
    R.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        R.run()
    torch.cuda.synchronize()
    dt_graph = (time.perf_counter() - t0) / steps
    R.release()
    dm.timing_enable(True)
    dm.deepflow(img1, img2, matches)
    torch.cuda.synchronize()
    rows = dm.timing_read()
    dm.timing_enable(False)
    agg = {}
    for name, level, count, ms in rows:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += count
        a[1] += ms
    # SOR launch on an n-pixel level (up to 10 half-sweeps on chip per
    # launch): every pixel's flow, increment, smoothness weight and five
    # system entries read once and its increment written once: 48 n bytes.
    # Pixel updates: every SOR sweep updates each pixel once.
    info = dm.flow_plan(W, H, int(matches.shape[0]))
    prm = dm.flow_params()
    sor_rows = [(level, count) for name, level, count, _ in rows if name == "df_sor"]
    sor_bytes = sum(48.0 * info.W[l] * info.H[l] * c for l, c in sor_rows)
    sor_updates = sum(float(info.W[l] * info.H[l]) * prm.n_fixed * prm.n_sor for l in {l for l, _ in sor_rows})
    sor_ms = agg.get("df_sor", [0, 0.0])[1]
    ach = sor_bytes / (sor_ms * 1e-3) / 1e9 if sor_ms else 0.0
    # end-point errors against the ground truth (interior, 16 px margin)
    flow = f.cpu().numpy()
    ys, xs = np.mgrid[16:H - 16, 16:W - 16]
    qx, qy = pair["flow"](xs.astype(np.float64), ys.astype(np.float64))
    epe = np.hypot(flow[16:H - 16, 16:W - 16, 0] - (qx - xs), flow[16:H - 16, 16:W - 16, 1] - (qy - ys))
    m = matches.cpu().numpy()
    mx, my = m[:, 0], m[:, 1]
    mqx, mqy = pair["flow"](mx, my)
    m_epe = np.hypot(m[:, 2] - mqx, m[:, 3] - mqy)
    return dict(ms_per_pair=round(dt * 1e3, 3), pairs_s=round(1.0 / dt, 3), ms_per_pair_graph=round(dt_graph * 1e3, 3),
                levels=int(info.n_levels), matches=int(matches.shape[0]),
                stage_ms={k: round(v[1], 3) for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1])[:6]},
                launches=int(sum(v[0] for v in agg.values())),
                sor_roofline={"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 4), "launches": int(agg.get("df_sor", [0])[0]),
                              "avg_us": round(sor_ms * 1e3 / max(1, agg.get("df_sor", [1])[0]), 2),
                              "pixel_updates_per_s": round(sor_updates / (sor_ms * 1e-3), 1) if sor_ms else None},
                epe_px={"mean": round(float(epe.mean()), 3), "median": round(float(np.median(epe)), 3),
                        "within_1px": round(float((epe < 1).mean()), 4)},
                match_epe_px={"mean": round(float(m_epe.mean()), 3), "median": round(float(np.median(m_epe)), 3)},
                workload="DeepFlow on the 512x256 pair, matches from the BF16 path, the paper's parameters "
                         "(eta 0.95: %d levels, 5 fixed points x 25 SOR sweeps per level), FP32" % info.n_levels)


def invariant_bench(dm, torch, img1, img2, plain_ms, steps, warmup):
    """Algorithm 2 on the pair: the full 9 x 8 grid, and per-stage times."""
    prm = dm.params(precision="bf16")
    info = dm.plan_invariant(img1.shape[1], img1.shape[0], img2.shape[1], img2.shape[0], prm)
    ws = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device="cuda")
    run = lambda: dm.match_invariant(img1, img2, prm, ws=ws)
    for _ in range(warmup):
        m = run()
    torch.cuda.synchronize()
    n = max(2, steps // 4)
    t0 = time.perf_counter()
    for _ in range(n):
        m = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    dm.timing_enable(True)
    run()
    torch.cuda.synchronize()
    stages = dm.timing_read()
    dm.timing_enable(False)
    per = {}
    for name, level, count, total in stages:
        key = name if level < 0 else f"{name}_l{level}"
        per[key] = per.get(key, 0.0) + total
    top = sorted(per.items(), key=lambda kv: -kv[1])[:6]
    return dict(pairs_s=round(1.0 / dt, 3), ms_per_step=round(dt * 1e3, 3), runs=int(info.n_runs),
                matches=int(len(m)), vs_plain=round(dt * 1e3 / plain_ms, 1),
                workspace_mb=round(info.workspace_bytes / 2**20, 1),
                top_stages_ms=[(k, round(v, 3)) for k, v in top],
                workload="the same 512x256 pair; sigma = -2..2 step 1/2, theta = 0..7 pi/4 (72 runs); "
                         "BF16 correlation, FP32 pyramid")


def _stored_oracle_matches():
    import numpy as np
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "c3_oracle.npz")
    return np.load(path)["matches"] if os.path.exists(path) else None


def oracle_agreement(matches):
    """Fraction of the stored oracle matches of the pair reproduced within 1 px."""
    ref = _stored_oracle_matches()
    return None if ref is None else round(within_1px(matches, ref), 5)


def oracle_score_error(matches):
    """Relative score error against the stored oracle matches, over the matches
    whose source and target pixels both equal the oracle's (and how many of the
    oracle's matches that is)."""
    import numpy as np
    ref = _stored_oracle_matches()
    if ref is None:
        return None
    g = {(int(r[0]), int(r[1])): r for r in matches}
    rel = []
    for r in ref:
        q = g.get((int(r[0]), int(r[1])))
        if q is not None and int(q[2]) == int(r[2]) and int(q[3]) == int(r[3]):
            rel.append(abs(float(q[4]) - float(r[4])) / abs(float(r[4])))
    if not rel:
        return {"same_coordinates": 0.0}
    rel = np.array(rel)
    return {"same_coordinates": round(len(rel) / len(ref), 5), "max": float("%.3g" % rel.max()),
            "median": float("%.3g" % np.median(rel))}


def copy_probe(torch):
    """A plain 1 GiB device-to-device copy: its FETCH_SIZE / WRITE_SIZE readings
    calibrate the HBM byte counters (1 GiB each way is the truth)."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def copy_bandwidth(torch, reps: int = 10) -> float:
    """Achievable HBM bandwidth on this GPU: a 1 GiB device-to-device copy
    (1 GiB read + 1 GiB written per copy), timed with HIP events; GB/s."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * (1 << 30) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the run, copy 1 GiB device to device (calibrates HBM byte counters)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 32-pair uneven batch")
    ap.add_argument("--no-approx", action="store_true", help="skip approximate DeepMatching")
    ap.add_argument("--no-invariant", action="store_true", help="skip scale and rotation invariant DeepMatching")
    ap.add_argument("--no-dmstar", action="store_true", help="skip the DM* entry points")
    ap.add_argument("--no-deepflow", action="store_true", help="skip DeepFlow")
    ap.add_argument("--only", choices=("all", "fwd_bf16", "fwd_bwd_bf16", "approx1024", "approx64", "invariant",
                                       "batch_fwd", "batch_fwd_bwd", "deepflow"),
                    default="all",
                    help="run only that pass (short profiler runs); prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the matcher has no multi-GPU path, "
                                   "run with --gpus 1"}))
        sys.exit(2)
    import torch
    import paper_1506_07656_amd as dm
    import synth

    pair = synth.make_pair("c3")
    img1 = torch.from_numpy(pair["img1"]).cuda()
    img2 = torch.from_numpy(pair["img2"]).cuda()
    if args.only == "fwd_bf16":
        dt, _, stages, pl = time_path(dm, torch, img1, img2, "bf16", args.steps, args.warmup)
        if args.copy_probe:
            copy_probe(torch)
        print(f"bf16 forward: {dt * 1e3:.3f} ms/pair", flush=True)
        for r in roofline_of(stages, pl, "bf16")[:8]:
            print(f"  {r['kernel']:<22} {r['avg_ms']:.4f} ms  {r['achieved']:.0f} {r['unit']}", flush=True)
        return
    if args.only == "invariant":
        prm = dm.params(precision="bf16")
        for _ in range(args.warmup):
            dm.match_invariant(img1, img2, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dm.match_invariant(img1, img2, prm)
        torch.cuda.synchronize()
        print(f"invariant (72 runs) bf16: {(time.perf_counter() - t0) / args.steps * 1e3:.3f} ms/pair", flush=True)
        return
    if args.only.startswith("approx"):
        D = int(args.only[len("approx"):])
        dt, _, _, _ = time_path(dm, torch, img1, img2, "bf16", args.steps, args.warmup, prototypes=D)
        print(f"approximate (D={D}) bf16 forward: {dt * 1e3:.3f} ms/pair", flush=True)
        return
    if args.only in ("batch_fwd", "batch_fwd_bwd"):   # the 32-pair uneven batch, autotuned, one graph replay per step
        import synth
        pairs = synth.make_batch(32)
        sizes = [(p["img1"].shape[1], p["img1"].shape[0], p["img2"].shape[1], p["img2"].shape[0]) for p in pairs]
        F = dm.Batch(sizes, dm.params(precision="bf16"), bwd=args.only == "batch_fwd_bwd", graph=True, autotune=True)
        F.set_images([torch.from_numpy(p["img1"]).cuda() for p in pairs],
                     [torch.from_numpy(p["img2"]).cuda() for p in pairs])
        for _ in range(max(1, args.warmup)):
            F.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            F.run()
        torch.cuda.synchronize()
        print(f"batch of 32 {args.only[6:]}: {(time.perf_counter() - t0) / args.steps * 1e3:.3f} ms", flush=True)
        F.release()
        return
    if args.only == "deepflow":
        m = dm.match_images(img1, img2, dm.params(precision="bf16"))
        r = deepflow_bench(dm, torch, pair, img1, img2, m, args.steps, args.warmup)
        print("deepflow: " + json.dumps(r), flush=True)
        return
    if args.only == "fwd_bwd_bf16":
        d1, d2 = dm.descriptors(img1), dm.descriptors(img2)
        dt, _ = time_fwd_bwd(dm, torch, d1, d2, "bf16", False, args.steps, args.warmup)
        if args.copy_probe:
            copy_probe(torch)
        print(f"bf16 forward + backward: {dt * 1e3:.3f} ms/pair", flush=True)
        return
    res = {}
    for prec in ("fp32", "bf16"):
        dt, matches, stages, pl = time_path(dm, torch, img1, img2, prec, args.steps, args.warmup)
        res[prec] = dict(ms=dt * 1e3, pairs_s=1.0 / dt, matches=matches, stages=stages, plan=pl)
    agree = within_1px(res["bf16"]["matches"], res["fp32"]["matches"])
    # fwd+bwd on leaf descriptors of the same pair
    d1 = dm.descriptors(img1)
    d2 = dm.descriptors(img2)
    fb = {}
    for prec in ("fp32", "bf16"):
        for rc in (False, True):
            dt, stages = time_fwd_bwd(dm, torch, d1, d2, prec, rc, max(3, args.steps // 2), 2)
            fb[f"{prec}{'_recompute' if rc else ''}"] = dict(pairs_s=round(1.0 / dt, 3), ms_per_step=round(dt * 1e3, 4),
                                                          stages=stages)
    head = res["bf16"]
    copy_gbs = copy_bandwidth(torch)
    rows = roofline_of(head["stages"], head["plan"], "bf16")
    dom = rows[0]
    rows32 = roofline_of(res["fp32"]["stages"], res["fp32"]["plan"], "fp32")
    out = {
        "metric": "pairs/s @512x256 fwd & fwd+bwd; BF16 vs FP32 plain at >=99% match agreement",
        "value": round(head["pairs_s"], 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "c3: 512x256 grayscale pair, blurred-noise content warped by a smooth field "
                               "(max 40 px) with gain; descriptors, pyramid to N_max=512, backtracking, "
                               "reciprocal matches", "W": 512, "H": 256, "N_max": head["plan"].N_max,
                   "global_batch": 1, "parallelism": "single GPU"},
        "fp32": {"pairs_s": round(res["fp32"]["pairs_s"], 3), "ms_per_step": round(res["fp32"]["ms"], 4),
                 "matches": int(len(res["fp32"]["matches"])),
                 "oracle_matches_within_1px": oracle_agreement(res["fp32"]["matches"]),
                 "oracle_score_rel_err": oracle_score_error(res["fp32"]["matches"])},
        "bf16": {"pairs_s": round(head["pairs_s"], 3), "ms_per_step": round(head["ms"], 4),
                 "matches": int(len(head["matches"])), "within_1px_of_fp32": round(agree, 5),
                 "oracle_matches_within_1px": oracle_agreement(head["matches"]),
                 "oracle_score_rel_err": oracle_score_error(head["matches"])},
        "fwd_bwd": {k: {kk: vv for kk, vv in v.items() if kk != "stages"} for k, v in fb.items()},
        "fwd_bwd_top_kernels_bf16": sorted([(n + ("" if l < 0 else "_l%d" % l), round(t / c, 4))
                                            for n, l, c, t in fb["bf16"]["stages"]], key=lambda x: -x[1])[:6],
        "fwd_bwd_top_kernels_fp32": sorted([(n + ("" if l < 0 else "_l%d" % l), round(t / c, 4))
                                            for n, l, c, t in fb["fp32"]["stages"]], key=lambda x: -x[1])[:6],
        "roofline": {"bound": dom["bound"], "kernel": dom["kernel"], "achieved": round(dom["achieved"], 2),
                     "peak": dom["peak"], "unit": dom["unit"], "frac": round(dom["frac"], 4),
                     "traffic": measured_traffic(dom["kernel"]),
                     "algorithmic_bytes": round(dom["work"]) if dom["unit"] == "GB/s" else None,
                     "avg_ms": round(dom["avg_ms"], 5),
                     # the same launch counted with the one-byte codes the library stores
                     "stored_achieved": round(dom.get("stored_achieved", 0.0), 2) or None,
                     "stored_frac": round(dom["stored_frac"], 4) if dom.get("stored_frac") else None,
                     # context: the bandwidth a plain 1 GiB copy reaches on this GPU
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(dom["achieved"] / copy_gbs, 4) if dom["unit"] == "GB/s" else None},
        "kernels_bf16": [dict({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items() if k != "work"},
                              traffic=measured_traffic(r["kernel"])) for r in rows],
        "kernels_fp32": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items() if k != "work"}
                         for r in rows32[:4]],
    }
    out["small_pairs"] = small_pairs(dm, torch, args.steps)
    if not args.no_approx:
        out["approx"] = approx_bench(dm, torch, img1, img2, head["matches"], head["plan"], args.steps, args.warmup)
    if not args.no_invariant:
        out["invariant"] = invariant_bench(dm, torch, img1, img2, head["ms"], args.steps, args.warmup)
    if not args.no_dmstar:
        out["dmstar"] = dmstar_bench(dm, torch, pair, img1, img2, head["matches"], head["ms"], args.steps,
                                     args.warmup)
    if not args.no_deepflow:
        out["deepflow"] = deepflow_bench(dm, torch, pair, img1, img2, torch.from_numpy(head["matches"]).cuda()
                                         if not torch.is_tensor(head["matches"]) else head["matches"],
                                         max(2, args.steps // 4), args.warmup)
    if not args.no_batch:
        out["batch"] = batch_bench(dm, torch, max(3, args.steps // 2))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pair)
    if args.copy_probe:
        copy_probe(torch)
        out["copy_probe_bytes"] = 1 << 30
    print(json.dumps(out))


if __name__ == "__main__":
    main()
