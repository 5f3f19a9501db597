"""ctypes binding of libdm.so.  Argument marshalling only: every stage of the
matching runs in the library's HIP kernels; torch supplies device memory and
the current stream.  There is no fallback: if the library is missing, every
call raises."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int, c_int32, c_size_t, c_uint64, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdm.so")

DM_MAX_LEVELS = 16
DM_FP32, DM_BF16, DM_FP64 = 0, 1, 2
PRECISIONS = {"fp32": DM_FP32, "bf16": DM_BF16, "fp64": DM_FP64}
STATUS = {0: "DM_OK", -1: "DM_ERR_INVALID_ARG", -2: "DM_ERR_SHAPE", -3: "DM_ERR_WORKSPACE",
          -4: "DM_ERR_CAPACITY", -5: "DM_ERR_UNSUPPORTED", -6: "DM_ERR_HIP"}


class DMError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


class Params(ctypes.Structure):
    _fields_ = [("nu1", c_float), ("nu2", c_float), ("nu3", c_float), ("sigmoid_slope", c_float),
                ("mu", c_float), ("intensity_scale", c_float), ("lam", c_float),
                ("max_patch", c_int32), ("precision", c_int32), ("prototypes", c_int32),
                ("kmeans_iters", c_int32), ("entry_points", c_int32), ("scoring", c_int32),
                ("reserved", c_int32 * 3)]


NOALLOC_MAX_BYTES = 128 << 20   # the static workspace of dm_match_images_noalloc

DM_ENTRIES_TOP = 0
DM_ENTRIES_LOCAL_MAXIMA = 1
DM_SCORE_PATH_SUM = 0
DM_SCORE_START_END = 1


class Match(ctypes.Structure):
    _fields_ = [("x1", c_int32), ("y1", c_int32), ("x2", c_int32), ("y2", c_int32), ("score", c_float)]


_L = DM_MAX_LEVELS


class PlanInfo(ctypes.Structure):
    _fields_ = [("W1", c_int32), ("H1", c_int32), ("W2", c_int32), ("H2", c_int32),
                ("lmax", c_int32), ("N_max", c_int32), ("n_atomic", c_int32), ("max_matches", c_int32),
                ("precision", c_int32),
                ("gx", c_int32 * _L), ("gy", c_int32 * _L), ("n_valid", c_int32 * _L),
                ("h", c_int32 * (_L + 1)), ("w", c_int32 * (_L + 1)),
                ("off_cp", c_uint64 * _L), ("off_code", c_uint64 * _L), ("off_u", c_uint64 * _L),
                ("off_top", c_uint64), ("off_desc1", c_uint64), ("off_desc2", c_uint64),
                ("off_bf1", c_uint64), ("off_bf2", c_uint64), ("off_valid", c_uint64),
                ("off_best", c_uint64), ("off_cell", c_uint64), ("off_misc", c_uint64),
                ("prototypes", c_int32), ("kmeans_chunks", c_int32),
                ("off_protos", c_uint64), ("off_assign", c_uint64), ("off_kstat", c_uint64),
                ("off_proto_img", c_uint64), ("off_proto_bf", c_uint64), ("off_kpart", c_uint64),
                ("workspace_bytes", c_uint64)]


class GradPlan(ctypes.Structure):
    _fields_ = [("geom", PlanInfo), ("recompute", c_int32), ("nsplit", c_int32),
                ("saved_bytes", c_uint64), ("scratch_bytes", c_uint64),
                ("off_cp", c_uint64 * _L), ("off_code", c_uint64 * _L), ("cp_in_saved", c_int32 * _L),
                ("off_top", c_uint64), ("off_valid", c_uint64), ("off_bf1", c_uint64), ("off_bf2", c_uint64),
                ("off_g", c_uint64 * 2), ("off_part", c_uint64), ("off_t", c_uint64), ("off_dense", c_uint64)]


DM_INV_MAX_RUNS = 72


class InvariantInfo(ctypes.Structure):
    _fields_ = [("n_runs", c_int32), ("max_matches", c_int32),
                ("run_k", c_int32 * DM_INV_MAX_RUNS), ("run_r", c_int32 * DM_INV_MAX_RUNS),
                ("run_W1", c_int32 * DM_INV_MAX_RUNS), ("run_H1", c_int32 * DM_INV_MAX_RUNS),
                ("run_W2", c_int32 * DM_INV_MAX_RUNS), ("run_H2", c_int32 * DM_INV_MAX_RUNS),
                ("off_best", c_uint64), ("off_cell", c_uint64), ("off_img1", c_uint64), ("off_img2", c_uint64),
                ("off_run", c_uint64), ("workspace_bytes", c_uint64)]


class StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("level", c_int32), ("count", c_int32), ("total_ms", ctypes.c_double)]


DM_MAX_BATCH = 256
DM_BATCH_BWD, DM_BATCH_GRAPH, DM_BATCH_AUTOTUNE = 1, 2, 4


class Pair(ctypes.Structure):
    _fields_ = [("img1", c_void_p), ("W1", c_int32), ("H1", c_int32), ("ld1", c_int32),
                ("img2", c_void_p), ("W2", c_int32), ("H2", c_int32), ("ld2", c_int32),
                ("dd1", c_void_p), ("dd2", c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_pairs", c_int32), ("n_launches", c_int32), ("max_matches", c_int32 * DM_MAX_BATCH),
                ("lmax", c_int32 * DM_MAX_BATCH), ("workspace_bytes", c_uint64)]


class BatchTiles(ctypes.Structure):
    _fields_ = [("level_rows", c_int32), ("bt_rows", c_int32), ("blocks_per_cu", c_int32 * 32),
                ("tuned", c_int32), ("tuned_ms", c_float)]


DM_FLOW_MAX_LEVELS = 128


class FlowParams(ctypes.Structure):
    _fields_ = [("sigma", c_float), ("eta", c_float), ("min_size", c_int32), ("n_fixed", c_int32),
                ("n_sor", c_int32), ("omega", c_float), ("kappa", c_float), ("beta", c_float), ("b", c_float),
                ("gamma", c_float), ("delta", c_float), ("eps", c_float), ("zeta", c_float),
                ("sigma_m", c_float), ("lam_scale", c_float), ("reserved", c_int32 * 4)]


class FlowInfo(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("W", c_int32 * DM_FLOW_MAX_LEVELS), ("H", c_int32 * DM_FLOW_MAX_LEVELS),
                ("workspace_bytes", c_uint64)]


# name -> (restype, argtypes); every symbol declared in include/dm.h.
SIGNATURES = {
    "dm_default_params": (c_int, [POINTER(Params)]),
    "dm_plan": (c_int, [POINTER(Params), c_int, c_int, c_int, c_int, POINTER(PlanInfo)]),
    "dm_descriptors": (c_int, [c_void_p, c_int, c_int, c_int, POINTER(Params), c_void_p, c_void_p]),
    "dm_match_descriptors": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, POINTER(Params),
                                     c_void_p, c_size_t, c_void_p, c_int, c_void_p, c_void_p]),
    "dm_match_images": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_int, c_int,
                                POINTER(Params), c_void_p, c_size_t, c_void_p, c_int, c_void_p, c_void_p]),
    "dm_match_images_noalloc": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_int, c_int,
                                        POINTER(Params), c_void_p, c_int, c_void_p, c_void_p]),
    "dm_plan_grad": (c_int, [POINTER(Params), c_int, c_int, c_int, c_int, c_int, POINTER(GradPlan)]),
    "dm_pyramid_forward": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, POINTER(Params), c_int,
                                   c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "dm_pyramid_backward": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, POINTER(Params), c_int,
                                    c_void_p, c_size_t, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                    c_void_p]),
    "dm_plan_batch": (c_int, [c_int, POINTER(Pair), POINTER(Params), c_int, POINTER(BatchInfo)]),
    "dm_match_batch": (c_int, [c_int, POINTER(Pair), POINTER(Params), c_int, c_void_p, c_size_t, c_void_p,
                               POINTER(c_int32), c_void_p, c_void_p]),
    "dm_batch_tiles_get": (c_int, [c_void_p, POINTER(BatchTiles)]),
    "dm_batch_release": (c_int, [c_void_p]),
    "dm_plan_invariant": (c_int, [POINTER(Params), c_int, c_int, c_int, c_int, ctypes.c_uint32, ctypes.c_uint32,
                                  POINTER(InvariantInfo)]),
    "dm_match_invariant": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_int, c_int, POINTER(Params),
                                   ctypes.c_uint32, ctypes.c_uint32, c_void_p, c_size_t, c_void_p, c_int, c_void_p,
                                   c_void_p]),
    "dm_flow_default_params": (c_int, [POINTER(FlowParams)]),
    "dm_flow_plan": (c_int, [c_int, c_int, c_int, POINTER(FlowParams), POINTER(FlowInfo)]),
    "dm_deepflow": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_int,
                            POINTER(FlowParams), c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "dm_flow_release": (c_int, [c_void_p]),
    "dm_timing_enable": (c_int, [c_int]),
    "dm_timing_read": (c_int, [POINTER(StageTime), c_int, POINTER(c_int)]),
    "dm_status_string": (c_char_p, [c_int]),
    "dm_last_error": (c_char_p, []),
    "dm_version": (c_char_p, []),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1506_07656_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise DMError(status, lib().dm_last_error().decode())


def params(**kw) -> Params:
    """Library defaults overridden by keyword (nu1, nu2, nu3, sigmoid_slope, mu,
    intensity_scale, lam, max_patch, precision in {'fp32','bf16','fp64'} or int,
    prototypes, kmeans_iters, entry_points in {'top', 'local_maxima'} or int,
    scoring in {'path_sum', 'start_end'} or int)."""
    p = Params()
    _check(lib().dm_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "entry_points" and isinstance(v, str):
            v = {"top": DM_ENTRIES_TOP, "local_maxima": DM_ENTRIES_LOCAL_MAXIMA}[v]
        if k == "scoring" and isinstance(v, str):
            v = {"path_sum": DM_SCORE_PATH_SUM, "start_end": DM_SCORE_START_END}[v]
        if k == "lambda":
            k = "lam"
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def plan(W1: int, H1: int, W2: int, H2: int, prm: Params | None = None) -> PlanInfo:
    prm = prm or params()
    out = PlanInfo()
    _check(lib().dm_plan(ctypes.byref(prm), W1, H1, W2, H2, ctypes.byref(out)))
    return out


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, ndim: int, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or t.dim() != ndim:
        raise ValueError(f"{name} must be {dtype} with {ndim} dims")
    return t


def workspace(pl: PlanInfo, device=None) -> torch.Tensor:
    """A device byte tensor of the planned workspace size (256-byte aligned by
    the caching allocator)."""
    return torch.empty(int(pl.workspace_bytes), dtype=torch.uint8, device=device or "cuda")


def descriptors(img: torch.Tensor, prm: Params | None = None) -> torch.Tensor:
    """H x W float32 image in [0, 1] -> H x W x 9 descriptors."""
    prm = prm or params()
    img = _dev(img, torch.float32, 2, "img")
    H, W = img.shape
    out = torch.empty((H, W, 9), dtype=torch.float32, device=img.device)
    _check(lib().dm_descriptors(c_void_p(img.data_ptr()), W, H, img.stride(0), ctypes.byref(prm),
                                c_void_p(out.data_ptr()), _stream()))
    return out


def _matches_tensor(buf: torch.Tensor, n: int) -> torch.Tensor:
    rec = buf[:n]
    out = torch.empty((n, 5), dtype=torch.float64, device=buf.device)
    out[:, :4] = rec[:, :4].to(torch.float64)
    out[:, 4] = rec[:, 4].view(torch.float32).to(torch.float64)
    return out


def match_descriptors(d1: torch.Tensor, d2: torch.Tensor, prm: Params | None = None,
                      ws: torch.Tensor | None = None, return_state: bool = False):
    """Descriptors (H x W x 9 float32) -> matches (n x 5: x1, y1, x2, y2, score)."""
    prm = prm or params()
    d1 = _dev(d1, torch.float32, 3, "d1")
    d2 = _dev(d2, torch.float32, 3, "d2")
    H1, W1, _ = d1.shape
    H2, W2, _ = d2.shape
    pl = plan(W1, H1, W2, H2, prm)
    ws = workspace(pl, d1.device) if ws is None else ws
    buf = torch.empty((pl.max_matches, 5), dtype=torch.int32, device=d1.device)
    n_out = torch.zeros(1, dtype=torch.int32, device=d1.device)
    _check(lib().dm_match_descriptors(c_void_p(d1.contiguous().data_ptr()), W1, H1,
                                      c_void_p(d2.contiguous().data_ptr()), W2, H2, ctypes.byref(prm),
                                      c_void_p(ws.data_ptr()), ws.numel(), c_void_p(buf.data_ptr()),
                                      pl.max_matches, c_void_p(n_out.data_ptr()), _stream()))
    m = _matches_tensor(buf, int(n_out.item()))
    return (m, ws, pl) if return_state else m


def match_images(img1: torch.Tensor, img2: torch.Tensor, prm: Params | None = None,
                 ws: torch.Tensor | None = None, return_state: bool = False):
    """Two H x W float32 images in [0, 1] -> matches (n x 5: x1, y1, x2, y2, score)."""
    prm = prm or params()
    img1 = _dev(img1, torch.float32, 2, "img1")
    img2 = _dev(img2, torch.float32, 2, "img2")
    H1, W1 = img1.shape
    H2, W2 = img2.shape
    pl = plan(W1, H1, W2, H2, prm)
    ws = workspace(pl, img1.device) if ws is None else ws
    buf = torch.empty((pl.max_matches, 5), dtype=torch.int32, device=img1.device)
    n_out = torch.zeros(1, dtype=torch.int32, device=img1.device)
    _check(lib().dm_match_images(c_void_p(img1.data_ptr()), W1, H1, img1.stride(0),
                                 c_void_p(img2.data_ptr()), W2, H2, img2.stride(0), ctypes.byref(prm),
                                 c_void_p(ws.data_ptr()), ws.numel(), c_void_p(buf.data_ptr()),
                                 pl.max_matches, c_void_p(n_out.data_ptr()), _stream()))
    m = _matches_tensor(buf, int(n_out.item()))
    return (m, ws, pl) if return_state else m


def match_images_noalloc(img1: torch.Tensor, img2: torch.Tensor, prm: Params | None = None) -> torch.Tensor:
    """match_images for callers that cannot allocate a workspace: the
    library's static device array of NOALLOC_MAX_BYTES serves as one (pairs
    whose workspace is larger are rejected).  Only the outputs are allocated
    here.  Calls that overlap on one GPU share that array and race."""
    prm = prm or params()
    img1 = _dev(img1, torch.float32, 2, "img1")
    img2 = _dev(img2, torch.float32, 2, "img2")
    H1, W1 = img1.shape
    H2, W2 = img2.shape
    pl = plan(W1, H1, W2, H2, prm)
    buf = torch.empty((pl.max_matches, 5), dtype=torch.int32, device=img1.device)
    n_out = torch.zeros(1, dtype=torch.int32, device=img1.device)
    _check(lib().dm_match_images_noalloc(c_void_p(img1.data_ptr()), W1, H1, img1.stride(0),
                                         c_void_p(img2.data_ptr()), W2, H2, img2.stride(0), ctypes.byref(prm),
                                         c_void_p(buf.data_ptr()), pl.max_matches, c_void_p(n_out.data_ptr()),
                                         _stream()))
    return _matches_tensor(buf, int(n_out.item()))


def flow_params(**kw) -> FlowParams:
    """The paper's DeepFlow parameters (dm_flow_default_params), with overrides."""
    p = FlowParams()
    _check(lib().dm_flow_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def flow_plan(W: int, H: int, max_matches: int = 0, prm: FlowParams | None = None) -> FlowInfo:
    info = FlowInfo()
    _check(lib().dm_flow_plan(W, H, max_matches, ctypes.byref(prm or flow_params()), ctypes.byref(info)))
    return info


def deepflow(img1: torch.Tensor, img2: torch.Tensor, matches: torch.Tensor | None = None,
             n_matches: torch.Tensor | None = None, prm: FlowParams | None = None,
             ws: torch.Tensor | None = None) -> torch.Tensor:
    """Flow (H x W x 2) from img1 to img2 (H x W float32 images in [0, 1])
    with DeepMatching's matches: an n x 4 or n x 5 device tensor of rows
    (x1, y1, x2, y2[, score]) as match_images returns them (any dtype; the
    coordinates are rounded to whole pixels), or the library's own n x 5
    int32 records; n_matches optionally a device count that limits how many
    rows are used."""
    prm = prm or flow_params()
    img1 = _dev(img1, torch.float32, 2, "img1")
    img2 = _dev(img2, torch.float32, 2, "img2")
    if img1.shape != img2.shape:
        raise ValueError("DeepFlow needs two images of one size")
    H, W = img1.shape
    if matches is None:
        matches = torch.zeros((0, 5), dtype=torch.int32, device=img1.device)
    if not matches.is_cuda or matches.dim() != 2 or matches.shape[1] not in (4, 5):
        raise ValueError("matches must be an n x 4 or n x 5 device tensor")
    if matches.dtype != torch.int32 or matches.shape[1] != 5:   # marshal into dm_match records
        rec = torch.zeros((matches.shape[0], 5), dtype=torch.int32, device=matches.device)
        rec[:, :4] = torch.round(matches[:, :4].to(torch.float64)).to(torch.int32)
        if matches.shape[1] == 5:
            rec[:, 4] = matches[:, 4].to(torch.float32).view(torch.int32)
        matches = rec
    matches = matches.contiguous()
    nm = matches.shape[0]
    if n_matches is None:
        n_matches = torch.full((1,), nm, dtype=torch.int32, device=img1.device)
    info = flow_plan(W, H, nm, prm)
    ws = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=img1.device) if ws is None else ws
    flow = torch.empty((H, W, 2), dtype=torch.float32, device=img1.device)
    _check(lib().dm_deepflow(c_void_p(img1.data_ptr()), c_void_p(img2.data_ptr()), W, H, img1.stride(0),
                             c_void_p(matches.data_ptr() if nm else None),
                             c_void_p(n_matches.data_ptr() if nm else None), nm, ctypes.byref(prm), 0,
                             c_void_p(flow.data_ptr()), c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return flow


DM_FLOW_GRAPH = 1


class DeepFlow:
    """Repeated DeepFlow on W x H pairs with up to max_matches matches, its
    launches captured into one HIP graph (DM_FLOW_GRAPH) and replayed.  The
    inputs, workspace and output live here so that every call presents the
    same arguments; set() copies a pair (and its matches) in, run() enqueues
    the flow on a side stream of default priority, joined with the current
    stream on entry and exit."""

    def __init__(self, W: int, H: int, max_matches: int, prm: FlowParams | None = None, graph: bool = True,
                 device="cuda"):
        self.W, self.H, self.max_matches = W, H, max_matches
        self.prm = prm or flow_params()
        self.flags = DM_FLOW_GRAPH if graph else 0
        self.img1 = torch.zeros((H, W), dtype=torch.float32, device=device)
        self.img2 = torch.zeros((H, W), dtype=torch.float32, device=device)
        self.matches = torch.zeros((max(1, max_matches), 5), dtype=torch.int32, device=device)
        self.n = torch.zeros(1, dtype=torch.int32, device=device)
        info = flow_plan(W, H, max_matches, self.prm)
        self.ws = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=device)
        self.flow = torch.zeros((H, W, 2), dtype=torch.float32, device=device)
        self.stream = torch.cuda.Stream(device=device)

    def set(self, img1: torch.Tensor, img2: torch.Tensor, matches: torch.Tensor | None = None,
            n_matches: torch.Tensor | None = None):
        """Copies the images and the first rows of matches (as deepflow()
        takes them) in; n_matches (device) may limit the count further."""
        self.img1.copy_(img1)
        self.img2.copy_(img2)
        k = 0 if matches is None else min(int(matches.shape[0]), self.max_matches)
        if k:
            rec = torch.zeros((k, 5), dtype=torch.int32, device=self.img1.device)
            rec[:, :4] = torch.round(matches[:k, :4].to(torch.float64)).to(torch.int32)
            self.matches[:k].copy_(rec)
        self.n.fill_(k)
        if n_matches is not None:
            torch.minimum(self.n, n_matches.to(torch.int32).reshape(1), out=self.n)

    def run(self) -> torch.Tensor:
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            _check(lib().dm_deepflow(c_void_p(self.img1.data_ptr()), c_void_p(self.img2.data_ptr()), self.W, self.H,
                                     self.W, c_void_p(self.matches.data_ptr()), c_void_p(self.n.data_ptr()),
                                     self.max_matches, ctypes.byref(self.prm), self.flags,
                                     c_void_p(self.flow.data_ptr()), c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                     c_void_p(self.stream.cuda_stream)))
        cur.wait_stream(self.stream)
        return self.flow

    def release(self):
        lib().dm_flow_release(c_void_p(self.ws.data_ptr()))


def plan_invariant(W1: int, H1: int, W2: int, H2: int, prm: Params | None = None, scales_mask: int = 0x1FF,
                   rotations_mask: int = 0xFF) -> InvariantInfo:
    prm = prm or params()
    out = InvariantInfo()
    _check(lib().dm_plan_invariant(ctypes.byref(prm), W1, H1, W2, H2, ctypes.c_uint32(scales_mask),
                                   ctypes.c_uint32(rotations_mask), ctypes.byref(out)))
    return out


def match_invariant(img1: torch.Tensor, img2: torch.Tensor, prm: Params | None = None, scales_mask: int = 0x1FF,
                    rotations_mask: int = 0xFF, ws: torch.Tensor | None = None, return_state: bool = False):
    """Scale and rotation invariant matches (Sec. 4.2) of two H x W float32
    images: sigma = k/2 for the set bits k + 4 of scales_mask, theta = r pi/4
    for the set bits r of rotations_mask.  Returns (n x 5: x1, y1, x2, y2,
    score), ordered by source cell."""
    prm = prm or params()
    img1 = _dev(img1, torch.float32, 2, "img1")
    img2 = _dev(img2, torch.float32, 2, "img2")
    H1, W1 = img1.shape
    H2, W2 = img2.shape
    info = plan_invariant(W1, H1, W2, H2, prm, scales_mask, rotations_mask)
    ws = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=img1.device) if ws is None else ws
    buf = torch.empty((info.max_matches, 5), dtype=torch.int32, device=img1.device)
    n_out = torch.zeros(1, dtype=torch.int32, device=img1.device)
    _check(lib().dm_match_invariant(c_void_p(img1.data_ptr()), W1, H1, img1.stride(0),
                                    c_void_p(img2.data_ptr()), W2, H2, img2.stride(0), ctypes.byref(prm),
                                    ctypes.c_uint32(scales_mask), ctypes.c_uint32(rotations_mask),
                                    c_void_p(ws.data_ptr()), ws.numel(), c_void_p(buf.data_ptr()),
                                    info.max_matches, c_void_p(n_out.data_ptr()), _stream()))
    m = _matches_tensor(buf, int(n_out.item()))
    return (m, ws, info) if return_state else m


class Matcher:
    """Preallocated workspace and output buffers for repeated matching of
    pairs of one size; run() only enqueues work on the current stream."""

    def __init__(self, W1: int, H1: int, W2: int, H2: int, prm: Params | None = None, device="cuda"):
        self.prm = prm or params()
        self.plan = plan(W1, H1, W2, H2, self.prm)
        self.shape = (W1, H1, W2, H2)
        self.ws = workspace(self.plan, device)
        self.buf = torch.empty((self.plan.max_matches, 5), dtype=torch.int32, device=device)
        self.n_out = torch.zeros(1, dtype=torch.int32, device=device)

    def run_images(self, img1: torch.Tensor, img2: torch.Tensor):
        W1, H1, W2, H2 = self.shape
        assert tuple(img1.shape) == (H1, W1) and tuple(img2.shape) == (H2, W2)
        _check(lib().dm_match_images(c_void_p(img1.data_ptr()), W1, H1, img1.stride(0),
                                     c_void_p(img2.data_ptr()), W2, H2, img2.stride(0), ctypes.byref(self.prm),
                                     c_void_p(self.ws.data_ptr()), self.ws.numel(), c_void_p(self.buf.data_ptr()),
                                     self.plan.max_matches, c_void_p(self.n_out.data_ptr()), _stream()))

    def run_descriptors(self, d1: torch.Tensor, d2: torch.Tensor):
        W1, H1, W2, H2 = self.shape
        assert d1.is_contiguous() and d2.is_contiguous()
        _check(lib().dm_match_descriptors(c_void_p(d1.data_ptr()), W1, H1, c_void_p(d2.data_ptr()), W2, H2,
                                          ctypes.byref(self.prm), c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                          c_void_p(self.buf.data_ptr()), self.plan.max_matches,
                                          c_void_p(self.n_out.data_ptr()), _stream()))

    def result(self) -> torch.Tensor:
        """Matches of the last run (synchronises on the count)."""
        return _matches_tensor(self.buf, int(self.n_out.item()))


def workspace_views(ws: torch.Tensor, pl: PlanInfo) -> dict:
    """Typed views of the pyramid a match call leaves in its workspace."""
    fsz = 8 if pl.precision == DM_FP64 else 4
    fdt = torch.float64 if pl.precision == DM_FP64 else torch.float32

    def view(off, count, dtype, shape, esz):
        return ws[off:off + count * esz].view(dtype).view(*shape)

    levels = []
    for lv in range(pl.lmax):
        shp = (pl.gy[lv], pl.gx[lv], pl.h[lv + 1], pl.w[lv + 1])
        if lv == 0 and pl.prototypes:   # the D prototype maps
            shp = (1, pl.prototypes, pl.h[1], pl.w[1])
        n = shp[0] * shp[1] * shp[2] * shp[3]
        d = dict(cp=view(pl.off_cp[lv], n, fdt, shp, fsz), code=view(pl.off_code[lv], n, torch.uint8, shp, 1))
        if lv >= 1:
            d["u"] = view(pl.off_u[lv], n, fdt, shp, fsz)
        levels.append(d)
    L = pl.lmax
    tshp = (pl.gy[L], pl.gx[L], pl.h[L], pl.w[L])
    top = view(pl.off_top, tshp[0] * tshp[1] * tshp[2] * tshp[3], fdt, tshp, fsz)
    out = dict(levels=levels, top=top)
    out["best"] = view(pl.off_best, pl.n_atomic, torch.int64, (pl.n_atomic,), 8)
    out["desc1"] = view(pl.off_desc1, pl.H1 * pl.W1 * 9, fdt, (pl.H1, pl.W1, 9), fsz)
    out["desc2"] = view(pl.off_desc2, pl.H2 * pl.W2 * 9, fdt, (pl.H2, pl.W2, 9), fsz)
    if pl.prototypes:
        D = pl.prototypes
        out["protos"] = view(pl.off_protos, D * 144, torch.float64, (D, 144), 8)
        out["assign"] = view(pl.off_assign, pl.n_atomic, torch.int32, (pl.gy[0], pl.gx[0]), 4)
        out["kstat"] = view(pl.off_kstat, 2, torch.int32, (2,), 4)
    return out


def plan_grad(W1: int, H1: int, W2: int, H2: int, prm: Params | None = None, recompute: bool = False) -> GradPlan:
    prm = prm or params()
    out = GradPlan()
    _check(lib().dm_plan_grad(ctypes.byref(prm), W1, H1, W2, H2, int(recompute), ctypes.byref(out)))
    return out


class Pyramid:
    """State of dm_pyramid_forward for one pair of descriptor fields: the
    `saved` buffer the backward needs and a transient `scratch` buffer."""

    def __init__(self, d1: torch.Tensor, d2: torch.Tensor, prm: Params | None = None, recompute: bool = False):
        self.prm = prm or params()
        fdt = torch.float64 if self.prm.precision == DM_FP64 else torch.float32
        self.d1 = _dev(d1, fdt, 3, "d1").contiguous()
        self.d2 = _dev(d2, fdt, 3, "d2").contiguous()
        H1, W1, _ = self.d1.shape
        H2, W2, _ = self.d2.shape
        self.dims = (W1, H1, W2, H2)
        self.recompute = bool(recompute)
        self.plan = plan_grad(W1, H1, W2, H2, self.prm, self.recompute)
        dev = self.d1.device
        self.saved = torch.empty(int(self.plan.saved_bytes), dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(int(self.plan.scratch_bytes), dtype=torch.uint8, device=dev)
        self.fdt = fdt

    def top_shape(self):
        g = self.plan.geom
        L = g.lmax
        return (g.gy[L], g.gx[L], g.h[L], g.w[L])

    def top(self) -> torch.Tensor:
        shp = self.top_shape()
        n = shp[0] * shp[1] * shp[2] * shp[3]
        es = 8 if self.fdt == torch.float64 else 4
        o = int(self.plan.off_top)
        return self.saved[o:o + n * es].view(self.fdt).view(*shp)

    def forward(self):
        W1, H1, W2, H2 = self.dims
        _check(lib().dm_pyramid_forward(c_void_p(self.d1.data_ptr()), W1, H1, c_void_p(self.d2.data_ptr()), W2, H2,
                                        ctypes.byref(self.prm), int(self.recompute), c_void_p(self.saved.data_ptr()),
                                        self.saved.numel(), c_void_p(self.scratch.data_ptr()), self.scratch.numel(),
                                        _stream()))
        return self.top()

    def backward(self, dtop: torch.Tensor):
        W1, H1, W2, H2 = self.dims
        dtop = dtop.to(self.fdt).contiguous()
        assert tuple(dtop.shape) == self.top_shape()
        dd1 = torch.empty_like(self.d1)
        dd2 = torch.empty_like(self.d2)
        _check(lib().dm_pyramid_backward(c_void_p(self.d1.data_ptr()), W1, H1, c_void_p(self.d2.data_ptr()), W2, H2,
                                         ctypes.byref(self.prm), int(self.recompute),
                                         c_void_p(self.saved.data_ptr()), self.saved.numel(),
                                         c_void_p(dtop.data_ptr()), c_void_p(dd1.data_ptr()), c_void_p(dd2.data_ptr()),
                                         c_void_p(self.scratch.data_ptr()), self.scratch.numel(), _stream()))
        return dd1, dd2


class DMPyramid(torch.autograd.Function):
    """C_top = pyramid(d1, d2) with the library's hand-written backward.

    forward(d1, d2, prm, recompute) -> C_top [gy, gx, h, w] of the top level
    (maps of non-existing top patches are zeros)."""

    @staticmethod
    def forward(ctx, d1, d2, prm=None, recompute=False):
        pyr = Pyramid(d1.detach(), d2.detach(), prm, recompute)
        top = pyr.forward().clone()
        ctx.pyr = pyr
        return top

    @staticmethod
    def backward(ctx, dtop):
        dd1, dd2 = ctx.pyr.backward(dtop)
        ctx.pyr = None
        return dd1, dd2, None, None


class Batch:
    """Many image pairs of uneven sizes matched together (dm_match_batch).

    Buffers (workspace, outputs, gradients) live here so that repeated
    run() calls present the same arguments and replay the cached schedule
    (with graph=True, one HIP graph launch per call).  Calls go to a side
    stream of default priority, joined with the current stream on entry and
    exit.  Images are copied into the batch's own input buffers by
    set_images(); run() takes no tensors."""

    def __init__(self, sizes, prm: Params | None = None, bwd: bool = False, graph: bool = True,
                 autotune: bool = False, device="cuda"):
        self.prm = prm or params()
        self.sizes = [tuple(int(v) for v in sz) for sz in sizes]   # (W1, H1, W2, H2)
        self.n = len(self.sizes)
        self.flags = (DM_BATCH_BWD if bwd else 0) | (DM_BATCH_GRAPH if graph else 0) | \
            (DM_BATCH_AUTOTUNE if autotune else 0)
        self.img1 = [torch.zeros((H1, W1), dtype=torch.float32, device=device) for W1, H1, _, _ in self.sizes]
        self.img2 = [torch.zeros((H2, W2), dtype=torch.float32, device=device) for _, _, W2, H2 in self.sizes]
        self.dd1 = [torch.zeros((H1, W1, 9), dtype=torch.float32, device=device) if bwd else None
                    for W1, H1, _, _ in self.sizes]
        self.dd2 = [torch.zeros((H2, W2, 9), dtype=torch.float32, device=device) if bwd else None
                    for _, _, W2, H2 in self.sizes]
        self.pairs = (Pair * self.n)()
        for k, (W1, H1, W2, H2) in enumerate(self.sizes):
            self.pairs[k] = Pair(self.img1[k].data_ptr(), W1, H1, W1, self.img2[k].data_ptr(), W2, H2, W2,
                                 self.dd1[k].data_ptr() if bwd else None, self.dd2[k].data_ptr() if bwd else None)
        self.info = BatchInfo()
        _check(lib().dm_plan_batch(self.n, self.pairs, ctypes.byref(self.prm), self.flags, ctypes.byref(self.info)))
        offs, o = [], 0
        for k in range(self.n):
            offs.append(o)
            o += self.info.max_matches[k]
        self.offsets = (c_int32 * self.n)(*offs)
        self.out = torch.empty((max(1, o), 5), dtype=torch.int32, device=device)
        self.n_out = torch.zeros(self.n, dtype=torch.int32, device=device)
        self.ws = torch.empty(int(self.info.workspace_bytes), dtype=torch.uint8, device=device)
        self.stream = torch.cuda.Stream(device=device)

    def set_images(self, imgs1, imgs2):
        for k in range(self.n):
            self.img1[k].copy_(imgs1[k])
            self.img2[k].copy_(imgs2[k])

    def run(self):
        """Enqueue the batch (on the side stream, ordered after the current
        stream's work; the current stream waits for it)."""
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            _check(lib().dm_match_batch(self.n, self.pairs, ctypes.byref(self.prm), self.flags,
                                        c_void_p(self.ws.data_ptr()), self.ws.numel(), c_void_p(self.out.data_ptr()),
                                        self.offsets, c_void_p(self.n_out.data_ptr()),
                                        c_void_p(self.stream.cuda_stream)))
        cur.wait_stream(self.stream)

    def matches(self) -> list:
        """Matches of the last run, one (n, 5) tensor per pair."""
        cnt = self.n_out.cpu().tolist()
        return [_matches_tensor(self.out[self.offsets[k]:], cnt[k]) for k in range(self.n)]

    def tiles(self) -> BatchTiles:
        t = BatchTiles()
        _check(lib().dm_batch_tiles_get(c_void_p(self.ws.data_ptr()), ctypes.byref(t)))
        return t

    def release(self):
        lib().dm_batch_release(c_void_p(self.ws.data_ptr()))

    def __del__(self):
        try:
            if _lib is not None and hasattr(self, "ws"):
                _lib.dm_batch_release(c_void_p(self.ws.data_ptr()))
        except Exception:
            pass


def top_loss(top: torch.Tensor) -> torch.Tensor:
    """Sum over top-level patches of the maximum of their map (the gradient
    goes to the first maximum in raster order)."""
    return top.reshape(top.shape[0] * top.shape[1], -1).max(1).values.sum()


def timing_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events on its stream."""
    _check(lib().dm_timing_enable(1 if on else 0))


def timing_read() -> list:
    """[(name, level, count, total_ms)] aggregated since timing_enable()."""
    n = c_int(0)
    _check(lib().dm_timing_read(None, 0, ctypes.byref(n)))
    arr = (StageTime * max(1, n.value))()
    _check(lib().dm_timing_read(arr, n.value, ctypes.byref(n)))
    return [(a.name.decode(), a.level, a.count, a.total_ms) for a in arr[:n.value]]


def version() -> str:
    return lib().dm_version().decode()
