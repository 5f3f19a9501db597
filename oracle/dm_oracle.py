"""FP64 CPU oracle of DeepMatching's hot path.

TEST INFRASTRUCTURE ONLY.  This module is the checker the GPU library is held
against.  Only the test suite, the smoke entry point and the CPU-baseline leg
of the benchmark may import it; the product path never does, and it shares no
code, table or helper with the GPU library.

It follows Revaud, Weinzaepfel, Harchaoui and Schmid, "DeepMatching:
Hierarchical Deformable Dense Matching" (IJCV 2016), in float64 NumPy:

* pixel descriptor ............ Sec. 3.2, paragraph "Pixel descriptor"
* bottom correlation .......... Sec. 3.2, Eqs. (3)-(4), Algorithm 1 (first loop)
* max-pool + subsample ........ Sec. 3.2, Eqs. (8)-(9)
* patch grids ................. Sec. 3.2, Eq. (7) and "Boundary effects"
* shift + average + rectify ... Sec. 3.2, Eqs. (5), (10)-(12), Algorithm 1
* backtracking + merge ........ Sec. 3.3, Eqs. (13)-(15)
* reciprocal verification ..... Sec. 3.3, Eq. (16)
* gradient of the top-level loss (no counterpart in the paper): the adjoint
  of each forward step above, written out by hand.

Where the GPU path uses a dense gather formulation of the backtracking, this
oracle keeps the paper's literal sets of tuples (N, p, p', s) and merges equal
(N, p, p') by keeping the highest score.

Readings taken where the paper is silent, ambiguous or inconsistent (the GPU
library takes the same ones):

 R1  A parent exists when its centre lies inside the image and at least one of
     its four children exists; the average runs over the existing children
     ("Boundary effects" example), not over all four as Eq. (7) literally says.
 R2  The neighbourhood Theta_i has radius N/8, i.e. the 3x3 window of Eq. (9)
     in subsampled units.
 R3  The shifted child map is read at q + o_i (the sign that makes an image
     match itself at the identity position, and the one the backtracking of
     Eq. (13) uses).
 R4  The bottom level is rectified too (Algorithm 1).
 R5  Target borders: the bottom correlation treats I' as zero outside; pooling
     ignores positions outside the map; an aggregated child read outside the
     map counts as 0 but the child still counts in the average; backtracking
     does not expand a child whose position falls outside the map.  Map sizes
     halve with rounding up.
 R6  Atomic centres are 2+4a with the whole 4x4 patch inside I (floor(W/4)
     columns); trailing pixels are never a source.
 R7  The pyramid top is Algorithm 1's loop bound (N < max(W, H)) or an
     explicit N_max, capped at the last level whose grid is non-empty.
 R8  A patch of even size N centred at p covers [p - N/2, p + N/2 - 1].
 R9  Argmax ties: first maximum in the order k = 3(m_y + 1) + (m_x + 1).
 R10 Descriptor: intensities scaled by 255; Gaussian "radius" nu = standard
     deviation, truncated at ceil(3 nu), replicated borders; central
     differences with replicated borders; orientations k*pi/4 with y down.
 R11 Match score: the top-level value plus the pooled child values along the
     backtracking path (Eq. (14)).
 R12 Reciprocal vicinities are the fixed 4x4 cells floor(p/4) and
     floor(p'/4); BestAt ties go to the smallest (p'_y, p'_x), BestAt' ties to
     the smallest (p_y, p_x, p'_y, p'_x).
 R13 Loss for the gradient: the sum over top-level patches of the maximum of
     their rectified map (ties: first in raster order).

 R14 Near-ties: decisions whose FP64 gap is below 2e-5 (1 + score) may go
     either way in FP32 (the GPU tests leave them out of exact comparisons).
 R15 lambda is a float32 parameter of the library.
 R16 Approximate DeepMatching (Sec. 4.1): k-means runs over the vectors of
     the atomic patches of I (the 16 pixel descriptors of the 4x4 patch in
     (dy, dx, channel) order, 144 values, norm 4 since every pixel descriptor
     has norm 1).  Keeping the centroids on the inputs' hypersphere means
     rescaling each one to norm 4 after every update.  D ranges over
     1 .. |G_4|; D = 0 is the exact method.
 R17 The paper does not say how k-means starts: centroid d starts as atomic
     patch floor((2d + 1) n / (2D)) of the n patches in raster order (evenly
     spread over the image, no random draw; D = n starts from every patch).
 R18 A fixed number of iterations (default 10), each an assignment then an
     update; a final assignment follows the last update.  Assignment: the
     nearest centroid on the sphere, i.e. the largest dot product; dot
     products within 1e-11 of the largest count as equal and the lowest
     index wins.  Update: the sum of the assigned vectors rescaled to norm 4;
     a centroid with no vector keeps its value.
 R19 Each atomic patch takes its prototype's bottom map C'_0; every level
     above is computed per patch as in the exact method (parents whose
     children have the same prototypes get equal maps; sharing them would
     save work but changes no value).
 R20 Scale and rotation invariant DM (Sec. 4.2, Algorithm 2): sigma takes
     half steps k/2, k in -4..4, and theta eighth turns r pi/4, r in 0..7 (the
     paper's grid).  The factors 2^(|k|/2) and the cosines and sines are
     exact table values (powers of two times sqrt(2), and 0, +-1,
     +-sqrt(1/2)), so every geometric quantity below is reproducible.
 R21 "I downsized by s" and "R_-theta * I' downsized by s" are one bilinear
     resampling each: output pixel (u, v) of the rotated canvas maps to
     q = R_theta((u, v) - c_out) + c_in in the downsized image, and q to
     s (q + 0.5) - 0.5 in the original (pixel centres aligned); neighbours
     outside the original count as 0.  The downsized image is
     floor(W/s) x floor(H/s) with centre c_in = ((W_s - 1)/2, (H_s - 1)/2);
     the rotated canvas is the bounding box ceil(W_s |cos| + H_s |sin|) x
     ceil(W_s |sin| + H_s |cos|) with centre c_out likewise; R_theta is
     [[cos, -sin], [sin, cos]] on (x, y) with y down.  No smoothing before
     the resampling.
 R22 Rectification: a run's tuple (p, p', s) maps to
     P = s1 (p + 0.5) - 0.5 and T = s2 (R_theta(p' - c_out) + c_in + 0.5) - 0.5,
     evaluated in FP64 in that order and rounded to the nearest pixel
     (floor(x + 0.5)); tuples whose T falls outside I' are dropped.  A run
     whose downsized I holds no atomic patch contributes nothing.
 R23 The union M' keeps the highest score of equal (P, T).  Reciprocal
     verification uses the fixed 4x4 cells of P in I and of T in I':
     BestAt(cell of P) is the best score, ties to the smallest (T_y, T_x), then
     the smallest (P_y, P_x); BestAt'(cell of T) as in R12.  The matches come
     out ordered by the source cell (row-major), at most one per cell.
 R24 DM* entry points (Sec. 3.3 names them only as local maxima over the
     correlation maps of every level; Table 1's middle configuration pairs
     them with the current path-sum scoring): the maps are those the method
     keeps, C_top and the pooled C'_l below it (a pooled cell stands for the
     position it was pooled from); a local maximum is positive, not below any
     of its 3 x 3 neighbours inside the map and above those before it in
     raster order (one maximum per plateau, since pooling repeats values in
     adjacent cells); an entry starts with its map value, tuples from above
     and entries merge by max at equal (N, p, p').
 R26 DM*'s start/end-point scoring (Sec. 5, the comparison with the earlier
     version, says only that an atomic correspondence was scored from the
     correlation values at the start and the end of its backtracking path):
     the score is the path sum of Eq. (14) restricted to the path's first
     and last nodes, i.e. the entry's value plus the atomic value C'_0 the
     path ends on (a path of one node, an entry at the bottom level, counts
     its value once); equal (N, p, p') still merge by max, which is exact
     because the end value depends on the atomic node alone.

Parity of the descriptor against the paper itself is unpinned (R10 fills in
details the paper does not give); it is pinned only by its invariants.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Child offsets o_i as (x, y), Eq. (5).
OFFSETS = ((-1, -1), (-1, +1), (+1, -1), (+1, +1))


@dataclass
class Params:
    """Method parameters (Sec. 5.2.1: nu1=0, mu=0.1 for uncompressed images;
    nu2=nu3=1, slope 0.2, lambda=1.4)."""
    nu1: float = 0.0
    nu2: float = 1.0
    nu3: float = 1.0
    slope: float = 0.2
    mu: float = 0.1
    scale: float = 255.0
    lam: float = 1.4
    max_patch: int = 0
    # Approximate DeepMatching (Sec. 4.1): D prototypes (0 = the exact
    # method) and the spherical k-means iterations (R16-R19).
    prototypes: int = 0
    kmeans_iters: int = 10
    # Entry points of the backtracking (Sec. 3.3, "Merging correspondences"):
    # 0 = every position of the top level; 1 = the earlier scheme (DM*,
    # compared in Table 1), local maxima of the maps of every level (R24).
    entry_points: int = 0
    # Scores of the atomic correspondences: 0 = the sum over the whole
    # backtracking path (Eq. (14)); 1 = the earlier scheme of Table 1, the
    # values at the path's start and end only (R26).
    scoring: int = 0


# ----------------------------------------------------------------------------
# Pixel descriptor (Sec. 3.2, "Pixel descriptor")
# ----------------------------------------------------------------------------

def gaussian_taps(sigma: float) -> np.ndarray:
    r = int(math.ceil(3.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-t * t / (2.0 * sigma * sigma))
    return g / g.sum()


def _smooth_axis(a: np.ndarray, g: np.ndarray, axis: int) -> np.ndarray:
    r = len(g) // 2
    n = a.shape[axis]
    out = np.zeros_like(a)
    for t in range(-r, r + 1):
        idx = np.clip(np.arange(n) + t, 0, n - 1)
        out += g[t + r] * np.take(a, idx, axis=axis)
    return out


def smooth(a: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian smoothing of an H x W (x C) array, replicated borders (R10)."""
    if sigma <= 0:
        return a
    g = gaussian_taps(sigma)
    return _smooth_axis(_smooth_axis(a, g, 1), g, 0)


def descriptors(img: np.ndarray, prm: Params = Params()) -> np.ndarray:
    """Per-pixel descriptor R_ij in R^9 (H x W x 9), unit l2 norm.

    Smooth (nu1), gradient, non-negative projections on the 8 orientations
    (cos k pi/4, sin k pi/4), smooth (nu2), sigmoid cap 2/(1+exp(-slope x))-1,
    smooth (nu3), append mu, l2-normalise."""
    J = prm.scale * np.asarray(img, dtype=np.float64)
    J = smooth(J, prm.nu1)
    H, W = J.shape
    xp = np.minimum(np.arange(W) + 1, W - 1)
    xm = np.maximum(np.arange(W) - 1, 0)
    yp = np.minimum(np.arange(H) + 1, H - 1)
    ym = np.maximum(np.arange(H) - 1, 0)
    gx = (J[:, xp] - J[:, xm]) / 2.0
    gy = (J[yp, :] - J[ym, :]) / 2.0
    O = np.stack([np.maximum(0.0, gx * math.cos(k * math.pi / 4) + gy * math.sin(k * math.pi / 4))
                  for k in range(1, 9)], axis=-1)
    O = smooth(O, prm.nu2)
    O = 2.0 / (1.0 + np.exp(-prm.slope * O)) - 1.0
    O = smooth(O, prm.nu3)
    d = np.concatenate([O, np.full((H, W, 1), prm.mu)], axis=-1)
    return d / np.sqrt((d * d).sum(-1, keepdims=True))


# ----------------------------------------------------------------------------
# Geometry: patch grids and map sizes (Sec. 3.2, Eq. (7), "Boundary effects")
# ----------------------------------------------------------------------------

def lattice_shape(level: int, W: int, H: int):
    """(ny, nx) of the lattice of candidate centres at a level.

    Level 0: atomic centres (2+4a, 2+4b) with the patch inside (R6).
    Level >= 1: centres (4a, 4b) inside the image."""
    if level == 0:
        return H // 4, W // 4
    return (H - 1) // 4 + 1, (W - 1) // 4 + 1


def lattice_centres(level: int, W: int, H: int):
    ny, nx = lattice_shape(level, W, H)
    base = 2 if level == 0 else 0
    return base + 4 * np.arange(ny), base + 4 * np.arange(nx)


def lattice_index(level: int, W: int, H: int, cy, cx):
    """Lattice indices (b, a) of centres at a level, and whether they exist."""
    ny, nx = lattice_shape(level, W, H)
    base = 2 if level == 0 else 0
    cy = np.asarray(cy)
    cx = np.asarray(cx)
    ok = ((cy - base) % 4 == 0) & ((cx - base) % 4 == 0)
    b = (cy - base) // 4
    a = (cx - base) // 4
    ok &= (b >= 0) & (b < ny) & (a >= 0) & (a < nx)
    return np.where(ok, b, 0), np.where(ok, a, 0), ok


def grids(W: int, H: int, lmax: int):
    """Boolean masks G_l over each level's lattice, for l = 0..lmax (R1)."""
    ny, nx = lattice_shape(0, W, H)
    G = [np.ones((ny, nx), dtype=bool)]
    for lv in range(1, lmax + 1):
        cy, cx = lattice_centres(lv, W, H)
        CY, CX = np.meshgrid(cy, cx, indexing="ij")
        g = np.zeros(CY.shape, dtype=bool)
        for ox, oy in OFFSETS:
            b, a, ok = lattice_index(lv - 1, W, H, CY + (2 ** lv) * oy, CX + (2 ** lv) * ox)
            g |= ok & G[lv - 1][b, a]
        G.append(g)
    return G


def pyramid_top(W: int, H: int, max_patch: int = 0) -> int:
    """Top level index lmax (N_max = 4 * 2^lmax), R7."""
    if max_patch:
        if max_patch < 4 or (max_patch & (max_patch - 1)):
            raise ValueError("max_patch must be a power of two >= 4")
        N = max_patch
    else:
        N = 4
        while N < max(W, H):          # Algorithm 1's loop bound
            N *= 2
    lmax = int(round(math.log2(N // 4)))
    G = grids(W, H, lmax)
    while lmax > 0 and not G[lmax].any():
        lmax -= 1
    return lmax


def map_dims(H2: int, W2: int, lmax: int):
    """(h_l, w_l) for l = 0..lmax+1: h_0 = H', h_l = ceil(h_{l-1}/2)."""
    h, w = [H2], [W2]
    for _ in range(lmax + 1):
        h.append((h[-1] + 1) // 2)
        w.append((w[-1] + 1) // 2)
    return h, w


# ----------------------------------------------------------------------------
# Bottom level (Eqs. (3)-(4)) and pyramid (Eqs. (8)-(12), Algorithm 1)
# ----------------------------------------------------------------------------

def bottom_scores(D1: np.ndarray, D2: np.ndarray, rows=None) -> np.ndarray:
    """A_0(p, q) = 1/16 sum_{i,j} R_ij(p)^T R'_ij(q), Eq. (3), for atomic
    centres p (patch rows `rows` of G_4) and every pixel q of I' (R5: I' is
    zero outside).  Returns shape (n_rows, nx0, H', W')."""
    H, W, C = D1.shape
    H2, W2, _ = D2.shape
    ny, nx = lattice_shape(0, W, H)
    rows = np.arange(ny) if rows is None else np.asarray(rows)
    cy = 2 + 4 * rows
    cx = 2 + 4 * np.arange(nx)
    D2p = np.zeros((H2 + 3, W2 + 3, C))
    D2p[2:2 + H2, 2:2 + W2] = D2
    # Patch vectors and target im2col over the 16 offsets of the 4x4 patch
    # (offsets -2..+1 around the centre, R8), in the same (dy, dx, c) order.
    offs = [(dy, dx) for dy in (-2, -1, 0, 1) for dx in (-2, -1, 0, 1)]
    P = np.concatenate([D1[np.ix_(cy + dy, cx + dx)].reshape(-1, C) for dy, dx in offs], axis=1)
    S = np.concatenate([D2p[2 + dy:2 + dy + H2, 2 + dx:2 + dx + W2].reshape(-1, C)
                        for dy, dx in offs], axis=1)
    A = P @ S.T
    return (A / 16.0).reshape(len(rows), nx, H2, W2)


def rectify(A: np.ndarray, lam: float) -> np.ndarray:
    """R_lambda, Eq. (11), on max(A, 0)."""
    return np.maximum(A, 0.0) ** lam


def pool_subsample(C: np.ndarray):
    """(S o P)(C), Eqs. (8)-(9): C'(r) = max_{m in {-1,0,1}^2} C(2r + m) over
    positions inside the map.  Returns (C', code, gap): code = 3(m_y+1)+(m_x+1)
    of the first maximum (R9), gap = best minus second-best candidate."""
    h, w = C.shape[-2:]
    h2, w2 = (h + 1) // 2, (w + 1) // 2
    Cp = np.full(C.shape[:-2] + (h + 3, w + 3), -np.inf)
    Cp[..., 1:1 + h, 1:1 + w] = C
    best = np.full(C.shape[:-2] + (h2, w2), -np.inf)
    second = np.full_like(best, -np.inf)
    code = np.zeros(best.shape, dtype=np.int8)
    for my in (-1, 0, 1):
        for mx in (-1, 0, 1):
            k = 3 * (my + 1) + (mx + 1)
            v = Cp[..., 1 + my:1 + my + 2 * h2:2, 1 + mx:1 + mx + 2 * w2:2]
            upd = v > best                      # strict: the first maximum wins
            np.maximum(second, np.minimum(v, best), out=second)
            np.copyto(code, np.int8(k), where=upd)
            np.maximum(best, v, out=best)
    return best, code, best - second


def risky(gap: np.ndarray) -> np.ndarray:
    """Gap as a risk margin: an exact tie (gap 0) comes from the same value
    reaching several candidates (overlapping pooling windows, equal sums) and
    is resolved by the tie rule in any precision, so it carries no risk."""
    return np.where(gap == 0, np.inf, gap)


def shift_read(M: np.ndarray, ox: int, oy: int) -> np.ndarray:
    """T applied as in R3: S(q) = M(q + o), 0 outside the map (R5)."""
    h, w = M.shape[-2:]
    Mp = np.zeros(M.shape[:-2] + (h + 2, w + 2))
    Mp[..., 1:1 + h, 1:1 + w] = M
    return Mp[..., 1 + oy:1 + oy + h, 1 + ox:1 + ox + w]


@dataclass
class Pyramid:
    W: int
    H: int
    W2: int
    H2: int
    lmax: int
    lam: float
    G: list
    h: list
    w: list
    Cp: list = field(default_factory=list)      # pooled maps C'_l, l < lmax
    code: list = field(default_factory=list)    # argmax codes of C'_l
    gap: list = field(default_factory=list)     # top-2 gaps of the pooling
    top: np.ndarray = None                      # C_lmax (unpooled)
    A: list = field(default_factory=list)       # pre-rectification maps (keep_full)
    protos: np.ndarray = None                   # approximate DM: prototypes (D x 144)
    assign: np.ndarray = None                   # approximate DM: prototype of each atomic patch


def aggregate(prev_pooled: np.ndarray, lv: int, pyr: Pyramid) -> np.ndarray:
    """A_l(p, q) = 1/|V(p)| sum_{i in V(p)} C'_{l-1}(p + 2^l o_i, q + o_i),
    Eqs. (6), (10), (12) with R1, R3, R5.  Invalid parents get NaN maps."""
    W, H = pyr.W, pyr.H
    cy, cx = lattice_centres(lv, W, H)
    CY, CX = np.meshgrid(cy, cx, indexing="ij")
    h, w = pyr.h[lv], pyr.w[lv]
    acc = np.zeros(CY.shape + (h, w))
    cnt = np.zeros(CY.shape)
    for ox, oy in OFFSETS:
        b, a, ok = lattice_index(lv - 1, W, H, CY + (2 ** lv) * oy, CX + (2 ** lv) * ox)
        ok &= pyr.G[lv - 1][b, a]
        child = np.where(ok[..., None, None], prev_pooled[b, a], 0.0)
        acc += shift_read(child, ox, oy)
        cnt += ok
    A = acc / np.maximum(cnt, 1)[..., None, None]
    A[~pyr.G[lv]] = np.nan
    return A


# ----------------------------------------------------------------------------
# Approximate DeepMatching: spherical k-means prototypes (Sec. 4.1, R16-R19)
# ----------------------------------------------------------------------------

KMEANS_TIE = 1e-11      # R18: dot products this close to the largest count as equal
SPHERE_RADIUS = 4.0     # R16: norm of an atomic patch vector


def kmeans_init(n: int, D: int) -> np.ndarray:
    """Indices of the D starting centroids among n patches (R17)."""
    if not 1 <= D <= n:
        raise ValueError("the number of prototypes must be in [1, number of atomic patches]")
    return (2 * np.arange(D, dtype=np.int64) + 1) * n // (2 * D)


def nearest_prototype(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Index of the nearest centroid of each row of X on the sphere: the
    largest dot product, ties within KMEANS_TIE to the lowest index (R18)."""
    S = X @ C.T
    return np.argmax(S >= S.max(axis=1, keepdims=True) - KMEANS_TIE, axis=1)


def atomic_patch_vectors(D1: np.ndarray) -> np.ndarray:
    """The 144-vector of every atomic patch of G_4 in lattice order: its 16
    pixel descriptors in (dy, dx) raster order, channels innermost (R8, R16)."""
    H, W, C = D1.shape
    ny, nx = lattice_shape(0, W, H)
    cy, cx = 2 + 4 * np.arange(ny), 2 + 4 * np.arange(nx)
    offs = [(dy, dx) for dy in (-2, -1, 0, 1) for dx in (-2, -1, 0, 1)]
    return np.concatenate([D1[np.ix_(cy + dy, cx + dx)].reshape(-1, C) for dy, dx in offs], axis=1)


def spherical_kmeans(X: np.ndarray, D: int, iters: int, radius: float = SPHERE_RADIUS):
    """Spherical k-means (Sec. 4.1): the D prototypes, each of norm `radius`,
    and the prototype of every row of X (R16-R18)."""
    C = X[kmeans_init(len(X), D)].astype(np.float64)
    C *= radius / np.linalg.norm(C, axis=1, keepdims=True)
    for _ in range(iters):
        a = nearest_prototype(X, C)
        for d in range(D):
            s = X[a == d].sum(axis=0)
            ns = np.linalg.norm(s)
            if ns > 0:
                C[d] = s * (radius / ns)
    return C, nearest_prototype(X, C)


def kmeans_objective(X: np.ndarray, C: np.ndarray, a: np.ndarray) -> float:
    """Sum over the rows of X of the dot product with their centroid, the
    quantity spherical k-means increases at every step."""
    return float(np.einsum("pk,pk->", X, C[a]))


def prototype_scores(C: np.ndarray, D2: np.ndarray) -> np.ndarray:
    """A_0 for prototype vectors instead of atomic patches: Eq. (3) with the
    patch vector replaced by its prototype (same (dy, dx, channel) order).
    Returns shape (D, H', W')."""
    H2, W2, Cc = D2.shape
    D2p = np.zeros((H2 + 3, W2 + 3, Cc))
    D2p[2:2 + H2, 2:2 + W2] = D2
    offs = [(dy, dx) for dy in (-2, -1, 0, 1) for dx in (-2, -1, 0, 1)]
    S = np.concatenate([D2p[2 + dy:2 + dy + H2, 2 + dx:2 + dx + W2].reshape(-1, Cc) for dy, dx in offs], axis=1)
    return ((C @ S.T) / 16.0).reshape(len(C), H2, W2)


def pyramid(D1: np.ndarray, D2: np.ndarray, prm: Params = Params(), keep_full: bool = False,
            row_chunk: int = 8, keep_bottom: bool = True) -> Pyramid:
    """Multi-level correlation pyramid, Algorithm 1.  keep_full keeps the
    pre-rectification maps for the gradient; keep_bottom=False leaves out the
    bottom one (full resolution), which pyramid_backward then recomputes in
    chunks of patch rows."""
    H, W, _ = D1.shape
    H2, W2, _ = D2.shape
    lmax = pyramid_top(W, H, prm.max_patch)
    G = grids(W, H, lmax)
    h, w = map_dims(H2, W2, lmax)
    pyr = Pyramid(W, H, W2, H2, lmax, prm.lam, G, h, w)
    ny0, nx0 = lattice_shape(0, W, H)
    if prm.prototypes > 0:
        # Approximate DeepMatching: C_0 and (S o P)(C_0) of the D prototypes,
        # then every atomic patch takes its prototype's (R19).
        if keep_full:
            raise ValueError("the gradient is defined for the exact method only (no prototypes)")
        X = atomic_patch_vectors(D1)
        pyr.protos, pyr.assign = spherical_kmeans(X, prm.prototypes, prm.kmeans_iters)
        a2 = pyr.assign.reshape(ny0, nx0)
        chunks = range(0, prm.prototypes, 64)
        if lmax == 0:
            pyr.top = np.concatenate([rectify(prototype_scores(pyr.protos[d:d + 64], D2), prm.lam)
                                      for d in chunks])[a2]
            return pyr
        pooled = [pool_subsample(rectify(prototype_scores(pyr.protos[d:d + 64], D2), prm.lam)) for d in chunks]
        pyr.Cp.append(np.concatenate([q[0] for q in pooled])[a2])
        pyr.code.append(np.concatenate([q[1] for q in pooled])[a2])
        pyr.gap.append(np.concatenate([q[2] for q in pooled])[a2])
        return _upper_levels(pyr, prm, keep_full)
    # Level 0: C_4 = R_lambda(I_4^F * I'), then S o P unless it is the top.
    parts_cp, parts_code, parts_gap, parts_A, parts_top = [], [], [], [], []
    for r0 in range(0, ny0, row_chunk):
        A0 = bottom_scores(D1, D2, np.arange(r0, min(ny0, r0 + row_chunk)))
        C0 = rectify(A0, prm.lam)
        if keep_full and (keep_bottom or lmax == 0):
            parts_A.append(A0)
        if lmax == 0:
            parts_top.append(C0)
        else:
            cp, cd, gp = pool_subsample(C0)
            parts_cp.append(cp)
            parts_code.append(cd)
            parts_gap.append(gp)
    if keep_full:
        pyr.A.append(np.concatenate(parts_A) if parts_A else None)
    if lmax == 0:
        pyr.top = np.concatenate(parts_top)
        return pyr
    pyr.Cp.append(np.concatenate(parts_cp))
    pyr.code.append(np.concatenate(parts_code))
    pyr.gap.append(np.concatenate(parts_gap))
    return _upper_levels(pyr, prm, keep_full)


def _upper_levels(pyr: Pyramid, prm: Params, keep_full: bool) -> Pyramid:
    """Levels 1..lmax of Algorithm 1 from the pooled level 0 in `pyr`."""
    lmax = pyr.lmax
    for lv in range(1, lmax + 1):
        A = aggregate(pyr.Cp[lv - 1], lv, pyr)
        C = rectify(A, prm.lam)
        if keep_full:
            pyr.A.append(A)
        if lv == lmax:
            pyr.top = C
        else:
            cp, cd, gp = pool_subsample(C)
            pyr.Cp.append(cp)
            pyr.code.append(cd)
            pyr.gap.append(gp)
    return pyr


# ----------------------------------------------------------------------------
# Top-down backtracking with merging (Sec. 3.3, Eqs. (13)-(15))
# ----------------------------------------------------------------------------

def _dedup_max(key: np.ndarray, s: np.ndarray):
    """Indices of the highest-score tuple of each key, and the gap to the
    runner-up (inf for singletons)."""
    order = np.lexsort((-s, key))
    k = key[order]
    first = np.ones(len(k), dtype=bool)
    first[1:] = k[1:] != k[:-1]
    keep = order[first]
    starts = np.flatnonzero(first)
    gap = np.full(len(starts), np.inf)
    has2 = np.append(starts[1:], len(k)) - starts > 1
    gap[has2] = s[order[starts[has2]]] - s[order[starts[has2] + 1]]
    return keep, gap


def backtrack(pyr: Pyramid, entries=None, level_entries=None, start_end: bool = False):
    """M' = B o ... o B (M), Eq. (15), merging equal (N, p, p') by max.

    start_end: score by the values at the start and end of each path (R26):
    B carries the score unchanged above the bottom level and adds the atomic
    value C'_0 in its last step.

    Entry points are all top-level (p, p') (Sec. 3.3, "Merging
    correspondences"), or the tuples of `level_entries` (a dict level ->
    (b, a, qy, qx, s, margin) arrays, `dmstar_entries`): those of the top
    level start the expansion and those of each lower level join the tuples
    that reach it before equal (N, p, p') merge.  Returns a dict of arrays
    over the atomic tuples: b, a (atomic lattice indices of p), qy, qx (pixel
    p' in I'), s (score), margin (smallest decision gap along the tuple's
    path: pooling argmaxes, and the local-maximum test of its entry)."""
    W, H, lmax = pyr.W, pyr.H, pyr.lmax
    Gt = pyr.G[lmax]
    if level_entries is not None:
        b, a, qy, qx, s, margin = (np.asarray(e) for e in level_entries[lmax])
    elif entries is None:
        bb, aa = np.nonzero(Gt)
        ht, wt = pyr.h[lmax], pyr.w[lmax]
        qy, qx = np.meshgrid(np.arange(ht), np.arange(wt), indexing="ij")
        n = len(bb)
        b = np.repeat(bb, ht * wt)
        a = np.repeat(aa, ht * wt)
        qy = np.tile(qy.ravel(), n)
        qx = np.tile(qx.ravel(), n)
    else:
        b, a, qy, qx = (np.asarray(e) for e in entries)
    if level_entries is None:
        s = pyr.top[b, a, qy, qx].astype(np.float64)
        margin = np.full(len(s), np.inf)
    for lv in range(lmax, 0, -1):
        h, w = pyr.h[lv], pyr.w[lv]
        cy, cx = lattice_centres(lv, W, H)
        out = {k: [] for k in ("b", "a", "qy", "qx", "s", "m")}
        for ox, oy in OFFSETS:
            cb, ca, ok = lattice_index(lv - 1, W, H, cy[b] + (2 ** lv) * oy, cx[a] + (2 ** lv) * ox)
            ok &= pyr.G[lv - 1][cb, ca]
            ry, rx = qy + oy, qx + ox
            ok &= (ry >= 0) & (ry < h) & (rx >= 0) & (rx < w)
            cb, ca, ry, rx = cb[ok], ca[ok], ry[ok], rx[ok]
            k = pyr.code[lv - 1][cb, ca, ry, rx].astype(np.int64)
            out["b"].append(cb)
            out["a"].append(ca)
            out["qy"].append(2 * ry + (k // 3 - 1))        # p'_i = 2(p' + o_i) + m_i, Eq. (13)
            out["qx"].append(2 * rx + (k % 3 - 1))
            step = pyr.Cp[lv - 1][cb, ca, ry, rx]
            out["s"].append(s[ok] if start_end and lv > 1 else s[ok] + step)   # Eq. (14); R26
            out["m"].append(np.minimum(margin[ok], risky(pyr.gap[lv - 1][cb, ca, ry, rx])))
        if level_entries is not None:   # the entries of level lv - 1 join before the merge
            for k, e in zip(("b", "a", "qy", "qx", "s", "m"), level_entries[lv - 1]):
                out[k].append(np.asarray(e))
        b, a, qy, qx, s, margin = (np.concatenate(out[k]) for k in ("b", "a", "qy", "qx", "s", "m"))
        ny, nx = lattice_shape(lv - 1, W, H)
        key = ((b * nx + a) * pyr.h[lv - 1] + qy) * pyr.w[lv - 1] + qx
        keep, _ = _dedup_max(key, s)
        b, a, qy, qx, s, margin = b[keep], a[keep], qy[keep], qx[keep], s[keep], margin[keep]
    return dict(b=b, a=a, qy=qy, qx=qx, s=s, margin=margin)


# ----------------------------------------------------------------------------
# Entry points of the earlier DeepMatching (DM*, Sec. 3.3 and Table 1): local
# maxima of the correlation maps of every level, scored by path sums (R24) or by
# the values at the start and end of each path (R26)
# ----------------------------------------------------------------------------

def local_maxima(M: np.ndarray, ids: np.ndarray | None = None):
    """R24: the local maxima of maps M[..., h, w] over their 3 x 3
    neighbourhoods (positions outside the map take no part): a positive value
    not below any neighbour and above the neighbours that come before it in
    raster order, so a plateau of equal values gives one maximum, at its
    first position.

    Returns the mask and each decision's margin.  The decision is the
    conjunction of one comparison per neighbour (and of the value with 0);
    a comparison's margin is the distance of the two values, except that
    equal values count as safe (inf) when they have the same identity in
    `ids` (a copy of one value: any evaluation ties them alike) and as 0
    otherwise (without `ids` every tie counts as 0).  A maximum changes when
    any comparison does (the smallest margin); a non-maximum only when every
    failing comparison does (the largest margin among them)."""
    h, w = M.shape[-2:]
    P = np.full(M.shape[:-2] + (h + 2, w + 2), -np.inf)
    P[..., 1:1 + h, 1:1 + w] = M
    if ids is not None:
        Q = np.full(M.shape[:-2] + (h + 2, w + 2), -1, dtype=np.int64)
        Q[..., 1:1 + h, 1:1 + w] = ids
    mask = M > 0
    m_all = np.abs(M)                      # the comparison with 0
    m_fail = np.where(mask, 0.0, np.abs(M))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            v = P[..., 1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
            ok = (M > v) if (dy, dx) < (0, 0) else (M >= v)
            mask &= ok
            with np.errstate(invalid="ignore"):   # -inf against -inf: no comparison, set below
                d = np.abs(M - v)
            if ids is None:
                same = np.zeros(M.shape, dtype=bool)
            else:
                same = Q[..., 1 + dy:1 + dy + h, 1 + dx:1 + dx + w] == ids
            mj = np.where(d > 0, d, np.where(same, np.inf, 0.0))
            mj = np.where(np.isinf(v), np.inf, mj)   # outside the map: no comparison
            m_all = np.minimum(m_all, mj)
            m_fail = np.where(ok, m_fail, np.maximum(m_fail, mj))
    return mask, np.where(mask, m_all, m_fail)


def dmstar_entries(pyr: Pyramid, tie: float = 2e-5):
    """Entry tuples of every level (R24): the local maxima of the top maps
    C_top, and of the pooled maps C'_l below the top, where pooled cell r of
    patch p stands for the node (l, p, 2r + m_l(p, r)) (the position it was
    pooled from) with score C'_l(p, r).  An entry's margin is that of its
    local-maximum decision, with the value identities of `pooling_stability`
    at `tie` (R14) telling copies from values that merely tie.  Returns
    {level: (b, a, qy, qx, s, margin)}."""
    out = {}
    _, tvid, pids = pooling_stability(pyr, tie)
    for lv in range(pyr.lmax + 1):
        M = pyr.top if lv == pyr.lmax else pyr.Cp[lv]
        ids = tvid if lv == pyr.lmax else pids[lv]
        mask, margin = local_maxima(np.nan_to_num(M, nan=-np.inf), ids)
        mask &= pyr.G[lv][..., None, None]
        b, a, ry, rx = np.nonzero(mask)
        if lv == pyr.lmax:
            qy, qx = ry, rx
        else:
            k = pyr.code[lv][b, a, ry, rx].astype(np.int64)
            qy, qx = 2 * ry + (k // 3 - 1), 2 * rx + (k % 3 - 1)
        out[lv] = (b, a, qy, qx, M[b, a, ry, rx].astype(np.float64), margin[b, a, ry, rx])
    return out


# ----------------------------------------------------------------------------
# Reciprocal verification (Sec. 3.3, Eq. (16))
# ----------------------------------------------------------------------------

def reciprocal(M: dict, W: int, H: int, W2: int, H2: int):
    """M'' = {t in M' : BestAt(p) = t = BestAt'(p')} with R12.

    Returns an (n, 5) array [x1, y1, x2, y2, score] sorted by (y1, x1), and
    the per-match margin (smallest decision gap: path argmaxes, BestAt and
    BestAt')."""
    b, a, qy, qx, s = M["b"], M["a"], M["qy"], M["qx"], M["s"]
    nx = lattice_shape(0, W, H)[1]
    n = len(s)
    if n == 0:
        return np.zeros((0, 5)), np.zeros(0)
    pid = b * nx + a
    # BestAt(p): max score, ties -> smallest (p'_y, p'_x).
    o1 = np.lexsort((qy * W2 + qx, -s, pid))
    f1 = np.ones(n, dtype=bool)
    f1[1:] = pid[o1][1:] != pid[o1][:-1]
    best_p = o1[f1]
    gap_p = np.full(n, np.inf)
    st = np.flatnonzero(f1)
    two = np.append(st[1:], n) - st > 1
    gap_p[best_p[two]] = s[o1[st[two]]] - s[o1[st[two] + 1]]
    # BestAt'(cell of p'): max score, ties -> smallest (p_y, p_x, p'_y, p'_x).
    cw = (W2 + 3) // 4
    cell = (qy // 4) * cw + (qx // 4)
    o2 = np.lexsort(((pid * H2 + qy) * W2 + qx, -s, cell))
    f2 = np.ones(n, dtype=bool)
    f2[1:] = cell[o2][1:] != cell[o2][:-1]
    best_c = o2[f2]
    gap_c = np.full(n, np.inf)
    st = np.flatnonzero(f2)
    two = np.append(st[1:], n) - st > 1
    gap_c[best_c[two]] = s[o2[st[two]]] - s[o2[st[two] + 1]]
    is_p = np.zeros(n, dtype=bool)
    is_p[best_p] = True
    is_c = np.zeros(n, dtype=bool)
    is_c[best_c] = True
    sel = np.flatnonzero(is_p & is_c)
    sel = sel[np.lexsort((a[sel], b[sel]))]
    out = np.stack([2 + 4 * a[sel], 2 + 4 * b[sel], qx[sel], qy[sel], s[sel]], axis=1).astype(np.float64)
    margin = np.minimum(M["margin"][sel], risky(np.minimum(gap_p[sel], gap_c[sel])))
    return out, margin


def match_descriptors(D1: np.ndarray, D2: np.ndarray, prm: Params = Params()):
    """Descriptors -> pyramid -> backtracking -> reciprocal matches."""
    # DM* entries need the value identities of pooling_stability, which read
    # the maps before rectification above level 0
    pyr = pyramid(D1, D2, prm, keep_full=bool(prm.entry_points), keep_bottom=False)
    M = backtrack(pyr, level_entries=dmstar_entries(pyr) if prm.entry_points else None,
                  start_end=prm.scoring == 1)
    out, margin = reciprocal(M, pyr.W, pyr.H, pyr.W2, pyr.H2)
    return out, margin, pyr, M


def match(img1: np.ndarray, img2: np.ndarray, prm: Params = Params()):
    """Images -> quasi-dense reciprocal matches [x1, y1, x2, y2, score]."""
    return match_descriptors(descriptors(img1, prm), descriptors(img2, prm), prm)


# ----------------------------------------------------------------------------
# Scale and rotation invariant DeepMatching (Sec. 4.2, Algorithm 2, R20-R23)
# ----------------------------------------------------------------------------

SQRT_HALF = 0.7071067811865476          # the double nearest to sqrt(1/2)
ROTATIONS = [(1.0, 0.0), (SQRT_HALF, SQRT_HALF), (0.0, 1.0), (-SQRT_HALF, SQRT_HALF),
             (-1.0, 0.0), (-SQRT_HALF, -SQRT_HALF), (0.0, -1.0), (SQRT_HALF, -SQRT_HALF)]   # (cos, sin) of r pi/4


def scale_factor(k: int) -> float:
    """2^(|k|/2) from exact operations (R20)."""
    k = abs(int(k))
    f = float(2 ** (k // 2))
    return f * math.sqrt(2.0) if k % 2 else f


def scale_pair(k: int):
    """(s1, s2) of Algorithm 2 for sigma = k/2: max(1, 2^sigma), max(1, 2^-sigma)."""
    return (scale_factor(k), 1.0) if k > 0 else (1.0, scale_factor(k))


def resampled_geometry(W: int, H: int, s: float, r: int):
    """Sizes and centres of the image downsized by s and rotated by -r pi/4
    (R21): (W_s, H_s, W_r, H_r, c_in, c_out)."""
    Ws, Hs = int(math.floor(W / s)), int(math.floor(H / s))
    c, sn = ROTATIONS[r]
    Wr = int(math.ceil(Ws * abs(c) + Hs * abs(sn)))
    Hr = int(math.ceil(Ws * abs(sn) + Hs * abs(c)))
    return Ws, Hs, Wr, Hr, ((Ws - 1) / 2.0, (Hs - 1) / 2.0), ((Wr - 1) / 2.0, (Hr - 1) / 2.0)


def canvas_to_source(u, v, s: float, r: int, cin, cout):
    """The composed map of R21 / R22: canvas pixel -> position in the
    original image, evaluated in this order."""
    c, sn = ROTATIONS[r]
    du, dv = u - cout[0], v - cout[1]
    qx = (c * du - sn * dv) + cin[0]
    qy = (sn * du + c * dv) + cin[1]
    return s * (qx + 0.5) - 0.5, s * (qy + 0.5) - 0.5


def resample(img: np.ndarray, s: float, r: int) -> np.ndarray:
    """img downsized by s and rotated by -r pi/4: one bilinear resampling,
    zero outside (R21)."""
    H, W = img.shape
    Ws, Hs, Wr, Hr, cin, cout = resampled_geometry(W, H, s, r)
    v, u = np.meshgrid(np.arange(Hr, dtype=np.float64), np.arange(Wr, dtype=np.float64), indexing="ij")
    x, y = canvas_to_source(u, v, s, r, cin, cout)
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = x - x0, y - y0
    x0, y0 = x0.astype(np.int64), y0.astype(np.int64)
    pad = np.zeros((H + 2, W + 2))
    pad[1:H + 1, 1:W + 1] = img
    out = np.zeros((Hr, Wr))
    for dy, wy in ((0, 1 - fy), (1, fy)):
        for dx, wx in ((0, 1 - fx), (1, fx)):
            yy, xx = y0 + dy, x0 + dx
            inside = (yy >= -1) & (yy <= H) & (xx >= -1) & (xx <= W)
            val = np.where(inside, pad[np.clip(yy + 1, 0, H + 1), np.clip(xx + 1, 0, W + 1)], 0.0)
            out += wy * wx * val
    return out


def round_half_up(x):
    return np.floor(np.asarray(x, dtype=np.float64) + 0.5).astype(np.int64)


def invariant_match(img1: np.ndarray, img2: np.ndarray, prm: Params = Params(), scales=range(-4, 5),
                    rotations=range(8)):
    """Algorithm 2: DM on every (sigma = k/2, theta = r pi/4) version of the
    pair, raw atomic correspondences rectified to the input images, their
    union, then one reciprocal verification (R20-R23).  Returns an (n, 5)
    array [x1, y1, x2, y2, score] ordered by source cell, and per-match
    margins (smallest decision gap, as in `reciprocal`)."""
    H1, W1 = img1.shape
    H2, W2 = img2.shape
    Px, Py, Tx, Ty, S, Mg = [], [], [], [], [], []
    for k in scales:
        s1, s2 = scale_pair(k)
        Ws1, Hs1, _, _, _, _ = resampled_geometry(W1, H1, s1, 0)
        if Ws1 < 4 or Hs1 < 4:
            continue                                      # no atomic patch (R22)
        D1 = descriptors(resample(img1, s1, 0), prm)
        for r in rotations:
            if min(resampled_geometry(W2, H2, s2, r)[2:4]) < 1:
                continue                                  # an empty image: nothing to add
            I2 = resample(img2, s2, r)
            M = backtrack(pyramid(D1, descriptors(I2, prm), prm))
            _, _, _, _, cin, cout = resampled_geometry(W2, H2, s2, r)
            px = round_half_up(s1 * ((2.0 + 4.0 * M["a"]) + 0.5) - 0.5)
            py = round_half_up(s1 * ((2.0 + 4.0 * M["b"]) + 0.5) - 0.5)
            tx, ty = canvas_to_source(M["qx"].astype(np.float64), M["qy"].astype(np.float64), s2, r, cin, cout)
            tx, ty = round_half_up(tx), round_half_up(ty)
            ok = (tx >= 0) & (tx < W2) & (ty >= 0) & (ty < H2)
            for L, v in ((Px, px), (Py, py), (Tx, tx), (Ty, ty), (S, M["s"]), (Mg, M["margin"])):
                L.append(v[ok])
    if not S or sum(len(v) for v in S) == 0:
        return np.zeros((0, 5)), np.zeros(0)
    px, py, tx, ty, s, mg = (np.concatenate(L) for L in (Px, Py, Tx, Ty, S, Mg))
    # Union: equal (P, T) keep the highest score (R23).
    pid, tid = py * W1 + px, ty * W2 + tx
    keep, gap = _dedup_max(pid * (W2 * H2) + tid, s)
    px, py, tx, ty, s, pid, tid = px[keep], py[keep], tx[keep], ty[keep], s[keep], pid[keep], tid[keep]
    mg = np.minimum(mg[keep], risky(gap))
    n = len(s)
    # BestAt per source cell: best score, ties -> smallest T, then smallest P.
    cw1, cw2 = (W1 + 3) // 4, (W2 + 3) // 4
    scell = (py // 4) * cw1 + px // 4
    o1 = np.lexsort((pid, tid, -s, scell))
    f1 = np.ones(n, dtype=bool)
    f1[1:] = scell[o1][1:] != scell[o1][:-1]
    best_p = o1[f1]
    gap_p = np.full(n, np.inf)
    st = np.flatnonzero(f1)
    two = np.append(st[1:], n) - st > 1
    gap_p[best_p[two]] = s[o1[st[two]]] - s[o1[st[two] + 1]]
    # BestAt' per target cell (R12): ties -> smallest (P_y, P_x, T_y, T_x).
    tcell = (ty // 4) * cw2 + tx // 4
    o2 = np.lexsort((tid, pid, -s, tcell))
    f2 = np.ones(n, dtype=bool)
    f2[1:] = tcell[o2][1:] != tcell[o2][:-1]
    best_c = o2[f2]
    gap_c = np.full(n, np.inf)
    st = np.flatnonzero(f2)
    two = np.append(st[1:], n) - st > 1
    gap_c[best_c[two]] = s[o2[st[two]]] - s[o2[st[two] + 1]]
    is_p = np.zeros(n, dtype=bool)
    is_p[best_p] = True
    is_c = np.zeros(n, dtype=bool)
    is_c[best_c] = True
    sel = np.flatnonzero(is_p & is_c)
    sel = sel[np.argsort(scell[sel], kind="stable")]
    out = np.stack([px[sel], py[sel], tx[sel], ty[sel], s[sel]], axis=1).astype(np.float64)
    return out, np.minimum(mg[sel], risky(np.minimum(gap_p[sel], gap_c[sel])))


# ----------------------------------------------------------------------------
# Gradient of L = sum_{p in G_top} max_q C_top(p, q) w.r.t. both descriptors
# ----------------------------------------------------------------------------

def top_loss(pyr: Pyramid) -> float:
    """R13: sum over existing top patches of the map maximum."""
    t = pyr.top[pyr.G[pyr.lmax]]
    return float(t.reshape(len(t), -1).max(1).sum())


def pyramid_backward(D1: np.ndarray, D2: np.ndarray, pyr: Pyramid, tie: float | None = None):
    """dL/dD1, dL/dD2 for the loss of `top_loss`, by hand-written adjoints of
    rectification, shift-average, max-pool/subsample (routed to the stored
    argmax) and the bottom correlation.  `pyr` must come from
    pyramid(..., keep_full=True).

    With `tie` set, also returns R1, R2 shaped like D1 and D2 and the list of
    risky decisions.  A decision (a pooling argmax that carries gradient, or
    the top map's maximum) is risky when `pooling_stability` finds that a
    less precise evaluation may take it the other way (R14); its gradient may
    then land on any candidate within tie * (1 + value) of the winner.  R is
    the magnitude of all such gradient, carried down the same adjoints as the
    gradient itself (absolute values, every candidate of a risky decision
    receiving the whole magnitude that reaches it), so it bounds how far each
    coordinate's gradient moves when any set of risky decisions goes another
    way.  Decisions are listed as (level, b, a, y, x): the pooled cell (y, x)
    of patch (b, a) at a level below the top, or the top map's first maximum
    (y, x) at level lmax."""
    if pyr.assign is not None:
        raise ValueError("the gradient is defined for the exact method only (no prototypes)")
    W, H, lmax, lam = pyr.W, pyr.H, pyr.lmax, pyr.lam
    top = pyr.top
    G = pyr.G[lmax]
    flat = np.where(G[..., None], top.reshape(top.shape[0], top.shape[1], -1), -np.inf)
    am = flat.argmax(-1)                                  # first maximum in raster order
    dC = np.zeros_like(top)
    bb, aa = np.nonzero(G)
    dC.reshape(top.shape[0], top.shape[1], -1)[bb, aa, am[bb, aa]] = 1.0
    risk = None
    if tie is not None:
        unstable, tvid, _ = pooling_stability(pyr, tie)
        mx = flat.max(-1, keepdims=True)
        near = (flat >= mx - tie * (1.0 + np.abs(mx))) & (mx > 0)
        if lmax == 0:   # the top is the bottom: distinct correlations
            at_risk = near.sum(-1) >= 2
        else:
            tv = tvid.reshape(flat.shape)
            winner = np.take_along_axis(tv, am[..., None], axis=-1)
            at_risk = (near & ((flat < mx) | (tv != winner))).any(-1)
        risk = (near & at_risk[..., None]).reshape(top.shape).astype(np.float64)
        w_top = top.shape[-1]
        decisions = [(lmax, int(b), int(a), int(am[b, a] // w_top), int(am[b, a] % w_top))
                     for b, a in zip(*np.nonzero(at_risk & G))]
    for lv in range(lmax, 0, -1):
        A = pyr.A[lv]
        fac = np.where(A > 0, lam * np.where(A > 0, A, 1.0) ** (lam - 1.0), 0.0)   # R_lambda'
        fac[~pyr.G[lv]] = 0.0
        dA = dC * fac
        # adjoint of the shifted average
        h, w = pyr.h[lv], pyr.w[lv]
        ny, nx = lattice_shape(lv - 1, W, H)
        dCp = np.zeros((ny, nx, h + 2, w + 2))
        cy, cx = lattice_centres(lv, W, H)
        CY, CX = np.meshgrid(cy, cx, indexing="ij")
        cnt = np.zeros(CY.shape)
        links = []
        for ox, oy in OFFSETS:
            cb, ca, ok = lattice_index(lv - 1, W, H, CY + (2 ** lv) * oy, CX + (2 ** lv) * ox)
            ok &= pyr.G[lv - 1][cb, ca] & pyr.G[lv]
            cnt += ok
            links.append((ox, oy, cb, ca, ok))
        if risk is not None:
            rA = risk * fac
            rCp = np.zeros((ny, nx, h + 2, w + 2))
        for ox, oy, cb, ca, ok in links:
            pb, pa = np.nonzero(ok)
            contrib = dA[pb, pa] / cnt[pb, pa][:, None, None]
            dCp[cb[pb, pa], ca[pb, pa], 1 + oy:1 + oy + h, 1 + ox:1 + ox + w] += contrib
            if risk is not None:
                rCp[cb[pb, pa], ca[pb, pa], 1 + oy:1 + oy + h, 1 + ox:1 + ox + w] += \
                    rA[pb, pa] / cnt[pb, pa][:, None, None]
        dCp = dCp[:, :, 1:1 + h, 1:1 + w]
        if risk is not None:
            rCp = rCp[:, :, 1:1 + h, 1:1 + w]
        if lv == 1:
            break   # dCp is the gradient of the pooled bottom maps C'_0
        dC = unpool_adjoint(dCp, pyr.code[lv - 1], pyr.h[lv - 1], pyr.w[lv - 1])
        if risk is not None:
            below = rectify(np.nan_to_num(pyr.A[lv - 1], nan=0.0), lam)
            risk, risky = unpool_risk(rCp, dCp, pyr.code[lv - 1], pyr.Cp[lv - 1], unstable[lv - 1], below, tie)
            decisions += [(lv - 1, *map(int, t)) for t in zip(*np.nonzero(risky))]
    # adjoint of the bottom correlation, Eq. (3), over chunks of patch rows
    # (the bottom maps are full resolution; a chunk at a time bounds memory)
    Hh, Ww, C = D1.shape
    H2, W2, _ = D2.shape
    ny0, nx0 = lattice_shape(0, W, H)
    cx = 2 + 4 * np.arange(nx0)
    D2p = np.zeros((H2 + 3, W2 + 3, C))
    D2p[2:2 + H2, 2:2 + W2] = D2
    dD1 = np.zeros_like(D1, dtype=np.float64)
    dD2p = np.zeros_like(D2p)
    if risk is not None:
        R1 = np.zeros(D1.shape)
        R2p = np.zeros(D2p.shape)
    chunk = ny0 if pyr.A[0] is not None else 4
    for r0 in range(0, ny0, chunk):
        rows = np.arange(r0, min(ny0, r0 + chunk))
        A0 = pyr.A[0][rows] if pyr.A[0] is not None else bottom_scores(D1, D2, rows)
        # gradient of C_0: the top's own (lmax = 0) or routed through the pool
        dC0 = dC[rows] if lmax == 0 else unpool_adjoint(dCp[rows], pyr.code[0][rows], H2, W2)
        fac0 = np.where(A0 > 0, lam * np.where(A0 > 0, A0, 1.0) ** (lam - 1.0), 0.0)
        g = (dC0 * fac0).reshape(len(rows) * nx0, H2 * W2) / 16.0
        cy = 2 + 4 * rows
        if risk is not None:
            if lmax == 0:
                r0map = risk[rows]
            else:
                r0map, risky = unpool_risk(rCp[rows], dCp[rows], pyr.code[0][rows], pyr.Cp[0][rows],
                                           unstable[0][rows], rectify(A0, lam), tie)
                decisions += [(0, int(b) + r0, *map(int, t)) for b, *t in zip(*np.nonzero(risky))]
            rg = (r0map * fac0).reshape(len(rows) * nx0, H2 * W2) / 16.0
        for dy in (-2, -1, 0, 1):
            for dx in (-2, -1, 0, 1):
                S = D2p[2 + dy:2 + dy + H2, 2 + dx:2 + dx + W2].reshape(-1, C)
                P = D1[np.ix_(cy + dy, cx + dx)].reshape(-1, C)
                dD1[np.ix_(cy + dy, cx + dx)] += (g @ S).reshape(len(rows), nx0, C)
                dD2p[2 + dy:2 + dy + H2, 2 + dx:2 + dx + W2] += (g.T @ P).reshape(H2, W2, C)
                if risk is not None:
                    R1[np.ix_(cy + dy, cx + dx)] += (rg @ np.abs(S)).reshape(len(rows), nx0, C)
                    R2p[2 + dy:2 + dy + H2, 2 + dx:2 + dx + W2] += (rg.T @ np.abs(P)).reshape(H2, W2, C)
    if risk is not None:
        return dD1, dD2p[2:2 + H2, 2:2 + W2], R1, R2p[2:2 + H2, 2:2 + W2], decisions
    return dD1, dD2p[2:2 + H2, 2:2 + W2]


def _mix64(h: np.ndarray, v: np.ndarray) -> np.ndarray:
    """One step of a 64-bit hash chain (the splitmix64 finaliser of h + v)."""
    with np.errstate(over="ignore"):
        z = h + v.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _value_ids(pyr: Pyramid, lv: int, pid_below: np.ndarray) -> np.ndarray:
    """Provenance of every value of C_lv (lv >= 1): a hash of the identities
    of the pooled child values it averages (Eq. (12)), -1 for a read outside
    the child's map, nothing for a missing child.  Equal ids mean the same
    child values added in the same order, hence bitwise equal results in any
    deterministic evaluation; ids are non-negative."""
    W, H = pyr.W, pyr.H
    h, w = pyr.h[lv], pyr.w[lv]
    cy, cx = lattice_centres(lv, W, H)
    CY, CX = np.meshgrid(cy, cx, indexing="ij")
    vid = np.zeros(CY.shape + (h, w), dtype=np.uint64)
    for ox, oy in OFFSETS:
        cb, ca, ok = lattice_index(lv - 1, W, H, CY + (2 ** lv) * oy, CX + (2 ** lv) * ox)
        ok &= pyr.G[lv - 1][cb, ca]
        pad = np.full(pid_below.shape[:-2] + (h + 2, w + 2), -1, dtype=np.int64)
        pad[..., 1:1 + h, 1:1 + w] = pid_below
        child = pad[cb, ca, 1 + oy:1 + oy + h, 1 + ox:1 + ox + w]
        vid = np.where(ok[..., None, None], _mix64(vid, child), vid)
    return (vid >> np.uint64(1)).astype(np.int64)


def pooling_stability(pyr: Pyramid, tie: float):
    """The decisions a less precise evaluation may take differently (R14).

    Returns (unstable, top_vid, pids): per level l < lmax, the pooled cells
    whose argmax (Eq. (9)) is at risk; the provenance ids of the top map; and
    per level l < lmax the identity of each pooled cell's value (equal ids:
    bitwise equal values in any evaluation that keeps the stable decisions).  A
    decision with a positive best value is at risk when a runner-up lies
    within tie * (1 + best) of it, unless the runner-up is an exact tie whose
    value has the same provenance as the winner's (`_value_ids`: the same
    stable child values, which every evaluation adds alike).  At level 0
    every exact tie counts, its candidates being distinct correlations.  A
    pooled cell passes on the provenance of its source position when its
    decision is stable, and an identity of its own otherwise."""
    out, pids = [], []
    pid = None
    for lv in range(pyr.lmax + 1):
        vid = None if lv == 0 else _value_ids(pyr, lv, pid)
        if lv == pyr.lmax:
            return out, vid, pids
        best, code = pyr.Cp[lv], pyr.code[lv]
        thr = tie * (1.0 + np.abs(best))
        h, w = best.shape[-2:]
        ry, rx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        sy, sx = 2 * ry + code // 3 - 1, 2 * rx + code % 3 - 1
        if lv == 0:
            unstable = (pyr.gap[lv] <= thr) & (best > 0)
            src = (sy * pyr.w[0] + sx).astype(np.int64)
        else:
            C = rectify(np.nan_to_num(pyr.A[lv], nan=0.0), pyr.lam)
            hp, wp = C.shape[-2:]
            Cpad = np.full(C.shape[:-2] + (hp + 3, wp + 3), -np.inf)
            Cpad[..., 1:1 + hp, 1:1 + wp] = C
            Vpad = np.full(C.shape[:-2] + (hp + 3, wp + 3), -1, dtype=np.int64)
            Vpad[..., 1:1 + hp, 1:1 + wp] = vid
            src = np.take_along_axis(vid.reshape(vid.shape[:-2] + (-1,)),
                                     (sy * wp + sx).reshape(code.shape[:-2] + (-1,)).astype(np.int64),
                                     axis=-1).reshape(code.shape)
            unstable = np.zeros(best.shape, dtype=bool)
            for my in (-1, 0, 1):
                for mx in (-1, 0, 1):
                    v = Cpad[..., 1 + my:1 + my + 2 * h:2, 1 + mx:1 + mx + 2 * w:2]
                    vv = Vpad[..., 1 + my:1 + my + 2 * h:2, 1 + mx:1 + mx + 2 * w:2]
                    unstable |= (v < best) & (v >= best - thr)
                    unstable |= (v == best) & (vv != src)
            unstable &= best > 0
        out.append(unstable)
        marker = -2 - np.arange(best.size, dtype=np.int64).reshape(best.shape)
        pid = np.where(unstable, marker, src)
        pids.append(pid)


def unpool_risk(rCp: np.ndarray, dCp: np.ndarray, code: np.ndarray, best: np.ndarray, unstable: np.ndarray,
                C: np.ndarray, tie: float):
    """The risk of `pyramid_backward` through S o P (Eqs. (8)-(9)): a stable
    cell routes its risk to its argmax position; an unstable cell
    (`pooling_stability`) that carries gradient or risk sends its whole
    magnitude |gradient| + risk to every position of its window within
    tie * (1 + best) of the best (C: the map below the pooling).  Returns the
    risk of that map and the mask of those unstable cells."""
    h, w = rCp.shape[-2:]
    hp, wp = C.shape[-2:]
    risky = ((rCp > 0) | (dCp != 0)) & unstable
    out = unpool_adjoint(np.where(risky, 0.0, rCp), code, hp, wp)
    mag = np.where(risky, np.abs(dCp) + rCp, 0.0)
    thr = best - tie * (1.0 + np.abs(best))
    Cpad = np.full(C.shape[:-2] + (hp + 3, wp + 3), -np.inf)
    Cpad[..., 1:1 + hp, 1:1 + wp] = C
    opad = np.zeros(Cpad.shape)
    for my in (-1, 0, 1):
        for mx in (-1, 0, 1):
            v = Cpad[..., 1 + my:1 + my + 2 * h:2, 1 + mx:1 + mx + 2 * w:2]
            opad[..., 1 + my:1 + my + 2 * h:2, 1 + mx:1 + mx + 2 * w:2] += np.where(v >= thr, mag, 0.0)
    return out + opad[..., 1:1 + hp, 1:1 + wp], risky


def unpool_adjoint(dCp: np.ndarray, code: np.ndarray, hp: int, wp: int) -> np.ndarray:
    """Adjoint of S o P (Eqs. (8)-(9)): each pooled gradient goes to the
    window position its stored argmax names, on the hp x wp map below."""
    h, w = dCp.shape[-2:]
    dC = np.zeros(dCp.shape[:-2] + (hp + 3, wp + 3))
    for my in (-1, 0, 1):
        for mx in (-1, 0, 1):
            k = 3 * (my + 1) + (mx + 1)
            sel = np.where(code == k, dCp, 0.0)
            dC[..., 1 + my:1 + my + 2 * h:2, 1 + mx:1 + mx + 2 * w:2] += sel
    return dC[..., 1:1 + hp, 1:1 + wp]
