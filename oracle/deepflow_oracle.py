"""FP64 CPU oracle of DeepFlow (Sec. 4.3): variational refinement of a flow
field with DeepMatching's matches as its matching term.

TEST INFRASTRUCTURE ONLY.  Like dm_oracle, this module is the checker the GPU
library is held against; only the tests, the smoke entry point and the
CPU-baseline leg of the benchmark may import it, and it shares no code with
the GPU library.

The energy (Sec. 4.3, Eq. (17)) is a data term (Eq. (18): colour and
gradient constancy, each normalised), a locally weighted smoothness term
(Eq. (19) with alpha(x)) and a matching term c phi Psi(|w - w'|^2), all
penalised by Psi(s^2) = sqrt(s^2 + eps^2).  It is minimised coarse to fine
with incremental warping (downsampling factor eta), a few fixed-point
iterations per level that freeze the penalisers' derivatives, and SOR on
the resulting linear system; the matching weight is beta^k = beta (k/k_max)^b
at level k.

Readings taken where the paper leaves the discretisation open (the GPU
library takes the same ones):

 D1  Images are grayscale (c = 1) with intensities in [0, 1], as given,
     smoothed by a Gaussian of standard deviation sigma truncated at
     ceil(3 sigma) with replicated borders.  The data and smoothness terms
     use that scale (the paper's kappa = 5 in alpha(x) and zeta = 0.1 only
     make sense on it: on 0..255 intensities alpha would vanish wherever
     there is texture); the matching weight phi reads lambda~ and Delta on
     0..255 intensities (its sigma_M = 50 and the factor 10 on lambda~ are on
     that scale: on [0, 1] intensities phi would be about 1e-3 and the
     matching term would vanish).
 D2  Level k has size round(W eta^k) x round(H eta^k); the coarsest level is
     the last whose smaller side is at least min_size (16).  Each level's
     images are a bilinear resampling (pixel centres aligned, coordinates
     clamped to the map) of the level below, the flow goes up a level by the
     same resampling, scaled by the ratio of the sizes; it starts at 0.
 D3  Spatial derivatives are central differences with replicated borders.
     The linearisation uses the average A = (I1 + I2(x + w)) / 2 of the
     first image and the warped second one for the spatial derivatives
     (A_x, A_y and, for gradient constancy, A_xx, A_xy, A_yy), I2w - I1 for
     the temporal one and the difference of the two images' spatial
     derivatives for I_xt, I_yt.  Warping is bilinear with coordinates
     clamped to the map.
 D4  Smoothness: alpha(x) = exp(-kappa |grad I1_k(x)|) at each level; the
     penaliser derivative psi'(|grad U|^2 + |grad V|^2) is taken per pixel
     (central differences); a 4-neighbour edge carries the mean of its two
     pixels' alpha psi'.
 D5  Psi'(s^2) = 1 / (2 sqrt(s^2 + eps^2)) for every term; the frozen-weight
     energy of a fixed-point iteration is the sum of the data quadratics, the
     edge terms g (|dU|^2 + |dV|^2) and w_M |w - w'|^2, and its minimiser
     solves a 2 x 2 system per pixel coupled through the edges.
 D6  SOR: red-black ordering (x + y even first), a 2 x 2 block update per
     pixel, relaxation omega = 1.6 (the paper gives the iteration count, not
     the factor).
 D7  Matching term: a match (x1, y1) -> (x2, y2) sets w'(x1, y1) =
     (x2 - x1, y2 - y1).  phi uses lambda~ = 10 x the smaller eigenvalue of
     the sum of grad I1 grad I1^T over the 3 x 3 window, and Delta =
     |I1(x) - I2(x + w')| + |grad I1(x) - grad I2(x + w')| (Euclidean norm of
     the gradient difference), read at the match's own target: the paper's
     x - w' is taken as the target x + w'.  The exponent is -Delta /
     (2 sigma_M).  At level k a match sits at the nearest level pixel of its
     source, its flow scaled by the level's size ratios; where several land
     on one pixel the first in the match list is kept (a rule that depends
     on the order only, not on the rounding of phi).
 D8  beta^k = beta (k / k_max)^b with k = 0 the finest level (no matching
     term there) and beta^0 = beta when there is a single level.

Every array is float64; images are (H, W) arrays indexed [y, x].
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class FlowParams:
    """Sec. 4.3 and the parameters of its experiments (eta, iterations, beta,
    gamma, delta, sigma, b); omega and min_size are readings D6 and D2."""
    sigma: float = 0.5
    eta: float = 0.95
    min_size: int = 16
    n_fixed: int = 5
    n_sor: int = 25
    omega: float = 1.6
    kappa: float = 5.0
    beta: float = 300.0
    b: float = 0.6
    gamma: float = 0.8
    delta: float = 0.0
    eps: float = 0.001
    zeta: float = 0.1
    sigma_m: float = 50.0
    lam_scale: float = 10.0


def psi(s2, eps):
    """Robust penaliser Psi(s^2) = sqrt(s^2 + eps^2) (Sec. 4.3)."""
    return np.sqrt(s2 + eps * eps)


def psi_prime(s2, eps):
    """dPsi / d(s^2) (D5)."""
    return 0.5 / np.sqrt(s2 + eps * eps)


# ---------------------------------------------------------------- image operations
def gauss_taps(sigma):
    r = int(math.ceil(3.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-x * x / (2.0 * sigma * sigma))
    return k / k.sum()


def smooth(img, sigma):
    """Separable Gaussian with replicated borders (D1)."""
    k = gauss_taps(sigma)
    r = len(k) // 2
    H, W = img.shape
    p = np.pad(img, ((0, 0), (r, r)), mode="edge")
    t = sum(k[i] * p[:, i:i + W] for i in range(len(k)))
    p = np.pad(t, ((r, r), (0, 0)), mode="edge")
    return sum(k[i] * p[i:i + H, :] for i in range(len(k)))


def bilinear(img, xs, ys):
    """img sampled at real coordinates (xs, ys), clamped to the map."""
    H, W = img.shape
    xs = np.clip(xs, 0.0, W - 1.0)
    ys = np.clip(ys, 0.0, H - 1.0)
    x0 = np.floor(xs).astype(np.int64)
    y0 = np.floor(ys).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    fx, fy = xs - x0, ys - y0
    top = img[y0, x0] * (1.0 - fx) + img[y0, x1] * fx
    bot = img[y1, x0] * (1.0 - fx) + img[y1, x1] * fx
    return top * (1.0 - fy) + bot * fy


def resize(img, W, H):
    """Bilinear resampling to W x H, pixel centres aligned (D2)."""
    h, w = img.shape
    xs = (np.arange(W, dtype=np.float64) + 0.5) * (w / W) - 0.5
    ys = (np.arange(H, dtype=np.float64) + 0.5) * (h / H) - 0.5
    X, Y = np.meshgrid(xs, ys)
    return bilinear(img, X, Y)


def grad(img):
    """Central differences with replicated borders (D3): (d/dx, d/dy)."""
    p = np.pad(img, 1, mode="edge")
    return 0.5 * (p[1:-1, 2:] - p[1:-1, :-2]), 0.5 * (p[2:, 1:-1] - p[:-2, 1:-1])


def warp(img, u, v):
    """img(x + u, y + v), bilinear (D3)."""
    H, W = img.shape
    X, Y = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    return bilinear(img, X + u, Y + v)


def level_sizes(W, H, p: FlowParams):
    """Sizes of levels 0 (finest) .. k_max (D2)."""
    sizes = [(W, H)]
    k = 1
    while True:
        w = int(math.floor(W * p.eta ** k + 0.5))
        h = int(math.floor(H * p.eta ** k + 0.5))
        if min(w, h) < p.min_size:
            break
        sizes.append((w, h))
        k += 1
    return sizes


# ---------------------------------------------------------------- matching term
def min_eig_autocorr(img):
    """lambda of D7 before scaling: the smaller eigenvalue of the 3 x 3 window
    sum of grad I grad I^T."""
    gx, gy = grad(img)
    def box(a):
        p = np.pad(a, 1, mode="edge")
        H, W = a.shape
        return sum(p[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3))
    a, b, c = box(gx * gx), box(gx * gy), box(gy * gy)
    return 0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2 + b * b)


def match_phi(I1, I2, matches, p: FlowParams):
    """phi of every match (D7) on the smoothed full-size images."""
    H, W = I1.shape
    if len(matches) == 0:
        return np.zeros(0)
    I1, I2 = 255.0 * I1, 255.0 * I2   # D1: phi on 0..255 intensities
    lam = p.lam_scale * np.maximum(min_eig_autocorr(I1), 0.0)
    g1x, g1y = grad(I1)
    g2x, g2y = grad(I2)
    x1 = np.clip(matches[:, 0].astype(np.int64), 0, W - 1)
    y1 = np.clip(matches[:, 1].astype(np.int64), 0, H - 1)
    x2 = np.clip(matches[:, 2].astype(np.int64), 0, W - 1)
    y2 = np.clip(matches[:, 3].astype(np.int64), 0, H - 1)
    delta = np.abs(I1[y1, x1] - I2[y2, x2]) + np.hypot(g1x[y1, x1] - g2x[y2, x2], g1y[y1, x1] - g2y[y2, x2])
    return np.sqrt(lam[y1, x1]) / (p.sigma_m * math.sqrt(2.0 * math.pi)) * np.exp(-delta / (2.0 * p.sigma_m))


def match_field(matches, phi, W, H, Wk, Hk):
    """w' and c phi at a level of size Wk x Hk (D7): arrays (Hk, Wk)."""
    up, vp, cphi = np.zeros((Hk, Wk)), np.zeros((Hk, Wk)), np.zeros((Hk, Wk))
    if len(matches) == 0:
        return up, vp, cphi
    sx, sy = Wk / W, Hk / H
    taken = np.zeros((Hk, Wk), dtype=bool)
    for i in range(len(matches)):
        x1, y1, x2, y2 = (float(v) for v in matches[i, :4])
        # nearest level pixel of the source centre (x1 + 0.5) sx - 0.5:
        # floor((2 x1 + 1) Wk / (2 W)), in integers (negative sources clamp to 0)
        xk = min(max((2 * int(x1) + 1) * Wk // (2 * W), 0), Wk - 1)
        yk = min(max((2 * int(y1) + 1) * Hk // (2 * H), 0), Hk - 1)
        if taken[yk, xk]:
            continue
        taken[yk, xk] = True
        up[yk, xk], vp[yk, xk], cphi[yk, xk] = (x2 - x1) * sx, (y2 - y1) * sy, phi[i]
    return up, vp, cphi


# ---------------------------------------------------------------- one level
def sym3(a, b, c):
    """Entries (11, 12, 13, 22, 23, 33) of the outer product [a, b, c]^T [a, b, c]."""
    return np.stack([a * a, a * b, a * c, b * b, b * c, c * c])


def level_tensors(I1, I2w, p: FlowParams):
    """Normalised data tensors J0 (colour) and Jxy (gradient) of Eq. (18)
    (D3): arrays (6, H, W) of their upper-triangle entries."""
    A = 0.5 * (I1 + I2w)
    Ax, Ay = grad(A)
    It = I2w - I1
    Axx, Axy = grad(Ax)
    _, Ayy = grad(Ay)
    g1x, g1y = grad(I1)
    g2x, g2y = grad(I2w)
    Ixt, Iyt = g2x - g1x, g2y - g1y
    z2 = p.zeta * p.zeta
    J0 = sym3(Ax, Ay, It) / (Ax * Ax + Ay * Ay + z2)
    Jxy = sym3(Axx, Axy, Ixt) / (Axx * Axx + Axy * Axy + z2) + sym3(Axy, Ayy, Iyt) / (Axy * Axy + Ayy * Ayy + z2)
    return J0, Jxy


def quad(J, du, dv):
    """(du, dv, 1) J (du, dv, 1)^T."""
    return (J[0] * du * du + 2 * J[1] * du * dv + 2 * J[2] * du + J[3] * dv * dv + 2 * J[4] * dv + J[5])


def frozen_weights(J0, Jxy, alpha, u, v, du, dv, up, vp, cphi, beta_k, p: FlowParams):
    """The penalisers' derivatives at the current increment (a fixed-point
    step, D4-D5): combined data tensor wJ (6, H, W), pixel smoothness weight
    a (H, W) and matching weight wM (H, W)."""
    wD0 = p.delta * psi_prime(quad(J0, du, dv), p.eps)
    wDxy = p.gamma * psi_prime(quad(Jxy, du, dv), p.eps)
    wJ = wD0 * J0 + wDxy * Jxy
    U, V = u + du, v + dv
    Ux, Uy = grad(U)
    Vx, Vy = grad(V)
    a = alpha * psi_prime(Ux * Ux + Uy * Uy + Vx * Vx + Vy * Vy, p.eps)
    wM = beta_k * cphi * psi_prime((U - up) ** 2 + (V - vp) ** 2, p.eps)
    return wJ, a, wM


def edge_weights(a):
    """Edge weights of D4: gh[y, x] between (x, x+1), gv[y, x] between (y, y+1)."""
    return 0.5 * (a[:, :-1] + a[:, 1:]), 0.5 * (a[:-1, :] + a[1:, :])


def sor(wJ, gh, gv, wM, u, v, du, dv, up, vp, n_iter, omega):
    """n_iter red-black block SOR sweeps (D6) on the linear system whose
    solution minimises the frozen-weight energy; returns (du, dv)."""
    H, W = u.shape
    du, dv = du.copy(), dv.copy()
    # neighbour weights of every pixel (0 past the border)
    gL = np.zeros((H, W)); gL[:, 1:] = gh
    gR = np.zeros((H, W)); gR[:, :-1] = gh
    gU = np.zeros((H, W)); gU[1:, :] = gv
    gD = np.zeros((H, W)); gD[:-1, :] = gv
    G = gL + gR + gU + gD
    a11 = wJ[0] + wM + G
    a12 = wJ[1]
    a22 = wJ[3] + wM + G
    b1 = -wJ[2] - wM * (u - up) - G * u
    b2 = -wJ[4] - wM * (v - vp) - G * v
    det = a11 * a22 - a12 * a12
    Y, X = np.mgrid[0:H, 0:W]
    colours = [((X + Y) & 1) == 0, ((X + Y) & 1) == 1]

    def nsum(g_l, g_r, g_u, g_d, f):
        s = np.zeros((H, W))
        s[:, 1:] += g_l[:, 1:] * f[:, :-1]
        s[:, :-1] += g_r[:, :-1] * f[:, 1:]
        s[1:, :] += g_u[1:, :] * f[:-1, :]
        s[:-1, :] += g_d[:-1, :] * f[1:, :]
        return s

    for _ in range(n_iter):
        for m in colours:
            su = nsum(gL, gR, gU, gD, u + du)
            sv = nsum(gL, gR, gU, gD, v + dv)
            r1, r2 = b1 + su, b2 + sv
            nu = (r1 * a22 - r2 * a12) / det
            nv = (a11 * r2 - a12 * r1) / det
            du = np.where(m, du + omega * (nu - du), du)
            dv = np.where(m, dv + omega * (nv - dv), dv)
    return du, dv


def frozen_energy(wJ, gh, gv, wM, u, v, du, dv, up, vp):
    """The quadratic energy a fixed-point step minimises (D5), written as
    its sum of terms (for the tests)."""
    U, V = u + du, v + dv
    e = quad(wJ, du, dv).sum()
    e += (gh * ((U[:, 1:] - U[:, :-1]) ** 2 + (V[:, 1:] - V[:, :-1]) ** 2)).sum()
    e += (gv * ((U[1:, :] - U[:-1, :]) ** 2 + (V[1:, :] - V[:-1, :]) ** 2)).sum()
    e += (wM * ((U - up) ** 2 + (V - vp) ** 2)).sum()
    return e


def solve_level(I1, I2, u, v, up, vp, cphi, beta_k, p: FlowParams, trace=None):
    """Fixed-point iterations with SOR at one level; returns the new (u, v).
    trace, when a list, receives the frozen energies before and after each
    SOR solve."""
    I2w = warp(I2, u, v)
    J0, Jxy = level_tensors(I1, I2w, p)
    gx, gy = grad(I1)
    alpha = np.exp(-p.kappa * np.hypot(gx, gy))
    du, dv = np.zeros_like(u), np.zeros_like(u)
    for _ in range(p.n_fixed):
        wJ, a, wM = frozen_weights(J0, Jxy, alpha, u, v, du, dv, up, vp, cphi, beta_k, p)
        gh, gv = edge_weights(a)
        e0 = frozen_energy(wJ, gh, gv, wM, u, v, du, dv, up, vp) if trace is not None else None
        du, dv = sor(wJ, gh, gv, wM, u, v, du, dv, up, vp, p.n_sor, p.omega)
        if trace is not None:
            trace.append((e0, frozen_energy(wJ, gh, gv, wM, u, v, du, dv, up, vp)))
    return u + du, v + dv


# ---------------------------------------------------------------- whole method
def prepare(img1, img2, p: FlowParams):
    """Smoothed images (D1)."""
    return smooth(np.asarray(img1, np.float64), p.sigma), smooth(np.asarray(img2, np.float64), p.sigma)


def deepflow(img1, img2, matches, p: FlowParams = FlowParams()):
    """Flow (H, W, 2) from img1 to img2 (float images in [0, 1], the same
    size) with matches (n, >= 4) rows (x1, y1, x2, y2, ...)."""
    img1 = np.asarray(img1, np.float64)
    img2 = np.asarray(img2, np.float64)
    assert img1.shape == img2.shape
    H, W = img1.shape
    I1, I2 = prepare(img1, img2, p)
    matches = np.asarray(matches, np.float64)
    if matches.size == 0:
        matches = np.zeros((0, 4))
    phi = match_phi(I1, I2, matches, p)
    sizes = level_sizes(W, H, p)
    kmax = len(sizes) - 1
    pyr1, pyr2 = [I1], [I2]
    for (w, h) in sizes[1:]:
        pyr1.append(resize(pyr1[-1], w, h))
        pyr2.append(resize(pyr2[-1], w, h))
    u = v = None
    for k in range(kmax, -1, -1):
        w, h = sizes[k]
        if u is None:
            u, v = np.zeros((h, w)), np.zeros((h, w))
        else:
            pw, ph = sizes[k + 1]
            u = resize(u, w, h) * (w / pw)
            v = resize(v, w, h) * (h / ph)
        beta_k = p.beta * ((k / kmax) ** p.b if kmax > 0 else 1.0)
        up, vp, cphi = match_field(matches, phi, W, H, w, h)
        u, v = solve_level(pyr1[k], pyr2[k], u, v, up, vp, cphi, beta_k, p)
    return np.stack([u, v], axis=-1)
