"""Pins of the DeepFlow oracle (Sec. 4.3) against what the mathematics fixes:
the penaliser's derivative, the frozen-weight energy that a fixed-point step
minimises (checked by finite differences of the energy written as its sum of
terms), exact 2 x 2 solves, resampling and warping on functions they
reproduce exactly, the eigenvalue against LAPACK, and recovery of a known
translation and of a flow that only the matches state."""
import math

import numpy as np
import pytest

from oracle import deepflow_oracle as F


def smooth_texture(W, H, t=(0.0, 0.0), seed=3):
    """A band-limited image I(x - tx, y - ty) in [0, 1]: a sum of sinusoids,
    so that every shift is exact."""
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(W, dtype=np.float64) - t[0], np.arange(H, dtype=np.float64) - t[1])
    img = np.zeros((H, W))
    for _ in range(12):
        fx, fy = rng.uniform(-0.35, 0.35, 2)
        img += rng.uniform(0.3, 1.0) * np.cos(fx * X + fy * Y + rng.uniform(0, 2 * np.pi))
    return 0.5 + 0.5 * img / 12.0


def test_psi_prime_is_the_derivative_of_psi():
    s2 = np.array([0.0, 1e-6, 0.3, 4.0, 1e3])
    for eps in (0.001, 0.1):
        h = 1e-4 * (s2 + eps * eps)   # central differences on the scale of s^2 + eps^2
        fd = (F.psi(s2 + h, eps) - F.psi(s2 - h, eps)) / (2 * h)
        assert np.allclose(F.psi_prime(s2, eps), fd, rtol=1e-6)


def random_frozen_problem(H, W, seed):
    rng = np.random.default_rng(seed)
    # positive semi-definite 3 x 3 data tensors per pixel: sums of outer products
    J = np.zeros((6, H, W))
    for _ in range(3):
        v = rng.normal(size=(3, H, W))
        J += rng.uniform(0.1, 1.0) * F.sym3(v[0], v[1], v[2])
    a = rng.uniform(0.05, 2.0, (H, W))
    gh, gv = F.edge_weights(a)
    wM = rng.uniform(0.0, 3.0, (H, W)) * (rng.random((H, W)) < 0.5)
    u, v, up, vp = (rng.normal(size=(H, W)) for _ in range(4))
    return J, gh, gv, wM, u, v, up, vp


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sor_minimises_the_frozen_energy(seed):
    """Red-black SOR converges to the increment at which every partial
    derivative of the frozen-weight energy (D5) vanishes; the derivatives are
    finite differences of the energy's plain sum, independent of the update
    formulas."""
    H, W = 5, 6
    J, gh, gv, wM, u, v, up, vp = random_frozen_problem(H, W, seed)
    du, dv = F.sor(J, gh, gv, wM, u, v, np.zeros((H, W)), np.zeros((H, W)), up, vp, 3000, 1.6)
    E = lambda a, b: F.frozen_energy(J, gh, gv, wM, u, v, a, b, up, vp)
    h = 1e-5
    g0 = []
    for arr in ("u", "v"):
        for y in range(H):
            for x in range(W):
                e = np.zeros((H, W)); e[y, x] = h
                if arr == "u":
                    g = (E(du + e, dv) - E(du - e, dv)) / (2 * h)
                    g_at0 = (E(e, 0 * dv) - E(-e, 0 * dv)) / (2 * h)
                else:
                    g = (E(du, dv + e) - E(du, dv - e)) / (2 * h)
                    g_at0 = (E(0 * du, e) - E(0 * du, -e)) / (2 * h)
                g0.append((g, g_at0))
    g = np.array(g0)
    assert np.abs(g[:, 0]).max() < 1e-6 * np.abs(g[:, 1]).max()
    # and it is a minimum: random perturbations raise the energy
    rng = np.random.default_rng(seed + 10)
    e_min = E(du, dv)
    for _ in range(20):
        assert E(du + 1e-3 * rng.normal(size=(H, W)), dv + 1e-3 * rng.normal(size=(H, W))) > e_min


def test_sor_single_pixel_is_the_exact_solve():
    """With no neighbours one unrelaxed sweep solves the pixel's 2 x 2 system."""
    J = F.sym3(np.array([[1.3]]), np.array([[-0.4]]), np.array([[0.7]])) + F.sym3(
        np.array([[0.2]]), np.array([[0.9]]), np.array([[-0.5]]))
    wM = np.array([[0.8]])
    u, v, up, vp = (np.array([[c]]) for c in (0.3, -0.2, 1.0, 0.5))
    gh, gv = np.zeros((1, 0)), np.zeros((0, 1))
    du, dv = F.sor(J, gh, gv, wM, u, v, np.zeros((1, 1)), np.zeros((1, 1)), up, vp, 1, 1.0)
    A = np.array([[J[0, 0, 0] + wM[0, 0], J[1, 0, 0]], [J[1, 0, 0], J[3, 0, 0] + wM[0, 0]]])
    b = np.array([-J[2, 0, 0] - wM[0, 0] * (u[0, 0] - up[0, 0]), -J[4, 0, 0] - wM[0, 0] * (v[0, 0] - vp[0, 0])])
    assert np.allclose([du[0, 0], dv[0, 0]], np.linalg.solve(A, b), rtol=1e-12)


def test_level_sizes_follow_eta_down_to_min_size():
    p = F.FlowParams()
    s = F.level_sizes(64, 48, p)
    assert s[0] == (64, 48) and s[1] == (61, 46)
    assert min(s[-1]) >= 16 and min(round(64 * 0.95 ** len(s)), round(48 * 0.95 ** len(s))) < 16
    assert len(F.level_sizes(512, 256, p)) == 55


def test_resampling_and_warping_on_exact_cases():
    rng = np.random.default_rng(5)
    img = rng.random((9, 13))
    assert np.array_equal(F.resize(img, 13, 9), img)
    assert np.allclose(F.resize(np.full((9, 13), 2.5), 7, 5), 2.5)
    # a linear ramp is reproduced wherever no coordinate is clamped
    X, Y = np.meshgrid(np.arange(40.0), np.arange(30.0))
    ramp = 0.3 * X - 0.7 * Y + 2.0
    r = F.resize(ramp, 38, 28)
    xs = (np.arange(38) + 0.5) * (40 / 38) - 0.5
    ys = (np.arange(28) + 0.5) * (30 / 28) - 0.5
    XS, YS = np.meshgrid(xs, ys)
    assert np.allclose(r[1:-1, 1:-1], (0.3 * XS - 0.7 * YS + 2.0)[1:-1, 1:-1])
    # warping: zero flow is the identity, an integer flow a shift
    assert np.array_equal(F.warp(img, np.zeros_like(img), np.zeros_like(img)), img)
    w = F.warp(img, np.ones_like(img), np.full_like(img, -1.0))
    assert np.array_equal(w[1:, :-1], img[:-1, 1:])
    # half-pixel flow averages neighbours
    h = F.warp(img, np.full_like(img, 0.5), np.zeros_like(img))
    assert np.allclose(h[:, :-1], 0.5 * (img[:, :-1] + img[:, 1:]))


def test_central_differences_and_smoothing():
    X, Y = np.meshgrid(np.arange(12.0), np.arange(10.0))
    gx, gy = F.grad(1.5 * X - 2.0 * Y + 0.25 * X * Y)
    assert np.allclose(gx[1:-1, 1:-1], (1.5 + 0.25 * Y)[1:-1, 1:-1])
    assert np.allclose(gy[1:-1, 1:-1], (-2.0 + 0.25 * X)[1:-1, 1:-1])
    k = F.gauss_taps(0.5)
    assert len(k) == 5 and np.isclose(k.sum(), 1.0) and np.allclose(k, k[::-1])
    assert np.allclose(F.smooth(np.full((6, 7), 3.0), 0.5), 3.0)
    # a Gaussian of a linear function leaves it unchanged away from the border
    s = F.smooth(1.5 * X - 2.0 * Y, 0.5)
    assert np.allclose(s[2:-2, 2:-2], (1.5 * X - 2.0 * Y)[2:-2, 2:-2])


def test_min_eigenvalue_against_lapack():
    rng = np.random.default_rng(9)
    img = F.smooth(rng.random((11, 14)), 0.5)
    lam = F.min_eig_autocorr(img)
    gx, gy = F.grad(img)
    p = lambda a: np.pad(a, 1, mode="edge")
    for y in range(11):
        for x in range(14):
            M = np.zeros((2, 2))
            for dy in range(3):
                for dx in range(3):
                    g = np.array([p(gx)[y + dy, x + dx], p(gy)[y + dy, x + dx]])
                    M += np.outer(g, g)
            assert np.isclose(lam[y, x], np.linalg.eigvalsh(M)[0], rtol=1e-9, atol=1e-9 * M.max())


def test_match_field_keeps_the_first_match_per_pixel():
    m = np.array([[10, 10, 12, 9], [11, 10, 15, 10], [40, 20, 41, 20]], np.float64)
    phi = np.array([0.2, 0.5, 0.1])
    up, vp, cphi = F.match_field(m, phi, 64, 32, 32, 16)   # half size: (10,10) and (11,10) meet at (5,5)
    assert cphi[5, 5] == 0.2 and up[5, 5] == 1.0 and vp[5, 5] == -0.5
    assert cphi[10, 20] == 0.1 and up[10, 20] == 0.5
    assert (cphi > 0).sum() == 2


def test_each_sor_solve_lowers_the_frozen_energy():
    I1 = smooth_texture(40, 32)
    I2 = smooth_texture(40, 32, t=(1.0, 0.5))
    p = F.FlowParams()
    z = np.zeros((32, 40))
    trace = []
    F.solve_level(I1, I2, z, z, z, z, z, 0.0, p, trace=trace)
    assert len(trace) == p.n_fixed and all(after < before for before, after in trace)


def test_translation_is_recovered():
    """I2(x) = I1(x - t): the flow from I1 to I2 is t (no matches).  The
    colour constancy term is on (delta = 1): on this smooth texture the
    gradient constancy term alone is weak next to the smoothness term, and 25
    SOR sweeps then leave the constant mode short of t."""
    t = (1.6, -0.9)
    I1, I2 = smooth_texture(64, 56), smooth_texture(64, 56, t=t)
    flow = F.deepflow(I1, I2, np.zeros((0, 4)), F.FlowParams(delta=1.0))
    inner = flow[10:-10, 10:-10]
    err = np.hypot(inner[..., 0] - t[0], inner[..., 1] - t[1])
    print(f"translation {t}: mean error {err.mean():.4f} px, max {err.max():.4f} px")
    assert err.mean() < 0.05 and err.max() < 0.25


def test_matches_alone_set_the_flow():
    """No data term (gamma = delta = 0): the matches, which all state the flow
    (3, -2), pull every coarse level to it, and the finest level (beta^0 = 0)
    keeps the smooth field it receives."""
    I1, I2 = smooth_texture(64, 48), smooth_texture(64, 48, seed=4)
    ys, xs = np.mgrid[2:48:4, 2:64:4]
    m = np.stack([xs.ravel(), ys.ravel(), xs.ravel() + 3, ys.ravel() - 2], axis=1).astype(np.float64)
    flow = F.deepflow(I1, I2, m, F.FlowParams(gamma=0.0, delta=0.0))
    inner = flow[6:-6, 6:-6]
    assert np.abs(inner[..., 0] - 3.0).max() < 0.05 and np.abs(inner[..., 1] + 2.0).max() < 0.05
