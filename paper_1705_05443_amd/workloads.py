"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the method: it only draws point sets and
right-hand sides (NumPy PCG64) with the shapes and distributions of the
paper's tests (uniform boxes as in Sec. 6.2, clustered volumes, the
Chebyshev / shifted point pairs of the Cauchy-like tests of Sec. 6.3).  It
imports nothing from the rest of the package.
"""
from __future__ import annotations

import numpy as np


def uniform(n: int, d: int, seed: int = 0) -> np.ndarray:
    """n points uniform in [0,1)^d, FP64, row-major (n, d)."""
    return np.random.default_rng(seed).random((n, d))


def clusters(n: int, d: int = 3, seed: int = 0, ncl: int = 8, sigma: float = 0.02,
             frac: float = 0.9) -> np.ndarray:
    """Mixture: frac of the points from ncl equal-weight Gaussian clusters
    (per-axis std sigma, centers uniform in [0.1,0.9]^d; samples falling
    outside the unit cube are redrawn), the rest uniform in [0,1)^d."""
    rng = np.random.default_rng(seed)
    centers = 0.1 + 0.8 * rng.random((ncl, d))
    nc = int(round(frac * n))
    lab = rng.integers(0, ncl, size=nc)
    pts = centers[lab] + sigma * rng.standard_normal((nc, d))
    bad = np.any((pts < 0.0) | (pts >= 1.0), axis=1)
    while bad.any():
        pts[bad] = centers[lab[bad]] + sigma * rng.standard_normal((int(bad.sum()), d))
        bad = np.any((pts < 0.0) | (pts >= 1.0), axis=1)
    out = np.concatenate([pts, rng.random((n - nc, d))], axis=0)
    return out[rng.permutation(n)]


def chebyshev_pair(n: int, seed: int = 0, shift: float = 1e-3, shift_x: bool = False):
    """(x, y) in 1D: one set at cos(pi(2i+1)/(2n)), the other shifted by
    shift*U(0,1).  Default: x = roots, y = x + shift*U.  With shift_x the
    roles swap (y = roots, x = roots + shift*U), which makes K.1 known in
    closed form for the 1/(x-y) kernel."""
    rng = np.random.default_rng(seed)
    roots = np.cos(np.pi * (2.0 * np.arange(n) + 1.0) / (2.0 * n))
    moved = roots + shift * rng.random(n)
    if shift_x:
        return moved[:, None].copy(), roots[:, None].copy()
    return roots[:, None].copy(), moved[:, None].copy()


def interlaced_pair(n: int, seed: int = 0, shift: float = 1e-7):
    """(x, y) in 1D as in eq. (6.3): x_k = k/(n+1), y_k = x_k + shift*U(0,1),
    k = 1..n, so each x_k has a y_k within shift of it."""
    rng = np.random.default_rng(seed)
    x = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    y = x + shift * rng.random(n)
    return x[:, None].copy(), y[:, None].copy()


def cauchy_like_generators(nx: int, ny: int, p: int = 2, seed: int = 0):
    """Generators (w, v) of a Cauchy-like matrix (eq. (6.1)), entries U(0,1) as in
    Sec. 6.3: w is (nx, p), v is (ny, p), row-major."""
    rng = np.random.default_rng(seed + 200)
    return rng.random((nx, p)), rng.random((ny, p))


def curve(name: str, n: int):
    """Nystrom data of the Laplace double-layer operator on a closed curve
    r(t), t in [0, 1), with the trapezoidal rule at t_k = k/n (weight 1/n):
    the ram head r(t) = (2 cos 2 pi t, 1 + sin 2 pi t - 1.4 cos^4 4 pi t)
    or the sunflower r(t) = rho(t) (cos 2 pi t, sin 2 pi t),
    rho = 1.3 + 1.25 cos 40 pi t (both counterclockwise).
    Returns points (n, 2) = r(t_k) and data (n, 3): the weighted normal
    m_k = (r2'(t_k), -r1'(t_k)) / n and the diagonal entry of the
    discretised operator K - I/2 at t_k, (1/n) (r1'' r2' - r2'' r1') /
    (4 pi |r'|^2) - 1/2 (the limit of the kernel at s = t, minus 1/2).
    These are the inputs of the problem, computed from the closed-form
    derivatives of the curve."""
    t = np.arange(n, dtype=np.float64) / n
    tp = 2.0 * np.pi
    if name == "ram_head":
        a, b = tp * t, 2.0 * tp * t
        r1, r2 = 2.0 * np.cos(a), 1.0 + np.sin(a) - 1.4 * np.cos(b) ** 4
        d1 = -2.0 * tp * np.sin(a)
        d2 = tp * np.cos(a) + 1.4 * 4.0 * np.cos(b) ** 3 * np.sin(b) * 2.0 * tp
        e1 = -2.0 * tp * tp * np.cos(a)
        e2 = (-tp * tp * np.sin(a)
              + 1.4 * 4.0 * (2.0 * tp) ** 2 * (np.cos(b) ** 4 - 3.0 * np.cos(b) ** 2 * np.sin(b) ** 2))
    elif name == "sunflower":
        th, ph = tp * t, 20.0 * tp * t
        rho, rp, rpp = 1.3 + 1.25 * np.cos(ph), -1.25 * 20.0 * tp * np.sin(ph), \
            -1.25 * (20.0 * tp) ** 2 * np.cos(ph)
        c, s_ = np.cos(th), np.sin(th)
        r1, r2 = rho * c, rho * s_
        d1, d2 = rp * c - tp * rho * s_, rp * s_ + tp * rho * c
        e1 = rpp * c - 2.0 * tp * rp * s_ - tp * tp * rho * c
        e2 = rpp * s_ + 2.0 * tp * rp * c - tp * tp * rho * s_
    else:
        raise ValueError(name)
    pts = np.stack([r1, r2], axis=1)
    sp2 = d1 * d1 + d2 * d2
    data = np.stack([d2 / n, -d1 / n,
                     (e1 * d2 - e2 * d1) / (4.0 * np.pi * sp2) / n - 0.5], axis=1)
    return np.ascontiguousarray(pts), np.ascontiguousarray(data)


def rhs(n: int, nrhs: int, seed: int = 0) -> np.ndarray:
    """Right-hand sides N(0,1), (n, nrhs) row-major, drawn from seed + 100."""
    return np.random.default_rng(seed + 100).standard_normal((n, nrhs))


# The five workloads (sizes, kernels and parameters).  The point sets are
# drawn by the functions above from the given seed.
CONFIGS = {
    "hss1d_inv_r_2048": dict(kind="uniform", n=2048, d=1, kernel="inv_r", adm=0, leaf=32,
                             order=10, tol=1e-10, eps_svd=1e-10, tau=0.6, nrhs=1,
                             root=((0.0,), 1.0), apply="f64"),
    "h2_2d_log_65536": dict(kind="uniform", n=65536, d=2, kernel="log_r", adm=1, leaf=64,
                            order=8, tol=1e-8, tau=0.7, nrhs=16, root=((0.0, 0.0), 1.0),
                            apply="f64"),
    "h2_3d_inv_r_clusters_1m": dict(kind="clusters", n=1 << 20, d=3, kernel="inv_r", adm=1,
                                    leaf=128, order=5, tol=1e-6, tau=0.7, nrhs=64,
                                    root=((0.0, 0.0, 0.0), 1.0), apply="f32"),
    # the same point set at the order that reaches 1e-6 against exact rows
    # (6^3 Chebyshev points, tol 1e-7) with FP64 apply; the coupling blocks
    # (5.5e10 FP64 entries, 437 GB) are evaluated inside each product
    "h2_3d_inv_r_clusters_1m_p6": dict(kind="clusters", n=1 << 20, d=3, kernel="inv_r", adm=1,
                                       leaf=128, order=6, tol=1e-7, tau=0.7, nrhs=64,
                                       root=((0.0, 0.0, 0.0), 1.0), apply="f64",
                                       coupling="evaluated"),
    # Laplace double layer (Sec. 6.4): HSS on the curve points, 5 x 5
    # interpolation points, tau 0.6, eps_svd 1e-11, leaf 50
    "hss_dl_ram_head_10240": dict(kind="curve", curve="ram_head", n=10240, d=2,
                                  kernel="double_layer", adm=0, leaf=50, order=5, tol=1e-10,
                                  eps_svd=1e-11, tau=0.6, nrhs=1, root=None, apply="f64"),
    "hss_dl_sunflower_10240": dict(kind="curve", curve="sunflower", n=10240, d=2,
                                   kernel="double_layer", adm=0, leaf=50, order=5, tol=1e-10,
                                   eps_svd=1e-11, tau=0.6, nrhs=1, root=None, apply="f64"),
    "hss1d_cauchy_1m": dict(kind="chebyshev_pair", n=1 << 20, d=1, kernel="cauchy", adm=0,
                            leaf=64, order=16, tol=1e-8, eps_svd=1e-9, tau=0.6, nrhs=256,
                            root=None, apply="f32"),
}


def points(cfg: dict, seed: int = 0, n: int | None = None):
    """(x, y) for a workload dict; y is None when Y = X."""
    n = cfg["n"] if n is None else n
    if cfg["kind"] == "uniform":
        return uniform(n, cfg["d"], seed), None
    if cfg["kind"] == "clusters":
        return clusters(n, cfg["d"], seed), None
    if cfg["kind"] == "chebyshev_pair":
        return chebyshev_pair(n, seed)
    if cfg["kind"] == "curve":  # the curve's points; its data from curve()
        return curve(cfg["curve"], n)[0], None
    raise ValueError(cfg["kind"])
