"""Seeded synthetic pansharpening scenes.

The paper evaluates on remote-sensing datasets that are not available here (Sec. IV-A).  This module stands in
for them with a fixed, seeded recipe whose shapes follow the paper's workloads (4-16 spectral bands, x4
resolution gap, Gaussian blur kernels that carry a sub-pixel misalignment):

* truth Z: ``n_ellipses`` random ellipses with shared geometry and per-band intensities U[0, 1] (hard edges,
  periodic wrap, overlaps add), plus a per-band low-frequency Gaussian random field (white noise filtered in the
  Fourier domain by a Gaussian of correlation length H/16 px, scaled to standard deviation ``grf_std``);
* PAN Y: a Dirichlet(1)-weighted sum of the bands plus white noise (standard deviation ``pan_noise``);
* blur kernel u: the unit-gain sampled Gaussian of eq. (gaussian_blur) in Sec. IV-B, here with an optional
  rotated anisotropic covariance; its peak (c_x, c_y) is the sub-pixel misalignment;
* LRMS X: each band circularly blurred by u, decimated by c at phase 0, plus white noise (``ms_noise``).

This is the observation simulator of Sec. IV-B, not the solver: the solver's own arithmetic lives in the HIP
library and, separately, in the oracle.  Both take their inputs from here, rounded once to float32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 210309943


def scene_rng(config: int, scene: int) -> np.random.Generator:
    """Generator for scene ``scene`` of workload ``config``; seeds never collide across workloads."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, int(config), int(scene)]))


@dataclasses.dataclass
class Scene:
    """One synthetic scene.  Arrays are C-contiguous float32, planar (band-major)."""

    X: np.ndarray  # LRMS [N][h][w]
    Y: np.ndarray  # PAN [H][W]
    u: np.ndarray  # blur kernel [n][n], centre at [(n-1)/2][(n-1)/2]
    Z: np.ndarray  # ground-truth HRMS [N][H][W]
    c: int  # decimation factor H/h

    @property
    def shape(self):
        N, h, w = self.X.shape
        return N, h, w, self.c, self.u.shape[0]


def gaussian_kernel(n: int, sigma_x: float, sigma_y: float | None = None, theta: float = 0.0,
                    cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """Unit-gain n x n sampled Gaussian (Sec. IV-B, eq. gaussian_blur), float64.

    Index [a][b] holds the tap at integer offset (y, x) = (a - R, b - R), R = (n-1)/2; rows are y, columns x.
    The peak sits at (x, y) = (cx, cy).  With sigma_y given, the covariance is R(theta) diag(sx^2, sy^2) R(theta)^T.
    """
    if n % 2 != 1 or n < 1:
        raise ValueError("kernel size must be odd")
    R = (n - 1) // 2
    sigma_y = sigma_x if sigma_y is None else sigma_y
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    dx, dy = xx - cx, yy - cy
    ct, st = math.cos(theta), math.sin(theta)
    along = ct * dx + st * dy
    across = -st * dx + ct * dy
    g = np.exp(-0.5 * ((along / sigma_x) ** 2 + (across / sigma_y) ** 2))
    return g / g.sum()


def motion_blur_kernel(R: int, sigma: float, d: float, theta: float, cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """Unit-gain (2R+1) x (2R+1) blur kernel of eq. (blur_kernel_final): the isotropic Gaussian of eq.
    (gaussian_blur) convolved with the d-wide motion blur of eq. (motion_blur) along direction theta, peak at
    (cx, cy), sampled at the integer offsets (App. B, steps I-III), float64.  Index [a][b] is the offset
    (y, x) = (a - R, b - R).  d = 0 gives the Gaussian itself."""
    n = 2 * R + 1
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    ct, st = math.cos(theta), math.sin(theta)
    xp = (xx - cx) * ct + (yy - cy) * st     # along the motion
    yp = -(xx - cx) * st + (yy - cy) * ct    # across it
    if d > 0:
        def cdf(x):
            return 0.5 * (1.0 + np.vectorize(math.erf)(x / (sigma * math.sqrt(2.0))))
        along = (cdf(xp + d / 2) - cdf(xp - d / 2)) / d
    else:
        along = np.exp(-0.5 * (xp / sigma) ** 2)
    g = along * np.exp(-0.5 * (yp / sigma) ** 2)
    assert g.shape == (n, n)
    return g / g.sum()


def _ellipse_layer(rng, H, W, n_ellipses):
    """Geometry of the shared ellipses: list of (rows, cols, mask)."""
    out = []
    for _ in range(n_ellipses):
        cyy, cxx = rng.uniform(0, H), rng.uniform(0, W)
        a, b = rng.uniform(H / 32, H / 4), rng.uniform(H / 32, H / 4)
        phi = rng.uniform(0, math.pi)
        ext = int(math.ceil(max(a, b))) + 1
        ext = min(ext, (min(H, W) - 1) // 2)
        oy, ox = np.mgrid[-ext:ext + 1, -ext:ext + 1].astype(np.float64)
        fy, fx = math.floor(cyy), math.floor(cxx)
        py, px = oy + fy - cyy, ox + fx - cxx
        cp, sp = math.cos(phi), math.sin(phi)
        e1 = (cp * px + sp * py) / a
        e2 = (-sp * px + cp * py) / b
        mask = (e1 * e1 + e2 * e2) <= 1.0
        rows = (np.arange(-ext, ext + 1) + fy) % H
        cols = (np.arange(-ext, ext + 1) + fx) % W
        out.append((rows, cols, mask))
    return out


def _grf(rng, H, W, corr, std):
    """Periodic low-frequency Gaussian random field of standard deviation ``std``."""
    noise = rng.standard_normal((H, W))
    ky = np.fft.fftfreq(H)[:, None]
    kx = np.fft.rfftfreq(W)[None, :]
    filt = np.exp(-2.0 * (math.pi * corr) ** 2 * (ky * ky + kx * kx))
    f = np.fft.irfft2(np.fft.rfft2(noise) * filt, s=(H, W))
    s = f.std()
    return f * (std / s) if s > 0 else f


def _simulate_lrms(Z_band, u, c):
    """Circular blur of one band by u (true convolution, centre of u at offset 0) then decimation at phase 0."""
    H, W = Z_band.shape
    n = u.shape[0]
    R = (n - 1) // 2
    otf = np.zeros((H, W))
    for a in range(n):
        for b in range(n):
            otf[(a - R) % H, (b - R) % W] += u[a, b]
    blurred = np.fft.irfft2(np.fft.rfft2(Z_band) * np.fft.rfft2(otf), s=(H, W))
    return blurred[::c, ::c]


def make_scene(rng: np.random.Generator, H: int, W: int, N: int, c: int, u: np.ndarray, *,
               n_ellipses: int = 40, grf_std: float = 0.05, pan_noise: float = 0.01,
               ms_noise: float = 0.01) -> Scene:
    """Draw one scene.  ``u`` is the (float64) blur kernel; it is stored rounded to float32."""
    if H % c or W % c:
        raise ValueError("H and W must be multiples of c")
    u32 = np.ascontiguousarray(u, dtype=np.float32)
    geom = _ellipse_layer(rng, H, W, n_ellipses)
    inten = rng.uniform(0.0, 1.0, size=(n_ellipses, N))
    weights = rng.dirichlet(np.ones(N))
    Z = np.zeros((N, H, W), dtype=np.float32)
    Y = np.zeros((H, W), dtype=np.float64)
    X = np.zeros((N, H // c, W // c), dtype=np.float32)
    for i in range(N):
        band = _grf(rng, H, W, H / 16.0, grf_std)
        for e, (rows, cols, mask) in enumerate(geom):
            band[np.ix_(rows, cols)] += inten[e, i] * mask
        Z[i] = band
        Y += weights[i] * band
        X[i] = _simulate_lrms(band, u32.astype(np.float64), c) + ms_noise * rng.standard_normal((H // c, W // c))
    Y += pan_noise * rng.standard_normal((H, W))
    return Scene(X=X, Y=Y.astype(np.float32), u=u32, Z=Z, c=c)


# ---------------------------------------------------------------------------------------------------------------
# The measured workloads.  Solver settings that the paper leaves open are fixed here (window radius r, lambda,
# epsilon; epsilon enters the matting matrix as eps/|w| + sigma^2).
# ---------------------------------------------------------------------------------------------------------------

@dataclasses.dataclass
class SolveSettings:
    r: int
    lam: float
    eps: float
    max_iters: int
    tol: float  # <= 0: run exactly max_iters iterations


def config_scene(config: int, scene: int = 0, *, side: int | None = None) -> tuple[Scene, SolveSettings]:
    """Scene ``scene`` of workload ``config`` (0..4) with its solver settings.

    0: 4 bands, 256^2 PAN, 64^2 LRMS, 9x9 Gaussian (sigma 1.5), r 1, lambda 1e-2, exactly 50 iterations.
    1: 8 bands, 2048^2 PAN, 512^2 LRMS, 17x17 anisotropic Gaussian (2.0, 1.4, random rotation), r 2, tol 1e-6.
    2: batch member: PAN side from {256, 384, ..., 1024}, 4 or 8 bands, 9..17 taps, sigma U(1, 2.5), r 1, tol 1e-6.
    3: warm-start set: scenes 0..1999 training (4 bands, 256^2), 2000.. evaluation (8 bands, 512^2), as 2.
    4: 16 bands, 4096^2 PAN, 1024^2 LRMS, 17x17 Gaussian sigma U(1.5, 2.5), LRMS noise 0.005, r 2, tol 1e-6.
    ``side`` overrides the PAN side (same recipe, smaller scene) for quick tests.
    """
    rng = scene_rng(config, scene)
    cx, cy = rng.uniform(-0.5, 0.5, size=2)
    eps = 1e-3
    if config == 0:
        H = side or 256
        u = gaussian_kernel(9, 1.5, cx=cx, cy=cy)
        sc = make_scene(rng, H, H, 4, 4, u)
        return sc, SolveSettings(r=1, lam=1e-2, eps=eps, max_iters=50, tol=0.0)
    if config == 1:
        H = side or 2048
        theta = rng.uniform(0, math.pi)
        u = gaussian_kernel(17, 2.0, 1.4, theta, cx=cx, cy=cy)
        sc = make_scene(rng, H, H, 8, 4, u)
        return sc, SolveSettings(r=2, lam=1e-2, eps=eps, max_iters=20000, tol=1e-6)
    if config in (2, 3):
        if config == 2:
            H = side or int(rng.choice(np.arange(256, 1025, 128)))
            N = 4 if rng.uniform() < 0.5 else 8
        elif scene < 2000:
            H, N = side or 256, 4
        else:
            H, N = side or 512, 8
        n = int(rng.choice(np.arange(9, 18, 2)))
        sigma = rng.uniform(1.0, 2.5)
        u = gaussian_kernel(n, sigma, cx=cx, cy=cy)
        sc = make_scene(rng, H, H, N, 4, u)
        return sc, SolveSettings(r=1, lam=1e-2, eps=eps, max_iters=20000, tol=1e-6)
    if config == 4:
        H = side or 4096
        sigma = rng.uniform(1.5, 2.5)
        u = gaussian_kernel(17, sigma, cx=cx, cy=cy)
        sc = make_scene(rng, H, H, 16, 4, u, ms_noise=0.005)
        return sc, SolveSettings(r=2, lam=1e-2, eps=eps, max_iters=20000, tol=1e-6)
    raise ValueError(f"unknown workload {config}")


def random_problem(rng: np.random.Generator, N: int, H: int, W: int, c: int, n: int):
    """Unstructured random inputs for operator tests: LRMS, PAN, a random positive unit-gain kernel, a plane set."""
    X = rng.standard_normal((N, H // c, W // c)).astype(np.float32)
    Y = rng.uniform(0, 1, (H, W)).astype(np.float32)
    u = rng.uniform(0.0, 1.0, (n, n))
    u = (u / u.sum()).astype(np.float32)
    P = rng.standard_normal((N, H, W)).astype(np.float32)
    return X, Y, u, P


def cnn_init_params(rng: np.random.Generator, layers=(2, 32, 32, 32, 32, 1), last_std: float = 1e-3):
    """Random initial weights of the warm-start network, flat float32 in the library's layout (per layer its
    W [out][in][3][3] then its b [out]): He-normal weights for the ReLU layers, a small normal last layer
    (the untrained network starts close to the plain upsampled band), zero biases."""
    out = []
    for k in range(len(layers) - 1):
        cin, cout = layers[k], layers[k + 1]
        std = last_std if k == len(layers) - 2 else math.sqrt(2.0 / (9 * cin))
        out.append(rng.normal(0.0, std, size=cout * cin * 9))
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)
