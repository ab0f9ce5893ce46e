"""Seeded synthetic inputs for the MRTLB-VANSE step.

This module only builds input fields (void fraction, forcing, populations);
it holds none of the scheme's arithmetic, so the GPU path and the oracle can
both be fed from it.  Every generator is deterministic in its seed and works
in float64 with numpy; coordinates are node indices (x, y) with node centres
at integer positions, and walls (when present) on the faces y = -1/2 and
y = ny - 1/2.

Workloads (sizes, fields and forcing as used by the tests and the benchmark):
  * ``periodic_wave``   -- 64x64 periodic lattice,
                           phi = 0.75 + 0.2 sin(2 pi x/64) cos(2 pi y/64).
  * ``channel_phi``     -- channel between walls: a tanh step of phi from 0.4
                           (lower half) to 1.0 (upper half), interface width 2
                           cells, plus seeded periodic-Gaussian-smoothed noise
                           of amplitude 0.05 (sigma = 8 cells), clipped to 1.
  * ``batch_lattices``  -- many periodic lattices with log-uniform sides.
  * ``solid_mask``, ``cylinder_channel`` -- solid nodes (uint8 masks).
  * ``mms_case``        -- manufactured void fraction, velocity and body force
                           of the paper's convergence tests (Sec. 3.4, Eq. 27-30
                           and Appendix C).
"""
from __future__ import annotations

import math

import numpy as np


def periodic_wave(nx: int = 64, ny: int = 64, base: float = 0.75, amp: float = 0.2):
    """phi(x, y) = base + amp * sin(2 pi x / nx) * cos(2 pi y / ny)."""
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    return base + amp * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)


def smoothed_noise(nx: int, ny: int, sigma: float, seed: int):
    """Standard normal field smoothed by a periodic Gaussian (FFT), scaled so
    that max |N| = 1."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal((ny, nx))
    kx = np.fft.fftfreq(nx)[None, :]
    ky = np.fft.fftfreq(ny)[:, None]
    kernel = np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx ** 2 + ky ** 2))
    sm = np.real(np.fft.ifft2(np.fft.fft2(n) * kernel))
    return sm / np.max(np.abs(sm))


def channel_phi(nx: int, ny: int, seed: int = 2409, lo: float = 0.4, hi: float = 1.0,
                width: float = 2.0, noise: float = 0.05, sigma: float = 8.0):
    """Channel void fraction: tanh step from ``lo`` (y < ny/2) to ``hi``
    (y > ny/2) of width ``width`` cells at mid-channel, plus smoothed noise of
    amplitude ``noise``; clipped to at most 1."""
    y = np.arange(ny)[:, None] + 0.5  # distance of node centres from the lower wall
    mid, half = 0.5 * (hi + lo), 0.5 * (hi - lo)
    step = mid - half * np.tanh((0.5 * ny - y) / width)
    eta = noise * smoothed_noise(nx, ny, sigma, seed) if noise > 0 else 0.0
    return np.minimum(1.0, step + eta) * np.ones((1, nx))


def discontinuous_block(n: int = 100, phi0: float = 0.5):
    """phi = phi0 on the square [0.4n, 0.6n]^2 and 1 elsewhere (Sec. 3.3, Eq. 24)."""
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    inside = (x >= 0.4 * n) & (x <= 0.6 * n) & (y >= 0.4 * n) & (y <= 0.6 * n)
    return np.where(inside, phi0, 1.0).astype(np.float64)


def random_populations(nx: int, ny: int, seed: int, level: float = 1.0,
                       spread: float = 0.05):
    """Positive random populations (9, ny, nx): magnitudes near level * w_i
    of the D2Q9 weights, each multiplied by (1 + spread * N(0, 1))."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rng = np.random.default_rng(seed)
    return level * w[:, None, None] * (1.0 + spread * rng.standard_normal((9, ny, nx)))


def batch_lattices(count: int = 256, seed: int = 4, lmin: int = 32, lmax: int = 512):
    """Independent periodic lattices: side L = round(exp U(ln lmin, ln lmax)),
    phi = 0.6 + 0.3 sin(2 pi kx x / L) sin(2 pi ky y / L) with kx, ky in
    {1..4}, force magnitude |G| ~ U[1e-7, 1e-5] along +x."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        L = int(round(math.exp(rng.uniform(math.log(lmin), math.log(lmax)))))
        kx, ky = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        g = float(rng.uniform(1e-7, 1e-5))
        x = np.arange(L)[None, :]
        y = np.arange(L)[:, None]
        phi = 0.6 + 0.3 * np.sin(2 * np.pi * kx * x / L) * np.sin(2 * np.pi * ky * y / L)
        out.append(dict(L=L, kx=kx, ky=ky, g=g, phi=phi))
    return out


# ---- manufactured solutions (Sec. 3.4) ------------------------------------

def _mms_coords(n: int, us: float, t: float):
    x = np.arange(n, dtype=np.float64)[None, :] * np.ones((n, 1))
    y = np.arange(n, dtype=np.float64)[:, None] * np.ones((1, n))
    xs = (2 * x - n + 1) / n  # Eq. (30)
    ys = (2 * y - n + 1) / n
    shift = 4.0 * us * t / n ** 2
    return xs, ys, xs + shift, ys + shift


def mms_case(case: str, n: int, a: float, b: float, us: float, nu: float, t: float = 0.0):
    """Manufactured void fraction phi~, velocity u~ and body force F^B on an
    n x n periodic lattice (node coordinates of Eq. 30, dx = 1/n).

    Case I  : Eq. (27) with the force of Eq. (C1).
    Case II : Eq. (28) with the force of Eq. (C2).
    Case III: Eq. (29) with the force of Eq. (C3) at time step t.
    Returns dict(phi, ux, uy, fx, fy).
    """
    xs, ys, xt, yt = _mms_coords(n, us, t)
    pi = np.pi
    n3 = float(n) ** 3
    if case == "I":
        sx, cx, sy, cy = np.sin(pi * xs), np.cos(pi * xs), np.sin(pi * ys), np.cos(pi * ys)
        phi = a + b * sx * sy
        ux = us / n * (-sx ** 2 * sy * cy)
        uy = us / n * (sy ** 2 * sx * cx)
        fx = (2 * pi * us ** 2 * phi / n3 * sx ** 3 * cx * sy ** 2
              + 4 * nu * pi ** 2 * us * b / n3 * sx ** 3 * cy ** 3
              + 4 * nu * pi ** 2 * us / n3 * sy * cy
              * (-6 * phi * sx ** 2 + 2 * a * cx ** 2 + 5 * b * sx * cx ** 2 * sy))
        fy = (2 * pi * us ** 2 * phi / n3 * sx ** 2 * sy ** 3 * cy
              - 4 * nu * pi ** 2 * us / n3 * sx * cx * cy ** 2 * (2 * a + 5 * b * sx * sy)
              + 4 * nu * pi ** 2 * us / n3 * cx * sy ** 2
              * (6 * a * sx + 6 * b * sx ** 2 * sy - b * cx ** 2 * sy))
    elif case == "II":
        sx, cx, sy, cy = np.sin(pi * xs), np.cos(pi * xs), np.sin(pi * ys), np.cos(pi * ys)
        phi = a * np.exp(-b * sx * sy)
        ux = us / n * np.exp(b * sx * sy)
        uy = ux.copy()
        fx = (2 * pi * us ** 2 * a * b / n3 * np.exp(b * sx * sy) * np.sin(pi * (xs + ys))
              - 4 * nu * pi ** 2 * us * a * b / (3 * n3) * (cx * cy - 7 * sx * sy))
        fy = fx.copy()
    elif case == "III":
        phi = a + b * np.sin(pi * xt) * np.sin(pi * yt)
        ux = us / n * (1.0 / phi - 2.0)
        uy = ux.copy()
        spp = np.sin(pi * (xt + yt))
        common = (-8 * pi * us ** 2 * b / n3 * spp
                  + 2 * pi * us ** 2 * b / (n3 * phi ** 2) * spp * (4 * phi ** 2 - 1))
        visc = 2 * nu * pi ** 2 * us * b / (3 * n3 * phi ** 2)
        fx = common + visc * (3 * b * np.cos(2 * pi * xt) + 4 * b * np.cos(2 * pi * yt) - 7 * b
                              + 8 * a * np.cos(pi * (xt + yt)) - 6 * a * np.cos(pi * (xt - yt)))
        fy = common + visc * (4 * b * np.cos(2 * pi * xt) + 3 * b * np.cos(2 * pi * yt) - 7 * b
                              + 8 * a * np.cos(pi * (xt + yt)) - 6 * a * np.cos(pi * (xt - yt)))
    else:
        raise ValueError(f"unknown manufactured case {case!r}")
    return dict(phi=phi, ux=ux, uy=uy, fx=fx, fy=fy)


def inclusion_phi(L: int, rng, rmin: float = 5.0, rmax: float = 50.0, fill: float = 0.15,
                  lo: float = 0.35, width: float = 2.0):
    """Periodic L x L void fraction with tanh-edged circular inclusions:
    phi = 1 - (1 - lo) max_k 1/2 (1 - tanh((d_k - r_k)/width)), radii
    r_k ~ U[rmin, rmax], count ceil(fill L^2 / (pi rbar^2)), uniform centres,
    periodic distance d_k.  Each inclusion is evaluated on a window around it."""
    rbar = 0.5 * (rmin + rmax)
    count = int(math.ceil(fill * L * L / (math.pi * rbar * rbar)))
    m = np.zeros((L, L))
    for _ in range(count):
        r = rng.uniform(rmin, rmax)
        cx, cy = rng.uniform(0, L, 2)
        h = int(min(L // 2, math.ceil(r + 10 * width)))
        xs = np.arange(int(cx) - h, int(cx) + h + 1)
        ys = np.arange(int(cy) - h, int(cy) + h + 1)
        if len(xs) > L:
            xs = np.arange(L)
        if len(ys) > L:
            ys = np.arange(L)
        dx = xs[None, :] - cx
        dy = ys[:, None] - cy
        dx = dx - L * np.round(dx / L)
        dy = dy - L * np.round(dy / L)
        v = 0.5 * (1 - np.tanh((np.sqrt(dx * dx + dy * dy) - r) / width))
        iy = np.mod(ys, L)[:, None]
        ix = np.mod(xs, L)[None, :]
        m[iy, ix] = np.maximum(m[iy, ix], v)
    return 1.0 - (1.0 - lo) * m


def served_requests(count: int = 40, rate: float = 4.0, seed: int = 5, lmin: int = 64,
                    lmax: int = 2048, beta0: float = 2e-3, beta1: float = 1e-2, g: float = 1e-6):
    """Solve requests for the serving loop: Poisson arrivals at `rate` per
    second; each a periodic L x L lattice, L = round(exp U(ln lmin, ln lmax)),
    with an inclusion void fraction (inclusion_phi), body force G = g along x
    and a linear drag beta = beta0 + beta1 (1 - phi) (background drag keeps a
    steady state reachable on a periodic domain)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        L = int(round(math.exp(rng.uniform(math.log(lmin), math.log(lmax)))))
        phi = inclusion_phi(L, rng)
        out.append(dict(rid=k, L=L, arrival=t, phi=phi, beta=beta0 + beta1 * (1.0 - phi), g=g))
    return out


def solid_mask(nx: int, ny: int, seed: int, discs: int = 3, rmin: float = 1.5,
               rmax: float = None, singles: int = None):
    """Solid nodes (uint8, 1 = solid): `discs` periodic discs of radius
    U[rmin, rmax] (rmax default min(nx, ny)/6) at uniform centres, plus
    `singles` isolated solid nodes (default nx*ny/200, at least 2) and one
    solid node on each edge row and column (next to walls and to the
    periodic seams).  A mask that leaves no fluid node is never returned."""
    rng = np.random.default_rng(seed)
    rmax = max(rmin, min(nx, ny) / 6.0) if rmax is None else rmax
    singles = max(2, nx * ny // 200) if singles is None else singles
    yy, xx = np.mgrid[0:ny, 0:nx]
    m = np.zeros((ny, nx), np.uint8)
    for _ in range(discs):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        r = rng.uniform(rmin, rmax)
        dx = xx - cx
        dy = yy - cy
        dx = dx - nx * np.round(dx / nx)
        dy = dy - ny * np.round(dy / ny)
        m[dx * dx + dy * dy < r * r] = 1
    for _ in range(singles):
        m[rng.integers(ny), rng.integers(nx)] = 1
    m[0, nx // 3] = m[ny - 1, nx // 2] = m[ny // 2, 0] = m[ny // 2, nx - 1] = 1
    if m.all():
        m[ny // 2, nx // 2] = 0
    return m


def cylinder_channel(nx: int, ny: int, radius: float):
    """A channel with walls in y and one solid disc (uint8 mask) centred at
    (nx/4, ny/2) -- flow past a cylinder between plates."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    return (((xx + 0.5 - nx / 4) ** 2 + (yy + 0.5 - ny / 2) ** 2) < radius ** 2).astype(np.uint8)
