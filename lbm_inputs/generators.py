"""Seeded generators of macroscopic fields and noise (numpy, float64).

Every field is returned as a C-contiguous float64 array of shape (ny, nx),
row index y, column index x.  Coordinates on the unit square are
x_i = i / nx and y_j = j / ny.  Seeds are explicit arguments so that the
oracle tests, the GPU parity tests and the benchmark draw identical inputs.
"""
from __future__ import annotations

import numpy as np


def shock_tube_1d(nx: int = 800):
    """Shock-tube initial data (section 6): density 1 on the left half of the
    tube and 0.5 on the right half, zero velocity.  Returns (rho, ux, uy) of
    shape (1, nx)."""
    rho = np.full((1, nx), 0.5)
    rho[0, : nx // 2] = 1.0
    zero = np.zeros((1, nx))
    return rho, zero.copy(), zero.copy()


def uniform_rest(nx: int, ny: int, rho0: float = 1.0):
    """Fluid at rest with uniform density (lid-driven cavity start)."""
    return np.full((ny, nx), rho0), np.zeros((ny, nx)), np.zeros((ny, nx))


def double_shear_layer(n: int, u0: float = 0.04, sharp: float = 80.0,
                       perturb: float = 0.004):
    """Periodic double shear layer on an n x n grid:
    u_x = u0 tanh(sharp (y - 1/4)) for y <= 1/2, u0 tanh(sharp (3/4 - y))
    above; u_y = perturb sin(2 pi (x + 1/4)); density 1."""
    x = np.arange(n) / n
    y = np.arange(n) / n
    X, Y = np.meshgrid(x, y)  # (ny, nx)
    ux = np.where(Y <= 0.5, u0 * np.tanh(sharp * (Y - 0.25)),
                  u0 * np.tanh(sharp * (0.75 - Y)))
    uy = perturb * np.sin(2.0 * np.pi * (X + 0.25))
    return np.ones((n, n)), np.ascontiguousarray(ux), np.ascontiguousarray(uy)


def spectral_velocity(n: int, k_peak: float = 16.0, u_rms: float = 0.05,
                      seed: int = 5):
    """Divergence-free random velocity on an n x n periodic grid from a
    random-phase streamfunction whose energy spectrum is
    E(k) ~ k^4 exp(-2 (k / k_peak)^2), scaled to an rms speed u_rms."""
    rng = np.random.default_rng(seed)
    kx = np.fft.rfftfreq(n, d=1.0 / n)          # 0 .. n/2
    ky = np.fft.fftfreq(n, d=1.0 / n)           # signed
    KX, KY = np.meshgrid(kx, ky)                # (n, n//2+1)
    K = np.sqrt(KX ** 2 + KY ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        # |psi_hat|^2 ~ E(k) / k^3 for a 2D streamfunction
        amp = np.where(K > 0, np.sqrt(K * np.exp(-2.0 * (K / k_peak) ** 2)), 0.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=amp.shape)
    psi_hat = amp * np.exp(1j * phase)
    ux = np.fft.irfft2(1j * 2 * np.pi * KY * psi_hat, s=(n, n))
    uy = np.fft.irfft2(-1j * 2 * np.pi * KX * psi_hat, s=(n, n))
    rms = np.sqrt(np.mean(ux ** 2 + uy ** 2))
    scale = u_rms / rms
    return (np.ones((n, n)), np.ascontiguousarray(ux * scale),
            np.ascontiguousarray(uy * scale))


def smooth_omega_field(nx: int, ny: int, lo: float = 1.0, hi: float = 1.95,
                       seed: int = 41, modes: int = 6):
    """Smooth per-site relaxation field with values in [lo, hi]: the mean
    (lo+hi)/2 plus (hi-lo)/2 times a sum of random low Fourier modes
    normalised to a maximum magnitude of 1."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    field = np.zeros((ny, nx))
    for _ in range(modes):
        kx, ky = rng.integers(1, 4, size=2)
        ph = rng.uniform(0, 2 * np.pi)
        field += rng.uniform(0.5, 1.0) * np.sin(2 * np.pi * (kx * X + ky * Y) + ph)
    field /= np.max(np.abs(field))
    return np.ascontiguousarray(0.5 * (lo + hi) + 0.5 * (hi - lo) * field)


def fourier_target(nx: int, ny: int, amp: float = 0.05, seed: int = 4,
                   modes: int = 4):
    """Smooth target velocity: the sum over `modes` random Fourier modes of
    amp * e_m * sin(2 pi k_m . x + phi_m), with k_m in {1..4}^2, e_m a random
    unit vector and phi_m uniform on [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    for _ in range(modes):
        kx, ky = rng.integers(1, 5, size=2)
        theta = rng.uniform(0, 2 * np.pi)
        ph = rng.uniform(0, 2 * np.pi)
        s = np.sin(2 * np.pi * (kx * X + ky * Y) + ph)
        ux += amp * np.cos(theta) * s
        uy += amp * np.sin(theta) * s
    return np.ascontiguousarray(ux), np.ascontiguousarray(uy)


def shear_wave(n: int, u0: float = 0.05):
    """Decaying shear wave (section 7) on an n x n periodic grid:
    density 1, u_x = 0, u_y = u0 sin(2 pi i / n) with i the column index."""
    x = np.arange(n)
    uy = np.tile(u0 * np.sin(2 * np.pi * x / n), (n, 1))
    return np.ones((n, n)), np.zeros((n, n)), np.ascontiguousarray(uy)


def uniform_noise(shape, seed: int, amp: float = 1.0):
    """Uniform noise on [-amp, amp) of the given shape."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=shape)


def taylor_green_3d(nx: int, ny: int = None, nz: int = None, u0: float = 0.05):
    """Three-dimensional Taylor-Green vortex on a periodic nx x ny x nz grid
    (arrays in (z, y, x) order), wavenumbers 2 pi / n along each axis:
    u_x = u0 sin(kx x) cos(ky y) cos(kz z), u_y = -u0 cos(kx x) sin(ky y)
    cos(kz z), u_z = 0, and the density of its pressure field,
    rho = 1 + (3 u0^2 / 16) (cos 2 kx x + cos 2 ky y) (cos 2 kz z + 2).
    The velocity is divergence-free when nx = ny."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    z, y, x = np.meshgrid(2 * np.pi * np.arange(nz) / nz, 2 * np.pi * np.arange(ny) / ny,
                          2 * np.pi * np.arange(nx) / nx, indexing="ij")
    ux = u0 * np.sin(x) * np.cos(y) * np.cos(z)
    uy = -u0 * np.cos(x) * np.sin(y) * np.cos(z)
    uz = np.zeros_like(ux)
    rho = 1.0 + (3.0 * u0 * u0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return rho, ux, uy, uz
