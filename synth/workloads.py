"""Input recipes (all numpy, float64, seeded with numpy.random.default_rng).

A source array has shape [nt] + level_shape and holds f(x, t_k) for t_k = k*tau,
k = 0..nt-1 (the samples f^(0..nt-1) that enter the right-hand side of the
all-at-once system).  ``level_shape`` is (nx,) in 1D and (ny, nx) in 2D, x fastest;
interior points x_i = i/(nx+1).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def grid_points(nx: int, ny: int = 0):
    x = np.arange(1, nx + 1) / (nx + 1.0)
    if not ny:
        return (x,)
    y = np.arange(1, ny + 1) / (ny + 1.0)
    X, Y = np.meshgrid(x, y, indexing="xy")
    return (X, Y)


def _times(nt: int, T: float):
    return (T / nt) * np.arange(nt)


def manufactured_1d(nx: int, nt: int, T: float = 1.0, noise_std: float = 0.0, seed: int = 1):
    """u = sin(pi x) sin(pi t) solves u_tt = u_xx, so f = 0, psi_0 = 0,
    psi_1 = pi sin(pi x); optional i.i.d. N(0, noise_std^2) source noise per
    (level, point).  Returns (src, psi0, psi1, exact) with exact at t_1..t_nt."""
    (x,) = grid_points(nx)
    t = _times(nt, T)
    src = np.zeros((nt, nx))
    if noise_std:
        src += noise_std * np.random.default_rng(seed).standard_normal((nt, nx))
    psi0 = np.zeros(nx)
    psi1 = np.pi * np.sin(np.pi * x)
    tk = (T / nt) * np.arange(1, nt + 1)
    exact = np.sin(np.pi * tk)[:, None] * np.sin(np.pi * x)[None, :]
    return src, psi0, psi1, exact


def manufactured_2d(nx: int, ny: int, nt: int, T: float = 1.0):
    """u = sin(pi x) sin(pi y) sin(pi t): f = pi^2 sin(pi x) sin(pi y) sin(pi t),
    psi_0 = 0, psi_1 = pi sin(pi x) sin(pi y).  Returns (src, psi0, psi1, exact)."""
    X, Y = grid_points(nx, ny)
    s = np.sin(np.pi * X) * np.sin(np.pi * Y)
    t = _times(nt, T)
    src = (np.pi ** 2) * np.sin(np.pi * t)[:, None, None] * s[None]
    psi0 = np.zeros_like(s)
    psi1 = np.pi * s
    tk = (T / nt) * np.arange(1, nt + 1)
    exact = np.sin(np.pi * tk)[:, None, None] * s[None]
    return src, psi0, psi1, exact


def random_source(nx: int, ny: int, nt: int, seed: int):
    """i.i.d. N(0, 1) source samples, zero initial data."""
    shape = (nt, ny, nx) if ny else (nt, nx)
    src = np.random.default_rng(seed).standard_normal(shape)
    z = np.zeros(shape[1:])
    return src, z, z.copy()


def gaussian_field_source(nx: int, ny: int, nt: int, T: float = 1.0, ell: float = 0.1, seed: int = 3):
    """Gaussian random field on the (t, y, x) grid: i.i.d. N(0,1) samples filtered in
    Fourier space by exp(-2 pi^2 ell^2 |k|^2) (k in cycles per unit on each axis),
    normalised to unit RMS.  Zero initial data."""
    shape = (nt, ny, nx) if ny else (nt, nx)
    white = np.random.default_rng(seed).standard_normal(shape)
    spacings = [T / nt] + ([1.0 / (ny + 1)] if ny else []) + [1.0 / (nx + 1)]
    spec = sfft.rfftn(white, workers=-1)
    del white
    k2 = None
    for ax, (n, d) in enumerate(zip(shape, spacings)):
        k = np.fft.rfftfreq(n, d=d) if ax == len(shape) - 1 else np.fft.fftfreq(n, d=d)
        kk = (k ** 2).reshape([-1 if a == ax else 1 for a in range(len(shape))])
        k2 = kk if k2 is None else k2 + kk
    spec *= np.exp(-2.0 * np.pi ** 2 * ell ** 2 * k2)
    field = sfft.irfftn(spec, s=shape, axes=tuple(range(len(shape))), workers=-1)
    del spec
    field /= np.sqrt(np.mean(field ** 2))
    z = np.zeros(shape[1:])
    return field, z, z.copy()


def jacobi_smoothed_source(nx: int, ny: int, nt: int, seed: int, sweeps: int = 3, omega: float = 2.0 / 3.0):
    """i.i.d. N(0,1) samples on every level, then ``sweeps`` weighted-Jacobi sweeps of
    the 2D discrete Laplace equation on each level with zero ghosts:
    v <- (1 - omega) v + omega * (sum of the 4 neighbours) / 4.  Zero initial data."""
    if not ny:
        raise ValueError("Jacobi-smoothed sources are two-dimensional")
    v = np.random.default_rng(seed).standard_normal((nt, ny, nx))
    for _ in range(sweeps):
        p = np.pad(v, ((0, 0), (1, 1), (1, 1)))
        nb = p[:, :-2, 1:-1] + p[:, 2:, 1:-1] + p[:, 1:-1, :-2] + p[:, 1:-1, 2:]
        v = (1.0 - omega) * v + omega * 0.25 * nb
    z = np.zeros((ny, nx))
    return v, z, z.copy()


SERVING_SHAPES = (
    [(nx, 0) for nx in (255, 1023, 4095)] + [(n, n) for n in (63, 127, 255)]
)
SERVING_NT = (64, 256, 1024)
SERVING_ALPHA = (1e-2, 1e-3)


def serving_trace(rate: float, count: int, seed: int = 5):
    """Poisson arrivals at ``rate`` requests/s: returns a list of dicts with the
    arrival time and a shape drawn uniformly from the serving mix
    {1D nx in (255,1023,4095), 2D nx=ny in (63,127,255)} x nt in (64,256,1024) x
    alpha in (1e-2,1e-3); request i's source uses seed 5000+i."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        nx, ny = SERVING_SHAPES[rng.integers(len(SERVING_SHAPES))]
        nt = SERVING_NT[rng.integers(len(SERVING_NT))]
        alpha = SERVING_ALPHA[rng.integers(len(SERVING_ALPHA))]
        out.append({"arrival": float(t[i]), "nx": nx, "ny": ny, "nt": nt,
                    "alpha": alpha, "seed": 5000 + i})
    return out


# Mixes of grids solved as one group, (nx, ny, nt, alpha) per member, sources from
# random_source with seed 50 + member index: many tiny 1D solves, small 2D and 1D
# solves, shapes of the serving mix (those with 256-thread tiles), and one C2-sized
# solve alone.
GROUP_MIXES = {
    "1d16": [(255, 0, 64, 1e-3)] * 16,
    "small8": [(63, 63, 64, 1e-3)] * 4 + [(1023, 0, 64, 1e-3)] * 4,
    "serving7": [(63, 63, 256, 1e-2), (127, 127, 64, 1e-3), (255, 0, 512, 1e-3), (1023, 0, 256, 1e-2),
                 (63, 63, 64, 1e-3), (255, 0, 256, 1e-2), (127, 127, 256, 1e-3)],
    "big1": [(255, 255, 256, 1e-3)],
}


# The five workloads (name -> description used in reports).
WORKLOADS = {
    "wave1d_63x64": "1D, nx=63, nt=64, T=1, manufactured u=sin(pi x)sin(pi t) + N(0, 0.1^2) source noise (seed 1)",
    "wave2d_255x255x256": "2D, nx=ny=255, nt=256, T=1, manufactured u=sin(pi x)sin(pi y)sin(pi t)",
    "wave2d_511x511x512": "2D, nx=ny=511, nt=512, T=1, Gaussian random-field source (ell=0.1, seed 3)",
    "batch64_wave2d_127x127x128": "64 RHS, 2D nx=ny=127, nt=128, N(0,1) sources (seed 4000+i) + 3 Jacobi sweeps",
    "serving_mix": "Poisson arrivals of mixed 1D/2D solves, nt in {64,256,1024}, alpha in {1e-2,1e-3}",
}
