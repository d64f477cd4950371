"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only produces problem data: per-cell wave speeds / wavenumbers,
Gaussian source centres, and the load vector of a Gaussian source.  It holds
none of the solver's arithmetic (no operator, smoother, transfer, coarse
stencil or Krylov code), so that the CPU oracle and the HIP path can both take
their inputs from here without sharing any of the method.

Conventions (shared with the library's documented layout):
  * the domain is the unit square [0,1]^2 (or the unit cube), split in N cells
    per direction of size h = 1/N; cell index is x-fastest;
  * the order-p space has (pN+1)^d nodes at the Gauss-Lobatto-Legendre (GLL)
    points of every cell, numbered lexicographically on the global node grid,
    x fastest;
  * a load vector is complex128 with shape (R, n_nodes).

Input recipe (project definitions; the paper's own experiments use constant k):
  * heterogeneous media: white noise N(0,1) per fine cell from numpy's PCG64
    with the given seed, filtered in Fourier space with the square root of the
    spectrum of the Gaussian covariance exp(-r^2 / (2 l^2)) on a zero-padded
    grid, then mapped affinely so that min = c_min and max = c_max exactly;
  * angular frequency omega = 2*pi*W*c_min so that the slowest speed has W
    wavelengths across the unit domain; k = omega / c per cell;
  * absorbing layer (the recipe of the paper's convergence tests, Sec. 7):
    over about 40 DOFs (40 / p cells) next to a flagged side the damping eps
    rises with a sin^2 profile from 0 to 2 k^2 / pi (D = 2 damping per
    wavelength, Sec. 5.2); here the layer takes the outer cells of the unit
    domain instead of cells added outside it;
  * Gaussian source g(x) = exp(-|x-x0|^2 / (2 sigma^2)), load vector by GLL
    quadrature on every cell: f_j = h^d * sum over cells containing node j of
    the tensor GLL weight of j in that cell times g(x_j).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "gll_points",
    "grf_speed",
    "constant_wavenumber",
    "wavenumber_from_speed",
    "gaussian_centres_grid",
    "gaussian_load",
    "absorbing_layer_eps",
    "random_complex",
    "config",
]


def gll_points(p: int):
    """GLL nodes and weights of degree p on [0, 1] (nodes ascending)."""
    if p < 1:
        raise ValueError("p must be >= 1")
    if p == 1:
        x = np.array([-1.0, 1.0])
    else:
        leg = np.polynomial.legendre.Legendre.basis(p)
        inner = np.sort(np.real(leg.deriv().roots()))
        x = np.concatenate([[-1.0], inner, [1.0]])
    leg = np.polynomial.legendre.Legendre.basis(p)
    w = 2.0 / (p * (p + 1) * leg(x) ** 2)
    # symmetrise against root-finder noise
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    return 0.5 * (x + 1.0), 0.5 * w


def grf_speed(n_cells: int, dim: int, ell: float, cmin: float, cmax: float,
              seed: int = 0) -> np.ndarray:
    """Per-cell wave speed from a seeded Gaussian random field.

    Returns an array of shape (N,)*dim indexed [..., iy, ix] (x fastest when
    flattened) with exact min cmin and max cmax.
    """
    h = 1.0 / n_cells
    pad = int(math.ceil(4.0 * ell / h))
    m = n_cells + 2 * pad
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((m,) * dim)
    freqs = [np.fft.fftfreq(m, d=h) * 2.0 * math.pi for _ in range(dim)]
    grids = np.meshgrid(*freqs, indexing="ij")
    kk = sum(g * g for g in grids)
    amp = np.exp(-0.25 * ell * ell * kk)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * amp))
    sl = tuple(slice(pad, pad + n_cells) for _ in range(dim))
    field = field[sl]
    lo, hi = field.min(), field.max()
    scale = (cmax - cmin) / (hi - lo) if hi > lo else 0.0  # a single cell: cmax below
    out = cmin + (field - lo) * scale
    out[np.unravel_index(np.argmin(field), field.shape)] = cmin
    out[np.unravel_index(np.argmax(field), field.shape)] = cmax
    return np.ascontiguousarray(out)


def constant_wavenumber(n_cells: int, dim: int, k: float) -> np.ndarray:
    return np.full((n_cells,) * dim, float(k))


def wavenumber_from_speed(speed: np.ndarray, wavelengths: float,
                          cmin: float | None = None) -> np.ndarray:
    """k = omega / c with omega chosen so the slowest speed has `wavelengths`
    wavelengths across the unit domain."""
    c0 = float(speed.min()) if cmin is None else float(cmin)
    omega = 2.0 * math.pi * wavelengths * c0
    return omega / speed


def absorbing_layer_eps(k: np.ndarray, p: int, sides, dofs: float = 40.0) -> np.ndarray:
    """Per-cell eps of absorbing layers along the sides flagged in `sides`
    (2*dim booleans, x-, x+, y-, y+, z-, z+) for the per-cell wavenumber k
    (indexed [z][y][x]).  Layer width L = dofs / p cells; a cell whose centre
    lies at distance d < L from a flagged side gets
    (2 k^2 / pi) sin^2(pi (L - d) / (2 L)); where layers meet, the larger."""
    k = np.asarray(k, dtype=np.float64)
    dim, N = k.ndim, k.shape[0]
    L = dofs / p
    centre = np.arange(N) + 0.5
    ramp = np.zeros((N,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[dim - 1 - a] = N  # axis a = x is the last array axis
        for hi in (0, 1):
            if not sides[2 * a + hi]:
                continue
            d = (N - centre) if hi else centre
            s = np.clip((L - d) / L, 0.0, 1.0).reshape(shape)
            ramp = np.maximum(ramp, np.sin(0.5 * math.pi * s) ** 2)
    return np.ascontiguousarray(2.0 * k * k / math.pi * ramp)


def gaussian_centres_grid(m: int, dim: int = 2) -> np.ndarray:
    """m^dim centres ((i+1/2)/m, ...) ordered x fastest."""
    c = (np.arange(m) + 0.5) / m
    grids = np.meshgrid(*([c] * dim), indexing="ij")
    # x fastest: last axis is slowest in the product order below
    pts = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    return pts


def gaussian_load(n_cells: int, p: int, centres, sigma: float,
                  dim: int = 2) -> np.ndarray:
    """Load vectors (R, (pN+1)^dim) for Gaussian sources by GLL quadrature."""
    centres = np.atleast_2d(np.asarray(centres, dtype=np.float64))
    h = 1.0 / n_cells
    xg, wg = gll_points(p)
    n1 = p * n_cells + 1
    # node coordinates and accumulated 1-D quadrature weights on the global grid
    coord = np.empty(n1)
    wsum = np.zeros(n1)
    for c in range(n_cells):
        coord[c * p: c * p + p + 1] = (c + xg) * h
        wsum[c * p: c * p + p + 1] += wg * h
    out = np.zeros((centres.shape[0], n1 ** dim), dtype=np.complex128)
    for r, x0 in enumerate(centres):
        g1 = [np.exp(-((coord - x0[d]) ** 2) / (2.0 * sigma * sigma)) for d in range(dim)]
        val = np.ones((1,))
        for d in reversed(range(dim)):  # slowest axis first -> x fastest
            val = np.multiply.outer(val, g1[d] * wsum)
        out[r] = val.ravel()
    return out


def mlp_samples(n: int, seed: int = 1, orders=(2, 4, 6, 8), eta_min: float = 0.3,
                eta_max: float = 2.1, shift_max: float = 0.05) -> np.ndarray:
    """Training inputs of the coarse-stencil surrogate: rows (eta_c, p, shift)
    with p uniform over `orders`, eta_c uniform on [eta_min, min(eta_max,
    0.95 * 2 pi / p)] (fine k h below 0.95 pi) and shift uniform on
    [0, shift_max]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.choice(np.asarray(orders, dtype=np.float64), size=n)
    hi = np.minimum(eta_max, 0.95 * 2.0 * math.pi / p)
    eta = eta_min + (hi - eta_min) * rng.random(n)
    shift = shift_max * rng.random(n)
    return np.ascontiguousarray(np.stack([eta, p, shift], axis=1))


def mlp_init(seed: int = 2, n_in: int = 3, width: int = 64, n_out: int = 2) -> np.ndarray:
    """Initial weights (float32, layout W1, b1, W2, b2, W3, b3): normal with
    standard deviation sqrt(1 / fan_in) for the matrices, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in [(n_in, width), (width, width), (width, n_out)]:
        parts.append(rng.standard_normal(fan_out * fan_in) * math.sqrt(1.0 / fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def random_complex(shape, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def config(name: str) -> dict:
    """Problem definitions of the five reference workloads.

    C1: 2-D Q2, 64x64 cells, constant k for 10 DOF/wavelength, Robin, one
        Gaussian (sigma = 2h) at the centre, alpha_s = 0.5, 8x8-cell
        subdomains, complex128, 1 RHS.
    C2: 2-D Q4, 200x200 cells, GRF speed (l = 0.05, [1.5, 4]) with 80
        wavelengths at the slowest speed, 16x16-cell subdomains.
    C3: C1 with 64 sources on a uniform 8x8 grid, mixed precision.
    C4: 3-D Q2, 75^3 cells, GRF (l = 0.1), 15 wavelengths, 8^3 subdomains,
        8 sources at {1/4, 3/4}^3.
    C5: 2-D Q4 64x64, GRF (l = 0.05), 10 DOF/wavelength at c_min.
    """
    name = name.upper()
    if name == "C1":
        n, p = 64, 2
        k = 2.0 * math.pi * 12.8
        return dict(name="C1", dim=2, n=n, p=p, k=constant_wavenumber(n, 2, k),
                    centres=np.array([[0.5, 0.5]]), sigma=2.0 / n, alpha_s=0.5,
                    l_dd=8, dtype="c128")
    if name == "C2":
        n, p = 200, 4
        c = grf_speed(n, 2, 0.05, 1.5, 4.0, seed=0)
        return dict(name="C2", dim=2, n=n, p=p, k=wavenumber_from_speed(c, 80.0),
                    centres=np.array([[0.5, 0.5]]), sigma=2.0 / n, alpha_s=0.5,
                    l_dd=16, dtype="c128")
    if name == "C3":
        d = config("C1")
        d.update(name="C3", centres=gaussian_centres_grid(8, 2), dtype="mixed")
        return d
    if name == "C4":
        n, p = 75, 2
        c = grf_speed(n, 3, 0.1, 1.5, 4.0, seed=0)
        return dict(name="C4", dim=3, n=n, p=p, k=wavenumber_from_speed(c, 15.0),
                    centres=gaussian_centres_grid(2, 3), sigma=2.0 / n, alpha_s=0.5,
                    l_dd=8, dtype="mixed")
    if name == "C5":
        n, p = 64, 4
        c = grf_speed(n, 2, 0.05, 1.5, 4.0, seed=0)
        # 10 DOF per wavelength at c_min: pN / W = 10
        return dict(name="C5", dim=2, n=n, p=p, k=wavenumber_from_speed(c, p * n / 10.0),
                    centres=np.array([[0.5, 0.5]]), sigma=2.0 / n, alpha_s=0.5,
                    l_dd=8, dtype="c128")
    raise KeyError(name)
