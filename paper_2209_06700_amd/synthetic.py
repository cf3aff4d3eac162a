"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the method's arithmetic: it evaluates a smooth
random field at given node coordinates and draws seeded random vectors.
Recipe of the smooth data (the "sum of 16 seeded Fourier modes, amplitudes
N(0,1)/k^2" workload): u(x,y,z) = sum_m a_m prod_d sin(kappa_{m,d} pi x_d) with
kappa_{m,d} uniform in {1..kmax} and a_m ~ N(0,1) / |kappa_m|^2, drawn from
numpy.random.default_rng(seed).
"""
from __future__ import annotations

import numpy as np


def grid_coords(ref_nodes, n_cells: int) -> np.ndarray:
    """1D node coordinates of a uniform n-cell partition of [0,1] whose cells
    carry the given reference nodes on [0,1] (shared end points once)."""
    ref = np.asarray(ref_nodes, dtype=float)
    k = ref.size - 1
    x = np.empty(n_cells * k + 1)
    for e in range(n_cells):
        x[e * k:(e + 1) * k + 1] = (e + ref) / n_cells
    return x


def fourier_modes(seed: int, n_modes: int = 16, kmax: int = 8):
    rng = np.random.default_rng(seed)
    kappa = rng.integers(1, kmax + 1, size=(n_modes, 3))
    amp = rng.standard_normal(n_modes) / np.sum(kappa ** 2, axis=1)
    return kappa, amp


def fourier_field(x1d: np.ndarray, seed: int, n_modes: int = 16, kmax: int = 8) -> np.ndarray:
    """The smooth random field at the tensor grid x1d^3, flattened x fastest,
    with the boundary nodes set to exactly zero."""
    kappa, amp = fourier_modes(seed, n_modes, kmax)
    N = x1d.size
    out = np.zeros((N, N, N))
    for (kx, ky, kz), a in zip(kappa, amp):
        sx, sy, sz = (np.sin(kk * np.pi * x1d) for kk in (kx, ky, kz))
        out += a * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    out[0] = out[-1] = 0.0
    out[:, 0] = out[:, -1] = 0.0
    out[:, :, 0] = out[:, :, -1] = 0.0
    return out.reshape(-1)


def random_vector(shape, seed: int, zero_boundary_N: int | None = None) -> np.ndarray:
    """Standard-normal values; if zero_boundary_N is given the trailing
    N^3 grid of every leading index gets a zero boundary."""
    v = np.random.default_rng(seed).standard_normal(shape)
    if zero_boundary_N is not None:
        N = zero_boundary_N
        g = v.reshape(-1, N, N, N)
        g[:, 0] = g[:, -1] = 0.0
        g[:, :, 0] = g[:, :, -1] = 0.0
        g[:, :, :, 0] = g[:, :, :, -1] = 0.0
    return v
