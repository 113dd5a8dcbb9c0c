"""Seeded synthetic inputs for the ES-BGK stream-collide workloads.

This module only draws macroscopic fields (density, velocity, temperature)
and per-domain parameters from fixed recipes and seeds.  It holds none of the
scheme's arithmetic, so both the GPU library's tests and the FP64 oracle can
consume the same host arrays.

Field arrays follow one convention everywhere: numpy shape (ny, nx) in 2D and
(nz, ny, nx) in 3D (x fastest in memory), velocity stacked as (D, ...).
All values are in the paper's dimensionless thermal units (rho0 = T0 = 1,
velocities in units of sqrt(R_g T0)).
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def _grid2(nx: int, ny: int):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y


def decay_2d(n: int = 32, amp_u: float = 1e-3, amp_T: float = 1e-3):
    """Plain-method decay case: rho = 1, T = 1 + amp_T cos(2 pi x/n),
    u_x = amp_u sin(2 pi y/n), u_y = 0 on an n x n periodic grid."""
    x, y = _grid2(n, n)
    rho = np.ones((n, n))
    u = np.zeros((2, n, n))
    u[0] = amp_u * np.sin(TWO_PI * y / n)
    T = 1.0 + amp_T * np.cos(TWO_PI * x / n)
    return rho, u, T


def waves_noise_2d(n: int = 4096, seed: int = 1611, amp: float = 1e-3, sigma: float = 1e-5, short: int = 32):
    """Superposed shear and thermal waves plus seeded Gaussian noise:
    u_x = amp [sin(2 pi y/n) + sin(2 pi y/short)] + noise,
    u_y = noise, T = 1 + amp [cos(2 pi x/n) + cos(2 pi x/short)] + noise,
    rho = 1.  Noise is N(0, sigma^2), drawn with numpy PCG64(seed) as three
    planes in the order u_x, u_y, T (x fastest)."""
    x, y = _grid2(n, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((3, n, n)) * sigma
    rho = np.ones((n, n))
    u = np.empty((2, n, n))
    u[0] = amp * (np.sin(TWO_PI * y / n) + np.sin(TWO_PI * y / short)) + noise[0]
    u[1] = noise[1]
    T = 1.0 + amp * (np.cos(TWO_PI * x / n) + np.cos(TWO_PI * x / short)) + noise[2]
    return rho, u, T


def random_state(dims, seed: int, amp_rho: float = 0.05, amp_u: float = 0.05, amp_T: float = 0.05, modes: int = 3):
    """Strongly perturbed smooth state for parity tests: a few random Fourier
    modes per field (amplitudes amp_*), plus a small white-noise component.
    dims = (nx, ny) or (nx, ny, nz)."""
    D = len(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(reversed(dims))
    axes = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    coords = list(reversed(axes))           # coords[d] varies along dims[d]

    def field(amp):
        out = np.zeros(shape)
        for _ in range(modes):
            ph = rng.uniform(0, TWO_PI)
            arg = ph
            for d in range(D):
                k = rng.integers(-2, 3)
                arg = arg + TWO_PI * k * coords[d] / dims[d]
            out += rng.uniform(0.3, 1.0) * np.cos(arg)
        out *= amp / modes
        out += 0.1 * amp * rng.standard_normal(shape)
        return out

    rho = 1.0 + field(amp_rho)
    u = np.stack([field(amp_u) for _ in range(D)])
    T = 1.0 + field(amp_T)
    return rho, u, T


def taylor_green_3d(n: int = 256, u0: float = 0.02, amp_T: float = 1e-2):
    """Thermal Taylor-Green vortex on an n^3 periodic grid, X = 2 pi i / n:
    u = u0 (sin X cos Y cos Z, -cos X sin Y cos Z, 0),
    T = 1 + amp_T cos X cos Y cos Z, rho = 1."""
    ax = TWO_PI * np.arange(n, dtype=np.float64) / n
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    u = np.empty((3, n, n, n))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    T = 1.0 + amp_T * np.cos(X) * np.cos(Y) * np.cos(Z)
    rho = np.ones((n, n, n))
    return rho, u, T


def batch_domains(count: int = 256, seed: int = 2409, amp: float = 1e-3):
    """Independent periodic 2D domains: side lengths drawn independently
    from {64, 96, ..., 512}, Pr ~ U[0.5, 2.0], N_f in {0, 1, 3},
    tau ~ U[0.55, 1.2], and a shear plus thermal wave with random phases.
    Returns a list of dicts (nx, ny, Pr, Nf, tau, phases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = np.arange(64, 513, 32)
    out = []
    for _ in range(count):
        nx, ny = (int(v) for v in rng.choice(sides, size=2))
        Pr = float(rng.uniform(0.5, 2.0))
        Nf = int(rng.choice([0, 1, 3]))
        tau = float(rng.uniform(0.55, 1.2))
        ph = rng.uniform(0, TWO_PI, size=2)
        out.append(dict(nx=nx, ny=ny, Pr=Pr, Nf=Nf, tau=tau, phases=(float(ph[0]), float(ph[1])), amp=amp))
    return out


def batch_fields(dom: dict):
    """Fields of one batch domain: u_x = amp sin(2 pi y/ny + p0),
    T = 1 + amp cos(2 pi x/nx + p1), u_y = 0, rho = 1."""
    nx, ny, amp = dom["nx"], dom["ny"], dom["amp"]
    x, y = _grid2(nx, ny)
    rho = np.ones((ny, nx))
    u = np.zeros((2, ny, nx))
    u[0] = amp * np.sin(TWO_PI * y / ny + dom["phases"][0])
    T = 1.0 + amp * np.cos(TWO_PI * x / nx + dom["phases"][1])
    return rho, u, T


def block_mean(a: np.ndarray, out_n: int) -> np.ndarray:
    """Average a square 2D array over (n/out_n)^2 blocks."""
    n = a.shape[-1]
    b = n // out_n
    return a.reshape(a.shape[:-2] + (out_n, b, out_n, b)).mean(axis=(-3, -1))
