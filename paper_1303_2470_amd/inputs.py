"""Seeded synthetic inputs: geometries, sorption rates and driving forces.

This module only *builds inputs* (solid/fluid masks, rate pairs, body forces,
test velocity fields). It holds none of the moment-propagation arithmetic, so
the GPU path and the CPU oracle can both draw their inputs from it.

Array convention: a mask is a ``uint8`` array of shape ``(nz, ny, nx)``
(x fastest in memory), 1 = solid node, 0 = fluid node, matching the node
index ``n = x + nx*(y + ny*z)``.

Workload recipes follow the paper's validation set-ups (slit pores, Sec. III;
face-centred cubic packing, Sec. III and Fig. 4) and the synthetic porous
media of the benchmark configurations (Boolean overlapping spheres).
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- geometries
def slit_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Slit pore: solid planes at z = 0 and z = nz-1, periodic in x and y.

    The pore holds ``nz - 2`` fluid layers; with half-way walls that is the
    slit width L of the paper's exact results (Eqs. 13-15).
    """
    if nz < 3:
        raise ValueError("a slit needs at least one fluid layer")
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[0] = 1
    m[-1] = 1
    return m


def bulk_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Fully periodic box with no solid node."""
    return np.zeros((nz, ny, nx), dtype=np.uint8)


def random_mask(nx: int, ny: int, nz: int, solid_fraction: float, seed: int) -> np.ndarray:
    """I.i.d. solid nodes with the given probability (tiny brute-force lattices)."""
    rng = np.random.default_rng(seed)
    m = (rng.random((nz, ny, nx)) < solid_fraction).astype(np.uint8)
    if m.all():
        m.flat[0] = 0
    return m


def sphere_pack(n: int, radius: float, porosity: float, seed: int,
                shape: tuple[int, int, int] | None = None) -> np.ndarray:
    """Boolean overlapping spheres on a periodic lattice.

    Integer centres are drawn uniformly on the lattice from ``default_rng(seed)``;
    a node is solid when its periodic squared distance to a centre is at most
    ``radius**2``. Spheres are added one at a time until the fluid fraction
    drops to ``porosity`` or below. Isolated pores are kept.
    """
    nz, ny, nx = shape if shape is not None else (n, n, n)
    rng = np.random.default_rng(seed)
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    r = int(math.floor(radius))
    off = np.arange(-r, r + 1)
    dz, dy, dx = np.meshgrid(off, off, off, indexing="ij")
    inside = dz * dz + dy * dy + dx * dx <= radius * radius
    dz, dy, dx = dz[inside], dy[inside], dx[inside]
    total = m.size
    solid = 0
    while (total - solid) / total > porosity:
        cz, cy, cx = rng.integers(0, nz), rng.integers(0, ny), rng.integers(0, nx)
        zz = (cz + dz) % nz
        yy = (cy + dy) % ny
        xx = (cx + dx) % nx
        newly = m[zz, yy, xx] == 0
        solid += int(np.count_nonzero(newly))
        m[zz, yy, xx] = 1
    return m


def fcc_mask(a: int, radius: float | None = None) -> np.ndarray:
    """One periodic unit cell (a^3 nodes) of a face-centred cubic sphere packing.

    Spheres sit at the cube corners and face centres; with the default radius
    ``a / (2*sqrt(2))`` neighbouring spheres touch, the compact packing of the
    paper's porous-medium example (Fig. 4), whose continuum porosity is
    ``1 - pi/(3*sqrt(2))``. Node centres are at integer coordinates + 1/2.
    """
    if radius is None:
        radius = a / (2.0 * math.sqrt(2.0))
    c = np.arange(a) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    centres = [(0, 0, 0), (0, a / 2, a / 2), (a / 2, 0, a / 2), (a / 2, a / 2, 0)]
    m = np.zeros((a, a, a), dtype=np.uint8)
    for (cx, cy, cz) in centres:
        ddx = np.abs(x - cx)
        ddx = np.minimum(ddx, a - ddx)
        ddy = np.abs(y - cy)
        ddy = np.minimum(ddy, a - ddy)
        ddz = np.abs(z - cz)
        ddz = np.minimum(ddz, a - ddz)
        m |= (ddx * ddx + ddy * ddy + ddz * ddz <= radius * radius).astype(np.uint8)
    return m


# ---------------------------------------------------------------- rates, forces
def loguniform_rates(n: int, lo: float, hi: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """``n`` pairs (k_a, k_d), each log-uniform on [lo, hi], from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log10(lo), math.log10(hi), size=(n, 2))
    k = 10.0 ** u
    return np.ascontiguousarray(k[:, 0]), np.ascontiguousarray(k[:, 1])


def poiseuille_force(peclet: float, d_b: float, width: float, tau: float = 1.0) -> float:
    """Body-force acceleration that targets a mean slit velocity Pe*D_b/width.

    Plane Poiseuille flow between walls ``width`` apart has mean velocity
    g*width^2/(12*nu), with the BGK viscosity nu = (tau - 1/2)/3.
    """
    nu = (tau - 0.5) / 3.0
    vbar = peclet * d_b / width
    return 12.0 * nu * vbar / (width * width)


def random_velocity(mask: np.ndarray, umax: float, seed: int) -> np.ndarray:
    """Random velocity field ``(3, nz, ny, nx)``, zero on solid nodes.

    Exercises the velocity dependence of the link probabilities in tests; it
    need not satisfy any flow equation (the Eq. 11 start is then not
    stationary, which exercises the source term).
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(-umax, umax, size=(3,) + mask.shape)
    u[:, mask.astype(bool)] = 0.0
    return u

