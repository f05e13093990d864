"""Seeded synthetic inputs for the two-component lattice-Boltzmann workloads.

This module only draws inputs: initial density fields, fixed sphere positions
and the solid mask they cover, a smooth target field for the gradient
objective, and sample sites.  It holds none of the lattice-Boltzmann
arithmetic, so both the CPU oracle and the GPU library can be fed from it
without sharing any part of the method.

Arrays are NumPy, C order ``[z][y][x]`` (x fastest), float64 unless stated.
The paper's own test boxes are synthetic too: periodic cubes at uniform
density, a two-component mix drawn at random per node, and randomly placed
spheres of radius 5.5 (Sec. 5, cases 1-3).
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "fluid_fields",
    "colour_fields",
    "particle_mass",
    "sphere_centres",
    "solid_mask",
    "smooth_target",
    "sample_sites",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named workload: lattice, storage, relaxation, coupling, noise, steps."""

    name: str
    shape: Tuple[int, int, int]          # (nz, ny, nx)
    storage: str                         # "f64" | "f32" | "f16s"
    tau: Tuple[float, float]
    G: float
    rho0: Tuple[float, float]
    amp: float                           # half-width of the uniform density noise
    steps: int
    seed: int
    spheres: int = 0
    radius: float = 0.0
    sphere_seed: Optional[int] = None
    sigma: float = 0.0                   # colour-gradient workloads: surface tension
    beta: float = 0.0                    # colour-gradient workloads: recolouring parameter

    @property
    def nodes(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz


# The Shan-Chen workloads: a small box the oracle runs in seconds, the 256^3
# spinodal throughput box (FP64, then FP32 / FP16-shifted storage), the
# 128^3 gradient box, and the 512^3 box with 2000 fixed spheres; then the
# single-fluid and colour-gradient boxes of the paper's cases 1 and 2.
WORKLOADS = {
    "mix32_f64": Workload("mix32_f64", (32, 32, 32), "f64", (1.0, 1.0), 3.5, (1.0, 1.0), 0.01, 200, 1),
    "spinodal256_f64": Workload("spinodal256_f64", (256, 256, 256), "f64", (0.8, 0.8), 3.5, (1.0, 1.0), 0.02, 1000, 2),
    "spinodal256_f32": Workload("spinodal256_f32", (256, 256, 256), "f32", (0.8, 0.8), 3.5, (1.0, 1.0), 0.02, 1000, 2),
    "spinodal256_f16s": Workload("spinodal256_f16s", (256, 256, 256), "f16s", (0.8, 0.8), 3.5, (1.0, 1.0), 0.02, 1000, 2),
    "adjoint128_f32": Workload("adjoint128_f32", (128, 128, 128), "f32", (1.0, 1.0), 3.5, (1.0, 1.0), 0.02, 500, 3),
    # single fluid (the paper's case 1: one fluid, fused BGK step, periodic cube); G and the second
    # component are unused
    "case1_256_f32": Workload("case1_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (1.0, 1.0), 0.02, 1000, 8),
    "case1_256_f64": Workload("case1_256_f64", (256, 256, 256), "f64", (1.0, 1.0), 0.0, (1.0, 1.0), 0.02, 1000, 8),
    "spheres512_f32": Workload("spheres512_f32", (512, 512, 512), "f32", (1.0, 1.0), 3.5, (1.0, 1.0), 0.02, 500, 7,
                               spheres=2000, radius=5.5, sphere_seed=6),
    # two immiscible fluids, colour-gradient model (the paper's case 2: every node pure red or pure
    # blue at random, at rest, periodic cube); tau of both pure fluids, surface tension sigma and
    # recolouring beta are not given by the paper; G, rho0 and amp are unused
    # moving rigid spheres of radius 5.5 in the single fluid (the paper's case 3 fractions 0.1%, 1% and
    # 10% of a 256^3 box: 24, 241 and 2407 spheres); at rest, fluid 1 +- U(0.02)
    "case3a_256_f32": Workload("case3a_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (1.0, 1.0), 0.02, 500, 11,
                               spheres=24, radius=5.5, sphere_seed=12),
    "case3b_256_f32": Workload("case3b_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (1.0, 1.0), 0.02, 500, 11,
                               spheres=241, radius=5.5, sphere_seed=13),
    "case3c_256_f32": Workload("case3c_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (1.0, 1.0), 0.02, 500, 11,
                               spheres=2407, radius=5.5, sphere_seed=14),
    "case3c_256_f64": Workload("case3c_256_f64", (256, 256, 256), "f64", (1.0, 1.0), 0.0, (1.0, 1.0), 0.02, 500, 11,
                               spheres=2407, radius=5.5, sphere_seed=14),
    # the paper's case 3: moving rigid spheres of radius 5.5 in the two immiscible fluids of case 2 (every
    # node pure red or pure blue at random, at rest), 0.1%, 1% and 10% of a 256^3 box (the sphere positions
    # of the single-fluid workloads above); uncovered nodes start at rho0 = (1/2, 1/2)
    "case3cg_a_256_f32": Workload("case3cg_a_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (0.5, 0.5), 0.0,
                                  500, 10, spheres=24, radius=5.5, sphere_seed=12, sigma=0.01, beta=0.7),
    "case3cg_b_256_f32": Workload("case3cg_b_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (0.5, 0.5), 0.0,
                                  500, 10, spheres=241, radius=5.5, sphere_seed=13, sigma=0.01, beta=0.7),
    "case3cg_c_256_f32": Workload("case3cg_c_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (0.5, 0.5), 0.0,
                                  500, 10, spheres=2407, radius=5.5, sphere_seed=14, sigma=0.01, beta=0.7),
    "case3cg_c_256_f64": Workload("case3cg_c_256_f64", (256, 256, 256), "f64", (1.0, 1.0), 0.0, (0.5, 0.5), 0.0,
                                  500, 10, spheres=2407, radius=5.5, sphere_seed=14, sigma=0.01, beta=0.7),
    "case2_32_f64": Workload("case2_32_f64", (32, 32, 32), "f64", (1.0, 1.0), 0.0, (1.0, 1.0), 0.0, 200, 9,
                             sigma=0.01, beta=0.7),
    "case2_256_f32": Workload("case2_256_f32", (256, 256, 256), "f32", (1.0, 1.0), 0.0, (1.0, 1.0), 0.0, 1000, 10,
                              sigma=0.01, beta=0.7),
    "case2_256_f64": Workload("case2_256_f64", (256, 256, 256), "f64", (1.0, 1.0), 0.0, (1.0, 1.0), 0.0, 1000, 10,
                              sigma=0.01, beta=0.7),
}


def fluid_fields(shape, amp: float, seed: int, rho0=(1.0, 1.0)):
    """Initial densities rho_A, rho_B = rho0 + U[-amp, amp], independent per node.

    One ``numpy.random.default_rng(seed)`` stream, drawn in C order over
    ``shape`` = (nz, ny, nx): all of component A first, then all of B.
    """
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    a = rho0[0] + rng.uniform(-amp, amp, size=shape)
    b = rho0[1] + rng.uniform(-amp, amp, size=shape)
    return np.ascontiguousarray(a, dtype=np.float64), np.ascontiguousarray(b, dtype=np.float64)


def colour_fields(shape, seed: int):
    """Initial densities of the colour-gradient workloads: each node is pure
    red (rho_r = 1, rho_b = 0) or pure blue (0, 1) with probability 1/2.

    One ``numpy.random.default_rng(seed)`` stream, one uniform draw per node in
    C order over ``shape``; red where the draw is below 1/2.
    """
    rng = np.random.default_rng(seed)
    red = rng.random(tuple(int(s) for s in shape)) < 0.5
    r = np.where(red, 1.0, 0.0)
    return np.ascontiguousarray(r, dtype=np.float64), np.ascontiguousarray(1.0 - r, dtype=np.float64)


# Particle mass of the moving-sphere workloads: a sphere 2.2 times as dense as
# the fluid (silica in water, as the paper's particles), fluid density 1.
PARTICLE_DENSITY_RATIO = 2.2


def particle_mass(radius: float) -> float:
    return PARTICLE_DENSITY_RATIO * (4.0 / 3.0) * np.pi * radius ** 3


def _min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.round(d / box)


def sphere_centres(shape, count: int, radius: float, seed: int, min_sep: Optional[float] = None):
    """Real-valued sphere centres, uniform in the periodic box, non-overlapping.

    Rejection sampling: a candidate is kept only if its minimum-image distance
    to every kept centre exceeds ``min_sep`` (default 2 * radius).  Returns an
    array ``[count, 3]`` of (x, y, z).
    """
    nz, ny, nx = shape
    box = np.array([nx, ny, nz], dtype=np.float64)
    min_sep = 2.0 * radius if min_sep is None else float(min_sep)
    rng = np.random.default_rng(seed)
    kept = np.empty((0, 3), dtype=np.float64)
    tries = 0
    while kept.shape[0] < count:
        tries += 1
        if tries > 1000 * count + 1000:
            raise RuntimeError("sphere_centres: box too crowded for the requested count")
        c = rng.uniform(0.0, 1.0, size=3) * box
        if kept.shape[0]:
            d = _min_image(kept - c, box)
            if np.min(np.einsum("ij,ij->i", d, d)) <= min_sep * min_sep:
                continue
        kept = np.vstack([kept, c])
    return kept


def solid_mask(shape, centres, radius: float) -> np.ndarray:
    """uint8 mask ``[z][y][x]``: 1 where a node lies within ``radius`` of a centre.

    Distances are minimum-image on the periodic box; a node at distance
    exactly ``radius`` counts as solid.
    """
    nz, ny, nx = shape
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    r2 = radius * radius
    reach = int(np.ceil(radius)) + 1
    for cx, cy, cz in np.asarray(centres, dtype=np.float64):
        xs = np.arange(int(np.floor(cx)) - reach, int(np.floor(cx)) + reach + 2)
        ys = np.arange(int(np.floor(cy)) - reach, int(np.floor(cy)) + reach + 2)
        zs = np.arange(int(np.floor(cz)) - reach, int(np.floor(cz)) + reach + 2)
        dx = xs - cx
        dy = ys - cy
        dz = zs - cz
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        hit = d2 <= r2
        zi, yi, xi = np.nonzero(hit)
        mask[zs[zi] % nz, ys[yi] % ny, xs[xi] % nx] = 1
    return mask


def smooth_target(shape, seed: int, modes: int = 4, amp: float = 0.05, kmax: int = 2) -> np.ndarray:
    """Smooth periodic field 1 + sum of a few cosines, scaled so max|t - 1| = amp."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    acc = np.zeros(shape, dtype=np.float64)
    for _ in range(modes):
        k = rng.integers(-kmax, kmax + 1, size=3)
        while not np.any(k):
            k = rng.integers(-kmax, kmax + 1, size=3)
        a = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        acc += a * np.cos(2.0 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + phi)
    acc *= amp / np.max(np.abs(acc))
    return 1.0 + acc


def sample_sites(shape, count: int, seed: int, exclude: Optional[np.ndarray] = None) -> np.ndarray:
    """``count`` distinct node coordinates ``[count, 3]`` as (x, y, z), optionally avoiding a mask."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    out = []
    seen = set()
    while len(out) < count:
        x, y, z = int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))
        if (x, y, z) in seen:
            continue
        if exclude is not None and exclude[z, y, x]:
            continue
        seen.add((x, y, z))
        out.append((x, y, z))
    return np.array(out, dtype=np.int64)
