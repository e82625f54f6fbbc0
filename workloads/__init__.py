"""Seeded synthetic inputs for the nodal-hexahedral H-field scattering solver.

This module only *describes* problems: a structured box mesh, per-element
relative permittivity/permeability, a per-element PEC mask, outer-face tags,
the free-space wavenumber and incident plane waves.  It contains none of the
finite element arithmetic, so both the CPU oracle's callers and the GPU
binding's callers can draw identical inputs from it without sharing any of
the method's code.

Geometry rules (staircased scatterers, element-centroid tests) and the
random draws follow the problem statement of the paper's section 2 (a
scatterer in a box truncated by an absorbing boundary, lit by a plane wave)
and its size statement in section 1 (10 nodes per wavelength).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

FACE_ABC = 0       # outer box face carries the absorbing boundary condition
FACE_NATURAL = 1   # outer box face left with the natural condition (no surface term)
FACE_SYM = 2       # symmetry plane, n . H = 0 (section 3.1.3, eq. (6a))
FACE_ANTISYM = 3   # antisymmetry plane, n x H = 0 (section 3.1.3, eq. (6b))

# Outer face order: -x, +x, -y, +y, -z, +z.
FACE_NAMES = ("-x", "+x", "-y", "+y", "-z", "+z")


@dataclasses.dataclass
class PlaneWave:
    """Incident field H_i(r) = p * exp(-j k0 d.r); |d| = 1 and p.d = 0."""
    d: np.ndarray          # (3,) float64
    p: np.ndarray          # (3,) complex128


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    h: Tuple[float, float, float]
    origin: Tuple[float, float, float]
    eps_r: np.ndarray      # (nz, ny, nx) complex128, x fastest in memory
    mu_r: np.ndarray       # (nz, ny, nx) complex128
    pec: np.ndarray        # (nz, ny, nx) uint8, 1 = element removed (perfect conductor)
    faces: Tuple[int, ...]  # 6 face tags (FACE_ABC / FACE_NATURAL / FACE_SYM / FACE_ANTISYM)
    k0: float
    penalty_s: float = 1.0
    name: str = ""

    @property
    def n_elements(self) -> int:
        return self.nx * self.ny * self.nz

    def grid_nodes(self) -> Tuple[int, int, int]:
        return (self.nz + 1, self.ny + 1, self.nx + 1)


def unit(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def random_wave(rng: np.random.Generator) -> PlaneWave:
    """Direction uniform on the sphere; linear polarisation at a uniform angle
    in the plane orthogonal to the direction."""
    d = unit(rng.standard_normal(3))
    # orthonormal pair (e1, e2) spanning the plane orthogonal to d
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = unit(a - d * np.dot(a, d))
    e2 = np.cross(d, e1)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    p = (math.cos(phi) * e1 + math.sin(phi) * e2).astype(np.complex128)
    return PlaneWave(d=d, p=p)


def element_centroids(nx, ny, nz, h, origin):
    """Centroid coordinates of every element as three (nz, ny, nx) arrays."""
    cx = origin[0] + (np.arange(nx) + 0.5) * h[0]
    cy = origin[1] + (np.arange(ny) + 0.5) * h[1]
    cz = origin[2] + (np.arange(nz) + 0.5) * h[2]
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    return X, Y, Z


def _blank(nx, ny, nz, h, origin, k0, faces=(FACE_ABC,) * 6, name=""):
    shape = (nz, ny, nx)
    return Problem(nx=nx, ny=ny, nz=nz, h=tuple(map(float, h)), origin=tuple(map(float, origin)),
                   eps_r=np.ones(shape, np.complex128), mu_r=np.ones(shape, np.complex128),
                   pec=np.zeros(shape, np.uint8), faces=tuple(faces), k0=float(k0), name=name)


def sphere_mask(p: Problem, center, radius) -> np.ndarray:
    """Staircased ball: an element belongs to it when its centroid lies within
    `radius` of `center` (ties included)."""
    X, Y, Z = element_centroids(p.nx, p.ny, p.nz, p.h, p.origin)
    r = np.sqrt((X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2)
    return r <= radius * (1.0 + 1e-12)


def box_mask(p: Problem, lo, hi) -> np.ndarray:
    """Staircased axis-aligned box: centroid inside [lo, hi] per axis."""
    X, Y, Z = element_centroids(p.nx, p.ny, p.nz, p.h, p.origin)
    return ((X >= lo[0]) & (X <= hi[0]) & (Y >= lo[1]) & (Y <= hi[1])
            & (Z >= lo[2]) & (Z <= hi[2]))


# --------------------------------------------------------------------------
# The five workloads.  Wavelength 1, so k0 = 2*pi and 10 nodes per wavelength
# means h = 0.1 unless stated otherwise.
# --------------------------------------------------------------------------

def free_cube(n: int = 10, wavelengths: float = 1.0) -> Tuple[Problem, List[PlaneWave]]:
    """Free-space cube, ABC on all faces, x-polarised wave travelling along +z."""
    h = wavelengths / n
    p = _blank(n, n, n, (h, h, h), (0.0, 0.0, 0.0), 2.0 * math.pi, name=f"free_cube_{n}")
    w = PlaneWave(d=np.array([0.0, 0.0, 1.0]), p=np.array([1.0, 0.0, 0.0], np.complex128))
    return p, [w]


def pec_cube(n: int = 30, seed: int = 43) -> Tuple[Problem, List[PlaneWave]]:
    """3-wavelength cube at 10 nodes per wavelength with a centred PEC cube of
    side one wavelength; one wave of seeded random direction/polarisation."""
    rng = np.random.default_rng(seed)
    h = 0.1
    p = _blank(n, n, n, (h, h, h), (0.0, 0.0, 0.0), 2.0 * math.pi, name=f"pec_cube_{n}")
    L = n * h
    side = 1.0
    lo = (L - side) / 2.0
    p.pec[box_mask(p, (lo,) * 3, (lo + side,) * 3)] = 1
    return p, [random_wave(rng)]


def pec_sphere_shell(n: int = 60, radius: float = 1.5, shell: float = 0.3,
                     seed: int = 44, nrhs: int = 1) -> Tuple[Problem, List[PlaneWave]]:
    """PEC sphere (staircased) centred in an n^3 box with h = 0.1 wavelength,
    wrapped in a dielectric shell radius < r <= radius + shell whose elements
    draw eps_r ~ U[2, 4] independently; mu_r = 1."""
    rng = np.random.default_rng(seed)
    h = 0.1
    L = n * h
    p = _blank(n, n, n, (h, h, h), (0.0, 0.0, 0.0), 2.0 * math.pi, name=f"pec_sphere_shell_{n}")
    c = (L / 2.0,) * 3
    ball = sphere_mask(p, c, radius)
    p.pec[ball] = 1
    if shell > 0:
        outer = sphere_mask(p, c, radius + shell) & ~ball
        p.eps_r[outer] = rng.uniform(2.0, 4.0, size=int(outer.sum()))
    waves = [random_wave(rng) for _ in range(nrhs)]
    return p, waves


def pec_sphere_batched(n: int = 40, radius: float = 1.0, nrhs: int = 64,
                       seed: int = 45) -> Tuple[Problem, List[PlaneWave]]:
    """PEC sphere of radius one wavelength centred in an n^3 box (h = 0.1),
    lit by `nrhs` waves with directions uniform on the sphere."""
    rng = np.random.default_rng(seed)
    h = 0.1
    L = n * h
    p = _blank(n, n, n, (h, h, h), (0.0, 0.0, 0.0), 2.0 * math.pi, name=f"pec_sphere_{n}_b{nrhs}")
    p.pec[sphere_mask(p, (L / 2.0,) * 3, radius)] = 1
    return p, [random_wave(rng) for _ in range(nrhs)]


@dataclasses.dataclass
class Request:
    arrival_s: float
    problem: Problem
    waves: List[PlaneWave]


def mirrored_pec_cube(n: int = 12, side: float = 0.4, cut_x: bool = False,
                      cut_y: bool = False) -> Tuple[Problem, List[PlaneWave]]:
    """Box of n^3 elements (n even, h = 0.1) centred on the origin around a
    centred PEC cube of the given side, ABC on the outer faces, lit by the
    x-polarised wave travelling along +z.  The problem is mirror-symmetric in
    x and in y, and so is this incident field: H is even under x -> -x
    (H_x even, H_y and H_z odd), so n x H = 0 on the plane x = 0, and odd
    under y -> -y (H_y odd), so n . H = 0 on y = 0.  cut_x keeps the half
    x >= 0 with its -x face tagged FACE_ANTISYM; cut_y keeps y >= 0 with its
    -y face tagged FACE_SYM.  The cut problem's nodal solution equals the
    whole box's restricted to the kept part."""
    if n % 2:
        raise ValueError("n must be even")
    h = 0.1
    half = n // 2
    full = _blank(n, n, n, (h, h, h), (-half * h, -half * h, -half * h), 2.0 * math.pi,
                  name=f"mirrored_pec_cube_{n}")
    s = side / 2.0
    full.pec = box_mask(full, (-s, -s, -s), (s, s, s)).astype(np.uint8)
    x0 = half if cut_x else 0
    y0 = half if cut_y else 0
    faces = list(full.faces)
    if cut_x:
        faces[0] = FACE_ANTISYM
    if cut_y:
        faces[2] = FACE_SYM
    p = dataclasses.replace(
        full, nx=n - x0, ny=n - y0,
        origin=(full.origin[0] + x0 * h, full.origin[1] + y0 * h, full.origin[2]),
        eps_r=np.ascontiguousarray(full.eps_r[:, y0:, x0:]), mu_r=np.ascontiguousarray(full.mu_r[:, y0:, x0:]),
        pec=np.ascontiguousarray(full.pec[:, y0:, x0:]), faces=tuple(faces),
        name=full.name + ("_x" if cut_x else "") + ("_y" if cut_y else ""))
    w = PlaneWave(d=np.array([0.0, 0.0, 1.0]), p=np.array([1.0, 0.0, 0.0], np.complex128))
    return p, [w]


def serving_request(rng: np.random.Generator, n_lo: int = 10, n_hi: int = 100,
                    nrhs_hi: int = 16) -> Tuple[Problem, List[PlaneWave]]:
    """One scattering request: n^3 mesh, n ~ U{n_lo..n_hi}; k0 ~ U[pi, 4 pi]
    with h = 0.1 * (2 pi / k0); a PEC box (side U[0.2, 0.5] L) or sphere
    (radius U[0.1, 0.3] L) centred at a random point of the middle 40 % of the
    box; 1..nrhs_hi random plane waves."""
    n = int(rng.integers(n_lo, n_hi + 1))
    k0 = float(rng.uniform(math.pi, 4.0 * math.pi))
    h = 0.1 * (2.0 * math.pi / k0)
    p = _blank(n, n, n, (h, h, h), (0.0, 0.0, 0.0), k0, name=f"req_n{n}")
    L = n * h
    c = L * (0.3 + 0.4 * rng.random(3))
    if rng.random() < 0.5:
        side = float(rng.uniform(0.2, 0.5)) * L
        p.pec[box_mask(p, c - side / 2, c + side / 2)] = 1
    else:
        rad = float(rng.uniform(0.1, 0.3)) * L
        p.pec[sphere_mask(p, c, rad)] = 1
    nrhs = int(rng.integers(1, nrhs_hi + 1))
    return p, [random_wave(rng) for _ in range(nrhs)]


def serving_stream(n_requests: int = 2000, rate_per_s: float = 10.0, seed: int = 46,
                   n_lo: int = 10, n_hi: int = 100, nrhs_hi: int = 16) -> List[Request]:
    """Poisson arrivals at `rate_per_s` of independent serving requests."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        prob, waves = serving_request(rng, n_lo, n_hi, nrhs_hi)
        out.append(Request(arrival_s=t, problem=prob, waves=waves))
    return out


def random_small(rng: np.random.Generator, n: Sequence[int] = (3, 3, 3),
                 n_pec: int = 1, eps_range=(1.0, 4.0), lossy: bool = False,
                 k0: float = 2.0 * math.pi, h=(0.1, 0.1, 0.1),
                 faces=(FACE_ABC,) * 6) -> Problem:
    """Tiny random problem for brute-force agreement tests: random eps per
    element (optionally lossy), `n_pec` random PEC elements."""
    nx, ny, nz = n
    p = _blank(nx, ny, nz, h, (0.0, 0.0, 0.0), k0, faces=faces, name=f"rand_{nx}x{ny}x{nz}")
    p.eps_r[:] = rng.uniform(*eps_range, size=(nz, ny, nx))
    if lossy:
        p.eps_r -= 1j * rng.uniform(0.0, 0.5, size=(nz, ny, nx))
    if n_pec:
        idx = rng.choice(nx * ny * nz, size=n_pec, replace=False)
        p.pec.reshape(-1)[idx] = 1
    return p


# The workloads by name, for the bench and the tests.
WORKLOADS = {
    "free_cube_10": lambda: free_cube(10),
    "pec_cube_30": lambda: pec_cube(30),
    "pec_sphere_shell_60": lambda: pec_sphere_shell(60),
    "pec_sphere_40_b64": lambda: pec_sphere_batched(40),
}
