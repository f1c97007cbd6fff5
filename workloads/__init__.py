"""Seeded synthetic inputs shared by the oracle, the GPU tests and the bench.

This module generates geometry and random inputs only: icosphere meshes,
the RWG edge table (topology), seeded rotations, incidence directions,
polarisations and test vectors, plus the workload recipes (sizes and pulse
numbers) of the sphere benchmarks.  It holds none of the method's
arithmetic (no basis functions, kernels, quadrature, grids or solvers), so
both the CPU oracle and the HIP library can consume its arrays without
sharing any computation.

Seed streams (numpy ``default_rng([seed, stream])``):
  1 rotation, 2 incidence directions, 3 polarisation angles,
  4 far-field directions, 5 composite geometry, 6 test vectors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C0 = 299_792_458.0

# ---------------------------------------------------------------- meshes

_PHI = (1.0 + math.sqrt(5.0)) / 2.0
_ICO_V = [(-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
          (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
          (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1)]
_ICO_F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
          (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
          (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
          (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]


def icosphere(level: int, radius: float = 1.0, rotation: np.ndarray | None = None):
    """Level-``level`` icosphere: the regular icosahedron, midpoint-subdivided
    ``level`` times, vertices projected onto the sphere of ``radius``.

    Returns (xyz float64 [nv,3], tri int32 [nt,3]) with counter-clockwise
    (outward-normal) vertex order.  Level 2 gives 320 triangles / 480 edges,
    level 4 gives 5120 triangles / 7680 edges.
    """
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in _ICO_V]
    faces = list(_ICO_F)
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    xyz = np.array(v) * radius
    tri = np.array(faces, dtype=np.int32)
    # orient every face outward (normal along the centroid direction)
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = np.einsum("ij,ij->i", nrm, p0 + p1 + p2) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    if rotation is not None:
        xyz = xyz @ np.asarray(rotation, dtype=np.float64).T
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tri)


def rwg_table(tri: np.ndarray) -> np.ndarray:
    """RWG edge table int32 [ns,4] = {t_plus, t_minus, edge_v0, edge_v1}.

    One row per edge shared by exactly two triangles, ordered by (v0, v1)
    with v0 < v1.  T+ is the triangle whose counter-clockwise boundary runs
    v0 -> v1, T- the one that runs v1 -> v0, so the basis current flows from
    T+ across the edge into T-.  Raises if the mesh is not a closed,
    consistently oriented 2-manifold.
    """
    owner: dict[tuple[int, int], int] = {}
    for t, (a, b, c) in enumerate(np.asarray(tri)):
        for p, q in ((a, b), (b, c), (c, a)):
            key = (int(p), int(q))
            if key in owner:
                raise ValueError(f"directed edge {key} used twice: inconsistent orientation")
            owner[key] = t
    rows = []
    for (p, q), t in owner.items():
        if p < q:
            if (q, p) not in owner:
                raise ValueError(f"edge ({p},{q}) has one triangle: open surface")
            rows.append((t, owner[(q, p)], p, q))
    rows.sort(key=lambda r: (r[2], r[3]))
    return np.array(rows, dtype=np.int32).reshape(-1, 4)


# ---------------------------------------------------------------- seeds

def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def random_rotation(seed: int) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion (stream 1)."""
    q = rng(seed, 1).standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def unit_vectors(seed: int, stream: int, n: int) -> np.ndarray:
    """n directions uniform on the sphere (normalised Gaussian 3-vectors)."""
    d = rng(seed, stream).standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def polarisations(seed: int, khat: np.ndarray) -> np.ndarray:
    """Random polarisation orthogonal to each k-hat (stream 3):
    p = cos(psi) e1 + sin(psi) e2, psi ~ U[0, 2pi), e1 = normalise(k x z)
    (x if k is parallel to z), e2 = k x e1."""
    khat = np.atleast_2d(khat)
    psi = rng(seed, 3).uniform(0.0, 2.0 * math.pi, len(khat))
    out = np.empty_like(khat)
    for i, k in enumerate(khat):
        e1 = np.cross(k, [0.0, 0.0, 1.0])
        if np.linalg.norm(e1) < 1e-12:
            e1 = np.array([1.0, 0.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(k, e1)
        out[i] = math.cos(psi[i]) * e1 + math.sin(psi[i]) * e2
    return out


def complex_normal(seed: int, shape, stream: int = 6) -> np.ndarray:
    """i.i.d. CN(0,1) test vectors (stream 6)."""
    g = rng(seed, stream)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / math.sqrt(2.0)


# ---------------------------------------------------------------- recipes

@dataclass
class Workload:
    """One synthetic benchmark problem (a sphere meshed as an icosphere)."""
    name: str
    level: int
    radius: float
    f0: float            # centre frequency [Hz]
    frac_bw: float       # half-bandwidth as a fraction of f0 (0.2 for +-20 %)
    nt: int              # time steps
    grid: int            # auxiliary grid nodes per axis (padded FFT length 2*grid)
    near_lambda: float   # near-zone distance in centre wavelengths
    ng: int = 0          # history depth, 0 = derive from beta
    beta: float = 0.2    # dt = beta / f_bw when ng == 0
    batch: int = 1
    rotate_seed: int | None = None
    dir_seed: int | None = None
    khat: tuple = (0.0, 0.0, -1.0)
    phat: tuple = (1.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)

    @property
    def f_bw(self) -> float:
        return self.frac_bw * self.f0

    @property
    def sigma(self) -> float:
        # the pulse band is f_c +- 3/(2 pi sigma); the band edge is f0*(1+frac)
        return 3.0 / (2.0 * math.pi * self.f_bw)

    @property
    def td(self) -> float:
        return 8.0 * self.sigma

    def mesh(self):
        rot = random_rotation(self.rotate_seed) if self.rotate_seed is not None else None
        xyz, tri = icosphere(self.level, self.radius, rot)
        return xyz, tri, rwg_table(tri)

    def incidence(self):
        """(khat [B,3], phat [B,3])."""
        if self.batch == 1 and self.dir_seed is None:
            return (np.array([self.khat], dtype=np.float64),
                    np.array([self.phat], dtype=np.float64))
        k = unit_vectors(self.dir_seed, 2, self.batch)
        return k, polarisations(self.dir_seed, k)


SPHERE_L2 = Workload("sphere_L2_r0.5_300MHz", level=2, radius=0.5, f0=300e6, frac_bw=0.20,
                     nt=200, grid=16, near_lambda=0.3, beta=0.2)
SPHERE_L4 = Workload("sphere_L4_r1_600MHz", level=4, radius=1.0, f0=600e6, frac_bw=0.30,
                     nt=500, grid=48, near_lambda=0.3, ng=24, rotate_seed=0)
SPHERE_L4_BATCH = Workload("sphere_L4_r1_600MHz_32dir", level=4, radius=1.0, f0=600e6,
                           frac_bw=0.10, nt=400, grid=48, near_lambda=0.3, ng=24,
                           rotate_seed=0, batch=32, dir_seed=0)
SPHERE_L4_ADJ = Workload("sphere_L4_r1_600MHz_adjoint", level=4, radius=1.0, f0=600e6,
                         frac_bw=0.30, nt=300, grid=48, near_lambda=0.3, ng=24, rotate_seed=0)
# mid-size parity case: level-3 sphere, 1920 RWG, several FFT tiles and ragged lines
SPHERE_L3 = Workload("sphere_L3_r1_300MHz", level=3, radius=1.0, f0=300e6, frac_bw=0.20,
                     nt=40, grid=18, near_lambda=0.2, ng=6, rotate_seed=3)

# narrow-band (+-1 %, chi ~ 101) variant of the level-2 sphere: the regime in
# which CPPIF envelope marching is stable, used for full-march parity
SPHERE_L2_NARROW = Workload("sphere_L2_r0.5_300MHz_narrow", level=2, radius=0.5, f0=300e6, frac_bw=0.01,
                            nt=60, grid=16, near_lambda=0.3, beta=0.2)

WORKLOADS = {w.name: w for w in (SPHERE_L2, SPHERE_L4, SPHERE_L4_BATCH, SPHERE_L4_ADJ, SPHERE_L3,
                                 SPHERE_L2_NARROW)}
