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


def rwg_table(tri: np.ndarray, open_ok: bool = False) -> np.ndarray:
    """RWG edge table int32 [ns,4] = {t_plus, t_minus, edge_v0, edge_v1}.

    One row per edge shared by exactly two triangles, ordered by (v0, v1)
    with v0 < v1.  T+ is the triangle whose counter-clockwise boundary runs
    v0 -> v1, T- the one that runs v1 -> v0, so the basis current flows from
    T+ across the edge into T-.  Raises if the mesh is not a consistently
    oriented 2-manifold, and, unless open_ok (a plate: its boundary edges
    carry no basis), if it is not closed.
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
        if (q, p) not in owner:
            if open_ok:
                continue
            raise ValueError(f"edge ({p},{q}) has one triangle: open surface")
        if p < q:
            rows.append((t, owner[(q, p)], p, q))
    rows.sort(key=lambda r: (r[2], r[3]))
    return np.array(rows, dtype=np.int32).reshape(-1, 4)


def _merge(parts):
    """Concatenate meshes (xyz, tri) into one."""
    xyz, tri, off = [], [], 0
    for v, t in parts:
        xyz.append(v)
        tri.append(t + off)
        off += len(v)
    return np.concatenate(xyz), np.concatenate(tri).astype(np.int32)


def _orient_outward(xyz, tri, centre):
    """Flip triangles whose normal points towards the centre of their
    (convex) object."""
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = np.einsum("ij,ij->i", nrm, (p0 + p1 + p2) / 3.0 - centre) < 0
    tri = tri.copy()
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def plate_mesh(size: float, edge: float):
    """Square PEC plate of side `size` in the z = 0 plane, centred at the
    origin: n x n squares (n = ceil(size / edge)), each split along the same
    diagonal into two triangles, counter-clockwise about +z."""
    n = max(1, int(math.ceil(size / edge)))
    g = np.linspace(-size / 2, size / 2, n + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    vid = lambda i, j: j * (n + 1) + i  # noqa: E731
    tri = []
    for j in range(n):
        for i in range(n):
            q = (vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1))
            tri += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    return xyz, np.array(tri, dtype=np.int32)


def box_mesh(centre, size, edge):
    """Closed surface of an axis-aligned box: each face a structured grid of
    rectangles no longer than `edge` per side, each split into two
    triangles; vertices shared along the box edges."""
    centre, size = np.asarray(centre, float), np.asarray(size, float)
    n = np.maximum(1, np.ceil(size / edge).astype(int))
    index, xyz, tri = {}, [], []

    def vid(i, j, k):
        key = (i, j, k)
        if key not in index:
            index[key] = len(xyz)
            xyz.append(centre - size / 2 + size * np.array([i, j, k]) / n)
        return index[key]

    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in (0, n[a]):
            for u in range(n[b]):
                for v in range(n[c]):
                    q = []
                    for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        ijk = [0, 0, 0]
                        ijk[a], ijk[b], ijk[c] = side, u + du, v + dv
                        q.append(vid(*ijk))
                    tri += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    xyz = np.array(xyz)
    return xyz, _orient_outward(xyz, np.array(tri, dtype=np.int32), centre)


def _zip_rings(ia, ta, ib, tb):
    """Triangles between two closed rings of vertices (indices ia, ib at
    angles ta, tb, increasing), advancing along the ring whose next vertex
    comes first in angle."""
    na, nb = len(ia), len(ib)
    i = j = 0
    tri = []
    while i < na or j < nb:
        a0, b0 = ia[i % na], ib[j % nb]
        na_ang = ta[(i + 1) % na] + (2 * math.pi if i + 1 >= na else 0.0)
        nb_ang = tb[(j + 1) % nb] + (2 * math.pi if j + 1 >= nb else 0.0)
        if j >= nb or (i < na and na_ang <= nb_ang):
            tri.append((a0, ia[(i + 1) % na], b0))
            i += 1
        else:
            tri.append((a0, ib[(j + 1) % nb], b0))
            j += 1
    return tri


def cylinder_mesh(centre, radius, height, axis, edge):
    """Closed surface of a circular cylinder along coordinate `axis`: the
    side a structured grid (n_theta around, n_h along), each cap concentric
    rings zipped together down to a centre vertex; the caps' outer rings
    are the side's end rings."""
    centre = np.asarray(centre, float)
    nt = max(8, int(math.ceil(2 * math.pi * radius / edge)))
    nh = max(1, int(math.ceil(height / edge)))
    nr = max(1, int(math.ceil(radius / edge)))
    b, c = (axis + 1) % 3, (axis + 2) % 3
    xyz, tri = [], []

    def point(r, th, z):
        p = centre.copy()
        p[b] += r * math.cos(th)
        p[c] += r * math.sin(th)
        p[axis] += z
        return p

    ang = 2 * math.pi * np.arange(nt) / nt
    side = []
    for h in range(nh + 1):
        row = []
        for t in range(nt):
            row.append(len(xyz))
            xyz.append(point(radius, ang[t], -height / 2 + height * h / nh))
        side.append(row)
    for h in range(nh):
        for t in range(nt):
            q = (side[h][t], side[h][(t + 1) % nt], side[h + 1][(t + 1) % nt], side[h + 1][t])
            tri += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    for h, z in ((0, -height / 2), (nh, height / 2)):
        outer, oang = side[h], ang
        for k in range(nr - 1, 0, -1):
            rk = radius * k / nr
            n_k = max(3, int(math.ceil(2 * math.pi * rk / edge)))
            kang = 2 * math.pi * (np.arange(n_k) + 0.5 * (k % 2)) / n_k
            ring = []
            for t in range(n_k):
                ring.append(len(xyz))
                xyz.append(point(rk, kang[t], z))
            tri += _zip_rings(outer, oang, ring, kang)
            outer, oang = ring, kang
        ctr = len(xyz)
        xyz.append(point(0.0, 0.0, z))
        m = len(outer)
        tri += [(outer[t], outer[(t + 1) % m], ctr) for t in range(m)]
    xyz = np.array(xyz)
    tri = np.array(tri, dtype=np.int32)
    # orient each triangle outward: side triangles radially, cap triangles along the axis
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    cen = (p0 + p1 + p2) / 3.0 - centre
    out = cen.copy()
    cap = np.abs(np.abs(cen[:, axis]) - height / 2) < 1e-9
    out[~cap, axis] = 0.0
    out[cap] = 0.0
    out[cap, axis] = np.sign(cen[cap, axis])
    flip = np.einsum("ij,ij->i", nrm, out) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return xyz, tri


def composite(seed: int, n: int = 6, cube: float = 5.4, smin: float = 0.5, smax: float = 3.0,
              edge: float = 0.02855, gap_edges: float = 2.0):
    """Union of n seeded, disjoint, axis-aligned boxes and cylinders (stream
    5) inside a cube of side `cube` centred at the origin: kind (box or
    cylinder, even odds), sizes log-uniform in [smin, smax] (box sides;
    cylinder diameter and height), a random axis for a cylinder, the
    position uniform where the object fits; placements whose bounding boxes
    come closer than gap_edges edge lengths to an earlier object are drawn
    again.  Returns (xyz, tri) meshed at edge length `edge`."""
    g = rng(seed, 5)
    placed, parts = [], []
    while len(placed) < n:
        kind = "box" if g.uniform() < 0.5 else "cylinder"
        if kind == "box":
            size = np.exp(g.uniform(math.log(smin), math.log(smax), 3))
            axis = -1
        else:
            d, hgt = np.exp(g.uniform(math.log(smin), math.log(smax), 2))
            axis = int(g.integers(0, 3))
            size = np.full(3, d)
            size[axis] = hgt
        if np.any(size > cube):
            continue
        centre = g.uniform(-cube / 2 + size / 2, cube / 2 - size / 2)
        lo, hi = centre - size / 2, centre + size / 2
        gap = gap_edges * edge
        if any(np.all(lo < h2 + gap) and np.all(l2 < hi + gap) for l2, h2 in placed):
            continue
        placed.append((lo, hi))
        if kind == "box":
            parts.append(box_mesh(centre, size, edge))
        else:
            parts.append(cylinder_mesh(centre, size[(axis + 1) % 3] / 2, size[axis], axis, edge))
    return _merge(parts)


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
    """One synthetic benchmark problem: a sphere meshed as an icosphere
    (level, radius), or, with composite_seed set, the composite object of
    ``composite`` meshed at edge length lambda_min / 10, lambda_min the
    wavelength at the top of the pulse band f0 (1 + frac_bw)."""
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
    composite_seed: int | None = None
    plate_size: float | None = None   # a square plate of this side (metres) in z = 0
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

    @property
    def edge(self) -> float:
        if "edge" in self.extra:
            return self.extra["edge"]
        return C0 / (self.f0 * (1.0 + self.frac_bw)) / 10.0

    def mesh(self):
        if self.plate_size is not None:
            xyz, tri = plate_mesh(self.plate_size, self.edge)
            return xyz, tri, rwg_table(tri, open_ok=True)
        if self.composite_seed is not None:
            xyz, tri = composite(self.composite_seed, edge=self.edge)
            return xyz, tri, rwg_table(tri)
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

# composite object: six seeded boxes and cylinders of 0.5-3 m, edge
# lambda_min/10 = 2.86 cm, 200 634 RWG; 192^3 grid (h = 2.45 cm), N_g = 32
COMPOSITE = Workload("composite6_1GHz", level=0, radius=0.0, f0=1e9, frac_bw=0.05, nt=1000, grid=192,
                     near_lambda=0.25, ng=32, composite_seed=0)
# the same recipe at 250 MHz (edge 11.4 cm, 12 321 RWG, 48^3 grid): the
# composite parity case at a size the oracle finishes in seconds
COMPOSITE_SMALL = Workload("composite6_250MHz", level=0, radius=0.0, f0=250e6, frac_bw=0.05, nt=200, grid=48,
                           near_lambda=0.25, ng=32, composite_seed=0)

# plate (Sec. 5.1: the paper's plates use the EFIE, alpha = 1): a 1 m square
# PEC plate at 300 MHz +-5 %, edge lambda_min / 10 (11 x 11 squares, 341 RWG),
# on a 16 x 16 x 8 grid (the plate lies in z = 0, midway between two node
# planes; 8 nodes is the grid's minimum along z)
PLATE_1M = Workload("plate_1m_300MHz", level=0, radius=0.0, f0=300e6, frac_bw=0.05, nt=80, grid=(16, 16, 8),
                    near_lambda=0.3, beta=0.2, plate_size=1.0)

# long histories for the multilevel time blocks of the delayed field: the
# level-4 sphere with N_g = 47 (levels of 3, 6, 12 and 24 steps, the top one
# ending inside the history) and the level-2 sphere with N_g = 95 (all five
# levels; its near zone spans the first 81 lags)
SPHERE_L4_NG47 = Workload("sphere_L4_r1_600MHz_ng47", level=4, radius=1.0, f0=600e6, frac_bw=0.30,
                          nt=200, grid=48, near_lambda=0.3, ng=47, rotate_seed=0)
SPHERE_L2_NG95 = Workload("sphere_L2_r0.5_300MHz_ng95", level=2, radius=0.5, f0=300e6, frac_bw=0.20,
                          nt=300, grid=16, near_lambda=0.3, ng=95)
# ... and with N_g = 150: two further 48-step segments past lag 95
SPHERE_L2_NG150 = Workload("sphere_L2_r0.5_300MHz_ng150", level=2, radius=0.5, f0=300e6, frac_bw=0.20,
                           nt=300, grid=16, near_lambda=0.3, ng=150)

WORKLOADS = {w.name: w for w in (SPHERE_L2, SPHERE_L4, SPHERE_L4_BATCH, SPHERE_L4_ADJ, SPHERE_L3,
                                 SPHERE_L2_NARROW, COMPOSITE, COMPOSITE_SMALL, PLATE_1M, SPHERE_L4_NG47,
                                 SPHERE_L2_NG95, SPHERE_L2_NG150)}

# size and bandwidth sweep of spheres (ET-AIM only): the band's top fixed at
# f_max = 300 MHz while chi = f_max / f_bw varies (f_c = f_max - f_bw), and
# the radius doubling with each icosphere level, so that the mesh keeps an
# edge of about 15 cm (lambda_min / 6.7); grids of about 8.5 cm spacing
SWEEP_F_MAX = 300e6
SWEEP_SIZES = ((2, 0.5, 16), (3, 1.0, 24), (4, 2.0, 48), (5, 4.0, 96), (6, 8.0, 192))   # level, radius, grid
SWEEP_CHI = (3, 10, 30, 100)


def sweep_workload(level: int, radius: float, grid: int, chi: float) -> Workload:
    """Sphere of the sweep at one size and bandwidth: beta = 1/5, near zone
    0.3 lambda_c, one incidence along -z; the march long enough for the
    pulse (t_d + 8 sigma) and one crossing of the sphere."""
    f_bw = SWEEP_F_MAX / chi
    f0 = SWEEP_F_MAX - f_bw
    sigma = 3.0 / (2.0 * math.pi * f_bw)
    dt = 0.2 / f_bw
    nt = int(math.ceil((16.0 * sigma + 2.0 * radius / C0) / dt)) + 4
    return Workload(f"sweep_L{level}_r{radius:g}_chi{chi:g}", level=level, radius=radius, f0=f0,
                    frac_bw=f_bw / f0, nt=nt, grid=grid, near_lambda=0.3, beta=0.2)


# plate sweep (ET-AIM only, the EFIE): squares of 1-8 m at the sweep's bands,
# edge about 10 cm (lambda_min / 10 at 300 MHz), grid spacing about 9 cm
PLATE_SWEEP_SIZES = ((1.0, 16), (2.0, 24), (4.0, 48), (8.0, 96))


def plate_sweep_workload(size: float, grid: int, chi: float) -> Workload:
    """Plate of the sweep at one size and bandwidth: beta = 1/5, near zone
    0.3 lambda_c, normal incidence along -z, x-polarised; the march long
    enough for the pulse and one crossing of the plate's diagonal."""
    f_bw = SWEEP_F_MAX / chi
    f0 = SWEEP_F_MAX - f_bw
    sigma = 3.0 / (2.0 * math.pi * f_bw)
    dt = 0.2 / f_bw
    nt = int(math.ceil((16.0 * sigma + math.sqrt(2.0) * size / C0) / dt)) + 4
    wl = Workload(f"plate_sweep_{size:g}m_chi{chi:g}", level=0, radius=0.0, f0=f0, frac_bw=f_bw / f0, nt=nt,
                  grid=(grid, grid, 8), near_lambda=0.3, beta=0.2, plate_size=size)
    # the mesh edge follows the band's top, not the centre: lambda_min / 10 at 300 MHz
    wl.extra["edge"] = C0 / SWEEP_F_MAX / 10.0
    return wl
