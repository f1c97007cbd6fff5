"""The seeded composite-object mesher (boxes and cylinders) and the hull
shortcut of the largest vertex distance, checked against closed forms:

* every surface is closed and consistently oriented (each directed edge's
  reverse occurs exactly once), with outward normals: the divergence-theorem
  volume is positive and equals the solid's volume (a box exactly; a
  cylinder as the prism over the inscribed regular polygon), and the area
  equals the closed form of the same solid;
* the composite is six disjoint closed components (Euler characteristic 2
  each) whose bounding boxes keep the stated gap, of the stated sizes, inside
  the cube;
* R_max (the largest vertex distance that fixes N_g and dt) from the hull
  vertices equals the brute force over all vertices, and a box's diagonal.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import physics as ph


def _closed_oriented(tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    keys = set(map(tuple, e.tolist()))
    assert len(keys) == len(e), "a directed edge occurs twice"
    assert all((b, a) in keys for a, b in e.tolist()), "an edge without its reverse"


def _volume_area(xyz, tri):
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    vol = float(np.einsum("ij,ij->i", p0, np.cross(p1, p2)).sum() / 6.0)
    area = float(np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1).sum() / 2.0)
    return vol, area


@pytest.mark.parametrize("size", [(0.5, 0.7, 1.3), (2.0, 0.5, 0.61)])
def test_box_is_closed_outward_and_exact(size):
    edge = 0.1
    xyz, tri = W.box_mesh((0.3, -0.2, 1.0), size, edge)
    _closed_oriented(tri)
    a, b, c = size
    vol, area = _volume_area(xyz, tri)
    assert vol == pytest.approx(a * b * c, rel=1e-12)
    assert area == pytest.approx(2 * (a * b + b * c + c * a), rel=1e-12)
    n = np.ceil(np.array(size) / edge).astype(int)
    assert len(tri) == 4 * (n[0] * n[1] + n[1] * n[2] + n[2] * n[0])
    assert ph.rmax_of(xyz) == pytest.approx(math.sqrt(a * a + b * b + c * c), rel=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("r,h", [(0.25, 0.9), (0.6, 0.3)])
def test_cylinder_is_closed_outward_and_exact(axis, r, h):
    edge = 0.07
    xyz, tri = W.cylinder_mesh((0.1, 0.2, -0.3), r, h, axis, edge)
    _closed_oriented(tri)
    n = max(8, math.ceil(2 * math.pi * r / edge))
    poly = 0.5 * n * r * r * math.sin(2 * math.pi / n)       # inscribed regular n-gon
    vol, area = _volume_area(xyz, tri)
    assert vol == pytest.approx(poly * h, rel=1e-12)
    assert area == pytest.approx(2 * poly + n * 2 * r * math.sin(math.pi / n) * h, rel=1e-12)
    # the cylinder's axis lies along `axis`
    ext = xyz.max(0) - xyz.min(0)
    assert ext[axis] == pytest.approx(h, rel=1e-12)


def _components(nv, tri):
    parent = np.arange(nv)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for t in tri:
        for u, v in ((t[0], t[1]), (t[1], t[2])):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[ru] = rv
    return len({find(a) for a in range(nv)})


def test_composite_recipe():
    wl = W.COMPOSITE_SMALL
    xyz, tri, rwg = wl.mesh()
    _closed_oriented(tri)
    assert _components(len(xyz), tri) == 6
    assert len(xyz) - len(rwg) + len(tri) == 12            # six spheres topologically
    vol, _ = _volume_area(xyz, tri)
    assert vol > 0
    # the same seed gives the same object, another seed another
    xyz2, tri2 = W.composite(0, edge=wl.edge)
    assert np.array_equal(xyz, xyz2) and np.array_equal(tri, tri2)
    assert not np.array_equal(W.composite(1, edge=wl.edge)[0][:10], xyz[:10])
    assert np.all(np.abs(xyz) <= 5.4 / 2 + 1e-12)


def test_composite_parts_are_disjoint_and_sized():
    """Rebuild the placements from the stream and check them directly."""
    edge = W.COMPOSITE.edge
    assert edge == pytest.approx(299_792_458.0 / 1.05e9 / 10)
    xyz, tri = W.composite(0, edge=edge)
    parent = np.arange(len(xyz))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for t in tri:
        for u, v in ((t[0], t[1]), (t[1], t[2])):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[ru] = rv
    roots = np.array([find(a) for a in range(len(xyz))])
    boxes = []
    for r in np.unique(roots):
        p = xyz[roots == r]
        boxes.append((p.min(0), p.max(0)))
        ext = p.max(0) - p.min(0)
        # (a cylinder's width is that of its inscribed polygon, >= d cos(pi / 8))
        assert np.all(ext >= 0.5 * math.cos(math.pi / 8) - 1e-9) and np.all(ext <= 3.0 + 1e-9)
    assert len(boxes) == 6
    for i in range(6):
        for j in range(i + 1, 6):
            (l1, h1), (l2, h2) = boxes[i], boxes[j]
            gap = np.maximum(l2 - h1, l1 - h2).max()          # separation along the best axis
            assert gap >= 2 * edge - 1e-9


def test_composite_size_at_one_gigahertz():
    xyz, tri, rwg = W.COMPOSITE.mesh()
    assert len(rwg) == 200_634
    lens = np.linalg.norm(xyz[rwg[:, 2]] - xyz[rwg[:, 3]], axis=1)
    # grid edges at most lambda_min / 10; the rectangles' diagonals and the
    # cap fans' spokes are longer
    assert np.median(lens) <= W.COMPOSITE.edge + 1e-12


def test_rmax_from_hull_equals_brute_force():
    xyz, _, _ = W.COMPOSITE_SMALL.mesh()
    assert len(xyz) > 2048                                   # the hull path
    best = 0.0
    for s in range(0, len(xyz), 256):
        d = xyz[s:s + 256, None, :] - xyz[None, :, :]
        best = max(best, float(np.sqrt((d * d).sum(-1)).max()))
    assert ph.rmax_of(xyz) == best


def test_sweep_recipes():
    """The sweep keeps the band's top at 300 MHz (f_c + f_bw) while chi =
    f_max / f_bw varies, marches past the pulse and one crossing, and keeps
    the sphere's mesh edge at about 15 cm as the radius doubles per level."""
    for level, radius, grid in W.SWEEP_SIZES:
        xyz, tri = W.icosphere(level, radius)
        e = np.linalg.norm(xyz[tri[:, 0]] - xyz[tri[:, 1]], axis=1)
        assert 0.10 < np.median(e) < 0.20, (level, radius, np.median(e))
        for chi in W.SWEEP_CHI:
            wl = W.sweep_workload(level, radius, grid, chi)
            assert wl.f0 + wl.f_bw == pytest.approx(300e6, rel=1e-12)
            assert 300e6 / wl.f_bw == pytest.approx(chi, rel=1e-12)
            dt = wl.beta / wl.f_bw
            assert wl.nt * dt >= 16 * wl.sigma + 2 * radius / 299_792_458.0


def test_plate_mesh_and_open_rwg_table():
    """The plate: area size^2, every normal +z, n^2 squares of two
    triangles, and RWG on the 3n^2 - 2n interior edges only (the 4n
    boundary edges carry no basis); a closed-surface RWG table refuses it."""
    size, edge = 1.3, 0.1
    xyz, tri = W.plate_mesh(size, edge)
    n = math.ceil(size / edge)
    assert len(tri) == 2 * n * n
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(p1 - p0, p2 - p0)
    assert np.all(cr[:, 2] > 0) and np.allclose(cr[:, :2], 0.0)
    assert 0.5 * cr[:, 2].sum() == pytest.approx(size * size, rel=1e-12)
    rwg = W.rwg_table(tri, open_ok=True)
    assert len(rwg) == 3 * n * n - 2 * n
    with pytest.raises(ValueError):
        W.rwg_table(tri)
    assert len(W.PLATE_1M.mesh()[2]) == 341
