"""ET-AIM pieces, written out plainly (oracle; test infrastructure only).

Sec. 4, stages (i)-(v) and eq. (5).  Readings (the paper defers the grid
rule to ref. [13] and the matrix entries to ref. [7]):

* Grid: cubic spacing h = max_a extent_a / (N_a - 4) over the vertex box,
  centred: x0_a = centre_a - h (N_a - 1)/2.  Basis centre c_k = mean of the
  two triangle centroids; stencil corner i0_a = floor((c_k,a - x0_a)/h) - 1;
  4 nodes per axis, 64 per basis.
* Projection (stage (i), moments up to order 3 matched, Sec. 5.1): per-axis
  degree <= 3 moments on the 4^3 stencil, i.e. the tensor cubic Lagrange
  projection  L[k,c,n] = int (S_k . e_c) l_n dS (c = x,y,z) and
  L[k,3,n] = int (div S_k) l_n dS, integrated exactly (degree <= 10) with the
  6 x 6 collapsed Gauss rule.  Local node index n = jx + 4 (jy + 4 jz), grid
  node index ix + Nx (iy + Ny iz).
* Grid Green functions (stage (ii)): G^A_m[d] = K_A(m, h|d|),
  G^phi_m[d] = K_phi(m, h|d|) for offsets |d_a| <= N_a - 1, G[0] = 0, m =
  0..N_g (truncated at N_g).
* Far part:  Z^FFT_m = sum_c L_c G^A_m L_c^T + L_q G^phi_m L_q^T.
* Near zone (stage (iv)): k' in N(k) iff |c_k - c_k'| <= d_near (k in N(k)).
  Pre-corrected Z^near_m = Z_m - Z^FFT_m on near pairs, m = 0..M_n with
  M_n = min(N_g, Q + floor((d_near + 2 r_max)/(c dt))), r_max the largest
  distance from a basis centre to its stencil nodes or support vertices.
* System (eq. (5), parentheses restored):
  (Z^near_0 + Z^FFT_0) I_l = V_l - sum_{m>=1} (Z^near_m + Z^FFT_m) I_{l-m}.

* CFIE (alpha < 1, ``oracle.mfie``): the far part is alpha times the EFIE
  far part above plus (1 - alpha) eta times the MFIE far part
  - sum_c H_c G^H_m L_c^T, on the same anterpolated components.  Each
  product is a channel (test projection, source component, Green table,
  coefficient); the EFIE has four, the CFIE seven.

Pins: projection moments vs the simplex monomial formula, FFT convolution
vs the literal double sum, symmetry, AIM accuracy on separated pairs.
"""
from __future__ import annotations

import math

import numpy as np

from . import cppif
from .geometry import Surface
from .kernels import EnvelopeKernel
from .physics import C0, ETA0
from .quadrature import collapsed_gauss, points

# threads of the 3-D transforms: 1 = numpy's FFT; more = scipy.fft with that
# many workers (the same transform, run on several cores; the timed CPU
# baseline sets it to the machine's core count)
FFT_WORKERS = 1


def _fftn(a):
    if FFT_WORKERS == 1:
        return np.fft.fftn(a)
    import scipy.fft
    return scipy.fft.fftn(a, workers=FFT_WORKERS)


def _ifftn(a):
    if FFT_WORKERS == 1:
        return np.fft.ifftn(a)
    import scipy.fft
    return scipy.fft.ifftn(a, workers=FFT_WORKERS)


class Grid:
    def __init__(self, xyz: np.ndarray, n):
        n = np.broadcast_to(np.asarray(n, dtype=np.int64), (3,)).copy()
        lo, hi = xyz.min(axis=0), xyz.max(axis=0)
        ext = hi - lo
        self.n = n
        self.h = float(np.max(ext / (n - 4)))
        centre = (lo + hi) / 2.0
        self.x0 = centre - self.h * (n - 1) / 2.0

    @property
    def nnodes(self) -> int:
        return int(np.prod(self.n))

    def node_xyz(self, ijk):
        return self.x0 + self.h * np.asarray(ijk, dtype=np.float64)


def stencil_corner(grid: Grid, c: np.ndarray) -> np.ndarray:
    return (np.floor((c - grid.x0) / grid.h) - 1).astype(np.int64)


def stencil_nodes(grid: Grid, i0: np.ndarray) -> np.ndarray:
    """Grid node index [ns,64] of the 4^3 stencil, local n = jx + 4(jy + 4 jz)."""
    j = np.arange(4)
    jx, jy, jz = np.meshgrid(j, j, j, indexing="ij")
    jx, jy, jz = (a.transpose(2, 1, 0).ravel() for a in (jx, jy, jz))   # jx fastest
    ix = i0[:, 0:1] + jx[None]
    iy = i0[:, 1:2] + jy[None]
    iz = i0[:, 2:3] + jz[None]
    if (ix.min() < 0 or iy.min() < 0 or iz.min() < 0 or ix.max() >= grid.n[0]
            or iy.max() >= grid.n[1] or iz.max() >= grid.n[2]):
        raise ValueError("stencil leaves the grid")
    return ix + grid.n[0] * (iy + grid.n[1] * iz)


def _lagrange4(u):
    """Cubic Lagrange basis on nodes 0,1,2,3 at local coordinate u [...]: [...,4]."""
    out = []
    for j in range(4):
        v = np.ones_like(u)
        for i in range(4):
            if i != j:
                v = v * (u - i) / (j - i)
        out.append(v)
    return np.stack(out, axis=-1)


def projection(surf: Surface, grid: Grid):
    """Moment-matching projection L [ns, 4, 64] and stencil corners i0 [ns,3]."""
    i0 = stencil_corner(grid, surf.c)
    bary, w = collapsed_gauss(6)
    L = np.zeros((surf.ns, 4, 64))
    for h in range(2):
        tri = surf.t[:, h]
        vt = surf.tv[tri]
        rp = points(vt, bary)                                   # [ns,P,3]
        u = (rp - grid.x0) / grid.h - i0[:, None, :]            # local coords
        lx, ly, lz = (_lagrange4(u[..., a]) for a in range(3))  # [ns,P,4]
        basis = np.einsum("kpa,kpb,kpc->kpcba", lx, ly, lz).reshape(surf.ns, -1, 64)
        area = surf.area[tri]
        ca = surf.s[:, h] * surf.length / (2.0 * area)
        cp = surf.s[:, h] * surf.length / area
        vfree = surf.xyz[surf.free[:, h]]
        Svec = ca[:, None, None] * (rp - vfree[:, None, :])   # [ns,P,3]
        wa = w[None, :] * area[:, None]
        for c in range(3):
            L[:, c, :] += np.einsum("kp,kp,kpn->kn", wa, Svec[..., c], basis)
        L[:, 3, :] += np.einsum("kp,k,kpn->kn", wa, cp, basis)
    return L, i0


def green_tables(grid: Grid, ms, dt: float, fc: float, basis=None):
    """G^A_m, G^phi_m on |offset| tables [len(ms), Nz, Ny, Nx] (index = |d|)."""
    nx, ny, nz = grid.n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    R = grid.h * np.sqrt((i * i + j * j + k * k).astype(np.float64))
    Rs = np.where(R == 0, 1.0, R)
    GA = np.zeros((len(ms),) + R.shape, dtype=np.complex128)
    GP = np.zeros_like(GA)
    for a, m in enumerate(ms):
        kn = EnvelopeKernel(m, dt, fc, basis)
        fa, fp = kn.f(R)
        GA[a] = np.where(R == 0, 0.0, kn.scale_a * fa / Rs)
        GP[a] = np.where(R == 0, 0.0, kn.scale_phi * fp / Rs)
    return GA, GP


def dense_node_matrix(grid: Grid, table: np.ndarray) -> np.ndarray:
    """Literal [N, N] matrix G[n, n'] = table[|dz|, |dy|, |dx|] (tiny grids)."""
    nx, ny, nz = grid.n
    idx = np.arange(grid.nnodes)
    ix, iy, iz = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    dx = np.abs(ix[:, None] - ix[None, :])
    dy = np.abs(iy[:, None] - iy[None, :])
    dz = np.abs(iz[:, None] - iz[None, :])
    return table[dz, dy, dx]


def near_pairs(surf: Surface, d_near: float):
    """(rows, cols) of all pairs with |c_k - c_k'| <= d_near, row-major sorted."""
    from scipy.spatial import cKDTree
    tree = cKDTree(surf.c)
    pairs = tree.query_pairs(d_near * (1 + 1e-9), output_type="ndarray")
    rows = np.concatenate([pairs[:, 0], pairs[:, 1], np.arange(surf.ns)])
    cols = np.concatenate([pairs[:, 1], pairs[:, 0], np.arange(surf.ns)])
    d = np.linalg.norm(surf.c[rows] - surf.c[cols], axis=1)
    keep = d <= d_near
    rows, cols = rows[keep], cols[keep]
    order = np.lexsort((cols, rows))
    return rows[order], cols[order]


def stencil_radius(surf: Surface, grid: Grid, i0: np.ndarray) -> float:
    j = np.arange(4)
    jx, jy, jz = np.meshgrid(j, j, j, indexing="ij")
    off = np.stack([jx.ravel(), jy.ravel(), jz.ravel()], axis=1)
    nodes = grid.x0 + grid.h * (i0[:, None, :] + off[None])
    r_st = np.linalg.norm(nodes - surf.c[:, None, :], axis=2).max(axis=1)
    r_sup = np.linalg.norm(surf.support_vertices() - surf.c[:, None, :], axis=2).max(axis=1)
    return float(np.maximum(r_st, r_sup).max())


def near_depth(d_near: float, r_max: float, dt: float, ng: int, q: int = cppif.Q) -> int:
    return int(min(ng, q + math.floor((d_near + 2.0 * r_max) / (C0 * dt))))


class AIM:
    """All L-B pieces for one problem (alpha = 1: EFIE; alpha < 1: CFIE)."""

    def __init__(self, surf: Surface, grid_n, d_near: float, dt: float, fc: float, ng: int,
                 alpha: float = 1.0, basis=None, fold_a=None):
        """basis: None (CPPIF) or an ``oracle.blif.Blif``; with a BLIF, fold_a
        [M-1, N_samp] folds the non-causal m = -(M-1)..-1 into m < N_samp
        (``oracle.blif``)."""
        self.surf, self.dt, self.fc, self.ng, self.d_near = surf, dt, fc, ng, d_near
        self.alpha = float(alpha)
        self.basis, self.fold_a = basis, fold_a
        self.mlo = 0 if basis is None else -(basis.M - 1)
        self.grid = Grid(surf.xyz, grid_n)
        self.L, self.i0 = projection(surf, self.grid)
        self.nodes = stencil_nodes(self.grid, self.i0)
        self.GA, self.GP = (self._folded(t) for t in green_tables(self.grid, range(self.mlo, ng + 1), dt, fc, basis))
        self.tables = {"A": self.GA, "P": self.GP}
        a = self.alpha
        # channels: (test projection [ns,64], source component, table, coefficient)
        self.channels = [(self.L[:, c, :], c, "A", a) for c in range(3)] + [(self.L[:, 3, :], 3, "P", a)]
        if a != 1.0:
            from . import mfie
            self.H = mfie.projection_curl(surf, self.grid, self.i0)
            self.GH = self._folded(mfie.green_table_h(self.grid, range(self.mlo, ng + 1), dt, fc, basis))
            self.tables["H"] = self.GH
            b = -(1.0 - a) * ETA0
            self.channels += [(self.H[:, c, :], c, "H", b) for c in range(3)]
        self.rows, self.cols = near_pairs(surf, d_near)
        self.r_max = stencil_radius(surf, self.grid, self.i0)
        self.mn = near_depth(d_near, self.r_max, dt, ng, cppif.Q if basis is None else basis.M)

    def _folded(self, tab):
        """Tables for m = mlo..ng -> m = 0..ng, the non-causal ones folded."""
        if self.mlo == 0:
            return tab
        from . import blif
        return blif.fold({m: tab[m - self.mlo] for m in range(self.mlo, self.ng + 1)}, self.fold_a, self.ng)

    def _exact(self, zfill_pairs, rows, cols):
        """Exact entries [M_n+1, P] (folded for a BLIF)."""
        if self.mlo == 0:
            return zfill_pairs(rows, cols, list(range(self.mn + 1)))
        from . import blif
        ms = list(range(self.mlo, self.mn + 1))
        z = zfill_pairs(rows, cols, ms)
        return blif.fold({m: z[i] for i, m in enumerate(ms)}, self.fold_a, self.mn)

    # ---- far part
    def anterpolate(self, x: np.ndarray) -> np.ndarray:
        """q [4, N] = L^T x (stage (i)), literal scatter-add."""
        q = np.zeros((4, self.grid.nnodes), dtype=np.complex128)
        for c in range(4):
            np.add.at(q[c], self.nodes.ravel(), (self.L[:, c, :] * x[:, None]).ravel())
        return q

    def interpolate(self, p) -> np.ndarray:
        """y [ns] = sum over channels of coef * T_ch p_ch (stage (iii)); p holds
        one potential grid per channel."""
        return sum(coef * np.einsum("kn,kn->k", T, p[i][self.nodes])
                   for i, (T, _, _, coef) in enumerate(self.channels))

    def propagate_direct(self, m: int, q: np.ndarray) -> list:
        """p_ch = G_m q_src per channel by the literal double sum over grid nodes
        (stage (ii))."""
        dense = {key: dense_node_matrix(self.grid, tab[m]) for key, tab in self.tables.items()}
        return [dense[key] @ q[src] for _, src, key, _ in self.channels]

    def ghat(self, m: int, key: str) -> np.ndarray:
        """FFT of the circulant embedding of table `key` at m, [2Nz, 2Ny, 2Nx];
        computed once per (m, key) and kept."""
        cache = self.__dict__.setdefault("_ghat", {})
        if (m, key) not in cache:
            cache[(m, key)] = _fftn(circulant(self.tables[key][m]))
        return cache[(m, key)]

    def green_hat(self, m: int, c: int) -> np.ndarray:
        """The EFIE's spectrum of component c: G^A_m (c < 3) or G^phi_m (c = 3)."""
        return self.ghat(m, "A" if c < 3 else "P")

    def spectra(self, x: np.ndarray) -> np.ndarray:
        """Forward FFT of the zero-padded anterpolated grid, [4, 2Nz, 2Ny, 2Nx]."""
        nx, ny, nz = self.grid.n
        q = self.anterpolate(x)
        out = np.zeros((4, 2 * nz, 2 * ny, 2 * nx), dtype=np.complex128)
        for c in range(4):
            out[c, :nz, :ny, :nx] = q[c].reshape(nz, ny, nx)
            out[c] = _fftn(out[c])
        return out

    def propagate_fft(self, m: int, q: np.ndarray) -> list:
        """p_ch = G_m q_src by zero-padded circulant FFT convolution (2N per axis)."""
        nx, ny, nz = self.grid.n
        qh = []
        for c in range(4):
            qq = np.zeros((2 * nz, 2 * ny, 2 * nx), dtype=np.complex128)
            qq[:nz, :ny, :nx] = q[c].reshape(nz, ny, nx)
            qh.append(_fftn(qq))
        return [_ifftn(self.ghat(m, key) * qh[src])[:nz, :ny, :nx].ravel() for _, src, key, _ in self.channels]

    def far_matvec(self, m: int, x: np.ndarray, direct: bool = False) -> np.ndarray:
        q = self.anterpolate(x)
        p = self.propagate_fft(m, q) if not direct else self.propagate_direct(m, q)
        return self.interpolate(p)

    def far_sum_rows(self, terms, rows) -> np.ndarray:
        """sum_i Z^FFT_{m_i} x_i on the given rows only, for terms = [(m_i,
        spectra(x_i))]: the products with the Green spectra are summed before
        one inverse transform per channel (the transform is linear), then
        interpolated at the stencils of ``rows``."""
        nx, ny, nz = self.grid.n
        rows = np.asarray(rows)
        y = 0
        for T, src, key, coef in self.channels:
            acc = np.zeros((2 * nz, 2 * ny, 2 * nx), dtype=np.complex128)
            for m, qh in terms:
                acc += self.ghat(m, key) * qh[src]
            p = _ifftn(acc)[:nz, :ny, :nx].ravel()
            y = y + coef * np.einsum("kn,kn->k", T[rows], p[self.nodes[rows]])
        return y

    def near_values_rows(self, zfill_pairs, rows):
        """Pre-corrected values [M_n+1, P] of the near pairs whose row is in
        ``rows`` (the pairs in CSR order: (self.rows[sel], self.cols[sel])).
        Returns (sel, values)."""
        sel = np.isin(self.rows, np.asarray(rows))
        rr, cc = self.rows[sel], self.cols[sel]
        ms = list(range(self.mn + 1))
        return sel, self._exact(zfill_pairs, rr, cc) - self.far_pairs(ms, rr, cc)

    def near_rows(self, sel, vals_m: np.ndarray, x: np.ndarray, rows) -> np.ndarray:
        """(Z^near_m x) on ``rows`` from the values of ``near_values_rows``."""
        rr, cc = self.rows[sel], self.cols[sel]
        y = np.zeros(self.surf.ns, dtype=np.complex128)
        np.add.at(y, rr, vals_m * x[cc])
        return y[np.asarray(rows)]

    def _full(self, T: np.ndarray) -> np.ndarray:
        ns = self.surf.ns
        out = np.zeros((ns, self.grid.nnodes))
        np.add.at(out, (np.repeat(np.arange(ns), 64), self.nodes.ravel()), T.ravel())
        return out

    def far_dense(self, m: int) -> np.ndarray:
        """Z^FFT_m as a dense [ns, ns] matrix (tiny problems)."""
        ns = self.surf.ns
        Z = np.zeros((ns, ns), dtype=np.complex128)
        dense = {key: dense_node_matrix(self.grid, tab[m]) for key, tab in self.tables.items()}
        for T, src, key, coef in self.channels:
            Z += coef * (self._full(T) @ (dense[key] @ self._full(self.L[:, src, :]).T))
        return Z

    def far_pairs(self, m, rows, cols) -> np.ndarray:
        """Z^FFT_m[rows[p], cols[p]] by the literal stencil double sum; m may be
        a list (result [len(m), P])."""
        ms = [m] if np.isscalar(m) else list(m)
        out = np.zeros((len(ms), len(rows)), dtype=np.complex128)
        nx, ny, nz = self.grid.n
        for s in range(0, len(rows), 512):
            r, c = rows[s:s + 512], cols[s:s + 512]
            na, nb = self.nodes[r], self.nodes[c]                  # [p,64]
            ia = np.stack([na % nx, (na // nx) % ny, na // (nx * ny)], -1)
            ib = np.stack([nb % nx, (nb // nx) % ny, nb // (nx * ny)], -1)
            d = np.abs(ia[:, :, None, :] - ib[:, None, :, :])       # [p,64,64,3]
            flat = (d[..., 2] * ny + d[..., 1]) * nx + d[..., 0]
            # stencil weight products per table: sum over its channels of coef T_r L_c
            prod = {}
            for T, src, key, coef in self.channels:
                w = coef * np.einsum("pn,pq->pnq", T[r], self.L[c, src])
                prod[key] = prod[key] + w if key in prod else w
            for i, mm in enumerate(ms):
                out[i, s:s + 512] = sum(np.einsum("pnq,pnq->p", w, self.tables[key][mm].ravel()[flat])
                                        for key, w in prod.items())
        return out[0] if np.isscalar(m) else out

    # ---- near part
    def near_values(self, zfill_pairs) -> np.ndarray:
        """Pre-corrected values [M_n+1, nnz]; ``zfill_pairs(rows, cols, ms)``
        returns the exact Z_m entries [len(ms), nnz]."""
        ms = list(range(self.mn + 1))
        exact = self._exact(zfill_pairs, self.rows, self.cols)
        far = self.far_pairs(ms, self.rows, self.cols)
        return exact - far

    def near_matvec(self, vals_m: np.ndarray, x: np.ndarray) -> np.ndarray:
        y = np.zeros(self.surf.ns, dtype=np.complex128)
        np.add.at(y, self.rows, vals_m * x[self.cols])
        return y


def circulant(table: np.ndarray) -> np.ndarray:
    """Embed an even |offset| table [nz,ny,nx] into the 2N-periodic circulant
    array: index i -> |i| for i < N, 2N - i for i > N, index N -> 0."""
    nz, ny, nx = table.shape

    def fold(n):
        i = np.arange(2 * n)
        f = np.where(i <= n, i, 2 * n - i)
        return f, i == n

    fz, bz = fold(nz)
    fy, by = fold(ny)
    fx, bx = fold(nx)
    fz_c, fy_c, fx_c = np.minimum(fz, nz - 1), np.minimum(fy, ny - 1), np.minimum(fx, nx - 1)
    out = table[fz_c[:, None, None], fy_c[None, :, None], fx_c[None, None, :]].copy()
    out[bz, :, :] = 0
    out[:, by, :] = 0
    out[:, :, bx] = 0
    return out
