// Host set-up of an ET-AIM problem: mesh/RWG validation, derived parameters,
// moment-matching projection, near zone and exact near-zone entries.
//
// Readings of the paper that this file implements (Sec. 3-5; the entries
// and the grid rule are deferred by the paper to its refs. [5], [7], [13]):
//  * time step / history: dt = beta/f_bw (Sec. 3), N_g = floor(Rmax/(c dt) + Q)
//    (Sec. 3 after eq. (4)); with N_g given, dt = Rmax/(c (N_g - Q + 1/2)).
//  * grid: cubic spacing h = max_a extent_a/(N_a - 4), centred on the vertex
//    box; basis centre c_k = mean of the two triangle centroids; 4^3 stencil
//    with corner floor((c_k - x0)/h) - 1.
//  * projection: moments up to order 3 per axis (Sec. 5.1), i.e. the tensor
//    cubic Lagrange projection, integrated exactly (6 x 6 Gauss-Legendre on
//    the collapsed square, exact to total degree 10).
//  * near zone: pairs of basis centres closer than d_near (stage (iv)).
//  * exact entries: differentiated EFIE with envelope kernels; 7 x 7
//    degree-5 rule on triangle pairs; on pairs sharing a vertex the f(0)/R
//    part is integrated in closed form over the source triangle (static
//    potentials of a flat triangle, Wilton et al. 1984 / Graglia 1993).
#include <cstdint>
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>

#include "context.hpp"

// host set-up keeps separate roundings (no contraction into fused multiply-adds)
#pragma clang fp contract(off)

namespace etaim {

namespace {

struct V3 {
    double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }
inline V3 vtx(const std::vector<double>& xyz, int i) { return {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]}; }

// 7-point degree-5 triangle rule (Radon 1948), barycentric, weights sum to 1.
struct Rule7 {
    double b[7][3], w[7];
    Rule7() {
        const double s15 = std::sqrt(15.0);
        const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
        const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
        const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                                  {a1, a1, 1 - 2 * a1}, {a1, 1 - 2 * a1, a1}, {1 - 2 * a1, a1, a1},
                                  {a2, a2, 1 - 2 * a2}, {a2, 1 - 2 * a2, a2}, {1 - 2 * a2, a2, a2}};
        const double ws[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
        std::memcpy(b, pts, sizeof(b));
        std::memcpy(w, ws, sizeof(w));
    }
};

// n-point Gauss-Legendre on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = 0.5 * (z + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Closed-form int_T 1/R dS' and int_T (r' - rho)/R dS' for a flat triangle
// (v[0], v[1], v[2] counter-clockwise about n) and observation point r;
// rho is the projection of r on the plane.
void tri_potentials(V3 r, const V3 v[3], double& I0, V3& I1, V3& rho) {
    V3 n = cross(v[1] - v[0], v[2] - v[0]);
    n = (1.0 / norm(n)) * n;
    const double d = dot(r - v[0], n);
    rho = r - d * n;
    const double ad = std::fabs(d);
    I0 = 0.0;
    I1 = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        const V3 a = v[i], b = v[(i + 1) % 3];
        V3 e = b - a;
        e = (1.0 / norm(e)) * e;
        const V3 u = cross(e, n);
        const double lp = dot(b - rho, e), lm = dot(a - rho, e), p0 = dot(a - rho, u);
        const double r02 = p0 * p0 + d * d;
        const double rp = std::sqrt(r02 + lp * lp), rm = std::sqrt(r02 + lm * lm);
        // ln((R+ + l+)/(R- + l-)); for l+ < 0 and l- < 0 the equal ratio
        // (R- - l-)/(R+ - l+) avoids cancellation
        double num, den;
        if (lp < 0 && lm < 0) {
            num = rm - lm;
            den = rp - lp;
        } else {
            num = rp + lp;
            den = rm + lm;
        }
        const double lr = (num > 0 && den > 0) ? std::log(num / den) : 0.0;
        double t1 = 0, t2 = 0;
        if (r02 > 0) {
            t1 = std::atan2(p0 * lp, r02 + ad * rp);
            t2 = std::atan2(p0 * lm, r02 + ad * rm);
        }
        I0 += p0 * lr - ad * (t1 - t2);
        I1 = I1 + (0.5 * (r02 * lr + lp * rp - lm * rm)) * u;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
int build_geometry(const etaim_mesh* m, const etaim_rwg* r, Geometry& g, std::string& err) {
    if (!m || !r || !m->xyz || !m->tri || !r->idx) {
        err = "null mesh or RWG pointer";
        return ETAIM_EINVAL;
    }
    if (m->nv < 3 || m->nt < 1 || r->ns < 1) {
        err = "mesh needs nv >= 3, nt >= 1 and ns >= 1";
        return ETAIM_EINVAL;
    }
    g.nv = m->nv;
    g.nt = m->nt;
    g.ns = r->ns;
    g.xyz.assign(m->xyz, m->xyz + 3 * (size_t)g.nv);
    g.tri.assign(m->tri, m->tri + 3 * (size_t)g.nt);
    for (double v : g.xyz)
        if (!std::isfinite(v)) {
            err = "non-finite vertex coordinate";
            return ETAIM_EINVAL;
        }
    g.area.resize(g.nt);
    g.cen.resize(3 * (size_t)g.nt);
    g.nrm.resize(3 * (size_t)g.nt);
    for (int t = 0; t < g.nt; ++t) {
        const int* tv = &g.tri[3 * (size_t)t];
        for (int j = 0; j < 3; ++j)
            if (tv[j] < 0 || tv[j] >= g.nv) {
                err = "triangle " + std::to_string(t) + " has a vertex index out of range";
                return ETAIM_EINVAL;
            }
        const V3 a = vtx(g.xyz, tv[0]), b = vtx(g.xyz, tv[1]), c = vtx(g.xyz, tv[2]);
        const V3 cr = cross(b - a, c - a);
        const double ar = 0.5 * norm(cr);
        if (!(ar > 0)) {
            err = "triangle " + std::to_string(t) + " is degenerate";
            return ETAIM_EINVAL;
        }
        g.area[t] = ar;
        const V3 nn = (1.0 / (2.0 * ar)) * cr;
        g.nrm[3 * t] = nn.x;
        g.nrm[3 * t + 1] = nn.y;
        g.nrm[3 * t + 2] = nn.z;
        g.cen[3 * t] = (a.x + b.x + c.x) / 3.0;
        g.cen[3 * t + 1] = (a.y + b.y + c.y) / 3.0;
        g.cen[3 * t + 2] = (a.z + b.z + c.z) / 3.0;
    }
    g.t.resize(2 * (size_t)g.ns);
    g.freev.resize(2 * (size_t)g.ns);
    g.loc.resize(2 * (size_t)g.ns);
    g.len.resize(g.ns);
    g.c.resize(3 * (size_t)g.ns);
    for (int k = 0; k < g.ns; ++k) {
        const int tp = r->idx[4 * (size_t)k], tm = r->idx[4 * (size_t)k + 1];
        const int e0 = r->idx[4 * (size_t)k + 2], e1 = r->idx[4 * (size_t)k + 3];
        if (tp < 0 || tp >= g.nt || tm < 0 || tm >= g.nt || tp == tm || e0 < 0 || e0 >= g.nv ||
            e1 < 0 || e1 >= g.nv || e0 == e1) {
            err = "RWG row " + std::to_string(k) + " has an invalid index";
            return ETAIM_EINVAL;
        }
        // T+ holds the directed edge e0 -> e1, T- the directed edge e1 -> e0
        const int tt[2] = {tp, tm};
        const int from[2] = {e0, e1}, to[2] = {e1, e0};
        for (int h = 0; h < 2; ++h) {
            const int* tv = &g.tri[3 * (size_t)tt[h]];
            int found = -1;
            for (int j = 0; j < 3; ++j)
                if (tv[j] == from[h] && tv[(j + 1) % 3] == to[h]) found = j;
            if (found < 0) {
                err = "RWG row " + std::to_string(k) + ": triangle " + std::to_string(tt[h]) +
                      " does not hold the edge with the orientation of " + (h ? "T-" : "T+");
                return ETAIM_EINVAL;
            }
            const int lf = (found + 2) % 3;  // the vertex not on the edge
            g.t[2 * k + h] = tt[h];
            g.loc[2 * k + h] = lf;
            g.freev[2 * k + h] = tv[lf];
        }
        const V3 a = vtx(g.xyz, e0), b = vtx(g.xyz, e1);
        g.len[k] = norm(b - a);
        for (int x = 0; x < 3; ++x) g.c[3 * k + x] = (g.cen[3 * tp + x] + g.cen[3 * tm + x]) / 2.0;
    }
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
static bool radix23(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

int derive_parameters(const Geometry& g, const etaim_params* p, Setup& s, std::string& err) {
    if (!(p->fc > 0) || p->nt_steps < 1 || p->batch < 1 || !(p->d_near >= 0) || !(p->tol > 0) ||
        p->restart < 1 || p->restart > 200 || p->maxit < 1 || p->ng < 0 || p->dt < 0 || p->sync_every < 0 ||
        p->sync_every > p->restart) {
        err = "invalid parameter (fc, nt_steps, batch, d_near, tol, restart, maxit, ng, dt, sync_every)";
        return ETAIM_EINVAL;
    }
    if (p->order != kQ) {
        err = "only the CPPIF of order 3 is supported";
        return ETAIM_EUNSUPPORTED;
    }
    if (p->precision != ETAIM_FP64 && p->precision != ETAIM_FP32) {
        err = "precision must be ETAIM_FP64 or ETAIM_FP32";
        return ETAIM_EINVAL;
    }
    if (p->formulation != ETAIM_EFIE && p->formulation != ETAIM_CFIE) {
        err = "formulation must be ETAIM_EFIE or ETAIM_CFIE";
        return ETAIM_EINVAL;
    }
    if (p->formulation == ETAIM_CFIE && !(p->alpha >= 0.0 && p->alpha < 1.0)) {
        err = "the CFIE's alpha must lie in [0, 1)";
        return ETAIM_EINVAL;
    }
    s.cfie = p->formulation == ETAIM_CFIE;
    s.alpha = s.cfie ? p->alpha : 1.0;
    if (p->basis != ETAIM_CPPIF && p->basis != ETAIM_BLIF) {
        err = "basis must be ETAIM_CPPIF or ETAIM_BLIF";
        return ETAIM_EINVAL;
    }
    // largest vertex-to-vertex distance
    double best = 0.0;
#pragma omp parallel for reduction(max : best) schedule(dynamic, 64)
    for (int i = 0; i < g.nv; ++i) {
        const double* a = &g.xyz[3 * (size_t)i];
        for (int j = 0; j < g.nv; ++j) {
            const double* b = &g.xyz[3 * (size_t)j];
            const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
            const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (d > best) best = d;
        }
    }
    s.rmax = best;
    if (p->dt > 0) {
        s.dt = p->dt;
        s.ng = p->ng > 0 ? p->ng : (int)std::floor(s.rmax / (kC0 * s.dt) + kQ);
    } else if (p->ng > 0) {
        s.ng = p->ng;
        if (p->ng <= kQ) {
            err = "ng must exceed the CPPIF order when dt is derived from it";
            return ETAIM_EINVAL;
        }
        s.dt = s.rmax / (kC0 * (p->ng - kQ + 0.5));
    } else {
        if (!(p->beta > 0) || !(p->f_bw > 0)) {
            err = "dt == 0 and ng == 0 need beta > 0 and f_bw > 0";
            return ETAIM_EINVAL;
        }
        s.dt = p->beta / p->f_bw;
        s.ng = (int)std::floor(s.rmax / (kC0 * s.dt) + kQ);
    }
    if (s.ng < 1 || s.ng > 4096) {
        err = "history depth out of range";
        return ETAIM_EINVAL;
    }
    if (p->basis == ETAIM_BLIF) {
        // the window's oversampling and the extrapolation of the M - 1 future samples
        const int M = p->order;
        const double beta = p->f_bw * s.dt;
        const int ns_ = p->nsamp > 0 ? p->nsamp : 3, nw = p->nomega > 0 ? p->nomega : 2 * ns_;
        if (!(p->f_bw > 0) || !(beta > 0.0 && beta < 0.5)) {
            err = "the BLIF needs f_bw > 0 with 0 < f_bw dt < 1/2";
            return ETAIM_EINVAL;
        }
        if (ns_ < 1 || ns_ > 4 || nw < ns_ || nw > 64 || s.ng < ns_) {
            err = "the BLIF's extrapolation needs 1 <= nsamp <= 4, nsamp <= nomega <= 64, nsamp <= N_g";
            return ETAIM_EINVAL;
        }
        s.tb.kind = 1;
        s.tb.M = M;
        const double a = kPi * M * (1.0 - 2.0 * beta), sha = std::sinh(a);
        double fct = 1.0;  // (2k+1)!
        for (int k = 0; k < kBlifTerms; ++k) {
            if (k > 0) fct *= (double)(2 * k) * (double)(2 * k + 1);
            s.tb.c[k] = std::pow(a, 2.0 * k + 1.0) / fct / sha;
        }
        s.mlo = -(M - 1);
        s.nsamp = ns_;
        // real least squares over the nw frequencies w dt = 2 pi beta x, x even on [-1, 1]:
        // rows (Re, Im) of exp(-j w p dt) a = exp(j w k dt), normal equations (nsamp <= 4)
        s.fold_a.assign((size_t)(M - 1) * ns_, 0.0);
        for (int k = 1; k < M; ++k) {
            double N[4][5] = {};
            for (int q = 0; q < nw; ++q) {
                const double x = nw == 1 ? 0.0 : -1.0 + 2.0 * q / (nw - 1);
                const double wd = 2.0 * kPi * beta * x;
                double re[4], im[4];
                for (int c = 0; c < ns_; ++c) {
                    re[c] = std::cos(wd * c);
                    im[c] = -std::sin(wd * c);
                }
                const double br = std::cos(wd * k), bi = std::sin(wd * k);
                for (int i = 0; i < ns_; ++i) {
                    for (int j = 0; j < ns_; ++j) N[i][j] += re[i] * re[j] + im[i] * im[j];
                    N[i][ns_] += re[i] * br + im[i] * bi;
                }
            }
            // Gaussian elimination with partial pivoting
            for (int i = 0; i < ns_; ++i) {
                int piv = i;
                for (int r = i + 1; r < ns_; ++r)
                    if (std::fabs(N[r][i]) > std::fabs(N[piv][i])) piv = r;
                for (int j = 0; j <= ns_; ++j) std::swap(N[i][j], N[piv][j]);
                if (!(std::fabs(N[i][i]) > 0)) {
                    err = "the BLIF's extrapolation fit is singular";
                    return ETAIM_EINVAL;
                }
                for (int r = i + 1; r < ns_; ++r) {
                    const double f = N[r][i] / N[i][i];
                    for (int j = i; j <= ns_; ++j) N[r][j] -= f * N[i][j];
                }
            }
            for (int i = ns_ - 1; i >= 0; --i) {
                double v = N[i][ns_];
                for (int j = i + 1; j < ns_; ++j) v -= N[i][j] * s.fold_a[(size_t)(k - 1) * ns_ + j];
                s.fold_a[(size_t)(k - 1) * ns_ + i] = v / N[i][i];
            }
        }
    }
    // grid
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = hi[a] = g.xyz[a];
        s.N[a] = p->grid[a];
        if (s.N[a] < 8) {
            err = "grid needs at least 8 nodes per axis";
            return ETAIM_EINVAL;
        }
        s.L[a] = 2 * s.N[a];
        if (s.L[a] > 2048) {
            err = "padded FFT length above 2048 is not supported";
            return ETAIM_EUNSUPPORTED;
        }
        if (!radix23(s.L[a])) {
            err = "padded FFT length 2*grid must be a product of 2 and 3";
            return ETAIM_EUNSUPPORTED;
        }
    }
    for (int i = 0; i < g.nv; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], g.xyz[3 * (size_t)i + a]);
            hi[a] = std::max(hi[a], g.xyz[3 * (size_t)i + a]);
        }
    double h = 0;
    for (int a = 0; a < 3; ++a) h = std::max(h, (hi[a] - lo[a]) / (double)(s.N[a] - 4));
    if (!(h > 0)) {
        err = "mesh has zero extent";
        return ETAIM_EINVAL;
    }
    s.h = h;
    for (int a = 0; a < 3; ++a) s.x0[a] = (lo[a] + hi[a]) / 2.0 - s.h * (double)(s.N[a] - 1) / 2.0;
    s.i0.resize(3 * (size_t)g.ns);
    for (int k = 0; k < g.ns; ++k)
        for (int a = 0; a < 3; ++a) {
            const int i0 = (int)std::floor((g.c[3 * k + a] - s.x0[a]) / s.h) - 1;
            if (i0 < 0 || i0 + 3 >= s.N[a]) {
                err = "stencil of basis " + std::to_string(k) + " leaves the grid";
                return ETAIM_EINVAL;
            }
            s.i0[3 * k + a] = i0;
        }
    // interpolation schedule: bases whose stencils overlap run close together
    // in time, so that their shared grid lines are L2 hits
    auto spread = [](uint64_t v) {
        uint64_t r = 0;
        for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1u) << (3 * b);
        return r;
    };
    std::vector<uint64_t> key(g.ns);
    for (int k = 0; k < g.ns; ++k)
        key[k] = spread((uint64_t)s.i0[3 * k]) | spread((uint64_t)s.i0[3 * k + 1]) << 1 |
                 spread((uint64_t)s.i0[3 * k + 2]) << 2;
    s.order.resize(g.ns);
    for (int k = 0; k < g.ns; ++k) s.order[k] = k;
    std::stable_sort(s.order.begin(), s.order.end(), [&](int a, int b) { return key[a] < key[b]; });
    s.d_near = p->d_near;
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
int build_projection(const Geometry& g, Setup& s, std::string& err) {
    (void)err;
    std::vector<double> gx, gw;
    gauss_legendre01(6, gx, gw);
    // collapsed square: l1 = u, l2 = (1-u) v, weight 2 (1-u) wu wv
    double qb[36][3], qw[36];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            const int q = 6 * a + b;
            qb[q][0] = gx[a];
            qb[q][1] = (1.0 - gx[a]) * gx[b];
            qb[q][2] = 1.0 - qb[q][0] - qb[q][1];
            qw[q] = 2.0 * (1.0 - gx[a]) * gw[a] * gw[b];
        }
    const int ns = g.ns;
    s.lam.assign((size_t)ns * 256, 0.0);
    // CFIE: the curl test projection H[k][c][n] = int ((S_k x n) x grad l_n)_c
    // (the tested n x curl of the interpolated potential), component 3 zero
    if (s.cfie) s.lamH.assign((size_t)ns * 256, 0.0);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < ns; ++k) {
        double* Lk = &s.lam[(size_t)k * 256];
        double* Hk = s.cfie ? &s.lamH[(size_t)k * 256] : nullptr;
        for (int h = 0; h < 2; ++h) {
            const int t = g.t[2 * k + h];
            const int* tv = &g.tri[3 * (size_t)t];
            const V3 v0 = vtx(g.xyz, tv[0]), v1 = vtx(g.xyz, tv[1]), v2 = vtx(g.xyz, tv[2]);
            const V3 vf = vtx(g.xyz, g.freev[2 * k + h]);
            const double sg = h == 0 ? 1.0 : -1.0;
            const double ca = sg * g.len[k] / (2.0 * g.area[t]);
            const double cp = sg * g.len[k] / g.area[t];
            for (int q = 0; q < 36; ++q) {
                const V3 r = qb[q][0] * v0 + qb[q][1] * v1 + qb[q][2] * v2;
                const double wa = qw[q] * g.area[t];
                // cubic Lagrange values l and derivatives dl (in the local
                // coordinate u) per axis
                double l[3][4], dl[3][4];
                const double rr[3] = {r.x, r.y, r.z};
                for (int a = 0; a < 3; ++a) {
                    const double u = (rr[a] - s.x0[a]) / s.h - (double)s.i0[3 * k + a];
                    for (int j = 0; j < 4; ++j) {
                        double v = 1.0, den = 1.0, d = 0.0;
                        for (int i = 0; i < 4; ++i)
                            if (i != j) {
                                v *= (u - i);
                                den *= (double)(j - i);
                            }
                        for (int skip = 0; skip < 4; ++skip) {
                            if (skip == j) continue;
                            double pr = 1.0;
                            for (int i = 0; i < 4; ++i)
                                if (i != j && i != skip) pr *= (u - i);
                            d += pr;
                        }
                        l[a][j] = v / den;
                        dl[a][j] = d / den;
                    }
                }
                const V3 S = ca * (r - vf);
                const double comp[4] = {S.x, S.y, S.z, cp};
                const V3 nt = {g.nrm[3 * (size_t)t], g.nrm[3 * (size_t)t + 1], g.nrm[3 * (size_t)t + 2]};
                const V3 Sn = cross(S, nt);
                for (int jz = 0; jz < 4; ++jz)
                    for (int jy = 0; jy < 4; ++jy)
                        for (int jx = 0; jx < 4; ++jx) {
                            const double b = wa * l[0][jx] * l[1][jy] * l[2][jz];
                            const int n = jx + 4 * (jy + 4 * jz);
                            for (int c = 0; c < 4; ++c) Lk[64 * c + n] += comp[c] * b;
                            if (Hk) {
                                const V3 gr = {dl[0][jx] * l[1][jy] * l[2][jz] / s.h,
                                               l[0][jx] * dl[1][jy] * l[2][jz] / s.h,
                                               l[0][jx] * l[1][jy] * dl[2][jz] / s.h};
                                const V3 v = cross(Sn, gr);
                                Hk[n] += wa * v.x;
                                Hk[64 + n] += wa * v.y;
                                Hk[128 + n] += wa * v.z;
                            }
                        }
            }
        }
    }
    // node-major transpose for the anterpolation gather
    const size_t N = (size_t)s.N[0] * s.N[1] * s.N[2];
    s.nptr.assign(N + 1, 0);
    auto node = [&](int k, int j) {
        const int jx = j & 3, jy = (j >> 2) & 3, jz = j >> 4;
        return (size_t)(s.i0[3 * k] + jx) +
               (size_t)s.N[0] * ((size_t)(s.i0[3 * k + 1] + jy) + (size_t)s.N[1] * (size_t)(s.i0[3 * k + 2] + jz));
    };
    for (int k = 0; k < ns; ++k)
        for (int j = 0; j < 64; ++j) s.nptr[node(k, j) + 1]++;
    for (size_t n = 0; n < N; ++n) s.nptr[n + 1] += s.nptr[n];
    s.nk.resize((size_t)ns * 64);
    s.nw.resize((size_t)ns * 64 * 4);
    std::vector<int> fill(s.nptr.begin(), s.nptr.end() - 1);
    for (int k = 0; k < ns; ++k)
        for (int j = 0; j < 64; ++j) {
            const size_t e = fill[node(k, j)]++;
            s.nk[e] = k;
            for (int c = 0; c < 4; ++c) s.nw[4 * e + c] = s.lam[(size_t)k * 256 + 64 * c + j];
        }
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
int build_near_zone(const Geometry& g, const etaim_params* p, Setup& s, std::string& err) {
    (void)p;
    const int ns = g.ns;
    const double dn = s.d_near;
    // cell list with cell size max(d_near, tiny)
    double lo[3] = {g.c[0], g.c[1], g.c[2]}, hi[3] = {g.c[0], g.c[1], g.c[2]};
    for (int k = 0; k < ns; ++k)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], g.c[3 * k + a]);
            hi[a] = std::max(hi[a], g.c[3 * k + a]);
        }
    double cell = dn;
    int nc[3];
    for (;;) {
        size_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            nc[a] = cell > 0 ? (int)std::floor((hi[a] - lo[a]) / cell) + 1 : 1;
            tot *= (size_t)nc[a];
        }
        if (tot <= (size_t)8 * ns + 64) break;
        cell = cell > 0 ? cell * 1.5 : (hi[0] - lo[0] + 1.0);
    }
    auto cid = [&](int k, int a) {
        int c = cell > 0 ? (int)std::floor((g.c[3 * k + a] - lo[a]) / cell) : 0;
        return std::min(std::max(c, 0), nc[a] - 1);
    };
    const size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
    std::vector<int> cstart(ncell + 1, 0), order(ns);
    std::vector<size_t> kc(ns);
    for (int k = 0; k < ns; ++k) {
        kc[k] = (size_t)cid(k, 0) + (size_t)nc[0] * ((size_t)cid(k, 1) + (size_t)nc[1] * cid(k, 2));
        cstart[kc[k] + 1]++;
    }
    for (size_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    {
        std::vector<int> f(cstart.begin(), cstart.end() - 1);
        for (int k = 0; k < ns; ++k) order[f[kc[k]]++] = k;
    }
    std::vector<std::vector<int>> rows(ns);
    const int reach = 1;
#pragma omp parallel for schedule(dynamic, 32)
    for (int k = 0; k < ns; ++k) {
        const int cx = cid(k, 0), cy = cid(k, 1), cz = cid(k, 2);
        std::vector<int>& out = rows[k];
        for (int z = std::max(cz - reach, 0); z <= std::min(cz + reach, nc[2] - 1); ++z)
            for (int y = std::max(cy - reach, 0); y <= std::min(cy + reach, nc[1] - 1); ++y)
                for (int x = std::max(cx - reach, 0); x <= std::min(cx + reach, nc[0] - 1); ++x) {
                    const size_t c = (size_t)x + (size_t)nc[0] * ((size_t)y + (size_t)nc[1] * z);
                    for (int e = cstart[c]; e < cstart[c + 1]; ++e) {
                        const int kk = order[e];
                        const double dx = g.c[3 * k] - g.c[3 * kk], dy = g.c[3 * k + 1] - g.c[3 * kk + 1],
                                     dz = g.c[3 * k + 2] - g.c[3 * kk + 2];
                        if (std::sqrt(dx * dx + dy * dy + dz * dz) <= dn) out.push_back(kk);
                    }
                }
        std::sort(out.begin(), out.end());
    }
    s.rowptr.assign(ns + 1, 0);
    for (int k = 0; k < ns; ++k) s.rowptr[k + 1] = s.rowptr[k] + (int)rows[k].size();
    if ((size_t)s.rowptr[ns] > (size_t)INT32_MAX / 2) {
        err = "near zone too large";
        return ETAIM_EINVAL;
    }
    s.col.resize(s.rowptr[ns]);
    for (int k = 0; k < ns; ++k) std::copy(rows[k].begin(), rows[k].end(), s.col.begin() + s.rowptr[k]);
    // largest distance from a basis centre to its stencil nodes or support vertices
    double rst = 0.0;
    for (int k = 0; k < ns; ++k) {
        for (int j = 0; j < 64; ++j) {
            const int jj[3] = {j & 3, (j >> 2) & 3, j >> 4};
            double d2 = 0;
            double dd[3];
            for (int a = 0; a < 3; ++a) dd[a] = (s.x0[a] + s.h * (double)(s.i0[3 * k + a] + jj[a])) - g.c[3 * k + a];
            d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
            rst = std::max(rst, std::sqrt(d2));
        }
        const int tp = g.t[2 * k], tm = g.t[2 * k + 1];
        (void)tm;
        int sup[4] = {g.freev[2 * k], g.freev[2 * k + 1], -1, -1};
        // the edge vertices are the two vertices of T+ other than its free vertex
        int n = 2;
        for (int j = 0; j < 3; ++j) {
            const int v = g.tri[3 * (size_t)tp + j];
            if (v != g.freev[2 * k]) sup[n++] = v;
        }
        for (int j = 0; j < 4; ++j) {
            double dd[3];
            for (int a = 0; a < 3; ++a) dd[a] = g.xyz[3 * (size_t)sup[j] + a] - g.c[3 * k + a];
            rst = std::max(rst, std::sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]));
        }
    }
    s.rst = rst;
    s.mn = std::min(s.ng, kQ + (int)std::floor((s.d_near + 2.0 * s.rst) / (kC0 * s.dt)));
    if (s.nsamp > s.mn + 1) {
        err = "the BLIF's nsamp exceeds the near-zone depth M_n + 1";
        return ETAIM_EINVAL;
    }
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
// Exact entries Z_m[k,k'] (m = 0..mn) of every near pair.
void exact_near_entries(const Geometry& g, const etaim_params* p, Setup& s) {
    const Rule7 rule;
    // stored m = 0..mn; computed m = mlo..mn (index i <-> m = mlo + i), the
    // BLIF's non-causal m < 0 folded into m < nsamp at the end of each pair
    const int M = s.mn + 1, mlo = s.mlo, ME = s.mn - mlo + 1;
    const double w = 2.0 * kPi * p->fc;
    EnvKernel K{s.dt, w, w / kC0, kC0 * s.dt};
    K.tb = s.tb;
    std::vector<zd> fa0(ME), fp0(ME), dfa0(ME), dfp0(ME);
    for (int m = 0; m < ME; ++m) K.origin(mlo + m, fa0[m], fp0[m], dfa0[m], dfp0[m]);
    const double sa = kMu0 / (4.0 * kPi), sp = 1.0 / (4.0 * kPi * eps0());
    // CFIE: alpha EFIE + (1 - alpha) eta MFIE (Sec. 2.1); MFIE Gram factors D_m
    const double al = s.alpha, bh = (1.0 - s.alpha) * std::sqrt(kMu0 / eps0());
    std::vector<zd> gm(ME);
    for (int m = 0; m < ME; ++m) gm[m] = K.gram(mlo + m);
    const size_t nnz = s.col.size();
    s.near_exact.assign(nnz * M, zd{0, 0});
#pragma omp parallel
    {
        std::vector<zd> IA(ME), IF(ME), IH(ME), ext(ME);
#pragma omp for schedule(dynamic, 16)
        for (int k = 0; k < g.ns; ++k) {
            for (int e = s.rowptr[k]; e < s.rowptr[k + 1]; ++e) {
                const int kk = s.col[e];
                std::fill(ext.begin(), ext.end(), zd{0, 0});
                zd* out = ext.data();
                for (int h = 0; h < 2; ++h)
                    for (int hh = 0; hh < 2; ++hh) {
                        const int ta = g.t[2 * k + h], tb = g.t[2 * kk + hh];
                        const int* A3 = &g.tri[3 * (size_t)ta];
                        const int* B3 = &g.tri[3 * (size_t)tb];
                        bool touch = false;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) touch |= A3[i] == B3[j];
                        const V3 va[3] = {vtx(g.xyz, A3[0]), vtx(g.xyz, A3[1]), vtx(g.xyz, A3[2])};
                        const V3 vb[3] = {vtx(g.xyz, B3[0]), vtx(g.xyz, B3[1]), vtx(g.xyz, B3[2])};
                        const V3 fa = vtx(g.xyz, g.freev[2 * k + h]);
                        const V3 fb = vtx(g.xyz, g.freev[2 * kk + hh]);
                        V3 ra[7], rb[7];
                        for (int q = 0; q < 7; ++q) {
                            ra[q] = rule.b[q][0] * va[0] + rule.b[q][1] * va[1] + rule.b[q][2] * va[2];
                            rb[q] = rule.b[q][0] * vb[0] + rule.b[q][1] * vb[1] + rule.b[q][2] * vb[2];
                        }
                        for (int m = 0; m < ME; ++m) IA[m] = IF[m] = zd{0, 0};
                        const double Aa = g.area[ta], Ab = g.area[tb];
                        for (int pq = 0; pq < 7; ++pq) {
                            const V3 da = ra[pq] - fa;
                            for (int qq = 0; qq < 7; ++qq) {
                                const V3 dv = ra[pq] - rb[qq];
                                const double R = std::sqrt(dv.x * dv.x + dv.y * dv.y + dv.z * dv.z);
                                const double W = rule.w[pq] * rule.w[qq] * (Aa * Ab);
                                const double D = dot(da, rb[qq] - fb);
                                for (int m = 0; m < ME; ++m) {
                                    zd ka, kp;
                                    if (touch && R == 0.0) {
                                        ka = dfa0[m];
                                        kp = dfp0[m];
                                    } else {
                                        zd fA, fP;
                                        K.eval(mlo + m, R, fA, fP);
                                        if (touch) {
                                            fA -= fa0[m];
                                            fP -= fp0[m];
                                        }
                                        ka = (1.0 / R) * fA;
                                        kp = (1.0 / R) * fP;
                                    }
                                    IA[m] += (W * D) * ka;
                                    IF[m] += W * kp;
                                }
                            }
                        }
                        if (touch) {
                            double sA = 0, sF = 0;
                            for (int pq = 0; pq < 7; ++pq) {
                                double I0;
                                V3 I1, rho;
                                tri_potentials(ra[pq], vb, I0, I1, rho);
                                const V3 Vj = I1 + I0 * (rho - fb);
                                const double wa = rule.w[pq] * Aa;
                                sA += wa * dot(ra[pq] - fa, Vj);
                                sF += wa * I0;
                            }
                            for (int m = 0; m < ME; ++m) {
                                IA[m] += sA * fa0[m];
                                IF[m] += sF * fp0[m];
                            }
                        }
                        const double sg = (h == 0 ? 1.0 : -1.0) * (hh == 0 ? 1.0 : -1.0);
                        const double cA = sg * g.len[k] * g.len[kk] / (4.0 * Aa * Ab);
                        const double cP = sg * g.len[k] * g.len[kk] / (Aa * Ab);
                        for (int m = 0; m < ME; ++m) out[m] += al * ((sa * cA) * IA[m] + (sp * cP) * IF[m]);
                        if (!s.cfie) continue;
                        if (ta == tb) {
                            // Gram term D_m / 2 <S_k, S_k'> on the shared triangle (exact, degree 2)
                            double gs = 0.0;
                            for (int q = 0; q < 7; ++q) gs += rule.w[q] * Aa * dot(ra[q] - fa, ra[q] - fb);
                            for (int m = 0; m < ME; ++m) out[m] += (bh * 0.5 * cA * gs) * gm[m];
                            continue;  // n x (Rhat x S') = 0 on a flat triangle with itself
                        }
                        // - int int g'_m(R) S_k . (n_a x (Rhat x S_k')),
                        // g'_m = -(1/4 pi) [fA/(c R) + fH/R^2]
                        const V3 na = {g.nrm[3 * (size_t)ta], g.nrm[3 * (size_t)ta + 1], g.nrm[3 * (size_t)ta + 2]};
                        for (int m = 0; m < ME; ++m) IH[m] = zd{0, 0};
                        for (int pq = 0; pq < 7; ++pq) {
                            const V3 da = ra[pq] - fa;
                            for (int qq = 0; qq < 7; ++qq) {
                                const V3 dv = ra[pq] - rb[qq];
                                const double R = std::sqrt(dv.x * dv.x + dv.y * dv.y + dv.z * dv.z);
                                if (!(R > 0.0)) continue;
                                const V3 rh = (1.0 / R) * dv;
                                const V3 db = rb[qq] - fb;
                                const double term = dot(da, rh) * dot(na, db) - dot(da, db) * dot(na, rh);
                                const double W = rule.w[pq] * rule.w[qq] * (Aa * Ab);
                                for (int m = 0; m < ME; ++m) {
                                    zd fA, fH;
                                    K.evalh(mlo + m, R, fA, fH);
                                    const zd gp = (-1.0 / (4.0 * kPi)) * ((1.0 / (kC0 * R)) * fA + (1.0 / (R * R)) * fH);
                                    IH[m] += (W * term) * gp;
                                }
                            }
                        }
                        for (int m = 0; m < ME; ++m) out[m] += (-bh * cA) * IH[m];
                    }
                // stored values: m = 0..mn, the non-causal ones folded in (BLIF)
                zd* dst = &s.near_exact[(size_t)e * M];
                for (int m = 0; m < M; ++m) dst[m] = ext[m - mlo];
                for (int kf = 1; kf <= -mlo; ++kf)
                    for (int q = 0; q < s.nsamp && q < M; ++q)
                        dst[q] += s.fold_a[(size_t)(kf - 1) * s.nsamp + q] * ext[-kf - mlo];
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Sparse approximate inverse of the step matrix on the near-zone pattern
// (right preconditioner of the per-step GMRES): column j of M minimises
// || Z0[I, J] m - e_j ||_2 over the near neighbours J of basis j, with I the
// rows that Z0[:, J] reaches (the neighbours of the neighbours).  Z0 on near
// pairs is the exact step entry (the pre-corrected AIM operator reproduces
// it there).  Each column is an independent small least-squares problem,
// solved by Householder QR.  M is returned in the near CSR layout: M[e] for
// e = (row i, column j) of the pattern, which is symmetric.
namespace {

using cz = std::complex<double>;

// least-squares solution of the n_r x n_c system S m = r (n_r >= n_c,
// column-major S, overwritten) by Householder QR
void lsq_householder(std::vector<cz>& S, int nr, int nc, std::vector<cz>& r, std::vector<cz>& m) {
    for (int k = 0; k < nc; ++k) {
        cz* a = &S[(size_t)k * nr];
        double sig = 0;
        for (int i = k; i < nr; ++i) sig += std::norm(a[i]);
        const double nrm = std::sqrt(sig);
        if (nrm == 0) continue;
        // v = a[k:] + e^{i arg a_k} |a| e_1; H = I - 2 v v^H / (v^H v)
        const cz ph = std::abs(a[k]) > 0 ? a[k] / std::abs(a[k]) : cz(1, 0);
        const cz alpha = -ph * nrm;
        a[k] -= alpha;
        double vv = 0;
        for (int i = k; i < nr; ++i) vv += std::norm(a[i]);
        for (int j = k + 1; j < nc; ++j) {
            cz* b = &S[(size_t)j * nr];
            cz d = 0;
            for (int i = k; i < nr; ++i) d += std::conj(a[i]) * b[i];
            d *= 2.0 / vv;
            for (int i = k; i < nr; ++i) b[i] -= d * a[i];
        }
        cz d = 0;
        for (int i = k; i < nr; ++i) d += std::conj(a[i]) * r[i];
        d *= 2.0 / vv;
        for (int i = k; i < nr; ++i) r[i] -= d * a[i];
        a[k] = alpha;  // R's diagonal; the rest of the reflector is no longer needed
    }
    m.assign(nc, cz(0, 0));
    for (int k = nc - 1; k >= 0; --k) {
        cz acc = r[k];
        for (int j = k + 1; j < nc; ++j) acc -= S[(size_t)j * nr + k] * m[j];
        const cz dkk = S[(size_t)k * nr + k];
        m[k] = std::abs(dkk) > 0 ? acc / dkk : cz(0, 0);
    }
}

}  // namespace

void sparse_approximate_inverse(const Setup& s, int ns, std::vector<zd>& M) {
    const int mv = s.mn + 1;
    const size_t nnz = s.col.size();
    M.assign(nnz, zd{0, 0});
    auto entry = [&](int i, int j, cz& v) {
        const int* b = s.col.data() + s.rowptr[i];
        const int* e = s.col.data() + s.rowptr[i + 1];
        const int* p = std::lower_bound(b, e, j);
        if (p == e || *p != j) return false;
        const zd z = s.near_exact[(size_t)(p - s.col.data()) * mv];
        v = cz(z.x, z.y);
        return true;
    };
#pragma omp parallel
    {
        std::vector<int> I;
        std::vector<cz> S, r, m;
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < ns; ++j) {
            const int j0 = s.rowptr[j], nc = s.rowptr[j + 1] - j0;
            if (nc == 0) continue;
            I.clear();
            for (int a = 0; a < nc; ++a) {
                const int k = s.col[j0 + a];
                I.insert(I.end(), s.col.begin() + s.rowptr[k], s.col.begin() + s.rowptr[k + 1]);
            }
            std::sort(I.begin(), I.end());
            I.erase(std::unique(I.begin(), I.end()), I.end());
            const int nr = (int)I.size();
            S.assign((size_t)nr * nc, cz(0, 0));
            r.assign(nr, cz(0, 0));
            for (int a = 0; a < nr; ++a) {
                if (I[a] == j) r[a] = cz(1, 0);
                for (int b = 0; b < nc; ++b) {
                    cz v;
                    if (entry(I[a], s.col[j0 + b], v)) S[(size_t)b * nr + a] = v;
                }
            }
            lsq_householder(S, nr, nc, r, m);
            // m[b] is M[col[j0 + b]][j]: stored at the pattern position (row col[j0 + b], column j)
            for (int b = 0; b < nc; ++b) {
                const int i = s.col[j0 + b];
                const int* bb = s.col.data() + s.rowptr[i];
                const int* ee = s.col.data() + s.rowptr[i + 1];
                const int* p = std::lower_bound(bb, ee, j);
                if (p != ee && *p == j) M[(size_t)(p - s.col.data())] = zd{m[b].real(), m[b].imag()};
            }
        }
    }
}

}  // namespace etaim
