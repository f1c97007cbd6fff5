// Host set-up of the ET-AIM library (the "matrix fill" of Sec. 4 stages
// (i)-(iv)) driven on the CPU, for builds with the address and
// undefined-behaviour sanitizers: geometry, derived parameters, projection,
// near zone, exact near entries and the sparse approximate inverse on a mesh
// read from a file, then the rejection paths of invalid meshes.
//
// Input file (little-endian): int32 nv, nt, ns; float64 xyz[nv][3];
// int32 tri[nt][3]; int32 rwg[ns][4]; float64 fc, beta, f_bw, d_near;
// int32 grid.  Prints one line of summary numbers.  With two more arguments
// (alpha, output path) the problem is the CFIE with that alpha (the EFIE for
// alpha = 1), with a third ("blif") on the BLIF basis, and the driver also
// writes, little-endian: int32 nnz, mn; int32 rowptr[ns+1], col[nnz];
// complex128 near_exact[nnz][mn+1]; float64 lamH[ns][4][64] (CFIE only).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1408_7060_amd/csrc/context.hpp"

using namespace etaim;

static bool rd(FILE* f, void* p, size_t n) { return std::fread(p, 1, n, f) == n; }

int main(int argc, char** argv) {
    if (argc != 2 && argc != 4 && argc != 5) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t nv, nt, ns, grid;
    double fc, beta, fbw, dnear;
    if (!rd(f, &nv, 4) || !rd(f, &nt, 4) || !rd(f, &ns, 4)) return 2;
    std::vector<double> xyz(3 * (size_t)nv);
    std::vector<int32_t> tri(3 * (size_t)nt), rwg(4 * (size_t)ns);
    if (!rd(f, xyz.data(), xyz.size() * 8) || !rd(f, tri.data(), tri.size() * 4) ||
        !rd(f, rwg.data(), rwg.size() * 4) || !rd(f, &fc, 8) || !rd(f, &beta, 8) || !rd(f, &fbw, 8) ||
        !rd(f, &dnear, 8) || !rd(f, &grid, 4))
        return 2;
    std::fclose(f);
    etaim_mesh m{nv, xyz.data(), nt, tri.data()};
    etaim_rwg r{ns, rwg.data()};
    etaim_params p{};
    p.fc = fc;
    p.beta = beta;
    p.f_bw = fbw;
    p.nt_steps = 10;
    p.order = 3;
    p.grid[0] = p.grid[1] = p.grid[2] = grid;
    p.d_near = dnear;
    p.precision = ETAIM_FP64;
    p.batch = 1;
    p.tol = 1e-6;
    p.restart = 20;
    p.maxit = 100;
    if (argc >= 4) {
        p.alpha = std::atof(argv[2]);
        p.formulation = p.alpha < 1.0 ? ETAIM_CFIE : ETAIM_EFIE;
        if (argc == 5 && std::string(argv[4]) == "blif") p.basis = ETAIM_BLIF;
    }
    Geometry g;
    Setup s;
    std::string err;
    if (build_geometry(&m, &r, g, err) || derive_parameters(g, &p, s, err) || build_projection(g, s, err) ||
        build_near_zone(g, &p, s, err)) {
        std::printf("setup failed: %s\n", err.c_str());
        return 1;
    }
    exact_near_entries(g, &p, s);
    std::vector<zd> M;
    sparse_approximate_inverse(s, g.ns, M);
    double sn = 0, sm = 0, sl = 0;
    for (const zd& v : s.near_exact) sn += std::abs(v.x) + std::abs(v.y);
    for (const zd& v : M) sm += std::abs(v.x) + std::abs(v.y);
    for (double v : s.lam) sl += std::abs(v);
    // rejection paths: a degenerate triangle, a non-finite vertex, an edge
    // that is not an edge of its triangles, an out-of-range index
    int rejected = 0;
    {
        std::vector<int32_t> t2 = tri;
        t2[1] = t2[0];
        etaim_mesh m2{nv, xyz.data(), nt, t2.data()};
        Geometry g2;
        rejected += build_geometry(&m2, &r, g2, err) != 0;
    }
    {
        std::vector<double> x2 = xyz;
        x2[0] = std::nan("");
        etaim_mesh m2{nv, x2.data(), nt, tri.data()};
        Geometry g2;
        rejected += build_geometry(&m2, &r, g2, err) != 0;
    }
    {
        std::vector<int32_t> r2 = rwg;
        r2[2] = r2[3];
        etaim_rwg rr{ns, r2.data()};
        Geometry g2;
        rejected += build_geometry(&m, &rr, g2, err) != 0;
    }
    {
        std::vector<int32_t> t2 = tri;
        t2[4] = nv;
        etaim_mesh m2{nv, xyz.data(), nt, t2.data()};
        Geometry g2;
        rejected += build_geometry(&m2, &r, g2, err) != 0;
    }
    if (argc >= 4) {
        FILE* o = std::fopen(argv[3], "wb");
        if (!o) return 2;
        const int32_t nnz = (int32_t)s.col.size(), mn = s.mn;
        std::fwrite(&nnz, 4, 1, o);
        std::fwrite(&mn, 4, 1, o);
        std::fwrite(s.rowptr.data(), 4, s.rowptr.size(), o);
        std::fwrite(s.col.data(), 4, s.col.size(), o);
        std::fwrite(s.near_exact.data(), sizeof(zd), s.near_exact.size(), o);
        if (!s.lamH.empty()) std::fwrite(s.lamH.data(), 8, s.lamH.size(), o);
        std::fclose(o);
    }
    std::printf("ns %d ng %d mn %d nnz %zu lam %.12e near %.12e sai %.12e rejected %d\n", g.ns, s.ng, s.mn,
                s.col.size(), sl, sn, sm, rejected);
    return 0;
}
