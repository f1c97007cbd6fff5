// Context of one ET-AIM problem: host set-up results and device buffers.
#pragma once

#include <string>
#include <vector>

#include "../../include/etaim.h"
#include "common.hpp"

namespace etaim {

struct Error {
    int code;
    std::string msg;
};

// Host geometry derived from the mesh and RWG table (Sec. 3: RWG basis on a
// triangular mesh).
struct Geometry {
    int nv = 0, nt = 0, ns = 0;
    std::vector<double> xyz;        // [nv][3]
    std::vector<int> tri;           // [nt][3]
    std::vector<double> area;       // [nt]
    std::vector<double> cen;        // [nt][3]
    std::vector<double> nrm;        // [nt][3]
    // per basis k and half h (0: T+, 1: T-)
    std::vector<int> t;             // [ns][2] triangle
    std::vector<int> freev;         // [ns][2] free vertex id
    std::vector<int> loc;           // [ns][2] local index of the free vertex
    std::vector<double> len;        // [ns]
    std::vector<double> c;          // [ns][3] basis centre
};

// Host set-up results (the "matrix fill" of Sec. 4 stages (i)-(iv)).
struct Setup {
    double dt = 0, h = 0, x0[3] = {0, 0, 0}, rmax = 0, rst = 0, d_near = 0;
    int ng = 0, mn = 0, N[3] = {0, 0, 0}, L[3] = {0, 0, 0};
    TBasis tb{};                    // temporal basis (CPPIF, or BLIF with its window series)
    int mlo = 0;                    // lowest m of the unfolded kernels (BLIF: -(M-1))
    int nsamp = 0;                  // BLIF: past samples of the extrapolation
    std::vector<double> fold_a;     // BLIF: [M-1][nsamp] extrapolation coefficients
    bool cfie = false;              // combined-field equation (Sec. 2.1)
    double alpha = 1.0;             // its weight of the EFIE
    std::vector<double> lam;        // [ns][4][64] projection weights
    std::vector<double> lamH;       // CFIE: [ns][4][64] curl test projection (component 3 zero)
    std::vector<int> i0;            // [ns][3] stencil corners
    std::vector<int> order;         // [ns] bases sorted by the Morton code of their stencil corner
    std::vector<int> rowptr, col;   // near-zone CSR (row-major, sorted columns)
    std::vector<zd> near_exact;     // [nnz][mn+1] exact Z_m entries (m fastest)
    // node-major transpose of the projection (anterpolation gather)
    std::vector<int> nptr;          // [N+1]
    std::vector<int> nk;            // [64 ns] basis index
    std::vector<double> nw;         // [64 ns][4] weights
};

// host set-up (setup.cpp)
int build_geometry(const etaim_mesh* m, const etaim_rwg* r, Geometry& g, std::string& err);
int derive_parameters(const Geometry& g, const etaim_params* p, Setup& s, std::string& err);
int build_projection(const Geometry& g, Setup& s, std::string& err);
int build_near_zone(const Geometry& g, const etaim_params* p, Setup& s, std::string& err);
void exact_near_entries(const Geometry& g, const etaim_params* p, Setup& s);
// sparse approximate inverse of Z0 on the near pattern, in the near CSR layout
void sparse_approximate_inverse(const Setup& s, int ns, std::vector<zd>& M);

}  // namespace etaim
