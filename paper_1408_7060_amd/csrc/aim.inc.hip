// ET-AIM grid kernels (Sec. 4 stages (i)-(iv)):
//  k_fwdx_gather  anterpolation (node-major gather of the projection) fused
//                 with the forward x-FFT of the zero-padded grid (LDS lines)
//  k_prescale, k_anterp_nz, k_xfwd, k_xinv
//                 the same x stage with register-resident lines: the
//                 anterpolated grid goes through its own buffer Q, zero
//                 outside the nodes some basis reaches
//  k_yzq_*        register-resident parity-quadrant variants of the plane
//                 kernels below; k_yzc_* the same with the z lines first
//                 (two tiles); k_ring_far the time-block history pass
//  k_yz_green     per x-frequency plane: 2-D (y,z) FFT, Green-spectrum
//                 multiply, inverse 2-D FFT, all in LDS
//  k_yz_commit    per plane: forward 2-D FFT into a history-ring slot
//  k_yz_delayed   per plane: k-space temporal sum over the history ring,
//                 inverse 2-D FFT
//  k_interp_near  interpolation (projection transposed) + near-zone SpMV
// Grid layouts (per excitation b and component c = x,y,z,charge; bc = 4b+c):
//  A: [bc][kx<Lx][z<Nz][y<Ny] (x-transformed, plane-major)
//  ring slot: [bc][kx<Lx][kz<Lz][ky<Ly] (LDS plane kernels) or quadrant-major
//  [bc][kx][q][kz'][ky'] (register plane kernels)   P, Q: [bc][z][x][y] (N per bc)
#pragma once
#include "fft.inc.hip"

namespace etaim {

struct GridDims {
    int N[3], L[3], B;
};

template <typename R>
__device__ __forceinline__ cplx<R> to_r(zd v) {
    return cplx<R>{(R)v.x, (R)v.y};
}

// Anterpolation + forward x-pass.  Block (512 threads): MR rows (y) of one
// (z, b), all 4 components -> 4*MR lines of length Lx, transformed in place
// in LDS.  x_in: [B][ns] complex128; dinv (optional): right preconditioner
// diag^-1 [ns].  Output in the plane-major layout A[bc][kx][z][y] (runs of
// MR consecutive y).
template <typename R>
__global__ void __launch_bounds__(kPlaneThreads) k_fwdx_gather(
    const zd* __restrict__ x_in, const zd* __restrict__ dinv, const int* __restrict__ nptr,
    const int* __restrict__ nk, const R* __restrict__ nw, cplx<R>* __restrict__ A, const cplx<R>* __restrict__ tw_g,
    Radix pl, GridDims g, int mr, int ns, int conj_in, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    extern __shared__ unsigned char smem_raw[];
    const int Lx = g.L[0], Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int ldl = Lx + 1, nl = 4 * mr;
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* tw = buf + nl * ldl;
    for (int i = threadIdx.x; i < Lx; i += blockDim.x) tw[i] = tw_g[i];
    const int y0 = blockIdx.x * mr, z = blockIdx.y, b = blockIdx.z;
    const zd* xb = x_in + (size_t)b * ns;
    for (int e = threadIdx.x; e < mr * Lx; e += blockDim.x) {
        const int r = e / Lx, x = e - r * Lx;
        const int y = y0 + r;
        cplx<R> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        if (x < Nx && y < Ny) {
            const int n = x + Nx * (y + Ny * z);
            for (int q = nptr[n]; q < nptr[n + 1]; ++q) {
                const int k = nk[q];
                zd v = xb[k];
                if (conj_in) v.y = -v.y;
                if (dinv) v = v * dinv[k];
                const cplx<R> vr = to_r<R>(v);
                const R* w = nw + 4 * (size_t)q;
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += w[c] * vr;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) buf[(c * mr + r) * ldl + x] = acc[c];
    }
    __syncthreads();
    plane_fft<R>(buf, nl, ldl, 1, pl, tw, false);
    const size_t plane = (size_t)Nz * Ny;
    for (int e = threadIdx.x; e < nl * Lx; e += blockDim.x) {
        const int r = e % mr, rest = e / mr;
        const int kx = rest % Lx, c = rest / Lx;
        const int y = y0 + r;
        if (y < Ny) A[(((size_t)b * 4 + c) * Lx + kx) * plane + (size_t)z * Ny + y] = buf[(c * mr + r) * ldl + kx];
    }
}

__device__ __forceinline__ int fold(int k, int n2) { return k <= n2 / 2 ? k : n2 - k; }


// ---------------------------------------------------------------------------
// Register x stage (N_x = N with a register codelet, padded length 2N).  The
// anterpolated grid and the potentials share one buffer laid out
// [bc][z][x][y] (y fastest): lines along x of consecutive (z, y) are
// consecutive addresses, so lanes that own consecutive lines coalesce.

// xs[k][b] = conj?(x[b][k]) dinv[k] in the working precision, [ns][B]: the
// anterpolation then reads the columns of one basis as one run.
template <typename R>
__global__ void k_prescale(const zd* __restrict__ x, const zd* __restrict__ dinv, cplx<R>* __restrict__ xs, int ns,
                           int B, int conj_in, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const size_t tot = (size_t)ns * B;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / B), b = (int)(e - (size_t)k * B);
        zd v = x[(size_t)b * ns + k];
        if (conj_in) v.y = -v.y;
        if (dinv) v = v * dinv[k];
        xs[e] = to_r<R>(v);
    }
}

// Anterpolation (Sec. 4 stage (i)): q_c[n] = sum_k Lambda^c_{k,n} xs[k] from
// the node-major projection (nptr, nk, nw[4]), no atomics, over the grid
// nodes that some basis reaches (nodes[j], as the index t of q[bc][z][x][y]
// within a component plane; the other nodes of q stay zero).  Thread (j, b),
// columns b fastest, so that a wave shares the entry loads of a node and
// reads each basis's columns as one run.
template <typename R>
__global__ void __launch_bounds__(256) k_anterp_nz(const cplx<R>* __restrict__ xs, const int* __restrict__ nodes,
                                                   int nnodes, const int* __restrict__ nptr,
                                                   const int* __restrict__ nk, const R* __restrict__ nw,
                                                   cplx<R>* __restrict__ q, GridDims g, int B,
                                                   const int* __restrict__ gate) {
#pragma clang fp contract(fast)  // fused multiply-adds
    if (gated_off(gate)) return;
    const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (e >= (size_t)nnodes * B) return;
    const int j = (int)(e / B), b = (int)(e - (size_t)j * B);
    const int Nx = g.N[0], Ny = g.N[1];
    const size_t N3 = (size_t)Nx * Ny * g.N[2];
    const int t = nodes[j], y = t % Ny, r = t / Ny, x = r % Nx, z = r / Nx;
    const size_t n = (size_t)x + (size_t)Nx * ((size_t)y + (size_t)Ny * z);
    cplx<R> acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = cplx<R>{0, 0};
    const int p1 = nptr[n + 1];
    for (int p = nptr[n]; p < p1; p += 4) {
        int k[4];
        R w[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool live = p + u < p1;
            k[u] = live ? nk[p + u] : 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) w[u][c] = live ? nw[4 * (size_t)(p + u) + c] : (R)0;
        }
        cplx<R> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = xs[(size_t)k[u] * B + b];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += w[u][c] * v[u];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) q[((size_t)b * 4 + c) * N3 + t] = acc[c];
}

// Forward x transform of the zero-padded lines: A[bc][kx][z][y] =
// sum_{x<N} q[bc][z][x][y] w_{2N}^{kx x}.  Lanes (2l, 2l+1) own line l =
// (z, y) of one bc with parity p: kx = 2a + p is the N-point DFT of
// q w_{2N}^{p x}.  Bit x of xmask[l] marks the nodes some basis reaches;
// the others read the zero block zsrc instead (cached, no HBM traffic).
template <typename R, int N>
__global__ void __launch_bounds__(256) k_xfwd(const cplx<R>* __restrict__ q, cplx<R>* __restrict__ A, GridDims g,
                                              const unsigned long long* __restrict__ xmask,
                                              const cplx<R>* __restrict__ zsrc, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int Ny = g.N[1], Nz = g.N[2], nl = Ny * Nz, bc = blockIdx.y;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, line = tid >> 1, p = tid & 1;
    if (line >= nl) return;
    const int z = line / Ny, y = line - z * Ny;
    const cplx<R>* src = q + (size_t)bc * N * nl + (size_t)z * N * Ny + y;
    const unsigned long long mk = xmask[line];
    cplx<R> u[N];
#pragma unroll
    for (int x = 0; x < N; ++x) u[x] = *(((mk >> x) & 1ull) ? src + (size_t)x * Ny : zsrc);
    if (p) {
#pragma unroll
        for (int x = 1; x < N; ++x) u[x] = tw96_mul<R>(u[x], (96 / (2 * N)) * x, false);
    }
    dft_small<R, N>(u, false);
    cplx<R>* dst = A + (size_t)bc * 2 * N * nl + (size_t)p * nl + line;
#pragma unroll
    for (int a = 0; a < N; ++a) dst[(size_t)2 * a * nl] = u[a];
}

// Inverse x transform kept to x < N: P[bc][z][x][y] = sum_{kx<2N}
// A[bc][kx][z][y] w_{2N}^{-kx x}.  Lane (2l + p) takes the N-point inverse
// DFT of A[2a + p] times w_{2N}^{-p x}; the lane pair adds its two halves,
// each lane keeping and storing half of the x range.
template <typename R, int N>
__global__ void __launch_bounds__(256) k_xinv(const cplx<R>* __restrict__ A, cplx<R>* __restrict__ P, GridDims g,
                                              const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int Ny = g.N[1], Nz = g.N[2], nl = Ny * Nz, bc = blockIdx.y;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, line = tid >> 1, p = tid & 1;
    if (line >= nl) return;  // both lanes of a pair leave together
    const cplx<R>* src = A + (size_t)bc * 2 * N * nl + (size_t)p * nl + line;
    cplx<R> u[N];
#pragma unroll
    for (int a = 0; a < N; ++a) u[a] = src[(size_t)2 * a * nl];
    dft_small<R, N>(u, true);
    if (p) {
#pragma unroll
        for (int x = 1; x < N; ++x) u[x] = tw96_mul<R>(u[x], (96 / (2 * N)) * x, true);
    }
    const int z = line / Ny, y = line - z * Ny;
    cplx<R>* dst = P + (size_t)bc * N * nl + (size_t)z * N * Ny + y;
    constexpr int H = N / 2;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        // lane p keeps x = p H + j and sends the partner its x = (1 - p) H + j
        const cplx<R> keep = p ? u[H + j] : u[j], send = p ? u[j] : u[H + j];
        const cplx<R> got{__shfl_xor(send.x, 1, 64), __shfl_xor(send.y, 1, 64)};
        dst[(size_t)(p * H + j) * Ny] = keep + got;
    }
}

// Shared shapes of the plane kernels: one block per (kx, bc) holds the
// (y, z) plane of one x-frequency as buf[z * ldp + y], z in [0, Lz),
// y in [0, Ly), ldp = Ly + 1.  A plane of the x-transformed grid is
// A[bc][kx][z < Nz][y < Ny]; a ring slot plane is [bc][kx][kz][ky].
template <typename R>
__device__ __forceinline__ void plane_load(cplx<R>* buf, const cplx<R>* __restrict__ src, const GridDims& g) {
    const int Ly = g.L[1], Lz = g.L[2], Ny = g.N[1], Nz = g.N[2], ldp = Ly + 1;
    for (int e = threadIdx.x; e < Lz * Ly; e += blockDim.x) {
        const int z = e / Ly, y = e - z * Ly;
        buf[z * ldp + y] = (z < Nz && y < Ny) ? src[z * Ny + y] : cplx<R>{0, 0};
    }
    __syncthreads();
}

template <typename R>
__device__ __forceinline__ void plane_store(const cplx<R>* buf, cplx<R>* __restrict__ dst, const GridDims& g) {
    const int Ly = g.L[1], Ny = g.N[1], Nz = g.N[2], ldp = Ly + 1;
    for (int e = threadIdx.x; e < Nz * Ny; e += blockDim.x) {
        const int z = e / Ny, y = e - z * Ny;
        dst[e] = buf[z * ldp + y];
    }
}

// forward y (rows z < Nz), forward z (all Ly columns)
template <typename R>
__device__ __forceinline__ void plane_forward(cplx<R>* buf, const GridDims& g, const Radix& ry, const Radix& rz,
                                              const cplx<R>* twy, const cplx<R>* twz) {
    const int ldp = g.L[1] + 1;
    plane_fft<R>(buf, g.N[2], ldp, 1, ry, twy, false);
    plane_fft<R>(buf, g.L[1], 1, ldp, rz, twz, false);
}

// inverse z (all Ly columns), inverse y (rows z < Nz)
template <typename R>
__device__ __forceinline__ void plane_inverse(cplx<R>* buf, const GridDims& g, const Radix& ry, const Radix& rz,
                                              const cplx<R>* twy, const cplx<R>* twz) {
    const int ldp = g.L[1] + 1;
    plane_fft<R>(buf, g.L[1], 1, ldp, rz, twz, true);
    plane_fft<R>(buf, g.N[2], ldp, 1, ry, twy, true);
}

// LDS of a plane kernel: the plane, then the y and z twiddle tables.
template <typename R>
__device__ __forceinline__ void plane_smem(const GridDims& g, const cplx<R>* __restrict__ twy_g,
                                           const cplx<R>* __restrict__ twz_g, cplx<R>*& buf, cplx<R>*& twy,
                                           cplx<R>*& twz) {
    extern __shared__ unsigned char smem_raw[];
    buf = reinterpret_cast<cplx<R>*>(smem_raw);
    twy = buf + (size_t)g.L[2] * (g.L[1] + 1);
    twz = twy + g.L[1];
    for (int i = threadIdx.x; i < g.L[1]; i += blockDim.x) twy[i] = twy_g[i];
    for (int i = threadIdx.x; i < g.L[2]; i += blockDim.x) twz[i] = twz_g[i];
}

// Matvec y/z stage, in place on A: one block per plane (kx, bc): 2-D FFT of
// the zero-padded plane, multiply by the folded Green spectrum
// G[t][kx'][kz'][ky'] of one m, inverse 2-D FFT, keep y < Ny, z < Nz.
template <typename R>
__global__ void __launch_bounds__(kPlaneThreads) k_yz_green(cplx<R>* __restrict__ A, const cplx<R>* __restrict__ G,
                                                            const cplx<R>* __restrict__ twy_g,
                                                            const cplx<R>* __restrict__ twz_g, Radix ry, Radix rz,
                                                            GridDims g, int conj_g, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    cplx<R>*buf, *twy, *twz;
    plane_smem<R>(g, twy_g, twz_g, buf, twy, twz);
    const int kx = blockIdx.x, bc = blockIdx.y;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], ldp = Ly + 1;
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    cplx<R>* pl = A + ((size_t)bc * Lx + kx) * ((size_t)g.N[2] * g.N[1]);
    plane_load<R>(buf, pl, g);
    plane_forward<R>(buf, g, ry, rz, twy, twz);
    const int t = (bc & 3) == 3 ? 1 : 0;
    const cplx<R>* Gk = G + ((size_t)t * gx + fold(kx, Lx)) * ((size_t)gz * gy);
    for (int e = threadIdx.x; e < Lz * Ly; e += blockDim.x) {
        const int kz = e / Ly, ky = e - kz * Ly;
        cplx<R> gv = Gk[(size_t)fold(kz, Lz) * gy + fold(ky, Ly)];
        if (conj_g) gv.y = -gv.y;
        buf[kz * ldp + ky] = buf[kz * ldp + ky] * gv;
    }
    __syncthreads();
    plane_inverse<R>(buf, g, ry, rz, twy, twz);
    plane_store<R>(buf, pl, g);
}

// Commit y/z stage: forward 2-D FFT of the plane into a ring slot plane.
template <typename R>
__global__ void __launch_bounds__(kPlaneThreads) k_yz_commit(const cplx<R>* __restrict__ A, cplx<R>* __restrict__ slot,
                                                             const cplx<R>* __restrict__ twy_g,
                                                             const cplx<R>* __restrict__ twz_g, Radix ry, Radix rz,
                                                             GridDims g) {
    cplx<R>*buf, *twy, *twz;
    plane_smem<R>(g, twy_g, twz_g, buf, twy, twz);
    const int kx = blockIdx.x, bc = blockIdx.y;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], ldp = Ly + 1;
    plane_load<R>(buf, A + ((size_t)bc * Lx + kx) * ((size_t)g.N[2] * g.N[1]), g);
    plane_forward<R>(buf, g, ry, rz, twy, twz);
    cplx<R>* o = slot + ((size_t)bc * Lx + kx) * ((size_t)Lz * Ly);
    for (int e = threadIdx.x; e < Lz * Ly; e += blockDim.x) {
        const int kz = e / Ly, ky = e - kz * Ly;
        o[e] = buf[kz * ldp + ky];
    }
}

// Delayed-field y/z stage: k-space temporal sum over the history ring
// acc = sum_{m=1}^{nm} G_m . ring[(cur - m) mod ng], inverse 2-D FFT, plane
// y < Ny, z < Nz written to A.  G: folded spectra [ng+1][2][gx][gz][gy].
template <typename R>
__global__ void __launch_bounds__(kPlaneThreads) k_yz_delayed(const cplx<R>* __restrict__ ring,
                                                              const cplx<R>* __restrict__ G, cplx<R>* __restrict__ A,
                                                              const cplx<R>* __restrict__ twy_g,
                                                              const cplx<R>* __restrict__ twz_g, Radix ry, Radix rz,
                                                              GridDims g, int ng, int cur, int nm, int conj_g,
                                                              const cplx<R>* __restrict__ Fj) {
    cplx<R>*buf, *twy, *twz;
    plane_smem<R>(g, twy_g, twz_g, buf, twy, twz);
    const int kx = blockIdx.x, bc = blockIdx.y;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], ldp = Ly + 1;
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    const size_t gsz = (size_t)2 * gx * gy * gz;
    const size_t slot_sz = (size_t)4 * g.B * Lx * Lz * Ly;
    const int t = (bc & 3) == 3 ? 1 : 0;
    const size_t goff = ((size_t)t * gx + fold(kx, Lx)) * ((size_t)gz * gy);
    const size_t roff = ((size_t)bc * Lx + kx) * ((size_t)Lz * Ly);
    for (int e = threadIdx.x; e < Lz * Ly; e += blockDim.x) {
        const int kz = e / Ly, ky = e - kz * Ly;
        const size_t gi = goff + (size_t)fold(kz, Lz) * gy + fold(ky, Ly);
        // Fj: the older history's part of the sum, formed beforehand
        cplx<R> acc = Fj ? Fj[roff + e] : cplx<R>{0, 0};
        for (int m = 1; m <= nm; ++m) {
            int s = (cur - m) % ng;
            if (s < 0) s += ng;
            cplx<R> gv = G[(size_t)m * gsz + gi];
            if (conj_g) gv.y = -gv.y;
            acc += gv * ring[(size_t)s * slot_sz + roff + e];
        }
        buf[kz * ldp + ky] = acc;
    }
    __syncthreads();
    plane_inverse<R>(buf, g, ry, rz, twy, twz);
    plane_store<R>(buf, A + ((size_t)bc * Lx + kx) * ((size_t)g.N[2] * g.N[1]), g);
}

// ---------------------------------------------------------------------------
// Register plane kernels (N_y = N_z = N non-zero rows and columns, padded
// length 2N, N | 48).  The zero-padded 2N x 2N transform of a plane X[z][y]
// splits by the parities of the wavenumbers: Y[2b + pz][2a + py] is the
// N x N DFT of X[z][y] w_{2N}^{pz z + py y}, and the kept outputs z, y < N
// of the inverse transform are the sum over the four parity quadrants of
// w_{2N}^{-(pz z + py y)} times their N x N inverse DFTs.  The row (y)
// transforms do not depend on pz (w_{2N}^{pz z} scales a whole row), so
// they run once per py and are then scaled into both pz tiles; on the way
// back the two pz halves are added before the inverse row transforms.  A
// task (thread) holds one row or column of N points in registers, so every
// 1-D transform is an N-point FFT with compile-time twiddles and no LDS
// traffic; the four quadrant tiles (N x (N+1) each, q = 2 pz + py) carry
// the row <-> column exchanges.  Tasks per phase: 2N rows, 4N columns.
// Ring slots of this path are quadrant-major: [bc][kx][q][kz'][ky'] with
// kz = 2 kz' + pz, ky = 2 ky' + py.  Blocks run bc fastest (grid (4B, L_x)),
// so the blocks of one XCD share the Green-spectrum plane of their kx in L2.
constexpr int kQuadThreads = 192;

// two complex values as one vector load
template <typename R>
struct Pair;
template <>
struct Pair<float> {
    using type = float4;
};
template <>
struct Pair<double> {
    using type = double4;
};

template <typename R, int N>
__device__ __forceinline__ cplx<R>* qtile(cplx<R>* t0, int q) {
    return t0 + q * N * (N + 1);
}

template <typename R, int N>
__device__ __forceinline__ void tile_row(cplx<R>* t, int z, cplx<R> (&u)[N], bool store) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (store)
            t[z * (N + 1) + j] = u[j];
        else
            u[j] = t[z * (N + 1) + j];
    }
}

template <typename R, int N>
__device__ __forceinline__ void tile_col(cplx<R>* t, int y, cplx<R> (&u)[N], bool store) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (store)
            t[j * (N + 1) + y] = u[j];
        else
            u[j] = t[j * (N + 1) + y];
    }
}

// tile 0 = X, tile 1 = X w_{2N}^{y} (the py = 1 pre-twiddle); twy[n] = w_{2N}^n
template <typename R, int N>
__device__ __forceinline__ void quad_stage(cplx<R>* t0, const cplx<R>* __restrict__ src,
                                           const cplx<R>* __restrict__ twy) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int z = e / N, y = e - z * N, o = z * (N + 1) + y;
        const cplx<R> v = src[e];
        t0[o] = v;
        qtile<R, N>(t0, 1)[o] = cmul_fma(v, twy[y]);
    }
}

// forward rows: task (py, z): N-point DFT of row z of tile py, kept in tile
// py (pz = 0) and, times w_{2N}^{z}, written to tile 2 + py (pz = 1)
template <typename R, int N>
__device__ __forceinline__ void quad_rows_forward(cplx<R>* t0, const cplx<R>* __restrict__ twz) {
    const int i = threadIdx.x;
    if (i < 2 * N) {
        const int py = i / N, z = i - py * N;
        cplx<R> u[N];
        tile_row<R, N>(qtile<R, N>(t0, py), z, u, false);
        dft_small<R, N>(u, false);
        tile_row<R, N>(qtile<R, N>(t0, py), z, u, true);
        const cplx<R> s = twz[z];
#pragma unroll
        for (int j = 0; j < N; ++j) u[j] = cmul_fma(u[j], s);
        tile_row<R, N>(qtile<R, N>(t0, 2 + py), z, u, true);
    }
}

// inverse rows: task (py, z): row z of tile py plus conj(w_{2N}^{z}) times
// row z of tile 2 + py, N-point inverse DFT, back into tile py
template <typename R, int N>
__device__ __forceinline__ void quad_rows_inverse(cplx<R>* t0, const cplx<R>* __restrict__ twz,
                                                  int i = threadIdx.x) {
    if (i < 2 * N) {
        const int py = i / N, z = i - py * N;
        cplx<R> u[N];
        tile_row<R, N>(qtile<R, N>(t0, py), z, u, false);
        const cplx<R> s = conjz(twz[z]);
        const cplx<R>* r1 = qtile<R, N>(t0, 2 + py) + z * (N + 1);
#pragma unroll
        for (int j = 0; j < N; ++j) u[j] += cmul_fma(r1[j], s);
        dft_small<R, N>(u, true);
        tile_row<R, N>(qtile<R, N>(t0, py), z, u, true);
    }
}

// out[z N + y] = tile0 + conj(w_{2N}^{y}) tile1 (the py = 1 post-twiddle)
template <typename R, int N>
__device__ __forceinline__ void quad_sum_store(cplx<R>* t0, cplx<R>* __restrict__ out,
                                               const cplx<R>* __restrict__ twy, int tid = threadIdx.x,
                                               int nth = blockDim.x) {
    for (int e = tid; e < N * N; e += nth) {
        const int z = e / N, y = e - z * N, o = z * (N + 1) + y;
        out[e] = t0[o] + cmul_fma(qtile<R, N>(t0, 1)[o], conjz(twy[y]));
    }
}

// folded Green spectrum at ky = 2 c + py, kz = 2 j + pz for one plane
template <typename R, int N>
__device__ __forceinline__ cplx<R> quad_green(const cplx<R>* __restrict__ Gk, int j, int c, int py, int pz,
                                              int conj_g) {
    cplx<R> gv = Gk[fold(2 * j + pz, 2 * N) * (N + 1) + fold(2 * c + py, 2 * N)];
    if (conj_g) gv.y = -gv.y;
    return gv;
}

// Matvec y/z stage on the register path, in place on A (as k_yz_green).
template <typename R, int N>
__global__ void __launch_bounds__(kQuadThreads) k_yzq_green(cplx<R>* __restrict__ A, const cplx<R>* __restrict__ G,
                                                            const cplx<R>* __restrict__ twy,
                                                            const cplx<R>* __restrict__ twz, GridDims g, int conj_g,
                                                            const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* t0 = reinterpret_cast<cplx<R>*>(smem_raw);
    const int bc = blockIdx.x, kx = blockIdx.y, Lx = g.L[0];
    cplx<R>* pl = A + ((size_t)bc * Lx + kx) * (size_t)(N * N);
    quad_stage<R, N>(t0, pl, twy);
    __syncthreads();
    quad_rows_forward<R, N>(t0, twz);
    __syncthreads();
    const int i = threadIdx.x;
    if (i < 4 * N) {
        const int q = i / N, c = i - q * N, py = q & 1, pz = q >> 1;
        const int gx = g.N[0] + 1, gg = N + 1;
        const cplx<R>* Gk = G + ((size_t)((bc & 3) == 3 ? 1 : 0) * gx + fold(kx, Lx)) * (size_t)(gg * gg);
        cplx<R> u[N];
        tile_col<R, N>(qtile<R, N>(t0, q), c, u, false);
        dft_small<R, N>(u, false);
#pragma unroll
        for (int j = 0; j < N; ++j) u[j] = cmul_fma(u[j], quad_green<R, N>(Gk, j, c, py, pz, conj_g));
        dft_small<R, N>(u, true);
        tile_col<R, N>(qtile<R, N>(t0, q), c, u, true);
    }
    __syncthreads();
    quad_rows_inverse<R, N>(t0, twz);
    __syncthreads();
    quad_sum_store<R, N>(t0, pl, twy);
}

// Matvec y/z stage with the z lines first: two N x (N+1) tiles (one per
// z parity pz) instead of four quadrant tiles, so that four blocks share a
// CU in FP32 at N = 48.  With kz = 2 kz' + pz and ky = 2 ky' + py:
//  1. task (pz, y): column y of the plane (read from HBM), times
//     w_{2N}^{pz z}, N-point DFT over z -> column y of tile pz (rows kz');
//  2. task (pz, py, kz'): row kz' of tile pz times w_{2N}^{py y}, DFT over
//     y, Green product, inverse DFT, times conj(w_{2N}^{py y}); the two py
//     rows are summed back into row kz' of tile pz;
//  3. task (pz, y): inverse DFT of column y of tile pz over kz', times
//     conj(w_{2N}^{pz z}); the two pz columns are summed into the plane.
// GT is the Green table with ky and kz exchanged ([ky fold][kz fold] per
// plane), so that the lanes of phase 2 (consecutive kz') read neighbouring
// entries.  Threads: 4N (2N busy in phases 1 and 3, parity-grouped by wave);
// in FP32 the registers
// are capped for three waves per SIMD (four blocks per CU at N = 48).
template <typename R, int N>
__global__ void __launch_bounds__(4 * N) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 1))) k_yzc_green(cplx<R>* __restrict__ A, const cplx<R>* __restrict__ GT,
                                                     const cplx<R>* __restrict__ twy,
                                                     const cplx<R>* __restrict__ twz, GridDims g, int conj_g,
                                                     const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* t0 = reinterpret_cast<cplx<R>*>(smem_raw);
    const int bc = blockIdx.x, kx = blockIdx.y, Lx = g.L[0];
    cplx<R>* pl = A + ((size_t)bc * Lx + kx) * (size_t)(N * N);
    const int i = threadIdx.x;
    // phases 1 and 3: the pz = 1 tasks start at lane 64 where the block has
    // room, so that the first wave holds only pz = 0 tasks and skips the
    // twiddles; phase 2: py-major, so that the first wave skips them there
    constexpr int OFF1 = 4 * N >= 64 + N ? 64 : N;
    const bool zt = i < N || (i >= OFF1 && i < OFF1 + N);
    const int zpz = i < N ? 0 : 1, zy = i < N ? i : i - OFF1;
    cplx<R> u[N];
    if (zt) {
        const int pz = zpz, y = zy;
#pragma unroll
        for (int z = 0; z < N; ++z) u[z] = pl[z * N + y];
        if (pz) {
#pragma unroll
            for (int z = 0; z < N; ++z) u[z] = cmul_fma(u[z], twz[z]);
        }
        dft_small<R, N>(u, false);
        tile_col<R, N>(qtile<R, N>(t0, pz), y, u, true);
    }
    __syncthreads();
    const int py = i / (2 * N), pz2 = (i / N) & 1, kz = i % N;
    {
        const int gx = g.N[0] + 1, gg = N + 1;
        const cplx<R>* Gk = GT + ((size_t)((bc & 3) == 3 ? 1 : 0) * gx + fold(kx, Lx)) * (size_t)(gg * gg);
        const int zf = fold(2 * kz + pz2, 2 * N);
        tile_row<R, N>(qtile<R, N>(t0, pz2), kz, u, false);
        if (py) {
#pragma unroll
            for (int y = 0; y < N; ++y) u[y] = cmul_fma(u[y], twy[y]);
        }
        dft_small<R, N>(u, false);
#pragma unroll
        for (int c = 0; c < N; ++c) {
            cplx<R> gv = Gk[fold(2 * c + py, 2 * N) * gg + zf];
            if (conj_g) gv.y = -gv.y;
            u[c] = cmul_fma(u[c], gv);
        }
        dft_small<R, N>(u, true);
        if (py) {
#pragma unroll
            for (int y = 0; y < N; ++y) u[y] = cmul_fma(u[y], conjz(twy[y]));
        }
    }
    __syncthreads();
    cplx<R>* row = qtile<R, N>(t0, pz2) + kz * (N + 1);
    if (py == 0) {
#pragma unroll
        for (int y = 0; y < N; ++y) row[y] = u[y];
    }
    __syncthreads();
    if (py == 1) {
#pragma unroll
        for (int y = 0; y < N; ++y) row[y] += u[y];
    }
    __syncthreads();
    if (zt) {
        const int pz = zpz, y = zy;
        tile_col<R, N>(qtile<R, N>(t0, pz), y, u, false);
        dft_small<R, N>(u, true);
        if (pz) {
#pragma unroll
            for (int z = 0; z < N; ++z) u[z] = cmul_fma(u[z], conjz(twz[z]));
        }
        tile_col<R, N>(qtile<R, N>(t0, pz), y, u, true);
    }
    __syncthreads();
    // quarter h of the z range of column y: the two parities summed
    {
        const int h = i / N, y = i - h * N;
        const cplx<R>* c0 = qtile<R, N>(t0, 0);
        const cplx<R>* c1 = qtile<R, N>(t0, 1);
#pragma unroll
        for (int z = h * (N / 4); z < (h + 1) * (N / 4); ++z)
            pl[z * N + y] = c0[z * (N + 1) + y] + c1[z * (N + 1) + y];
    }
}

// Commit y/z stage with the z lines first (two tiles, as k_yzc_green):
// z columns per parity into the tiles, then the row tasks (pz, py, kz')
// transform their rows; the py = 0 rows, then the py = 1 rows go back into
// the tiles and out to the ring slot's quadrants q = 2 pz + py (coalesced).
template <typename R, int N>
__global__ void __launch_bounds__(4 * N) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 1)))
k_yzc_commit(const cplx<R>* __restrict__ A, cplx<R>* __restrict__ slot, const cplx<R>* __restrict__ twy,
             const cplx<R>* __restrict__ twz, GridDims g, StepRef sr, int ng) {
    if (step_off(sr)) return;
    // replayed: slot is the ring's base and the step picks its slot
    if (const StepDesc* d = step_of(sr))
        slot += (size_t)(d->cur % ng) * (4 * (size_t)g.B * g.L[0] * 4 * N * N);
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* t0 = reinterpret_cast<cplx<R>*>(smem_raw);
    constexpr int NN = N * N;
    const int bc = blockIdx.x, kx = blockIdx.y, Lx = g.L[0];
    const cplx<R>* pl = A + ((size_t)bc * Lx + kx) * (size_t)NN;
    cplx<R>* out = slot + ((size_t)bc * Lx + kx) * (size_t)(4 * NN);
    const int i = threadIdx.x;
    // as in k_yzc_green: pz = 1 column tasks from lane 64 where the block has
    // room, row tasks py-major, so that the first wave skips the twiddles
    constexpr int OFF1 = 4 * N >= 64 + N ? 64 : N;
    const bool zt = i < N || (i >= OFF1 && i < OFF1 + N);
    const int zpz = i < N ? 0 : 1, zy = i < N ? i : i - OFF1;
    cplx<R> u[N];
    if (zt) {
        const int pz = zpz, y = zy;
#pragma unroll
        for (int z = 0; z < N; ++z) u[z] = pl[z * N + y];
        if (pz) {
#pragma unroll
            for (int z = 0; z < N; ++z) u[z] = cmul_fma(u[z], twz[z]);
        }
        dft_small<R, N>(u, false);
        tile_col<R, N>(qtile<R, N>(t0, pz), y, u, true);
    }
    __syncthreads();
    const int py = i / (2 * N), pz2 = (i / N) & 1, kz = i % N;
    tile_row<R, N>(qtile<R, N>(t0, pz2), kz, u, false);
    __syncthreads();
    if (py) {
#pragma unroll
        for (int y = 0; y < N; ++y) u[y] = cmul_fma(u[y], twy[y]);
    }
    dft_small<R, N>(u, false);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (py == h) tile_row<R, N>(qtile<R, N>(t0, pz2), kz, u, true);
        __syncthreads();
        for (int e = i; e < 2 * NN; e += 4 * N) {
            const int pz = e / NN, r = e - pz * NN;
            out[(size_t)(2 * pz + h) * NN + r] = qtile<R, N>(t0, pz)[(r / N) * (N + 1) + r % N];
        }
        __syncthreads();
    }
}

// GT[p][a][b] = G[p][b][a] for the n x n planes p of a folded Green table
template <typename R>
__global__ void k_green_transpose(const cplx<R>* __restrict__ G, cplx<R>* __restrict__ GT, size_t planes, int n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t nn = (size_t)n * n;
    if (i >= planes * nn) return;
    const size_t p = i / nn;
    const int r = (int)(i - p * nn), a = r / n, b = r - a * n;
    GT[i] = G[p * nn + (size_t)b * n + a];
}

// Commit y/z stage on the register path: forward transforms of the plane
// into a quadrant-major ring slot plane.
template <typename R, int N>
__global__ void __launch_bounds__(kQuadThreads) k_yzq_commit(const cplx<R>* __restrict__ A, cplx<R>* __restrict__ slot,
                                                             const cplx<R>* __restrict__ twy,
                                                             const cplx<R>* __restrict__ twz, GridDims g) {
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* t0 = reinterpret_cast<cplx<R>*>(smem_raw);
    const int bc = blockIdx.x, kx = blockIdx.y, Lx = g.L[0];
    quad_stage<R, N>(t0, A + ((size_t)bc * Lx + kx) * (size_t)(N * N), twy);
    __syncthreads();
    quad_rows_forward<R, N>(t0, twz);
    __syncthreads();
    const int i = threadIdx.x;
    if (i < 4 * N) {
        const int q = i / N, c = i - q * N;
        cplx<R> u[N];
        tile_col<R, N>(qtile<R, N>(t0, q), c, u, false);
        dft_small<R, N>(u, false);
        cplx<R>* o = slot + (((size_t)bc * Lx + kx) * 4 + q) * (size_t)(N * N) + c;
#pragma unroll
        for (int j = 0; j < N; ++j) o[j * N] = u[j];
    }
}

// inverse column and row transforms of the quadrant tiles and the quadrant
// sum into one plane of A, by threads tid < nth of the block (every thread
// of the block must call it: it synchronises the block)
template <typename R, int N>
__device__ __forceinline__ void quad_inverse_store(cplx<R>* t0, cplx<R>* __restrict__ out,
                                                   const cplx<R>* __restrict__ twy, const cplx<R>* __restrict__ twz,
                                                   int tid, int nth) {
    if (tid < 4 * N) {
        const int q = tid / N, c = tid - q * N;
        cplx<R> u[N];
        tile_col<R, N>(qtile<R, N>(t0, q), c, u, false);
        dft_small<R, N>(u, true);
        tile_col<R, N>(qtile<R, N>(t0, q), c, u, true);
    }
    __syncthreads();
    quad_rows_inverse<R, N>(t0, twz, tid);
    __syncthreads();
    quad_sum_store<R, N>(t0, out, twy, tid, nth);
}

// tile position of point e of a quadrant-major plane
template <int N>
__device__ __forceinline__ int quad_tile_pos(int e) {
    const int qq = e / (N * N), rr = e - qq * N * N;
    return qq * N * (N + 1) + (rr / N) * (N + 1) + rr % N;
}

// Delayed-field y/z stage on the register path.  The k-space temporal sum
// over the quadrant-major ring streams the history.  A block owns the two
// planes (bc, kx) and (bc + 4, kx) of one kx and component, which share
// every Green value: each Green load serves two ring loads.  The block's
// 512 threads own consecutive pairs of spectrum points (one vector load of
// the ring per pair and plane, coalesced) and accumulate over m in
// registers; the sums go to two sets of quadrant tiles (150 KB in FP32),
// and each half of the block then transforms one plane.
constexpr int kDelayThreads = 512;

template <typename R, int N>
__global__ void __launch_bounds__(kDelayThreads) k_yzq_delayed(const cplx<R>* __restrict__ ring,
                                                              const cplx<R>* __restrict__ G, cplx<R>* __restrict__ A,
                                                              const cplx<R>* __restrict__ twy,
                                                              const cplx<R>* __restrict__ twz, GridDims g, int ng,
                                                              int cur, int nm, int conj_g,
                                                              const cplx<R>* __restrict__ Fj, StepRef sr) {
    if (step_off(sr)) return;
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* t0 = reinterpret_cast<cplx<R>*>(smem_raw);
    constexpr int NN = N * N, PAIRS = 4 * NN / 2, PER = 6, CHUNK = PER * kDelayThreads, TS = 4 * N * (N + 1);
    if (const StepDesc* d = step_of(sr)) {
        // Fj is the base of the block sums here: slot fj of this step, if any
        cur = d->cur;
        nm = d->nm;
        Fj = d->fj >= 0 ? Fj + (size_t)d->fj * (4 * (size_t)g.B * g.L[0] * 4 * NN) : nullptr;
    }
    // plane pair p: bc0 = 8 (p / 4) + p % 4 and bc0 + 4 (the same component c)
    const int p = blockIdx.x, bc0 = 8 * (p >> 2) + (p & 3);
    const int kx = blockIdx.y, Lx = g.L[0];
    const int gx = g.N[0] + 1, gg = N + 1;
    const size_t gsz = (size_t)2 * gx * gg * gg;
    const size_t slot_sz = (size_t)4 * g.B * Lx * 4 * NN;
    const size_t roff0 = ((size_t)bc0 * Lx + kx) * (size_t)(4 * NN);
    const size_t roff1 = roff0 + (size_t)4 * Lx * (4 * NN);
    const size_t goff = ((size_t)((bc0 & 3) == 3 ? 1 : 0) * gx + fold(kx, Lx)) * (size_t)(gg * gg);
    for (int c0 = 0; c0 < PAIRS; c0 += CHUNK) {
        // point pair i: points 2 i, 2 i + 1 of the plane's quadrant-major
        // spectrum (N is even, so a pair never straddles a quadrant row)
        int gi[PER][2];
        cplx<R> acc0[PER][2], acc1[PER][2];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = c0 + threadIdx.x + r * kDelayThreads;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = 2 * i + h, qq = e / NN, rr = e - qq * NN;
                const int kz = 2 * (rr / N) + (qq >> 1), ky = 2 * (rr % N) + (qq & 1);
                gi[r][h] = fold(kz, 2 * N) * gg + fold(ky, 2 * N);
                acc0[r][h] = cplx<R>{0, 0};
                acc1[r][h] = cplx<R>{0, 0};
            }
            // the older history's part of the sum, precomputed for this step's time block
            if (Fj != nullptr && i < PAIRS) {
                *reinterpret_cast<typename Pair<R>::type*>(acc0[r]) =
                    *reinterpret_cast<const typename Pair<R>::type*>(Fj + roff0 + 2 * i);
                *reinterpret_cast<typename Pair<R>::type*>(acc1[r]) =
                    *reinterpret_cast<const typename Pair<R>::type*>(Fj + roff1 + 2 * i);
            }
        }
        for (int m = 1; m <= nm; ++m) {
            int s = (cur - m) % ng;
            if (s < 0) s += ng;
            const cplx<R>* rs0 = ring + (size_t)s * slot_sz + roff0;
            const cplx<R>* rs1 = ring + (size_t)s * slot_sz + roff1;
            const cplx<R>* Gm = G + (size_t)m * gsz + goff;
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int i = c0 + threadIdx.x + r * kDelayThreads;
                if (i < PAIRS) {
                    cplx<R> v0[2], v1[2];
                    *reinterpret_cast<typename Pair<R>::type*>(v0) =
                        *reinterpret_cast<const typename Pair<R>::type*>(rs0 + 2 * i);
                    *reinterpret_cast<typename Pair<R>::type*>(v1) =
                        *reinterpret_cast<const typename Pair<R>::type*>(rs1 + 2 * i);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        cplx<R> gv = Gm[gi[r][h]];
                        if (conj_g) gv.y = -gv.y;
                        acc0[r][h] += cmul_fma(gv, v0[h]);
                        acc1[r][h] += cmul_fma(gv, v1[h]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = c0 + threadIdx.x + r * kDelayThreads;
            if (i < PAIRS) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int o = quad_tile_pos<N>(2 * i + h);
                    t0[o] = acc0[r][h];
                    t0[TS + o] = acc1[r][h];
                }
            }
        }
    }
    __syncthreads();
    const int half = threadIdx.x >= kDelayThreads / 2 ? 1 : 0;
    quad_inverse_store<R, N>(t0 + half * TS, A + ((size_t)(bc0 + 4 * half) * Lx + kx) * (size_t)NN, twy, twz,
                             threadIdx.x - half * (kDelayThreads / 2), kDelayThreads / 2);
}

constexpr int kDelay1Threads = 256;

// One plane per block (any batch; used where two planes' tiles do not fit
// the LDS, e.g. FP64 at N = 48).
template <typename R, int N>
__global__ void __launch_bounds__(kDelay1Threads) k_yzq_delayed1(const cplx<R>* __restrict__ ring,
                                                              const cplx<R>* __restrict__ G, cplx<R>* __restrict__ A,
                                                              const cplx<R>* __restrict__ twy,
                                                              const cplx<R>* __restrict__ twz, GridDims g, int ng,
                                                              int cur, int nm, int conj_g,
                                                              const cplx<R>* __restrict__ Fj, StepRef sr) {
    if (step_off(sr)) return;
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* t0 = reinterpret_cast<cplx<R>*>(smem_raw);
    // the plane's 4 N^2 points as pairs; the sum runs in chunks of PER pairs
    // per thread so that the accumulators stay within half the VGPR file
    constexpr int NN = N * N, PAIRS = 4 * NN / 2, PER = 9, CHUNK = PER * kDelay1Threads;
    if (const StepDesc* d = step_of(sr)) {
        cur = d->cur;
        nm = d->nm;
        Fj = d->fj >= 0 ? Fj + (size_t)d->fj * (4 * (size_t)g.B * g.L[0] * 4 * NN) : nullptr;
    }
    const int bc = blockIdx.x, kx = blockIdx.y, Lx = g.L[0];
    const int gx = g.N[0] + 1, gg = N + 1;
    const size_t gsz = (size_t)2 * gx * gg * gg;
    const size_t slot_sz = (size_t)4 * g.B * Lx * 4 * NN;
    const size_t roff = ((size_t)bc * Lx + kx) * (size_t)(4 * NN);
    const size_t goff = ((size_t)((bc & 3) == 3 ? 1 : 0) * gx + fold(kx, Lx)) * (size_t)(gg * gg);
    for (int c0 = 0; c0 < PAIRS; c0 += CHUNK) {
        // point pair i: points 2 i, 2 i + 1 of the plane's quadrant-major
        // spectrum (N is even, so a pair never straddles a quadrant row)
        int gi[PER][2];
        cplx<R> acc[PER][2];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = c0 + threadIdx.x + r * kDelay1Threads;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = 2 * i + h, qq = e / NN, rr = e - qq * NN;
                const int kz = 2 * (rr / N) + (qq >> 1), ky = 2 * (rr % N) + (qq & 1);
                gi[r][h] = fold(kz, 2 * N) * gg + fold(ky, 2 * N);
                acc[r][h] = cplx<R>{0, 0};
            }
            if (Fj != nullptr && i < PAIRS)
                *reinterpret_cast<typename Pair<R>::type*>(acc[r]) =
                    *reinterpret_cast<const typename Pair<R>::type*>(Fj + roff + 2 * i);
        }
        for (int m = 1; m <= nm; ++m) {
            int s = (cur - m) % ng;
            if (s < 0) s += ng;
            const cplx<R>* rs = ring + (size_t)s * slot_sz + roff;
            const cplx<R>* Gm = G + (size_t)m * gsz + goff;
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int i = c0 + threadIdx.x + r * kDelay1Threads;
                if (i < PAIRS) {
                    cplx<R> v[2];
                    *reinterpret_cast<typename Pair<R>::type*>(v) =
                        *reinterpret_cast<const typename Pair<R>::type*>(rs + 2 * i);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        cplx<R> gv = Gm[gi[r][h]];
                        if (conj_g) gv.y = -gv.y;
                        acc[r][h] += cmul_fma(gv, v[h]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = c0 + threadIdx.x + r * kDelay1Threads;
            if (i < PAIRS) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = 2 * i + h, qq = e / NN, rr = e - qq * NN;
                    t0[qq * N * (N + 1) + (rr / N) * (N + 1) + rr % N] = acc[r][h];
                }
            }
        }
    }
    __syncthreads();
    quad_inverse_store<R, N>(t0, A + ((size_t)bc * Lx + kx) * (size_t)(N * N), twy, twz, threadIdx.x, blockDim.x);
}

// History part of the delayed field for a block of pb steps starting at
// march step r0.  At step r0 + j the sum over m splits at m = j: the terms
// m > j read history older than r0, all known at the block's start, and are
// summed for the whole block in one pass over the ring,
//   F[j][p] = sum_{m = j+1}^{ng} G_m[p] ring[r0 + j - m][p],  j < pb,
// for every spectrum point p (quadrant-major, all bc and kx; history steps
// before 0 are zero); the j terms m <= j (the block's own, newer steps) are
// added at the step itself.  Each history slot is read once per block and
// feeds all pb outputs.  A thread owns one 16-byte vector of points (two in
// FP32) of one component c and kx and loops over the batch columns b: the
// points' Green values, the same for every b, are loaded once and stay in
// registers (NGX >= ng of them, a compile-time bound).  Ring reads and F
// writes are streaming (non-temporal).
constexpr int kFarMaxNg = 32, kFarMaxBlock = 8;

template <typename R>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int P = 2;
};
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int P = 1;
};

// ---------------------------------------------------------------------------
// Line-pass y/z engine (any grid whose lines fit the LDS line kernel, also
// where a padded (y, z) plane does not fit the LDS): the y and z transforms
// as separate passes over a full-spectrum work array S[bc][kx][kz][ky]
// (the ring-slot layout of this engine), k_lines for the y passes and the
// forward z pass, and these two kernels.

// Matvec z stage, in place on S: lines along z of one (bc, kx) plane, mt
// consecutive ky per block; the zero-padded forward transform of rows
// z < Nz, the product with the folded Green spectrum, the inverse
// transform, rows z < Nz stored back.
template <typename R>
__global__ void __launch_bounds__(kPlaneThreads) k_zlines_green(cplx<R>* __restrict__ S, const cplx<R>* __restrict__ G,
                                                               const cplx<R>* __restrict__ twz_g, Radix rz, GridDims g,
                                                               int mt, int conj_g, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    extern __shared__ unsigned char smem_raw[];
    const int Lz = g.L[2], Ly = g.L[1], Lx = g.L[0], Nz = g.N[2], ldl = Lz + 1;
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* tw = buf + mt * ldl;
    for (int i = threadIdx.x; i < Lz; i += blockDim.x) tw[i] = twz_g[i];
    const int ky0 = blockIdx.x * mt, pl = blockIdx.y, kx = pl % Lx, bc = pl / Lx;
    cplx<R>* base = S + (size_t)pl * Lz * Ly;
    // rows z (the line points) outer, consecutive ky (the lines) inner: coalesced
    for (int e = threadIdx.x; e < mt * Lz; e += blockDim.x) {
        const int p = e / mt, l = e - p * mt, ky = ky0 + l;
        cplx<R> v{0, 0};
        if (ky < Ly && p < Nz) v = base[(size_t)p * Ly + ky];
        buf[l * ldl + p] = v;
    }
    __syncthreads();
    plane_fft<R>(buf, mt, ldl, 1, rz, tw, false);
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    const int t = (bc & 3) == 3 ? 1 : 0;
    const cplx<R>* Gk = G + ((size_t)t * gx + fold(kx, Lx)) * ((size_t)gz * gy);
    for (int e = threadIdx.x; e < mt * Lz; e += blockDim.x) {
        const int p = e / mt, l = e - p * mt, ky = ky0 + l;
        if (ky < Ly) {
            cplx<R> gv = Gk[(size_t)fold(p, Lz) * gy + fold(ky, Ly)];
            if (conj_g) gv.y = -gv.y;
            buf[l * ldl + p] = buf[l * ldl + p] * gv;
        }
    }
    __syncthreads();
    plane_fft<R>(buf, mt, ldl, 1, rz, tw, true);
    for (int e = threadIdx.x; e < mt * Nz; e += blockDim.x) {
        const int p = e / mt, l = e - p * mt, ky = ky0 + l;
        if (ky < Ly) base[(size_t)p * Ly + ky] = buf[l * ldl + p];
    }
}

// The same z stage with four-step z lines (L_z = A B, both factors register
// codelets): the forward transform's first step loads rows z < N_z of MT
// consecutive ky (lanes over the lines, so each row's loads are one run),
// the second step, the Green product and the inverse's first step run in
// the registers of the (ky, k1) tasks, and the inverse's second step stores
// rows z < N_z back.
template <typename R, int A, int B>
__global__ void __launch_bounds__((lines4_threads<R, A, B>())) k_zg4(cplx<R>* __restrict__ S,
                                                                  const cplx<R>* __restrict__ G,
                                                                  const cplx<R>* __restrict__ twz_g, GridDims g,
                                                                  int conj_g, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    constexpr int MT = lines4_mt<R>(), L = A * B;
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* Y = tw + L;
    for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twz_g[i];
    const int Ly = g.L[1], Lx = g.L[0], Nz = g.N[2];
    const int ky0 = blockIdx.x * MT, pl = blockIdx.y, kx = pl % Lx, bc = pl / Lx;
    cplx<R>* base = S + (size_t)pl * L * Ly;
    __syncthreads();
    for (int t = threadIdx.x; t < MT * B; t += blockDim.x) {
        const int l = t % MT, n2 = t / MT, ky = ky0 + l;
        cplx<R> u[A];
        // the padded half (z >= N_z = L/2, i.e. n1 >= A/2) is zero
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) {
            const int z = n2 + B * n1;
            u[n1] = (n1 < A / 2 && ky < Ly) ? base[(size_t)z * Ly + ky] : cplx<R>{0, 0};
        }
        l4_fwd_first<R, A, B, MT, true>(u, Y, tw, l, n2);
    }
    __syncthreads();
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    const cplx<R>* Gk = G + ((size_t)((bc & 3) == 3 ? 1 : 0) * gx + fold(kx, Lx)) * ((size_t)gz * gy);
    for (int t = threadIdx.x; t < MT * A; t += blockDim.x) {
        const int l = t % MT, k1 = t / MT, ky = ky0 + l;
        const int fy = fold(ky < Ly ? ky : 0, Ly);
        cplx<R> u[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) u[n2] = Y[l4_y<R, A, B, true>(l, k1, n2)];
        dft_small<R, B>(u, false);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            cplx<R> gv = Gk[(size_t)fold(k1 + A * k2, L) * gy + fy];
            if (conj_g) gv.y = -gv.y;
            u[k2] = u[k2] * gv;
        }
        // the task rewrites only the Y entries it has just read
        l4_inv_first<R, A, B, MT, true>(u, Y, tw, l, k1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < MT * B; t += blockDim.x) {
        const int l = t % MT, n2 = t / MT, ky = ky0 + l;
        cplx<R> u[A];
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) u[k1] = Y[l4_y<R, A, B, true>(l, k1, n2)];
        dft_small<R, A>(u, true);
        if (ky < Ly)
#pragma unroll
            for (int n1 = 0; n1 < A / 2; ++n1) base[(size_t)(n2 + B * n1) * Ly + ky] = u[n1];
    }
}

// Delayed-field sum of the line-pass engine: S = sum_{m=1}^{nm} G_m . ring
// slot (cur - m) mod ng over every spectrum point [bc][kx][kz][ky]; a thread
// owns one 16-byte vector of points (two in FP32) of one plane row and
// loops over m.
template <typename R>
__global__ void __launch_bounds__(256) k_delay_sum(const cplx<R>* __restrict__ ring, const cplx<R>* __restrict__ G,
                                                   cplx<R>* __restrict__ S, GridDims g, int ng, int cur, int nm,
                                                   int conj_g, const cplx<R>* __restrict__ Fj) {
    using V = typename Vec16<R>::type;
    constexpr int P = Vec16<R>::P;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    const size_t plane = (size_t)Ly * Lz, slot = (size_t)4 * g.B * Lx * plane;
    const size_t gid = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) * P;
    if (gid >= slot) return;
    // Ly is even, so the P points share one (bc, kx, kz) row
    const size_t pl = gid / plane;
    const int r = (int)(gid - pl * plane), kz = r / Ly, ky = r - kz * Ly;
    const int kx = (int)(pl % Lx), bc = (int)(pl / Lx);
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    const size_t gsz = (size_t)2 * gx * gy * gz;
    const size_t goff = (((size_t)((bc & 3) == 3 ? 1 : 0) * gx + fold(kx, Lx)) * gz + fold(kz, Lz)) * gy;
    const R sg = conj_g ? R(-1) : R(1);
    cplx<R> acc[P];
    if (Fj) {
        // time blocks: the step's block sum of the older history, then its nm
        // newest terms
        const V f = __builtin_nontemporal_load(reinterpret_cast<const V*>(Fj + gid));
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] = cplx<R>{f[2 * q], f[2 * q + 1]};
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] = cplx<R>{0, 0};
    }
    for (int m = 1; m <= nm; ++m) {
        int s = (cur - m) % ng;
        if (s < 0) s += ng;
        const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(ring + (size_t)s * slot + gid));
#pragma unroll
        for (int q = 0; q < P; ++q) {
            cplx<R> gv = G[(size_t)m * gsz + goff + fold(ky + q, Ly)];
            gv.y *= sg;
            acc[q] += cmul_fma(gv, cplx<R>{t[2 * q], t[2 * q + 1]});
        }
    }
    V o;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        o[2 * q] = acc[q].x;
        o[2 * q + 1] = acc[q].y;
    }
    *reinterpret_cast<V*>(S + gid) = o;
}

template <typename R, int N, int NGX>
__global__ void __launch_bounds__(256) k_ring_far(const cplx<R>* __restrict__ ring, const cplx<R>* __restrict__ G,
                                                  cplx<R>* __restrict__ F, GridDims g, int ng, int r0, int pb,
                                                  int conj_g, StepRef sr) {
    if (step_off(sr)) return;
    if (const StepDesc* d = step_of(sr)) r0 = d->r0;
    using V = typename Vec16<R>::type;
    constexpr int P = Vec16<R>::P, NN = N * N, PP = 4 * NN;
    const int Lx = g.L[0];
    const size_t slot = (size_t)4 * g.B * Lx * PP;
    const size_t gid = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) * P;
    if (gid >= (size_t)4 * Lx * PP) return;
    // PP is even, so the P points share (c, kx) and one quadrant row
    const int pl = (int)(gid / PP), e = (int)(gid - (size_t)pl * PP);
    const int kx = pl >> 2, c = pl & 3;
    const int gx = g.N[0] + 1, gg = N + 1;
    const size_t gsz = (size_t)2 * gx * gg * gg;
    // all loads unconditional (dead terms read a live address and are
    // zeroed), so that the compiler issues them back to back
    const R sg = conj_g ? R(-1) : R(1);
    cplx<R> gr[NGX + 1][P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int ee = e + p, qq = ee / NN, rr = ee - qq * NN;
        const size_t gp = ((size_t)(c == 3 ? 1 : 0) * gx + fold(kx, Lx)) * (size_t)(gg * gg) +
                          fold(2 * (rr / N) + (qq >> 1), 2 * N) * gg + fold(2 * (rr % N) + (qq & 1), 2 * N);
#pragma unroll
        for (int m = 1; m <= NGX; ++m) {
            const R mk = m <= ng ? R(1) : R(0);
            const cplx<R> v = G[(size_t)(m <= ng ? m : ng) * gsz + gp];
            gr[m][p] = cplx<R>{v.x * mk, v.y * (sg * mk)};
        }
    }
    for (int b = 0; b < g.B; ++b) {
        const size_t off = ((size_t)(4 * b + c) * Lx + kx) * PP + e;
        cplx<R> acc[kFarMaxBlock][P];
#pragma unroll
        for (int j = 0; j < kFarMaxBlock; ++j)
#pragma unroll
            for (int p = 0; p < P; ++p) acc[j][p] = cplx<R>{0, 0};
        // history step h = r0 - hp feeds output j through m = j + hp (the
        // outputs j >= pb accumulate dead sums and are not stored); the slots
        // are loaded eight at a time ahead of their products
        constexpr int CH = 8;
#pragma unroll
        for (int hp0 = 1; hp0 <= NGX; hp0 += CH) {
            if (hp0 > ng) break;
            cplx<R> q[CH][P];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int hp = hp0 + u < ng ? hp0 + u : ng;
                const int h = r0 - hp;
                const V t = __builtin_nontemporal_load(
                    reinterpret_cast<const V*>(ring + (size_t)((h > 0 ? h : 0) % ng) * slot + off));
#pragma unroll
                for (int p = 0; p < P; ++p) q[u][p] = cplx<R>{t[2 * p], t[2 * p + 1]};
                if (h < 0 || hp0 + u > ng)
#pragma unroll
                    for (int p = 0; p < P; ++p) q[u][p] = cplx<R>{0, 0};
            }
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int j = 0; j < kFarMaxBlock; ++j) {
                    const int m = j + hp0 + u;
                    if (m <= NGX)
#pragma unroll
                        for (int p = 0; p < P; ++p) acc[j][p] += cmul_fma(gr[m][p], q[u][p]);
                }
        }
#pragma unroll
        for (int j = 0; j < kFarMaxBlock; ++j)
            if (j < pb) {
                V t;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    t[2 * p] = acc[j][p].x;
                    t[2 * p + 1] = acc[j][p].y;
                }
                __builtin_nontemporal_store(t, reinterpret_cast<V*>(F + (size_t)j * slot + off));
            }
    }
}

// Time-block pass of the line-pass engine (spectrum slots [bc][kx][kz][ky]):
// F[j] = sum_{hp=1}^{min(ng, r0)} G_{j+hp} . ring slot (r0 - hp) mod ng for
// the pb steps r0 + j of a block (terms with j + hp > ng dropped).  A thread
// owns one 16-byte vector of points of one component, kx and kz and loops
// over the batch, so that its Green values are loaded once for all columns;
// history slots are loaded eight at a time ahead of their products.
template <typename R, int NGX>
__global__ void __launch_bounds__(256) k_ring_far3(const cplx<R>* __restrict__ ring, const cplx<R>* __restrict__ G,
                                                   cplx<R>* __restrict__ F, GridDims g, int ng, int r0, int pb,
                                                   int conj_g) {
    using V = typename Vec16<R>::type;
    constexpr int P = Vec16<R>::P;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    const size_t plane = (size_t)Ly * Lz, col = 4 * (size_t)Lx * plane, slot = (size_t)g.B * col;
    const size_t gid = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) * P;
    if (gid >= col) return;
    // Ly is even, so the P points share one (c, kx, kz) row
    const size_t pl = gid / plane;
    const int r = (int)(gid - pl * plane), kz = r / Ly, ky = r - kz * Ly;
    const int kx = (int)(pl % Lx), c = (int)(pl / Lx);
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    const size_t gsz = (size_t)2 * gx * gy * gz;
    const size_t goff = (((size_t)(c == 3 ? 1 : 0) * gx + fold(kx, Lx)) * gz + fold(kz, Lz)) * gy;
    const R sg = conj_g ? R(-1) : R(1);
    cplx<R> gr[NGX + 1][P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int fy = fold(ky + q, Ly);
#pragma unroll
        for (int m = 1; m <= NGX; ++m) {
            const R mk = m <= ng ? R(1) : R(0);
            const cplx<R> v = G[(size_t)(m <= ng ? m : ng) * gsz + goff + fy];
            gr[m][q] = cplx<R>{v.x * mk, v.y * (sg * mk)};
        }
    }
    for (int b = 0; b < g.B; ++b) {
        const size_t off = (size_t)b * col + gid;
        cplx<R> acc[kFarMaxBlock][P];
#pragma unroll
        for (int j = 0; j < kFarMaxBlock; ++j)
#pragma unroll
            for (int q = 0; q < P; ++q) acc[j][q] = cplx<R>{0, 0};
        constexpr int CH = 8;
#pragma unroll
        for (int hp0 = 1; hp0 <= NGX; hp0 += CH) {
            if (hp0 > ng) break;
            cplx<R> t[CH][P];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int hp = hp0 + u < ng ? hp0 + u : ng;
                const int h = r0 - hp;
                const V v = __builtin_nontemporal_load(
                    reinterpret_cast<const V*>(ring + (size_t)((h > 0 ? h : 0) % ng) * slot + off));
#pragma unroll
                for (int q = 0; q < P; ++q) t[u][q] = cplx<R>{v[2 * q], v[2 * q + 1]};
                if (h < 0 || hp0 + u > ng)
#pragma unroll
                    for (int q = 0; q < P; ++q) t[u][q] = cplx<R>{0, 0};
            }
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int j = 0; j < kFarMaxBlock; ++j) {
                    const int m = j + hp0 + u;
                    if (m <= NGX)
#pragma unroll
                        for (int q = 0; q < P; ++q) acc[j][q] += cmul_fma(gr[m][q], t[u][q]);
                }
        }
#pragma unroll
        for (int j = 0; j < kFarMaxBlock; ++j)
            if (j < pb) {
                V v;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    v[2 * q] = acc[j][q].x;
                    v[2 * q + 1] = acc[j][q].y;
                }
                __builtin_nontemporal_store(v, reinterpret_cast<V*>(F + (size_t)j * slot + off));
            }
    }
}

// ---------------------------------------------------------------------------
// Multilevel time blocks of the delayed field: the temporal direction of the
// blocked space-time transforms that evaluate the right-hand side of eq. (5)
// (Sec. 4).  The lags m >= kMlBase of the history sum are split into levels
// k = 0, 1, ... holding the lags [S_k, 2 S_k), S_k = kMlBase 2^k; the lags
// below kMlBase are summed directly at each step.  Once steps e - S_k + 1
// .. e are in the ring (e + 1 a multiple of S_k), level k forms its share of
// the sums of the next S_k steps,
//   acc[e + 1 + t] += sum_{u=0}^{S_k-1} G_{S_k+u} s_{e+1+t-S_k-u},  t < S_k,
// as the valid half of a length-2S_k circular convolution (overlap-save) of
// the window s_{e-2S_k+1 .. e} with the zero-padded lag segment: a forward
// register DFT of the window, the product with the segment's DFT (set up
// once, 1/(2 S_k) folded in), an inverse DFT.  A step moves O(log N_g)
// spectra and spends O(log^2 N_g) flops per point instead of N_g of each.
// Window steps below 0, or older than the ring (e - h >= ng: they meet only
// lags beyond ng), enter as zeros.  The accumulator ring has na = S_top
// slots (step l in slot l mod na): the top level's pass is the first to
// reach every step and writes its sums, the lower levels add theirs.
// Lags from 2 S_top = 96 on are taken by further segments of the top
// length, segment j (j >= 1) holding the lags [S_top (j + 1), S_top (j + 2)):
// the same overlap-save pass over a window that ends S_top j steps earlier.
constexpr int kMlBase = 3, kMlLevels = 5;  // S = 3, 6, 12, 24, 48: lags up to 95
constexpr int kMlExtraMax = 20;            // further 48-step segments: lags up to 1055
// levels passed together in one sweep (their windows nest), the rest alone
constexpr int kMlFused = 3;
__host__ __device__ constexpr int ml_s(int k) { return kMlBase << k; }
// first of level k's 2 S_k segment spectra in the level table; the further
// segments j >= 1 of the top length follow the five levels
__host__ __device__ constexpr int ml_off(int k) { return k == 0 ? 0 : ml_off(k - 1) + 2 * ml_s(k - 1); }
__host__ __device__ constexpr int ml_off_extra(int j) { return ml_off(kMlLevels) + 2 * ml_s(kMlLevels - 1) * (j - 1); }
// the largest history the levels and the further segments reach
__host__ __device__ constexpr int ml_max_ng() { return ml_s(kMlLevels - 1) * (kMlExtraMax + 2) - 1; }

template <typename R, int M>
__device__ __forceinline__ void ml_dft(cplx<R> (&u)[M], bool inverse) {
    if constexpr (M == 96) {
        // two interleaved 48-point transforms and one radix-2 stage
        cplx<R> ev[48], od[48];
#pragma unroll
        for (int n = 0; n < 48; ++n) {
            ev[n] = u[2 * n];
            od[n] = u[2 * n + 1];
        }
        dft_small<R, 48>(ev, inverse);
        dft_small<R, 48>(od, inverse);
#pragma unroll
        for (int k = 0; k < 48; ++k) {
            const cplx<R> t = tw96_mul<R>(od[k], k, inverse);
            u[k] = ev[k] + t;
            u[k + 48] = cplx<R>{ev[k].x - t.x, ev[k].y - t.y};
        }
    } else {
        dft_small<R, M>(u, inverse);
    }
}

// folded Green-table index of spectrum point `off` of a ring slot: plain
// slots [bc][kx][kz][ky] (QN = 0) or parity quadrants [bc][kx][quadrant
// rows] of a 2QN x 2QN plane (QN = N of the register engines)
template <int QN>
__device__ __forceinline__ size_t ml_gidx(size_t off, const GridDims& g) {
    const int Lx = g.L[0], gx = g.N[0] + 1;
    if constexpr (QN == 0) {
        const int Ly = g.L[1], Lz = g.L[2];
        const size_t plane = (size_t)Ly * Lz, pl = off / plane;
        const int r = (int)(off - pl * plane), kz = r / Ly, ky = r - kz * Ly;
        const int kx = (int)(pl % Lx), c = (int)((pl / Lx) & 3);
        const int gy = g.N[1] + 1, gz = g.N[2] + 1;
        return (((size_t)(c == 3 ? 1 : 0) * gx + fold(kx, Lx)) * gz + fold(kz, Lz)) * gy + fold(ky, Ly);
    } else {
        constexpr int NN = QN * QN, PP = 4 * NN, gg = QN + 1;
        const size_t pl = off / PP;
        const int e = (int)(off - pl * PP), qq = e / NN, rr = e - qq * NN;
        const int kx = (int)(pl % Lx), c = (int)((pl / Lx) & 3);
        return ((size_t)(c == 3 ? 1 : 0) * gx + fold(kx, Lx)) * (size_t)(gg * gg) +
               fold(2 * (rr / QN) + (qq >> 1), 2 * QN) * gg + fold(2 * (rr % QN) + (qq & 1), 2 * QN);
    }
}

// one complex value as an 8- or 16-byte vector, for streaming (non-temporal)
// loads and stores
template <typename R>
struct CVec;
template <>
struct CVec<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct CVec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <typename R>
__device__ __forceinline__ cplx<R> nt_load(const cplx<R>* p) {
    const typename CVec<R>::type v = __builtin_nontemporal_load(reinterpret_cast<const typename CVec<R>::type*>(p));
    return cplx<R>{v[0], v[1]};
}
template <typename R>
__device__ __forceinline__ void nt_store(cplx<R>* p, cplx<R> c) {
    typename CVec<R>::type v;
    v[0] = c.x;
    v[1] = c.y;
    __builtin_nontemporal_store(v, reinterpret_cast<typename CVec<R>::type*>(p));
}

// level K's sums from the tail of the window (its own 2 S_K steps), added
// into out[t], t < S_K; then the next level up to K1
template <typename R, int K, int K1, int W, int S1>
__device__ __forceinline__ void ml_levels(const cplx<R> (&win)[W], cplx<R> (&out)[S1], const cplx<R>* __restrict__ gam,
                                          size_t gstride, size_t gi) {
    constexpr int S = ml_s(K), M = 2 * S;
    cplx<R> u[M];
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = win[W - M + j];
    ml_dft<R, M>(u, false);
#pragma unroll
    for (int w = 0; w < M; ++w) u[w] = cmul_fma(u[w], gam[(size_t)(ml_off(K) + w) * gstride + gi]);
    ml_dft<R, M>(u, true);
#pragma unroll
    for (int t = 0; t < S; ++t) out[t] += u[S + t];
    if constexpr (K < K1) ml_levels<R, K + 1, K1, W, S1>(win, out, gam, gstride, gi);
}

// The passes of levels K0..K1 at step e in one sweep, one spectrum point per
// thread (slot = points of a ring slot, gstride = folded points per lag of
// the tables, gam = the level table; a further segment: K0 = K1 = the top
// level, gam shifted so that its spectra stand where the top level's do,
// dly = its delay S_top j): the window of the last 2 S_K1 spectra
// serves every level, their sums are added in registers (K0 first) to the
// accumulator slots of steps e + 1 .. e + S_K1, which are loaded with the
// window (first: the top level is K1, whose sums start those slots).  Sums of steps below lo
// are not written (a rebuild from the ring at step lo passes the levels'
// last blocks, whose earlier steps are already consumed).  conj_g: the sum
// with conj(G) (adjoint march), as conj of the sum with G over the
// conjugated history.
template <typename R, int K0, int K1, int QN>
__global__ void __launch_bounds__(256) k_ml_pass(const cplx<R>* __restrict__ ring, const cplx<R>* __restrict__ gam,
                                                 cplx<R>* __restrict__ acc, GridDims g, size_t slot, size_t gstride,
                                                 int ng, int e, int na, int conj_g, int first, int lo,
                                                 int dly) {
    constexpr int S1 = ml_s(K1), W = 2 * S1;
    const size_t off = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (off >= slot) return;
    const size_t gi = ml_gidx<QN>(off, g);
    const R sg = conj_g ? R(-1) : R(1);
    cplx<R> win[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int h = e - dly - W + 1 + j;
        cplx<R> v{0, 0};
        if (h >= 0 && e - h < ng) v = nt_load(ring + (size_t)(h % ng) * slot + off);
        win[j] = cplx<R>{v.x, sg * v.y};
    }
    // the accumulators, conjugated with the window where conj_g is set
    cplx<R> out[S1];
#pragma unroll
    for (int t = 0; t < S1; ++t) {
        cplx<R> a{0, 0};
        if (!first && e + 1 + t >= lo) a = nt_load(acc + (size_t)((e + 1 + t) % na) * slot + off);
        out[t] = cplx<R>{a.x, sg * a.y};
    }
    ml_levels<R, K0, K1, W, S1>(win, out, gam, gstride, gi);
#pragma unroll
    for (int t = 0; t < S1; ++t)
        if (e + 1 + t >= lo)
            nt_store(acc + (size_t)((e + 1 + t) % na) * slot + off, cplx<R>{out[t].x, sg * out[t].y});
}

// The level tables: gam[ml_off(k) + w][q] = (1/M) sum_{u<S} G_{S+u}[q]
// exp(-2 pi i w u / M), M = 2 S = 2 S_k, for every folded point q, with
// G_m = 0 beyond m = ng (FP64 arithmetic on the FP64 Green table); the
// further segments j at ml_off_extra(j), from G_{S_top (j + 1) + u}.
template <typename R>
__global__ void k_ml_gamma(const zd* __restrict__ G, cplx<R>* __restrict__ gam, size_t gstride, int ng, int nlev,
                           int nextra) {
    const size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (q >= gstride) return;
    // levels k < nlev (lag base S_k), then the further segments j = 1..nextra
    // (lag base S_top (j + 1)), each 2 S spectra of its S lags
    for (int k = 0; k < nlev + nextra; ++k) {
        const int top = k >= nlev;
        const int S = top ? ml_s(kMlLevels - 1) : ml_s(k), M = 2 * S;
        const int base = top ? S * (k - nlev + 2) : S;
        const int off = top ? ml_off_extra(k - nlev + 1) : ml_off(k);
        for (int w = 0; w < M; ++w) {
            double re = 0, im = 0;
            for (int u = 0; u < S && base + u <= ng; ++u) {
                double sn, cs;
                sincospi(-2.0 * (double)((w * u) % M) / (double)M, &sn, &cs);
                const zd v = G[(size_t)(base + u) * gstride + q];
                re += v.x * cs - v.y * sn;
                im += v.x * sn + v.y * cs;
            }
            gam[(size_t)(off + w) * gstride + q] = cplx<R>{(R)(re / M), (R)(im / M)};
        }
    }
}

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Interpolation + near-zone SpMV, one wavefront per basis k, all columns b.
// mode 0 (matvec):  y[b][k] = sum_c sum_j L[k][c][j] P[bc][node_j]
//                              + sum_e val[e][m] xr[col_e][b]
// mode 1 (delayed): y[b][k] = V[b][k] - (interp(P) + sum_{m=1}^{nmh}
//                              val[e][m] hist[(cur-m) mod mn][col_e][b])
// mode 2: y[b][k] += interp(P);  mode 3: y[b][k] -= interp(P)  (no near
// zone: the CFIE's MFIE far part, lam then its curl test projection)
// xr = the scaled columns dinv . x and hist the current history, both in
// the working precision with the columns of one basis contiguous ([ns][B]).
// Lane j of the wave owns stencil node j (and near-zone entries e0 + j,
// e0 + j + 64, ...) for up to kInterpCols columns at once; the 64-lane sums
// of all columns then take one transposing butterfly (each exchange halves
// the columns a lane carries) instead of one full reduction per column.
constexpr int kInterpCols = 32;

template <typename R>
__global__ void __launch_bounds__(256) k_interp_near(
    const cplx<R>* __restrict__ P, const R* __restrict__ lam, const int* __restrict__ i0,
    const int* __restrict__ order, GridDims g,
    const int* __restrict__ rowptr, const int* __restrict__ col, const cplx<R>* __restrict__ val, int mv,
    const cplx<R>* __restrict__ xr, int m, const cplx<R>* __restrict__ hist, int mn, int cur,
    int nmh, const zd* __restrict__ V, zd* __restrict__ y, int ns, int mode, int conj_v,
    const int* __restrict__ gate, StepRef sr = {}) {
    if (gated_off(gate) || step_off(sr)) return;
    if (const StepDesc* d = step_of(sr)) {
        // replayed delayed field: this step's excitation from the call's array
        cur = d->cur;
        nmh = d->nmh;
        V = d->V + (size_t)d->cur * g.B * ns;
    }
    const int lane = threadIdx.x & 63;
    // consecutive blocks land on different XCDs (round-robin dispatch), so
    // give each XCD one contiguous run of the Morton-ordered bases: its L2
    // then holds one surface patch of the grid
    const int per = gridDim.x / kXcds;
    const int lb = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int slot = lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slot >= ns) return;
    const int k = order[slot];
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2], B = g.B;
    const size_t N = (size_t)Nx * Ny * Nz;
    // P is [bc][z][x][y]: lanes take the stencil with y fastest (32-byte runs)
    const int jy = lane & 3, jx = (lane >> 2) & 3, jz = lane >> 4, j = jx + 4 * jy + 16 * jz;
    const size_t node = (size_t)(i0[3 * k + 1] + jy) + (size_t)Ny * ((size_t)(i0[3 * k] + jx) + (size_t)Nx * (i0[3 * k + 2] + jz));
    R w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = lam[(size_t)k * 256 + 64 * c + j];
    const int e0 = rowptr[k], e1 = mode >= 2 ? e0 : rowptr[k + 1];
    for (int b0 = 0; b0 < B; b0 += kInterpCols) {
        const int nb = min(kInterpCols, B - b0);
        cplx<R> acc[kInterpCols];
#pragma unroll
        for (int bb = 0; bb < kInterpCols; ++bb) {
            acc[bb] = cplx<R>{0, 0};
            if (bb < nb) {
                const cplx<R>* pb = P + (size_t)(b0 + bb) * 4 * N + node;
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[bb] += w[c] * pb[(size_t)c * N];
            }
        }
        // near zone: lane = (entry slot, column) with the columns innermost, so
        // that the lanes of one entry read one coalesced run of its basis's
        // columns and share the entry's loads
        int C = 1;
        while (C < nb) C <<= 1;
        const int E = 64 / C, bcol = lane & (C - 1), eslot = lane / C;
        cplx<R> nacc{0, 0};
        // four entries per slot at a time, their loads issued together
        constexpr int U = 4;
        for (int e = e0 + eslot; e < e1; e += U * E) {
            int cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cc[u] = e + u * E < e1 ? col[e + u * E] : -1;
            if (mode == 0) {
                if (m <= mv - 1) {
                    cplx<R> v[U], xv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        v[u] = cplx<R>{0, 0};
                        xv[u] = cplx<R>{0, 0};
                        if (cc[u] >= 0) {
                            v[u] = val[(size_t)(e + u * E) * mv + m];
                            if (bcol < nb) xv[u] = xr[(size_t)cc[u] * B + b0 + bcol];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (conj_v) v[u].y = -v[u].y;
                        nacc += v[u] * xv[u];
                    }
                }
            } else {
                for (int mm = 1; mm <= nmh; ++mm) {
                    int s = (cur - mm) % mn;
                    if (s < 0) s += mn;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (cc[u] < 0) continue;
                        cplx<R> v = val[(size_t)(e + u * E) * mv + mm];
                        if (conj_v) v.y = -v.y;
                        if (bcol < nb) nacc += v * hist[((size_t)s * ns + cc[u]) * B + b0 + bcol];
                    }
                }
            }
        }
        // sum over the entry slots: every lane then holds its column's total
        for (int o = C; o < 64; o <<= 1) {
            nacc.x += __shfl_xor(nacc.x, o, 64);
            nacc.y += __shfl_xor(nacc.y, o, 64);
        }
        // transposing butterfly over the top log2(kInterpCols) lane bits: after
        // the exchange over a bit a lane keeps half its partial sums, those of
        // the half its bit selects; the lower bits then pair up, and the GL
        // lanes GL bb + {0 .. GL - 1} hold the full sum of column bb
        constexpr int GL = 64 / kInterpCols;
#pragma unroll
        for (int h = kInterpCols / 2, bit = 32; h >= 1; h >>= 1, bit >>= 1) {
            const bool up = (lane & bit) != 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const cplx<R> keep = up ? acc[i + h] : acc[i];
                const cplx<R> send = up ? acc[i] : acc[i + h];
                acc[i] = keep + cplx<R>{__shfl_xor(send.x, bit, 64), __shfl_xor(send.y, bit, 64)};
            }
        }
        cplx<R> tot = acc[0];
#pragma unroll
        for (int bit = GL / 2; bit >= 1; bit >>= 1)
            tot += cplx<R>{__shfl_xor(tot.x, bit, 64), __shfl_xor(tot.y, bit, 64)};
        const int bb = lane / GL;
        // the near-zone total of column bb sits in lane bb (entry slot 0)
        const cplx<R> near{__shfl(nacc.x, bb, 64), __shfl(nacc.y, bb, 64)};
        tot += near;
        if (lane % GL == 0 && bb < nb) {
            const size_t o = (size_t)(b0 + bb) * ns + k;
            if (mode == 0)
                y[o] = zd{(double)tot.x, (double)tot.y};
            else if (mode == 1)
                y[o] = zd{V[o].x - (double)tot.x, V[o].y - (double)tot.y};
            else if (mode == 2)
                y[o] = zd{y[o].x + (double)tot.x, y[o].y + (double)tot.y};
            else
                y[o] = zd{y[o].x - (double)tot.x, y[o].y - (double)tot.y};
        }
    }
}

// Interpolation + near-zone SpMV by grid tiles (the same sums as
// k_interp_near).  The bases are grouped by the tile of their stencil
// corner (kTileX x kTileY x kTileZ corners); a block takes one tile and a
// group of GC columns: it loads the tile's node box (the corners plus the
// stencil's 3-node reach, y fastest, so that the loads are runs of kBoxY
// nodes) of the 4 GC potential planes into LDS, then its waves take the
// tile's bases one by one as k_interp_near does, lane j on stencil node j,
// reading the potentials from LDS.  Blocks run tile-fastest within a column
// group, each XCD a contiguous run of the Morton-ordered tiles.
constexpr int kTileX = 4, kTileY = 8, kTileZ = 4;
constexpr int kBoxX = kTileX + 3, kBoxY = kTileY + 3, kBoxZ = kTileZ + 3, kBoxN = kBoxX * kBoxY * kBoxZ;

constexpr int kTileThreads = 1024;

template <typename R, int GC>
__global__ void __launch_bounds__(kTileThreads) k_interp_tile(
    const cplx<R>* __restrict__ P, const R* __restrict__ lam, const int* __restrict__ i0,
    const int* __restrict__ tptr, const int* __restrict__ tbase, const int* __restrict__ torg, int ntiles,
    GridDims g, const int* __restrict__ rowptr, const int* __restrict__ col, const cplx<R>* __restrict__ val,
    int mv, const cplx<R>* __restrict__ xr, int m, const cplx<R>* __restrict__ hist, int mn, int cur, int nmh,
    const zd* __restrict__ V, zd* __restrict__ y, int ns, int mode, int conj_v, const int* __restrict__ gate,
    StepRef sr) {
    if (gated_off(gate) || step_off(sr)) return;
    if (const StepDesc* d = step_of(sr)) {
        cur = d->cur;
        nmh = d->nmh;
        V = d->V + (size_t)d->cur * g.B * ns;
    }
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* box = reinterpret_cast<cplx<R>*>(smem_raw);
    // block -> (column group, tile): each XCD (round-robin dispatch) gets one
    // contiguous run of the logical blocks
    const int per = gridDim.x / kXcds;
    const int lb = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const int ngroups = (g.B + GC - 1) / GC;
    if (lb >= ntiles * ngroups) return;
    const int t = lb % ntiles, b0 = (lb / ntiles) * GC;
    const int nb = min(GC, g.B - b0);
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2], B = g.B;
    const size_t N = (size_t)Nx * Ny * Nz;
    const int ox = torg[3 * t], oy = torg[3 * t + 1], oz = torg[3 * t + 2];
    // the box as rows of kBoxY y-nodes, one row per 16 lanes (y = lane % 16):
    // each load instruction takes four coalesced runs
    constexpr int ROWS = 4 * GC * kBoxZ * kBoxX;
    for (int e = threadIdx.x; e < ROWS * 16; e += blockDim.x) {
        const int ly = e & 15, row = e >> 4;
        if (ly >= kBoxY) continue;
        const int lx = row % kBoxX, r2 = row / kBoxX, lz = r2 % kBoxZ, bcl = r2 / kBoxZ;
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        cplx<R> v{0, 0};
        if (bcl < 4 * nb && gx < Nx && gy < Ny && gz < Nz)
            v = P[(size_t)(4 * b0 + bcl) * N + (size_t)gy + (size_t)Ny * ((size_t)gx + (size_t)Nx * gz)];
        box[row * kBoxY + ly] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int jy = lane & 3, jx = (lane >> 2) & 3, jz = lane >> 4, j = jx + 4 * jy + 16 * jz;
    // near zone: lane = (entry slot, column), columns innermost
    constexpr int C = GC, E = 64 / GC, GL = 64 / GC;
    const int bcol = lane & (C - 1), eslot = lane / C;
    for (int q = tptr[t] + wave; q < tptr[t + 1]; q += nw) {
        const int k = tbase[q];
        const int lx = i0[3 * k] - ox + jx, ly = i0[3 * k + 1] - oy + jy, lz = i0[3 * k + 2] - oz + jz;
        const int o = (lz * kBoxX + lx) * kBoxY + ly;
        R w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) w[c] = lam[(size_t)k * 256 + 64 * c + j];
        cplx<R> acc[GC];
#pragma unroll
        for (int bb = 0; bb < GC; ++bb) {
            acc[bb] = cplx<R>{0, 0};
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[bb] += w[c] * box[(size_t)(4 * bb + c) * kBoxN + o];
        }
        cplx<R> nacc{0, 0};
        const int e0 = rowptr[k], e1 = rowptr[k + 1];
        constexpr int U = 4;
        for (int e = e0 + eslot; e < e1; e += U * E) {
            int cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cc[u] = e + u * E < e1 ? col[e + u * E] : -1;
            if (mode == 0) {
                if (m <= mv - 1) {
                    cplx<R> v[U], xv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        v[u] = cplx<R>{0, 0};
                        xv[u] = cplx<R>{0, 0};
                        if (cc[u] >= 0) {
                            v[u] = val[(size_t)(e + u * E) * mv + m];
                            if (bcol < nb) xv[u] = xr[(size_t)cc[u] * B + b0 + bcol];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (conj_v) v[u].y = -v[u].y;
                        nacc += v[u] * xv[u];
                    }
                }
            } else {
                for (int mm = 1; mm <= nmh; ++mm) {
                    int sl = (cur - mm) % mn;
                    if (sl < 0) sl += mn;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (cc[u] < 0) continue;
                        cplx<R> v = val[(size_t)(e + u * E) * mv + mm];
                        if (conj_v) v.y = -v.y;
                        if (bcol < nb) nacc += v * hist[((size_t)sl * ns + cc[u]) * B + b0 + bcol];
                    }
                }
            }
        }
        for (int sft = C; sft < 64; sft <<= 1) {
            nacc.x += __shfl_xor(nacc.x, sft, 64);
            nacc.y += __shfl_xor(nacc.y, sft, 64);
        }
        // transposing butterfly over the top log2(GC) lane bits, then the GL
        // lanes of each column group summed: lane GL bb + i holds column bb
#pragma unroll
        for (int h = GC / 2, bit = 32; h >= 1; h >>= 1, bit >>= 1) {
            const bool up = (lane & bit) != 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const cplx<R> keep = up ? acc[i + h] : acc[i];
                const cplx<R> send = up ? acc[i] : acc[i + h];
                acc[i] = keep + cplx<R>{__shfl_xor(send.x, bit, 64), __shfl_xor(send.y, bit, 64)};
            }
        }
        cplx<R> tot = acc[0];
#pragma unroll
        for (int bit = GL / 2; bit >= 1; bit >>= 1)
            tot += cplx<R>{__shfl_xor(tot.x, bit, 64), __shfl_xor(tot.y, bit, 64)};
        const int bb = lane / GL;
        const cplx<R> near{__shfl(nacc.x, bb, 64), __shfl(nacc.y, bb, 64)};
        tot += near;
        if (lane % GL == 0 && bb < nb) {
            const size_t oo = (size_t)(b0 + bb) * ns + k;
            if (mode == 0)
                y[oo] = zd{(double)tot.x, (double)tot.y};
            else
                y[oo] = zd{V[oo].x - (double)tot.x, V[oo].y - (double)tot.y};
        }
    }
}

// ---------------------------------------------------------------------------
// Set-up kernels (FP64): Green tables, circulant embedding, folding,
// pre-correction, excitation.

// G[m][t][k][j][i] for |offset| (i,j,k) < (Nx,Ny,Nz); t = 0: (mu/4pi) fA/R,
// t = 1: (1/4 pi eps) fphi/R; zero at the origin.  With a BLIF the
// non-causal m = -1..-nk fold into m < np: G~_m = G_m + sum_k a[k-1][m] G_{-k}.
__global__ void k_green_table(zd* __restrict__ G, GridDims g, int ng, double h, EnvKernel K, double sa,
                              double sp, TFold fo) {
    const size_t n3 = (size_t)g.N[0] * g.N[1] * g.N[2];
    const size_t tot = (size_t)(ng + 1) * n3;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(e / n3);
        const size_t r = e - (size_t)m * n3;
        const int i = (int)(r % g.N[0]);
        const int j = (int)((r / g.N[0]) % g.N[1]);
        const int k = (int)(r / ((size_t)g.N[0] * g.N[1]));
        const double R = h * sqrt((double)(i * i + j * j + k * k));
        zd a{0, 0}, p{0, 0};
        if (R != 0.0) {
            zd fa, fp;
            K.eval(m, R, fa, fp);
            a = (sa / R) * fa;
            p = (sp / R) * fp;
            if (m < fo.np)
                for (int kf = 1; kf <= fo.nk; ++kf) {
                    K.eval(-kf, R, fa, fp);
                    a += (fo.a[kf - 1][m] * sa / R) * fa;
                    p += (fo.a[kf - 1][m] * sp / R) * fp;
                }
        }
        G[((size_t)m * 2 + 0) * n3 + r] = a;
        G[((size_t)m * 2 + 1) * n3 + r] = p;
    }
}

// CFIE: G[m][0][k][j][i] = scale exp(-j k R) [T'/dt + j w T](tau) / (4 pi R)
// (the MFIE's potential, zero at the origin), G[m][1] = 0
__global__ void k_green_table_h(zd* __restrict__ G, GridDims g, int ng, double h, EnvKernel K, double scale,
                                TFold fo) {
    const size_t n3 = (size_t)g.N[0] * g.N[1] * g.N[2];
    const size_t tot = (size_t)(ng + 1) * n3;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(e / n3);
        const size_t r = e - (size_t)m * n3;
        const int i = (int)(r % g.N[0]);
        const int j = (int)((r / g.N[0]) % g.N[1]);
        const int k = (int)(r / ((size_t)g.N[0] * g.N[1]));
        const double R = h * sqrt((double)(i * i + j * j + k * k));
        zd v{0, 0};
        if (R != 0.0) {
            zd fa, fh;
            K.evalh(m, R, fa, fh);
            v = (scale / (4.0 * kPi * R)) * fh;
            if (m < fo.np)
                for (int kf = 1; kf <= fo.nk; ++kf) {
                    K.evalh(-kf, R, fa, fh);
                    v += (fo.a[kf - 1][m] * scale / (4.0 * kPi * R)) * fh;
                }
        }
        G[((size_t)m * 2 + 0) * n3 + r] = v;
        G[((size_t)m * 2 + 1) * n3 + r] = zd{0, 0};
    }
}

// circulant embedding of one |offset| table into the padded [Lz][Ly][Lx] grid
__global__ void k_circulant(const zd* __restrict__ tab, zd* __restrict__ out, GridDims g) {
    const size_t tot = (size_t)g.L[0] * g.L[1] * g.L[2];
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % g.L[0]);
        const int y = (int)((e / g.L[0]) % g.L[1]);
        const int z = (int)(e / ((size_t)g.L[0] * g.L[1]));
        zd v{0, 0};
        if (x != g.N[0] && y != g.N[1] && z != g.N[2]) {
            const int i = x < g.N[0] ? x : g.L[0] - x;
            const int j = y < g.N[1] ? y : g.L[1] - y;
            const int k = z < g.N[2] ? z : g.L[2] - z;
            v = tab[((size_t)k * g.N[1] + j) * g.N[0] + i];
        }
        out[e] = v;
    }
}

// keep the unique octant (k <= N per axis) of a padded spectrum [kz][ky][kx],
// scaled, in the plane-major layout out[kx'][kz'][ky']
__global__ void k_fold(const zd* __restrict__ full, zd* __restrict__ out, GridDims g, double scale) {
    const int gx = g.N[0] + 1, gy = g.N[1] + 1, gz = g.N[2] + 1;
    const size_t tot = (size_t)gx * gy * gz;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(e % gy);
        const int z = (int)((e / gy) % gz);
        const int x = (int)(e / ((size_t)gy * gz));
        const zd v = full[((size_t)z * g.L[1] + y) * g.L[0] + x];
        out[e] = zd{v.x * scale, v.y * scale};
    }
}

// Pre-correction: val[e][m] = exact[e][m] - sum_c sum_{n,n'} L[k][c][n]
//   G_m^c[|node_n - node_n'|] L[k'][c][n'] for every near pair e = (k, k').
// CFIE (lamH set): minus also sum_{c<3} sum_{n,n'} H[k][c][n] GH_m[..] L[k'][c][n'].
// One wavefront per pair; lane = local node n of k.
__global__ void __launch_bounds__(64) k_precorrect(zd* __restrict__ val, const double* __restrict__ lam,
                                                   const int* __restrict__ i0, const int* __restrict__ rowof,
                                                   const int* __restrict__ col, const zd* __restrict__ G,
                                                   GridDims g, int mv, int nnz, const double* __restrict__ lamH,
                                                   const zd* __restrict__ GH) {
    __shared__ double lk2[256];
    const int e = blockIdx.x;
    if (e >= nnz) return;
    const int lane = threadIdx.x;
    const int k = rowof[e], k2 = col[e];
#pragma unroll
    for (int c = 0; c < 4; ++c) lk2[64 * c + lane] = lam[(size_t)k2 * 256 + 64 * c + lane];
    __syncthreads();
    const int jx = lane & 3, jy = (lane >> 2) & 3, jz = lane >> 4;
    const int ax = i0[3 * k] + jx, ay = i0[3 * k + 1] + jy, az = i0[3 * k + 2] + jz;
    const int bx = i0[3 * k2], by = i0[3 * k2 + 1], bz = i0[3 * k2 + 2];
    double lk[4], hk[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) lk[c] = lam[(size_t)k * 256 + 64 * c + lane];
    if (lamH) {
#pragma unroll
        for (int c = 0; c < 3; ++c) hk[c] = lamH[(size_t)k * 256 + 64 * c + lane];
    }
    const size_t n3 = (size_t)g.N[0] * g.N[1] * g.N[2];
    for (int m = 0; m < mv; ++m) {
        const zd* GA = G + ((size_t)m * 2 + 0) * n3;
        const zd* GP = G + ((size_t)m * 2 + 1) * n3;
        zd acc{0, 0};
        for (int q = 0; q < 64; ++q) {
            const int dx = abs(ax - (bx + (q & 3)));
            const int dy = abs(ay - (by + ((q >> 2) & 3)));
            const int dz = abs(az - (bz + (q >> 4)));
            const size_t off = ((size_t)dz * g.N[1] + dy) * g.N[0] + dx;
            const zd ga = GA[off], gp = GP[off];
            const double sA = lk[0] * lk2[q] + lk[1] * lk2[64 + q] + lk[2] * lk2[128 + q];
            const double sP = lk[3] * lk2[192 + q];
            acc += sA * ga;
            acc += sP * gp;
            if (lamH) {
                const double sH = hk[0] * lk2[q] + hk[1] * lk2[64 + q] + hk[2] * lk2[128 + q];
                acc += sH * GH[((size_t)m * 2) * n3 + off];
            }
        }
        const double re = wave_sum<double>(acc.x), im = wave_sum<double>(acc.y);
        if (lane == 0) {
            zd& v = val[(size_t)e * mv + m];
            v = zd{v.x - re, v.y - im};
        }
    }
}

// Plane-wave excitation, eq. (1) with (d/dt + j w) applied:
// V[l][b][k] = sum_{half,q} (Sq . p) [g'(tau) + j w g(tau)] exp(-j w (r.k/c + td))
// Sq[k][h][q][3]: quadrature-weighted basis values; rq: points.
// CFIE (Snq set): the projection is alpha (Sq . p) + (1 - alpha) (Snq . (khat x p)),
// Snq = the weighted S x n, i.e. alpha S . E~ + (1 - alpha) S . (n x (khat x E~))
__global__ void k_excitation(zd* __restrict__ V, const double* __restrict__ Sq, const double* __restrict__ rq,
                             const double* __restrict__ khat, const double* __restrict__ phat, int nt, int nb,
                             int ns, double dt, double sigma, double td, double w, const double* __restrict__ Snq,
                             double alpha) {
    const size_t tot = (size_t)nt * nb * ns;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % ns);
        const int b = (int)((e / ns) % nb);
        const int l = (int)(e / ((size_t)ns * nb));
        const double t = (double)(l + 1) * dt;
        const double* kh = khat + 3 * b;
        const double* ph = phat + 3 * b;
        double sr = 0, si = 0;
        for (int q = 0; q < 14; ++q) {
            const double* S = Sq + ((size_t)k * 14 + q) * 3;
            const double* r = rq + ((size_t)k * 14 + q) * 3;
            const double rk = (r[0] * kh[0] + r[1] * kh[1] + r[2] * kh[2]) / kC0;
            const double tau = t - rk - td;
            const double gg = exp(-tau * tau / (2.0 * sigma * sigma));
            const double dg = -(tau / (sigma * sigma)) * gg;
            double proj = S[0] * ph[0] + S[1] * ph[1] + S[2] * ph[2];
            if (Snq) {
                const double* Sn = Snq + ((size_t)k * 14 + q) * 3;
                const double hx = kh[1] * ph[2] - kh[2] * ph[1], hy = kh[2] * ph[0] - kh[0] * ph[2],
                             hz = kh[0] * ph[1] - kh[1] * ph[0];
                proj = alpha * proj + (1.0 - alpha) * (Sn[0] * hx + Sn[1] * hy + Sn[2] * hz);
            }
            const double arg = w * (rk + td);
            const double c = cos(arg), s = -sin(arg);
            // (dg + j w gg) (c + j s)
            sr += proj * (dg * c - w * gg * s);
            si += proj * (dg * s + w * gg * c);
        }
        V[e] = zd{sr, si};
    }
}

// Far-field operator taps F[tap][d][x][k] (complex128):
//   -(mu/4pi) [I - d d] sum_q Sq[k][q] [T'(tau)/dt + j w T(tau)] exp(j kc d.r_q),
//   tau = (m_lo + tap) + d.r_q/(c dt).
__global__ void k_farfield_taps(zd* __restrict__ F, const double* __restrict__ Sq, const double* __restrict__ rq,
                                const double* __restrict__ dirs, int nd, int ns, int ntap, int m_lo, double dt,
                                double w, double mu4pi, TBasis tb) {
    const size_t tot = (size_t)ntap * nd * ns;
    const double kc = w / kC0, cdt = kC0 * dt;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % ns);
        const int d = (int)((e / ns) % nd);
        const int tap = (int)(e / ((size_t)ns * nd));
        const double* u = dirs + 3 * d;
        double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int q = 0; q < 14; ++q) {
            const double* S = Sq + ((size_t)k * 14 + q) * 3;
            const double* r = rq + ((size_t)k * 14 + q) * 3;
            const double dr = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
            double T[4];
            if (!tb.eval((double)(m_lo + tap) + dr / cdt, T)) continue;
            const double c = cos(kc * dr), s = sin(kc * dr);
            // (T'/dt + j w T) (c + j s)
            const double fr = T[1] / dt * c - w * T[0] * s;
            const double fi = T[1] / dt * s + w * T[0] * c;
            for (int x = 0; x < 3; ++x) {
                acc[x][0] += S[x] * fr;
                acc[x][1] += S[x] * fi;
            }
        }
        // transverse projection and scale
        const double pr = u[0] * acc[0][0] + u[1] * acc[1][0] + u[2] * acc[2][0];
        const double pi = u[0] * acc[0][1] + u[1] * acc[1][1] + u[2] * acc[2][1];
        for (int x = 0; x < 3; ++x) {
            const double vr = acc[x][0] - u[x] * pr, vi = acc[x][1] - u[x] * pi;
            F[(((size_t)tap * nd + d) * 3 + x) * ns + k] = zd{-mu4pi * vr, -mu4pi * vi};
        }
    }
}

// U[l][b][d][x] = sum_tap sum_k F[tap][d][x][k] I[l - (m_lo+tap)][b][k]; block per output.
__global__ void __launch_bounds__(256) k_farfield_apply(zd* __restrict__ U, const zd* __restrict__ F,
                                                        const zd* __restrict__ I, int nt, int B, int nd, int ns,
                                                        int ntap, int m_lo) {
    __shared__ double sh[256];
    const int o = blockIdx.x;  // ((l*B + b)*nd + d)*3 + x
    const int x = o % 3, d = (o / 3) % nd, b = (o / (3 * nd)) % B, l = o / (3 * nd * B);
    double re = 0, im = 0;
    for (int tap = 0; tap < ntap; ++tap) {
        const int j = l - (m_lo + tap);
        if (j < 0 || j >= nt) continue;
        const zd* f = F + (((size_t)tap * nd + d) * 3 + x) * ns;
        const zd* v = I + ((size_t)j * B + b) * ns;
        for (int k = threadIdx.x; k < ns; k += 256) {
            re += f[k].x * v[k].x - f[k].y * v[k].y;
            im += f[k].x * v[k].y + f[k].y * v[k].x;
        }
    }
    sh[threadIdx.x] = re;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double rs = sh[0];
    __syncthreads();
    sh[threadIdx.x] = im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) U[o] = zd{rs, sh[0]};
}

// S[j][b][k] = sum_tap sum_{d,x} conj(F[tap][d][x][k]) U[j + m_lo + tap][b][d][x]
// Co-polarised RCS from far-field envelopes (Sec. 2.4), one thread per
// (frequency i, incidence b, direction d): the envelope's Fourier transform
// at df[i] (samples at t = (l+1) dt), projected on pol[d], over the incident
// Gaussian envelope's transform G[i]: sigma = 4 pi |pol . U(df)|^2 / G^2.
__global__ void k_rcs(double* __restrict__ out, const zd* __restrict__ U, const double* __restrict__ pol,
                      const double* __restrict__ df, const double* __restrict__ G, int nt, int B, int nd, int nf,
                      double dt) {
    const size_t tot = (size_t)nf * B * nd;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int d = (int)(e % nd);
        const size_t r = e / nd;
        const int b = (int)(r % B), i = (int)(r / B);
        const double px = pol[3 * d], py = pol[3 * d + 1], pz = pol[3 * d + 2];
        const double w = -2.0 * kPi * df[i] * dt;
        zd acc{0, 0};
        for (int l = 0; l < nt; ++l) {
            const zd* u = U + (((size_t)l * B + b) * nd + d) * 3;
            const zd v = zd{px * u[0].x + py * u[1].x + pz * u[2].x, px * u[0].y + py * u[1].y + pz * u[2].y};
            double sn, cs;
            sincos(w * (l + 1.0), &sn, &cs);
            acc += v * zd{cs, sn};
        }
        const double a2 = (acc.x * acc.x + acc.y * acc.y) * dt * dt;
        out[e] = 4.0 * kPi * a2 / (G[i] * G[i]);
    }
}

__global__ void k_farfield_adjoint(zd* __restrict__ S, const zd* __restrict__ F, const zd* __restrict__ U, int nt,
                                   int B, int nd, int ns, int ntap, int m_lo) {
    const size_t tot = (size_t)nt * B * ns;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % ns);
        const int b = (int)((e / ns) % B);
        const int j = (int)(e / ((size_t)ns * B));
        double re = 0, im = 0;
        for (int tap = 0; tap < ntap; ++tap) {
            const int l = j + m_lo + tap;
            if (l < 0 || l >= nt) continue;
            for (int d = 0; d < nd; ++d)
                for (int x = 0; x < 3; ++x) {
                    const zd f = F[(((size_t)tap * nd + d) * 3 + x) * ns + k];
                    const zd u = U[(((size_t)l * B + b) * nd + d) * 3 + x];
                    re += f.x * u.x + f.y * u.y;
                    im += f.x * u.y - f.y * u.x;
                }
        }
        S[e] = zd{re, im};
    }
}

}  // namespace etaim
