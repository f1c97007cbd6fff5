// FP64 kernels of right-preconditioned restarted GMRES (Sec. 5.1: diagonally
// preconditioned GMRES), one Krylov space per excitation column b.
// Vectors are [B][ns] complex128; the basis is [restart+1][B][ns].
#pragma once
#include "common.hpp"

namespace etaim {

__device__ __forceinline__ double block_sum256(double v, double* sh) {
    // deterministic tree over a 256-thread block
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Block of the column reductions: 1024 threads, so that the few blocks of
// a reduction (one per column) keep enough loads in flight
constexpr int kRedThreads = 1024;

// deterministic sum over a kRedThreads block, valid in thread 0: a fixed
// butterfly within each wave, then the wave sums in order
__device__ __forceinline__ double block_sum_t0(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kRedThreads / 64; ++q) r += sh[q];
    return r;
}

// h[i][b] = <V_i[b], w[b]> = sum_k conj(V_i[b][k]) w[b][k], i < nv.  grid (nv, B)
__global__ void __launch_bounds__(kRedThreads) k_dots(const zd* __restrict__ V, const zd* __restrict__ w,
                                                      zd* __restrict__ h, int ns, int B,
                                                      const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    __shared__ double sh[2][kRedThreads / 64];
    const int i = blockIdx.x, b = blockIdx.y;
    const zd* v = V + ((size_t)i * B + b) * ns;
    const zd* x = w + (size_t)b * ns;
    double re = 0, im = 0;
    for (int k = threadIdx.x; k < ns; k += kRedThreads) {
        const zd a = v[k], c = x[k];
        re += a.x * c.x + a.y * c.y;
        im += a.x * c.y - a.y * c.x;
    }
    re = block_sum_t0(re, sh[0]);
    im = block_sum_t0(im, sh[1]);
    if (threadIdx.x == 0) h[(size_t)i * B + b] = zd{re, im};
}

// The same dot products over long columns, split over nchunk blocks per
// (i, b): each block sums one contiguous chunk (part[(i B + b) nchunk + c]),
// then k_dots_fin adds the chunks in order (deterministic, no atomics).
__global__ void __launch_bounds__(kRedThreads) k_dots_part(const zd* __restrict__ V, const zd* __restrict__ w,
                                                           zd* __restrict__ part, int ns, int B, int nchunk,
                                                           const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    __shared__ double sh[2][kRedThreads / 64];
    const int i = blockIdx.x, b = blockIdx.y, ch = blockIdx.z;
    const int len = (ns + nchunk - 1) / nchunk, k0 = ch * len, k1 = min(ns, k0 + len);
    const zd* v = V + ((size_t)i * B + b) * ns;
    const zd* x = w + (size_t)b * ns;
    double re = 0, im = 0;
    for (int k = k0 + threadIdx.x; k < k1; k += kRedThreads) {
        const zd a = v[k], c = x[k];
        re += a.x * c.x + a.y * c.y;
        im += a.x * c.y - a.y * c.x;
    }
    re = block_sum_t0(re, sh[0]);
    im = block_sum_t0(im, sh[1]);
    if (threadIdx.x == 0) part[((size_t)i * B + b) * nchunk + ch] = zd{re, im};
}
// h[e] = sum_c part[e nchunk + c], e < n
__global__ void k_dots_fin(const zd* __restrict__ part, zd* __restrict__ h, int n, int nchunk,
                           const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    zd acc{0, 0};
    for (int ch = 0; ch < nchunk; ++ch) acc += part[(size_t)e * nchunk + ch];
    h[e] = acc;
}
// nrm[b] = ||w[b]|| over nchunk chunks per column (sum of squares in part,
// finished by k_norm_fin)
__global__ void __launch_bounds__(kRedThreads) k_norm_part(const zd* __restrict__ w, double* __restrict__ part,
                                                           int ns, int nchunk, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    __shared__ double sh[kRedThreads / 64];
    const int b = blockIdx.x, ch = blockIdx.y;
    const int len = (ns + nchunk - 1) / nchunk, k0 = ch * len, k1 = min(ns, k0 + len);
    const zd* x = w + (size_t)b * ns;
    double s = 0;
    for (int k = k0 + threadIdx.x; k < k1; k += kRedThreads) s += x[k].x * x[k].x + x[k].y * x[k].y;
    s = block_sum_t0(s, sh);
    if (threadIdx.x == 0) part[(size_t)b * nchunk + ch] = s;
}
__global__ void k_norm_fin(const double* __restrict__ part, double* __restrict__ nrm, int B, int nchunk,
                           const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[(size_t)b * nchunk + ch];
    nrm[b] = sqrt(s);
}

// w[b] -= sum_{i<nv} h[i][b] V_i[b]  (one classical Gram-Schmidt pass)
__global__ void __launch_bounds__(256) k_orth(const zd* __restrict__ V, zd* __restrict__ w, const zd* __restrict__ h,
                                              int nv, int ns, int B, const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int b = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= ns) return;
    zd acc = w[(size_t)b * ns + k];
    for (int i = 0; i < nv; ++i) acc -= h[(size_t)i * B + b] * V[((size_t)i * B + b) * ns + k];
    w[(size_t)b * ns + k] = acc;
}

// nrm[b] = ||w[b]||  (kRedThreads per block)
__global__ void __launch_bounds__(kRedThreads) k_norm(const zd* __restrict__ w, double* __restrict__ nrm, int ns,
                                                      const int* __restrict__ gate = nullptr, StepRef sr = {}) {
    if (gated_off(gate) || step_off(sr)) return;
    // replayed step: its row of the call's per-step norms [steps][B]
    if (const StepDesc* d = step_of(sr)) nrm = d->nrm + (size_t)d->i * gridDim.x;
    __shared__ double sh[kRedThreads / 64];
    const int b = blockIdx.x;
    const zd* x = w + (size_t)b * ns;
    double s = 0;
    for (int k = threadIdx.x; k < ns; k += kRedThreads) s += x[k].x * x[k].x + x[k].y * x[k].y;
    s = block_sum_t0(s, sh);
    if (threadIdx.x == 0) nrm[b] = sqrt(s);
}

// out[b] = w[b] / nrm[b] (0 if nrm == 0)
__global__ void k_scale(const zd* __restrict__ w, const double* __restrict__ nrm, zd* __restrict__ out, int ns,
                        int B, const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    const size_t tot = (size_t)ns * B;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / ns);
        const double n = nrm[b];
        const double s = n > 0 ? 1.0 / n : 0.0;
        out[e] = zd{w[e].x * s, w[e].y * s};
    }
}

// r = rhs - r  (r holds A x on entry)
__global__ void k_residual(const zd* __restrict__ rhs, zd* __restrict__ r, size_t n,
                           const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        r[e] = rhs[e] - r[e];
}

// Start of a cycle: beta = ||r||; column active iff beta > tol * bnorm.
// g[b] = (beta, 0, ...), jcnt = 0.  flag[0] = number of active columns,
// flag[1] set on a non-finite residual.  One block, one thread per column
// (strided); flag must be zero on entry.
__global__ void __launch_bounds__(256) k_cycle_start(const double* __restrict__ beta, const double* __restrict__ bnorm,
                                                     int* __restrict__ active, int* __restrict__ jcnt,
                                                     zd* __restrict__ g, double* __restrict__ resid,
                                                     int* __restrict__ flag, int B, int ldg, double tol,
                                                     const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const double be = beta[b];
        const bool fin = isfinite(be);
        const int a = (fin && be > tol * bnorm[b]) ? 1 : 0;
        active[b] = a;
        jcnt[b] = 0;
        resid[b] = bnorm[b] > 0 ? be / bnorm[b] : 0.0;
        for (int i = 0; i < ldg; ++i) g[(size_t)b * ldg + i] = zd{0, 0};
        g[(size_t)b * ldg] = zd{be, 0};
        if (a) atomicAdd(&flag[0], 1);
        if (!fin) atomicOr(&flag[1], 1);
    }
}

// Arnoldi column j for each active column b: Hessenberg entries
// h1 + h2 (the two classical Gram-Schmidt passes) and h_{j+1,j} = nrm[b],
// previous Givens rotations, a new rotation, residual estimate |g_{j+1}|.
// One block, one thread per column (strided); flag[0] must be zero on entry,
// flag[1] (non-finite) is sticky until the next cycle start.
__global__ void __launch_bounds__(256) k_arnoldi_update(const zd* __restrict__ h1, const zd* __restrict__ h2,
                                                        const double* __restrict__ nrm, zd* __restrict__ H,
                                                        double* __restrict__ cs, zd* __restrict__ sn,
                                                        zd* __restrict__ g, int* __restrict__ active,
                                                        int* __restrict__ jcnt, double* __restrict__ resid,
                                                        const double* __restrict__ bnorm, int* __restrict__ flag,
                                                        int j, int B, int restart, double tol,
                                                        const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int ldh = restart + 1;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        if (!active[b]) continue;
        zd* col = H + ((size_t)b * restart + j) * ldh;
        for (int i = 0; i <= j; ++i) col[i] = h1[(size_t)i * B + b] + h2[(size_t)i * B + b];
        col[j + 1] = zd{nrm[b], 0};
        double* c = cs + (size_t)b * restart;
        zd* s = sn + (size_t)b * restart;
        for (int i = 0; i < j; ++i) {
            const zd a = col[i], bb = col[i + 1];
            col[i] = c[i] * a + s[i] * bb;
            col[i + 1] = c[i] * bb - conjz(s[i]) * a;
        }
        const zd a = col[j];
        const double bv = col[j + 1].x;
        const double aa = sqrt(a.x * a.x + a.y * a.y);
        const double r = sqrt(aa * aa + bv * bv);
        double cj;
        zd sj;
        if (aa == 0.0) {
            cj = 0.0;
            sj = zd{1.0, 0.0};
        } else {
            cj = aa / r;
            sj = zd{a.x / aa * bv / r, a.y / aa * bv / r};
        }
        c[j] = cj;
        s[j] = sj;
        col[j] = cj * a + sj * col[j + 1];
        col[j + 1] = zd{0, 0};
        zd* gb = g + (size_t)b * ldh;
        const zd gj = gb[j];
        gb[j] = cj * gj;
        gb[j + 1] = zd{0, 0} - conjz(sj) * gj;
        const double est = sqrt(gb[j + 1].x * gb[j + 1].x + gb[j + 1].y * gb[j + 1].y);
        resid[b] = bnorm[b] > 0 ? est / bnorm[b] : 0.0;
        jcnt[b] = j + 1;
        if (!isfinite(est)) {
            atomicOr(&flag[1], 1);
            active[b] = 0;
        } else if (est <= tol * bnorm[b] || nrm[b] == 0.0 || j + 1 == restart) {
            active[b] = 0;
        }
        if (active[b]) atomicAdd(&flag[0], 1);
    }
}

// Gate of one Arnoldi step, flag = {active columns, non-finite, live,
// steps taken this cycle, step budget}: the step is live while a column is
// active, nothing went non-finite and the budget lasts.  One thread.
__global__ void k_gate(int* __restrict__ flag, const int* __restrict__ step_live = nullptr) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int live =
        (flag[0] > 0 && flag[1] == 0 && flag[4] > 0 && (step_live == nullptr || *step_live != 0)) ? 1 : 0;
    flag[2] = live;
    if (live) {
        flag[3] += 1;
        flag[4] -= 1;
    }
}

// Back-substitution R y = g per column (size jcnt[b]); y[b][i].
__global__ void k_backsolve(const zd* __restrict__ H, const zd* __restrict__ g, const int* __restrict__ jcnt,
                            zd* __restrict__ y, int B, int restart, const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int ldh = restart + 1;
    const int n = jcnt[b];
    zd* yb = y + (size_t)b * restart;
    for (int i = n - 1; i >= 0; --i) {
        zd acc = g[(size_t)b * ldh + i];
        for (int q = i + 1; q < n; ++q) acc -= H[((size_t)b * restart + q) * ldh + i] * yb[q];
        const zd d = H[((size_t)b * restart + i) * ldh + i];
        const double dd = d.x * d.x + d.y * d.y;
        yb[i] = dd > 0 ? zd{(acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd} : zd{0, 0};
    }
}

// x[b] += dinv . sum_{i<jcnt[b]} y[b][i] V_i[b]
__global__ void __launch_bounds__(256) k_update_x(zd* __restrict__ x, const zd* __restrict__ V,
                                                  const zd* __restrict__ y, const int* __restrict__ jcnt,
                                                  const zd* __restrict__ dinv, int ns, int B, int restart,
                                                  const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    const int b = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= ns) return;
    const int n = jcnt[b];
    if (n == 0) return;
    zd acc{0, 0};
    for (int i = 0; i < n; ++i) acc += y[(size_t)b * restart + i] * V[((size_t)i * B + b) * ns + k];
    const zd d = dinv[k];
    x[(size_t)b * ns + k] += acc * d;
}

// y[b] = op(M) x[b] (or y[b] += op(M) x[b]) for every column b, M a complex
// CSR matrix on the near-zone pattern; op(M) = M, or with conj = 1 the
// conjugated values (the host passes the transposed copy for M^H).
__global__ void k_spmv_cols(const int* __restrict__ rowptr, const int* __restrict__ col, const zd* __restrict__ M,
                            const zd* __restrict__ x, zd* __restrict__ y, int ns, int B, int conj, int accumulate,
                            const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const size_t tot = (size_t)ns * B;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / ns), i = (int)(e - (size_t)b * ns);
        const zd* xb = x + (size_t)b * ns;
        zd acc{0, 0};
        for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            zd v = M[q];
            if (conj) v.y = -v.y;
            acc += v * xb[col[q]];
        }
        y[e] = accumulate ? y[e] + acc : acc;
    }
}

// (op(M) x)[b][i] from the columns of x transposed to xt[k][b] (FP64), for
// lanes on consecutive columns b of row i: each matrix entry is one broadcast
// load and each x row one coalesced run; entries go in groups of four with
// their loads issued together.
__device__ __forceinline__ zd spmv_row_col(const int* __restrict__ rowptr, const int* __restrict__ col,
                                           const zd* __restrict__ M, const zd* __restrict__ xt, int i, int b, int B,
                                           int conj) {
    const double sg = conj ? -1.0 : 1.0;
    zd acc{0, 0};
    const int q1 = rowptr[i + 1];
    for (int q = rowptr[i]; q < q1; q += 4) {
        zd v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool live = q + u < q1;
            const int cu = live ? col[q + u] : 0;
            v[u] = live ? M[q + u] : zd{0, 0};
            xv[u] = xt[(size_t)cu * B + b];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += zd{v[u].x, sg * v[u].y} * xv[u];
    }
    return acc;
}

// (op(M) x)[b][i] for few columns: a group of kSpmvLanes lanes per (row i,
// column b) runs over the row's entries (coalesced entry loads), then sums
// across the group.  x[b][k] is read at x + k xs_k + b xs_b.  rows_out:
// out[i B + b] in the working precision (the operator's scaled-column
// layout); otherwise y[b][i] (FP64), added to y when accumulate.
constexpr int kSpmvLanes = 16;
template <typename R>
__global__ void __launch_bounds__(256) k_spmv_grp(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                  const zd* __restrict__ M, const zd* __restrict__ x, long long xs_k,
                                                  long long xs_b, cplx<R>* __restrict__ out, zd* __restrict__ y,
                                                  int ns, int B, int conj, int accumulate,
                                                  const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t pr = t / kSpmvLanes;
    const int g = (int)(t % kSpmvLanes);
    const bool live = pr < (size_t)ns * B;
    const int i = live ? (int)(pr / B) : 0, b = live ? (int)(pr % B) : 0;
    const double sg = conj ? -1.0 : 1.0;
    zd acc{0, 0};
    if (live) {
        const int q1 = rowptr[i + 1];
        for (int q = rowptr[i] + g; q < q1; q += kSpmvLanes) {
            const zd v = M[q];
            acc += zd{v.x, sg * v.y} * x[(size_t)col[q] * xs_k + (size_t)b * xs_b];
        }
    }
#pragma unroll
    for (int o = kSpmvLanes / 2; o > 0; o >>= 1) {
        acc.x += __shfl_xor(acc.x, o, 64);
        acc.y += __shfl_xor(acc.y, o, 64);
    }
    if (!live || g != 0) return;
    if (out)
        out[(size_t)i * B + b] = to_r<R>(acc);
    else {
        zd& d = y[(size_t)b * ns + i];
        d = accumulate ? d + acc : acc;
    }
}

// out[i][b] = (op(M) x)[b][i] in the working precision, the layout the
// operator's anterpolation and near zone read
template <typename R>
__global__ void __launch_bounds__(256) k_spmv_rows(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                   const zd* __restrict__ M, const zd* __restrict__ xt,
                                                   cplx<R>* __restrict__ out, int ns, int B, int conj,
                                                   const int* __restrict__ gate) {
    if (gated_off(gate)) return;
    const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (e >= (size_t)ns * B) return;
    const int i = (int)(e / B), b = (int)(e - (size_t)i * B);
    out[e] = to_r<R>(spmv_row_col(rowptr, col, M, xt, i, b, B, conj));
}

// y[b][i] += (op(M) x)[b][i] (FP64, columns of y contiguous)
__global__ void __launch_bounds__(256) k_spmv_rows_add(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                       const zd* __restrict__ M, const zd* __restrict__ xt,
                                                       zd* __restrict__ y, int ns, int B, int conj,
                                                       const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (e >= (size_t)ns * B) return;
    const int i = (int)(e / B), b = (int)(e - (size_t)i * B);
    y[(size_t)b * ns + i] += spmv_row_col(rowptr, col, M, xt, i, b, B, conj);
}

// u[b] = sum_{i < jcnt[b]} y[b][i] V_i[b]  (the Krylov combination before a
// right preconditioner that is not diagonal)
__global__ void __launch_bounds__(256) k_krylov_combine(zd* __restrict__ u, const zd* __restrict__ V,
                                                        const zd* __restrict__ y, const int* __restrict__ jcnt, int ns,
                                                        int B, int restart, const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    const int b = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= ns) return;
    const int n = jcnt[b];
    zd acc{0, 0};
    for (int i = 0; i < n; ++i) acc += y[(size_t)b * restart + i] * V[((size_t)i * B + b) * ns + k];
    u[(size_t)b * ns + k] = acc;
}

__global__ void k_copy_conj(const zd* __restrict__ in, zd* __restrict__ out, size_t n, int conj) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        zd v = in[e];
        if (conj) v.y = -v.y;
        out[e] = v;
    }
}

// Extrapolation orders: the polynomial through the last p solutions at the
// next step, x = sum_i (-1)^(i+1) C(p, i) x_{-i}, p = 1 .. kMaxGuess
constexpr int kMaxGuess = 6;
__constant__ double kExtrap[kMaxGuess][kMaxGuess] = {{1, 0, 0, 0, 0, 0},       {2, -1, 0, 0, 0, 0},
                                                      {3, -3, 1, 0, 0, 0},      {4, -6, 4, -1, 0, 0},
                                                      {5, -10, 10, -5, 1, 0},   {6, -15, 20, -15, 6, -1}};

// Initial guess of a time step: x = sum_{i=1}^{p} a_i I_{l - dir i}, the
// polynomial through the last p solutions evaluated one step ahead
// (a_i = (-1)^(i+1) C(p, i)); p = 0 gives zero.  The march picks p as the
// order whose prediction of the step just solved was closest.
__global__ void k_extrap(const zd* __restrict__ I, zd* __restrict__ x, size_t nB, long long l, int dir, int p,
                         const int* __restrict__ pdev, StepRef sr = {}) {
    if (step_off(sr)) return;
    if (const StepDesc* d = step_of(sr)) {
        I = d->I;
        l = d->cur;
        p = d->p;
        if (!d->pdev) pdev = nullptr;
    }
    // p caps the order (history available); pdev, when given, holds the order chosen on the device
    if (pdev) p = min(p, *pdev);
    const auto& a = kExtrap;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nB; e += (size_t)gridDim.x * blockDim.x) {
        zd acc{0, 0};
        for (int i = 1; i <= p; ++i) {
            const zd v = I[(size_t)(l - (long long)dir * i) * nB + e];
            acc.x += a[p - 1][i - 1] * v.x;
            acc.y += a[p - 1][i - 1] * v.y;
        }
        x[e] = acc;
    }
}

// Squared error of each extrapolation order p = 1..pmax at the step just
// solved, ||I_l - sum_i a_i I_{l - dir i}||^2: per-block partial sums
// part[blk][p-1] (grid-stride), then k_pred_err_sum adds the blocks in
// order (deterministic).
constexpr int kPredBlocks = 256;
__global__ void __launch_bounds__(kRedThreads) k_pred_err(const zd* __restrict__ I, size_t nB, long long l, int dir,
                                                          int pmax, double* __restrict__ part, StepRef sr = {}) {
    if (step_off(sr)) return;
    if (const StepDesc* d = step_of(sr)) {
        I = d->I;
        l = d->cur;
        pmax = d->pmax;
    }
    __shared__ double sh[kMaxGuess][kRedThreads / 64];
    const auto& a = kExtrap;
    double s[kMaxGuess] = {0, 0, 0, 0, 0, 0};
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nB; e += (size_t)gridDim.x * blockDim.x) {
        const zd x = I[(size_t)l * nB + e];
        zd v[kMaxGuess];
        for (int i = 1; i <= pmax; ++i) v[i - 1] = I[(size_t)(l - (long long)dir * i) * nB + e];
        for (int p = 1; p <= pmax; ++p) {
            double rx = x.x, ry = x.y;
            for (int i = 1; i <= p; ++i) {
                rx -= a[p - 1][i - 1] * v[i - 1].x;
                ry -= a[p - 1][i - 1] * v[i - 1].y;
            }
            s[p - 1] += rx * rx + ry * ry;
        }
    }
    for (int p = 0; p < kMaxGuess; ++p) {
        const double t = block_sum_t0(s[p], sh[p]);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * kMaxGuess + p] = t;
    }
}

__global__ void __launch_bounds__(256) k_pred_err_sum(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ err, int pmax, int* __restrict__ pbest,
                                                      StepRef sr = {}) {
    if (step_off(sr)) return;
    if (const StepDesc* d = step_of(sr)) pmax = d->pmax;
    __shared__ double sh[256];
    double e[kMaxGuess];
    for (int p = 0; p < kMaxGuess; ++p) {
        double s = 0;
        for (int b = threadIdx.x; b < nblk; b += 256) s += part[(size_t)b * kMaxGuess + p];
        e[p] = block_sum256(s, sh);
        if (threadIdx.x == 0) err[p] = e[p];
    }
    // the order that predicted best (the lowest on ties)
    if (threadIdx.x == 0) {
        int best = 1;
        for (int p = 2; p <= pmax; ++p)
            if (e[p - 1] < e[best - 1]) best = p;
        *pbest = best;
    }
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v, const int* __restrict__ gate = nullptr) {
    if (gated_off(gate)) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// out[e][m] = in[perm[e]][m] (rows of mv values)
__global__ void k_permute_rows(const zd* __restrict__ in, zd* __restrict__ out, const int* __restrict__ perm, int n,
                               int mv) {
    const size_t tot = (size_t)n * mv;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < tot; i += (size_t)gridDim.x * blockDim.x) {
        const size_t e = i / mv, m = i - e * mv;
        out[i] = in[(size_t)perm[e] * mv + m];
    }
}

template <typename R>
__global__ void k_to_r(const zd* __restrict__ in, cplx<R>* __restrict__ out, size_t n) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        out[e] = cplx<R>{(R)in[e].x, (R)in[e].y};
}

// The replayed step's solution x into the call's I_out[cur] ([N_t][B][ns]).
__global__ void k_store_step(const zd* __restrict__ x, size_t nB, StepRef sr) {
    if (step_off(sr)) return;
    const StepDesc* d = step_of(sr);
    zd* out = d->I + (size_t)d->cur * nB;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nB; e += (size_t)gridDim.x * blockDim.x)
        out[e] = x[e];
}

// The replayed step's solution into its slot of the current history
// [M_n][ns][B] in the working precision (columns of a basis contiguous).
template <typename R>
__global__ void k_store_hist(const zd* __restrict__ x, cplx<R>* __restrict__ hist, int ns, int B, int mn,
                             StepRef sr) {
    if (step_off(sr)) return;
    const StepDesc* d = step_of(sr);
    cplx<R>* out = hist + (size_t)(d->cur % mn) * ns * B;
    const size_t tot = (size_t)ns * B;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / B), b = (int)(e - (size_t)k * B);
        const zd v = x[(size_t)b * ns + k];
        out[e] = cplx<R>{(R)v.x, (R)v.y};
    }
}

// Start of a run of replayed steps (one thread): ctl = {descriptor index, live}.
__global__ void k_step_ctl(int* __restrict__ ctl, int idx) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ctl[0] = idx;
    ctl[1] = 1;
}

// After a replayed step's GMRES cycle (one thread): a column still active
// (not converged within the captured Arnoldi steps) or a non-finite residual
// stops the replays (live = 0) before the step commits anything.
// flag = the Arnoldi flags {active columns, non-finite, ...}.
__global__ void k_step_check(const int* __restrict__ flag, int* __restrict__ live) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (*live != 0 && (flag[0] > 0 || flag[1] != 0)) *live = 0;
}

// End of a replayed step (one thread): its Arnoldi step count and largest
// residual estimate into the per-step records, and the descriptor counter
// moves on.
__global__ void k_step_end(const int* __restrict__ flag, const double* __restrict__ resid, int B,
                           int* __restrict__ iters, double* __restrict__ res, int* __restrict__ ctr,
                           const int* __restrict__ live) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || *live == 0) return;
    double w = 0;
    for (int b = 0; b < B; ++b) w = fmax(w, resid[b]);
    iters[*ctr] = flag[3];
    res[*ctr] = w;
    *ctr += 1;
}

template <typename R>
__global__ void k_real_to_r(const double* __restrict__ in, R* __restrict__ out, size_t n) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        out[e] = (R)in[e];
}

}  // namespace etaim
