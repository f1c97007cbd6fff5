// Radix-2/3/4 Stockham FFT of many lines held in LDS, and the line-pass
// kernel built on it.  Each pass of radix R with p = product of the radices
// already done maps butterfly i (k = i mod p) to
//   inputs  x[i + j L/R], twiddled by w^(j k L/(pR)), w = exp(-2 pi i/L)
//   outputs y[(i - k) R + k + j p]
// (self-sorting, no bit reversal).  Two LDS buffers ping-pong between passes.
#pragma once
#include "common.hpp"

namespace etaim {

struct Radix {
    int L, n, r[16];
};

inline Radix make_radix(int L) {
    Radix p{};
    p.L = L;
    int n = L;
    while (n % 4 == 0) {
        p.r[p.n++] = 4;
        n /= 4;
    }
    while (n % 2 == 0) {
        p.r[p.n++] = 2;
        n /= 2;
    }
    while (n % 3 == 0) {
        p.r[p.n++] = 3;
        n /= 3;
    }
    return p;
}

template <typename R>
__device__ __forceinline__ cplx<R> mul_i(cplx<R> a, bool inverse) {
    // multiply by -i (forward) or +i (inverse)
    return inverse ? cplx<R>{-a.y, a.x} : cplx<R>{a.y, -a.x};
}

template <typename R, int RAD>
__device__ __forceinline__ void dft_small(cplx<R> (&u)[RAD], bool inverse) {
    if constexpr (RAD == 2) {
        const cplx<R> a = u[0], b = u[1];
        u[0] = a + b;
        u[1] = a - b;
    } else if constexpr (RAD == 3) {
        const R s = inverse ? (R)0.86602540378443864676 : (R)-0.86602540378443864676;
        const cplx<R> t = u[1] + u[2];
        const cplx<R> d = u[1] - u[2];
        const cplx<R> m = u[0] - (R)0.5 * t;
        const cplx<R> id{-s * d.y, s * d.x};  // i s d
        u[0] = u[0] + t;
        u[1] = m + id;
        u[2] = m - id;
    } else {
        const cplx<R> a = u[0] + u[2], b = u[0] - u[2];
        const cplx<R> c = u[1] + u[3], d = mul_i(u[1] - u[3], inverse);
        u[0] = a + c;
        u[2] = a - c;
        u[1] = b + d;
        u[3] = b - d;
    }
}

template <typename R, int RAD>
__device__ __forceinline__ void stockham_pass(const cplx<R>* __restrict__ src, cplx<R>* __restrict__ dst,
                                              int nl, int L, int ldl, int p,
                                              const cplx<R>* __restrict__ tw, bool inverse) {
    const int nb = L / RAD;
    const int tstep = L / (p * RAD);
    for (int e = threadIdx.x; e < nl * nb; e += blockDim.x) {
        const int line = e / nb;
        const int i = e - line * nb;
        const int k = i % p;
        const cplx<R>* s = src + line * ldl;
        cplx<R>* d = dst + line * ldl;
        cplx<R> u[RAD];
#pragma unroll
        for (int j = 0; j < RAD; ++j) u[j] = s[i + j * nb];
        if (k) {
#pragma unroll
            for (int j = 1; j < RAD; ++j) {
                cplx<R> w = tw[j * k * tstep];
                if (inverse) w.y = -w.y;
                u[j] = u[j] * w;
            }
        }
        dft_small<R, RAD>(u, inverse);
        const int base = (i - k) * RAD + k;
#pragma unroll
        for (int j = 0; j < RAD; ++j) d[base + j * p] = u[j];
    }
}

// FFT of nl lines of length pl.L stored at a[line*ldl + point]; returns the
// buffer holding the result (a or b).  Must be called by the whole block.
template <typename R>
__device__ cplx<R>* lds_fft(cplx<R>* a, cplx<R>* b, int nl, int ldl, const Radix& pl,
                            const cplx<R>* __restrict__ tw, bool inverse) {
    int p = 1;
    for (int s = 0; s < pl.n; ++s) {
        const int r = pl.r[s];
        if (r == 4)
            stockham_pass<R, 4>(a, b, nl, pl.L, ldl, p, tw, inverse);
        else if (r == 2)
            stockham_pass<R, 2>(a, b, nl, pl.L, ldl, p, tw, inverse);
        else
            stockham_pass<R, 3>(a, b, nl, pl.L, ldl, p, tw, inverse);
        __syncthreads();
        cplx<R>* t = a;
        a = b;
        b = t;
        p *= r;
    }
    return a;
}

// Generic pass: lines indexed by (f, s), f in [0,nf) grouped MT per block
// (blockIdx.x), s = blockIdx.y.  Element (line, point) lives at
// base + f*in_f + s*in_s + point*in_p.  Points >= in_len load as zero; the
// first out_len outputs are stored.
struct LineArgs {
    Radix pl;
    int nf, in_len, out_len, mt;
    long long in_f, in_s, in_p, out_f, out_s, out_p;
    int inverse;
};

template <typename R>
__global__ void __launch_bounds__(256) k_lines(const cplx<R>* in, cplx<R>* out,
                                               const cplx<R>* __restrict__ tw, LineArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int L = a.pl.L, ldl = L + 1, mt = a.mt;
    cplx<R>* b0 = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* b1 = b0 + mt * ldl;
    const int f0 = blockIdx.x * mt;
    const long long s = blockIdx.y;
    const cplx<R>* ibase = in + s * a.in_s;
    cplx<R>* obase = out + s * a.out_s;
    const int tot = mt * L;
    if (a.in_p == 1) {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int l = e / L, p = e - l * L;
            const int f = f0 + l;
            cplx<R> v{(R)0, (R)0};
            if (f < a.nf && p < a.in_len) v = ibase[f * a.in_f + p];
            b0[l * ldl + p] = v;
        }
    } else {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int p = e / mt, l = e - p * mt;
            const int f = f0 + l;
            cplx<R> v{(R)0, (R)0};
            if (f < a.nf && p < a.in_len) v = ibase[f * a.in_f + p * a.in_p];
            b0[l * ldl + p] = v;
        }
    }
    __syncthreads();
    cplx<R>* res = lds_fft<R>(b0, b1, mt, ldl, a.pl, tw, a.inverse != 0);
    const int tot_o = mt * a.out_len;
    if (a.out_p == 1) {
        for (int e = threadIdx.x; e < tot_o; e += blockDim.x) {
            const int l = e / a.out_len, p = e - l * a.out_len;
            const int f = f0 + l;
            if (f < a.nf) obase[f * a.out_f + p] = res[l * ldl + p];
        }
    } else {
        for (int e = threadIdx.x; e < tot_o; e += blockDim.x) {
            const int p = e / mt, l = e - p * mt;
            const int f = f0 + l;
            if (f < a.nf) obase[f * a.out_f + p * a.out_p] = res[l * ldl + p];
        }
    }
}

}  // namespace etaim
