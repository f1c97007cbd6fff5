// Mixed-radix (2, 3, 4, 6, 8, 12, 16) Stockham FFT of many lines held in LDS, and the line-pass
// kernel built on it.  Each pass of radix R with p = product of the radices
// already done maps butterfly i (k = i mod p) to
//   inputs  x[i + j L/R], twiddled by w^(j k L/(pR)), w = exp(-2 pi i/L)
//   outputs y[(i - k) R + k + j p]
// (self-sorting, no bit reversal), in place in one LDS buffer.
#pragma once
#include "common.hpp"

namespace etaim {

struct Radix {
    int L, n, r[16];
};

// Radix plan: fewest passes first (16, 12, 8, 6, 4, 3, 2).
inline Radix make_radix(int L) {
    Radix p{};
    p.L = L;
    int n = L;
    const int order[7] = {16, 12, 8, 6, 4, 3, 2};
    while (n > 1) {
        bool found = false;
        for (int r : order)
            if (n % r == 0) {
                p.r[p.n++] = r;
                n /= r;
                found = true;
                break;
            }
        if (!found || p.n >= 16) {
            p.n = 0;  // unsupported factor: caller checks p.n
            return p;
        }
    }
    return p;
}

// a * b with two products and two fused multiply-adds
template <typename R>
__device__ __forceinline__ cplx<R> cmul_fma(cplx<R> a, cplx<R> b) {
    return cplx<R>{fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}

template <typename R>
__device__ __forceinline__ cplx<R> mul_i(cplx<R> a, bool inverse) {
    // multiply by -i (forward) or +i (inverse)
    return inverse ? cplx<R>{-a.y, a.x} : cplx<R>{a.y, -a.x};
}

// exp(-2 pi i m / 48) for m = 0..47 written as (cos, sin) of multiples of
// 7.5 degrees: covers the twiddles of every composite codelet below
// (N = 6, 8, 12, 16 all divide 48).
__device__ __forceinline__ void w48(int m, double& c, double& s) {
    // cos(k * pi / 24), k = 0..12 (quarter wave), exact decimal expansions
    const double q[13] = {1.0,
                          0.99144486137381041114,
                          0.96592582628906828675,
                          0.92387953251128675613,
                          0.86602540378443864676,
                          0.79335334029123516458,
                          0.70710678118654752440,
                          0.60876142900872063942,
                          0.5,
                          0.38268343236508977173,
                          0.25881904510252076235,
                          0.13052619222005159155,
                          0.0};
    m %= 48;
    // angle = 2 pi m / 48 = m * 7.5 deg = m * pi / 24
    const int quad = m / 12, r = m % 12;
    double cr = q[r], sr = q[12 - r];
    // rotate by quad * 90 degrees
    for (int i = 0; i < quad; ++i) {
        const double t = cr;
        cr = -sr;
        sr = t;
    }
    c = cr;
    s = -sr;  // exp(-i angle)
}

// exp(-2 pi i m / 96) for m = 0..95 (multiples of 3.75 degrees): the
// parity pre-twiddles w_{2N}^n of the register plane kernels (2N | 96).
__device__ __forceinline__ void w96(int m, double& c, double& s) {
    // cos(k * pi / 48), k = 0..24 (quarter wave), exact decimal expansions
    const double q[25] = {1.0,
                          0.997858923238603506738,
                          0.991444861373810411145,
                          0.980785280403230449126,
                          0.965925826289068286750,
                          0.946930129495105664256,
                          0.923879532511286756128,
                          0.896872741532688303894,
                          0.866025403784438646764,
                          0.831469612302545237079,
                          0.793353340291235164580,
                          0.751839807478977396408,
                          0.707106781186547524401,
                          0.659345815100068868425,
                          0.608761429008720639416,
                          0.555570233019602224743,
                          0.5,
                          0.442288690219001281995,
                          0.382683432365089771728,
                          0.321439465303161580701,
                          0.258819045102520762349,
                          0.195090322016128267848,
                          0.130526192220051591548,
                          0.065403129230143066815,
                          0.0};
    m %= 96;
    const int quad = m / 24, r = m % 24;
    double cr = q[r], sr = q[24 - r];
    for (int i = 0; i < quad; ++i) {
        const double t = cr;
        cr = -sr;
        sr = t;
    }
    c = cr;
    s = -sr;  // exp(-i angle)
}

template <typename R, int RAD>
__device__ __forceinline__ void dft_small(cplx<R> (&u)[RAD], bool inverse);

// v * exp(-+2 pi i m / 48) for a compile-time m (after unrolling): exact
// swaps and negations at multiples of 90 degrees, sqrt(1/2) (a +- b) at odd
// multiples of 45 degrees, otherwise two products and two fused
// multiply-adds
template <typename R>
__device__ __forceinline__ cplx<R> tw48_mul(cplx<R> v, int m, bool inverse) {
    m %= 48;
    if (inverse) m = (48 - m) % 48;  // conj(w^m) = w^(48 - m)
    const R h = (R)0.70710678118654752440;
    switch (m) {
        case 0: return v;
        case 12: return cplx<R>{v.y, -v.x};
        case 24: return cplx<R>{-v.x, -v.y};
        case 36: return cplx<R>{-v.y, v.x};
        case 6: return cplx<R>{h * (v.x + v.y), h * (v.y - v.x)};
        case 18: return cplx<R>{h * (v.y - v.x), -h * (v.x + v.y)};
        case 30: return cplx<R>{-h * (v.x + v.y), h * (v.x - v.y)};
        case 42: return cplx<R>{h * (v.x - v.y), h * (v.x + v.y)};
        default: {
            double c, s;
            w48(m, c, s);
            const R cr = (R)c, sr = (R)s;
            return cplx<R>{fma(v.x, cr, -(v.y * sr)), fma(v.x, sr, v.y * cr)};
        }
    }
}

// v * exp(-+2 pi i m / 96) for a compile-time m, exact at multiples of 90
// degrees and sqrt(1/2) (a +- b) at odd multiples of 45 degrees
template <typename R>
__device__ __forceinline__ cplx<R> tw96_mul(cplx<R> v, int m, bool inverse) {
    m %= 96;
    if (m % 2 == 0) return tw48_mul<R>(v, m / 2, inverse);
    if (inverse) m = 96 - m;
    double c, s;
    w96(m, c, s);
    return cmul_fma(v, cplx<R>{(R)c, (R)s});
}

// composite codelet of size N1*N2 in registers: X[k2 + N2 k1] =
// sum_n1 W_N1^{n1 k1} W_N^{n1 k2} sum_n2 W_N2^{n2 k2} x[n1 + N1 n2]
template <typename R, int N1, int N2>
__device__ __forceinline__ void dft_composite(cplx<R> (&u)[N1 * N2], bool inverse) {
    constexpr int N = N1 * N2;
    cplx<R> y[N1][N2];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        cplx<R> v[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) v[n2] = u[n1 + N1 * n2];
        dft_small<R, N2>(v, inverse);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            y[n1][k2] = tw48_mul<R>(v[k2], (48 / N) * n1 * k2, inverse);
        }
    }
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
        cplx<R> v[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) v[n1] = y[n1][k2];
        dft_small<R, N1>(v, inverse);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) u[k2 + N2 * k1] = v[k1];
    }
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
        const cplx<R> m{fma((R)-0.5, t.x, u[0].x), fma((R)-0.5, t.y, u[0].y)};
        u[0] = u[0] + t;
        // m +- i s d
        u[1] = cplx<R>{fma(-s, d.y, m.x), fma(s, d.x, m.y)};
        u[2] = cplx<R>{fma(s, d.y, m.x), fma(-s, d.x, m.y)};
    } else if constexpr (RAD == 4) {
        const cplx<R> a = u[0] + u[2], b = u[0] - u[2];
        const cplx<R> c = u[1] + u[3], d = mul_i(u[1] - u[3], inverse);
        u[0] = a + c;
        u[2] = a - c;
        u[1] = b + d;
        u[3] = b - d;
    } else if constexpr (RAD == 6) {
        dft_composite<R, 2, 3>(u, inverse);
    } else if constexpr (RAD == 8) {
        dft_composite<R, 2, 4>(u, inverse);
    } else if constexpr (RAD == 12) {
        dft_composite<R, 4, 3>(u, inverse);
    } else if constexpr (RAD == 24) {
        dft_composite<R, 8, 3>(u, inverse);
    } else if constexpr (RAD == 48) {
        dft_composite<R, 16, 3>(u, inverse);
    } else {
        static_assert(RAD == 16, "unsupported radix");
        dft_composite<R, 4, 4>(u, inverse);
    }
}

// ---------------------------------------------------------------------------
// In-place FFT of nl lines held in one LDS buffer: element (line, point) at
// buf[line*lstride + point*pstride].  A pass of radix RAD has nl * L/RAD
// butterflies e = i*nl + line (line fastest), so the lanes of a wavefront
// touch consecutive lines: with a line stride of 1 (columns) or an odd
// stride L+1 (rows) the LDS accesses spread over all banks for every
// butterfly index i and output position.  Thread tid owns e = tid + q*blockDim,
// q < NPT; (line, i) advance incrementally (no division per butterfly).
// Inputs are staged in registers, the block synchronises, and outputs are
// written to the same buffer.  plane_fits() is the host-side condition.
constexpr int kPlaneThreads = 1024;
// butterflies per thread per pass, by radix: nl * L <= 12288 fits every radix
__host__ __device__ constexpr int plane_npt(int r) {
    return r == 16 ? 1 : r == 12 ? 1 : r == 8 ? 2 : r == 6 ? 2 : r == 4 ? 3 : r == 3 ? 4 : 6;
}

template <typename R, int RAD, int NPT>
__device__ __forceinline__ void plane_pass(cplx<R>* buf, int nl, int lstride, int pstride, int L, int p,
                                           const cplx<R>* tw, bool inverse) {
    const int nb = L / RAD, tstep = L / (p * RAD);
    const int dl = blockDim.x % nl, di = blockDim.x / nl;
    const int line0 = threadIdx.x % nl, i0 = threadIdx.x / nl;
    const bool pow2 = (p & (p - 1)) == 0;
    cplx<R> u[NPT][RAD];
    {
        int line = line0, i = i0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            if (i < nb) {
                const cplx<R>* src = buf + line * lstride + i * pstride;
#pragma unroll
                for (int j = 0; j < RAD; ++j) u[q][j] = src[j * nb * pstride];
            }
            line += dl;
            i += di;
            if (line >= nl) {
                line -= nl;
                ++i;
            }
        }
    }
    __syncthreads();
    {
        int line = line0, i = i0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            if (i < nb) {
                const int k = pow2 ? (i & (p - 1)) : i % p;
                if (k) {
#pragma unroll
                    for (int j = 1; j < RAD; ++j) {
                        cplx<R> w = tw[j * k * tstep];
                        if (inverse) w.y = -w.y;
                        u[q][j] = u[q][j] * w;
                    }
                }
                dft_small<R, RAD>(u[q], inverse);
                cplx<R>* dst = buf + line * lstride + ((i - k) * RAD + k) * pstride;
#pragma unroll
                for (int j = 0; j < RAD; ++j) dst[j * p * pstride] = u[q][j];
            }
            line += dl;
            i += di;
            if (line >= nl) {
                line -= nl;
                ++i;
            }
        }
    }
    __syncthreads();
}

template <typename R>
__device__ void plane_fft(cplx<R>* buf, int nl, int lstride, int pstride, const Radix& pl, const cplx<R>* tw,
                          bool inverse) {
    int p = 1;
    for (int s = 0; s < pl.n; ++s) {
        const int r = pl.r[s];
        switch (r) {
            case 16: plane_pass<R, 16, plane_npt(16)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
            case 12: plane_pass<R, 12, plane_npt(12)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
            case 8: plane_pass<R, 8, plane_npt(8)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
            case 6: plane_pass<R, 6, plane_npt(6)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
            case 4: plane_pass<R, 4, plane_npt(4)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
            case 3: plane_pass<R, 3, plane_npt(3)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
            default: plane_pass<R, 2, plane_npt(2)>(buf, nl, lstride, pstride, pl.L, p, tw, inverse); break;
        }
        p *= r;
    }
}

// host check: every pass of an FFT of nl lines of length pl.L fits the
// per-thread register staging of kPlaneThreads threads
inline bool plane_fits(int nl, const Radix& pl) {
    if (pl.n == 0) return false;
    for (int s = 0; s < pl.n; ++s) {
        const int r = pl.r[s];
        const long tot = (long)nl * (pl.L / r);
        if (tot > (long)plane_npt(r) * kPlaneThreads) return false;
    }
    return true;
}

// Generic pass: lines indexed by (f, s), f in [0,nf) grouped MT per block
// (blockIdx.x), s = blockIdx.y = s1*ns0 + s0.  Element (line, point) lives at
// base + f*in_f + s0*in_s + s1*in_s1 + point*in_p.  Points >= in_len load as
// zero; the first out_len outputs are stored.  The MT lines are transformed
// in place in LDS (plane_fft, kPlaneThreads threads).
struct LineArgs {
    Radix pl;
    int nf, in_len, out_len, mt;
    long long in_f, in_s, in_p, out_f, out_s, out_p;
    int inverse;
    // slow index s = s1 * ns0 + s0 -> offset s0 * in_s + s1 * in_s1 (same for out)
    int ns0;
    long long in_s1, out_s1;
    const int* gate;  // optional GMRES gate
};

template <typename R>
__global__ void __launch_bounds__(kPlaneThreads) k_lines(const cplx<R>* in, cplx<R>* out,
                                                         const cplx<R>* __restrict__ tw_g, LineArgs a) {
    if (gated_off(a.gate)) return;
    extern __shared__ unsigned char smem_raw[];
    const int L = a.pl.L, ldl = L + 1, mt = a.mt;
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* tw = buf + mt * ldl;
    for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = tw_g[i];
    const int f0 = blockIdx.x * mt;
    const long long s0 = blockIdx.y % a.ns0, s1 = blockIdx.y / a.ns0;
    const cplx<R>* ibase = in + s0 * a.in_s + s1 * a.in_s1;
    cplx<R>* obase = out + s0 * a.out_s + s1 * a.out_s1;
    const int tot = mt * L;
    if (a.in_p == 1) {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int l = e / L, p = e - l * L;
            const int f = f0 + l;
            cplx<R> v{(R)0, (R)0};
            if (f < a.nf && p < a.in_len) v = ibase[f * a.in_f + p];
            buf[l * ldl + p] = v;
        }
    } else {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int p = e / mt, l = e - p * mt;
            const int f = f0 + l;
            cplx<R> v{(R)0, (R)0};
            if (f < a.nf && p < a.in_len) v = ibase[f * a.in_f + p * a.in_p];
            buf[l * ldl + p] = v;
        }
    }
    __syncthreads();
    plane_fft<R>(buf, mt, ldl, 1, a.pl, tw, a.inverse != 0);
    const int tot_o = mt * a.out_len;
    if (a.out_p == 1) {
        for (int e = threadIdx.x; e < tot_o; e += blockDim.x) {
            const int l = e / a.out_len, p = e - l * a.out_len;
            const int f = f0 + l;
            if (f < a.nf) obase[f * a.out_f + p] = buf[l * ldl + p];
        }
    } else {
        for (int e = threadIdx.x; e < tot_o; e += blockDim.x) {
            const int p = e / mt, l = e - p * mt;
            const int f = f0 + l;
            if (f < a.nf) obase[f * a.out_f + p * a.out_p] = buf[l * ldl + p];
        }
    }
}

// ---------------------------------------------------------------------------
// Four-step line FFT for L = A B points with both factors register codelets
// (A, B dividing 48).  Index maps n = n2 + B n1, k = k1 + A k2 give
//   X[k1 + A k2] = sum_n2 W_B^{n2 k2} W_L^{n2 k1} sum_n1 W_A^{n1 k1} x[n2 + B n1]
// (W_L^{nk} = W_L^{n2 k1} W_B^{n2 k2} W_A^{n1 k1}).  A block takes MT lines:
// tasks (line, n2) do the A-point DFTs in registers, scale by W_L^{n2 k1}
// and write Y[line][k1][n2] to LDS; after one barrier, tasks (line, k1) read
// their B values and do the B-point DFTs in registers.  The inverse runs
// the same steps mirrored with conjugate twiddles (unnormalised).  Loads of
// points >= in_len read as zero; outputs >= out_len are not stored.
//
// LF (lines fastest): lanes run over consecutive lines, for layouts whose
// lines are adjacent in memory (a line's points strided); otherwise lanes
// run over a line's points, for layouts whose points are adjacent.  Y is
// laid out to match: [k1][n2][line] (LF) or [line][k1][n2 + pad] (points
// fastest, rows of B + 1), so that the lanes of a wave touch consecutive
// LDS words in both phases.
template <typename R>
__host__ __device__ constexpr int lines4_mt() {
    return sizeof(R) == 4 ? 16 : 8;
}
template <typename R, int A, int B>
__host__ __device__ constexpr int lines4_threads() {
    return lines4_mt<R>() * (A > B ? A : B);
}
// lanes over the lines: the k1 rows of Y are padded by 128 bytes, so that
// the four (FP32) or eight (FP64) k1 rows one wave reads in the second
// step fall on alternate halves of the LDS banks
template <typename R>
__host__ __device__ constexpr int lines4_pad() {
    return 128 / (int)sizeof(cplx<R>);
}
template <typename R, int A, int B, bool LF>
__host__ __device__ constexpr int lines4_ysize() {
    return LF ? A * (B * lines4_mt<R>() + lines4_pad<R>()) : lines4_mt<R>() * A * (B + 1);
}
template <typename R, int A, int B, bool LF>
__host__ __device__ constexpr size_t lines4_lds() {
    return (size_t)(A * B + lines4_ysize<R, A, B, LF>()) * sizeof(cplx<R>);
}

template <typename R, int A, int B, bool LF>
__device__ __forceinline__ int l4_y(int l, int k1, int n2) {
    constexpr int MT = lines4_mt<R>();
    return LF ? k1 * (B * MT + lines4_pad<R>()) + n2 * MT + l : (l * A + k1) * (B + 1) + n2;
}

// tasks over (line, j), j < J: t -> (l, j)
template <int J, int MT, bool LF>
__device__ __forceinline__ void l4_task(int t, int& l, int& j) {
    if (LF) {
        l = t % MT;
        j = t / MT;
    } else {
        j = t % J;
        l = t / J;
    }
}

// forward: x (stride B per n1, loaded by the caller into u) -> Y
template <typename R, int A, int B, int MT, bool LF>
__device__ __forceinline__ void l4_fwd_first(cplx<R> (&u)[A], cplx<R>* Y, const cplx<R>* tw, int l, int n2) {
    dft_small<R, A>(u, false);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) Y[l4_y<R, A, B, LF>(l, k1, n2)] = k1 ? u[k1] * tw[n2 * k1] : u[k1];
}

// inverse: X (stride A per k2, in u) -> Y
template <typename R, int A, int B, int MT, bool LF>
__device__ __forceinline__ void l4_inv_first(cplx<R> (&u)[B], cplx<R>* Y, const cplx<R>* tw, int l, int k1) {
    dft_small<R, B>(u, true);
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
        cplx<R> v = u[n2];
        if (n2 && k1) {
            cplx<R> w = tw[n2 * k1];
            w.y = -w.y;
            v = v * w;
        }
        Y[l4_y<R, A, B, LF>(l, k1, n2)] = v;
    }
}

// HALF: the zero-padded half is known at compile time (forward: in_len =
// L/2, so n1 >= A/2 load as zero; inverse: out_len = L/2, so only n1 < A/2
// are stored), and the codelets drop the work on those constant zeros and
// unused outputs.
template <typename R, int A, int B, bool LF, bool HALF>
__global__ void __launch_bounds__((lines4_threads<R, A, B>())) k_lines4(const cplx<R>* in, cplx<R>* out,
                                                                     const cplx<R>* __restrict__ tw_g,
                                                                     LineArgs a) {
    if (gated_off(a.gate)) return;
    constexpr int MT = lines4_mt<R>(), L = A * B;
    extern __shared__ unsigned char smem_raw[];
    cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* Y = tw + L;
    for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = tw_g[i];
    const int f0 = blockIdx.x * MT;
    const long long s0 = blockIdx.y % a.ns0, s1 = blockIdx.y / a.ns0;
    const cplx<R>* ibase = in + s0 * a.in_s + s1 * a.in_s1;
    cplx<R>* obase = out + s0 * a.out_s + s1 * a.out_s1;
    __syncthreads();
    if (!a.inverse) {
        for (int t = threadIdx.x; t < MT * B; t += blockDim.x) {
            int l, n2;
            l4_task<B, MT, LF>(t, l, n2);
            const int f = f0 + l;
            cplx<R> u[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) {
                const int n = n2 + B * n1;
                if (HALF && n1 >= A / 2)
                    u[n1] = cplx<R>{0, 0};
                else
                    u[n1] = (f < a.nf && (HALF || n < a.in_len)) ? ibase[f * a.in_f + n * a.in_p] : cplx<R>{0, 0};
            }
            l4_fwd_first<R, A, B, MT, LF>(u, Y, tw, l, n2);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < MT * A; t += blockDim.x) {
            int l, k1;
            l4_task<A, MT, LF>(t, l, k1);
            const int f = f0 + l;
            cplx<R> u[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) u[n2] = Y[l4_y<R, A, B, LF>(l, k1, n2)];
            dft_small<R, B>(u, false);
            if (f < a.nf)
#pragma unroll
                for (int k2 = 0; k2 < B; ++k2) {
                    const int k = k1 + A * k2;
                    if (k < a.out_len) obase[f * a.out_f + k * a.out_p] = u[k2];
                }
        }
    } else {
        for (int t = threadIdx.x; t < MT * A; t += blockDim.x) {
            int l, k1;
            l4_task<A, MT, LF>(t, l, k1);
            const int f = f0 + l;
            cplx<R> u[B];
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) {
                const int k = k1 + A * k2;
                u[k2] = (f < a.nf && k < a.in_len) ? ibase[f * a.in_f + k * a.in_p] : cplx<R>{0, 0};
            }
            l4_inv_first<R, A, B, MT, LF>(u, Y, tw, l, k1);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < MT * B; t += blockDim.x) {
            int l, n2;
            l4_task<B, MT, LF>(t, l, n2);
            const int f = f0 + l;
            cplx<R> u[A];
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) u[k1] = Y[l4_y<R, A, B, LF>(l, k1, n2)];
            dft_small<R, A>(u, true);
            if (f < a.nf)
#pragma unroll
                for (int n1 = 0; n1 < (HALF ? A / 2 : A); ++n1) {
                    const int n = n2 + B * n1;
                    if (HALF || n < a.out_len) obase[f * a.out_f + n * a.out_p] = u[n1];
                }
        }
    }
}

// the (A, B) split of a line length with a four-step kernel, A <= B; false if none
inline bool lines4_split(int L, int& A, int& B) {
    switch (L) {
        case 96: A = 8; B = 12; return true;
        case 144: A = 12; B = 12; return true;
        case 192: A = 8; B = 24; return true;
        case 288: A = 12; B = 24; return true;
        case 384: A = 16; B = 24; return true;
        case 576: A = 24; B = 24; return true;
        default: return false;
    }
}

}  // namespace etaim
