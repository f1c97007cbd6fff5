// Shared definitions of the ET-AIM library (host set-up and device code).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace etaim {

constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
// MI355X: 8 XCDs, each with its own L2; consecutive workgroups of a launch
// are dispatched to the XCDs round-robin
constexpr int kXcds = 8;

// Device-side gate of the batched GMRES iteration: kernels of an Arnoldi
// step that are launched ahead of the host's convergence check (or replayed
// from a captured graph) return at once when the step is not live.
__device__ __forceinline__ bool gated_off(const int* gate) { return gate != nullptr && *gate == 0; }

constexpr double kMu0 = 4.0e-7 * kPi;
// eps0 = 1/(mu0 c^2), evaluated at run time to keep one definition
__host__ __device__ inline double eps0() { return 1.0 / (kMu0 * kC0 * kC0); }
constexpr int kQ = 3;  // CPPIF order

template <typename R>
struct cplx {
    R x, y;
};
using zd = cplx<double>;
using zf = cplx<float>;

// Per-step values of a forward march replayed from a captured whole-step
// graph.  The host writes one descriptor per step before the replays; the
// graph's kernels read sd[*ctr], and its last kernel advances *ctr.  *live
// drops to 0 when a step does not converge within the graph's Arnoldi
// steps: every later node of the graph (and of the steps enqueued after
// it) then returns at once, and the host completes that step eagerly.
struct StepDesc {
    int cur;   // the step (index of V and I)
    int i;     // the step's index within the march call
    int r0;    // first step of its time block
    int nm;    // history terms of the per-step delayed sum
    int fj;    // block-sum slot of the step (-1: none)
    int nmh;   // near-history terms, min(M_n, cur)
    int p;     // extrapolation order cap of the initial guess
    int pdev;  // 1: the order is the one chosen on the device (pnext)
    int pmax;  // extrapolation orders compared after the step
    int pad;
    // the call's arrays: excitation and solutions [N_t][B][ns], current norms [steps][B]
    const cplx<double>* V;
    cplx<double>* I;
    double* nrm;
};
struct StepRef {
    const StepDesc* sd = nullptr;  // nullptr: an eager launch (values from the arguments)
    const int* ctr = nullptr;
    const int* live = nullptr;
};
__device__ __forceinline__ const StepDesc* step_of(StepRef s) { return s.sd ? s.sd + *s.ctr : nullptr; }
__device__ __forceinline__ bool step_off(StepRef s) { return s.live != nullptr && *s.live == 0; }

template <typename R>
__host__ __device__ inline cplx<R> mk(R a, R b) { return cplx<R>{a, b}; }
template <typename R>
__host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__host__ __device__ inline cplx<R> conjz(cplx<R> a) { return {a.x, -a.y}; }
template <typename R>
__host__ __device__ inline cplx<R>& operator+=(cplx<R>& a, cplx<R> b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <typename R>
__host__ __device__ inline cplx<R>& operator-=(cplx<R>& a, cplx<R> b) {
    a.x -= b.x;
    a.y -= b.y;
    return a;
}

// ---------------------------------------------------------------------------
// CPPIF temporal basis of order 3 (Sec. 3 eq. (3)): on the piece
// tau in (i-1, i], i = 0..3, T is the Lagrange weight of sample n-i for the
// cubic through samples n, n-1, n-2, n-3.  With s = tau - i in (-1, 0]:
//   T = prod_{k != i} (s + k) / prod_{k != i} (k - i),
// a cubic in s whose roots are -k for the three k != i.  Breakpoints belong
// to the left piece (i = ceil(tau)); T = 0 outside (-1, 3].
// d[0..3] receive T, dT/dtau, d2T/dtau2, d3T/dtau3 of piece i at s.
__host__ __device__ inline void cppif_piece(int i, double s, double d[4]) {
    double a[3];
    int n = 0;
    double den = 1.0;
    for (int k = 0; k <= kQ; ++k) {
        if (k == i) continue;
        a[n++] = (double)k;
        den *= (double)(k - i);
    }
    const double e1 = a[0] + a[1] + a[2];
    const double e2 = a[0] * a[1] + a[1] * a[2] + a[2] * a[0];
    const double e3 = a[0] * a[1] * a[2];
    d[0] = (((s + e1) * s + e2) * s + e3) / den;
    d[1] = ((3.0 * s + 2.0 * e1) * s + e2) / den;
    d[2] = (6.0 * s + 2.0 * e1) / den;
    d[3] = 6.0 / den;
}

// T and its first two derivatives at tau (zero outside the support).
__host__ __device__ inline bool cppif_eval(double tau, double d[4]) {
    if (!(tau > -1.0 && tau <= (double)kQ)) {
        d[0] = d[1] = d[2] = d[3] = 0.0;
        return false;
    }
    const int i = (int)ceil(tau);
    cppif_piece(i, tau - (double)i, d);
    return true;
}

// ---------------------------------------------------------------------------
// Band-limited interpolatory basis (BLIF, Sec. 3 and Sec. 3.1.2) of half
// width M: T = sinc(tau) W(tau) on -M < tau <= M, W Knab's approximate
// prolate window sinh(a sqrt(u)) / (sqrt(u) sinh a), u = 1 - (tau/M)^2,
// a = pi M (1 - 2 beta), beta = f_bw dt.  W is summed as its power series
// in u (c[k] = a^(2k+1) / ((2k+1)! sinh a)), which is entire, so T and its
// derivatives follow from the product rule; the sinc's derivatives are
// taken in closed form, or by their Taylor series near tau = 0.
constexpr int kBlifTerms = 24;

struct TBasis {
    int kind = 0;  // 0: CPPIF of order kQ, 1: BLIF
    int M = kQ;    // BLIF half width
    double c[kBlifTerms] = {};

    // lower and upper ends of the support (lo < tau <= hi)
    __host__ __device__ double lo() const { return kind == 0 ? -1.0 : -(double)M; }
    __host__ __device__ double hi() const { return kind == 0 ? (double)kQ : (double)M; }

    __host__ __device__ void blif_at(double t, double d[4]) const {
        const double MM = (double)M * (double)M;
        const double u = 1.0 - t * t / MM, u1 = -2.0 * t / MM, u2 = -2.0 / MM;
        // window series and its first three u-derivatives (Horner)
        double w0 = 0, w1 = 0, w2 = 0, w3 = 0;
        for (int k = kBlifTerms - 1; k >= 0; --k) {
            const double kk = (double)k;
            w0 = w0 * u + c[k];
            if (k >= 1) w1 = w1 * u + c[k] * kk;
            if (k >= 2) w2 = w2 * u + c[k] * kk * (kk - 1.0);
            if (k >= 3) w3 = w3 * u + c[k] * kk * (kk - 1.0) * (kk - 2.0);
        }
        const double W0 = w0, W1 = w1 * u1, W2 = w2 * u1 * u1 + w1 * u2, W3 = w3 * u1 * u1 * u1 + 3.0 * w2 * u1 * u2;
        // sinc derivatives in tau
        double S0, S1, S2, S3;
        const double pi = kPi;
        if (fabs(t) < 0.25) {
            // sin(pi t)/(pi t) = sum_j (-1)^j (pi t)^(2j) / (2j+1)!
            S0 = S1 = S2 = S3 = 0.0;
            double fac = 1.0;  // (2j+1)!
            double sgn = 1.0;
            for (int j = 0; j < 16; ++j) {
                const int e = 2 * j;
                if (j > 0) fac *= (double)(e) * (double)(e + 1);
                const double coef = sgn * pow(pi, (double)e) / fac;
                S0 += coef * pow(t, (double)e);
                if (e >= 1) S1 += coef * e * pow(t, (double)(e - 1));
                if (e >= 2) S2 += coef * e * (e - 1) * pow(t, (double)(e - 2));
                if (e >= 3) S3 += coef * e * (e - 1) * (e - 2) * pow(t, (double)(e - 3));
                sgn = -sgn;
            }
        } else {
            const double x = pi * t, sx = sin(x), cx = cos(x), x2 = x * x;
            S0 = sx / x;
            S1 = pi * (x * cx - sx) / x2;
            S2 = pi * pi * (-x2 * sx - 2.0 * x * cx + 2.0 * sx) / (x2 * x);
            S3 = pi * pi * pi * (-x2 * x * cx + 3.0 * x2 * sx + 6.0 * x * cx - 6.0 * sx) / (x2 * x2);
        }
        d[0] = S0 * W0;
        d[1] = S1 * W0 + S0 * W1;
        d[2] = S2 * W0 + 2.0 * S1 * W1 + S0 * W2;
        d[3] = S3 * W0 + 3.0 * S2 * W1 + 3.0 * S1 * W2 + S0 * W3;
    }
    // T and its first three derivatives at tau (zero outside the support)
    __host__ __device__ bool eval(double tau, double d[4]) const {
        if (kind == 0) return cppif_eval(tau, d);
        if (!(tau > lo() && tau <= hi())) {
            d[0] = d[1] = d[2] = d[3] = 0.0;
            return false;
        }
        blif_at(tau, d);
        return true;
    }
    // T and its derivatives at tau = m approached from below (R -> 0+): the
    // CPPIF's piece m, the BLIF's value; false where they vanish
    __host__ __device__ bool origin(int m, double d[4]) const {
        if (kind == 0) {
            if (m < 0 || m > kQ) {
                d[0] = d[1] = d[2] = d[3] = 0.0;
                return false;
            }
            cppif_piece(m, 0.0, d);
            return true;
        }
        return eval((double)m, d);
    }
};

// the BLIF's fold of the non-causal m = -1..-nk into m < np (nk = 0: none)
struct TFold {
    int nk = 0, np = 0;
    double a[2][4] = {};
};

// Envelope kernel factors for interaction offset m at distance R
// (differentiated EFIE, Lorenz gauge, envelope Green function
// delta(t - R/c) exp(-j k R)/(4 pi R), d/dt -> d/dt + j w):
//   fA   = exp(-j k R) [T''/dt^2 + 2 j w T'/dt - w^2 T](m - R/(c dt))
//   fphi = exp(-j k R) T(m - R/(c dt))
// so that K_A = (mu/4pi) fA / R and K_phi = (1/(4 pi eps)) fphi / R.
struct EnvKernel {
    double dt, w, k, cdt;
    TBasis tb{};
    __host__ __device__ void eval(int m, double R, zd& fa, zd& fp) const {
        const double tau = (double)m - R / cdt;
        double d[4];
        if (!tb.eval(tau, d)) {
            fa = {0.0, 0.0};
            fp = {0.0, 0.0};
            return;
        }
        const double c = cos(k * R), s = -sin(k * R);
        const zd ph{c, s};
        const zd pa{d[2] / (dt * dt) - w * w * d[0], 2.0 * w * d[1] / dt};
        fa = ph * pa;
        fp = zd{c * d[0], s * d[0]};
    }
    // CFIE: fA as eval and fH = exp(-j k R) [T'/dt + j w T](m - R/(c dt)),
    // the temporal factor of the MFIE's potential
    __host__ __device__ void evalh(int m, double R, zd& fa, zd& fh) const {
        const double tau = (double)m - R / cdt;
        double d[4];
        if (!tb.eval(tau, d)) {
            fa = {0.0, 0.0};
            fh = {0.0, 0.0};
            return;
        }
        const double c = cos(k * R), s = -sin(k * R);
        const zd ph{c, s};
        const zd pa{d[2] / (dt * dt) - w * w * d[0], 2.0 * w * d[1] / dt};
        fa = ph * pa;
        fh = ph * zd{d[1] / dt, w * d[0]};
    }
    // [T'/dt + j w T] at tau = m on piece m (the MFIE's Gram factor D_m)
    __host__ __device__ zd gram(int m) const {
        double d[4];
        if (!tb.origin(m, d)) return zd{0.0, 0.0};
        return zd{d[1] / dt, w * d[0]};
    }
    // value and R-derivative at R = 0+ (piece m, tau -> m-)
    __host__ __device__ void origin(int m, zd& fa0, zd& fp0, zd& dfa0, zd& dfp0) const {
        double d[4];
        if (!tb.origin(m, d)) {
            fa0 = fp0 = dfa0 = dfp0 = zd{0.0, 0.0};
            return;
        }
        const zd pa{d[2] / (dt * dt) - w * w * d[0], 2.0 * w * d[1] / dt};
        const zd dpa{d[3] / (dt * dt) - w * w * d[1], 2.0 * w * d[2] / dt};
        fa0 = pa;
        fp0 = zd{d[0], 0.0};
        const zd mjk{0.0, -k};
        dfa0 = mjk * pa - (1.0 / cdt) * dpa;
        dfp0 = mjk * fp0 - zd{d[1] / cdt, 0.0};
    }
};

}  // namespace etaim
