// C ABI of the ET-AIM marching library: context set-up, the AIM operator
// (Sec. 4 stages (i)-(iv)), the delayed field, GMRES (stage (v), Sec. 5.1),
// the forward and adjoint marches of eq. (5), excitation and export.
#include <chrono>
#include <cstdlib>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "aim.inc.hip"
#include "context.hpp"
#include "krylov.inc.hip"

using namespace etaim;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(e_ == hipErrorOutOfMemory ? ETAIM_ENOMEM : ETAIM_EHIP,                     \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                       \
    } while (0)

#define CHK(expr)                     \
    do {                              \
        int r_ = (expr);              \
        if (r_ != ETAIM_OK) return r_; \
    } while (0)

constexpr int kLdsBudget = 64 * 1024;
// largest grid y dimension of a launch
constexpr size_t kMaxGridY = 65535;
// batches up to this many columns apply the preconditioner with lane groups per row
constexpr int kSpmvGroupMaxB = 4;
// most blocks one dot product or norm is split over
constexpr int kRedMaxChunks = 64;

int pick_lines(int L, size_t elem, int cap) {
    int mt = (int)(kLdsBudget / (2 * (size_t)(L + 1) * elem));
    return std::max(1, std::min(mt, cap));
}

int blocks_for(size_t n, int threads = 256) {
    size_t b = (n + threads - 1) / threads;
    return (int)std::min<size_t>(std::max<size_t>(b, 1), 65535 * 8);
}

}  // namespace

struct etaim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    etaim_params prm{};
    Geometry geo;
    Setup st;
    GridDims gd{};
    Radix rx{}, ry{}, rz{};
    int ns = 0, B = 0, prec = 0, mv = 0, nnz = 0, ldg = 0, ncu = 256;
    size_t N3 = 0, Np = 0, gfold = 0;
    int64_t dev_bytes = 0;
    std::vector<void*> allocs;
    // FP64 device arrays
    zd *dinv = nullptr, *dinv_c = nullptr, *diag = nullptr, *near64 = nullptr, *nearT64 = nullptr, *ghat64 = nullptr;
    double* lam64 = nullptr;
    int *i0 = nullptr, *korder = nullptr, *rowptr = nullptr, *col = nullptr, *rowof = nullptr, *nptr = nullptr, *nk = nullptr;
    double *Sq = nullptr, *rq = nullptr;
    // CFIE (Sec. 2.1): the MFIE's curl test projection, its Green spectra
    // (G^H, zero), the excitation's weighted S x n; the MFIE far part runs as
    // a second pass of the far pipeline with these in place of the EFIE's
    // (PassSwap), on the same anterpolated currents and history ring
    double *lamH64 = nullptr, *Snq = nullptr;
    zd* ghatH64 = nullptr;
    void *lamH_r = nullptr, *ghatH_r = nullptr, *ghatHT_r = nullptr, *farH = nullptr;
    int farH_slots = 0, farH_r0 = -1, pass = 0;
    // working-precision arrays (float or double)
    void *lam_r = nullptr, *nw_r = nullptr, *near_r = nullptr, *nearT_r = nullptr, *ghat_r = nullptr, *tw_r[3] = {};
    void* ghatT_r = nullptr;  // ky/kz-exchanged copy for the z-lines-first plane kernel
    void *A = nullptr, *P = nullptr, *ring = nullptr;
    void* S = nullptr;  // line-pass engine: full-spectrum work array [bc][kx][kz][ky] (allocated on first use)
    // register x stage: anterpolated grid q[bc][z][x][y], zero outside the
    // nodes some basis reaches (anodes, as plane indices)
    void* Q = nullptr;
    int* anodes = nullptr;
    unsigned long long* xmask = nullptr;  // [z][y]: bit x set where node (x, y, z) is reached
    int n_anodes = 0;
    zd* hist = nullptr;  // [mn][ns][B] in the working precision (sized for complex128)
    // Krylov (FP64)
    zd *Vk = nullptr, *w = nullptr, *h1 = nullptr, *h2 = nullptr, *H = nullptr, *sn = nullptr, *g = nullptr,
       *yv = nullptr, *xk = nullptr, *rhs = nullptr, *zero = nullptr;
    double *cs = nullptr, *nrm = nullptr, *beta = nullptr, *bnorm = nullptr, *resid = nullptr;
    int *active = nullptr, *jcnt = nullptr, *flag = nullptr;
    double* perr = nullptr;  // extrapolation errors of the step just solved (+ block partials)
    // near-zone sparse approximate inverse (right preconditioner) and its transposed copy
    zd *sai = nullptr, *saiT = nullptr, *zt = nullptr;
    // partial sums of the dot products and norms split over several blocks
    void* redpart = nullptr;
    int precond = 1;  // 0: Jacobi diag(Z0)^-1, 1: near-zone sparse approximate inverse
    // interpolation by grid tiles: tile -> bases (CSR), tile origins [ntiles][3]
    int interp_engine = 0, ntiles = 0;
    int *tptr = nullptr, *tbase = nullptr, *torg = nullptr;
    // delayed field in time blocks (register engine): far part of the history
    // sum once per block of delay_block steps into far, near part per step
    int delay_block = 6, far_slots = 0, far_r0 = -1;
    int check_cols = 0;  // FP64 companion: history steps transformed together
    void* far = nullptr;
    // multilevel time blocks of the delayed field (delay_mode 1): level tables
    // [ml_off(ml_levels)][2 gfold], accumulator ring [ml_na][ring slot];
    // ml_step: the step whose sum the accumulators hold complete (-1: rebuild
    // them from the ring), ml_conj: built with conj(G); the *H copies belong
    // to the CFIE's MFIE pass (PassSwap exchanges them)
    int delay_mode = 0, ml_levels = 0, ml_extra = 0, ml_na = 0, ml_step = -1, ml_conj = 0, ml_stepH = -1,
        ml_conjH = 0;
    void *ml_gam = nullptr, *ml_acc = nullptr, *ml_gamH = nullptr, *ml_accH = nullptr;
    int* flag_h = nullptr;
    double* res_h = nullptr;  // pinned: per-column residuals [B], then per-column norms [B]
    int* pnext = nullptr;     // device: extrapolation order chosen for the next step
    // batched-GMRES schedule: steps per host check, captured Arnoldi steps
    int sync_every = 1;
    int iter_hint = 0;  // Arnoldi steps of the last solve of the march (first chunk size)
    // forward march state: the next step the history rings are ready for (-1:
    // none), and the initial-guess order carried into it
    int next_step = -1, guess_p_next = 1;
    bool guess_dev_next = false;
    bool use_graph = false, capturing = false;
    bool no_solver = false;  // an operator-only context (the FP64 check companion): no preconditioner set-up
    int ring_cols = 0;       // columns of a spectrum-ring slot (0: B)
    int check_next = 0;      // companion: the first step its history does not hold yet
    int check_synced = -1;   // the step at which the companion's history continues this context's march
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraphExec_t> graphs[2];  // [conj][j]
    // whole-step graphs of the forward march (ETAIM_F_STEP_GRAPH): device step
    // descriptors of the current call, {descriptor index, live}, per-step
    // Arnoldi steps and residual estimates, pinned readback; graphs by variant
    bool step_graph = false;
    StepDesc* sdesc = nullptr;
    int* sctl = nullptr;
    int* siters = nullptr;
    double* sres = nullptr;
    int* sctl_h = nullptr;
    std::map<int, hipGraphExec_t> step_graphs;
    // launch shapes (0 = automatic); the autotuner sets them
    int gather_rows_t = 0, lines_x_t = 0, interp_waves = 4;
    int yz_engine = 0;  // 0: LDS plane kernels, 1: register quadrant kernels, 2: as 1 with z-lines-first matvec and commit
    int guess_order = kMaxGuess;  // solutions extrapolated into a step's initial guess (0..kMaxGuess)
    int x_engine = 0;   // 0: LDS line kernels, 1: register line kernels
    void* xs = nullptr; // [ns][B] scaled columns for the register anterpolation
    hipEvent_t ev[8] = {};  // march phase events, two sets (steps alternate)
    hipEvent_t evg[2] = {}; // around a run of replayed whole-step graphs
    // FP64 residual check of an FP32 march (ETAIM_F_RESIDUAL_CHECK): an FP64
    // context of the same problem for the monitored column 0, on this stream
    etaim_ctx* check = nullptr;
    // per-kernel-class tracing
    bool prof = false;
    uint32_t prof_mask = 0;  // traced kernel classes, bit ETAIM_K_*
    double k_ms[ETAIM_K_COUNT] = {}, k_bytes[ETAIM_K_COUNT] = {};
    int64_t k_n[ETAIM_K_COUNT] = {};
    std::vector<hipEvent_t> pool;
    struct Pending {
        int cls, ev;
        double bytes;
    };
    std::vector<Pending> pending;
    int pool_next = 0;

    template <typename T>
    int alloc(T*& p, size_t n) {
        void* q = nullptr;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc(&q, n * sizeof(T));
        if (e != hipSuccess) return fail(ETAIM_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
        allocs.push_back(q);
        dev_bytes += (int64_t)(n * sizeof(T));
        p = reinterpret_cast<T*>(q);
        return ETAIM_OK;
    }
    int allocv(void*& p, size_t bytes) {
        unsigned char* q = nullptr;
        CHK(alloc(q, bytes));
        p = q;
        return ETAIM_OK;
    }
    template <typename T>
    int upload(T*& p, const std::vector<T>& v) {
        CHK(alloc(p, v.size()));
        HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return ETAIM_OK;
    }
    ~etaim_ctx() {
        delete check;
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : evg)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : pool) (void)hipEventDestroy(e);
        if (flag_h) (void)hipHostFree(flag_h);
        if (res_h) (void)hipHostFree(res_h);
        for (auto& v : graphs)
            for (auto& x : v)
                if (x) (void)hipGraphExecDestroy(x);
        for (auto& kv : step_graphs) (void)hipGraphExecDestroy(kv.second);
        if (sctl_h) (void)hipHostFree(sctl_h);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (void* p : allocs) (void)hipFree(p);
    }
};

namespace {

// The CFIE's MFIE pass: while one lives, the far pipeline (Green spectra,
// interpolation weights, time-block sums) sees the MFIE's arrays in place of
// the EFIE's; the anterpolation, the transforms and the history ring are
// shared.  Both passes keep their block sums of the same block (far_r0).
struct PassSwap {
    etaim_ctx* c;
    explicit PassSwap(etaim_ctx* cc) : c(cc) { swap(); }
    ~PassSwap() { swap(); }
    void swap() {
        std::swap(c->ghat_r, c->ghatH_r);
        std::swap(c->ghatT_r, c->ghatHT_r);
        std::swap(c->lam_r, c->lamH_r);
        std::swap(c->far, c->farH);
        std::swap(c->far_slots, c->farH_slots);
        std::swap(c->far_r0, c->farH_r0);
        std::swap(c->ml_gam, c->ml_gamH);
        std::swap(c->ml_acc, c->ml_accH);
        std::swap(c->ml_step, c->ml_stepH);
        std::swap(c->ml_conj, c->ml_conjH);
        c->pass ^= 1;
    }
};

// the block whose time-block sums both passes hold (-1: none)
// (-1 also invalidates the multilevel accumulators: the history changed)
inline void set_far_r0(etaim_ctx* c, int r0) {
    c->far_r0 = c->farH_r0 = r0;
    if (r0 < 0) c->ml_step = c->ml_stepH = -1;
}

// Tracing: an event pair around each launch of a class (when enabled).  A
// class of one kernel passes the pair to the launch itself (launch_timed):
// the events then take the dispatch's own start and end, with no queue gap.
struct Trace {
    etaim_ctx* c;
    int cls, idx = -1;
    double bytes;
    bool ext;
    Trace(etaim_ctx* c_, int cls_, double bytes_, bool ext_ = false) : c(c_), cls(cls_), bytes(bytes_), ext(ext_) {
        if (!c->prof || c->capturing || !((c->prof_mask >> cls) & 1u)) return;
        if ((size_t)(c->pool_next + 2) > c->pool.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                c->pool.push_back(e);
            }
        }
        idx = c->pool_next;
        c->pool_next += 2;
        if (!ext) (void)hipEventRecord(c->pool[idx], c->stream);
    }
    hipEvent_t ev0() const { return idx >= 0 ? c->pool[idx] : nullptr; }
    hipEvent_t ev1() const { return idx >= 0 ? c->pool[idx + 1] : nullptr; }
    ~Trace() {
        if (idx < 0) return;
        if (!ext) (void)hipEventRecord(c->pool[idx + 1], c->stream);
        c->pending.push_back({cls, idx, bytes});
    }
};

// the one launch of an ext-mode trace (a plain launch when tracing is off)
template <typename F, typename... Args>
void launch_timed(const Trace& t, F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st, Args... args) {
    if (t.ev0())
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, st, t.ev0(), t.ev1(), 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

// traced launches held before the march resolves them
constexpr size_t kTraceBatch = 2048;

// resolve pending event pairs (waits on the stream)
int trace_flush(etaim_ctx* c) {
    if (c->pending.empty()) return ETAIM_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    for (const auto& p : c->pending) {
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, c->pool[p.ev], c->pool[p.ev + 1]));
        c->k_ms[p.cls] += t;
        c->k_bytes[p.cls] += p.bytes;
        c->k_n[p.cls] += 1;
    }
    c->pending.clear();
    c->pool_next = 0;
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
// pass launchers (templated on the working precision)

template <typename R>
int lines_per_block(const Radix& pl) {
    int mt = 64;
    while (mt > 1 && ((size_t)mt * (pl.L + 1) + pl.L) * sizeof(cplx<R>) > (size_t)kLdsBudget) mt /= 2;
    while (mt > 1 && !plane_fits(mt, pl)) mt /= 2;
    return mt;
}

// a radix plan whose lines the LDS line kernel can take (at least one line
// per block within the LDS budget)
template <typename R>
bool line_fits(const Radix& pl) {
    const int mt = lines_per_block<R>(pl);
    return plane_fits(mt, pl) && ((size_t)mt * (pl.L + 1) + pl.L) * sizeof(cplx<R>) <= (size_t)kLdsBudget;
}

// one four-step line launch; the LDS attribute is raised once per instance
// where the block's buffers pass 64 KB
template <typename R, int A, int B, bool LF, bool HALF>
int launch_l4(etaim_ctx* c, dim3 grid, const cplx<R>* in, cplx<R>* out, const cplx<R>* tw, const LineArgs& a) {
    constexpr size_t lds = lines4_lds<R, A, B, LF>();
    static bool attr = false;
    if (lds > 64 * 1024 && !attr) {
        HIPCHK(hipFuncSetAttribute((const void*)k_lines4<R, A, B, LF, HALF>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr = true;
    }
    hipLaunchKernelGGL((k_lines4<R, A, B, LF, HALF>), grid, dim3(lines4_threads<R, A, B>()), lds, c->stream, in, out,
                       tw, a);
    HIPCHK(hipGetLastError());
    return ETAIM_OK;
}
template <typename R, int A, int B>
int launch_l4(etaim_ctx* c, bool lf, dim3 grid, const cplx<R>* in, cplx<R>* out, const cplx<R>* tw,
              const LineArgs& a) {
    // the zero-padded forward input or the pruned inverse output, fixed at compile time
    const int L = A * B;
    const bool half = a.inverse ? (a.out_len == L / 2 && a.in_len == L) : (a.in_len == L / 2 && a.out_len == L);
    if (half)
        return lf ? launch_l4<R, A, B, true, true>(c, grid, in, out, tw, a)
                  : launch_l4<R, A, B, false, true>(c, grid, in, out, tw, a);
    return lf ? launch_l4<R, A, B, true, false>(c, grid, in, out, tw, a)
              : launch_l4<R, A, B, false, false>(c, grid, in, out, tw, a);
}
// the four-step instances of lines4_split
#define ETAIM_L4_SPLITS(X) X(8, 12) X(12, 12) X(8, 24) X(12, 24) X(16, 24) X(24, 24)

template <typename R>
int launch_lines(etaim_ctx* c, const cplx<R>* in, cplx<R>* out, const cplx<R>* tw, const Radix& pl, int nf,
                 int nslow, int in_len, int out_len, long long in_f, long long in_s, long long in_p,
                 long long out_f, long long out_s, long long out_p, bool inverse, int ns0 = 0,
                 long long in_s1 = 0, long long out_s1 = 0, const int* gate = nullptr, int mt = 0) {
    LineArgs a{};
    a.gate = gate;
    a.ns0 = ns0 > 0 ? ns0 : nslow;
    a.in_s1 = in_s1;
    a.out_s1 = out_s1;
    a.pl = pl;
    a.nf = nf;
    a.in_len = in_len;
    a.out_len = out_len;
    a.in_f = in_f;
    a.in_s = in_s;
    a.in_p = in_p;
    a.out_f = out_f;
    a.out_s = out_s;
    a.out_p = out_p;
    a.inverse = inverse ? 1 : 0;
    int A4 = 0, B4 = 0;
    if (lines4_split(pl.L, A4, B4)) {
        // register four-step lines; lanes over the lines where the lines are adjacent
        const bool lf = in_f == 1 || out_f == 1;
        const dim3 grid4((nf + lines4_mt<R>() - 1) / lines4_mt<R>(), nslow);
#define ETAIM_L4_CASE(AA, BB) \
    if (A4 == AA && B4 == BB) return launch_l4<R, AA, BB>(c, lf, grid4, in, out, tw, a);
        ETAIM_L4_SPLITS(ETAIM_L4_CASE)
#undef ETAIM_L4_CASE
    }
    a.mt = mt > 0 ? mt : lines_per_block<R>(pl);
    const size_t lds = ((size_t)a.mt * (pl.L + 1) + pl.L) * sizeof(cplx<R>);
    dim3 grid((nf + a.mt - 1) / a.mt, nslow);
    hipLaunchKernelGGL(k_lines<R>, grid, dim3(kPlaneThreads), lds, c->stream, in, out, tw, a);
    HIPCHK(hipGetLastError());
    return ETAIM_OK;
}

// N of the register x-line kernels (N_x = N, N | 48 with a register codelet), 0 if none
int xline_n(const etaim_ctx* c) {
    const int n = c->gd.N[0];
    if (c->gd.L[0] != 2 * n) return 0;
    return (n == 16 || n == 24 || n == 48) ? n : 0;
}

// the register x stage applies: a register x-line codelet, or four-step
// lines of length L_x (the anterpolated grid is then transformed by them)
bool xreg_ok(const etaim_ctx* c) {
    int A = 0, B = 0;
    return xline_n(c) > 0 || (c->gd.L[0] == 2 * c->gd.N[0] && lines4_split(c->gd.L[0], A, B));
}

// N of the register quadrant kernels for this grid (N_y = N_z = N, N | 48
// with a register codelet), 0 if they do not apply
int quad_n(const etaim_ctx* c) {
    const int n = c->gd.N[1];
    if (c->gd.N[2] != n || c->gd.L[1] != 2 * n || c->gd.L[2] != 2 * n) return 0;
    return (n == 16 || n == 24 || n == 48) ? n : 0;
}

// columns per block of the grid-tile interpolation (a power of two, its LDS
// box of 4 GC potential planes within 69 KB)
template <typename R>
int interp_tile_gc(const etaim_ctx* c) {
    const int cap = sizeof(R) == 4 ? 4 : 2;
    int gc = 1;
    while (gc < cap && gc < c->B) gc *= 2;
    return gc;
}
template <typename R>
size_t interp_tile_lds(const etaim_ctx* c) {
    return (size_t)4 * interp_tile_gc<R>(c) * kBoxN * sizeof(cplx<R>);
}

template <typename R>
struct Ops {
    static cplx<R>* A(etaim_ctx* c) { return (cplx<R>*)c->A; }
    static cplx<R>* P(etaim_ctx* c) { return (cplx<R>*)c->P; }
    static cplx<R>* Q(etaim_ctx* c) { return (cplx<R>*)c->Q; }
    static const cplx<R>* tw(etaim_ctx* c, int a) { return (const cplx<R>*)c->tw_r[a]; }
    static const cplx<R>* ghat(etaim_ctx* c) { return (const cplx<R>*)c->ghat_r; }
    static const cplx<R>* ghatT(etaim_ctx* c) { return (const cplx<R>*)c->ghatT_r; }
    // near-zone values; the adjoint (conjugated) operators use the transposed
    // values: the exact entries are symmetric only up to quadrature
    static const cplx<R>* nearv(etaim_ctx* c, int conj) {
        return (const cplx<R>*)(conj ? c->nearT_r : c->near_r);
    }
    static cplx<R>* ring(etaim_ctx* c) { return (cplx<R>*)c->ring; }
    static cplx<R>* S(etaim_ctx* c) { return (cplx<R>*)c->S; }

    // ---- line-pass y/z engine (yz_engine 3): S = the y/z spectrum of the A planes
    static int ensure_S(etaim_ctx* c) {
        if (c->S) return ETAIM_OK;
        if (c->capturing) return fail(ETAIM_EUNSUPPORTED, "the line-pass work array is not allocated");
        return c->allocv(c->S, (size_t)4 * c->B * c->Np * sizeof(cplx<R>));
    }
    // A[bc][kx][z][y] -> S rows z < Nz: zero-padded forward y transforms
    static int ylines_fwd(etaim_ctx* c, const int* gate) {
        const GridDims& g = c->gd;
        const long long Ny = g.N[1], Nz = g.N[2], Ly = g.L[1], Lz = g.L[2];
        return launch_lines<R>(c, A(c), S(c), tw(c, 1), c->ry, (int)Nz, 4 * c->B * g.L[0], (int)Ny, (int)Ly, Ny,
                               Ny * Nz, 1, Ly, Ly * Lz, 1, false, 0, 0, 0, gate);
    }
    // S rows z < Nz -> A[bc][kx][z][y]: inverse y transforms kept to y < Ny
    static int ylines_inv(etaim_ctx* c, const int* gate) {
        const GridDims& g = c->gd;
        const long long Ny = g.N[1], Nz = g.N[2], Ly = g.L[1], Lz = g.L[2];
        return launch_lines<R>(c, S(c), A(c), tw(c, 1), c->ry, (int)Nz, 4 * c->B * g.L[0], (int)Ly, (int)Ny, Ly,
                               Ly * Lz, 1, Ny, Ny * Nz, 1, true, 0, 0, 0, gate);
    }
    // S rows z < Nz: forward z transforms, product with the Green spectrum G,
    // inverse, rows z < Nz stored back (four-step register lines where L_z
    // splits, else the LDS passes)
    template <int A, int B>
    static int zg4(etaim_ctx* c, const cplx<R>* G, int conj, const int* gate) {
        constexpr size_t lds = lines4_lds<R, A, B, true>();
        static bool attr = false;
        if (lds > 64 * 1024 && !attr) {
            HIPCHK(hipFuncSetAttribute((const void*)k_zg4<R, A, B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
            attr = true;
        }
        const GridDims& g = c->gd;
        const int mt = lines4_mt<R>();
        hipLaunchKernelGGL((k_zg4<R, A, B>), dim3((g.L[1] + mt - 1) / mt, 4 * c->B * g.L[0]),
                           dim3(lines4_threads<R, A, B>()), lds, c->stream, S(c), G, tw(c, 2), g, conj, gate);
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    static int zlines_green(etaim_ctx* c, const cplx<R>* G, int conj, const int* gate) {
        const GridDims& g = c->gd;
        int A4 = 0, B4 = 0;
        if (lines4_split(g.L[2], A4, B4)) {
#define ETAIM_ZG4_CASE(AA, BB) \
    if (A4 == AA && B4 == BB) return zg4<AA, BB>(c, G, conj, gate);
            ETAIM_L4_SPLITS(ETAIM_ZG4_CASE)
#undef ETAIM_ZG4_CASE
        }
        const int mt = lines_per_block<R>(c->rz);
        const size_t lds = ((size_t)mt * (g.L[2] + 1) + g.L[2]) * sizeof(cplx<R>);
        hipLaunchKernelGGL(k_zlines_green<R>, dim3((g.L[1] + mt - 1) / mt, 4 * c->B * g.L[0]), dim3(kPlaneThreads),
                           lds, c->stream, S(c), G, tw(c, 2), c->rz, g, mt, conj, gate);
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    // S rows z < Nz -> out (every kz): zero-padded forward z transforms
    static int zlines_fwd(etaim_ctx* c, cplx<R>* out) {
        const GridDims& g = c->gd;
        const long long Nz = g.N[2], Ly = g.L[1], Lz = g.L[2];
        return launch_lines<R>(c, S(c), out, tw(c, 2), c->rz, (int)Ly, 4 * c->B * g.L[0], (int)Nz, (int)Lz, 1,
                               Ly * Lz, Ly, 1, Ly * Lz, Ly, false);
    }
    // S (every kz) -> S rows z < Nz: inverse z transforms, in place
    static int zlines_inv(etaim_ctx* c) {
        const GridDims& g = c->gd;
        const long long Nz = g.N[2], Ly = g.L[1], Lz = g.L[2];
        return launch_lines<R>(c, S(c), S(c), tw(c, 2), c->rz, (int)Ly, 4 * c->B * g.L[0], (int)Lz, (int)Nz, 1,
                               Ly * Lz, Ly, 1, Ly * Lz, Ly, true);
    }

    // anterpolate x (optionally scaled by dinv) and forward x pass -> A
    static int gather_rows(etaim_ctx* c) {
        // 4 * mr lines of length Lx in one LDS buffer (in-place FFT)
        const int Lx = c->gd.L[0];
        if (c->gather_rows_t > 0) return c->gather_rows_t;
        int mr = sizeof(R) == 4 ? 16 : 8;
        while (mr > 1 && (!plane_fits(4 * mr, c->rx) ||
                          (4 * (size_t)mr * (Lx + 1) + Lx) * sizeof(cplx<R>) > (size_t)160 * 1024))
            mr /= 2;
        return mr;
    }
    static size_t gather_lds(etaim_ctx* c) {
        return ((size_t)4 * gather_rows(c) * (c->gd.L[0] + 1) + c->gd.L[0]) * sizeof(cplx<R>);
    }
    // xs_ready: the scaled columns are already in c->xs ([ns][B], register x stage only)
    static int forward_x(etaim_ctx* c, const zd* x, const zd* dinv, int conj_in, const int* gate = nullptr,
                         bool xs_ready = false) {
        const GridDims& g = c->gd;
        const int mr = gather_rows(c);
        dim3 grid((g.N[1] + mr - 1) / mr, g.N[2], c->B);
        const double s = sizeof(cplx<R>), nB = (double)c->B * c->ns;
        const double a_sz = 4.0 * c->B * g.L[0] * g.N[2] * g.N[1] * s;
        Trace t(c, ETAIM_K_ANTERP_X, nB * 16 + 64.0 * c->ns * (4 + 4 * sizeof(R)) + (c->N3 + 1) * 4.0 + a_sz +
                                         (dinv ? c->ns * 16.0 : 0.0));
        if (c->x_engine == 1) {
            cplx<R>* xs = (cplx<R>*)c->xs;
            if (!xs_ready)
                hipLaunchKernelGGL(k_prescale<R>, dim3(blocks_for(nB)), dim3(256), 0, c->stream, x, dinv, xs, c->ns,
                                   c->B, conj_in, gate);
            if (c->n_anodes > 0)
                hipLaunchKernelGGL(k_anterp_nz<R>, dim3(blocks_for((size_t)c->n_anodes * c->B)), dim3(256), 0,
                                   c->stream, xs, c->anodes, c->n_anodes, c->nptr, c->nk, (const R*)c->nw_r, Q(c), g,
                                   c->B, gate);
            if (!xline_n(c)) {
                // four-step lines along x, q[bc][z][x][y] -> A[bc][kx][z][y], zero-padded
                const long long Lx = g.L[0], Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
                return launch_lines<R>(c, Q(c), A(c), tw(c, 0), c->rx, (int)Ny, (int)(4 * c->B * Nz), (int)Nx,
                                       (int)Lx, 1, Nx * Ny, Ny, 1, Ny, Nz * Ny, false, (int)Nz, Nz * Nx * Ny,
                                       Lx * Nz * Ny, gate);
            }
            const dim3 gx((2 * g.N[1] * g.N[2] + 255) / 256, 4 * c->B);
            const cplx<R>* zsrc = (const cplx<R>*)c->zero;
            switch (xline_n(c)) {
                case 16: hipLaunchKernelGGL((k_xfwd<R, 16>), gx, dim3(256), 0, c->stream, Q(c), A(c), g, c->xmask, zsrc, gate); break;
                case 24: hipLaunchKernelGGL((k_xfwd<R, 24>), gx, dim3(256), 0, c->stream, Q(c), A(c), g, c->xmask, zsrc, gate); break;
                case 48: hipLaunchKernelGGL((k_xfwd<R, 48>), gx, dim3(256), 0, c->stream, Q(c), A(c), g, c->xmask, zsrc, gate); break;
                default: return fail(ETAIM_EUNSUPPORTED, "register x-line kernels need N_x in {16, 24, 48}");
            }
            HIPCHK(hipGetLastError());
            return ETAIM_OK;
        }
        hipLaunchKernelGGL(k_fwdx_gather<R>, grid, dim3(kPlaneThreads), gather_lds(c), c->stream, x, dinv, c->nptr,
                           c->nk, (const R*)c->nw_r, A(c), tw(c, 0), c->rx, g, mr, c->ns, conj_in, gate);
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    // inverse x pass A[bc][kx][z][y] -> P[bc][z][y][x]
    static int inverse_x(etaim_ctx* c, const int* gate = nullptr) {
        const GridDims& g = c->gd;
        const long long Lx = g.L[0], Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
        const double s = sizeof(cplx<R>), bc = 4.0 * c->B;
        // one register kernel (events on its dispatch) or the line launches
        Trace t(c, ETAIM_K_FFT_X_INV, bc * Lx * Nz * Ny * s + bc * c->N3 * s, c->x_engine == 1 && xline_n(c) > 0);
        if (c->x_engine == 1 && xline_n(c)) {
            const dim3 gx((unsigned)((2 * Ny * Nz + 255) / 256), (unsigned)(4 * c->B));
            switch (xline_n(c)) {
                case 16: launch_timed(t, k_xinv<R, 16>, gx, dim3(256), 0, c->stream, A(c), P(c), g, gate); break;
                case 24: launch_timed(t, k_xinv<R, 24>, gx, dim3(256), 0, c->stream, A(c), P(c), g, gate); break;
                case 48: launch_timed(t, k_xinv<R, 48>, gx, dim3(256), 0, c->stream, A(c), P(c), g, gate); break;
                default: return fail(ETAIM_EUNSUPPORTED, "register x-line kernels need N_x in {16, 24, 48}");
            }
            HIPCHK(hipGetLastError());
            return ETAIM_OK;
        }
        // lines (y fastest) of the LDS line kernel, written to P[bc][z][x][y]
        return launch_lines<R>(c, A(c), P(c), tw(c, 0), c->rx, (int)Ny, (int)(4 * c->B * Nz), (int)Lx, (int)Nx, 1,
                               Ny, Nz * Ny, 1, Nx * Ny, Ny, true, (int)Nz, Lx * Nz * Ny, Nz * Nx * Ny, gate,
                               c->lines_x_t);
    }
    static size_t plane_lds(etaim_ctx* c) {
        return ((size_t)c->gd.L[2] * (c->gd.L[1] + 1) + c->gd.L[1] + c->gd.L[2]) * sizeof(cplx<R>);
    }
    static size_t quad_lds(etaim_ctx* c) { return (size_t)4 * quad_n(c) * (quad_n(c) + 1) * sizeof(cplx<R>); }
    static size_t zline_lds(etaim_ctx* c) { return (size_t)2 * quad_n(c) * (quad_n(c) + 1) * sizeof(cplx<R>); }
    static int yz_green(etaim_ctx* c, int m, int conj, const int* gate = nullptr) {
        const GridDims& g = c->gd;
        dim3 grid(g.L[0], 4 * c->B);
        const double s = sizeof(cplx<R>);
        if (c->yz_engine == 3) {
            CHK(ensure_S(c));
            Trace t(c, ETAIM_K_YZ_GREEN, 2.0 * 4 * c->B * g.L[0] * g.N[2] * g.N[1] * s + 2.0 * c->gfold * s);
            CHK(ylines_fwd(c, gate));
            CHK(zlines_green(c, ghat(c) + (size_t)m * 2 * c->gfold, conj, gate));
            return ylines_inv(c, gate);
        }
        Trace t(c, ETAIM_K_YZ_GREEN, 2.0 * 4 * c->B * g.L[0] * g.N[2] * g.N[1] * s + 2.0 * c->gfold * s, true);
        if (c->yz_engine == 2) {
            const cplx<R>* G = ghatT(c) + (size_t)m * 2 * c->gfold;
            const size_t lds = zline_lds(c);
            grid = dim3(4 * c->B, g.L[0]);
            switch (quad_n(c)) {
                case 16: launch_timed(t, k_yzc_green<R, 16>, grid, dim3(4 * 16), lds, c->stream, A(c), G, tw(c, 1), tw(c, 2), g, conj, gate); break;
                case 24: launch_timed(t, k_yzc_green<R, 24>, grid, dim3(4 * 24), lds, c->stream, A(c), G, tw(c, 1), tw(c, 2), g, conj, gate); break;
                case 48: launch_timed(t, k_yzc_green<R, 48>, grid, dim3(4 * 48), lds, c->stream, A(c), G, tw(c, 1), tw(c, 2), g, conj, gate); break;
                default: return fail(ETAIM_EUNSUPPORTED, "register plane kernels need N_y = N_z in {16, 24, 48}");
            }
            HIPCHK(hipGetLastError());
            return ETAIM_OK;
        }
        if (c->yz_engine == 1) {
            const cplx<R>* G = ghat(c) + (size_t)m * 2 * c->gfold;
            const size_t lds = quad_lds(c);
            grid = dim3(4 * c->B, g.L[0]);
            switch (quad_n(c)) {
                case 16: launch_timed(t, k_yzq_green<R, 16>, grid, dim3(kQuadThreads), lds, c->stream, A(c), G, tw(c, 1), tw(c, 2), g, conj, gate); break;
                case 24: launch_timed(t, k_yzq_green<R, 24>, grid, dim3(kQuadThreads), lds, c->stream, A(c), G, tw(c, 1), tw(c, 2), g, conj, gate); break;
                case 48: launch_timed(t, k_yzq_green<R, 48>, grid, dim3(kQuadThreads), lds, c->stream, A(c), G, tw(c, 1), tw(c, 2), g, conj, gate); break;
                default: return fail(ETAIM_EUNSUPPORTED, "register plane kernels need N_y = N_z in {16, 24, 48}");
            }
            HIPCHK(hipGetLastError());
            return ETAIM_OK;
        }
        launch_timed(t, k_yz_green<R>, grid, dim3(kPlaneThreads), plane_lds(c), c->stream, A(c),
                     ghat(c) + (size_t)m * 2 * c->gfold, tw(c, 1), tw(c, 2), c->ry, c->rz, g, conj, gate);
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    static int interp_near(etaim_ctx* c, int mode, const zd* x, const zd* dinv, int m, int cur, int nmh,
                           const zd* V, zd* y, int conj_v, int conj_x, const int* gate = nullptr,
                           StepRef sr = {}) {
        // whole multiple of the XCD count: the kernel's block -> basis map is a bijection
        const int wpb = c->interp_waves;
        dim3 grid(((c->ns + wpb - 1) / wpb + kXcds - 1) / kXcds * kXcds);
        const double s = sizeof(cplx<R>), nB = (double)c->B * c->ns;
        const double nvals = mode == 0 ? (m <= c->st.mn ? 1.0 : 0.0) : (double)nmh;
        Trace t(c, ETAIM_K_INTERP_NEAR,
                4.0 * c->B * c->N3 * s + c->ns * (256.0 * sizeof(R) + 12.0) + (c->ns + 1) * 4.0 + c->nnz * 4.0 +
                    c->nnz * nvals * s + (mode == 0 ? nB * 16 : (nmh + 1) * nB * 16) + nB * 16);
        cplx<R>* xs = (cplx<R>*)c->xs;
        // the near zone reads the scaled columns [ns][B]; the register x stage
        // has already written them for this x
        if (mode == 0 && (c->x_engine != 1 || conj_x))
            hipLaunchKernelGGL(k_prescale<R>, dim3(blocks_for(nB)), dim3(256), 0, c->stream, x, dinv, xs, c->ns, c->B,
                               conj_x, gate);
        if (c->interp_engine == 1 && c->ntiles > 0 && mode <= 1) {
            const int gc = interp_tile_gc<R>(c);
            const int nblk = c->ntiles * ((c->B + gc - 1) / gc);
            const dim3 tg((nblk + kXcds - 1) / kXcds * kXcds);
            const size_t lds = interp_tile_lds<R>(c);
#define ETAIM_TILE(GC)                                                                                               \
    hipLaunchKernelGGL((k_interp_tile<R, GC>), tg, dim3(kTileThreads), lds, c->stream, (const cplx<R>*)P(c), (const R*)c->lam_r, \
                       c->i0, c->tptr, c->tbase, c->torg, c->ntiles, c->gd, c->rowptr, c->col, nearv(c, conj_v), c->mv, \
                       (const cplx<R>*)xs, m, (const cplx<R>*)c->hist, std::max(c->st.mn, 1), cur, nmh, V, y, c->ns,   \
                       mode, conj_v, gate, sr)
            switch (gc) {
                case 1: ETAIM_TILE(1); break;
                case 2: ETAIM_TILE(2); break;
                default: ETAIM_TILE(4); break;
            }
#undef ETAIM_TILE
            HIPCHK(hipGetLastError());
            return ETAIM_OK;
        }
        hipLaunchKernelGGL(k_interp_near<R>, grid, dim3(64 * wpb), 0, c->stream, (const cplx<R>*)P(c),
                           (const R*)c->lam_r, c->i0, c->korder, c->gd, c->rowptr, c->col, nearv(c, conj_v), c->mv,
                           (const cplx<R>*)xs, m, (const cplx<R>*)c->hist, std::max(c->st.mn, 1), cur, nmh, V, y,
                           c->ns, mode, conj_v, gate, sr);
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    // y = conj?(Z_m) (dinv . x)
    // (xs_ready: x is given as the scaled columns in c->xs, register x stage only)
    static int apply(etaim_ctx* c, int m, const zd* x, const zd* dinv, zd* y, int conj,
                     const int* gate = nullptr, bool xs_ready = false) {
        if (c->st.cfie && conj) return fail(ETAIM_EUNSUPPORTED, "the CFIE's transposed operators are not built");
        CHK(forward_x(c, x, dinv, 0, gate, xs_ready));
        CHK(yz_green(c, m, conj, gate));
        CHK(inverse_x(c, gate));
        CHK(interp_near(c, 0, x, dinv, m, 0, 0, nullptr, y, conj, 0, gate));
        if (!c->st.cfie) return ETAIM_OK;
        // the MFIE far part, added to y (the register x stage's scaled
        // columns are in place after the first pass)
        PassSwap ps(c);
        CHK(forward_x(c, x, dinv, 0, gate, xs_ready || c->x_engine == 1));
        CHK(yz_green(c, m, conj, gate));
        CHK(inverse_x(c, gate));
        return interp_near(c, 2, x, dinv, m, 0, 0, nullptr, y, conj, 0, gate);
    }
    // rhs = V - sum_{m>=1} conj?(Z_m) I_{cur-m} from the rings (cur >= 1).
    // Captured into a whole-step graph (sr.sd set) the step's values come from
    // its descriptor; graph_far then says whether the time-block pass runs.
    static bool blocks_on(const etaim_ctx* c) {
        return (c->yz_engine >= 1) && c->delay_block > 1 && c->st.ng <= kFarMaxNg && c->delay_block <= kFarMaxBlock;
    }
    // the block sums' pb spectrum slots (reallocated when a longer block is set)
    static int ensure_far(etaim_ctx* c, int pb) {
        if (c->far_slots >= pb) return ETAIM_OK;
        if (c->capturing) return fail(ETAIM_EUNSUPPORTED, "the time-block sums are not allocated");
        const size_t slot = (size_t)4 * c->B * c->Np;
        if (c->far) {
            auto it = std::find(c->allocs.begin(), c->allocs.end(), c->far);
            if (it != c->allocs.end()) c->allocs.erase(it);
            HIPCHK(hipFree(c->far));
            c->dev_bytes -= (int64_t)((size_t)c->far_slots * slot * sizeof(cplx<R>));
            c->far = nullptr;
            c->far_slots = 0;
        }
        CHK(c->allocv(c->far, (size_t)pb * slot * sizeof(cplx<R>)));
        c->far_slots = pb;
        return ETAIM_OK;
    }
    // multilevel time blocks (delay_mode 1): eager steps, N_g within the
    // levels' reach
    static bool ml_on(const etaim_ctx* c, bool graph) {
        return c->delay_mode == 1 && !graph && c->st.ng >= kMlBase && c->st.ng <= ml_max_ng();
    }
    // level tables from the FP64 Green spectra (the MFIE's in the CFIE's
    // second pass) and the accumulator ring
    static int ml_setup(etaim_ctx* c) {
        if (c->ml_acc) return ETAIM_OK;
        const int ng = c->st.ng;
        int nlev = 0;
        while (nlev < kMlLevels && ml_s(nlev) <= ng) ++nlev;
        // further top-length segments for the lags from 2 S_top on
        const int st = ml_s(kMlLevels - 1);
        const int nextra = nlev == kMlLevels ? std::max(0, (ng + 1 + st - 1) / st - 2) : 0;
        const size_t gs = 2 * c->gfold, slot = (size_t)4 * c->B * c->Np;
        const int na = ml_s(nlev - 1);
        cplx<R>* gam = nullptr;
        cplx<R>* acc = nullptr;
        CHK(c->alloc(gam, (size_t)(nextra ? ml_off_extra(nextra + 1) : ml_off(nlev)) * gs));
        hipLaunchKernelGGL(k_ml_gamma<R>, dim3(blocks_for(gs)), dim3(256), 0, c->stream,
                           c->pass ? c->ghatH64 : c->ghat64, gam, gs, ng, nlev, nextra);
        HIPCHK(hipGetLastError());
        CHK(c->alloc(acc, (size_t)na * slot));
        c->ml_gam = gam;
        c->ml_acc = acc;
        c->ml_levels = nlev;
        c->ml_extra = nextra;
        c->ml_na = na;
        c->ml_step = -1;
        return ETAIM_OK;
    }
    // the passes of levels k0..k1 at step e in one sweep (first: k1 is the
    // top level, whose sums start the accumulator slots; sums of steps below
    // lo are not written); seg >= 1: the further top-length segment seg
    static int ml_pass(etaim_ctx* c, int k0, int k1, int e, int conj, int first, int lo, int seg = 0) {
        const size_t slot = (size_t)4 * c->B * c->Np, gs = 2 * c->gfold;
        const double s = sizeof(cplx<R>), S1 = ml_s(k1);
        double gam_b = 0;
        for (int k = k0; k <= k1; ++k) gam_b += 2.0 * ml_s(k) * gs * s;
        Trace t(c, ETAIM_K_RING_FAR, (2.0 * S1 + (first ? 1.0 : 2.0) * S1) * slot * s + gam_b, true);
        const dim3 grid((unsigned)((slot + 255) / 256));
        const cplx<R>* rg = (const cplx<R>*)ring(c);
        // a further segment's spectra where the kernel looks for the top level's
        const cplx<R>* gm = (const cplx<R>*)c->ml_gam +
                            (seg ? (std::ptrdiff_t)(ml_off_extra(seg) - ml_off(kMlLevels - 1)) * (std::ptrdiff_t)gs : 0);
        const int dly = seg * ml_s(kMlLevels - 1);
        cplx<R>* acc = (cplx<R>*)c->ml_acc;
        const GridDims& g = c->gd;
        // parity quadrants for the register plane engines, plain slots for
        // the LDS plane and line-pass engines
        const int qn = c->yz_engine == 1 || c->yz_engine == 2 ? quad_n(c) : 0;
#define ETAIM_ML(K0, K1, QQ)                                                                                        \
    launch_timed(t, k_ml_pass<R, K0, K1, QQ>, grid, dim3(256), 0, c->stream, rg, gm, acc, g, slot, gs, c->st.ng, e, \
                 c->ml_na, conj, first, lo, dly)
#define ETAIM_ML_Q(K0, K1)                                                                               \
    switch (qn) {                                                                                        \
        case 0: ETAIM_ML(K0, K1, 0); break;                                                              \
        case 16: ETAIM_ML(K0, K1, 16); break;                                                            \
        case 24: ETAIM_ML(K0, K1, 24); break;                                                            \
        case 48: ETAIM_ML(K0, K1, 48); break;                                                            \
        default: return fail(ETAIM_EUNSUPPORTED, "multilevel time blocks: no slot layout for this engine"); \
    }
        static_assert(kMlFused == 3 && kMlLevels == 5, "the pass table below covers these levels");
        if (seg && (k0 != kMlLevels - 1 || k1 != kMlLevels - 1))
            return fail(ETAIM_EINVAL, "multilevel time blocks: a further segment has the top length");
        const int key = 10 * k0 + k1;
        switch (key) {
            case 0: ETAIM_ML_Q(0, 0) break;
            case 1: ETAIM_ML_Q(0, 1) break;
            case 2: ETAIM_ML_Q(0, 2) break;
            case 33: ETAIM_ML_Q(3, 3) break;
            case 44: ETAIM_ML_Q(4, 4) break;
            default: return fail(ETAIM_EINVAL, "multilevel time blocks: no pass for these levels");
        }
#undef ETAIM_ML_Q
#undef ETAIM_ML
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    // the passes due at step e (the levels k with S_k | e + 1 among `due`, a
    // bit per level), in a fixed order: the top level first (it starts the
    // slots it reaches), the further top-length segments, then the fused low
    // levels 0..kt, then the other levels upwards; a march and a rebuild run
    // the same passes in the same order, so their sums round alike
    static int ml_event(etaim_ctx* c, int e, unsigned due, int conj, int lo) {
        const int top = c->ml_levels - 1;
        const bool top_due = (due >> top) & 1u;
        int kt = -1;
        for (int k = 0; k < std::min(kMlFused, c->ml_levels); ++k)
            if ((due >> k) & 1u) kt = k;
        if (top_due && top >= kMlFused) CHK(ml_pass(c, top, top, e, conj, 1, lo));
        if (top_due)
            for (int j = 1; j <= c->ml_extra; ++j) CHK(ml_pass(c, top, top, e, conj, 0, lo, j));
        if (kt >= 0) CHK(ml_pass(c, 0, kt, e, conj, top_due && kt == top ? 1 : 0, lo));
        for (int k = kMlFused; k < top; ++k)
            if ((due >> k) & 1u) CHK(ml_pass(c, k, k, e, conj, 0, lo));
        return ETAIM_OK;
    }
    // bring the accumulators to step cur: the passes of the blocks that end
    // at cur - 1 after a step cur - 1, else a rebuild from the ring (every
    // level's last completed block before cur, grouped by step)
    static int ml_advance(etaim_ctx* c, int cur, int conj) {
        CHK(ml_setup(c));
        if (c->ml_step >= 0 && c->ml_conj == conj) {
            if (c->ml_step == cur) return ETAIM_OK;
            if (c->ml_step == cur - 1) {
                unsigned due = 0;
                for (int k = 0; k < c->ml_levels; ++k)
                    if (cur % ml_s(k) == 0) due |= 1u << k;
                if (due) CHK(ml_event(c, cur - 1, due, conj, 0));
                c->ml_step = cur;
                return ETAIM_OK;
            }
        }
        // steps before the top level's first block (cur < S_top) start from
        // these zeros, as they do in a march begun at step 0
        const size_t slot = (size_t)4 * c->B * c->Np;
        HIPCHK(hipMemsetAsync(c->ml_acc, 0, (size_t)c->ml_na * slot * sizeof(cplx<R>), c->stream));
        // level k's last block ends at e_k = S_k floor(cur / S_k) - 1; the
        // higher the level, the earlier (S_k divides S_{k+1})
        for (int k = c->ml_levels - 1; k >= 0; --k) {
            const int e = ml_s(k) * (cur / ml_s(k)) - 1;
            if (e < 0 || (k + 1 < c->ml_levels && e == ml_s(k + 1) * (cur / ml_s(k + 1)) - 1)) continue;
            unsigned due = 0;
            for (int j = 0; j < c->ml_levels; ++j)
                if (ml_s(j) * (cur / ml_s(j)) - 1 == e) due |= 1u << j;
            CHK(ml_event(c, e, due, conj, cur));
        }
        c->ml_step = cur;
        c->ml_conj = conj;
        return ETAIM_OK;
    }
    static int delayed(etaim_ctx* c, int cur, const zd* V, zd* rhs, int conj, StepRef sr = {}, int graph_far = 0) {
        if (c->st.cfie && conj) return fail(ETAIM_EUNSUPPORTED, "the CFIE's adjoint march is not built");
        CHK(delayed_pass(c, cur, V, rhs, conj, sr, graph_far, 1));
        if (!c->st.cfie) return ETAIM_OK;
        // the MFIE far part of the history sum, subtracted from rhs
        PassSwap ps(c);
        return delayed_pass(c, cur, V, rhs, conj, sr, graph_far, 3);
    }
    // one pass of the delayed field; the interpolation in `mode` (1: rhs =
    // V - far - near history; 3: rhs -= far)
    static int delayed_pass(etaim_ctx* c, int cur, const zd* V, zd* rhs, int conj, StepRef sr, int graph_far,
                            int mode) {
        const GridDims& g = c->gd;
        const int nm = std::min(c->st.ng, cur);
        const int ng = c->st.ng;
        const bool graph = sr.sd != nullptr;
        // time blocks (register engine): at step r0 + j the terms that read history
        // older than r0 (m > j) are summed for the whole block at its first step, the
        // j terms of the block's own steps at the step itself
        const int pb = c->delay_block;
        // multilevel time blocks: lags below kMlBase summed here, the rest
        // from the step's accumulator slot
        const bool ml = ml_on(c, graph) && cur >= 1;
        const bool blocked = !ml && blocks_on(c) && cur >= 1;
        const int r0 = blocked ? cur - (cur - 1) % pb : 0;
        const bool far_pass = graph ? (blocked && graph_far != 0) : (blocked && c->far_r0 != r0);
        if (graph && blocked && (!c->far || c->far_slots < pb))
            return fail(ETAIM_EUNSUPPORTED, "whole-step graph: the time-block sums are not allocated");
        const int nmx = ml ? std::min(nm, kMlBase - 1) : blocked ? std::min(cur - r0, ng) : nm;
        const cplx<R>* Fml = nullptr;
        if (ml) {
            CHK(ml_advance(c, cur, conj));
            Fml = (const cplx<R>*)c->ml_acc + (size_t)(cur % c->ml_na) * 4 * c->B * c->Np;
        }
        {
            const double s = sizeof(cplx<R>), slot_b = 4.0 * c->B * c->Np * s, green_b = 2.0 * c->gfold * s;
            double bytes = nmx * (slot_b + green_b) + 4.0 * c->B * g.L[0] * g.N[2] * g.N[1] * s;
            if (blocked || ml) bytes += slot_b;
            if (c->yz_engine == 3) {
                // the sum over the history into S (from the step's block sum with
                // time blocks), then the inverse z and y passes
                if (graph) return fail(ETAIM_EUNSUPPORTED, "whole-step graph: needs the register plane kernels");
                CHK(ensure_S(c));
                const size_t slot = (size_t)4 * c->B * c->Np;
                const cplx<R>* Fj = Fml;
                if (blocked) {
                    CHK(ensure_far(c, pb));
                    if (far_pass) {
                        Trace tf(c, ETAIM_K_RING_FAR, std::min(ng, r0) * slot_b + ng * green_b + pb * slot_b);
                        // one thread per 16-byte vector of one column's points
                        const size_t pts = (size_t)4 * c->Np * sizeof(cplx<R>) / 16;
                        const dim3 gf((unsigned)((pts + 255) / 256));
                        cplx<R>* F = (cplx<R>*)c->far;
                        const cplx<R>* rg = (const cplx<R>*)ring(c);
                        if (ng <= 16)
                            hipLaunchKernelGGL((k_ring_far3<R, 16>), gf, dim3(256), 0, c->stream, rg, ghat(c), F, g, ng,
                                               r0, pb, conj);
                        else if (ng <= 24)
                            hipLaunchKernelGGL((k_ring_far3<R, 24>), gf, dim3(256), 0, c->stream, rg, ghat(c), F, g, ng,
                                               r0, pb, conj);
                        else
                            hipLaunchKernelGGL((k_ring_far3<R, 32>), gf, dim3(256), 0, c->stream, rg, ghat(c), F, g, ng,
                                               r0, pb, conj);
                        HIPCHK(hipGetLastError());
                        c->far_r0 = r0;
                    }
                    Fj = (const cplx<R>*)c->far + (size_t)(cur - r0) * slot;
                }
                Trace t(c, ETAIM_K_YZ_DELAYED, bytes);
                const size_t vecs = (size_t)4 * c->B * c->Np * sizeof(cplx<R>) / 16;
                hipLaunchKernelGGL(k_delay_sum<R>, dim3((unsigned)((vecs + 255) / 256)), dim3(256), 0, c->stream,
                                   (const cplx<R>*)ring(c), ghat(c), S(c), g, ng, cur, nmx, conj, Fj);
                HIPCHK(hipGetLastError());
                CHK(zlines_inv(c));
                CHK(ylines_inv(c, nullptr));
            } else if (c->yz_engine >= 1) {
                const size_t slot = (size_t)4 * c->B * c->Np;
                const cplx<R>* Fj = Fml;
                if (blocked) {
                    if (!graph) CHK(ensure_far(c, pb));
                    if (far_pass) {
                        Trace tf(c, ETAIM_K_RING_FAR, std::min(ng, r0) * slot_b + ng * green_b + pb * slot_b, true);
                        // one thread per 16-byte vector of points of one component and kx
                        const size_t pts = (size_t)4 * g.L[0] * 4 * (size_t)g.N[1] * g.N[2] * sizeof(cplx<R>) / 16;
                        const dim3 gf((unsigned)((pts + 255) / 256));
                        cplx<R>* F = (cplx<R>*)c->far;
                        const cplx<R>* rg = (const cplx<R>*)ring(c);
#define ETAIM_FAR(NN, NG) launch_timed(tf, k_ring_far<R, NN, NG>, gf, dim3(256), 0, c->stream, rg, ghat(c), F, g, ng, r0, pb, conj, sr)
#define ETAIM_FAR_NG(NN) \
    if (ng <= 16) ETAIM_FAR(NN, 16); else if (ng <= 24) ETAIM_FAR(NN, 24); else ETAIM_FAR(NN, 32);
                        switch (quad_n(c)) {
                            case 16: ETAIM_FAR_NG(16) break;
                            case 24: ETAIM_FAR_NG(24) break;
                            case 48: ETAIM_FAR_NG(48) break;
                            default: return fail(ETAIM_EUNSUPPORTED, "register plane kernels need N_y = N_z in {16, 24, 48}");
                        }
#undef ETAIM_FAR_NG
#undef ETAIM_FAR
                        HIPCHK(hipGetLastError());
                        if (!graph) c->far_r0 = r0;
                    }
                    // replayed: the kernel takes the block sums' base and the step's slot
                    Fj = (const cplx<R>*)c->far + (graph ? 0 : (size_t)(cur - r0) * slot);
                }
                Trace t(c, ETAIM_K_YZ_DELAYED, bytes, true);
                // plane pairs (bc, bc + 4) sharing the Green loads where the batch is even and two
                // planes' tiles fit the LDS; one plane per block otherwise
                const bool pair = c->B % 2 == 0 && 2 * quad_lds(c) <= (size_t)160 * 1024;
                const dim3 grid(pair ? 2 * c->B : 4 * c->B, g.L[0]);
                const dim3 blk(pair ? kDelayThreads : kDelay1Threads);
                const size_t lds = (pair ? 2 : 1) * quad_lds(c);
                const cplx<R>* rg = (const cplx<R>*)ring(c);
#define ETAIM_DELAYED(NN)                                                                                     \
    if (pair)                                                                                                  \
        launch_timed(t, k_yzq_delayed<R, NN>, grid, blk, lds, c->stream, rg, ghat(c), A(c), tw(c, 1), tw(c, 2), \
                     g, ng, cur, nmx, conj, Fj, sr);                                                           \
    else                                                                                                       \
        launch_timed(t, k_yzq_delayed1<R, NN>, grid, blk, lds, c->stream, rg, ghat(c), A(c), tw(c, 1),         \
                     tw(c, 2), g, ng, cur, nmx, conj, Fj, sr);
                switch (quad_n(c)) {
                    case 16: ETAIM_DELAYED(16) break;
                    case 24: ETAIM_DELAYED(24) break;
                    case 48: ETAIM_DELAYED(48) break;
                    default: return fail(ETAIM_EUNSUPPORTED, "register plane kernels need N_y = N_z in {16, 24, 48}");
                }
#undef ETAIM_DELAYED
            } else {
                if (graph) return fail(ETAIM_EUNSUPPORTED, "whole-step graph: needs the register plane kernels");
                Trace t(c, ETAIM_K_YZ_DELAYED, bytes, true);
                launch_timed(t, k_yz_delayed<R>, dim3(g.L[0], 4 * c->B), dim3(kPlaneThreads), plane_lds(c), c->stream,
                             (const cplx<R>*)ring(c), ghat(c), A(c), tw(c, 1), tw(c, 2), c->ry, c->rz, g, c->st.ng,
                             cur, ml ? nmx : nm, conj, Fml);
            }
        }
        HIPCHK(hipGetLastError());
        CHK(inverse_x(c, sr.live));
        const int nmh = std::min(c->st.mn, cur);
        return interp_near(c, mode, nullptr, nullptr, 0, cur, nmh, V, rhs, conj, 0, sr.live, sr);
    }
    // push the converged I_cur into the spectrum ring and the current ring
    static int commit(etaim_ctx* c, int cur, const zd* x, StepRef sr = {}) {
        const size_t slot_sz = (size_t)4 * c->B * c->Np;
        if (sr.sd) {
            // replayed: the commit kernel and the history store take the step from its descriptor
            CHK(commit_slot(c, ring(c), x, sr));
            if (c->st.mn >= 1) {
                const size_t n = (size_t)c->B * c->ns;
                hipLaunchKernelGGL(k_store_hist<R>, dim3(blocks_for(n)), dim3(256), 0, c->stream, x, (cplx<R>*)c->hist,
                                   c->ns, c->B, c->st.mn, sr);
                HIPCHK(hipGetLastError());
            }
            return ETAIM_OK;
        }
        CHK(commit_slot(c, ring(c) + (size_t)(cur % c->st.ng) * slot_sz, x));
        if (c->st.mn >= 1) {
            const size_t n = (size_t)c->B * c->ns;
            // current history slot in the working precision, columns of a basis contiguous
            hipLaunchKernelGGL(k_prescale<R>, dim3(blocks_for(n)), dim3(256), 0, c->stream, x, nullptr,
                               (cplx<R>*)c->hist + (size_t)(cur % c->st.mn) * n, c->ns, c->B, 0, nullptr);
            HIPCHK(hipGetLastError());
        }
        return ETAIM_OK;
    }
    // anterpolate + forward FFT of the B columns of x into the spectrum slot
    // `slot` (replayed: the ring's base, the kernel picks the step's slot)
    static int commit_slot(etaim_ctx* c, cplx<R>* slot, const zd* x, StepRef sr = {}) {
        CHK(forward_x(c, x, nullptr, 0, sr.live));
        if (sr.sd && c->yz_engine != 2)
            return fail(ETAIM_EUNSUPPORTED, "whole-step graph: needs the z-lines-first plane kernels");
        const GridDims& g = c->gd;
        if (c->yz_engine == 3) {
            CHK(ensure_S(c));
            const double s = sizeof(cplx<R>);
            Trace t(c, ETAIM_K_YZ_COMMIT, 4.0 * c->B * g.L[0] * g.N[2] * g.N[1] * s + 4.0 * c->B * c->Np * s);
            CHK(ylines_fwd(c, nullptr));
            return zlines_fwd(c, slot);
        }
        {
            const double s = sizeof(cplx<R>);
            Trace t(c, ETAIM_K_YZ_COMMIT, 4.0 * c->B * g.L[0] * g.N[2] * g.N[1] * s + 4.0 * c->B * c->Np * s, true);
            if (c->yz_engine == 2) {
                const dim3 grid(4 * c->B, g.L[0]);
                const size_t lds = zline_lds(c);
                const cplx<R>* a = (const cplx<R>*)A(c);
                switch (quad_n(c)) {
                    case 16: launch_timed(t, k_yzc_commit<R, 16>, grid, dim3(4 * 16), lds, c->stream, a, slot, tw(c, 1), tw(c, 2), g, sr, c->st.ng); break;
                    case 24: launch_timed(t, k_yzc_commit<R, 24>, grid, dim3(4 * 24), lds, c->stream, a, slot, tw(c, 1), tw(c, 2), g, sr, c->st.ng); break;
                    case 48: launch_timed(t, k_yzc_commit<R, 48>, grid, dim3(4 * 48), lds, c->stream, a, slot, tw(c, 1), tw(c, 2), g, sr, c->st.ng); break;
                    default: return fail(ETAIM_EUNSUPPORTED, "register plane kernels need N_y = N_z in {16, 24, 48}");
                }
            } else if (c->yz_engine == 1) {
                const dim3 grid(4 * c->B, g.L[0]);
                const size_t lds = quad_lds(c);
                const cplx<R>* a = (const cplx<R>*)A(c);
                switch (quad_n(c)) {
                    case 16: launch_timed(t, k_yzq_commit<R, 16>, grid, dim3(kQuadThreads), lds, c->stream, a, slot, tw(c, 1), tw(c, 2), g); break;
                    case 24: launch_timed(t, k_yzq_commit<R, 24>, grid, dim3(kQuadThreads), lds, c->stream, a, slot, tw(c, 1), tw(c, 2), g); break;
                    case 48: launch_timed(t, k_yzq_commit<R, 48>, grid, dim3(kQuadThreads), lds, c->stream, a, slot, tw(c, 1), tw(c, 2), g); break;
                    default: return fail(ETAIM_EUNSUPPORTED, "register plane kernels need N_y = N_z in {16, 24, 48}");
                }
            } else
            launch_timed(t, k_yz_commit<R>, dim3(g.L[0], 4 * c->B), dim3(kPlaneThreads), plane_lds(c), c->stream,
                         (const cplx<R>*)A(c), slot, tw(c, 1), tw(c, 2), c->ry, c->rz, g);
        }
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    // allow the plane kernels and the gather their dynamic LDS
    static int set_lds(etaim_ctx* c) {
        // (a plane larger than the LDS runs on the line-pass engine instead)
        const int bytes = (int)std::min(plane_lds(c), (size_t)160 * 1024);
        for (const void* f : {(const void*)k_yz_green<R>, (const void*)k_yz_commit<R>, (const void*)k_yz_delayed<R>})
            HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
        for (const void* f : {(const void*)k_yzq_green<R, 16>, (const void*)k_yzq_green<R, 24>,
                              (const void*)k_yzq_green<R, 48>, (const void*)k_yzq_commit<R, 16>,
                              (const void*)k_yzq_commit<R, 24>, (const void*)k_yzq_commit<R, 48>,
                              (const void*)k_yzq_delayed<R, 16>, (const void*)k_yzq_delayed<R, 24>,
                              (const void*)k_yzq_delayed<R, 48>, (const void*)k_yzq_delayed1<R, 16>,
                              (const void*)k_yzq_delayed1<R, 24>, (const void*)k_yzq_delayed1<R, 48>,
                              (const void*)k_yzc_green<R, 16>, (const void*)k_yzc_green<R, 24>,
                              (const void*)k_yzc_green<R, 48>, (const void*)k_yzc_commit<R, 16>,
                              (const void*)k_yzc_commit<R, 24>, (const void*)k_yzc_commit<R, 48>})
            HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        HIPCHK(hipFuncSetAttribute((const void*)k_zlines_green<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
        for (const void* f : {(const void*)k_interp_tile<R, 1>, (const void*)k_interp_tile<R, 2>,
                              (const void*)k_interp_tile<R, 4>})
            HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        // the gather's LDS grows with its tuned row count
        HIPCHK(hipFuncSetAttribute((const void*)k_fwdx_gather<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
        return ETAIM_OK;
    }
};

// ---------------------------------------------------------------------------
// Outcome of one time step's solve.
struct StepResult {
    int iters = 0, cols_iters = 0;
    bool noconv = false, nonfinite = false;
    double resid = 0;
};

// One Arnoldi step j for every active column: matvec, two classical
// Gram-Schmidt passes, norm, scale, Givens update (flag[0] = columns still
// active afterwards).  With a gate every kernel first checks the step's
// live flag (k_gate), so steps can be enqueued ahead of the host's
// convergence check or replayed from a captured graph.
// blocks per dot product or norm: one per 16 K entries, at most 64
inline int red_chunks(int ns) { return std::max(1, std::min(kRedMaxChunks, ns / 16384)); }

template <typename R>
int arnoldi_step(etaim_ctx* c, int j, int conj, const int* gate, const int* step_live = nullptr) {
    const int B = c->B, ns = c->ns, rs = c->prm.restart;
    const size_t nB = (size_t)B * ns;
    const zd* dinv = conj ? c->dinv_c : c->dinv;
    zd* vj = c->Vk + (size_t)j * nB;
    zd* vn = c->Vk + (size_t)(j + 1) * nB;
    if (gate) hipLaunchKernelGGL(k_gate, dim3(1), dim3(64), 0, c->stream, c->flag, step_live);
    // few columns: lane groups per row (the column-lane kernels would leave
    // most lanes idle)
    const bool grp = B <= kSpmvGroupMaxB;
    const unsigned gblocks = (unsigned)((nB * kSpmvLanes + 255) / 256);
    if (c->precond == 1 && c->x_engine == 1) {
        // w = Z (M v_j), M the near-zone sparse approximate inverse (M^H for the
        // adjoint): v_j transposed to [ns][B], then M v_j straight into the
        // operator's scaled-column buffer
        {
            Trace tp(c, ETAIM_K_KRYLOV, (double)c->nnz * 20.0 + 2.0 * (double)nB * 16.0 + (double)nB * sizeof(cplx<R>));
            if (grp) {
                hipLaunchKernelGGL(k_spmv_grp<R>, dim3(gblocks), dim3(256), 0, c->stream, c->rowptr, c->col,
                                   conj ? c->saiT : c->sai, vj, 1LL, (long long)ns, (cplx<R>*)c->xs, (zd*)nullptr, ns,
                                   B, conj, 0, gate);
            } else {
                hipLaunchKernelGGL(k_prescale<double>, dim3(blocks_for(nB)), dim3(256), 0, c->stream, vj, nullptr,
                                   (cplx<double>*)c->zt, ns, B, 0, gate);
                hipLaunchKernelGGL(k_spmv_rows<R>, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->rowptr, c->col,
                                   conj ? c->saiT : c->sai, c->zt, (cplx<R>*)c->xs, ns, B, conj, gate);
            }
        }
        CHK(Ops<R>::apply(c, 0, nullptr, nullptr, c->w, conj, gate, true));
    } else if (c->precond == 1) {
        // w = Z (M v_j), M the near-zone sparse approximate inverse (M^H for the adjoint)
        {
            Trace tp(c, ETAIM_K_KRYLOV, (double)c->nnz * 20.0 + 2.0 * (double)nB * 16.0);
            if (grp)
                hipLaunchKernelGGL(k_spmv_grp<R>, dim3(gblocks), dim3(256), 0, c->stream, c->rowptr, c->col,
                                   conj ? c->saiT : c->sai, vj, 1LL, (long long)ns, (cplx<R>*)nullptr, c->zt, ns, B,
                                   conj, 0, gate);
            else
                hipLaunchKernelGGL(k_spmv_cols, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->rowptr, c->col,
                                   conj ? c->saiT : c->sai, vj, c->zt, ns, B, conj, 0, gate);
        }
        CHK(Ops<R>::apply(c, 0, c->zt, nullptr, c->w, conj, gate));
    } else {
        CHK(Ops<R>::apply(c, 0, vj, dinv, c->w, conj, gate));
    }
    dim3 gd(j + 1, B), go((ns + 255) / 256, B);
    Trace tk(c, ETAIM_K_KRYLOV, (4.0 * (j + 1) + 8.0) * (double)nB * 16.0);
    // long columns: each dot product and norm over several blocks, finished in order
    const int nch = red_chunks(ns);
    auto dots = [&](zd* h) {
        if (nch == 1) {
            hipLaunchKernelGGL(k_dots, gd, dim3(kRedThreads), 0, c->stream, c->Vk, c->w, h, ns, B, gate);
            return;
        }
        hipLaunchKernelGGL(k_dots_part, dim3(j + 1, B, nch), dim3(kRedThreads), 0, c->stream, c->Vk, c->w,
                           (zd*)c->redpart, ns, B, nch, gate);
        hipLaunchKernelGGL(k_dots_fin, dim3(((j + 1) * B + 63) / 64), dim3(64), 0, c->stream, (const zd*)c->redpart,
                           h, (j + 1) * B, nch, gate);
    };
    dots(c->h1);
    hipLaunchKernelGGL(k_orth, go, dim3(256), 0, c->stream, c->Vk, c->w, c->h1, j + 1, ns, B, gate);
    dots(c->h2);
    hipLaunchKernelGGL(k_orth, go, dim3(256), 0, c->stream, c->Vk, c->w, c->h2, j + 1, ns, B, gate);
    if (nch == 1) {
        hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, c->w, c->nrm, ns, gate);
    } else {
        hipLaunchKernelGGL(k_norm_part, dim3(B, nch), dim3(kRedThreads), 0, c->stream, c->w, (double*)c->redpart, ns,
                           nch, gate);
        hipLaunchKernelGGL(k_norm_fin, dim3((B + 63) / 64), dim3(64), 0, c->stream, (const double*)c->redpart, c->nrm,
                           B, nch, gate);
    }
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->w, c->nrm, vn, ns, B, gate);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flag, 1, 0, gate);
    hipLaunchKernelGGL(k_arnoldi_update, dim3(1), dim3(256), 0, c->stream, c->h1, c->h2, c->nrm, c->H, c->cs, c->sn,
                       c->g, c->active, c->jcnt, c->resid, c->bnorm, c->flag, j, B, rs, c->prm.tol, gate);
    HIPCHK(hipGetLastError());
    return ETAIM_OK;
}

// Arnoldi step j as a replayed HIP graph, captured on first use (per
// direction of the operator).  Capture runs on a private stream; replays
// go to the context's stream.
template <typename R>
int arnoldi_step_graph(etaim_ctx* c, int j, int conj) {
    auto& v = c->graphs[conj];
    if (v.size() < (size_t)c->prm.restart) v.resize(c->prm.restart, nullptr);
    if (!v[j]) {
        if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        c->capturing = true;
        const hipError_t e0 = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        const int rc = e0 == hipSuccess ? arnoldi_step<R>(c, j, conj, c->flag + 2) : (int)ETAIM_EHIP;
        hipGraph_t g = nullptr;
        const hipError_t e1 = e0 == hipSuccess ? hipStreamEndCapture(c->stream, &g) : e0;
        c->stream = user;
        c->capturing = false;
        if (rc != ETAIM_OK || e1 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return rc != ETAIM_OK ? rc : fail(ETAIM_EHIP, std::string("graph capture failed: ") +
                                                              hipGetErrorString(e1));
        }
        hipGraphExec_t x = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) return fail(ETAIM_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e2));
        v[j] = x;
    }
    HIPCHK(hipGraphLaunch(v[j], c->stream));
    return ETAIM_OK;
}

// GMRES for one time step: x (in: initial guess, out: solution).
// Every column b of the batch has its own Krylov space; columns leave the
// iteration as they converge (device-side masks).
template <typename R>
int gmres(etaim_ctx* c, const zd* rhs, zd* x, int conj, StepResult& res) {
    const int B = c->B, ns = c->ns, rs = c->prm.restart;
    const size_t nB = (size_t)B * ns;
    const double tol = c->prm.tol;
    const zd* dinv = conj ? c->dinv_c : c->dinv;
    // gated schedule: several steps per host check, or graph replays (direct
    // gated launches while profiling, so that every kernel is traced)
    const bool graph = c->use_graph && !c->prof;
    const bool gated = graph || c->sync_every > 1;
    const int chunk = gated ? std::max(c->sync_every, 1) : 1;
    hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, rhs, c->bnorm, ns, nullptr);
    int total = 0;
    double prev_worst = 0;
    for (int cycle = 0;; ++cycle) {
        // r = rhs - A x
        CHK(Ops<R>::apply(c, 0, x, nullptr, c->w, conj));
        hipLaunchKernelGGL(k_residual, dim3(blocks_for(nB)), dim3(256), 0, c->stream, rhs, c->w, nB);
        hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, c->w, c->beta, ns, nullptr);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flag, 4, 0, nullptr);
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flag + 4, 1,
                           std::max(c->prm.maxit - total, 0), nullptr);
        hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(256), 0, c->stream, c->beta, c->bnorm, c->active, c->jcnt,
                           c->g, c->resid, c->flag, B, c->ldg, tol);
        // the first cycle of a gated solve goes straight on to its Arnoldi steps:
        // the gate holds them back if no column is active, and the host reads the
        // cycle start's flags and residuals with the first chunk's
        const bool defer = gated && cycle == 0;
        if (defer) {
            HIPCHK(hipMemcpyAsync(c->res_h + B, c->resid, B * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        } else {
            // flags and the true residuals of the cycle start in one readback
            HIPCHK(hipMemcpyAsync(c->flag_h, c->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipMemcpyAsync(c->res_h, c->resid, B * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            if (c->flag_h[1]) {
                res.nonfinite = true;
                break;
            }
            if (c->flag_h[0] == 0) break;
            if (total >= c->prm.maxit) {
                res.noconv = true;
                break;
            }
            // stagnation: the true residual at a restart did not drop below half of
            // the previous restart's (e.g. a tolerance below the working precision)
            double worst = 0;
            for (int b = 0; b < B; ++b) worst = std::max(worst, c->res_h[b]);
            if (cycle > 0 && worst > 0.5 * prev_worst) {
                res.noconv = true;
                break;
            }
            prev_worst = worst;
        }
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->w, c->beta, c->Vk, ns, B,
                           nullptr);
        const int base = total;
        // first chunk of a solve: as many steps as the previous solve took (the
        // count is steady along a march), so that no step is enqueued past
        // convergence; sync_every steps per chunk after that
        int j1 = 0;
        for (int j0 = 0; j0 < rs; j0 = j1) {
            const int len = (cycle == 0 && j0 == 0 && gated && c->iter_hint > 0) ? c->iter_hint : chunk;
            j1 = std::min(j0 + len, rs);
            std::vector<size_t> mark(j1 - j0);
            for (int j = j0; j < j1; ++j) {
                mark[j - j0] = c->pending.size();
                if (graph)
                    CHK(arnoldi_step_graph<R>(c, j, conj));
                else
                    CHK(arnoldi_step<R>(c, j, conj, gated ? c->flag + 2 : nullptr));
            }
            HIPCHK(hipMemcpyAsync(c->flag_h, c->flag, 5 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipMemcpyAsync(c->res_h, c->resid, B * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            HIPCHK(hipGetLastError());
            if (defer && j0 == 0) {
                // the deferred cycle start: its residuals for the next restart's stagnation test
                prev_worst = 0;
                for (int b = 0; b < B; ++b) prev_worst = std::max(prev_worst, c->res_h[B + b]);
            }
            if (gated) {
                // steps enqueued past convergence did no work (the gate is
                // monotone, so they are the chunk's last): drop their traces
                const int live = base + c->flag_h[3] - total;
                if (live >= 0 && live < j1 - j0) c->pending.resize(mark[live]);
            }
            total = gated ? base + c->flag_h[3] : total + 1;
            res.iters = total;
            if (c->flag_h[1]) res.nonfinite = true;
            if (c->flag_h[0] == 0 || c->flag_h[1] || total >= c->prm.maxit) break;
        }
        hipLaunchKernelGGL(k_backsolve, dim3((B + 63) / 64), dim3(64), 0, c->stream, c->H, c->g, c->jcnt, c->yv, B,
                           rs);
        if (c->precond == 1) {
            // x += M (V y): the combination, transposed to [ns][B] (in w, free
            // until the next cycle start), then the rows of M on the lanes' columns
            hipLaunchKernelGGL(k_krylov_combine, dim3((ns + 255) / 256, B), dim3(256), 0, c->stream, c->zt, c->Vk,
                               c->yv, c->jcnt, ns, B, rs);
            if (B <= kSpmvGroupMaxB) {
                hipLaunchKernelGGL(k_spmv_grp<double>, dim3((unsigned)((nB * kSpmvLanes + 255) / 256)), dim3(256), 0,
                                   c->stream, c->rowptr, c->col, conj ? c->saiT : c->sai, c->zt, 1LL, (long long)ns,
                                   (cplx<double>*)nullptr, x, ns, B, conj, 1, nullptr);
            } else {
                hipLaunchKernelGGL(k_prescale<double>, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->zt, nullptr,
                                   (cplx<double>*)c->w, ns, B, 0, nullptr);
                hipLaunchKernelGGL(k_spmv_rows_add, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->rowptr, c->col,
                                   conj ? c->saiT : c->sai, c->w, x, ns, B, conj);
            }
        } else {
            hipLaunchKernelGGL(k_update_x, dim3((ns + 255) / 256, B), dim3(256), 0, c->stream, x, c->Vk, c->yv,
                               c->jcnt, dinv, ns, B, rs);
        }
        HIPCHK(hipGetLastError());
        if (res.nonfinite) break;
        // every column converged by its Arnoldi residual estimate: done, unless
        // the true residual is to confirm it at a new cycle start
        if ((c->prm.flags & ETAIM_F_IMPLICIT_STOP) && c->flag_h[0] == 0) break;
    }
    // final residual (the last readback): the true residual of the last cycle
    // start, or the Arnoldi estimate of the last step under ETAIM_F_IMPLICIT_STOP
    res.resid = 0;
    for (int b = 0; b < B; ++b) res.resid = std::max(res.resid, c->res_h[b]);
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
// Whole-step graphs (ETAIM_F_STEP_GRAPH).  One forward time step as a captured
// graph: the delayed field (with or without the time-block pass: two
// variants), the extrapolated initial guess, one GMRES cycle of J
// device-gated Arnoldi steps ending on the residual estimate, the step
// check, the store of the solution, the commit, the growth-detector norms,
// the extrapolation-order selection (with or without: two variants) and the
// step end.  Every per-step value comes from the descriptor sdesc[ctl[0]];
// the step end advances ctl[0]; ctl[1] = 0 (set by the step check) makes
// every later node return.
constexpr int kStepChunk = 8;  // replayed steps enqueued per host check

int step_graph_setup(etaim_ctx* c) {
    if (c->sdesc) return ETAIM_OK;
    const size_t n = (size_t)std::max(c->prm.nt_steps, 1);
    CHK(c->alloc(c->sdesc, n));
    CHK(c->alloc(c->sctl, 2));
    CHK(c->alloc(c->siters, n));
    CHK(c->alloc(c->sres, n));
    HIPCHK(hipHostMalloc((void**)&c->sctl_h, 4 * sizeof(int), hipHostMallocDefault));
    return ETAIM_OK;
}

template <typename R>
int step_body(etaim_ctx* c, int J, int far, int pred) {
    const StepRef sr{c->sdesc, c->sctl, c->sctl + 1};
    const int* live = c->sctl + 1;
    const int B = c->B, ns = c->ns, rs = c->prm.restart;
    const size_t nB = (size_t)B * ns;
    // rhs = V_l - sum_{m>=1} Z_m I_{l-m} (cur = 1 only selects the blocked kernels)
    CHK(Ops<R>::delayed(c, 1, nullptr, c->rhs, 0, sr, far));
    hipLaunchKernelGGL(k_extrap, dim3(blocks_for(nB)), dim3(256), 0, c->stream, (const zd*)nullptr, c->xk, nB, 0LL, 1,
                       0, (const int*)c->pnext, sr);
    // GMRES, one cycle (the first cycle of the gated eager solve)
    hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, c->rhs, c->bnorm, ns, live, StepRef{});
    CHK(Ops<R>::apply(c, 0, c->xk, nullptr, c->w, 0, live));
    hipLaunchKernelGGL(k_residual, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->rhs, c->w, nB, live);
    hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, c->w, c->beta, ns, live, StepRef{});
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flag, 4, 0, live);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flag + 4, 1, c->prm.maxit, live);
    hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(256), 0, c->stream, c->beta, c->bnorm, c->active, c->jcnt, c->g,
                       c->resid, c->flag, B, c->ldg, c->prm.tol, live);
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->w, c->beta, c->Vk, ns, B, live);
    for (int j = 0; j < J; ++j) CHK(arnoldi_step<R>(c, j, 0, c->flag + 2, live));
    hipLaunchKernelGGL(k_backsolve, dim3((B + 63) / 64), dim3(64), 0, c->stream, c->H, c->g, c->jcnt, c->yv, B, rs,
                       live);
    if (c->precond == 1) {
        hipLaunchKernelGGL(k_krylov_combine, dim3((ns + 255) / 256, B), dim3(256), 0, c->stream, c->zt, c->Vk, c->yv,
                           c->jcnt, ns, B, rs, live);
        // the same product as the eager solve's end (bit-identical replays)
        if (B <= kSpmvGroupMaxB) {
            hipLaunchKernelGGL(k_spmv_grp<double>, dim3((unsigned)((nB * kSpmvLanes + 255) / 256)), dim3(256), 0,
                               c->stream, c->rowptr, c->col, c->sai, c->zt, 1LL, (long long)ns, (cplx<double>*)nullptr,
                               c->xk, ns, B, 0, 1, live);
        } else {
            hipLaunchKernelGGL(k_prescale<double>, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->zt, nullptr,
                               (cplx<double>*)c->w, ns, B, 0, live);
            hipLaunchKernelGGL(k_spmv_rows_add, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->rowptr, c->col,
                               c->sai, c->w, c->xk, ns, B, 0, live);
        }
    } else {
        hipLaunchKernelGGL(k_update_x, dim3((ns + 255) / 256, B), dim3(256), 0, c->stream, c->xk, c->Vk, c->yv,
                           c->jcnt, c->dinv, ns, B, rs, live);
    }
    hipLaunchKernelGGL(k_step_check, dim3(1), dim3(64), 0, c->stream, c->flag, c->sctl + 1);
    // the solution, the rings, the detector's norms, the next extrapolation order
    hipLaunchKernelGGL(k_store_step, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->xk, nB, sr);
    CHK(Ops<R>::commit(c, 0, c->xk, sr));
    hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, c->xk, nullptr, ns, live, sr);
    if (pred) {
        hipLaunchKernelGGL(k_pred_err, dim3(kPredBlocks), dim3(kRedThreads), 0, c->stream, (const zd*)nullptr, nB, 0LL,
                           1, 0, c->perr + kMaxGuess, sr);
        hipLaunchKernelGGL(k_pred_err_sum, dim3(1), dim3(256), 0, c->stream, (const double*)(c->perr + kMaxGuess),
                           kPredBlocks, c->perr, 0, c->pnext, sr);
    }
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, c->stream, c->flag, c->resid, B, c->siters, c->sres, c->sctl,
                       (const int*)(c->sctl + 1));
    HIPCHK(hipGetLastError());
    return ETAIM_OK;
}

// the executable graph of a step variant, captured on first use
template <typename R>
int step_graph_get(etaim_ctx* c, int J, int far, int pred, hipGraphExec_t& out) {
    const int key = (J * 2 + far) * 2 + pred;
    auto it = c->step_graphs.find(key);
    if (it != c->step_graphs.end()) {
        out = it->second;
        return ETAIM_OK;
    }
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    c->capturing = true;
    const hipError_t e0 = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    const int rc = e0 == hipSuccess ? step_body<R>(c, J, far, pred) : (int)ETAIM_EHIP;
    hipGraph_t g = nullptr;
    const hipError_t e1 = e0 == hipSuccess ? hipStreamEndCapture(c->stream, &g) : e0;
    c->stream = user;
    c->capturing = false;
    if (rc != ETAIM_OK || e1 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc != ETAIM_OK ? rc : fail(ETAIM_EHIP, std::string("step graph capture failed: ") + hipGetErrorString(e1));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(ETAIM_EHIP, std::string("step graph instantiation failed: ") + hipGetErrorString(e2));
    c->step_graphs[key] = x;
    out = x;
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
// FP64 residual check of eq. (5) (the late-time check of the precision form).
// Every kCheckEvery steps (step r with (r + 1) % kCheckEvery == 0) and at the
// last step of a call, the march forms in FP64
//   res_l = ||V_l - sum_{m=0}^{min(N_g, l)} Z_m I_{l-m}|| / ||V_l - sum_{m>=1} Z_m I_{l-m}||
// with the FP64 operators.  An FP64 march checks every column on the context
// itself (rhs of the step, one FP64 matvec); an FP32 march checks column 0
// on an FP64 companion context, which commits that column of every solution
// into its own FP64 history and forms the delayed field from it.
constexpr int kCheckEvery = 16;
constexpr int kCheckBatch = 16;  // history steps transformed together by the FP64 companion
constexpr double kCheckGridBytes = 8e9;

int device_setup(etaim_ctx* c);

// history steps the FP64 companion transforms together: kCheckBatch, fewer
// where the per-column FP64 grid buffers (work spectrum, planes, grids) of a
// large grid would pass kCheckGridBytes
int check_batch(const etaim_ctx* c) {
    const double per = 16.0 * (4.0 * (double)c->Np + 4.0 * c->gd.L[0] * (double)c->gd.N[1] * c->gd.N[2] +
                               8.0 * (double)c->N3);
    return (int)std::max(1.0, std::min((double)kCheckBatch, std::floor(kCheckGridBytes / per)));
}

int checker_create(etaim_ctx* c) {
    if (c->check) return ETAIM_OK;
    const int cb = check_batch(c);
    std::unique_ptr<etaim_ctx> k(new etaim_ctx());
    k->prm = c->prm;
    k->prm.precision = ETAIM_FP64;
    k->prm.batch = cb;
    k->prm.flags = 0;
    k->geo = c->geo;
    k->st = c->st;
    k->ns = c->ns;
    k->B = cb;  // grid buffers for the batched history transforms
    k->ring_cols = 1;    // the history of one column
    k->prec = ETAIM_FP64;
    k->mv = c->mv;
    k->nnz = c->nnz;
    k->gd = c->gd;
    k->gd.B = cb;
    k->rx = make_radix(k->gd.L[0]);
    k->ry = make_radix(k->gd.L[1]);
    k->rz = make_radix(k->gd.L[2]);
    k->N3 = c->N3;
    k->Np = c->Np;
    k->gfold = c->gfold;
    k->device = c->device;
    k->ncu = c->ncu;
    k->stream = c->stream;
    k->no_solver = true;
    k->yz_engine = quad_n(k.get()) ? 2 : 0;
    k->x_engine = xreg_ok(k.get()) ? 1 : 0;
    k->delay_block = 1;  // the delayed field is formed only at check steps: direct sum
    k->check_cols = cb;
    CHK(device_setup(k.get()));
    // the line-pass work spectrum sized for the widest batch of history transforms
    if (k->yz_engine == 3) CHK(Ops<double>::ensure_S(k.get()));
    k->B = 1;  // its operators act on the one monitored column
    k->gd.B = 1;
    c->check = k.release();
    return ETAIM_OK;
}

// an empty companion history that starts at step `from` (read from I_out later)
int checker_reset(etaim_ctx* c, int from) {
    etaim_ctx* k = c->check;
    HIPCHK(hipMemsetAsync(k->ring, 0, (size_t)k->st.ng * 4 * k->Np * sizeof(zd), k->stream));
    if (k->st.mn >= 1) HIPCHK(hipMemsetAsync(k->hist, 0, (size_t)k->st.mn * k->ns * sizeof(zd), k->stream));
    set_far_r0(k, -1);
    k->check_next = std::max(from, 0);
    return ETAIM_OK;
}

// the companion's history up to step hi - 1: column 0 of steps check_next..hi-1
// of I_out (only the last N_g of them matter), in runs of consecutive ring
// slots transformed together as the columns of one batch, and the last M_n
// of them into its current ring
int checker_fill(etaim_ctx* c, const zd* I, int hi) {
    etaim_ctx* k = c->check;
    const int ng = k->st.ng, mn = k->st.mn, ns = k->ns;
    const int lo = std::max(k->check_next, hi - ng);
    const size_t step = (size_t)c->B * ns;  // stride of I_out's steps
    for (int s = lo; s < hi;) {
        const int run = std::min({k->check_cols, hi - s, ng - s % ng});
        HIPCHK(hipMemcpy2DAsync(k->xk, (size_t)ns * sizeof(zd), I + (size_t)s * step, step * sizeof(zd),
                                (size_t)ns * sizeof(zd), run, hipMemcpyDeviceToDevice, k->stream));
        k->B = run;
        k->gd.B = run;
        const int rc = Ops<double>::commit_slot(k, (cplx<double>*)k->ring + (size_t)(s % ng) * 4 * k->Np, k->xk);
        k->B = 1;
        k->gd.B = 1;
        CHK(rc);
        s += run;
    }
    for (int s = std::max(lo, hi - mn); s < hi && mn >= 1; ++s)
        hipLaunchKernelGGL(k_prescale<double>, dim3(blocks_for((size_t)ns)), dim3(256), 0, k->stream,
                           I + (size_t)s * step, nullptr, (cplx<double>*)k->hist + (size_t)(s % mn) * ns, ns, 1, 0,
                           nullptr);
    HIPCHK(hipGetLastError());
    k->check_next = std::max(k->check_next, hi);
    return ETAIM_OK;
}

// residual and right-hand-side norms of step r into out[0..cols) and out[cols..2 cols)
template <typename R>
int check_step(etaim_ctx* c, int r, const zd* Vl, const zd* I, const zd* Il, double* out) {
    if (c->prec == ETAIM_FP64) {
        // the rhs of this step is still in c->rhs: r = rhs - Z0 I_l, all columns
        const size_t nB = (size_t)c->B * c->ns;
        CHK(Ops<double>::apply(c, 0, Il, nullptr, c->w, 0));
        hipLaunchKernelGGL(k_residual, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->rhs, c->w, nB);
        hipLaunchKernelGGL(k_norm, dim3(c->B), dim3(kRedThreads), 0, c->stream, c->w, out, c->ns, nullptr);
        hipLaunchKernelGGL(k_norm, dim3(c->B), dim3(kRedThreads), 0, c->stream, c->rhs, out + c->B, c->ns,
                           nullptr);
        HIPCHK(hipGetLastError());
        return ETAIM_OK;
    }
    etaim_ctx* k = c->check;
    const size_t n = (size_t)k->ns;
    CHK(checker_fill(c, I, r));
    if (r >= 1)
        CHK(Ops<double>::delayed(k, r, Vl, k->rhs, 0));
    else
        HIPCHK(hipMemcpyAsync(k->rhs, Vl, n * sizeof(zd), hipMemcpyDeviceToDevice, k->stream));
    CHK(Ops<double>::apply(k, 0, Il, nullptr, k->w, 0));
    hipLaunchKernelGGL(k_residual, dim3(blocks_for(n)), dim3(256), 0, k->stream, k->rhs, k->w, n);
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(kRedThreads), 0, k->stream, k->w, out, k->ns, nullptr);
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(kRedThreads), 0, k->stream, k->rhs, out + 1, k->ns, nullptr);
    HIPCHK(hipGetLastError());
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
// Steps first .. first + count - 1 of a march (the adjoint march: first = 0).
// With first > 0 the history rings continue from the last forward march on
// this context (or a loaded state) that ended at step first; otherwise they
// start empty.  Per-call arrays (norms, stats) are indexed by r - first.
template <typename R>
int march_impl(etaim_ctx* c, const zd* V, zd* I, etaim_stats* st, bool adjoint, int first, int count) {
    const int nt = count, B = c->B, ns = c->ns;
    const size_t nB = (size_t)B * ns;
    const int conj = adjoint ? 1 : 0;
    if (first == 0) {
        HIPCHK(hipMemsetAsync(c->ring, 0, (size_t)c->st.ng * 4 * B * c->Np * sizeof(cplx<R>), c->stream));
        set_far_r0(c, -1);  // the block sums belong to the previous history
        c->iter_hint = 0;
        if (c->st.mn >= 1) HIPCHK(hipMemsetAsync(c->hist, 0, (size_t)c->st.mn * nB * sizeof(zd), c->stream));
    }
    c->next_step = -1;  // valid again once this call completes its steps
    const int check_synced = c->check_synced;
    c->check_synced = -1;
    // excitation norms per step of this call (instability detector)
    std::vector<double> nV((size_t)nt * B), nI((size_t)nt, 0.0);
    {
        double* d = nullptr;
        CHK(c->alloc(d, (size_t)nt * B));
        hipLaunchKernelGGL(k_norm, dim3(nt * B), dim3(kRedThreads), 0, c->stream, V + (size_t)first * nB, d, ns, nullptr);
        HIPCHK(hipMemcpyAsync(nV.data(), d, nV.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        c->allocs.pop_back();
        c->dev_bytes -= (int64_t)((size_t)nt * B * sizeof(double));
        HIPCHK(hipFree(d));
    }
    // the excitation's largest norm and the step of the call (in marching
    // order) where it peaks: growth counts as late-time only after it
    double vmax = 0;
    int vpeak = 0;
    for (int q = 0; q < nt; ++q) {
        const int lq = adjoint ? nt - 1 - q : q;
        for (int b = 0; b < B; ++b)
            if (nV[(size_t)lq * B + b] > vmax) {
                vmax = nV[(size_t)lq * B + b];
                vpeak = q;
            }
    }
    int steps = 0, tot_iters = 0, max_iters = 0, first_noconv = -1, unstable = -1;
    double maxres = 0, ms_rhs = 0, ms_solve = 0, ms_commit = 0;
    bool nonfinite = false;
    // per-step current norms on the device [nt][B] (instability detector); with
    // ETAIM_F_FAIL_ON_UNSTABLE the host reads them every step, otherwise once
    // at the end, so that steps are enqueued without waiting for the last one
    const bool eager_detect = (c->prm.flags & ETAIM_F_FAIL_ON_UNSTABLE) != 0;
    double* nrm_all = nullptr;
    CHK(c->alloc(nrm_all, (size_t)nt * B));
    // FP64 residual check of eq. (5) (forward marches with ETAIM_F_RESIDUAL_CHECK)
    const bool checking = !adjoint && (c->prm.flags & ETAIM_F_RESIDUAL_CHECK) != 0;
    const int ccols = c->prec == ETAIM_FP64 ? B : 1;
    std::vector<int> chk_steps;
    double* chk = nullptr;
    if (checking) {
        for (int r = first; r < first + nt; ++r)
            if ((r + 1) % kCheckEvery == 0 || r == first + nt - 1) chk_steps.push_back(r);
        CHK(c->alloc(chk, 2 * (size_t)ccols * chk_steps.size()));
        if (c->prec != ETAIM_FP64) {
            CHK(checker_create(c));
            // the companion's history: kept when this call continues the march
            // it follows, else the monitored column of the steps before `first`,
            // read from I_out at the first check
            if (first == 0 || check_synced != first) CHK(checker_reset(c, first - c->st.ng));
        }
    }
    size_t nchk = 0;
    const int W = 32;
    auto detect = [&](int r) {
        // late-time growth: monotone growth by > 10x over W steps that begin
        // after the excitation's peak plus N_g steps (the pulse has crossed the
        // object, so the current of a stable march decays with the excitation;
        // a current that grows with a rising pulse is not flagged)
        if (unstable >= 0 || r < W || r - W + 1 <= vpeak + c->st.ng) return;
        bool mono = nI[r] > 10.0 * nI[r - W];
        for (int q = r - W + 1; q <= r && mono; ++q) mono = nI[q] > nI[q - 1];
        if (mono) unstable = r;
    };
    // phase times of a step, read once its events are complete
    auto phase_ms = [&](int r) -> int {
        hipEvent_t* ev = c->ev + 4 * (r & 1);
        float t01 = 0, t12 = 0, t23 = 0;
        HIPCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
        HIPCHK(hipEventElapsedTime(&t12, ev[1], ev[2]));
        HIPCHK(hipEventElapsedTime(&t23, ev[2], ev[3]));
        ms_rhs += t01;
        ms_solve += t12;
        ms_commit += t23;
        return ETAIM_OK;
    };
    // extrapolation order of the next initial guess: known on the host while
    // fewer than two orders can be compared, else chosen on the device
    int guess_p = c->guess_order == 0 ? 0 : 1;
    bool guess_dev = false;
    if (first > 0) {
        guess_p = c->guess_p_next;
        guess_dev = c->guess_dev_next;
    }
    // the eager step whose phase events have not been read yet (-1: none)
    int ev_step = -1;
    double ms_graph = 0;
    int graph_steps = 0, graph_halts = 0;
    // one step launched kernel by kernel; 1: the march stops after it
    auto eager_step = [&](int r) -> int {
        const int i = r - first;  // index within this call
        const int l = adjoint ? nt - 1 - r : r;
        const zd* Vl = V + (size_t)l * nB;
        zd* Il = I + (size_t)l * nB;
        hipEvent_t* ev = c->ev + 4 * (r & 1);
        HIPCHK(hipEventRecord(ev[0], c->stream));
        if (r >= 1) {
            CHK(Ops<R>::delayed(c, r, Vl, c->rhs, conj));
        } else {
            HIPCHK(hipMemcpyAsync(c->rhs, Vl, nB * sizeof(zd), hipMemcpyDeviceToDevice, c->stream));
        }
        HIPCHK(hipEventRecord(ev[1], c->stream));
        // initial guess: extrapolation of the last p solutions, p the order
        // that best predicted the previous step (at most guess_order)
        hipLaunchKernelGGL(k_extrap, dim3(blocks_for(nB)), dim3(256), 0, c->stream, (const zd*)I, c->xk, nB,
                           (long long)l, adjoint ? -1 : 1, guess_dev ? r : std::min(r, guess_p),
                           guess_dev ? (const int*)c->pnext : nullptr, StepRef{});
        HIPCHK(hipGetLastError());
        StepResult sr;
        CHK(gmres<R>(c, c->rhs, c->xk, conj, sr));
        c->iter_hint = std::min(sr.iters, c->prm.restart);
        // gmres has waited on the stream: the previous step's events are complete
        if (ev_step >= 0) {
            CHK(phase_ms(ev_step));
            ev_step = -1;
        }
        HIPCHK(hipEventRecord(ev[2], c->stream));
        HIPCHK(hipMemcpyAsync(Il, c->xk, nB * sizeof(zd), hipMemcpyDeviceToDevice, c->stream));
        if (checking && nchk < chk_steps.size() && chk_steps[nchk] == r) {
            CHK(check_step<R>(c, r, Vl, I, Il, chk + 2 * (size_t)ccols * nchk));
            ++nchk;
        }
        CHK(Ops<R>::commit(c, r, c->xk));
        hipLaunchKernelGGL(k_norm, dim3(B), dim3(kRedThreads), 0, c->stream, c->xk, nrm_all + (size_t)i * B, ns,
                           nullptr, StepRef{});
        const int pmax = std::min(r, c->guess_order);
        if (pmax >= 2) {
            hipLaunchKernelGGL(k_pred_err, dim3(kPredBlocks), dim3(kRedThreads), 0, c->stream, (const zd*)I, nB,
                               (long long)l, adjoint ? -1 : 1, pmax, c->perr + kMaxGuess, StepRef{});
            hipLaunchKernelGGL(k_pred_err_sum, dim3(1), dim3(256), 0, c->stream, (const double*)(c->perr + kMaxGuess),
                               kPredBlocks, c->perr, pmax, c->pnext, StepRef{});
            guess_dev = true;
        } else {
            guess_p = c->guess_order == 0 ? 0 : 1;
            guess_dev = false;
        }
        HIPCHK(hipEventRecord(ev[3], c->stream));
        ev_step = r;
        HIPCHK(hipGetLastError());
        // kernel traces are resolved in batches (each flush waits on the stream)
        if (c->pending.size() >= kTraceBatch) CHK(trace_flush(c));
        if (eager_detect) {
            HIPCHK(hipMemcpyAsync(c->res_h + B, nrm_all + (size_t)i * B, B * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            for (int b = 0; b < B; ++b) nI[i] = std::max(nI[i], c->res_h[B + b]);
        }
        steps = i + 1;
        tot_iters += sr.iters;
        max_iters = std::max(max_iters, sr.iters);
        maxres = std::max(maxres, sr.resid);
        if (st && st->iters_per_step) st->iters_per_step[i] = sr.iters;
        if (sr.nonfinite) {
            nonfinite = true;
            return 1;
        }
        if (sr.noconv && first_noconv < 0) {
            first_noconv = r;
            if (!(c->prm.flags & ETAIM_F_CONTINUE_ON_NOCONV)) return 1;
        }
        if (eager_detect) {
            detect(i);
            if (unstable >= 0) return 1;
        }
        return 0;
    };
    // whole-step graph replays: forward marches with the estimate stop, the
    // register engines, no tracing and no per-step growth check
    const bool graph_mode = !adjoint && c->step_graph && c->delay_mode == 0 && !c->prof && !eager_detect &&
                            (c->prm.flags & ETAIM_F_IMPLICIT_STOP) && c->yz_engine == 2 && c->x_engine == 1 &&
                            xline_n(c) > 0 && quad_n(c) > 0;
    const bool blocked = Ops<R>::blocks_on(c);
    const int pb = c->delay_block, ng = c->st.ng;
    auto block_start = [&](int r) { return r - (r - 1) % pb; };
    if (graph_mode) {
        CHK(step_graph_setup(c));
        std::vector<StepDesc> d((size_t)nt);
        for (int r = first; r < first + nt; ++r) {
            StepDesc& e = d[(size_t)(r - first)];
            e.cur = r;
            e.i = r - first;
            e.r0 = blocked ? block_start(r) : 0;
            e.nm = blocked ? std::min(r - e.r0, ng) : std::min(ng, r);
            e.fj = blocked ? r - e.r0 : -1;
            e.nmh = std::min(c->st.mn, r);
            // replayed steps follow a step that compared >= 2 orders when guess_order >= 2
            e.pdev = c->guess_order >= 2 ? 1 : 0;
            e.p = e.pdev ? r : std::min(r, c->guess_order == 0 ? 0 : 1);
            e.pmax = std::min(r, c->guess_order);
            e.pad = 0;
            e.V = V;
            e.I = I;
            e.nrm = nrm_all;
        }
        HIPCHK(hipMemcpy(c->sdesc, d.data(), d.size() * sizeof(StepDesc), hipMemcpyHostToDevice));
    }
    std::vector<int> it_h(kStepChunk);
    std::vector<double> res_hv(kStepChunk);
    for (int r = first; r < first + nt;) {
        if (!graph_mode || r < 3 || r == first) {
            const int rc = eager_step(r);
            if (rc < 0) return rc;
            if (rc == 1) break;
            ++r;
            continue;
        }
        // a run a..b of replayed steps, ending at the next residual check
        const int a = r;
        int b = std::min(first + nt - 1, a + kStepChunk - 1);
        int chk_at = -1;
        if (checking && nchk < chk_steps.size() && chk_steps[nchk] <= b) b = chk_at = chk_steps[nchk];
        const int J = std::max(2, std::min(c->iter_hint + 1, c->prm.restart));
        hipLaunchKernelGGL(k_step_ctl, dim3(1), dim3(64), 0, c->stream, c->sctl, a - first);
        HIPCHK(hipEventRecord(c->evg[0], c->stream));
        for (int q = a; q <= b; ++q) {
            const int far = blocked && c->far_r0 != block_start(q) ? 1 : 0;
            if (far) set_far_r0(c, block_start(q));
            const int pred = std::min(q, c->guess_order) >= 2 ? 1 : 0;
            hipGraphExec_t gx = nullptr;
            CHK(step_graph_get<R>(c, J, far, pred, gx));
            HIPCHK(hipGraphLaunch(gx, c->stream));
        }
        if (chk_at >= 0)
            CHK(check_step<R>(c, chk_at, V + (size_t)chk_at * nB, I, I + (size_t)chk_at * nB,
                              chk + 2 * (size_t)ccols * nchk));
        HIPCHK(hipEventRecord(c->evg[1], c->stream));
        HIPCHK(hipMemcpyAsync(c->sctl_h, c->sctl, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (ev_step >= 0) {
            CHK(phase_ms(ev_step));
            ev_step = -1;
        }
        {
            float t = 0;
            HIPCHK(hipEventElapsedTime(&t, c->evg[0], c->evg[1]));
            ms_graph += t;
        }
        const int done = c->sctl_h[0] - (a - first);
        if (done < 0 || done > b - a + 1) return fail(ETAIM_EHIP, "whole-step graph: inconsistent step counter");
        if (done > 0) {
            HIPCHK(hipMemcpy(it_h.data(), c->siters + (a - first), done * sizeof(int), hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(res_hv.data(), c->sres + (a - first), done * sizeof(double), hipMemcpyDeviceToHost));
        }
        int hint = 0;
        graph_steps += done;
        for (int q = 0; q < done; ++q) {
            const int i = a - first + q;
            steps = i + 1;
            tot_iters += it_h[q];
            max_iters = std::max(max_iters, it_h[q]);
            maxres = std::max(maxres, res_hv[q]);
            hint = std::max(hint, it_h[q]);
            if (st && st->iters_per_step) st->iters_per_step[i] = it_h[q];
        }
        if (done > 0) {
            c->iter_hint = std::min(hint, c->prm.restart);
            const int qlast = a + done - 1;
            guess_dev = std::min(qlast, c->guess_order) >= 2;
            if (!guess_dev) guess_p = c->guess_order == 0 ? 0 : 1;
        }
        if (c->sctl_h[1] != 0) {
            if (chk_at >= 0) ++nchk;
            r = b + 1;
            continue;
        }
        // step h did not converge within J Arnoldi steps (or went non-finite):
        // nothing after its GMRES ran, for it or the steps enqueued after it.
        // Its time block's sums are in place (their pass ran at or before h).
        const int h = a + done;
        ++graph_halts;
        if (blocked) set_far_r0(c, block_start(h));
        // a residual check enqueued after the halt read solutions that were not
        // computed: it is not counted, and the FP64 history refills from h on
        if (c->check) c->check->check_next = std::min(c->check->check_next, h);
        const int rc = eager_step(h);
        if (rc < 0) return rc;
        if (rc == 1) break;
        r = h + 1;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(trace_flush(c));
    if (ev_step >= 0) CHK(phase_ms(ev_step));
    if (!eager_detect && steps >= 1) {
        std::vector<double> na((size_t)steps * B);
        HIPCHK(hipMemcpy(na.data(), nrm_all, na.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int r = 0; r < steps; ++r) {
            for (int b = 0; b < B; ++b) nI[r] = std::max(nI[r], na[(size_t)r * B + b]);
            detect(r);
        }
    }
    // (the delayed field may have allocated after nrm_all: remove it by value)
    auto it = std::find(c->allocs.begin(), c->allocs.end(), (void*)nrm_all);
    if (it != c->allocs.end()) c->allocs.erase(it);
    c->dev_bytes -= (int64_t)((size_t)nt * B * sizeof(double));
    HIPCHK(hipFree(nrm_all));
    int n_checks = 0, worst_step = -1;
    double worst = 0;
    if (chk) {
        std::vector<double> cn(2 * (size_t)ccols * nchk);
        if (nchk > 0) HIPCHK(hipMemcpy(cn.data(), chk, cn.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t q = 0; q < nchk; ++q)
            for (int b = 0; b < ccols; ++b) {
                const double rn = cn[2 * ccols * q + b], bn = cn[2 * ccols * q + ccols + b];
                const double e = bn > 0 ? rn / bn : (rn > 0 ? INFINITY : 0.0);  // k_norm gives 2-norms
                if (worst_step < 0 || !(e <= worst)) {  // a NaN residual counts as the worst
                    worst = e;
                    worst_step = chk_steps[q];
                }
            }
        n_checks = (int)nchk;
        it = std::find(c->allocs.begin(), c->allocs.end(), (void*)chk);
        if (it != c->allocs.end()) c->allocs.erase(it);
        c->dev_bytes -= (int64_t)(2 * (size_t)ccols * chk_steps.size() * sizeof(double));
        HIPCHK(hipFree(chk));
    }
    if (st) {
        st->steps_done = steps;
        st->total_iters = tot_iters;
        st->max_iters = max_iters;
        st->first_noconv_step = first_noconv;
        st->unstable_step = unstable >= 0 ? first + unstable : -1;
        st->ms_rhs = ms_rhs;
        st->ms_solve = ms_solve;
        st->ms_commit = ms_commit;
        st->ms_total = ms_rhs + ms_solve + ms_commit + ms_graph;
        st->max_rel_residual = maxres;
        st->residual_checks = n_checks;
        st->residual_worst_step = worst_step;
        st->max_residual64 = worst;
        st->graph_steps = graph_steps;
        st->graph_halts = graph_halts;
    }
    if (!adjoint && steps == nt && !nonfinite) {
        if (checking && c->check) c->check_synced = first + steps;
        c->next_step = first + steps;
        c->guess_p_next = guess_p;
        c->guess_dev_next = guess_dev;
    }
    if (nonfinite) return fail(ETAIM_ENONFINITE, "non-finite GMRES residual at step " + std::to_string(first + steps - 1));
    if (first_noconv >= 0 && !(c->prm.flags & ETAIM_F_CONTINUE_ON_NOCONV))
        return fail(ETAIM_ENOCONV, "GMRES reached maxit at step " + std::to_string(first_noconv));
    if (unstable >= 0 && (c->prm.flags & ETAIM_F_FAIL_ON_UNSTABLE))
        return fail(ETAIM_EUNSTABLE, "late-time growth detected at step " + std::to_string(first + unstable));
    return ETAIM_OK;
}

// ---------------------------------------------------------------------------
// device set-up: Green tables and spectra, pre-correction, precision copies
template <typename R>
int make_working(etaim_ctx* c) {
    const size_t nB = (size_t)c->B;
    if (c->st.cfie) {
        // the MFIE pass's interpolation weights and Green spectra
        const size_t nl = (size_t)c->ns * 256, ngh = (size_t)(c->st.ng + 1) * 2 * c->gfold;
        if constexpr (sizeof(R) == sizeof(double)) {
            c->lamH_r = c->lamH64;
            c->ghatH_r = c->ghatH64;
        } else {
            float* lh = nullptr;
            zf* gh = nullptr;
            CHK(c->alloc(lh, nl));
            hipLaunchKernelGGL(k_real_to_r<float>, dim3(blocks_for(nl)), dim3(256), 0, c->stream, c->lamH64, lh, nl);
            CHK(c->alloc(gh, ngh));
            hipLaunchKernelGGL(k_to_r<float>, dim3(blocks_for(ngh)), dim3(256), 0, c->stream, c->ghatH64, gh, ngh);
            HIPCHK(hipGetLastError());
            c->lamH_r = lh;
            c->ghatH_r = gh;
        }
    }
    if constexpr (sizeof(R) == sizeof(double)) {
        c->lam_r = c->lam64;
        c->near_r = c->near64;
        c->nearT_r = c->nearT64;
        c->ghat_r = c->ghat64;
        double* nw = nullptr;
        CHK(c->upload(nw, c->st.nw));
        c->nw_r = nw;
    } else {
        float *lam = nullptr, *nw = nullptr;
        zf *nearv = nullptr, *gh = nullptr;
        CHK(c->alloc(lam, (size_t)c->ns * 256));
        hipLaunchKernelGGL(k_real_to_r<float>, dim3(blocks_for((size_t)c->ns * 256)), dim3(256), 0, c->stream,
                           c->lam64, lam, (size_t)c->ns * 256);
        double* nw64 = nullptr;
        CHK(c->upload(nw64, c->st.nw));
        CHK(c->alloc(nw, c->st.nw.size()));
        hipLaunchKernelGGL(k_real_to_r<float>, dim3(blocks_for(c->st.nw.size())), dim3(256), 0, c->stream, nw64, nw,
                           c->st.nw.size());
        CHK(c->alloc(nearv, (size_t)c->nnz * c->mv));
        hipLaunchKernelGGL(k_to_r<float>, dim3(blocks_for((size_t)c->nnz * c->mv)), dim3(256), 0, c->stream,
                           c->near64, nearv, (size_t)c->nnz * c->mv);
        zf* nearT = nullptr;
        CHK(c->alloc(nearT, (size_t)c->nnz * c->mv));
        hipLaunchKernelGGL(k_to_r<float>, dim3(blocks_for((size_t)c->nnz * c->mv)), dim3(256), 0, c->stream,
                           c->nearT64, nearT, (size_t)c->nnz * c->mv);
        c->nearT_r = nearT;
        const size_t ng = (size_t)(c->st.ng + 1) * 2 * c->gfold;
        CHK(c->alloc(gh, ng));
        hipLaunchKernelGGL(k_to_r<float>, dim3(blocks_for(ng)), dim3(256), 0, c->stream, c->ghat64, gh, ng);
        HIPCHK(hipGetLastError());
        c->lam_r = lam;
        c->nw_r = nw;
        c->near_r = nearv;
        c->ghat_r = gh;
    }
    if (const int qn = quad_n(c)) {
        const size_t planes = (size_t)(c->st.ng + 1) * 2 * (c->gd.N[0] + 1), n1 = (size_t)qn + 1;
        cplx<R>* gt = nullptr;
        CHK(c->alloc(gt, planes * n1 * n1));
        hipLaunchKernelGGL(k_green_transpose<R>, dim3(blocks_for(planes * n1 * n1)), dim3(256), 0, c->stream,
                           (const cplx<R>*)c->ghat_r, gt, planes, (int)n1);
        HIPCHK(hipGetLastError());
        c->ghatT_r = gt;
        if (c->st.cfie) {
            cplx<R>* gth = nullptr;
            CHK(c->alloc(gth, planes * n1 * n1));
            hipLaunchKernelGGL(k_green_transpose<R>, dim3(blocks_for(planes * n1 * n1)), dim3(256), 0, c->stream,
                               (const cplx<R>*)c->ghatH_r, gth, planes, (int)n1);
            HIPCHK(hipGetLastError());
            c->ghatHT_r = gth;
        }
    }
    for (int a = 0; a < 3; ++a) {
        const int L = c->gd.L[a];
        std::vector<cplx<R>> tw(L);
        for (int n = 0; n < L; ++n) {
            const double ang = 2.0 * kPi * (double)n / (double)L;
            tw[n] = cplx<R>{(R)std::cos(ang), (R)(-std::sin(ang))};
        }
        cplx<R>* d = nullptr;
        CHK(c->upload(d, tw));
        c->tw_r[a] = d;
    }
    CHK(c->allocv(c->A, 4 * nB * (size_t)c->gd.N[2] * c->gd.N[1] * c->gd.L[0] * sizeof(cplx<R>)));
    CHK(c->allocv(c->P, 4 * nB * c->N3 * sizeof(cplx<R>)));
    if (xreg_ok(c)) {
        CHK(c->allocv(c->Q, 4 * nB * c->N3 * sizeof(cplx<R>)));
        HIPCHK(hipMemsetAsync(c->Q, 0, 4 * nB * c->N3 * sizeof(cplx<R>), c->stream));
    }
    CHK(c->allocv(c->xs, nB * (size_t)c->ns * sizeof(cplx<R>)));
    const size_t ring_cols = c->ring_cols > 0 ? (size_t)c->ring_cols : nB;
    CHK(c->allocv(c->ring, (size_t)c->st.ng * 4 * ring_cols * c->Np * sizeof(cplx<R>)));
    // plane kernels: LDS and per-thread register staging limits; where the
    // padded (y, z) plane does not fit, the line-pass engine takes the y/z stage
    const bool plane_ok = Ops<R>::plane_lds(c) <= 160 * 1024 && plane_fits(c->gd.N[2], c->ry) &&
                          plane_fits(c->gd.L[1], c->rz);
    if (c->yz_engine == 0 && !plane_ok) c->yz_engine = 3;
    if (Ops<R>::gather_lds(c) > 160 * 1024 || !plane_fits(4, c->rx) ||
        (c->yz_engine == 3 && !(line_fits<R>(c->ry) && line_fits<R>(c->rz))))
        return fail(ETAIM_EUNSUPPORTED, "the padded grid's lines do not fit the LDS line kernels");
    // the line launches index (bc, kx) or (bc, z) planes by the grid's y dimension
    if ((c->yz_engine == 3 && 4 * nB * c->gd.L[0] > kMaxGridY) || ((c->x_engine == 0 || !xline_n(c)) && 4 * nB * c->gd.N[2] > kMaxGridY))
        return fail(ETAIM_EUNSUPPORTED, "batch too large for the line kernels at this grid (4 B L_x planes)");
    CHK(Ops<R>::set_lds(c));
    return ETAIM_OK;
}

int device_setup(etaim_ctx* c) {
    Setup& s = c->st;
    const int ns = c->ns;
    // FP64 arrays
    CHK(c->upload(c->lam64, s.lam));
    if (s.cfie) CHK(c->upload(c->lamH64, s.lamH));
    CHK(c->upload(c->i0, s.i0));
    CHK(c->upload(c->korder, s.order));
    CHK(c->upload(c->rowptr, s.rowptr));
    CHK(c->upload(c->col, s.col));
    std::vector<int> rowof(c->nnz);
    for (int k = 0; k < ns; ++k)
        for (int e = s.rowptr[k]; e < s.rowptr[k + 1]; ++e) rowof[e] = k;
    CHK(c->upload(c->rowof, rowof));
    CHK(c->upload(c->nptr, s.nptr));
    {
        // grid nodes that some basis reaches, as plane indices t = y + Ny (x + Nx z)
        const int Nx = s.N[0], Ny = s.N[1], Nz = s.N[2];
        std::vector<int> an;
        for (int z = 0; z < Nz; ++z)
            for (int x = 0; x < Nx; ++x)
                for (int y = 0; y < Ny; ++y) {
                    const size_t n = (size_t)x + (size_t)Nx * ((size_t)y + (size_t)Ny * z);
                    if (s.nptr[n + 1] > s.nptr[n]) an.push_back(y + Ny * (x + Nx * z));
                }
        c->n_anodes = (int)an.size();
        if (!an.empty()) CHK(c->upload(c->anodes, an));
        std::vector<unsigned long long> xm((size_t)Ny * Nz, 0ull);
        for (int t : an) {
            const int y = t % Ny, r = t / Ny, x = r % Nx, z = r / Nx;
            if (x < 64) xm[(size_t)z * Ny + y] |= 1ull << x;
        }
        CHK(c->upload(c->xmask, xm));
    }
    CHK(c->upload(c->nk, s.nk));
    {
        // interpolation tiles: the bases (in their Morton order) grouped by the
        // tile of their stencil corner, the tiles in the Morton order of their index
        std::map<long long, std::vector<int>> by_tile;
        auto spread = [](uint64_t v) {
            uint64_t r = 0;
            for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1u) << (3 * b);
            return r;
        };
        for (int q = 0; q < ns; ++q) {
            const int k = s.order[q];
            const uint64_t tx = (uint64_t)(s.i0[3 * k] / kTileX), ty = (uint64_t)(s.i0[3 * k + 1] / kTileY),
                           tz = (uint64_t)(s.i0[3 * k + 2] / kTileZ);
            by_tile[(long long)(spread(tx) | spread(ty) << 1 | spread(tz) << 2)].push_back(k);
        }
        std::vector<int> tptr(1, 0), tbase, torg;
        for (const auto& kv : by_tile) {
            const int k = kv.second.front();
            torg.push_back(s.i0[3 * k] / kTileX * kTileX);
            torg.push_back(s.i0[3 * k + 1] / kTileY * kTileY);
            torg.push_back(s.i0[3 * k + 2] / kTileZ * kTileZ);
            tbase.insert(tbase.end(), kv.second.begin(), kv.second.end());
            tptr.push_back((int)tbase.size());
        }
        c->ntiles = (int)by_tile.size();
        CHK(c->upload(c->tptr, tptr));
        CHK(c->upload(c->tbase, tbase));
        CHK(c->upload(c->torg, torg));
    }
    CHK(c->upload(c->near64, s.near_exact));
    // diagonal of Z0 = exact self entry (pre-correction restores it)
    std::vector<zd> diag(ns), dinv(ns), dinv_c(ns);
    for (int k = 0; k < ns; ++k) {
        zd d{0, 0};
        for (int e = s.rowptr[k]; e < s.rowptr[k + 1]; ++e)
            if (s.col[e] == k) d = s.near_exact[(size_t)e * c->mv];
        const double dd = d.x * d.x + d.y * d.y;
        if (!(dd > 0)) return fail(ETAIM_EINVAL, "zero diagonal entry of Z0 at basis " + std::to_string(k));
        diag[k] = d;
        dinv[k] = zd{d.x / dd, -d.y / dd};
        dinv_c[k] = zd{d.x / dd, d.y / dd};
    }
    CHK(c->upload(c->diag, diag));
    CHK(c->upload(c->dinv, dinv));
    CHK(c->upload(c->dinv_c, dinv_c));
    // Green tables (FP64) and pre-correction
    zd* gtab = nullptr;
    CHK(c->alloc(gtab, (size_t)(s.ng + 1) * 2 * c->N3));
    const double w = 2.0 * kPi * c->prm.fc;
    EnvKernel K{s.dt, w, w / kC0, kC0 * s.dt};
    K.tb = s.tb;
    // the BLIF's fold of its non-causal tables (none for the CPPIF)
    TFold fo{};
    if (s.mlo < 0) {
        fo.nk = -s.mlo;
        fo.np = s.nsamp;
        for (int kf = 0; kf < fo.nk; ++kf)
            for (int q = 0; q < fo.np; ++q) fo.a[kf][q] = s.fold_a[(size_t)kf * s.nsamp + q];
    }
    // the CFIE weighs the EFIE's tables by alpha and adds the MFIE's, -(1 - alpha) eta G^H
    const double sa = s.alpha * kMu0 / (4.0 * kPi), sp = s.alpha / (4.0 * kPi * eps0());
    hipLaunchKernelGGL(k_green_table, dim3(blocks_for((size_t)(s.ng + 1) * c->N3)), dim3(256), 0, c->stream, gtab,
                       c->gd, s.ng, s.h, K, sa, sp, fo);
    HIPCHK(hipGetLastError());
    zd* gtabH = nullptr;
    if (s.cfie) {
        CHK(c->alloc(gtabH, (size_t)(s.ng + 1) * 2 * c->N3));
        const double sh = -(1.0 - s.alpha) * std::sqrt(kMu0 / eps0());
        hipLaunchKernelGGL(k_green_table_h, dim3(blocks_for((size_t)(s.ng + 1) * c->N3)), dim3(256), 0, c->stream,
                           gtabH, c->gd, s.ng, s.h, K, sh, fo);
        HIPCHK(hipGetLastError());
    }
    if (c->nnz > 0)
        hipLaunchKernelGGL(k_precorrect, dim3(c->nnz), dim3(64), 0, c->stream, c->near64, c->lam64, c->i0, c->rowof,
                           c->col, gtab, c->gd, c->mv, c->nnz, (const double*)c->lamH64, (const zd*)gtabH);
    HIPCHK(hipGetLastError());
    // Green spectra: circulant embedding, full FP64 3-D FFT, fold, / Np
    CHK(c->alloc(c->ghat64, (size_t)(s.ng + 1) * 2 * c->gfold));
    zd* full = nullptr;
    CHK(c->alloc(full, c->Np));
    std::vector<zd> tw64[3];
    zd* twd[3];
    for (int a = 0; a < 3; ++a) {
        const int L = c->gd.L[a];
        tw64[a].resize(L);
        for (int n = 0; n < L; ++n) {
            const double ang = 2.0 * kPi * (double)n / (double)L;
            tw64[a][n] = zd{std::cos(ang), -std::sin(ang)};
        }
        CHK(c->upload(twd[a], tw64[a]));
    }
    const long long Lx = c->gd.L[0], Ly = c->gd.L[1], Lz = c->gd.L[2];
    if (s.cfie) {
        // the MFIE pass's spectra: G^H in slot 0, zero in slot 1 (its charge component)
        CHK(c->alloc(c->ghatH64, (size_t)(s.ng + 1) * 2 * c->gfold));
        HIPCHK(hipMemsetAsync(c->ghatH64, 0, (size_t)(s.ng + 1) * 2 * c->gfold * sizeof(zd), c->stream));
    }
    for (int m = 0; m <= s.ng; ++m)
        for (int t = 0; t < (s.cfie ? 3 : 2); ++t) {
            // t = 0, 1: the EFIE's A and phi tables; t = 2: the MFIE's G^H
            const zd* src = t < 2 ? gtab + ((size_t)m * 2 + t) * c->N3 : gtabH + (size_t)m * 2 * c->N3;
            zd* dst = t < 2 ? c->ghat64 + ((size_t)m * 2 + t) * c->gfold : c->ghatH64 + (size_t)m * 2 * c->gfold;
            hipLaunchKernelGGL(k_circulant, dim3(blocks_for(c->Np)), dim3(256), 0, c->stream, src, full, c->gd);
            CHK(launch_lines<double>(c, full, full, twd[0], c->rx, (int)Ly, (int)Lz, (int)Lx, (int)Lx, Lx, Ly * Lx, 1,
                                     Lx, Ly * Lx, 1, false));
            CHK(launch_lines<double>(c, full, full, twd[1], c->ry, (int)Lx, (int)Lz, (int)Ly, (int)Ly, 1, Ly * Lx, Lx,
                                     1, Ly * Lx, Lx, false));
            CHK(launch_lines<double>(c, full, full, twd[2], c->rz, (int)Lx, (int)Ly, (int)Lz, (int)Lz, 1, Lx,
                                     Ly * Lx, 1, Lx, Ly * Lx, false));
            hipLaunchKernelGGL(k_fold, dim3(blocks_for(c->gfold)), dim3(256), 0, c->stream, full, dst, c->gd,
                               1.0 / (double)c->Np);
            HIPCHK(hipGetLastError());
        }
    HIPCHK(hipStreamSynchronize(c->stream));
    // transposed near-zone values (the pattern is symmetric): nearT[e] = near[e'] with e' = (col[e], row[e])
    {
        std::vector<int> tperm(c->nnz);
        for (int k = 0; k < ns; ++k)
            for (int e = s.rowptr[k]; e < s.rowptr[k + 1]; ++e) {
                const int k2 = s.col[e];
                const int* base = s.col.data();
                const int* b = base + s.rowptr[k2];
                const int* end = base + s.rowptr[k2 + 1];
                const int* f = std::lower_bound(b, end, k);
                if (f == end || *f != k) return fail(ETAIM_EINVAL, "near-zone pattern is not symmetric");
                tperm[e] = (int)(f - base);
            }
        int* tp = nullptr;
        CHK(c->upload(tp, tperm));
        CHK(c->alloc(c->nearT64, (size_t)c->nnz * c->mv));
        hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for((size_t)c->nnz * c->mv)), dim3(256), 0, c->stream,
                           c->near64, c->nearT64, tp, c->nnz, c->mv);
        HIPCHK(hipGetLastError());
        // sparse approximate inverse of Z0 on the near pattern, and M^T's values for M^H
        if (!c->no_solver) {
            std::vector<zd> Mv;
            sparse_approximate_inverse(s, ns, Mv);
            CHK(c->upload(c->sai, Mv));
            CHK(c->alloc(c->saiT, (size_t)c->nnz));
            hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for((size_t)c->nnz)), dim3(256), 0, c->stream, c->sai,
                               c->saiT, tp, c->nnz, 1);
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(c->stream));
        auto it = std::find(c->allocs.begin(), c->allocs.end(), (void*)tp);
        c->allocs.erase(it);
        HIPCHK(hipFree(tp));
        c->dev_bytes -= (int64_t)(tperm.size() * sizeof(int));
    }
    // release set-up temporaries (gtab, gtabH, full, twd)
    for (void* p : {(void*)twd[2], (void*)twd[1], (void*)twd[0], (void*)full, (void*)gtab, (void*)gtabH}) {
        if (!p) continue;
        auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
        if (it != c->allocs.end()) c->allocs.erase(it);
        HIPCHK(hipFree(p));
    }
    c->dev_bytes -= (int64_t)(((size_t)(s.ng + 1) * 2 * c->N3 * (s.cfie ? 2 : 1) + c->Np) * sizeof(zd));
    // excitation / far-field quadrature data: 14 points per basis (7 per half)
    {
        const double s15 = std::sqrt(15.0);
        const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
        const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
        const double bq[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, 1 - 2 * a1}, {a1, 1 - 2 * a1, a1},
                                 {1 - 2 * a1, a1, a1},        {a2, a2, 1 - 2 * a2}, {a2, 1 - 2 * a2, a2},
                                 {1 - 2 * a2, a2, a2}};
        const double wq[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
        std::vector<double> Sq((size_t)ns * 14 * 3), rq((size_t)ns * 14 * 3), Snq(s.cfie ? (size_t)ns * 14 * 3 : 0);
        const Geometry& G = c->geo;
        for (int k = 0; k < ns; ++k)
            for (int h = 0; h < 2; ++h) {
                const int t = G.t[2 * k + h];
                const double sg = h == 0 ? 1.0 : -1.0;
                const double coef = sg * G.len[k] / (2.0 * G.area[t]);
                const int* tv = &G.tri[3 * (size_t)t];
                const int f = G.freev[2 * k + h];
                for (int q = 0; q < 7; ++q) {
                    const size_t o = ((size_t)k * 14 + h * 7 + q) * 3;
                    for (int x = 0; x < 3; ++x) {
                        const double r = bq[q][0] * G.xyz[3 * (size_t)tv[0] + x] + bq[q][1] * G.xyz[3 * (size_t)tv[1] + x] +
                                         bq[q][2] * G.xyz[3 * (size_t)tv[2] + x];
                        rq[o + x] = r;
                        Sq[o + x] = wq[q] * G.area[t] * coef * (r - G.xyz[3 * (size_t)f + x]);
                    }
                    if (s.cfie) {
                        // weighted S x n of this half's triangle
                        const double* nn = &G.nrm[3 * (size_t)t];
                        const double* S = &Sq[o];
                        Snq[o] = S[1] * nn[2] - S[2] * nn[1];
                        Snq[o + 1] = S[2] * nn[0] - S[0] * nn[2];
                        Snq[o + 2] = S[0] * nn[1] - S[1] * nn[0];
                    }
                }
            }
        CHK(c->upload(c->Sq, Sq));
        if (s.cfie) CHK(c->upload(c->Snq, Snq));
        CHK(c->upload(c->rq, rq));
    }
    CHK(c->prec == ETAIM_FP32 ? make_working<float>(c) : make_working<double>(c));
    // history of currents, Krylov space
    const size_t nB = (size_t)c->B * ns;
    const int rs = c->prm.restart;
    c->ldg = rs + 1;
    CHK(c->alloc(c->hist, (size_t)std::max(s.mn, 1) * nB));
    CHK(c->alloc(c->Vk, (size_t)(rs + 1) * nB));
    CHK(c->alloc(c->w, nB));
    CHK(c->alloc(c->xk, nB));
    CHK(c->alloc(c->zt, nB));
    CHK(c->alloc(c->rhs, nB));
    CHK(c->alloc(c->zero, nB));
    HIPCHK(hipMemsetAsync(c->zero, 0, nB * sizeof(zd), c->stream));
    CHK(c->allocv(c->redpart, (size_t)(rs + 1) * c->B * kRedMaxChunks * sizeof(zd)));
    CHK(c->alloc(c->h1, (size_t)(rs + 1) * c->B));
    CHK(c->alloc(c->h2, (size_t)(rs + 1) * c->B));
    CHK(c->alloc(c->H, (size_t)c->B * rs * (rs + 1)));
    CHK(c->alloc(c->sn, (size_t)c->B * rs));
    CHK(c->alloc(c->cs, (size_t)c->B * rs));
    CHK(c->alloc(c->g, (size_t)c->B * (rs + 1)));
    CHK(c->alloc(c->yv, (size_t)c->B * rs));
    CHK(c->alloc(c->nrm, c->B));
    CHK(c->alloc(c->beta, c->B));
    CHK(c->alloc(c->bnorm, c->B));
    CHK(c->alloc(c->resid, c->B));
    CHK(c->alloc(c->active, c->B));
    CHK(c->alloc(c->jcnt, c->B));
    CHK(c->alloc(c->flag, 8));
    CHK(c->alloc(c->perr, kMaxGuess + kMaxGuess * kPredBlocks));
    HIPCHK(hipHostMalloc((void**)&c->flag_h, 8 * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->res_h, 2 * (size_t)c->B * sizeof(double), hipHostMallocDefault));
    CHK(c->alloc(c->pnext, 1));
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
    for (auto& e : c->evg) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipStreamSynchronize(c->stream));
    return ETAIM_OK;
}

#include "tune.inc.hip"

int check_ctx(const etaim_ctx* c) {
    if (!c) return fail(ETAIM_EINVAL, "null context");
    return ETAIM_OK;
}

}  // namespace

// Staging of the no-allocation excitation entry point: the incidence
// directions and polarisations [2][nb][3] of one call.  Each device holds
// its own copy for the life of the process; every call on a device shares
// it.  Host code never uses the array's name as an address (on the host it
// is a stand-in symbol): the device address comes from hipGetSymbolAddress,
// once per device, at context creation.
constexpr int kNoallocMaxDirs = 4096;
static __device__ __align__(256) double scratch[6 * kNoallocMaxDirs];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device dev, which must be current
int scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(ETAIM_EUNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return ETAIM_OK;
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ETAIM_EHIP, "hipGetSymbolAddress returned no address for the staging array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
    return ETAIM_OK;
}

double* scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}
}  // namespace

// ===========================================================================
extern "C" {

const char* etaim_last_error(void) { return g_err.c_str(); }

int etaim_create(etaim_ctx** out, const etaim_mesh* mesh, const etaim_rwg* rwg, const etaim_params* params,
                 void* hip_stream) {
    g_err.clear();
    if (!out || !params) return fail(ETAIM_EINVAL, "null output or parameter pointer");
    *out = nullptr;
    std::unique_ptr<etaim_ctx> c(new etaim_ctx());
    c->prm = *params;
    std::string err;
    int rc = build_geometry(mesh, rwg, c->geo, err);
    if (rc) return fail(rc, err);
    rc = derive_parameters(c->geo, params, c->st, err);
    if (rc) return fail(rc, err);
    rc = build_projection(c->geo, c->st, err);
    if (rc) return fail(rc, err);
    rc = build_near_zone(c->geo, params, c->st, err);
    if (rc) return fail(rc, err);
    c->ns = c->geo.ns;
    c->B = params->batch;
    c->sync_every = std::max(params->sync_every, 1);
    c->use_graph = (params->flags & ETAIM_F_GRAPH) != 0;
    c->step_graph = (params->flags & ETAIM_F_STEP_GRAPH) != 0;
    c->prec = params->precision;
    c->mv = c->st.mn + 1;
    c->nnz = (int)c->st.col.size();
    for (int a = 0; a < 3; ++a) {
        c->gd.N[a] = c->st.N[a];
        c->gd.L[a] = c->st.L[a];
    }
    c->gd.B = c->B;
    c->rx = make_radix(c->gd.L[0]);
    c->ry = make_radix(c->gd.L[1]);
    c->rz = make_radix(c->gd.L[2]);
    c->yz_engine = quad_n(c.get()) ? 2 : 0;
    c->x_engine = xreg_ok(c.get()) ? 1 : 0;
    // histories longer than the one-level time blocks take, within the
    // levels' reach: multilevel time blocks
    c->delay_mode = (c->st.ng > kFarMaxNg && c->st.ng <= ml_max_ng()) ? 1 : 0;
    c->N3 = (size_t)c->gd.N[0] * c->gd.N[1] * c->gd.N[2];
    c->Np = (size_t)c->gd.L[0] * c->gd.L[1] * c->gd.L[2];
    c->gfold = (size_t)(c->gd.N[0] + 1) * (c->gd.N[1] + 1) * (c->gd.N[2] + 1);
    exact_near_entries(c->geo, params, c->st);
    if (hipGetDevice(&c->device) != hipSuccess) return fail(ETAIM_EHIP, "no HIP device");
    rc = scratch_init(c->device);
    if (rc) return rc;
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || c->ncu < 1)
        c->ncu = 256;
    c->stream = (hipStream_t)hip_stream;
    rc = device_setup(c.get());
    if (rc) return rc;
    if (c->delay_mode == 1) {
        // the multilevel buffers (accumulators of S_top slots and the level
        // tables, per far pass) must leave room for the march's others: else
        // the direct sum stays the default
        const int ng = c->st.ng, st = ml_s(kMlLevels - 1);
        int nlev = 0;
        while (nlev < kMlLevels && ml_s(nlev) <= ng) ++nlev;
        const int nextra = nlev == kMlLevels ? std::max(0, (ng + 1 + st - 1) / st - 2) : 0;
        const double cs = c->prm.precision == ETAIM_FP32 ? 8.0 : 16.0;
        const double need = (c->st.cfie ? 2.0 : 1.0) * cs *
                            ((double)ml_s(nlev - 1) * 4.0 * c->B * c->Np +
                             (double)(nextra ? ml_off_extra(nextra + 1) : ml_off(nlev)) * 2.0 * c->gfold);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess || need > 0.5 * (double)fr) c->delay_mode = 0;
    }
    *out = c.release();
    return ETAIM_OK;
}

int etaim_describe(const etaim_ctx* c, etaim_derived* o) {
    CHK(check_ctx(c));
    if (!o) return fail(ETAIM_EINVAL, "null output");
    o->dt = c->st.dt;
    o->h = c->st.h;
    for (int a = 0; a < 3; ++a) {
        o->origin[a] = c->st.x0[a];
        o->grid[a] = c->st.N[a];
        o->padded[a] = c->st.L[a];
    }
    o->rmax = c->st.rmax;
    o->stencil_radius = c->st.rst;
    o->ns = c->ns;
    o->ng = c->st.ng;
    o->mn = c->st.mn;
    o->nnz = c->nnz;
    o->batch = c->B;
    o->precision = c->prec;
    o->device_bytes = c->dev_bytes;
    return ETAIM_OK;
}

int etaim_excitation_planewave(etaim_ctx* c, int32_t nb, const double* khat, const double* phat, double sigma,
                               double td, void* V) {
    CHK(check_ctx(c));
    if (nb != c->B || !khat || !phat || !V || !(sigma > 0))
        return fail(ETAIM_EINVAL, "excitation needs nb == batch, khat, phat, V and sigma > 0");
    std::vector<double> kp(6 * (size_t)nb);
    std::memcpy(kp.data(), khat, 3 * nb * sizeof(double));
    std::memcpy(kp.data() + 3 * nb, phat, 3 * nb * sizeof(double));
    double* d = nullptr;
    CHK(c->upload(d, kp));
    const size_t tot = (size_t)c->prm.nt_steps * nb * c->ns;
    hipLaunchKernelGGL(k_excitation, dim3(blocks_for(tot)), dim3(256), 0, c->stream, (zd*)V, c->Sq, c->rq, d,
                       d + 3 * nb, c->prm.nt_steps, nb, c->ns, c->st.dt, sigma, td, 2.0 * kPi * c->prm.fc,
                       (const double*)c->Snq, c->st.alpha);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->allocs.pop_back();
    c->dev_bytes -= (int64_t)(kp.size() * sizeof(double));
    HIPCHK(hipFree(d));
    return ETAIM_OK;
}

int etaim_excitation_planewave_noalloc(etaim_ctx* c, int32_t nb, const double* khat, const double* phat,
                                       double sigma, double td, void* V) {
    CHK(check_ctx(c));
    if (nb > kNoallocMaxDirs)
        return fail(ETAIM_EINVAL, "no-allocation excitation: nb = " + std::to_string(nb) + " exceeds its limit of " +
                                      std::to_string(kNoallocMaxDirs) + " directions");
    if (nb != c->B || !khat || !phat || !V || !(sigma > 0))
        return fail(ETAIM_EINVAL, "excitation needs nb == batch, khat, phat, V and sigma > 0");
    double* d = scratch_of(c->device);
    if (!d) return fail(ETAIM_EHIP, "the staging array of this device has no address");
    HIPCHK(hipMemcpyAsync(d, khat, 3 * (size_t)nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(d + 3 * (size_t)nb, phat, 3 * (size_t)nb * sizeof(double), hipMemcpyHostToDevice,
                          c->stream));
    const size_t tot = (size_t)c->prm.nt_steps * nb * c->ns;
    hipLaunchKernelGGL(k_excitation, dim3(blocks_for(tot)), dim3(256), 0, c->stream, (zd*)V, c->Sq, c->rq, d,
                       d + 3 * (size_t)nb, c->prm.nt_steps, nb, c->ns, c->st.dt, sigma, td, 2.0 * kPi * c->prm.fc,
                       (const double*)c->Snq, c->st.alpha);
    HIPCHK(hipGetLastError());
    // the staging is free for the next call (and the caller's host arrays) once this returns
    HIPCHK(hipStreamSynchronize(c->stream));
    return ETAIM_OK;
}

int etaim_apply_z(etaim_ctx* c, int32_t m, const void* x, void* y) {
    CHK(check_ctx(c));
    if (m < 0 || m > c->st.ng || !x || !y) return fail(ETAIM_EINVAL, "apply_z needs 0 <= m <= ng and x, y");
    if (c->prec == ETAIM_FP32)
        CHK(Ops<float>::apply(c, m, (const zd*)x, nullptr, (zd*)y, 0));
    else
        CHK(Ops<double>::apply(c, m, (const zd*)x, nullptr, (zd*)y, 0));
    return trace_flush(c);
}

int etaim_delayed_field(etaim_ctx* c, const void* hist, void* b) {
    CHK(check_ctx(c));
    if (!hist || !b) return fail(ETAIM_EINVAL, "null pointer");
    const int ng = c->st.ng;
    const size_t nB = (size_t)c->B * c->ns;
    auto run = [&](auto tag) -> int {
        using R = decltype(tag);
        HIPCHK(hipMemsetAsync(c->ring, 0, (size_t)ng * 4 * c->B * c->Np * sizeof(cplx<R>), c->stream));
        set_far_r0(c, -1);
        c->next_step = -1;  // the rings now hold the injected history
        c->check_synced = -1;
        if (c->st.mn >= 1) HIPCHK(hipMemsetAsync(c->hist, 0, (size_t)c->st.mn * nB * sizeof(zd), c->stream));
        for (int m = ng; m >= 1; --m) CHK(Ops<R>::commit(c, ng - m, (const zd*)hist + (size_t)(m - 1) * nB));
        CHK(Ops<R>::delayed(c, ng, c->zero, (zd*)b, 0));
        hipLaunchKernelGGL(k_residual, dim3(blocks_for(nB)), dim3(256), 0, c->stream, c->zero, (zd*)b, nB);
        HIPCHK(hipGetLastError());
        return trace_flush(c);
    };
    return c->prec == ETAIM_FP32 ? run(float{}) : run(double{});
}

int etaim_march(etaim_ctx* c, const void* V, void* I_out, int32_t nsteps, etaim_stats* st) {
    CHK(check_ctx(c));
    if (!V || !I_out) return fail(ETAIM_EINVAL, "null V or I_out");
    if (nsteps < 0 || nsteps > c->prm.nt_steps) return fail(ETAIM_EINVAL, "nsteps out of range");
    const int n = nsteps > 0 ? nsteps : c->prm.nt_steps;
    return c->prec == ETAIM_FP32 ? march_impl<float>(c, (const zd*)V, (zd*)I_out, st, false, 0, n)
                                 : march_impl<double>(c, (const zd*)V, (zd*)I_out, st, false, 0, n);
}

int etaim_march_continue(etaim_ctx* c, const void* V, void* I_out, int32_t first, int32_t nsteps,
                         etaim_stats* st) {
    CHK(check_ctx(c));
    if (!V || !I_out) return fail(ETAIM_EINVAL, "null V or I_out");
    if (first < 1 || nsteps < 1 || first + nsteps > c->prm.nt_steps)
        return fail(ETAIM_EINVAL, "steps out of range: need 1 <= first, first + nsteps <= nt_steps");
    if (c->next_step != first)
        return fail(ETAIM_EINVAL, "the history is not at step " + std::to_string(first) + " (it is at " +
                                      std::to_string(c->next_step) + ")");
    return c->prec == ETAIM_FP32 ? march_impl<float>(c, (const zd*)V, (zd*)I_out, st, false, first, nsteps)
                                 : march_impl<double>(c, (const zd*)V, (zd*)I_out, st, false, first, nsteps);
}

// ---- march state (history rings and the carried initial-guess order)
namespace {
struct StateHeader {
    char magic[8];
    int32_t version, prec, B, ns, ng, mn, next_step, guess_p, guess_dev, pnext;
    int32_t quad, pad;  // ring slots by parity quadrants (register plane engines) or plain
    int64_t Np, ring_bytes, hist_bytes;
};
constexpr int32_t kStateVersion = 2;
constexpr char kStateMagic[8] = {'E', 'T', 'A', 'I', 'M', 'S', 'T', '1'};

size_t ring_bytes(const etaim_ctx* c) {
    return (size_t)c->st.ng * 4 * c->B * c->Np * (c->prec == ETAIM_FP32 ? sizeof(zf) : sizeof(zd));
}
size_t hist_bytes(const etaim_ctx* c) { return (size_t)std::max(c->st.mn, 1) * c->B * c->ns * sizeof(zd); }
}  // namespace

int etaim_state_size(const etaim_ctx* c, size_t* bytes) {
    CHK(check_ctx(c));
    if (!bytes) return fail(ETAIM_EINVAL, "null bytes");
    *bytes = sizeof(StateHeader) + ring_bytes(c) + hist_bytes(c);
    return ETAIM_OK;
}

int etaim_state_save(const etaim_ctx* c, void* host, size_t bytes) {
    CHK(check_ctx(c));
    if (!host) return fail(ETAIM_EINVAL, "null host pointer");
    const size_t rb = ring_bytes(c), hb = hist_bytes(c);
    if (bytes != sizeof(StateHeader) + rb + hb) return fail(ETAIM_EINVAL, "state size mismatch");
    if (c->next_step < 1) return fail(ETAIM_EINVAL, "no forward march state to save");
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    h.version = kStateVersion;
    h.quad = (c->yz_engine == 1 || c->yz_engine == 2) ? 1 : 0;
    h.prec = c->prec;
    h.B = c->B;
    h.ns = c->ns;
    h.ng = c->st.ng;
    h.mn = c->st.mn;
    h.next_step = c->next_step;
    h.guess_p = c->guess_p_next;
    h.guess_dev = c->guess_dev_next ? 1 : 0;
    h.Np = (int64_t)c->Np;
    h.ring_bytes = (int64_t)rb;
    h.hist_bytes = (int64_t)hb;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&h.pnext, c->pnext, sizeof(int), hipMemcpyDeviceToHost));
    unsigned char* p = (unsigned char*)host;
    std::memcpy(p, &h, sizeof h);
    HIPCHK(hipMemcpy(p + sizeof h, c->ring, rb, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(p + sizeof h + rb, c->hist, hb, hipMemcpyDeviceToHost));
    return ETAIM_OK;
}

int etaim_state_load(etaim_ctx* c, const void* host, size_t bytes) {
    CHK(check_ctx(c));
    if (!host) return fail(ETAIM_EINVAL, "null host pointer");
    const size_t rb = ring_bytes(c), hb = hist_bytes(c);
    if (bytes != sizeof(StateHeader) + rb + hb) return fail(ETAIM_EINVAL, "state size mismatch");
    StateHeader h;
    std::memcpy(&h, host, sizeof h);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != kStateVersion)
        return fail(ETAIM_EINVAL, "not a march state of this library");
    if (h.quad != ((c->yz_engine == 1 || c->yz_engine == 2) ? 1 : 0))
        return fail(ETAIM_EINVAL, "the state's spectrum ring is laid out for the other class of y/z engines "
                                  "(parity quadrants or plain): set the y/z engine it was saved with");
    if (h.prec != c->prec || h.B != c->B || h.ns != c->ns || h.ng != c->st.ng || h.mn != c->st.mn ||
        h.Np != (int64_t)c->Np || h.ring_bytes != (int64_t)rb || h.hist_bytes != (int64_t)hb)
        return fail(ETAIM_EINVAL, "the state belongs to a different problem (precision, batch, mesh or grid)");
    if (h.next_step < 1 || h.next_step > c->prm.nt_steps) return fail(ETAIM_EINVAL, "corrupt state: step");
    // extrapolation orders index the 6 x 6 coefficient table of the initial guess
    if (h.guess_p < 0 || h.guess_p > kMaxGuess || h.pnext < 1 || h.pnext > kMaxGuess || h.guess_dev < 0 ||
        h.guess_dev > 1)
        return fail(ETAIM_EINVAL, "corrupt state: initial-guess order");
    const unsigned char* p = (const unsigned char*)host;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->ring, p + sizeof h, rb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->hist, p + sizeof h + rb, hb, hipMemcpyHostToDevice));
    // the loading context's cap on the extrapolation order applies from the first step on
    const int pcap = std::max(c->guess_order, 1);
    const int pnext = std::min(h.pnext, pcap);
    HIPCHK(hipMemcpy(c->pnext, &pnext, sizeof(int), hipMemcpyHostToDevice));
    c->next_step = h.next_step;
    c->guess_p_next = std::min(h.guess_p, c->guess_order);
    c->guess_dev_next = h.guess_dev != 0 && c->guess_order >= 2;
    set_far_r0(c, -1);  // block sums are recomputed from the loaded ring
    c->iter_hint = 0;
    c->check_synced = -1;  // the residual check's FP64 history is rebuilt from I_out
    return ETAIM_OK;
}

int etaim_adjoint_march(etaim_ctx* c, const void* S, void* Lambda, etaim_stats* st) {
    CHK(check_ctx(c));
    if (!S || !Lambda) return fail(ETAIM_EINVAL, "null S or Lambda");
    if (c->st.cfie) return fail(ETAIM_EUNSUPPORTED, "the CFIE's adjoint march is not built");
    // Z^H = conj(Z): every operator is complex-symmetric, so the adjoint
    // march runs the same kernels with conjugated Green spectra, near-zone
    // values and preconditioner, backward in time
    return c->prec == ETAIM_FP32 ? march_impl<float>(c, (const zd*)S, (zd*)Lambda, st, true, 0, c->prm.nt_steps)
                                 : march_impl<double>(c, (const zd*)S, (zd*)Lambda, st, true, 0, c->prm.nt_steps);
}

int etaim_export(const etaim_ctx* c, int32_t what, void* host, size_t bytes) {
    CHK(check_ctx(c));
    if (!host) return fail(ETAIM_EINVAL, "null host pointer");
    const Setup& s = c->st;
    auto put = [&](const void* src, size_t n, bool device) -> int {
        if (n != bytes) return fail(ETAIM_EINVAL, "export size mismatch: expected " + std::to_string(n));
        if (device) {
            HIPCHK(hipStreamSynchronize(c->stream));
            HIPCHK(hipMemcpy(host, src, n, hipMemcpyDeviceToHost));
        } else {
            std::memcpy(host, src, n);
        }
        return ETAIM_OK;
    };
    switch (what) {
        case 0: return put(s.lam.data(), s.lam.size() * sizeof(double), false);
        case 1: return put(s.i0.data(), s.i0.size() * sizeof(int), false);
        case 2: return put(s.rowptr.data(), s.rowptr.size() * sizeof(int), false);
        case 3: return put(s.col.data(), s.col.size() * sizeof(int), false);
        case 4: {
            const size_t n = (size_t)c->nnz * c->mv;
            if (bytes != n * sizeof(zd)) return fail(ETAIM_EINVAL, "export size mismatch");
            std::vector<zd> v(n), o(n);
            HIPCHK(hipStreamSynchronize(c->stream));
            HIPCHK(hipMemcpy(v.data(), c->near64, n * sizeof(zd), hipMemcpyDeviceToHost));
            for (int e = 0; e < c->nnz; ++e)
                for (int m = 0; m < c->mv; ++m) o[(size_t)m * c->nnz + e] = v[(size_t)e * c->mv + m];
            std::memcpy(host, o.data(), bytes);
            return ETAIM_OK;
        }
        case 5: return put(c->diag, (size_t)c->ns * sizeof(zd), true);
        case 6: {
            // stored plane-major [m][t][kx][kz][ky]; exported as [m][t][kz][ky][kx]
            const size_t n = (size_t)(s.ng + 1) * 2 * c->gfold;
            if (bytes != n * sizeof(zd)) return fail(ETAIM_EINVAL, "export size mismatch");
            std::vector<zd> v(n);
            HIPCHK(hipStreamSynchronize(c->stream));
            HIPCHK(hipMemcpy(v.data(), c->ghat64, n * sizeof(zd), hipMemcpyDeviceToHost));
            const int gx = c->gd.N[0] + 1, gy = c->gd.N[1] + 1, gz = c->gd.N[2] + 1;
            zd* o = (zd*)host;
            for (size_t mt = 0; mt < (size_t)(s.ng + 1) * 2; ++mt)
                for (int x = 0; x < gx; ++x)
                    for (int z = 0; z < gz; ++z)
                        for (int y = 0; y < gy; ++y)
                            o[mt * c->gfold + ((size_t)z * gy + y) * gx + x] =
                                v[mt * c->gfold + ((size_t)x * gz + z) * gy + y];
            return ETAIM_OK;
        }
        case 7:
            if (!s.cfie) return fail(ETAIM_EINVAL, "export 7 (curl test projection) needs the CFIE");
            return put(s.lamH.data(), s.lamH.size() * sizeof(double), false);
        default: return fail(ETAIM_EINVAL, "unknown export id");
    }
}

int etaim_set_profiling_mask(etaim_ctx* c, uint32_t classes) {
    CHK(check_ctx(c));
    if (classes >> ETAIM_K_COUNT) return fail(ETAIM_EINVAL, "profiling mask names an unknown kernel class");
    CHK(trace_flush(c));
    c->prof_mask = classes;
    c->prof = classes != 0;
    if (c->prof)
        for (int i = 0; i < ETAIM_K_COUNT; ++i) c->k_ms[i] = c->k_bytes[i] = 0, c->k_n[i] = 0;
    return ETAIM_OK;
}

int etaim_set_delay_mode(etaim_ctx* c, int32_t mode) {
    CHK(check_ctx(c));
    if (mode != 0 && mode != 1) return fail(ETAIM_EINVAL, "delay mode must be 0 or 1");
    if (mode == 1 && c->st.ng > ml_max_ng())
        return fail(ETAIM_EUNSUPPORTED, "multilevel time blocks reach lags up to " +
                                            std::to_string(ml_max_ng()) + ", N_g is " +
                                            std::to_string(c->st.ng));
    if (c->delay_mode != mode) {
        c->delay_mode = mode;
        set_far_r0(c, -1);
    }
    return ETAIM_OK;
}

int etaim_get_delay_mode(const etaim_ctx* c, int32_t* mode) {
    CHK(check_ctx(c));
    if (!mode) return fail(ETAIM_EINVAL, "null pointer");
    *mode = c->delay_mode;
    return ETAIM_OK;
}

int etaim_set_profiling(etaim_ctx* c, int32_t on) {
    return etaim_set_profiling_mask(c, on ? (1u << ETAIM_K_COUNT) - 1u : 0u);
}

int etaim_kernel_stats(const etaim_ctx* c, int32_t cls, double* ms, double* bytes, int64_t* launches) {
    CHK(check_ctx(c));
    if (cls < 0 || cls >= ETAIM_K_COUNT || !ms || !bytes || !launches)
        return fail(ETAIM_EINVAL, "kernel_stats needs a valid class and outputs");
    *ms = c->k_ms[cls];
    *bytes = c->k_bytes[cls];
    *launches = c->k_n[cls];
    return ETAIM_OK;
}

int etaim_autotune(etaim_ctx* c, int32_t budget_ms, const char* cache_path, etaim_tuning* out) {
    g_err.clear();
    CHK(check_ctx(c));
    if (budget_ms < 1) return fail(ETAIM_EINVAL, "budget_ms must be >= 1");
    const std::string key = tune_key(c);
    etaim_tuning t{};
    if (cache_path && cache_lookup(cache_path, key, t)) {
        Shape s;
        CHK(shape_from_c(c, &t, s));
        const bool ok = c->prec == ETAIM_FP32 ? shape_fits<float>(c, s) : shape_fits<double>(c, s);
        if (ok) {
            put_shape(c, s);
            if (out) *out = t;
            return ETAIM_OK;
        }
        // a record that no longer fits the kernels: tune again
    }
    const Shape saved = get_shape(c);
    const bool prof = c->prof;
    const int rc = c->prec == ETAIM_FP32 ? autotune_impl<float>(c, budget_ms, &t)
                                         : autotune_impl<double>(c, budget_ms, &t);
    c->prof = prof;
    if (rc != ETAIM_OK) {
        put_shape(c, saved);
        return rc;
    }
    if (cache_path) CHK(cache_append(cache_path, key, t));
    if (out) *out = t;
    return ETAIM_OK;
}

int etaim_get_tuning(const etaim_ctx* c, etaim_tuning* out) {
    g_err.clear();
    CHK(check_ctx(c));
    if (!out) return fail(ETAIM_EINVAL, "null output");
    *out = etaim_tuning{};
    if (c->prec == ETAIM_FP32)
        shape_to_c<float>(c, get_shape(c), out);
    else
        shape_to_c<double>(c, get_shape(c), out);
    return ETAIM_OK;
}

int etaim_set_tuning(etaim_ctx* c, const etaim_tuning* t) {
    g_err.clear();
    CHK(check_ctx(c));
    if (!t) return fail(ETAIM_EINVAL, "null tuning");
    Shape s;
    CHK(shape_from_c(c, t, s));
    const bool ok = c->prec == ETAIM_FP32 ? shape_fits<float>(c, s) : shape_fits<double>(c, s);
    if (!ok) return fail(ETAIM_EUNSUPPORTED, "the setting does not fit the kernels' LDS or register staging");
    put_shape(c, s);
    return ETAIM_OK;
}

void etaim_destroy(etaim_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"

namespace {
int farfield_taps(etaim_ctx* c, int nd, const double* dirs, zd*& F, double*& dd, int& ntap, int& m_lo) {
    double rad = 0;
    for (double v : c->geo.xyz) rad = std::max(rad, std::fabs(v));
    const double smax = rad * std::sqrt(3.0) / (kC0 * c->st.dt);
    m_lo = (int)std::floor(c->st.tb.lo() - smax);
    const int m_hi = (int)std::ceil(c->st.tb.hi() + smax);
    ntap = m_hi - m_lo + 1;
    std::vector<double> dv(dirs, dirs + 3 * (size_t)nd);
    CHK(c->upload(dd, dv));
    CHK(c->alloc(F, (size_t)ntap * nd * 3 * c->ns));
    const size_t tot = (size_t)ntap * nd * c->ns;
    hipLaunchKernelGGL(k_farfield_taps, dim3(blocks_for(tot)), dim3(256), 0, c->stream, F, c->Sq, c->rq, dd, nd,
                       c->ns, ntap, m_lo, c->st.dt, 2.0 * kPi * c->prm.fc, kMu0 / (4.0 * kPi), c->st.tb);
    HIPCHK(hipGetLastError());
    return ETAIM_OK;
}
int release_last(etaim_ctx* c, int n) {
    for (int i = 0; i < n && !c->allocs.empty(); ++i) {
        HIPCHK(hipFree(c->allocs.back()));
        c->allocs.pop_back();
    }
    return ETAIM_OK;
}
}  // namespace

extern "C" {
int etaim_farfield(etaim_ctx* c, int32_t nd, const double* dirs, const void* I, void* U) {
    CHK(check_ctx(c));
    if (nd < 1 || !dirs || !I || !U) return fail(ETAIM_EINVAL, "farfield needs nd >= 1, dirs, I and U");
    zd* F = nullptr;
    double* dd = nullptr;
    int ntap = 0, m_lo = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t before = c->dev_bytes;
    CHK(farfield_taps(c, nd, dirs, F, dd, ntap, m_lo));
    const int nout = c->prm.nt_steps * c->B * nd * 3;
    hipLaunchKernelGGL(k_farfield_apply, dim3(nout), dim3(256), 0, c->stream, (zd*)U, F, (const zd*)I,
                       c->prm.nt_steps, c->B, nd, c->ns, ntap, m_lo);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(release_last(c, 2));
    c->dev_bytes = before;
    return ETAIM_OK;
}

int etaim_farfield_adjoint(etaim_ctx* c, int32_t nd, const double* dirs, const void* Ubar, void* S) {
    CHK(check_ctx(c));
    if (nd < 1 || !dirs || !Ubar || !S) return fail(ETAIM_EINVAL, "farfield_adjoint needs nd >= 1, dirs, Ubar, S");
    zd* F = nullptr;
    double* dd = nullptr;
    int ntap = 0, m_lo = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t before = c->dev_bytes;
    CHK(farfield_taps(c, nd, dirs, F, dd, ntap, m_lo));
    const size_t tot = (size_t)c->prm.nt_steps * c->B * c->ns;
    hipLaunchKernelGGL(k_farfield_adjoint, dim3(blocks_for(tot)), dim3(256), 0, c->stream, (zd*)S, F,
                       (const zd*)Ubar, c->prm.nt_steps, c->B, nd, c->ns, ntap, m_lo);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(release_last(c, 2));
    c->dev_bytes = before;
    return ETAIM_OK;
}

int etaim_rcs(etaim_ctx* c, int32_t nd, const double* pol, int32_t nf, const double* df, double pulse_sigma,
              const void* U, double* sigma_out) {
    CHK(check_ctx(c));
    if (nd < 1 || nf < 1 || !pol || !df || !U || !sigma_out || !(pulse_sigma > 0))
        return fail(ETAIM_EINVAL, "rcs needs nd >= 1, nf >= 1, pol, df, pulse_sigma > 0, U, sigma_out");
    // the incident envelope's transform: g = exp(-t^2 / 2 sigma^2) -> sigma sqrt(2 pi) exp(-2 pi^2 sigma^2 df^2)
    std::vector<double> host((size_t)3 * nd + 2 * (size_t)nf);
    std::memcpy(host.data(), pol, sizeof(double) * 3 * nd);
    for (int i = 0; i < nf; ++i) {
        host[3 * (size_t)nd + i] = df[i];
        host[3 * (size_t)nd + nf + i] =
            pulse_sigma * std::sqrt(2.0 * kPi) * std::exp(-2.0 * kPi * kPi * pulse_sigma * pulse_sigma * df[i] * df[i]);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t before = c->dev_bytes;
    double* d = nullptr;
    CHK(c->upload(d, host));
    const size_t tot = (size_t)nf * c->B * nd;
    hipLaunchKernelGGL(k_rcs, dim3(blocks_for(tot)), dim3(256), 0, c->stream, sigma_out, (const zd*)U, d,
                       d + 3 * (size_t)nd, d + 3 * (size_t)nd + nf, c->prm.nt_steps, c->B, nd, nf, c->st.dt);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(release_last(c, 1));
    c->dev_bytes = before;
    return ETAIM_OK;
}

int etaim_db_error(int32_t n, const double* sigma, const double* sigma_ref, const double* w, double floor_db,
                   double* err) {
    if (n < 1 || !sigma || !sigma_ref || !w || !err || !(floor_db > 0))
        return fail(ETAIM_EINVAL, "db_error needs n >= 1, sigma, sigma_ref, w, floor_db > 0, err");
    double peak = 0;
    for (int i = 0; i < n; ++i) peak = std::max(peak, sigma_ref[i]);
    if (!(peak > 0)) return fail(ETAIM_EINVAL, "the reference pattern has no positive value");
    const double th = 10.0 * std::log10(peak) - floor_db;
    auto thr = [&](double v) { return std::max(10.0 * std::log10(std::max(v, 1e-300)), th) - th; };
    double num = 0, den = 0;
    for (int i = 0; i < n; ++i) {
        const double a = thr(sigma[i]), b = thr(sigma_ref[i]);
        num += (a - b) * (a - b) * w[i];
        den += b * b * w[i];
    }
    *err = num / den;
    return ETAIM_OK;
}
}  // extern "C"
