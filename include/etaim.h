/*
 * etaim.h - C ABI of the MI355X envelope-tracking adaptive integral method
 * (ET-AIM) marching library (Kaur & Yilmaz, "Empirical Comparison of
 * Envelope-Tracking and Time-Domain Adaptive Integral Methods for Surface
 * Integral Equations", arXiv 1408.7060).
 *
 * The calls follow the paper's statement of the problem (Sec. 3, eq. (3)-(4)
 * and Sec. 4, eq. (5)): a PEC surface meshed with triangles and expanded in
 * RWG functions S_k, a causal piecewise-polynomial temporal basis T of order
 * Q = 3, a time step dt and the incident-envelope excitation V_l go in; the
 * current-envelope samples I_l, l = 1..N_t, and scattered far-field
 * envelopes come out.  The method's parameters (auxiliary grid size,
 * near-zone distance, solver tolerance) are those of Sec. 5.1.
 *
 * Conventions (every call):
 *  - Return value: ETAIM_OK (0) or a negative ETAIM_E* code; the message of
 *    the last failure on the calling thread is etaim_last_error().  No C++
 *    exception crosses this boundary.
 *  - Complex arrays are interleaved (re, im) float64 pairs ("complex128"),
 *    row-major, so they match the storage of torch.complex128 tensors.
 *  - Mesh, RWG and parameter structs are HOST pointers, read during the call
 *    only.  Excitation, current, history, field and output arrays are DEVICE
 *    pointers on the context's device; the caller owns them.
 *  - The context owns every internal device buffer (projection weights,
 *    Green spectra, near-zone matrices, history rings, Krylov space) and
 *    frees them in etaim_destroy.
 *  - A context is bound to the device current at etaim_create and to the
 *    HIP stream given there; calls are ordered on that stream.  Calls that
 *    return statistics synchronise the stream.  Contexts are not
 *    thread-safe: use one context per thread.
 *  - Input validation happens before any device work: an invalid argument
 *    returns ETAIM_EINVAL and leaves the context unchanged.
 */
#ifndef ETAIM_H
#define ETAIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ETAIM_OK 0
#define ETAIM_EINVAL (-1)      /* bad argument, mesh, RWG table or parameter */
#define ETAIM_ENOMEM (-2)      /* device or host allocation failed */
#define ETAIM_EHIP (-3)        /* HIP runtime error */
#define ETAIM_ENOCONV (-4)     /* GMRES reached maxit at some step */
#define ETAIM_ENONFINITE (-5)  /* NaN/Inf in a residual */
#define ETAIM_EUNSTABLE (-6)   /* late-time growth detector fired */
#define ETAIM_EUNSUPPORTED (-7)

/* working precision of the grid/FFT/near-zone arithmetic (Krylov is FP64) */
#define ETAIM_FP64 0
#define ETAIM_FP32 1

/* flags */
#define ETAIM_F_CONTINUE_ON_NOCONV 1 /* keep marching after a step hits maxit */
#define ETAIM_F_FAIL_ON_UNSTABLE 2   /* return ETAIM_EUNSTABLE instead of only flagging */
#define ETAIM_F_GRAPH 4              /* capture each Arnoldi step j of the batched GMRES once as a
                                        HIP graph and replay it (device-side gating, see sync_every);
                                        while profiling is on the same steps run as direct launches */
#define ETAIM_F_IMPLICIT_STOP 8      /* end a step's GMRES as soon as every column's Givens residual
                                        estimate meets the tolerance; without it the solver
                                        recomputes the true residual b - Z x at a new cycle start
                                        and stops only if that meets the tolerance too (one operator
                                        application more per step) */
#define ETAIM_F_STEP_GRAPH 32        /* replay every time step of a forward march (from its fourth step
                                        and from the second step of a call on) from captured HIP graphs:
                                        delayed field, one GMRES cycle of device-gated Arnoldi steps,
                                        commit and bookkeeping in one graph, its per-step values read
                                        from device descriptors; several steps are enqueued per host
                                        check.  A step that has not converged within the captured
                                        Arnoldi steps stops the replays on the device and is completed
                                        eagerly.  Needs ETAIM_F_IMPLICIT_STOP and the register engines;
                                        otherwise, while profiling, for the adjoint march and with
                                        ETAIM_F_FAIL_ON_UNSTABLE the steps run eagerly.  Results equal
                                        the eager march bit for bit. */
#define ETAIM_F_RESIDUAL_CHECK 16    /* forward marches check eq. (5) in FP64 every 16 steps (step l
                                        with (l + 1) % 16 == 0) and at the last step of the call:
                                        ||V_l - sum_{m>=0} Z_m I_{l-m}|| / ||V_l - sum_{m>=1} Z_m I_{l-m}||
                                        with the FP64 operators, for every column of an FP64 march and
                                        for column 0 of an FP32 one (its FP64 history is kept by an
                                        internal FP64 context of the same problem, about 1.4 GB at the
                                        level-4 size); results in etaim_stats */

/* Integral equation (Sec. 2.1).  ETAIM_EFIE: the time-differentiated EFIE
 * on the envelopes.  ETAIM_CFIE: alpha EFIE + (1 - alpha) eta MFIE, the
 * MFIE taken on the exterior of the closed surface (outward normals, the
 * mesh's counter-clockwise order), differentiated in time like the EFIE:
 *   Z^H_m = D_m / 2 <S_k, S_k'> - int int g'_m(R) S_k . (n x (Rhat x S_k')),
 *   g'_m = -(exp(-j k_c R)/4 pi) [P_A(tau)/(c R) + (T'/dt + j w_c T)(tau)/R^2],
 * D_m = (T'/dt + j w_c T)(m) (piece m), the same 7 x 7 rule (zero on a
 * triangle with itself).  Its far part is the curl of the interpolated
 * potential: test projection H[k,:,n] = int (S_k x n) x grad l_n over the
 * stencil's Lagrange functions, Green table exp(-j k_c R)(T'/dt + j w_c
 * T)(tau)/(4 pi R) on the EFIE's anterpolated currents and forward
 * spectra.  The excitation adds (1 - alpha) <S_k, n x (khat x D E~_inc)>.
 * With ETAIM_CFIE the forward operators and the forward march are
 * supported; the adjoint (transposed) operators and march return
 * ETAIM_EUNSUPPORTED. */
#define ETAIM_EFIE 0
#define ETAIM_CFIE 1

/* Temporal basis (Sec. 3).  ETAIM_CPPIF: the causal cubic interpolant of
 * order Q = 3.  ETAIM_BLIF: the band-limited interpolatory function of half
 * width M = 3, T = sinc(tau) W(tau) on -M < tau <= M with Knab's window
 * W = sinh(a sqrt(u)) / (sqrt(u) sinh a), u = 1 - (tau/M)^2,
 * a = pi M (1 - 2 beta), beta = f_bw dt (f_bw is then required, with
 * 0 < beta < 1/2).  Its M - 1 future samples are extrapolated from the last
 * nsamp ones, I_{l+k} ~ sum_p a_kp I_{l-p}, a_k the least-squares fit of
 * exp(j w k dt) by exp(-j w p dt) at nomega frequencies spread evenly over
 * |w| <= 2 pi f_bw (Sec. 3.1.2 cites the scheme; this fit is the library's
 * reading), and folded into the marching matrices:
 * Z~_p = Z_p + sum_k a_kp Z_{-k} for p < nsamp.  N_g = floor(Rmax/(c dt) + M).
 * The march, its operators and the far field then run unchanged. */
#define ETAIM_CPPIF 0
#define ETAIM_BLIF 1

typedef struct etaim_ctx etaim_ctx;

/* Triangle mesh of the closed PEC surface (Sec. 3, RWG on a triangular
 * mesh).  xyz: host float64 [nv][3] in metres; tri: host int32 [nt][3]
 * vertex indices, counter-clockwise about the outward normal. */
typedef struct {
    int32_t nv;
    const double *xyz;
    int32_t nt;
    const int32_t *tri;
} etaim_mesh;

/* RWG table: host int32 [ns][4] = {t_plus, t_minus, edge_v0, edge_v1}.
 * T+ must contain the directed edge v0 -> v1 in its counter-clockwise
 * order, T- the directed edge v1 -> v0; the basis current flows from T+
 * into T- (S_k = +l/(2A+) (r - v+) on T+, -l/(2A-) (r - v-) on T-). */
typedef struct {
    int32_t ns;
    const int32_t *idx;
} etaim_rwg;

typedef struct {
    double fc;          /* centre (carrier) frequency f_c [Hz], > 0 */
    double dt;          /* time step [s]; 0 => derived (see ng, beta, f_bw) */
    double beta;        /* dt = beta / f_bw when dt == 0 and ng == 0 (Sec. 3) */
    double f_bw;        /* essential half bandwidth [Hz] for the beta rule */
    int32_t nt_steps;   /* N_t >= 1 */
    int32_t order;      /* CPPIF order Q, or BLIF half width M; only 3 is supported */
    int32_t grid[3];    /* auxiliary grid nodes per axis (>= 8 each); padded
                           FFT lengths 2*grid must be products of 2 and 3 */
    double d_near;      /* near-zone distance [m] between basis centres */
    int32_t ng;         /* history depth N_g; 0 => floor(Rmax/(c dt) + Q).
                           With dt == 0 and ng > 0: dt = Rmax/(c (ng - Q + 1/2)) */
    int32_t precision;  /* ETAIM_FP64 or ETAIM_FP32 */
    int32_t batch;      /* B >= 1 excitations marched together */
    double tol;         /* GMRES relative residual tolerance (Sec. 5.1) */
    int32_t restart;    /* GMRES restart length, 1..200 */
    int32_t maxit;      /* max GMRES iterations per step */
    int32_t flags;      /* ETAIM_F_* */
    int32_t sync_every; /* Arnoldi steps enqueued per host convergence check; 0 or 1 => check after
                           every step.  Steps enqueued past convergence return at once on the
                           device (a gate flag), so results do not depend on it. */
    int32_t formulation; /* ETAIM_EFIE (0) or ETAIM_CFIE (1), Sec. 2.1 */
    double alpha;        /* ETAIM_CFIE: weight of the EFIE, 0 <= alpha < 1 (the paper's spheres:
                            0.5, Sec. 5.1); ignored for ETAIM_EFIE */
    int32_t basis;       /* temporal basis: ETAIM_CPPIF (0) or ETAIM_BLIF (1) */
    int32_t nsamp;       /* ETAIM_BLIF: past samples the future ones are extrapolated from
                            (1..4; 0 => 3, the paper's N_samp) */
    int32_t nomega;      /* ETAIM_BLIF: frequencies of the extrapolation's fit (nsamp..64;
                            0 => 2 nsamp, the paper's N_omega) */
} etaim_params;

typedef struct {
    double dt, h, origin[3], rmax, stencil_radius;
    int32_t ns, ng, mn, nnz, batch, precision;
    int32_t grid[3], padded[3];
    int64_t device_bytes;
} etaim_derived;

typedef struct {
    int32_t steps_done;        /* steps completed by the last march */
    int32_t total_iters;       /* GMRES iterations summed over steps and columns */
    int32_t max_iters;         /* largest per-step, per-column iteration count */
    int32_t first_noconv_step; /* -1 if every step converged */
    int32_t unstable_step;     /* -1, or the step where late-time growth was flagged: the
                                  current norm grew monotonically by more than 10x over 32 steps
                                  of this call that begin more than N_g steps after the step
                                  where the excitation's norm peaked (the pulse has crossed the
                                  object) */
    double ms_rhs, ms_solve, ms_commit, ms_total;  /* device time per phase */
    double max_rel_residual;   /* largest final relative residual (estimate) */
    int32_t *iters_per_step;   /* optional caller host buffer [N_t] (or NULL) */
    int32_t residual_checks;     /* FP64 checks of eq. (5) made (ETAIM_F_RESIDUAL_CHECK), else 0 */
    int32_t residual_worst_step; /* step of the largest checked residual (-1: none) */
    double max_residual64;       /* largest FP64 relative residual of eq. (5) over the checks */
    int32_t graph_steps;         /* steps replayed from whole-step graphs (ETAIM_F_STEP_GRAPH) */
    int32_t graph_halts;         /* replayed steps that did not converge within their graph's
                                    Arnoldi steps and were completed eagerly */
} etaim_stats;

/* Context set-up (the paper's "matrix fill", Sec. 4 stages (i)-(iv), not
 * timed in marching): validates the mesh and RWG table, derives dt, N_g,
 * the grid (h, origin) and the near-zone depth M_n, computes the
 * moment-matching projection (moments up to order 3, Sec. 5.1), the grid
 * Green functions and their spectra (m = 0..N_g), the exact near-zone
 * entries and their pre-correction, and allocates the history rings.
 * *out receives the context; hip_stream is a hipStream_t (NULL = default).
 * Errors: EINVAL (invalid mesh/RWG/params, a stencil outside the grid),
 * ENOMEM, EHIP, EUNSUPPORTED (order != 3, radix other than 2/3). */
int etaim_create(etaim_ctx **out, const etaim_mesh *mesh, const etaim_rwg *rwg,
                 const etaim_params *params, void *hip_stream);

/* Derived quantities of a context (host struct filled in). */
int etaim_describe(const etaim_ctx *ctx, etaim_derived *out);

/* Excitation vectors of the cosine-modulated Gaussian plane wave, eq. (1)
 * (Sec. 2.2), tested at t = l dt, l = 1..N_t (eq. (4)):
 *   V_l[k] = int S_k . (d/dt + j w_c) E~(r, l dt) dS,
 *   E~ = p g(tau) exp(-j w_c (r.k/c + t_d)), g = exp(-tau^2/2 sigma^2),
 *   tau = t - r.k/c - t_d.
 * khat, phat: host float64 [nb][3] (unit, orthogonal); sigma, td [s].
 * V: device complex128 [N_t][nb][ns].  nb must equal the context batch. */
int etaim_excitation_planewave(etaim_ctx *ctx, int32_t nb, const double *khat,
                               const double *phat, double sigma, double td, void *V);

/* etaim_excitation_planewave for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same vectors, computed by the same kernel, with the
 * directions and polarisations staged in a fixed per-device array instead
 * of a per-call allocation.  The call allocates and frees nothing.  Limit:
 * nb <= 4096 (ETAIM_EINVAL beyond, with a message naming the limit).  The
 * array (48 KiB per device, held until the process ends) is shared by every
 * call on a device and keeps the last call's contents: calls that overlap
 * on one device, from different host threads or streams, race.  The call
 * synchronises the context's stream before it returns. */
int etaim_excitation_planewave_noalloc(etaim_ctx *ctx, int32_t nb, const double *khat,
                                       const double *phat, double sigma, double td, void *V);

/* Forward march of eq. (5) (Sec. 4 stage (v); GMRES as in Sec. 5.1, right-
 * preconditioned by default with a sparse approximate inverse of Z0 on the
 * near-zone pattern, or with the paper's diagonal (Jacobi) preconditioner
 * when etaim_tuning.precond = 0): for l = 1..n solve
 *   (Z0near + Z0fft) I_l = V_l - sum_{m=1}^{N_g} (Zmnear + Zmfft) I_{l-m},
 * starting from a zero history, n = nsteps (1..N_t; 0 means N_t).
 * V, I_out: device complex128 [N_t][B][ns] (the first n steps are used).
 * stats may be NULL.  Errors: ENOCONV (unless CONTINUE_ON_NOCONV),
 * ENONFINITE, EUNSTABLE (with FAIL_ON_UNSTABLE). */
int etaim_march(etaim_ctx *ctx, const void *V, void *I_out, int32_t nsteps, etaim_stats *stats);

/* Continue a forward march (checkpoint/resume of the time marching, eq. (5)):
 * steps first .. first + nsteps - 1, with the history rings as the last
 * etaim_march / etaim_march_continue on this context left them, or as
 * etaim_state_load set them, at step `first` (ETAIM_EINVAL otherwise).
 * V and I_out are the full device arrays [N_t][B][ns]; I_out must hold the
 * solutions of the steps before `first` (the initial guess extrapolates the
 * last guess_order solutions, at most 6: etaim_tuning.guess_order).  The
 * result equals that of one uninterrupted march; stats
 * cover this call's steps (iters_per_step[0] is step `first`). */
int etaim_march_continue(etaim_ctx *ctx, const void *V, void *I_out, int32_t first, int32_t nsteps,
                         etaim_stats *stats);

/* March state for checkpoint/resume: the spectrum ring (N_g slots), the
 * current ring (M_n steps), the next step and the carried initial-guess
 * order.  etaim_state_size gives the bytes; save copies the state of the
 * last completed forward march to caller-owned host memory (ETAIM_EINVAL if
 * there is none, or after etaim_delayed_field / an adjoint march / a change
 * between the register plane engines (yz_engine 1, 2: ring slots by parity
 * quadrants) and the LDS or line-pass engines (0, 3: plain slots) replaced
 * the rings); load restores it into a context of the same problem
 * (precision, batch, mesh, grid, N_g, M_n) whose y/z engine lays the ring
 * out the same way (ETAIM_EINVAL otherwise).  At the bench workload the
 * state is 21.7 GB. */
int etaim_state_size(const etaim_ctx *ctx, size_t *bytes);
int etaim_state_save(const etaim_ctx *ctx, void *host, size_t bytes);
int etaim_state_load(etaim_ctx *ctx, const void *host, size_t bytes);

/* y = (Zmnear + Zmfft) x for 0 <= m <= N_g (Sec. 4 stages (i)-(iv)).
 * x, y: device complex128 [B][ns]. */
int etaim_apply_z(etaim_ctx *ctx, int32_t m, const void *x, void *y);

/* Delayed field b = sum_{m=1}^{N_g} (Zmnear + Zmfft) hist[m-1] for an
 * injected history hist[m-1] = I_{l-m} (the right-hand-side sum of eq. (5)).
 * hist: device complex128 [N_g][B][ns]; b: device complex128 [B][ns]. */
int etaim_delayed_field(etaim_ctx *ctx, const void *hist, void *b);

/* Scattered far-field envelopes (Sec. 2.4 post-processing):
 *   u_d(l dt) = -(mu/4pi) [I - d d] sum_{k',l'} I_l'[k'] int S_k'
 *               [T'(tau')/dt + j w_c T(tau')] exp(j k_c d.r') dS',
 *   tau' = l - l' + d.r'/(c dt).
 * dirs: host float64 [nd][3] unit vectors; I: device complex128
 * [N_t][B][ns]; U: device complex128 [N_t][B][nd][3]. */
int etaim_farfield(etaim_ctx *ctx, int32_t nd, const double *dirs, const void *I, void *U);

/* Adjoint of etaim_farfield: S = F^H Ubar, S device complex128 [N_t][B][ns]. */
int etaim_farfield_adjoint(etaim_ctx *ctx, int32_t nd, const double *dirs, const void *Ubar,
                           void *S);

/* Co-polarised radar cross section from far-field envelopes (Sec. 2.4):
 * for frequency f_c + df[i], incidence b and direction d,
 *   sigma_out[i][b][d] = 4 pi |pol_d . U_bd(df_i)|^2 / G(df_i)^2,
 *   U_bd(df) = dt sum_l U[l][b][d] exp(-j 2 pi df (l+1) dt),
 *   G(df) = pulse_sigma sqrt(2 pi) exp(-2 pi^2 pulse_sigma^2 df^2),
 * i.e. the far field per unit incident field at that frequency: the
 * envelope's Fourier transform over that of the Gaussian pulse of eq. (1)
 * of width pulse_sigma (its delay and carrier phase drop out of |.|).
 * U: device complex128 [N_t][B][nd][3] as etaim_farfield writes it; pol:
 * host [nd][3] unit vectors (theta-hat for sigma_theta-theta); df: host
 * [nf] in Hz; sigma_out: device double [nf][B][nd], in m^2. */
int etaim_rcs(etaim_ctx *ctx, int32_t nd, const double *pol, int32_t nf, const double *df,
              double pulse_sigma, const void *U, double *sigma_out);

/* Thresholded dB-error norm of eq. (2) (Sec. 2.4) between two RCS patterns
 * sampled on n directions with quadrature weights w (sin(theta) on a
 * (theta, phi) grid): values are mapped to max(10 log10 sigma, TH) - TH with
 * TH = 10 log10(max sigma_ref) - floor_db (the paper uses 80 dB), then
 * err = sum w (a - b)^2 / sum w b^2.  Host arrays; needs no context. */
int etaim_db_error(int32_t n, const double *sigma, const double *sigma_ref, const double *w, double floor_db,
                   double *err);

/* Adjoint march, backward in time with the conjugate Green spectra and
 * conjugate near-zone values (the operators are complex-symmetric):
 *   Z0^H lambda_l = S_l - sum_{m=1}^{N_g} Zm^H lambda_{l+m}, l = N_t..1.
 * S, Lambda: device complex128 [N_t][B][ns].  For J = |F I|^2 and
 * S = F^H F I, dJ/d conj(V) = Lambda.  The call takes no checkpoint
 * interval: eq. (5) is linear in I, so the adjoint needs only S (which the
 * caller forms from the forward currents it holds), never the forward
 * history rings, and there is no forward state to recompute. */
int etaim_adjoint_march(etaim_ctx *ctx, const void *S, void *Lambda, etaim_stats *stats);

/* Kernel classes traced by etaim_set_profiling (HIP events recorded on the
 * context stream around every launch of the class, with the algorithmic
 * bytes of that launch: compulsory reads + writes of its inputs/outputs). */
#define ETAIM_K_ANTERP_X 0    /* anterpolation gather + forward x-FFT */
#define ETAIM_K_YZ_GREEN 1    /* per x-frequency plane: 2-D FFT, Green multiply, inverse 2-D FFT */
#define ETAIM_K_FFT_X_INV 2   /* inverse x-FFT pass */
#define ETAIM_K_INTERP_NEAR 3 /* interpolation + near-zone SpMV */
#define ETAIM_K_YZ_DELAYED 4  /* k-space temporal sum over the history + inverse 2-D FFT */
#define ETAIM_K_YZ_COMMIT 5   /* forward 2-D FFT into the history ring */
#define ETAIM_K_KRYLOV 6      /* GMRES vector kernels */
#define ETAIM_K_RING_FAR 7    /* time-block pass over the history ring (the terms a block's steps
                                 take from history older than the block, once per block; with
                                 the multilevel delay mode, each level's pass) */
#define ETAIM_K_COUNT 8

/* Delayed-field algorithm (the right-hand side of eq. (5), evaluated with
 * blocked space-time transforms, Sec. 4; its O(log^2 N_g) temporal cost,
 * Sec. 1 and Sec. 4).  mode 0 (the default where N_g <= 32): the k-space
 * temporal sum over the stored spectra, in time blocks of
 * etaim_tuning.delay_block steps.  mode 1 (the default where
 * 32 < N_g <= 1055 and its buffers take at most half the device memory
 * left free by etaim_create): multilevel time blocks: the lags 1..2 are summed at
 * every step; the lags [3 * 2^k, 6 * 2^k), k = 0..4, form level k, whose
 * share of the next 3 * 2^k steps' sums is computed once those steps' last
 * block of history is stored, as a length-6 * 2^k temporal DFT convolution
 * per spectrum point (overlap-save) added to a ring of per-step
 * accumulators; the lags from 96 on form further 48-step segments
 * [48 (j + 1), 48 (j + 2)), j = 1..20, passed with the top level over
 * windows 48 j steps older; equal to mode 0 up to rounding.  Mode 1 is
 * taken by every y/z engine in eager steps (whole-step graphs are not
 * replayed while it is set); it allocates 3 * 2^K spectrum slots
 * of accumulators (K = the top level) and the level tables on first use.
 * Changing the mode invalidates derived history sums, not the history.
 * With ETAIM_CFIE the MFIE pass keeps level tables and accumulators of its
 * own.  Errors: EINVAL (mode not 0 or 1), EUNSUPPORTED (mode 1 with
 * N_g > 1055). */
int etaim_set_delay_mode(etaim_ctx *ctx, int32_t mode);

/* Current delay mode (host out). */
int etaim_get_delay_mode(const etaim_ctx *ctx, int32_t *mode);

/* Turn per-class kernel tracing on (1) or off (0); turning it on clears the
 * counters.  Tracing adds two event records per launch. */
int etaim_set_profiling(etaim_ctx *ctx, int32_t on);

/* Trace only the kernel classes whose bit (1 << ETAIM_K_*) is set in
 * classes (0: off); clears the counters when any bit is set.  Single-kernel
 * classes (ETAIM_K_YZ_GREEN, _FFT_X_INV with the register x lines,
 * _YZ_DELAYED, _YZ_COMMIT, _RING_FAR) carry their events on the dispatch
 * itself; the others record event markers between launches, which cost
 * stream time.  ETAIM_EINVAL for a bit at or above ETAIM_K_COUNT. */
int etaim_set_profiling_mask(etaim_ctx *ctx, uint32_t classes);

/* Accumulated device time [ms], algorithmic bytes and launch count of one
 * kernel class since tracing was turned on (host outputs). */
int etaim_kernel_stats(const etaim_ctx *ctx, int32_t cls, double *ms, double *bytes, int64_t *launches);

/* Launch shapes and schedule of the batched march.  They change speed
 * only: every admissible setting computes the same operator (the FFT plans
 * differ in rounding order only, the schedules not at all). */
typedef struct {
    int32_t radix[3][8];     /* FFT radix plan per axis x, y, z: pass radices in order
                                (each 2, 3, 4, 6, 8, 12 or 16), product = padded length,
                                0-terminated */
    int32_t gather_rows;     /* grid rows per anterpolation block (>= 1) */
    int32_t lines_per_block; /* lines per block of the inverse x pass (>= 1) */
    int32_t interp_waves;    /* bases (one wavefront each) per interpolation block, 1..4 */
    int32_t sync_every;      /* Arnoldi steps per host convergence check, 1..restart */
    int32_t graph;           /* 1: replay captured Arnoldi steps (ETAIM_F_GRAPH); 2: replay whole
                                time steps of forward marches (ETAIM_F_STEP_GRAPH) */
    int32_t yz_engine;       /* y/z plane stage: 0 LDS-staged radix passes over the whole padded
                                plane, 1 register-resident parity quadrants (needs N_y = N_z in
                                {16, 24, 48}), 2 as 1 but the matvec and commit plane transforms take
                                the z lines first and hold two tiles instead of four, 3 separate
                                y- and z-line passes over a full-spectrum work array (any grid whose
                                lines fit the LDS line kernel; chosen by itself where the padded
                                plane does not fit the LDS) */
    int32_t x_engine;        /* x stage: 0 LDS-staged lines with the anterpolation fused in,
                                1 register-resident lines after a separate anterpolation
                                (needs N_x in {16, 24, 48}) */
    int32_t guess_order;     /* GMRES initial guess of step l: the polynomial through the last
                                p solutions evaluated at step l, p <= guess_order chosen as the
                                order that best predicted step l-1 (0: zero guess, 1: the
                                previous solution, up to 6: quintic); the converged solution
                                does not depend on it beyond the tolerance (default 6) */
    int32_t precond;         /* right preconditioner of the per-step GMRES: 0 Jacobi diag(Z0)^-1
                                (the paper's choice), 1 sparse approximate inverse of Z0 on the
                                near-zone pattern (default; M^H for the adjoint) */
    int32_t delay_block;     /* delayed field of the register engine in time blocks of this many
                                steps (1..8; 1: the direct sum over all N_g history steps at every
                                step): at step r0 + j of a block the terms that read history older
                                than r0 are summed for the whole block in one pass at r0, the j
                                terms of the block's own steps at the step; equal to the direct sum
                                up to rounding (default 6; used when N_g <= 32 in delay
                                mode 0, etaim_set_delay_mode) */
    int32_t interp_engine;   /* interpolation + near zone: 0 one wavefront per basis gathering its
                                stencil from HBM/L2 (interp_waves bases per block), 1 by grid tiles:
                                a block loads a tile's node box of a group of columns into LDS and
                                its wavefronts take the tile's bases from there */
    double apply_ms;         /* out: measured matvec time [ms] (0 if not measured) */
    double solve_ms;         /* out: measured GMRES solve of the tuning right-hand side [ms] (0 if not
                                measured) */
} etaim_tuning;

/* Autotuner of the batching form: times the admissible radix plans, launch
 * shapes and GMRES schedules on this context (AIM matvecs on a seeded
 * random vector; GMRES solves of a seeded right-hand side with zero history),
 * checks each candidate's matvec against the current setting (relative L2
 * <= 1e-4 in FP32, 1e-10 in FP64; others are skipped), and keeps the fastest.
 * budget_ms bounds the timing work (>= 1; candidates are tried in order of
 * expected benefit).  cache_path (host string or NULL): a JSON-lines file; a
 * record whose key matches this problem's shape (precision, batch, ns,
 * grid, near-zone size, restart, formulation) is applied without timing, otherwise the
 * result is appended.  out (host, may be NULL) receives the setting.  Must
 * not run while a march is in flight on the context's stream.  Errors:
 * EINVAL (budget < 1), EHIP, or the cache file cannot be written (EINVAL). */
int etaim_autotune(etaim_ctx *ctx, int32_t budget_ms, const char *cache_path, etaim_tuning *out);

/* Current setting (host out). */
int etaim_get_tuning(const etaim_ctx *ctx, etaim_tuning *out);

/* Apply a setting; EINVAL if a radix plan does not multiply to the padded
 * length or uses another radix, EUNSUPPORTED if a plan or shape does not fit
 * the kernels' LDS and register staging (or an engine 1 on another grid). */
int etaim_set_tuning(etaim_ctx *ctx, const etaim_tuning *t);

/* Copy a set-up array to host memory for inspection.  what: 0 projection
 * weights float64 [ns][4][64], 1 stencil corners int32 [ns][3], 2 near-zone
 * row pointers int32 [ns+1], 3 column indices int32 [nnz], 4 pre-corrected
 * near values complex128 [mn+1][nnz] (m-major), 5 diagonal of Z0 complex128
 * [ns], 6 folded Green spectra complex128 [ng+1][2][gz+1][gy+1][gx+1]
 * (g = grid size, already divided by the padded size; with ETAIM_CFIE the
 * EFIE's, weighted by alpha), 7 (ETAIM_CFIE) the MFIE's curl test projection
 * float64 [ns][4][64] (component 3 zero).  bytes must equal the array size. */
int etaim_export(const etaim_ctx *ctx, int32_t what, void *host, size_t bytes);

/* Message of the last failing call on this thread ("" if none). */
const char *etaim_last_error(void);

/* Frees the context and everything it owns (NULL is a no-op). */
void etaim_destroy(etaim_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ETAIM_H */
