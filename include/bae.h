/*
 * bae.h - C ABI of the MI355X (gfx950) library for the unfitted boundary algebraic
 * equation (BAE) method with free-space lattice Green's functions (arXiv 2502.05507).
 *
 * Problem (paper Sec. 2, eq. "elliptic"):  -Lap u + sigma u = f in Omega,  u = g on the
 * boundary, sigma >= 0, Omega given by a level set (interior where phi < 0, Sec. 4.2),
 * discretised by the 7-point stencil on a uniform grid of spacing h (eq. "discrete").
 * The library implements Algorithm 1 (Sec. 3.5), double-layer formulation:
 *   LGF table  G_s, s = sigma h^2 (Sec. 2.2, eqs. "lgf", "lgf_bessel", 1/48 table of Sec. 4)
 *   point sets M+, gamma+-, N+, D_n, E and the hat-function closure Phi (Sec. 2.1, 3.2)
 *   matrix-free double layer  v(m) = sum_{n in gamma-} D(m,n) q_d(n),
 *       D(m,n) = sum_{k in D_n} [G_s(m-n) - G_s(m-k)]                    (Sec. 3.2)
 *   BAE operator  A = Phi+ D+ + Phi- D-,  GMRES on A q_d = b            (Sec. 3.4, eq. "double_bae")
 *   b = g(x*) - Phi u_p,  u_gamma = [D+ q_d; D- q_d],  u = u_p + D q_d on M+   (Algorithm 1)
 *
 * Conventions
 *   - Every call returns an int status: BAE_OK (0), BAE_NOT_CONVERGED (1, results valid),
 *     or a negative error code; bae_last_error() gives a message for the calling thread.
 *   - Grid node (i,j,k) sits at origin + h*(i,j,k); node arrays are [n0][n1][n2], k fastest.
 *   - gamma- (the unknowns' index set) and gamma+ are returned in lexicographic order of
 *     (i,j,k).  Vectors "on gamma" are [gamma+ ; gamma-] in that order.
 *   - Multi-RHS arrays are [nrhs][len], row major.
 *   - "_dev" pointers are device pointers on the context's device (e.g. from torch tensors);
 *     other pointers are host memory owned by the caller.  The library never keeps a
 *     caller pointer beyond the call.
 *   - stream arguments are hipStream_t passed as void* (NULL = the default stream).
 *   - Kernel sign convention: positive, L = (6+s) I - sum of the 6 shifts, G_0(0) = 0.25273...
 */
#ifndef BAE_H
#define BAE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define BAE_OK 0
#define BAE_NOT_CONVERGED 1      /* GMRES hit maxit; density/history still valid */
#define BAE_ERR_ARG (-1)         /* bad argument (null pointer, size, enum)        */
#define BAE_ERR_GEOMETRY (-2)    /* empty M+, interior within 2 nodes of the grid edge */
#define BAE_ERR_NONFINITE (-3)   /* NaN/Inf in level set, boundary data or source  */
#define BAE_ERR_OOM (-4)         /* device allocation failed                       */
#define BAE_ERR_HIP (-5)         /* a HIP runtime call failed                       */
#define BAE_ERR_STATE (-6)       /* call out of order (e.g. solve before set_rhs)   */
#define BAE_ERR_ADMISSION (-7)   /* a served request exceeds the whole memory budget */

/* ------------------------------------------------------------------ enums */
#define BAE_LS_SPHERE 1     /* params[0] = radius                                     */
#define BAE_LS_ELLIPSOID 2  /* params[0..2] = semi-axes (axis aligned)               */
#define BAE_LS_TORUS 3      /* params[0] = R (centre line, xy plane), params[1] = r  */
#define BAE_LS_STAR 4       /* r0*(1 + amp*sin(m theta)*cos(k phi)): params = r0, amp, m, k;
                               theta polar angle from +z, phi = atan2(y, x)           */
#define BAE_LS_SAMPLED 5    /* phi given at the nodes; crossings by linear interpolation */

#define BAE_PREC_FP64 0     /* FP64 LGF sum                                           */
#define BAE_PREC_FP32 1     /* FP32 LGF sum, compensated accumulation                 */
#define BAE_PREC_FFT 2      /* the LGF sum as an FFT convolution on the grid box, FP64
                               (fast summation: O(B log B) for a box of B nodes instead
                               of O(|targets| |sources|))                               */

#define BAE_SOLVE_FP64 0          /* plain FP64 GMRES                                 */
#define BAE_SOLVE_FP32_REFINED 1  /* FP64 iterative refinement around FP32-matvec GMRES */
#define BAE_SOLVE_FFT 2           /* FP64 GMRES whose matvecs are FFT convolutions        */

#define BAE_LAYER_DOUBLE 0        /* double-layer formulation (Sec. 3.4 eq. "double_bae") */
#define BAE_LAYER_SINGLE 1        /* single-layer formulation (Sec. 3.4)                 */
#define BAE_LAYER_DIRECT 2        /* direct formulation (Sec. 3.1, eq. "direct_sys"): the
                                     unknowns are v on gamma itself                      */

#define BAE_PARTICULAR_FREE 0     /* u_p: the free-space volume potential (LGF sum, FFT)  */
#define BAE_PARTICULAR_BOX 1      /* u_p: Algorithm 1's finite-grid G_h[chi_{M+} f]      */

/* ------------------------------------------------------------------ structs */
typedef struct bae_grid {
    int32_t n[3];        /* nodes per axis, in [5, 2049]                            */
    double origin[3];    /* coordinates of node (0,0,0)                             */
    double h;            /* grid spacing (> 0)                                      */
    double sigma;        /* sigma = kappa^2 >= 0                                    */
} bae_grid;

typedef struct bae_levelset {
    int32_t kind;              /* BAE_LS_*                                          */
    double center[3];
    double params[8];
    const double* phi_samples; /* BAE_LS_SAMPLED: n0*n1*n2 host doubles, else NULL  */
} bae_levelset;

typedef struct bae_options {   /* zero-initialise for defaults                      */
    int32_t device;            /* HIP device ordinal                                */
    int32_t near_radius_fp64;  /* must be 0: the LDS table radii are fixed by the     */
    int32_t near_radius_fp32;  /* kernels (47 / 60 for sigma = 0, 46 / 59 otherwise)  */
    int32_t max_krylov;        /* Krylov basis capacity per RHS (default 400)       */
    int32_t max_rhs;           /* right-hand sides the context can hold (default 16) */
    int32_t sum_wait_polls;    /* polls of each bounded wait in the LGF sum's work hand-off
                                  before the sum gives up and the call reports BAE_ERR_HIP
                                  (0: default 2^22, ~0.1 s; < 0: none, every wait gives up at
                                  once -- for tests of that failure path)               */
} bae_options;

typedef struct bae_sizes {
    int64_t n_mplus, n_gamma_plus, n_gamma_minus, n_ext, n_edges;
    int64_t n_sources;         /* |gamma- u E|                                      */
    int64_t n_targets;         /* |gamma| = |gamma+| + |gamma-|                     */
    int64_t n_empty_d;         /* gamma- nodes with empty D_n (zero density column)  */
    int32_t max_offset;        /* largest |component| of an offset in N+ u E         */
    int32_t table_radius;      /* radius of the resident FP64 table                  */
    int64_t table_entries;
    int64_t device_bytes;      /* device memory held by the context                 */
    int32_t lds_radius_fp32;   /* offsets up to this max-norm come from the LDS table */
    int32_t lds_radius_fp64;
    int32_t far_field_fp32;    /* 1: the FP32 sum uses a far-field expansion beyond  */
    int32_t far_field_fp64;    /*    the LDS radius (sigma = 0, or the checked        */
                               /*    sigma > 0 form in FP32); 0: the exact table      */
    double far_field_err_fp32; /* sigma > 0: largest relative error of that form      */
                               /* against the context's table (-1 when not checked)   */
    int32_t conv_box[3];       /* the FFT convolution (BAE_PREC_FFT): extents of its box  */
    int32_t conv_fft[3];       /*   and its FFT lengths (zeros until first used)       */
} bae_sizes;

typedef struct bae_solve_params {
    int32_t precision;         /* BAE_SOLVE_* (FFT: every matvec an FFT convolution) */
    double tol;                /* relative residual target ||b - A q|| / ||b||      */
    int32_t maxit;             /* GMRES iterations per (inner) solve; <= max_krylov */
    double inner_tol;          /* refined mode: floor of the inner FP32 GMRES tolerance
                                  (default 1e-6); each outer step asks for
                                  max(floor, 0.5 tol / current residual), capped at 0.1 */
    int32_t max_outer;         /* refinement steps (default 8)                       */
    int32_t compute_grid;      /* also form u on N+: Algorithm 1's reconstruction
                                  u = u_p + G_h[chi_{M-} L_h (u_gamma - u_p)] (one box
                                  solve per RHS)                                      */
    int32_t recycle_dim;       /* refined mode: the first inner solve's Krylov space (at
                                  most this many vectors) augments the later inner
                                  solves (GCRO); 0 = automatic (64 once a matvec has
                                  1e8 pair interactions, else none), < 0 = none       */
    int32_t formulation;       /* BAE_LAYER_DOUBLE (default, 0): (Phi+ D+ + Phi- D-) q = b;
                                  BAE_LAYER_SINGLE: (Phi+ S+ + Phi- S-) q = b with the
                                  single layer S(m,n) = G(m - n) on gamma- sources
                                  (Sec. 3.4); the density, u_gamma and u are those of
                                  the chosen layer.
                                  BAE_LAYER_DIRECT: the direct system (Sec. 3.1)
                                  [(I - P+) v+ - P- v- ; Phi+ v+ + Phi- v-] = [0 ; b] for v
                                  on gamma ([gamma+; gamma-], the "density" returned, of
                                  length |gamma|); u_gamma = v + u_p.  Its first use on a
                                  context sets up the gamma x gamma sum and |gamma|-long
                                  Krylov vectors (BAE_ERR_STATE while the context belongs
                                  to a batch)                                          */
    const double* x0_dev;      /* initial densities [nrhs][|gamma-|] (device, FP64), or NULL
                                  for x0 = 0 (the paper's choice, Sec. 4); GMRES then solves
                                  A d = b - A x0 and returns x0 + d.  Read during the solve
                                  (bae_solve: ordered after the null stream's work;
                                  bae_solve_async: after its stream's)                 */
} bae_solve_params;

typedef struct bae_result {
    int32_t status;            /* BAE_OK or BAE_NOT_CONVERGED                       */
    int32_t iterations;        /* total GMRES iterations (all inner solves)         */
    int32_t outer_steps;       /* refinement steps (0 for FP64)                      */
    int32_t converged;
    double rel_residual_est;   /* last Givens estimate                               */
    double rel_residual_true;  /* ||b - A64 q|| / ||b|| with the FP64 operator       */
    double seconds;            /* wall time of the solve on the host                 */
    int64_t matvecs_fp64, matvecs_fp32;
} bae_result;

typedef struct bae_ctx bae_ctx;

/* ------------------------------------------------------------------ status */
const char* bae_status_string(int status);
/* Message of the last error on the calling thread ("" if none). */
const char* bae_last_error(void);

/* ------------------------------------------------------------------ LGF (Sec. 2.2) */
/* Entries in the 1/48-symmetric table: (R+1)(R+2)(R+3)/6. */
int64_t bae_lgf_table_size(int32_t R);
/*
 * G_s(a,b,c) for 0 <= a <= b <= c <= R, s = sigma h^2 >= 0, in FP64, written to out_dev
 * (device, bae_lgf_table_size(R) doubles) at index c(c+1)(c+2)/6 + b(b+1)/2 + a.
 * Bessel-integral form of Sec. 2.2 with exp(-(6+s)t): composite Gauss-Legendre in ln t on
 * [0, T*], large-argument (Hankel) series of I_n integrated term by term beyond T*.
 * R in [0, 4096]; s finite and >= 0, else BAE_ERR_ARG.  Runs on `stream`, asynchronous.
 */
int bae_lgf_table(double s, int32_t R, double* out_dev, void* stream);
/*
 * bae_lgf_table for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same table, with their scratch (quadrature nodes, weights and scaled Bessel values) in a
 * static device array of 8.9 MB that each GPU the library runs on holds until the process
 * ends; no hipMalloc, hipFree or stream synchronisation, asynchronous on `stream` (a stream
 * of the current device).  R in [0, 2048] (BAE_ERR_ARG beyond: the scratch holds the rule
 * for at most that radius); s finite and >= 0.  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (other streams, other threads) race.
 */
int bae_lgf_table_noalloc(double s, int32_t R, double* out_dev, void* stream);

/* ------------------------------------------------------------------ context (Alg. 1 setup) */
/*
 * Classify the grid (M+, gamma+-, N+, D_n, E; Sec. 2.1, 3.2), find one boundary point
 * x* per gamma- node on the edge to the M+ neighbour with the smallest crossing t
 * (ties: -x,+x,-y,+y,-z,+z), build Phi, and make the LGF table for s = sigma h^2 resident
 * (Alg. 1 "PrecomputeLGF").  Structs are copied; phi_samples is read during the call only.
 * Errors: BAE_ERR_ARG, BAE_ERR_GEOMETRY, BAE_ERR_NONFINITE, BAE_ERR_OOM, BAE_ERR_HIP.
 */
int bae_create(const bae_grid* grid, const bae_levelset* ls, const bae_options* opt, bae_ctx** out);
int bae_destroy(bae_ctx* ctx);
int bae_get_sizes(const bae_ctx* ctx, bae_sizes* out);
/* Node sets as (i,j,k) triples, lexicographic; buffers of 3*count int32 (any may be NULL). */
int bae_get_sets(const bae_ctx* ctx, int32_t* gamma_plus, int32_t* gamma_minus, int32_t* ext);
/*
 * Dirichlet closure per gamma- node (lexicographic): boundary point xstar (3 doubles),
 * partner index into gamma+ (int32), weight t in [0,1): row (1-t) u(q) + t u(p) = g(x*).
 * Callers evaluate g at xstar and pass it to bae_set_rhs.  Any pointer may be NULL.
 */
int bae_get_boundary_points(const bae_ctx* ctx, double* xstar, int32_t* partner, double* t);

/*
 * Right-hand sides: g_xstar [nrhs][|gamma-|] (host), f_grid [nrhs][n0 n1 n2] (host, or
 * NULL for f = 0).  With f the particular solution u_p = h^2 sum_{M+} G_s(m-n) f(n) (the
 * free-space volume potential) is formed on gamma by the LGF sum as an FP64 FFT convolution
 * on the box of N+ u E (set up on first use), and b = g - Phi u_p.
 * nrhs in [1, max_rhs].  BAE_ERR_NONFINITE on NaN/Inf input.
 */
int bae_set_rhs(bae_ctx* ctx, int32_t nrhs, const double* g_xstar, const double* f_grid);
/*
 * The same with Algorithm 1's particular solution on the finite grid: u_p = G_h[chi_{M+} f],
 * G_h the inverse of the 7-point operator on the interior nodes of the box with u = 0 on its
 * boundary nodes (Sec. 2.1), by sine transforms along the three axes (DST-I, each an FFT of
 * length 2(N_d + 1); any n0 x n1 x n2 grid), instead of the free-space volume potential.  u,
 * u_gamma and the grid solution are the same discrete solution either way; the density q
 * differs.  With f == NULL it equals bae_set_rhs.  The context keeps u_p on the device
 * ((n0-2)(n1-2)(n2-2) doubles per RHS) for the grid solution.
 */
int bae_set_rhs_box(bae_ctx* ctx, int32_t nrhs, const double* g_xstar, const double* f_grid);
/*
 * Device form of bae_set_rhs / bae_set_rhs_box, asynchronous on `stream`: g_dev
 * [nrhs][|gamma-|] and f_dev [nrhs][n0 n1 n2] (or NULL for f = 0) are device FP64 arrays
 * (e.g. torch tensors) that must stay valid until `stream` has passed this call's work.
 * particular: BAE_PARTICULAR_FREE or BAE_PARTICULAR_BOX (as bae_set_rhs_box).
 * Nothing is read back: a non-finite g or f is flagged on the device and the next solve
 * fails with BAE_ERR_NONFINITE.  The first call with f on a context does one-time set-up
 * (index maps, work list) on the host and the context's own stream.  Errors: BAE_ERR_ARG.
 */
int bae_set_rhs_device(bae_ctx* ctx, int32_t nrhs, const double* g_dev, const double* f_dev, int32_t particular,
                       void* stream);
/* u_p of right-hand side r on the whole grid (n0*n1*n2, k fastest; zero on the box boundary)
   after bae_set_rhs_box with f; caller-owned host buffer.  BAE_ERR_STATE otherwise. */
int bae_get_particular(const bae_ctx* ctx, int32_t r, double* up_grid);

/*
 * Solve A q_d = b for every RHS (GMRES, x0 = 0, no preconditioner: Sec. 4), then form
 * u_gamma (and u on N+ if params->compute_grid).  results: nrhs entries (may be NULL).
 * Returns BAE_NOT_CONVERGED if any RHS missed the tolerance.
 */
int bae_solve(bae_ctx* ctx, const bae_solve_params* params, bae_result* results);
/* Outputs of the last solve, RHS r (or every RHS for r = -1, [nrhs][len]; host buffers):
   the density (|gamma-|, or |gamma| after a direct-formulation solve: bae_get_density_length),
   u_gamma (|gamma|), u on the grid (n0 n1 n2, NaN outside N+; needs compute_grid), residual
   history (r >= 0 only).  Errors: BAE_ERR_ARG, BAE_ERR_STATE (no solve yet). */
int bae_get_density(const bae_ctx* ctx, int32_t r, double* q);
int bae_get_gamma_values(const bae_ctx* ctx, int32_t r, double* u_gamma);
int bae_get_solution(const bae_ctx* ctx, int32_t r, double* u_grid);
int bae_get_history(const bae_ctx* ctx, int32_t r, double* hist, int32_t cap, int32_t* len);
/* Length per RHS of the last solve's density: |gamma-| for the layer potentials (solo,
   batched or served), |gamma| for the direct formulation (Sec. 3.1).  Size the buffers of
   bae_get_density / bae_get_density_device from it.  Errors: BAE_ERR_ARG, BAE_ERR_STATE (no
   solve yet). */
int bae_get_density_length(const bae_ctx* ctx, int64_t* len);
/*
 * Asynchronous solve (Algorithm 1's solve step, as bae_solve): its device work is ordered
 * after everything queued on `stream` so far (a PyTorch caller passes its current stream;
 * no device synchronisation) and runs on the context's own stream, driven by a host thread
 * of the context, and the call returns at once.  Argument errors are reported here; errors
 * of the solve itself by bae_solve_wait.  Any other call on the context (set_rhs, getters,
 * applies, another solve) first waits for the solve's host thread.
 */
int bae_solve_async(bae_ctx* ctx, const bae_solve_params* params, void* stream);
/* done = 1 once the asynchronous solve has finished (or none is running), else 0; never blocks. */
int bae_solve_poll(const bae_ctx* ctx, int32_t* done);
/* Waits for the asynchronous solve, copies its results (nrhs entries, may be NULL) and makes
   `stream` wait for every output of the solve on the device.  Returns the solve's status
   (BAE_OK, BAE_NOT_CONVERGED or its error); BAE_ERR_STATE if no solve was started. */
int bae_solve_wait(bae_ctx* ctx, void* stream, bae_result* results);
/* Device forms of the getters, asynchronous on `stream`: RHS r, or every RHS for r = -1
   ([nrhs][len]); q_dev bae_get_density_length doubles, u_dev |gamma| or n0 n1 n2 doubles per
   RHS. */
int bae_get_density_device(const bae_ctx* ctx, int32_t r, double* q_dev, void* stream);
int bae_get_gamma_values_device(const bae_ctx* ctx, int32_t r, double* u_dev, void* stream);
int bae_get_solution_device(const bae_ctx* ctx, int32_t r, double* u_dev, void* stream);

/* ------------------------------------------------------------------ operators (hot path) */
/*
 * Double layer potential on gamma (Sec. 3.2): v = [D+ q; D- q] for nrhs densities.
 * q_dev [nrhs][|gamma-|] FP64 (device), v_dev [nrhs][|gamma|] FP64 (device).
 * precision BAE_PREC_FP64 or BAE_PREC_FP32 (FP32 kernel sum, FP64 in/out).
 * Asynchronous on `stream`; q_dev/v_dev must not alias.
 */
int bae_apply_double_layer(bae_ctx* ctx, const double* q_dev, double* v_dev, int32_t nrhs,
                           int32_t precision, void* stream);
/*
 * Single layer potential on gamma (Sec. 3.4, S(m,n) = G(m - n) on gamma- sources):
 * v = [S+ q; S- q].  Same arguments, layouts and errors as bae_apply_double_layer.
 */
int bae_apply_single_layer(bae_ctx* ctx, const double* q_dev, double* v_dev, int32_t nrhs,
                           int32_t precision, void* stream);
/*
 * The direct system's operator (Sec. 3.1): y = [v+ - P+ v+ - P- v- ; Phi+ v+ + Phi- v-] with
 * (P+ v+)(p*) = -sum_edges G(q - p*) v(p), (P- v-)(p*) = sum_edges G(p - p*) v(q) over the
 * neighbour pairs p in gamma+, q in gamma-.  v_dev, y_dev: [nrhs][|gamma|] FP64 device,
 * [gamma+; gamma-] order; precision of the LGF sum as in bae_apply_double_layer.  The first
 * call sets up the direct formulation (see bae_solve_params.formulation).  Asynchronous on
 * `stream` after that set-up.
 */
int bae_apply_direct(bae_ctx* ctx, const double* v_dev, double* y_dev, int32_t nrhs, int32_t precision, void* stream);
/* The BAE operator A q = Phi+ D+ q + Phi- D- q (Sec. 3.4, eq. "double_bae").
   q_dev, aq_dev: [nrhs][|gamma-|] FP64 device. */
int bae_apply_operator(bae_ctx* ctx, const double* q_dev, double* aq_dev, int32_t nrhs,
                       int32_t precision, void* stream);
/*
 * The LGF sum of Sec. 3.2 by itself, for timing its kernel: forms the source weights of the
 * densities q_dev once (as bae_apply_double_layer does), then launches the sum over
 * gamma x (gamma- u E) `repeats` times in a row into the context's partial-sum scratch,
 * which the next operator call overwrites.  No result is returned and nothing is reduced.
 * q_dev [nrhs][|gamma-|] FP64 (device), 1 <= nrhs <= max_rhs, precision BAE_PREC_FP64 or
 * BAE_PREC_FP32, 1 <= repeats <= 1000.  Asynchronous on `stream`; the context's scratch is
 * shared with every other call on it.  Errors: BAE_ERR_ARG (null pointer, nrhs, precision or
 * repeats out of range), BAE_ERR_HIP (a failed launch).
 */
int bae_lgf_sum_repeat(bae_ctx* ctx, const double* q_dev, int32_t nrhs, int32_t precision, int32_t repeats,
                       void* stream);
/*
 * Pair counts of the LGF sum over gamma x (gamma- u E) as the kernel classifies them for
 * `precision` (per wavefront of 64 Morton-ordered targets and block of 64 sources):
 * counts[0] pairs in blocks within the LDS table radius (table lookups), [1] in all-far
 * blocks (far field: q = 4 in FP64; sigma > 0: global-table gathers), [2] in FP32 far
 * blocks (the q = 2 lattice form past its gap for sigma = 0, the checked Yukawa form beyond
 * the LDS radius for sigma > 0), [3] / [4] pairs of mixed blocks within / beyond the LDS
 * radius.  Host computation (no device work); for flop accounting.  counts: 5 int64.
 */
int bae_sum_stats(const bae_ctx* ctx, int32_t precision, int64_t* counts);
/*
 * The kernel the LGF sum uses, at `count` integer offsets (offsets_dev: [count][3] int32,
 * device) -> out_dev (count FP64): near table or far-field expansion exactly as the sum
 * evaluates it at `precision`.  For checking the far field and table lookups.
 */
int bae_lgf_eval(bae_ctx* ctx, const int32_t* offsets_dev, int64_t count, double* out_dev,
                 int32_t precision, void* stream);

/* ------------------------------------------------------------------ batched solves */
typedef struct bae_batch bae_batch;
/*
 * Group n contexts for lock-step solving (the batched form of Algorithm 1's solve step).
 * Every context must hold exactly one RHS (bae_set_rhs with nrhs = 1) and live on the
 * same device.  The batch keeps pointers to the contexts: they must outlive it and must
 * not be used concurrently with it.  Each GMRES phase is one launch for all problems; the
 * LGF sum is a persistent kernel over (problem, target tile, source chunk) items.
 */
int bae_batch_create(bae_ctx* const* ctxs, int32_t n, bae_batch** out);
/*
 * Time the LGF-sum tiling candidates (source blocks per chunk in {2, 4, 8, 16, 32, 64} x
 * persistent grid of {1, 2, 4} workgroups per compute unit) on this batch at `precision`,
 * keep the fastest, and append it to the tuning cache
 * ($BAE_AUTOTUNE_CACHE, else ~/.cache/bae_autotune.txt; keyed by GPU arch, log2 of the
 * pair count and of the batch size) that bae_batch_create reads.  chosen: 2 int32 (or NULL).
 */
int bae_batch_autotune(bae_batch* b, int32_t precision, int32_t* chosen);
/*
 * Solve every problem (GMRES x0 = 0, FP64 or FP32-refined as in bae_solve).  use_graph = 1
 * captures 8 GMRES iterations once as a HIP graph and replays it; 0 launches eagerly.
 * results: n entries (or NULL).  Densities, u_gamma and histories land in each context
 * (bae_get_density / bae_get_gamma_values / bae_get_history).
 */
int bae_batch_solve(bae_batch* b, const bae_solve_params* params, int32_t use_graph, bae_result* results);
/*
 * Pair counts of the batched LGF sum (Sec. 3.2) summed over the batch's problems, in the
 * classes of bae_sum_stats, as the batched kernel classifies them: its LDS table holds the
 * general layout (radius 59 in FP32, 46 in FP64), so a problem's counts can differ from its
 * solo ones.  Host computation; counts: 5 int64.  Errors: BAE_ERR_ARG.
 */
int bae_batch_sum_stats(const bae_batch* b, int32_t precision, int64_t* counts);
int bae_batch_destroy(bae_batch* b);

/* ------------------------------------------------------------------ serving (continuous batching) */
typedef struct bae_server bae_server;
/* Boundary data callback: g_out[i] = g(xyz[3i], xyz[3i+1], xyz[3i+2]) for i < count.  It is
   called on the server's set-up thread when a request is admitted. */
typedef void (*bae_boundary_fn)(void* user, int64_t count, const double* xyz, double* g_out);

typedef struct bae_server_options {
    int32_t device;
    int32_t max_slots;         /* requests on the device at once                       */
    int64_t hbm_budget;        /* device bytes all admitted requests may hold together  */
    int32_t precision;         /* BAE_SOLVE_FP64 or BAE_SOLVE_FP32_REFINED              */
    double tol;                /* relative residual target (default 1e-10)             */
    int32_t maxit;             /* GMRES iterations per (inner) solve                   */
    int32_t max_krylov;        /* Krylov capacity per request (default 200)            */
    int32_t iters_per_step;    /* GMRES iterations between scheduling points (default 4) */
    int32_t setup_threads;     /* host threads that classify geometries and build contexts
                                  (default 4, at most 16)                                */
} bae_server_options;

typedef struct bae_request {   /* one Dirichlet problem, f = 0 (sigma >= 0)             */
    bae_grid grid;
    bae_levelset levelset;     /* sampled level sets are copied at submit              */
    bae_boundary_fn g;
    void* user;                /* passed to g; must stay valid until the request is done */
} bae_request;

typedef struct bae_request_info {
    int32_t state;             /* 0 waiting, 1 running, 2 done, 3 failed               */
    int64_t n_gamma_minus, n_targets, bytes;
    double t_submit, t_admit, t_done;   /* seconds since the server started             */
} bae_request_info;

typedef struct bae_server_stats {
    int64_t submitted, admitted, completed, failed, steps, max_active, peak_bytes;
    int64_t bytes_in_use, waiting, running;
} bae_server_stats;

/*
 * Start a server: set-up threads classify the geometry of the first waiting requests (which
 * gives each one's device footprint before any allocation), admit requests in arrival order
 * when a slot is free and the footprint fits in hbm_budget, and build each one's context
 * (point sets, LGF table, boundary data through its callback; the callback may run on any of
 * these threads, one call at a time per request) on the context's own stream while the
 * batch runs; a scheduler
 * thread adds set-up requests to the running batch at the next step, advances all running
 * requests together (one launch per GMRES phase), and retires finished ones, releasing
 * their slot and memory.  A request larger than the whole budget fails with
 * BAE_ERR_ADMISSION; any other set-up failure fails that request only.
 */
int bae_server_create(const bae_server_options* opt, bae_server** out);
int bae_server_submit(bae_server* s, const bae_request* req, uint64_t* ticket);
/* Block until the request is done (timeout_s < 0: no limit).  Returns its status
   (BAE_OK / BAE_NOT_CONVERGED) or the error that failed it. */
int bae_server_wait(bae_server* s, uint64_t ticket, double timeout_s, bae_result* res, bae_request_info* info);
/* The request's state without blocking: 0 waiting, 1 admitted (set-up or running), 2 done,
   3 failed (its error then comes from bae_server_wait).  Errors: BAE_ERR_ARG (unknown ticket). */
int bae_server_poll(bae_server* s, uint64_t ticket, int32_t* state);
/* Copy a done request's density (|gamma-|) and u_gamma (|gamma|) out and forget it. */
int bae_server_fetch(bae_server* s, uint64_t ticket, double* q, int64_t q_cap, double* u_gamma, int64_t u_cap);
int bae_server_stats_get(bae_server* s, bae_server_stats* out);
/* Finish the running requests, fail the waiting ones, stop the thread. */
int bae_server_destroy(bae_server* s);

#ifdef __cplusplus
}
#endif
#endif /* BAE_H */
