/*
 * ehh.h -- C ABI of the MI355X elastic Helmholtz hybrid multigrid / domain
 * decomposition solver (Treister & Yovel, "A hybrid shifted Laplacian multigrid
 * and domain decomposition preconditioner for the elastic Helmholtz equations").
 *
 * The system (section 2.1 and section 3, eq. (14)) is the mixed staggered
 * discretisation
 *
 *     [ grad_h^T A_e(mu) grad_h - w^2 M    grad_h        ] [u]   [q]
 *     [ grad_h^T                          -D_c(1/(l+mu)) ] [p] = [0]
 *
 * with M = A_f(rho (1 - i gamma/w)) (eq. (5)).  The preconditioner approximately
 * inverts the shifted operator, in which M becomes A_f(rho (1 - i (gamma/w + alpha)))
 * on the u block only (eq. (10) with M_s = A_f(rho), section 3; the shift is
 * given the sign of the attenuation), by one multigrid cycle (Algorithm 1 applied
 * recursively) with damped red-black cell-wise Vanka relaxation, Galerkin coarse
 * operators (eq. (9)), staggered bilinear transfers and an exact coarsest solve,
 * optionally wrapped in overlapping domain decomposition with absorbing padding
 * (section 2.3, section 4, Algorithm 2).  The outer solver is FGMRES(m) from a
 * zero initial guess (section 6).
 *
 * Grid, unknowns and vector layout
 *   Cells: n[0] x n[1] (x n[2]) of size h; x is axis 0, depth is the last axis.
 *   Media (lambda, mu, rho, gamma) are cell arrays, x fastest.
 *   u_k lives on the interior faces normal to axis k (the normal displacement
 *   vanishes on the walls); p lives on cells.  Component k has
 *   prod_a (a == k ? n_a - 1 : n_a) unknowns, x fastest; p has prod n_a.
 *   A complex vector of one right-hand side is 2 N reals: the real parts of
 *   [u_0, u_1, (u_2), p] followed by their imaginary parts (N = unknowns).
 *   Several right-hand sides are stored back to back (stride 2 N reals).
 *
 * Units
 *   Every vector at this ABI is in the library's nondimensional scaling:
 *   h -> 1, lambda, mu -> lambda/mu_bar, mu/mu_bar, rho -> rho/rho_bar and
 *   w -> w h sqrt(rho_bar/mu_bar), with mu_bar = mean(mu) (mean(lambda+2mu) if mu
 *   is zero everywhere) and rho_bar = mean(rho).  A force q [SI] enters the
 *   u rows as q h^2/mu_bar; p_SI = p mu_bar / h.  Relative residuals are taken in
 *   the 2-norm of these vectors.  ehh_scaling() returns mu_bar, rho_bar and the
 *   nondimensional w.
 *
 * Memory and streams
 *   Pointers marked (device) are HIP device pointers; the caller owns them and
 *   keeps them alive until the work on `stream` (a hipStream_t, NULL = default
 *   stream) has completed.  The handle owns everything it allocates.  A handle
 *   may be used from one host thread at a time.  Calls return a status; on
 *   failure ehh_last_error() gives a message (thread-local).  EHH_ERR_INVALID
 *   is returned before any device work is enqueued.
 */
#ifndef EHH_H
#define EHH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EHH_MAX_LEVELS 8
#define EHH_MAX_RESTART 16

typedef struct ehh_ctx* ehh_handle_t;

typedef enum {
    EHH_OK = 0,
    EHH_NOT_CONVERGED = 1,      /* maxit reached: x holds the last iterate */
    EHH_ERR_INVALID = -1,       /* bad argument; nothing was enqueued */
    EHH_ERR_HIP = -2,           /* a HIP call failed (message has the HIP string) */
    EHH_ERR_OOM = -3,           /* device allocation failed; nothing leaked */
    EHH_ERR_BREAKDOWN = -4,     /* NaN/Inf in media or right-hand side, or Krylov breakdown */
    EHH_ERR_UNSUPPORTED = -5
} ehh_status_t;

typedef struct {
    int32_t dim;            /* 2 or 3 */
    int32_t n[3];           /* cells along x, y, z (n[2] ignored when dim == 2) */
    double  h;              /* cell size [m], > 0 */
    double  omega;          /* angular frequency [rad/s], > 0 */
    double  shift;          /* alpha >= 0 of the shifted preconditioning operator */
    int32_t abl_cells[3];   /* absorbing layer width per axis, on both sides (>= 0) */
    double  abl_max;        /* gamma/omega reached at the wall, per axis (section 2.1: 1) */
    double  atten0;         /* constant attenuation gamma_0 [1/s] added everywhere */
    double  mu_bar;         /* stiffness unit [Pa] of the nondimensional scaling; 0 = mean(mu) */
    double  rho_bar;        /* density unit [kg/m^3]; 0 = mean(rho).  Fix both to keep the
                               units of the vectors unchanged across model updates. */
} ehh_problem_t;

typedef struct {
    int32_t levels;         /* multigrid levels, 1..EHH_MAX_LEVELS; every (sub)domain
                               axis must be divisible by 2^(levels-1) */
    int32_t cycle;          /* recursive calls per coarse-grid correction: 1 = V, 2 = W */
    int32_t cycle_level;    /* levels >= cycle_level make `cycle` calls, the finer ones a
                               single call (0: every level; e.g. 1 = V on the finest
                               level, W below) */
    int32_t nu1, nu2;       /* red-black relaxation steps before / after the correction */
    int32_t vanka;          /* 1 = full cell block, 0 = economic (diagonal u part) */
    int32_t precond_bits;   /* 64: complex128 cycle; 32: complex64 cycle (FP32
                               accumulation) with an FP64 coarsest solve */
    int32_t restart;        /* FGMRES restart length m, 1..EHH_MAX_RESTART */
    int32_t dd_parts[3];    /* subdomains per axis; all 1 = no domain decomposition */
    int32_t dd_overlap;     /* overlap between neighbouring subdomains [cells] */
    int32_t dd_pad;         /* absorbing padding on interior subdomain sides [cells] */
    int32_t dd_colors;      /* 1 = one colour, local corrections averaged on the
                               overlaps; 0 = multicolour schedule of Algorithm 2 */
    double  damping[EHH_MAX_LEVELS];  /* Vanka damping per level, finest first */
    int32_t coarse_bits;    /* 32 (default) or 16: with the complex64 cycle, the stored
                               rows of the Galerkin levels (2D and 3D) are kept in FP16,
                               scaled by a power of two per level, and summed in FP32 (the
                               paper's half-precision storage of coarse data, section 3);
                               the 2D levels served by LDS-staged tiles (>= 256^2 cells with
                               more than 8 sources) read the FP32 compact stencil instead */
    int32_t coarse_dd_parts[3];  /* DD as the coarsest-level solver (MG-DD, section 4;
                               with dd_parts > 1 as well: DD-MG-DD): subdomains per axis of
                               every hierarchy's coarsest level; all 1 (default) = the
                               exact solve by a dense inverse.  Each subdomain's operator
                               is the coarsest Galerkin operator restricted to its cells
                               and their interior faces, inverted exactly (FP64); one
                               coarsest solve is one sweep over them */
    int32_t coarse_dd_overlap;   /* overlap of those subdomains [coarsest cells] (default 2) */
    int32_t coarse_dd_colors;    /* 0 (default): Algorithm 2 over the coarsest level's
                               subdomains (each colour from the residual left by the
                               previous ones); 1: one colour, corrections averaged */
    int32_t dd_batch;       /* 1 (default): with domain decomposition, each step of the
                               subdomains' cycles (and their gathers and scatters) runs
                               for all subdomains of a colour in one launch over a flat
                               (subdomain, block) list, up to 8 subdomains per launch;
                               0: one launch per subdomain and step */
    double  damping_p[EHH_MAX_LEVELS];  /* Vanka damping of the pressure row of a cell
                               block per level (component-dependent damping (w_u, w_p),
                               section 5.2; damping[] then damps the displacement rows);
                               0 (default) = damping[l] */
    int32_t reorth;         /* Gram-Schmidt in the FGMRES Arnoldi step: 0 (default) =
                               classical Gram-Schmidt, repeated once for a right-hand
                               side whose first pass kept less than 0.1 of |w| (the test
                               of Daniel, Gragg, Kaufman and Stewart with bound 0.1);
                               1 = always two passes (CGS2) */
} ehh_options_t;

typedef struct {
    int32_t status;         /* ehh_status_t of this right-hand side */
    int32_t iters;          /* preconditioner applications */
    double  rel_res_est;    /* Arnoldi estimate |b - A x| / |b| at exit */
    double  rel_res_true;   /* recomputed |b - A x| / |b| at exit (FP64) */
    double  conv_factor;    /* (r_k / r_5)^(1/(k-5)) over the estimates (section 5.4) */
} ehh_stats_t;

/* Defaults: 3 levels, V(1,1) (cycle_level 0), full Vanka, damping 0.75/0.5/0.25..., 64-bit
 * cycle, restart 5, no domain decomposition. */
void ehh_default_options(ehh_options_t* opt);

/* Build the operator, its shifted multigrid hierarchy (Galerkin coarse levels
 * and the inverse of every coarsest operator) and, with domain decomposition,
 * one padded subdomain hierarchy per subdomain (section 2.1 for the
 * coefficients, eq. (9) for the hierarchy, section 4 for the subdomains).
 *   lambda, mu, rho: FP64 cell arrays [Pa, Pa, kg/m^3], x fastest; rho > 0,
 *                    mu >= 0, lambda + mu > 0.  Host arrays are copied to the
 *                    device during the call; arrays in device memory (as the
 *                    runtime reports the pointer) are read in place, e.g. a
 *                    model updated on the device between solves.  Either way
 *                    the handle keeps only its own nondimensional coefficients
 *                    and the caller may reuse the arrays once the call returns.
 *   gamma:           FP64 physical attenuation [1/s] per cell (host or device,
 *                    as above), or NULL.
 *   stream:          work is enqueued on it; the call synchronises it before
 *                    returning.
 *   out:             receives the handle (set only on EHH_OK).
 * Errors: EHH_ERR_INVALID (sizes, levels, options, null media), EHH_ERR_BREAKDOWN
 * (non-finite or non-physical media),
 * EHH_ERR_OOM (nothing is kept: a later setup starts afresh), EHH_ERR_HIP. */
int32_t ehh_setup_operator(const ehh_problem_t* problem, const double* lambda,
                           const double* mu, const double* rho, const double* gamma,
                           const ehh_options_t* options, void* stream, ehh_handle_t* out);

/* Release every device buffer of the handle (waits for the device's work).
 * The buffers go to the library's device memory cache, from which later
 * handles take buffers of the same size class instead of calling hipMalloc;
 * the cache holds at most EHH_CACHE_MB MiB (environment, default 32768) and is
 * emptied for a device when an allocation there fails. */
void ehh_destroy(ehh_handle_t h);

/* Return the cached device buffers of every device to the driver (hipFree).
 * Handles that are alive keep their buffers.  Thread-safe; buffers released
 * by other threads while it runs may stay cached. */
void ehh_release_cached_memory(void);

/* counts[4] = unknowns of u_0, u_1, u_2 (0 in 2D), p; *stride = 2 * N reals
 * between consecutive right-hand sides. */
int32_t ehh_vector_layout(ehh_handle_t h, int64_t counts[4], int64_t* stride);

/* out[0] = mu_bar [Pa], out[1] = rho_bar [kg/m^3], out[2] = nondimensional omega. */
int32_t ehh_scaling(ehh_handle_t h, double out[3]);

/* y = A x for nrhs right-hand sides (FP64, global layout), A the system of eq. (14)
 * (shifted = 0) or the shifted preconditioning operator (shifted = 1).
 * x, y: (device), distinct. */
int32_t ehh_apply(ehh_handle_t h, int32_t shifted, const double* x, double* y,
                  int32_t nrhs, void* stream);

/* One multigrid cycle (Algorithm 1, recursive, zero initial guess) of the shifted
 * operator of subdomain `sub` (0 without domain decomposition): e ~ A_s^{-1} r.
 * r, e: (device) vectors in the subdomain's level-0 layout (ehh_level_info),
 * float when precond_bits == 32, double when 64; r and e distinct.
 * The cycle precision is not an argument: it is fixed at setup
 * (ehh_options_t.precond_bits), because the hierarchy's coefficients are built
 * in that precision; the subdomain index takes its place, since with domain
 * decomposition every padded subdomain has its own hierarchy. */
int32_t ehh_vcycle(ehh_handle_t h, int32_t sub, const void* r, void* e, int32_t nrhs,
                   void* stream);

/* z = M^{-1} v: the preconditioner of the outer Krylov method -- one cycle of the
 * global shifted hierarchy, or with domain decomposition one cycle per padded
 * subdomain combined by overlap averaging (one colour) or Algorithm 2.
 * v, z: (device) FP64, global layout, distinct. */
int32_t ehh_precondition(ehh_handle_t h, const double* v, double* z, int32_t nrhs,
                         void* stream);

/* Solve A x = b for nrhs right-hand sides with right-preconditioned FGMRES(m)
 * from x = 0 until |b - A x| <= tol |b| per right-hand side (section 6).
 * b, x: (device) FP64 global layout; stats: host array of nrhs entries or NULL.
 * Returns EHH_OK when every right-hand side converged, EHH_NOT_CONVERGED when
 * maxit preconditioner applications were reached for some (x holds the last
 * iterates), EHH_ERR_BREAKDOWN on a non-finite residual.  Synchronises `stream`
 * once per iteration to read the residual estimates. */
int32_t ehh_solve(ehh_handle_t h, const double* b, double* x, int32_t nrhs, double tol,
                  int32_t maxit, ehh_stats_t* stats, void* stream);

/* Solve the adjoint system A^H y = g.  A of eq. (14) is complex symmetric
 * (A^T = A), so A^H = conj(A): the call solves A conj(y) = conj(g) with the same
 * preconditioned FGMRES and conjugates the result.  g, y: (device) FP64 global
 * layout, distinct.  Stats and returns as ehh_solve (the residual norms of the
 * conjugated system equal those of the adjoint one). */
int32_t ehh_solve_adjoint(ehh_handle_t h, const double* g, double* y, int32_t nrhs, double tol,
                          int32_t maxit, ehh_stats_t* stats, void* stream);

/* Derivatives of a real misfit L(x_1..x_nrhs) with respect to the cell media,
 * by the adjoint-state method (section 1 motivates the solver by full-waveform
 * inversion): with A x_r = b_r and A^H y_r = dL/dx_r (the real-layout gradient
 * read as a complex vector), dL/dm_c = -Re sum_r y_r^H (dA/dm_c) x_r for
 * m = lambda, mu, rho at every cell c, A the unshifted operator of eq. (14).
 * Derivatives are per SI unit (Pa, kg/m^3) at the handle's fixed scaling
 * mu_bar, rho_bar (attenuation and omega held fixed).
 *   y, x: (device) FP64 global layout, nrhs vectors each.
 *   grad_lambda, grad_mu, grad_rho: (device) FP64 cell arrays, x fastest,
 *   distinct; overwritten (accumulate = 0) or added to (accumulate = 1).
 * Deterministic: each cell sums its right-hand sides in a fixed order. */
int32_t ehh_media_gradient(ehh_handle_t h, const double* y, const double* x, int32_t nrhs,
                           double* grad_lambda, double* grad_mu, double* grad_rho,
                           int32_t accumulate, void* stream);

/* Per-step entry points of the multigrid path (for checking each kernel).
 * Vectors are (device) in the level's layout and the cycle precision. */
int32_t ehh_num_subdomains(ehh_handle_t h);
/* n_local[3]: padded local cells; origin[3]: global cell of local cell 0;
 * lo[3], hi[3]: owned extent [lo, hi) in global cells. */
int32_t ehh_subdomain_info(ehh_handle_t h, int32_t sub, int32_t n_local[3],
                           int32_t origin[3], int32_t lo[3], int32_t hi[3]);
int32_t ehh_level_info(ehh_handle_t h, int32_t sub, int32_t level, int32_t n[3],
                       int64_t counts[4], int64_t* stride);
/* y = A_level x (level 0: the shifted fine operator; level > 0: Galerkin). */
int32_t ehh_level_apply(ehh_handle_t h, int32_t sub, int32_t level, const void* x,
                        void* y, int32_t nrhs, void* stream);
/* One damped red-black half-sweep on colour (0 = red: even index sum) with the
 * residual taken at the start of the half-sweep; e_in == NULL means e_in = 0. */
int32_t ehh_level_relax(ehh_handle_t h, int32_t sub, int32_t level, int32_t colour,
                        const void* b, const void* e_in, void* e_out, int32_t nrhs,
                        void* stream);
/* rc = P^T (b - A_level e) on level + 1. */
int32_t ehh_level_restrict(ehh_handle_t h, int32_t sub, int32_t level, const void* b,
                           const void* e, void* rc, int32_t nrhs, void* stream);
/* e += P ec, ec on level + 1. */
int32_t ehh_level_prolong(ehh_handle_t h, int32_t sub, int32_t level, const void* ec,
                          void* e, int32_t nrhs, void* stream);
/* e = A_coarsest^{-1} r (FP64 dense inverse; r, e in the cycle precision), or
 * with coarse_dd_parts one sweep of the coarsest-level DD from e = 0 (FP64). */
int32_t ehh_coarse_solve(ehh_handle_t h, int32_t sub, const void* r, void* e,
                         int32_t nrhs, void* stream);

/* Launch-shape autotuner.  For every level (on the first subdomain, applied to
 * all), the half-sweep and the residual are launched with each candidate
 * number of source groups per launch (the heuristic one, 1, 2, 4, ..., up to
 * nrhs) on zeroed workspaces and timed with HIP events on `stream` (best of
 * three rounds of 8 launches); another shape replaces the heuristic one when
 * it is at least 2 % faster.  The choice only changes which grid rows handle
 * which sources, so results are the same to the bit for any table.
 * table[2 * levels] receives (half-sweep groups, residual groups) per level,
 * finest first (0 = the heuristic); captured graphs are rebuilt.  Synchronises
 * `stream`. */
int32_t ehh_autotune(ehh_handle_t h, int32_t nrhs, int32_t* table, int32_t len, void* stream);
/* Install a table from ehh_autotune (e.g. kept in a cache across runs);
 * len = 2 * levels, entries in [0, 4096]. */
int32_t ehh_set_tuning(ehh_handle_t h, const int32_t* table, int32_t len);

/* Measurement of the preconditioner's kernels (the cycle's HBM roofline).
 * One application z = M^{-1} v (as ehh_precondition) is run with every kernel
 * launch recorded; then each distinct kernel's launches of that application are
 * replayed, with the same arguments and in their order, from a HIP graph on
 * `stream`, `reps` times, each launch preceded by a write of the caller's
 * eviction buffer (device, evict_bytes, a multiple of 4; NULL and 0 for none)
 * so that it finds the caches as cold as inside a solve; the eviction writes
 * alone are timed the same way and subtracted (HIP events, best of three);
 * the launches are also replayed back to back without the writes; and the
 * whole application's launches are replayed in their order without graphs,
 * each launch timed by start and stop events that its dispatch records itself
 * (hipExtLaunchKernel), so that no launch gap is counted and every launch
 * finds the caches as the preceding launches of the application left them.
 * out[cap] receives one entry per kernel in order of first launch, *count how
 * many were written.  v: (device) as for ehh_precondition; z and the handle's
 * workspaces are overwritten by the replays (z's content afterwards is
 * unspecified).  Synchronises `stream`. */
typedef struct {
    char    kernel[128];    /* kernel name as kernel traces print it, e.g.
                               "k_relax_st2d<double, false, false>" */
    int32_t launches;       /* launches in one preconditioner application */
    double  avg_us;         /* average duration of one launch after the eviction write
                               (its data from HBM) */
    double  avg_us_warm;    /* the same launches replayed back to back without it (their
                               data partly in L2 / MALL, as a small level's inside a solve) */
    double  bytes;          /* algorithmic HBM bytes per launch: every vector entry the
                               kernel must read or write once, the operator's compact
                               coefficients once (mean over its launches) */
    double  bytes_model;    /* the same under the per-cell cycle model: V unknowns per
                               cell of w bytes per source (3 V w for a half-sweep from
                               e_in, 2 V w from zero) plus the level's coefficients per
                               cell (fine 4 reals; Galerkin 29 complex in 2D, 169 in 3D) */
    double  avg_us_seq;     /* average duration of one launch in the in-order replay of
                               the application (the dispatch's own start to end) */
} ehh_kernel_time_t;
int32_t ehh_profile_precondition(ehh_handle_t h, const double* v, double* z, int32_t nrhs, int32_t reps,
                                 void* evict, int64_t evict_bytes, ehh_kernel_time_t* out, int32_t cap,
                                 int32_t* count, void* stream);

/* The coarsest solve of ehh_coarse_solve, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It allocates nothing: the column-segment partial sums
 * of its kernels live in a library-wide device array of 2^22 doubles (32 MiB)
 * per device, which each device that the library runs on holds until the
 * process ends.  Every call rewrites the partial sums it reads, so nothing
 * carries over between calls; calls that overlap in time on one device share
 * that array and race.  The handle's device must be current.  r, e: (device)
 * as for ehh_coarse_solve.  Returns EHH_ERR_UNSUPPORTED (nothing launched)
 * when the coarsest size and nrhs need more partial sums than the array holds
 * (e.g. 3,008 unknowns: up to 32 right-hand sides fit), and for a coarsest
 * level solved by DD (coarse_dd_parts), whose workspaces it cannot allocate. */
int32_t ehh_coarse_solve_noalloc(ehh_handle_t h, int32_t sub, const void* r, void* e,
                                 int32_t nrhs, void* stream);

const char* ehh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EHH_H */
