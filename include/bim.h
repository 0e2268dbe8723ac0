/*
 * bim.h -- C ABI of the MI355X (gfx950) Stokes layer-potential library.
 *
 * Method: C. Sorgentone, A.-K. Tornberg, "A highly accurate boundary integral
 * equation method for surfactant-laden drops in 3D" (arXiv:1707.02156).
 * The library evaluates, for N drops whose surfaces are spherical-harmonic
 * expansions, the interfacial velocity of the second-kind boundary integral
 * equation of Sec. 1:
 *
 *   (lambda_i + 1) u(x0) = 2 u_inf(x0) - 1/(4 pi) sum_j int_{gamma_j} f . G ds
 *                          + sum_j (lambda_j - 1)/(4 pi) int_{gamma_j} u . T . n ds
 *
 * with G = I/r + xh xh/r^3, T = -6 xh xh xh / r^5, xh = x0 - x, solved in the
 * Galerkin form of Sec. 1.2 (unknowns: spherical-harmonic coefficients of u).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Degree-q grid (Sec. 2.1): q+1 Gauss-Legendre latitudes, theta ascending
 *   (index j = 0..q), times 2q longitudes phi_k = pi k / q (k = 0..2q-1);
 *   N(q) = 2q(q+1) nodes, flat index j*2q + k.
 * Basis (Sec. 1.1, Appendix A): Y_n^m = Ptilde_n^m(cos theta) e^{i m phi},
 *   orthonormal, Condon-Shortley phase.
 * Real scalar field of degree p: the m >= 0 coefficients f_n^m as interleaved
 *   (re, im) doubles at complex index n(n+1)/2 + m, i.e. (p+1)(p+2) doubles;
 *   f_n^{-m} = (-1)^m conj(f_n^m) is implied (Sec. 1.2). Im f_n^0 and
 *   Im f_p^p must be zero (the latter is not representable on the grid).
 * Multi-drop vector arrays are component-major:
 *   coef[c][drop][(p_d+1)(p_d+2)]   and   grid[c][drop][N(p_d)],
 *   c = 0,1,2 (x, y, z); drops in the order given to bim_set_drops.
 *
 * Ownership: the caller owns every pointer it passes; the library copies
 * inputs into context-owned device memory and writes outputs into the
 * caller's buffers. mem_kind 0 = host pointer, 1 = device pointer (HIP
 * device memory on the context's device). Device outputs are written
 * asynchronously on the context stream; host outputs are complete on return.
 *
 * Errors: every function returns a status (0 = BIM_OK, < 0 = error). No C++
 * exception or abort crosses the ABI. bim_last_error() gives a per-context
 * message. A context is not thread-safe; use one per thread or stream.
 */
#ifndef BIM_H
#define BIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BIM_OK = 0,
    BIM_EINVAL = -1,   /* invalid argument or input (p out of range, NaN, lambda < 0, empty drop) */
    BIM_ENOMEM = -2,   /* device or host allocation failed */
    BIM_EDEVICE = -3,  /* HIP runtime error */
    BIM_ENOCONV = -4,  /* GMRES did not reach the tolerance; output holds the last iterate */
    BIM_ESTATE = -5,   /* call out of order (e.g. evaluation before bim_set_drops) */
    BIM_EAGAIN = -6,   /* server request not finished within the wait time */
    BIM_EBUSY = -7     /* server queue full: the request was refused (max_queue) */
};

enum { BIM_MEM_HOST = 0, BIM_MEM_DEVICE = 1 };

enum { BIM_EOS_UNIFORM = 0, BIM_EOS_LINEAR = 1, BIM_EOS_LANGMUIR = 2 };

enum { BIM_PREC_FP64 = 0, BIM_PREC_MIXED = 1 };

typedef struct bim_ctx_s *bim_ctx;

typedef struct {
    int device;          /* HIP device ordinal */
    int precision;       /* BIM_PREC_FP64: every step in FP64.
                            BIM_PREC_MIXED: the direct pair sums (regular rule on the standard and
                            upsampled grids of the other drops, Sec. 2.1, 2.3) in FP32 arithmetic,
                            coordinates taken relative to the source drop's centre, runs of 16
                            sources summed in FP32 and accumulated in FP64; the fast summation
                            keeps its stored source harmonics in FP32 (multipoles accumulated in
                            FP64); on the matrix-core transform path (xform_path) the density
                            synthesis of the double-layer operator and the analyses of the
                            operator output and right-hand side take FP32 operands with FP32
                            accumulation (Sec. 1.1, 2.1); the singular self-integrals, the single
                            layer's force density, nearest-region quadrature and GMRES stay in
                            FP64 (relative error of the velocity about 1e-6) */
    double A_tilde;      /* Omega_1 threshold in units of h (Sec. 2.3; paper uses 5) */
    int U_tilde;         /* Omega_1 grid degree factor: sources on the degree U_tilde*p grid */
    int U_sing;          /* singular rule grid degree factor (q = U_sing*p; 1 = paper) */
    int U_geom;          /* de-aliasing grid factor for curvature and force (Sec. 1.3) */
    int lambda_rule;     /* 0: double layer of drop j weighted by lambda_j (source);
                            1: weighted by lambda_i of the target drop (as printed) */
    double gmres_tol;    /* relative residual tolerance (Euclidean norm of coefficients) */
    int gmres_restart;   /* Krylov dimension before restart */
    int gmres_maxit;     /* total iteration cap */
    int singular_path;   /* singular self-integral (Sec. 2.2):
                            0: batched pipeline over all targets of a drop (Legendre stages on the
                               matrix cores); the drop's double layer on itself is stored as a matrix
                               (N(p) x 6 x (p+1)(p+2) doubles per drop) when a double layer is applied;
                            1: rotation and quadrature on every application (no matrix);
                            2: one fused workgroup per target (stored matrix as in 0) */
    void *stream;        /* hipStream_t to run on; NULL = the context creates its own */
    int near_rule;       /* targets in Omega_2 (nearest node of another drop within h, Sec. 2.3):
                            0: the Omega_1 rule (upsampled regular quadrature);
                            1: the special quadrature of Sec. 2.3 (closest point by damped Newton,
                               on-surface value from the source drop's self-interaction expansion,
                               exterior limit for the double layer, regular values at
                               x* + h sqrt(l) d, l = 1..near_L, Lagrange interpolation) */
    int near_L;          /* interpolation points of the special quadrature, 2..16 (paper: 8) */
    int fmm_order;       /* fast summation of far drop pairs (the O(N^2) pair sums of Sec. 2.1 and
                            2.3, which the paper proposes to replace by fast summation, Sec. 6):
                            0 = off (every pair summed directly); -1 = order chosen by timing at
                            the first velocity evaluation after bim_set_drops (0, 8, 12, 16, 20, 24
                            or 30: for a given fmm_eps only the cost depends on the order);
                            P in 2..30 = multipole order of a
                            drop-level fast multipole method on four harmonic potentials (Laplace
                            multipoles of each source drop, translated to local expansions of each
                            target drop, evaluated at its nodes). A drop pair (i, j) takes it when
                            all targets of i are in the same region of j (0 or 1, no Omega_2) and
                            rho^(P+1) <= fmm_eps, rho = (a_i + a_j) / |c_i - c_j| (bounding radii
                            and centres of i's nodes and of j's source grid); the others are
                            summed directly */
    double fmm_eps;      /* truncation bound of a far pair, in (0, 1) */
    int pair_tune;       /* 1: the work-item shape of the direct pair sums (targets per lane 1, 2
                            or 4; sources per item) is chosen by timing a double-layer pair pass
                            of each candidate at the first evaluation after bim_set_drops, and
                            kept for later contexts of the same problem shape (same number of
                            pairs to two digits, targets, fast-summation order) in the process;
                            0: a rule from the pair count. Only the speed depends on it */
    int xform_path;      /* spherical-harmonic transforms of value fields inside the velocity
                            evaluation (density values on the nodes, Galerkin analysis; Sec. 1.1,
                            2.1): 1: scalar FMA kernels (FP64); 2: Legendre and Fourier sums as
                            16x16x4 matrix-core contractions (FP64, or FP32 in the mixed form);
                            0: whichever of the two is faster, timed once per problem shape and
                            precision at first use and kept for the process. Derivative fields
                            and degrees above 63 (analysis grids above 63) take the scalar
                            kernels */
    double pipe_budget_gb; /* device memory for the intermediates of the batched singular pipeline
                            (singular_path 0), GB: the (drop, latitude) units of a degree group
                            run in chunks that fit it (about 80 MB per latitude at p = 48, 24 MB
                            at p = 32); larger chunks mean fewer, fuller launches. Default 8 */
} bim_options;

typedef struct {
    int gmres_iterations;     /* Arnoldi steps performed (0 if all lambda = 1) */
    double gmres_residual;    /* final relative residual */
    int n_targets;            /* grid targets over all drops */
    int n_omega1;             /* (target, source drop) pairs in Omega_1 */
    int n_omega2;             /* pairs in Omega_2 (near_rule selects their quadrature) */
    int n_matvec;             /* operator applications in the solve */
    double ms_total;          /* wall time of the call */
    int n_fmm_pairs;          /* drop pairs taken by the fast summation (fmm_order != 0) */
    int fmm_order;            /* multipole order in use (0: every pair summed directly) */
    int pair_targets_per_lane;  /* work-item shape of the direct pair sums in use: targets per lane */
    int pair_sources_per_item;  /* and sources per item (0: from the pair count) */
    int xform_matrix_cores;     /* transforms on the matrix cores: bit 0 synthesis, bit 1 analysis */
} bim_report;

/* Library version (major*10000 + minor*100 + patch). */
int bim_version(void);
/* Static string for a status code. */
const char *bim_status_string(int status);
/* Fill defaults: A_tilde 5, U_tilde 4, U_sing 1, U_geom 2, lambda_rule 0,
 * gmres_tol 1e-10, restart 50, maxit 500, singular_path 0, device 0, FP64,
 * stream NULL, near_rule 1, near_L 8, fmm_order 0 (off), fmm_eps 1e-10, pair_tune 1,
 * xform_path 0, pipe_budget_gb 8. */
int bim_default_options(bim_options *opt);

/* Create a context on opt->device. Allocates nothing large until drops are set. */
int bim_create(const bim_options *opt, bim_ctx *out);
int bim_destroy(bim_ctx ctx);
const char *bim_last_error(bim_ctx ctx);

/* Drop surfaces x(theta, phi) = sum x_n^m Y_n^m (Sec. 1.1, eq. of the surface
 * expansion). p[d] in [2, 64]; xcoef component-major as in the header;
 * lambda[d] >= 0 is the viscosity ratio of drop d. Builds or reuses the
 * per-degree tables (Gauss-Legendre grid, Legendre functions, Wigner-d
 * rotations of Appendix B). Resets the surfactant to uniform tension 1. */
int bim_set_drops(bim_ctx ctx, int n_drops, const int *p, const double *xcoef,
                  const double *lambda, int mem_kind);

/* Surface tension from the surfactant concentration Gamma (Sec. 1, equation
 * of state): eos UNIFORM sigma = sigma0 (gamma_coef may be NULL);
 * LINEAR sigma = 1 - E xs Gamma; LANGMUIR sigma = 1 + E ln(1 - xs Gamma).
 * gamma_coef: one scalar field per drop, [drop][(p+1)(p+2)]. */
int bim_set_tension(bim_ctx ctx, const double *gamma_coef, int eos, double E, double xs,
                    double sigma0, int mem_kind);

/* Independent systems in one context (batched evaluation): system_of_drop[d]
 * >= 0 for each drop set by bim_set_drops (which resets all to 0). Drops of
 * different systems do not interact (no pair sums; bim_regions reports -2);
 * bim_eval_velocity solves all systems in one GMRES with the tolerance scaled
 * by min_s ||b_s|| / ||b||, so that every system's own relative residual is at
 * most gmres_tol; the report's gmres_residual is that per-system bound. */
int bim_set_systems(bim_ctx ctx, const int *system_of_drop);

/* Far field u_inf(x) = U0 + gradU x (gradU row-major 3x3). */
int bim_set_farfield(bim_ctx ctx, const double U0[3], const double gradU[9]);

/* Interfacial force f = 2 sigma K n - grad_gamma sigma (Sec. 1), computed on
 * the degree U_geom*p grid and analysed to degree p (Sec. 1.3). Output:
 * coefficients, component-major. */
int bim_force(bim_ctx ctx, double *f_coef, int mem_kind);

/* Region of every grid target w.r.t. every drop (Sec. 2.3): -1 own drop,
 * -2 drop of another system (bim_set_systems),
 * 0 Omega_0 (dist > A_tilde h_j), 1 Omega_1 (h_j < dist <= A_tilde h_j),
 * 2 Omega_2 (dist <= h_j); dist = distance to the nearest node of drop j's
 * degree-p grid, h_j = R_j pi/(p_j+1), R_j the volume-equivalent radius.
 * regions: int8 [target][drop]; dist (may be NULL): double [target][drop]
 * (own-drop entries are 0). Targets are numbered over all drops in order.
 * Requesting dist computes every nearest-node distance; without it, pairs
 * whose region a bounding-sphere bound already fixes skip the node scan. */
int bim_regions(bim_ctx ctx, int8_t *regions, double *dist, int mem_kind);

/* Single-layer velocity at every grid target:
 *   out(x0) = -1/(8 pi) sum_j int_{gamma_j} f . G ds
 * (the velocity for lambda = 1 and u_inf = 0). The self term uses the
 * rotated-pole singular rule (Sec. 2.2, Theorem 1, Appendix B); other drops
 * use the regular rule on the standard or upsampled grid by region (Sec. 2.1,
 * 2.3). f_coef = NULL uses the interfacial force. out: grid, component-major. */
int bim_single_layer(bim_ctx ctx, const double *f_coef, double *out, int mem_kind);

/* Double layer of a velocity given by coefficients u_coef (component-major):
 * mode 0: out = grid values of 1/(4 pi) sum_j int_{gamma_j} u . T . n ds (unweighted);
 * mode 1: out = coefficients of the Galerkin second-kind operator
 *         (lambda_i + 1) u_i - P_i[ sum_j (lambda_j - 1)/(4 pi) D_j[u] ],
 *         P_i the analysis of Sec. 2.1 on drop i's grid. */
int bim_apply_double_layer(bim_ctx ctx, const double *u_coef, double *out, int mode, int mem_kind);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operator as bim_apply_double_layer (modes 0 and 1) with nothing allocated.
 * u_coef and out are device pointers (HIP device memory on the context's
 * device), written/read on the context stream. The pair partial sums use a
 * static device array of 256 MiB (one per GPU, held until the process ends);
 * every other buffer is the context's own, so the context must have applied
 * bim_apply_double_layer in the same mode to the same drops first (regions,
 * work lists, stored singular rows and buffers built). Errors: BIM_ESTATE when
 * that preparation is missing, kernel timing is on, or a step would need to
 * allocate; BIM_ENOMEM when the partial sums need more than the 256 MiB (the
 * message gives the size); BIM_EDEVICE when the array's device address is
 * unavailable. Calls that overlap on one GPU (other contexts or threads)
 * share the array and race; the array keeps the last call's contents and
 * needs no clearing (every slot read in a call is written in it). */
int bim_apply_double_layer_noalloc(bim_ctx ctx, const double *u_coef, double *out, int mode);

/* Full velocity: right-hand side 2 u_inf - (1/4pi) sum_j S_j[f], Galerkin
 * projection and GMRES solve of the second-kind equation when any lambda != 1.
 * out_kind bit 0: 0 = grid values, 1 = coefficients; bit 1: 0 = host, 1 = device.
 * rep may be NULL. Returns BIM_ENOCONV (with the last iterate written) if GMRES
 * stops at gmres_maxit above the tolerance. */
int bim_eval_velocity(bim_ctx ctx, double *u_out, int out_kind, bim_report *rep);

/* One coupled step of the drops and their insoluble surfactant (Sec. 3,
 * Algorithm 1): explicit midpoint rule for the drop coefficients and the
 * second-order IMEX scheme of Sec. 3.2 for the surfactant coefficients set by
 * bim_set_tension (without them only the drops move):
 *   u0 = velocity(t); x_h = x + dt/2 u0;
 *   (I - dt/(2 Pe) L) Gamma_h = Gamma + dt/2 fE(x, u0, Gamma) by GMRES with the
 *   sphere's diagonal 1 + dt/(2 Pe) n(n+1)/R^2 as right preconditioner
 *   (R the drop's volume-equivalent radius at x_h, Sec. 3.2.1);
 *   u_h = velocity(t + dt/2); x' = x + dt u_h;
 *   Gamma' = Gamma + dt (fE(x_h, u_h, Gamma_h) + L Gamma_h / Pe),
 * with L the Laplace-Beltrami operator and fE = -Gamma div_s u (the rate at
 * nodes that move with the velocity; it conserves surfactant mass), both
 * evaluated on the degree U_geom p grid and projected to degree p.
 * Error estimates: drop = ||x'_midpoint - x'_Euler|| / ||x'|| (2-norm of all
 * position coefficients); surfactant = max over drops of the relative change
 * of int Gamma dS (conservation error). The step is accepted when
 * max(err) < tol, or always when tol <= 0; the context then holds the new
 * state, otherwise it keeps the state at t. dt_next = dt (0.9 tol/err)^(1/2)
 * (dt when tol <= 0 or err = 0). Pe > 0; Pe = +infinity switches diffusion
 * off. Errors: BIM_EINVAL (dt <= 0 or not finite, Pe <= 0 or NaN, tol not
 * finite), BIM_ESTATE (no drops), BIM_ENOCONV (a GMRES solve did not
 * converge; the state at t is kept). rep may be NULL. */
typedef struct {
    double dt_next;
    double err_drop;
    double err_surf;
    double mass0, mass1;   /* total surfactant over all drops at t and at t + dt */
    int accepted;
    int gmres_velocity[2]; /* GMRES iterations of the velocity solves at t and t + dt/2 */
    int gmres_imex;        /* GMRES iterations of the IMEX stage solve (0 without diffusion) */
    double ms_total;
} bim_step_report;
int bim_time_step(bim_ctx ctx, double dt, double Pe, double tol, bim_step_report *rep);

/* Current drop coefficients ([3][sum (p+1)(p+2)], component-major) and
 * surfactant coefficients ([sum (p+1)(p+2)]); either pointer may be NULL.
 * BIM_ESTATE when gamma_coef is requested and no surfactant was set. */
int bim_get_state(bim_ctx ctx, double *xcoef, double *gamma_coef, int mem_kind);

/* Angle reparametrization of every drop (Sec. 4, Algorithm 2). The surface
 * keeps its expansion (zero-padded to degree q = U_rep p); only the parameter
 * angles of the degree-q grid nodes move: each pseudo-time step solves, per
 * node, [x_t.x_t x_t.x_p; x_t.x_p x_p.x_p] alpha = (w.x_t, w.x_p) with
 * w = -(I - n n) grad E and grad E = sum_{n >= n_cut} x~_n^m Y_n^m (perfect
 * low-pass filter, x~ the current coefficients, n_cut the smallest l >= 2
 * whose coefficient-magnitude tail sum_{n>=l} sum_m |x~_n^m| is below P_cut
 * times that of l = 1), then (theta, phi) += dtau alpha. It stops when the
 * largest |g| = |(I - n n) grad E| over the nodes is below eps or after
 * imax - 1 steps; each drop stops on its own residual (the drops of one
 * degree run as one batch on the device). The drop coefficients, and the surfactant coefficients when
 * set, become the analysis of the initial expansions at the final angles,
 * truncated to degree p (the surfactant stays the same function of the
 * surface points). The paper's values are U_rep = 2, dtau = 1, imax = 30.
 * Errors: BIM_EINVAL (U_rep < 1, U_rep p > 64, P_cut outside (0, 1], eps
 * < 0 or not finite, imax < 1, dtau <= 0 or not finite), BIM_ESTATE (no
 * drops). rep may be NULL. */
typedef struct {
    int moves;      /* pseudo-time steps taken (largest over the drops) */
    int ncut_min;   /* smallest final n_cut over the drops */
    double gnorm;   /* largest final max |g| over the drops */
    double ms_total;
} bim_rep_report;
int bim_reparametrize(bim_ctx ctx, int U_rep, double P_cut, double eps, int imax, double dtau, bim_rep_report *rep);

/* Stand-alone transforms on the context's device and stream (Sec. 1.1, 2.1).
 * Synthesis: nf scalar fields of degree p (each (p+1)(p+2) doubles,
 * consecutive) to grid values on the degree-q grid (q >= p), derivative
 * orders (dt, dp) in theta and phi, dt + dp <= 2; grid [field][N(q)].
 * Analysis: nf grid fields on the degree-q grid to coefficients of degree
 * p <= q. Pointers are device pointers when mem_kind = 1. Value fields with
 * p <= 63 (analysis: q <= 63) run on the matrix cores, with FP32 operands and
 * accumulation in a mixed-precision context; the rest on the scalar FP64
 * kernels. */
int bim_sh_synthesize(bim_ctx ctx, int p, int q, int nf, const double *coef, int dt, int dp,
                      double *grid, int mem_kind);
int bim_sh_analyze(bim_ctx ctx, int q, int p, int nf, const double *grid, double *coef, int mem_kind);

/* Block until all work queued by the context is complete. */
int bim_synchronize(bim_ctx ctx);

/* Kernel timing: HIP events recorded around each launch of the main kernels,
 * on the stream the launch goes to (the context stream; the singular pipeline
 * of a velocity evaluation runs on a second stream of the context). enable = 1 clears the totals and starts recording,
 * 0 stops. Kernel names: "pipe_rotate", "pipe_legendre", "pipe_fourier",
 * "pipe_adjrot" (batched singular pipeline), "sing_fused" (fused singular
 * rule), "sing_rotate" and "sing_v1" (per-application singular path),
 * "dl_apply" (stored double layer times a density), "pair_sl", "pair_dl"
 * (pair sums), "near" (nearest-region interpolation points and
 * interpolation), "synthesis", "analysis", "classify". Each timed launch adds an
 * event pair to the stream, which delays the next launch by a few
 * microseconds; bim_profile_select limits timing to chosen kernels. */
int bim_profile(bim_ctx ctx, int enable);
/* Restricts event timing to the kernels named in a comma-separated list
 * (NULL or "" = all kernels). Launch counts, flops and bytes are still
 * totalled for every kernel. Takes effect at the next bim_profile(ctx, 1). */
int bim_profile_select(bim_ctx ctx, const char *names);
/* Totals since the last enable: launches, summed event time (ms), algorithmic
 * flops and bytes of those launches. Unknown names give zeros. Synchronizes
 * the context's streams. */
int bim_profile_query(bim_ctx ctx, const char *name, int *launches, double *ms, double *flops, double *bytes);

/* ------------------------------------------------------------------------
 * Request server: independent drop systems (each a full velocity
 * evaluation, bim_eval_velocity) submitted at any time and run concurrently.
 * The server holds `slots` contexts, each with its own HIP stream (default
 * priority) and host worker thread; the per-degree tables of a context and
 * its device buffers stay resident between requests (buffers grow to the
 * largest request a slot has served and are not freed until the server is
 * destroyed; the admission budget counts each running request's estimate). A queued request is admitted, first come first
 * served, when a slot is free and its estimated device memory
 * (bim_server_footprint) fits in hbm_budget_gb next to the running requests;
 * the device work of admitted requests overlaps (three slots by default: on
 * the serving stream of 1-8 drops of degree 8-32 they keep the median latency
 * of four and a lower tail, since a large request shares the device with
 * fewer others). With max_batch > 1 a free
 * slot also takes further queued requests of the same tension parameters and
 * solves them together as independent systems (bim_set_systems): each
 * result then meets gmres_tol on its own but differs from the result of the
 * request alone at that level.
 * ---------------------------------------------------------------------- */
typedef struct bim_server_s *bim_server;

typedef struct {
    int slots;              /* concurrent batches, 1..64 (default 3) */
    double hbm_budget_gb;   /* admission budget, GB of estimated device memory (default 64) */
    bim_options opt;        /* options of every context; opt.stream must be NULL */
    int max_batch;          /* requests a free slot takes from the queue at once, run as independent
                               systems of one context (bim_set_systems); 1 = one at a time (default) */
    int max_batch_drops;    /* drops per batch at most (default 128) */
    int max_queue;          /* requests waiting for a slot at most; a submit beyond it is refused
                               with BIM_EBUSY, so an overloaded server sheds load at the door
                               instead of growing its queue without bound (0 = no limit, the
                               default) */
} bim_server_options;

/* Defaults: 3 slots, 64 GB, max_batch 1, max_batch_drops 128, max_queue 0, opt from
 * bim_default_options with pair_tune 0 and xform_path 1 (no timing of work
 * shapes on the request path) and pipe_budget_gb 0.75. */
int bim_server_default_options(bim_server_options *opt);
int bim_server_create(const bim_server_options *opt, bim_server *out);
/* Finishes the running requests, drops the queued ones, frees everything. */
int bim_server_destroy(bim_server srv);
/* Queue one system: drops, surface coefficients, viscosity ratios and
 * surfactant as for bim_set_drops / bim_set_tension (host pointers, copied
 * before return; gamma_coef may be NULL for eos UNIFORM). out_kind 0: grid
 * velocity, 1: coefficients (as bim_eval_velocity, host). *id names the
 * request in bim_server_wait. */
int bim_server_submit(bim_server srv, int n_drops, const int *p, const double *xcoef, const double *lambda,
                      const double *gamma_coef, int eos, double E, double xs, double sigma0, int out_kind,
                      uint64_t *id);
/* Wait up to timeout_s seconds (< 0: no limit, 0: poll) for request id.
 * Done: copies the velocity to out (may be NULL; size as bim_eval_velocity),
 * the report to rep (may be NULL) and, if times_ms is not NULL, the queueing,
 * service and total times in ms; releases the request and returns its status
 * (BIM_OK, BIM_ENOCONV, ...). Not done: BIM_EAGAIN. Unknown id: BIM_EINVAL. */
int bim_server_wait(bim_server srv, uint64_t id, double timeout_s, double *out, bim_report *rep,
                    double *times_ms);
/* Estimated device memory in bytes of one request with these degrees. */
int bim_server_footprint(const bim_options *opt, int n_drops, const int *p, double *bytes);

/* Host-side tables (no device needed; the same routines build the device
 * tables). Gauss-Legendre nodes t[0..q] (descending, theta ascending) and
 * weights of the degree-q grid (Sec. 2.1). */
int bim_host_gauss_legendre(int q, double *t, double *w);
/* Ptilde_n^m(t) and its first and second theta-derivatives at -1 < t < 1 for
 * 0 <= m <= n <= nmax, at index n(n+1)/2 + m (Sec. 1.1, Appendix A). D1 and D2
 * may be NULL. */
int bim_host_legendre(int nmax, double t, double *P, double *D1, double *D2);
/* Wigner small-d matrix of degree n at angle beta (Appendix B):
 * d[(m'+n)(2n+1) + (m+n)] = d^n_{m'm}(beta), -n <= m', m <= n. */
int bim_host_wigner_d(int n, double beta, double *d);

#ifdef __cplusplus
}
#endif

#endif /* BIM_H */
