/*
 * eigenwave.h -- C ABI of the MI355X (gfx950) WaveHoltz-filter eigensolver.
 *
 * The library computes eigenpairs of the Dirichlet Laplacian on boxes near a
 * target frequency omega with the EigenWave method: the WaveHoltz operator S
 * (one wave-solve over N_p periods plus a trapezoidal time filter) is applied
 * once per Arnoldi step, and the eigenvalues of L_h are recovered from the
 * eigenvectors of S by a Rayleigh quotient stage.
 *
 * Conventions shared by every entry point
 *   - Every call returns ew_status: 0 on success, a negative code otherwise;
 *     ew_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses the ABI.  On error the contents of output
 *     buffers are unspecified.
 *   - Vectors hold the active (interior) grid points only, as FP64,
 *     lexicographic with x fastest (the paper's matrix-vector routine,
 *     Alg. "WaveHoltz matrix-vector product"; boundary points are constraint
 *     equations and never enter the vectors).  A grid with n[d] interior
 *     points per dimension has n_active = prod n[d] entries.
 *   - "_dev" pointers are device (HBM) addresses on the device that was
 *     current when the object was created; "_host" pointers are host memory.
 *     The caller owns every buffer it passes; the library owns its workspace,
 *     allocated by *_create and released by *_destroy.
 *   - Device work is ordered on the hip stream given at creation (a
 *     hipStream_t passed as void*; NULL = the null stream).  Calls marked
 *     "stream-ordered" return before the device work finishes; calls marked
 *     "host-blocking" synchronise the stream before returning.
 *   - Objects are not thread-safe: one host thread at a time per object.
 */
#ifndef EIGENWAVE_H
#define EIGENWAVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EW_OK = 0,
    EW_ERR_INVALID_ARG = -1,       /* an argument violates the documented range */
    EW_ERR_OOM = -2,               /* device or host allocation failed */
    EW_ERR_HIP = -3,               /* a HIP runtime call failed */
    EW_ERR_MG_NOT_CONVERGED = -4,  /* multigrid hit mg_max_cycles before mg_tol */
    EW_ERR_NONFINITE = -5,         /* a NaN or Inf appeared in a norm */
    EW_ERR_NOT_CONVERGED = -6,     /* eigensolver hit max_wave_solves */
    EW_ERR_UNSUPPORTED = -7        /* valid but not implemented combination */
} ew_status;

enum { EW_TS_EXPLICIT = 0, EW_TS_IMPLICIT = 1 };
enum { EW_FILTER_ALPHA_D = 0, EW_FILTER_QUARTER = 1 };
enum { EW_PREC_FP64 = 0, EW_PREC_MIXED = 1 };
enum { EW_PRED_ZERO = 0, EW_PRED_SCALED = 1, EW_PRED_CNN = 2, EW_PRED_EXTRAP = 3, EW_PRED_PROJ = 4 };

typedef struct ew_op_s* ew_op;

/* Grid: a box [0,len_0] x [0,len_1] (x [0,len_2]) with n[d] active points per
 * dimension.  dim in {2,3}; 1 <= n[d] <= 65535 for d < dim (entries beyond dim
 * are ignored); order in {2,4}: the 2nd-order (5/7-point) or 4th-order
 * (width-5 cross) Laplacian L_h of eq. eigBVPdiscrete.
 *
 * walls[d][0] (x_d = 0) and walls[d][1] (x_d = len_d) are EW_WALL_DIRICHLET
 * (0, the default) or EW_WALL_NEUMANN (the boundary operator of Sec. "Problem
 * specification and the EigenWave algorithm" may be either).  A Dirichlet
 * wall is not an active point: value 0, and order 4 closes the stencil by odd
 * reflection (u_{-1} = -u_{1}), the form the paper's compatibility conditions
 * take for a flat wall (Sec. "Discrete approximations").  A Neumann wall point
 * is active, and ghosts mirror the interior evenly about it (u_{-k} = u_{k}).
 * Spacing h_d = len_d / (n_d + 1 - number of Neumann walls of dimension d);
 * an axis with a Neumann wall needs n_d >= 3.  With Neumann walls L_h is
 * self-adjoint in the inner product weighted by 1/2 per Neumann wall a point
 * lies on; ew_eigs works in those weighted coordinates and returns the grid
 * functions.  Multigrid coarsening keeps the wall points (n = 2 n_c + 1,
 * 2 n_c or 2 n_c - 1 for zero, one or two Neumann walls of an axis); boxes
 * with Neumann walls run the tiled multigrid kernels on every level (not the
 * single-workgroup coarse kernel), and the implicit guesses PROJ and CNN are
 * not available there (EW_ERR_UNSUPPORTED). */
enum { EW_WALL_DIRICHLET = 0, EW_WALL_NEUMANN = 1 };
typedef struct {
    int dim;
    int64_t n[3];
    double len[3];
    int order;
    int walls[3][2];
} ew_grid_desc;

/* Operator: one wave-solve plus time filter, S v (eqs. explicitScheme or
 * implicitScheme, and filterQuadrature).
 *   omega > 0          target frequency; T_f = n_p * 2 pi / omega.
 *   ts                 EW_TS_EXPLICIT: leapfrog, dt from cfl (0 < cfl <= 1) with
 *                      dt_max = 2/sqrt(rho), rho = sum_d c/h_d^2 (c = 4 for order
 *                      2, 16/3 for order 4), N_t = ceil(T_f/(cfl dt_max));
 *                      EW_TS_IMPLICIT: trapezoidal, N_t = n_p * n_its (n_its >= 5,
 *                      Sec. "Discrete time-stepping analysis").
 *   n_p >= 1           number of periods.
 *   adjust_omega       nonzero: use the adjusted frequency of eq. adjustedOmega
 *                      (implicit only).
 *   filter_const       EW_FILTER_ALPHA_D: cos(omega t) - alpha_d/2 (eq. alphad);
 *                      EW_FILTER_QUARTER: cos(omega t) - 1/4.
 *   precision          EW_PREC_FP64, or EW_PREC_MIXED: FP32 state, stencils,
 *                      smoother and filter accumulation, FP64 multigrid defect
 *                      correction (implicit) and FP64 vectors at the boundary.
 *   mg_tol, mg_nu1, mg_nu2, mg_max_cycles, mg_coarse_sweeps
 *                      implicit only: V(nu1,nu2) cycles of red-black
 *                      Gauss-Seidel multigrid on M = I - (dt^2/2) L_h (eq.
 *                      impMatrix) until ||b - M x||_2 <= mg_tol ||b||_2;
 *                      mg_coarse_sweeps sweeps on a coarsest level of more
 *                      than one point.
 *   mg_coarse_points   largest level (in points) that is handed to the
 *                      single-workgroup kernel that runs all remaining coarser
 *                      levels in LDS; 0 = the largest that fits (<= 8192 points
 *                      and 160 KB of LDS for the arrays of all those levels).
 *                      Results do not depend on it beyond rounding order.
 *   predictor          initial guess of each implicit solve: EW_PRED_ZERO, or
 *                      EW_PRED_SCALED (x0 = b / (1 + a omega^2), exact for
 *                      every mode with lambda = omega since M phi = (1 + a mu) phi), or
 *                      EW_PRED_EXTRAP (linear extrapolation in time,
 *                      W^{n+1} ~ 2 W^n - W^{n-1}, i.e. x0 = b), or
 *                      EW_PRED_PROJ (projection on earlier solves: x0 is the
 *                      combination of the last proj_window solutions x_k
 *                      (M x_k = b_k, kept in FP32 across wave-solves) that is
 *                      closest to the new solution in the M-norm, found from
 *                      the Gram matrix x_i . b_j and the products x_k . b;
 *                      P. F. Fischer's method for successive right-hand
 *                      sides), or EW_PRED_CNN (the PROJ guess, or zero with
 *                      proj_window < 0 or an empty window, corrected at the
 *                      steps n >= 1 by the learned network of ew_cnn_* from
 *                      its residual; 2D FP64 only; needs ew_op_set_cnn, else
 *                      it is that base guess).  Whatever the guess, the
 *                      multigrid iterates to mg_tol, so results agree with
 *                      the zero guess to that tolerance.
 *   proj_window        solves kept for PROJ and CNN: 0 = 24, at most 32,
 *                      negative = none.
 *   mg_max_levels      implicit only: most multigrid levels (the finest
 *                      counts as one); 0 = coarsen while every n_d is odd
 *                      and >= 3.  A truncated hierarchy ends on a level that
 *                      gets mg_coarse_sweeps sweeps, which solve it well when
 *                      (dt^2/2)/h_coarse^2 is small (M is then strongly
 *                      diagonally dominant).  EW_MG_LEVELS_AUTO (-1): stop
 *                      at the first level whose Gauss-Seidel contraction
 *                      bound, rho_J^2 with rho_J the ratio of M's
 *                      off-diagonal row sum to its diagonal (a = dt^2/2:
 *                      2 a S / (1 + 2 a S) for order 2, (34/12) a S /
 *                      (1 + (30/12) a S) for order 4, S = sum_d 1/h_d^2 on
 *                      that level), raised to mg_coarse_sweeps, is <= 0.1.
 *   mg_relax           implicit solves: relaxation weight w of the
 *                      finest level's red-black half-sweeps,
 *                      x_i += w (b - M x)_i / M_ii (w > 1: over-relaxed
 *                      red-black Gauss-Seidel); 0 = the default 1.2; else in
 *                      (0, 2).
 *   mg_relax_coarse    the same weight on every coarser level (a level of one
 *                      point always uses 1, an exact solve); 0 = the default
 *                      1.05; else in (0, 2).  The defaults took the fewest
 *                      V-cycles per solve on the 2D and 3D workloads tried.
 *                      On a mapped grid both weigh the zebra-line (or, on
 *                      lines too long for LDS, point) relaxation,
 *                      x <- x + w (relaxed value - x), and default to 1: the
 *                      best weights depend on the map. */
enum { EW_MG_LEVELS_AUTO = -1 };
typedef struct {
    double omega;
    int ts;
    double cfl;
    int n_its;
    int n_p;
    int adjust_omega;
    int filter_const;
    int precision;
    double mg_tol;
    int mg_nu1;
    int mg_nu2;
    int mg_max_cycles;
    int mg_coarse_sweeps;
    int mg_coarse_points;
    int predictor;
    int proj_window;
    int mg_max_levels;
    double mg_relax;
    double mg_relax_coarse;
} ew_op_desc;

/* Read-only facts about an operator. */
typedef struct {
    int64_t n_active;     /* length of every vector */
    int n_t;              /* time steps per wave-solve */
    double dt;            /* time step */
    double omega_used;    /* frequency used in the filter (adjusted or not) */
    double t_final;       /* T_f */
    double alpha_d;       /* eq. alphad at omega_used * dt */
    int mg_levels;        /* multigrid levels (implicit), else 0 */
    double mg_relax;      /* relaxation weight of the finest level's box smoother in use */
    double mg_relax_coarse; /* ... and of the coarser levels */
} ew_op_info;

/* Cumulative counters of an operator (reset by ew_op_reset_stats). */
typedef struct {
    int64_t wave_solves;      /* applications of S */
    int64_t time_steps;       /* time levels advanced */
    int64_t pt_updates;       /* active points x time levels advanced */
    int64_t mg_solves;        /* implicit solves */
    int64_t mg_cycles;        /* V-cycles over all implicit solves */
    int64_t laplacian_applies;
    int64_t cnn_guesses;      /* initial guesses made by the network */
    int64_t guess_probes;     /* solves measured by ew_op_probe_guesses */
    double base_rel_res_sum;  /* sum of ||b - M x0||/||b|| of the base guesses measured */
    double guess_rel_res_sum; /* the same for the guesses the multigrid started from */
} ew_op_stats;

/* Create an operator on the current device.  The filter weights c_n, dt and
 * N_t are computed once here in FP64.  Errors: EW_ERR_INVALID_ARG for any
 * violated range above, EW_ERR_OOM, EW_ERR_HIP. */
ew_status ew_op_create(const ew_grid_desc* grid, const ew_op_desc* desc, void* hip_stream, ew_op* out);

/* Create an explicit operator on a single curvilinear grid (the mapping
 * method of Sec. "Discrete approximations": a smooth invertible map x = G(r)
 * of the unit square, the equations written in r by the chain rule).  The
 * paper prints no discrete form; this library uses the order-2 conservative
 * one,
 *   J L_h u = D+r(A11 D-r u) + D+s(A22 D-s u) + D0r(B D0s u) + D0s(B D0r u),
 * J = x_r y_s - x_s y_r, J a^11 = (x_s^2 + y_s^2)/J, J a^22 = (x_r^2 + y_r^2)/J,
 * B = J a^12 = -(x_r x_s + y_r y_s)/J, A11 (A22) at a half point the mean of
 * J a^11 (J a^22) at its two nodes, metric derivatives by centred
 * differences of the coordinates, Dirichlet walls.  L_h is self-adjoint in
 * the J-weighted inner product; ew_eigs works in y = J^{1/2} u and returns
 * grid functions.  The explicit step uses dt_max = 2 / sqrt(rho) with rho the
 * Gershgorin bound max (1/J) sum |weights of J L_h| (ew_op_mapped_rho).  The
 * implicit scheme solves M = I - (dt^2/2) L_h by multigrid whose coarse
 * levels carry the Galerkin product R M P of the level above (bilinear P,
 * full weighting R = P^T/4; every coarse node is a fine node; n halves as
 * (n - 1)/2 while both sizes are odd and >= 3, with mg_max_levels and
 * EW_MG_LEVELS_AUTO as for boxes, the latter judged on each level's
 * operator),
 * zebra line relaxation along the first index (each grid line j of one
 * parity solved exactly with lines j +- 1 held; levels with n[0] > 2816
 * fall back to red-black point Gauss-Seidel, whose corner neighbours enter
 * with their previous values), full weighting and bilinear prolongation;
 * ew_op_mg_solve, ew_op_mg_vcycle and ew_op_mg_half_sweep apply to it.
 *   grid      dim 2, order 2, Dirichlet walls; n[0] x n[1] active points at
 *             r = (i + 1)/(n[0] + 1), s = (j + 1)/(n[1] + 1); len is unused.
 *   desc      explicit or implicit, precision EW_PREC_FP64; implicit guesses
 *             EW_PRED_ZERO, EW_PRED_SCALED or EW_PRED_EXTRAP.
 *   xy_host   host array of 2 (n[0] + 4)(n[1] + 4) doubles: x, then y, of
 *             nodes i in [-2, n[0] + 1], j in [-2, n[1] + 1] (the walls are
 *             i = -1 and i = n[0], plus one layer beyond each) at
 *             (i + 2) + (n[0] + 4)(j + 2).  Read during the call only.
 * Errors: EW_ERR_INVALID_ARG (ranges of ew_op_create, null or non-finite
 * coordinates, a Jacobian that is not positive at some node, walls
 * included), EW_ERR_UNSUPPORTED (3D, order 4, Neumann walls, mixed
 * precision, the PROJ and CNN guesses), EW_ERR_OOM, EW_ERR_HIP.  The
 * network and batched entry points do not apply to such an operator. */
ew_status ew_op_create_mapped(const ew_grid_desc* grid, const ew_op_desc* desc, const double* xy_host,
                              void* hip_stream, ew_op* out);
/* The Gershgorin bound rho of a mapped operator (EW_ERR_INVALID_ARG for any
 * other operator). */
ew_status ew_op_mapped_rho(ew_op op, double* rho_host);
void ew_op_destroy(ew_op op);
ew_status ew_op_get_info(ew_op op, ew_op_info* out);
ew_status ew_op_get_stats(ew_op op, ew_op_stats* out);
ew_status ew_op_reset_stats(ew_op op);
/* Measurement of the initial guesses (implicit FP64 operators): while on,
 * every solve of a step n >= 1 computes ||b - M x0||_2 / ||b||_2 for the base
 * guess of its predictor and for the guess the multigrid starts from (they
 * differ for EW_PRED_CNN with a network attached, where the base is the
 * projection guess) and adds them to ew_op_stats (base_rel_res_sum,
 * guess_rel_res_sum, guess_probes).  It costs a residual pass and a host
 * round trip per measured guess; results do not change.  Host only. */
ew_status ew_op_probe_guesses(ew_op op, int on);

/* out_dev = S v_dev (both n_active FP64, device; may not alias).  This is the
 * paper's matVec (Alg. "WaveHoltz matrix-vector product"): the vector is the
 * initial condition W^0 with zero velocity, W is advanced N_t steps, and
 * out = sum_n c_n W^n with trapezoidal c_n (eq. filterQuadrature).
 * Stream-ordered for explicit; implicit blocks the host once per multigrid
 * cycle to test convergence.  Explicit 2D FP64 operators too large for the
 * single-workgroup wave-solve (about 8192 points) and mapped operators
 * advance several steps per launch and allocate two more time levels (16 B
 * per point, held until ew_op_destroy) at their first call.  EW_ERR_MG_NOT_CONVERGED if a solve fails, EW_ERR_OOM if that
 * allocation does. */
ew_status ew_op_apply_filter(ew_op op, const double* v_dev, double* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): out_dev =
 * S v_dev as ew_op_apply_filter computes it for an explicit operator created
 * from the same descriptors, with no operator object.  The time plan (dt,
 * N_t, the weights c_n) is computed on the host for each call; the time levels
 * live in a device array of 2^23 doubles (64 MiB) that the library holds on
 * each GPU it runs on until the process ends, its address resolved on the
 * first call on that GPU.  The call makes no device or pinned-host
 * allocation, creates no event and does not synchronise: it is stream-ordered
 * on hip_stream (NULL = the null stream) of the current device.
 *   grid, desc  as for ew_op_create, with desc->ts = EW_TS_EXPLICIT and
 *               precision EW_PREC_FP64 or EW_PREC_MIXED; at most 2^22 active
 *               points (2047^2 fits).
 *   v_dev, out_dev  n_active FP64 device vectors (may not alias); read and
 *               written only by the stream-ordered work.
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on one GPU (other streams, other host threads) race and give undefined
 * results; calls ordered on one stream are safe.  Nothing of an earlier
 * call's contents enters a result (every array is written before it is
 * read).  Small grids take the per-step kernels (ew_op_apply_filter may run
 * them in one workgroup), so results agree with it to rounding.
 * Errors: EW_ERR_INVALID_ARG (the ranges of ew_op_create, null pointers,
 * aliasing, more than 2^22 points), EW_ERR_UNSUPPORTED (implicit stepping),
 * EW_ERR_HIP. */
ew_status ew_apply_filter_noalloc(const ew_grid_desc* grid, const ew_op_desc* desc, const double* v_dev,
                                  double* out_dev, void* hip_stream);

/* out_dev = L_h v_dev (FP64, device; may not alias), the operator of eq.
 * eigBVPdiscrete with the order's closure.  Stream-ordered. */
ew_status ew_op_apply_laplacian(ew_op op, const double* v_dev, double* out_dev);

/* Solve M x = b with M = I - (dt^2/2) L_h of the operator (implicit only) by
 * multigrid from the initial guess in x_dev, to the operator's mg_tol.
 * b_dev, x_dev: n_active FP64 device vectors (may not alias).  cycles_host and
 * rel_res_host (may be NULL) receive the V-cycle count and the final
 * ||b - M x||_2 / ||b||_2.  Host-blocking. */
ew_status ew_op_mg_solve(ew_op op, const double* b_dev, double* x_dev, int* cycles_host, double* rel_res_host);

/* One V-cycle x <- V(x, b) on the finest level (FP64 operators only; for
 * component parity tests).  Stream-ordered. */
ew_status ew_op_mg_vcycle(ew_op op, const double* b_dev, double* x_dev);

/* One half-sweep of the finest level's smoother (FP64 operators only).
 * Boxes: every point whose 0-based index sum has parity `colour` gets
 * x_i += (b - M x)_i / M_ii, all from the values before the half-sweep.
 * Mapped grids with n[0] <= 2816: every line j with j % 2 == colour is
 * replaced by the exact solution of its own equations (M x = b on the line)
 * with the values on lines j +- 1 held; wider mapped grids: the point rule.
 * Stream-ordered. */
ew_status ew_op_mg_half_sweep(ew_op op, const double* b_dev, double* x_dev, int colour);

/* Eigensolver (Alg. "Krylov-Schur" interface of the paper):
 *   k >= 1 wanted pairs (largest |beta|, the paper's "largestAbs"), Krylov
 *   dimension m with k < m <= n_active and m <= 4096, Ritz tolerance tol_ritz
 *   (relative |S y - theta y| / |theta|) and L_h residual tolerance tol_res
 *   (||L y + mu y||_2 / (mu ||y||_2)), wave-solve cap max_wave_solves.
 *   The start vector is v0_dev if non-NULL, else SplitMix64 uniform[-1,1) of
 *   stream `seed`; deflation probes (fresh starts that find further copies of
 *   repeated eigenvalues) use streams seed+1, seed+2, ...  n_keep (0 = default
 *   max(k, (m+k)/2)) Ritz vectors are kept at each restart. */
typedef struct {
    int k;
    int m;
    double tol_ritz;
    double tol_res;
    int64_t max_wave_solves;
    uint64_t seed;
    const double* v0_dev;
    int n_keep;
    int max_probes;
} ew_eigs_desc;

typedef struct {
    int n_conv;               /* converged pairs found (may exceed k) */
    int n_returned;           /* pairs written (min(n_conv, k_cap)) */
    int64_t wave_solves;
    int64_t restarts;
    int64_t probes;
    int64_t time_steps;
    int64_t pt_updates;
    int64_t mg_cycles;
    double seconds;           /* wall time of the call */
    double max_res;           /* largest L_h residual among returned pairs */
} ew_eigs_stats;

/* Run the eigensolver.  Outputs (k_cap entries each, first n_returned valid,
 * ordered by |beta| descending): mu_host = lambda_h^2, beta_host = eigenvalue
 * of S, res_host = L_h residual ||L z + mu z|| / (max(mu, 1) ||z||),
 * Y_dev = eigenvectors (n_active x k_cap FP64 column-major on the device,
 * unit 2-norm grid functions, each signed so that its entry of largest
 * magnitude (the first such) is positive; may be NULL).  With Neumann walls
 * (or on a mapped grid) the Krylov vectors, v0_dev and the residuals are in
 * the coordinates y = W^{1/2} u (W = 1/2 per Neumann wall a point lies on;
 * W = J on a mapped grid), where S and L_h are symmetric.
 * Host-blocking.  EW_ERR_NOT_CONVERGED if max_wave_solves is reached first.
 * With the environment variable EW_EIGS_PROGRESS set (to anything but "0"),
 * each convergence test prints one line to stderr (run, basis size,
 * wave-solves, restarts, leading converged Ritz pairs). */
ew_status ew_eigs(ew_op op, const ew_eigs_desc* desc, int k_cap, double* mu_host, double* beta_host,
                  double* res_host, double* Y_dev, ew_eigs_stats* stats);

/* The projected eigenproblem of the Krylov-Schur restart (Alg. "IRAM"; Sec.
 * "Using Arnoldi-based algorithms"): A = Q diag(w) Q^T for a symmetric n x n
 * matrix, the routine ew_eigs uses on its projected matrices.  a_host is
 * row-major n x n (only symmetric input is meaningful; the matrix is read,
 * not modified); w_host receives n eigenvalues (unordered), q_host (n x n,
 * row-major, may be NULL) the orthonormal eigenvectors as columns.  Orders up
 * to 64: cyclic Jacobi; above: Householder tridiagonalisation and implicit
 * QR with Wilkinson shifts.  Host only, no device work.  Errors:
 * EW_ERR_INVALID_ARG (n < 1, n > 8192, NULL a_host or w_host). */
ew_status ew_sym_eig(int n, const double* a_host, double* w_host, double* q_host);

/* Kernel timing inside an operator (the tracing facility).  Between
 * ew_op_profile_begin and ew_op_profile_end, every launch of kernel class
 * `kclass` that the operator issues on multigrid level `level` (any level if
 * level < 0; levels count from 0 = finest) is bracketed by hipEvents recorded
 * on the operator's stream.  bytes_alg accumulates, per launch, the
 * algorithmic bytes of that kernel: every array it must read or write counted
 * once at its storage precision.  At most 65536 launches are timed per
 * session.  ew_op_profile_end is host-blocking. */
enum {
    EW_K_LEAPFROG = 0,  /* explicit step + filter accumulation (a whole wave-solve on small 2D grids) */
    EW_K_SMOOTH = 1,    /* red-black Gauss-Seidel sweep reading the iterate (on 2D levels a
                           launch runs two consecutive sweeps from one pass over x and b) */
    EW_K_RESTRICT = 2,  /* residual + full-weighting restriction */
    EW_K_PROLONG = 3,   /* prolongation + correction (fused with the first post-sweep) */
    EW_K_RESNORM = 4,   /* residual norm (convergence test) */
    EW_K_UPDATE = 5,    /* implicit update + filter accumulation */
    EW_K_COARSE = 6,    /* coarse-level V-cycle in one workgroup */
    EW_K_SMOOTH_ZERO = 7 /* first sweep (2D: first two) from a zero iterate (iterate not read) */
};
typedef struct {
    int64_t launches;
    double total_ms;
    double bytes_alg;
} ew_kernel_profile;
ew_status ew_op_profile_begin(ew_op op, int kclass, int level);
ew_status ew_op_profile_end(ew_op op, ew_kernel_profile* out);

/* Number of filter periods N_p for k wanted eigenpairs (Sec. "Changing the
 * number of filter periods"; Sec. "Estimating the EigenWave convergence
 * rate": the main lobe of the filter narrows like 1/N_p, the estimated
 * convergence rate at the lobe's edge hardly depends on N_p, and the most
 * efficient runs hold about the wanted eigenvalues above beta ~ 0.8).
 * Returns the largest N_p <= np_max for which at least k frequencies of the
 * continuous Dirichlet Laplacian on the box, lambda = pi sqrt(sum_d
 * (m_d / len_d)^2), have continuous filter value beta(lambda; w, N_p) (eq.
 * filterThreeSincs) >= beta_r, and 1 if even N_p = 1 holds fewer.  w is the
 * frequency the operator's filter uses for desc (adjusted with desc->n_its
 * when desc->adjust_omega; desc->n_p is ignored).  n_lobe_out receives the
 * count for the returned N_p.  Outputs may be NULL.  Host only, no device
 * work.  Errors: EW_ERR_INVALID_ARG (dim, lengths, omega, k < 1, beta_r
 * outside [0.5, 1), np_max outside [1, 4096], more than 5e7 modes);
 * EW_ERR_UNSUPPORTED for Neumann walls (the rule counts Dirichlet modes). */
ew_status ew_choose_periods(const ew_grid_desc* grid, const ew_op_desc* desc, int k, double beta_r, int np_max,
                            int* n_p_out, int* n_lobe_out);

/* ------------------------------------------------------------------------
 * Batched form: many independent 2D Dirichlet rectangles, explicit leapfrog,
 * FP64 vectors and Arnoldi.  The time levels and the filter accumulation are
 * FP32 (precision EW_PREC_MIXED) or FP64 (EW_PREC_FP64), one precision and
 * one stencil order for all problems.  With FP32 state, problems with
 * nx, ny <= 128 run their whole wave-solve inside one workgroup and larger
 * ones advance one time step per batched launch, whose tile height is chosen
 * at creation by timing the candidates on the batch (ew_batch_info.tune_us);
 * with FP64 state every problem advances 8 steps (order 2) or 4 (order 4)
 * per batched launch, in tiles that overlap by the steps' reach.  One batched
 * wave-solve is a captured hipGraph (a graph of ordinary launches, not a
 * persistent kernel) replayed on a private stream and joined to the caller's
 * stream with events.
 * ------------------------------------------------------------------------ */
typedef struct ew_batch_s* ew_batch;

typedef struct {
    int nprob;
    int n_small;                 /* problems solved inside one workgroup */
    int n_large;                 /* problems advanced by the batched step kernel */
    int max_steps_large;         /* longest N_t among the batched-launch problems */
    int step_rows_per_thread;    /* FP32 state: tile height chosen by the autotuner (rows = 4 x this); FP64: 0 */
    double tune_us[4];           /* FP32 state: time per step launch for 1, 2, 4, 8 rows per thread; FP64: 0 */
    int64_t total_steps;         /* sum of N_t over the problems */
    int64_t pt_updates_per_wave_solve;
    int state_fp64;              /* 1: FP64 time levels and accumulation; 0: FP32 */
    int steps_per_launch;        /* time steps per batched launch: 1 with FP32 state, 8 / (order / 2) with FP64 */
} ew_batch_info;

/* grids[i], descs[i] describe problem i (same rules as ew_op_create, plus:
 * dim 2, Dirichlet walls, ts EW_TS_EXPLICIT, precision EW_PREC_MIXED or
 * EW_PREC_FP64, one order and one precision for all; EW_ERR_UNSUPPORTED or
 * EW_ERR_INVALID_ARG otherwise).
 * Allocates every problem's workspace, autotunes and captures the graph.
 * Host-blocking. */
ew_status ew_batch_create(int nprob, const ew_grid_desc* grids, const ew_op_desc* descs, void* hip_stream,
                          ew_batch* out);
void ew_batch_destroy(ew_batch b);
ew_status ew_batch_get_info(ew_batch b, ew_batch_info* out);
/* n_active and N_t of problem i (either output may be NULL). */
ew_status ew_batch_n_active(ew_batch b, int i, int64_t* n_active, int* n_t);
/* out_dev[i] = S_i v_dev[i] for every problem (host arrays of nprob device
 * pointers to n_active_i FP64 values; out may not alias v).  Stream-ordered
 * on the stream given at creation. */
ew_status ew_batch_apply_filter(ew_batch b, const double* const* v_dev, double* const* out_dev);
/* The eigensolver of ew_eigs for every problem, advanced in lock-step
 * (descs: nprob entries).  Outputs of problem i start at i*k_cap in mu_host,
 * beta_host, res_host; n_conv_host[i] (may be NULL) gets its converged count;
 * Y_dev (may be NULL) is a host array of nprob device pointers, each to
 * n_active_i x k_cap FP64.  stats (may be NULL) sums over the problems.
 * Host-blocking.  EW_ERR_NOT_CONVERGED if any problem hit its budget. */
ew_status ew_batch_eigs(ew_batch b, const ew_eigs_desc* descs, int k_cap, double* mu_host, double* beta_host,
                        double* res_host, int* n_conv_host, double* const* Y_dev, ew_eigs_stats* stats);

/* ------------------------------------------------------------------------
 * Learned warm start for the implicit solves (not part of the paper's method:
 * the paper solves each implicit step by multigrid to a relative residual
 * tolerance, Sec. "An optimal O(N) eigenvalue solver", so an initial guess
 * saves cycles only through its residual).  A small network corrects a base
 * guess x0 of M x = b from that guess's residual; the multigrid still
 * iterates to mg_tol, so a poor guess costs cycles, never accuracy.
 *
 * Network (3057 parameters, FP32 master copy, BF16 in the products with FP32
 * accumulation): input planes r/s, b/s_b, c2 = a w^2/(1 + a w^2) and
 * c3 = min(a/h^2, 100)/100 (r = b - M x0, s = RMS of r, s_b = RMS of b over
 * the grid, a = dt^2/2, w = omega_used, h the spacing of the first axis; every
 * plane is zero outside the grid); 3x3 convolution 4->16, bias, ReLU; 3x3
 * 16->16, bias, ReLU; 3x3 16->1, bias.  Output y gives the guess x0 + s y.
 * Parameter vector order: W1[16][4][3][3], b1[16], W2[16][16][3][3], b2[16],
 * W3[1][16][3][3], b3[1]; W[o][i][ky][kx] multiplies the input at row offset
 * ky-1 and column offset kx-1.
 *
 * Training data are crops: an output window of crop x crop points (crop a
 * multiple of 16, 16..256) with the two field planes (r/s, b/s_b) over the
 * window plus 3 points on every side (zero outside the grid), the target r/s
 * over the window, and per crop c2, c3, a/h_x^2, a/h_y^2 and the rectangle of
 * the padded window that lies inside the grid.  Loss: the mean over all
 * window points of the batch of e^2, e = target - M y on the points whose
 * stencil neighbours lie inside the window or beyond a wall of the grid (M =
 * I - a L_h with L_h's wall closure, in units of the spacing), e = 0 on the
 * other points; it is the squared initial residual left by the guess, divided
 * by s^2.  Training: Adam (Kingma and Ba) on minibatches drawn with
 * replacement by SplitMix64.
 * ------------------------------------------------------------------------ */
#define EW_CNN_PARAMS 3057
#define EW_CNN_HALO 3

typedef struct ew_cnn_s* ew_cnn;
typedef struct ew_cnn_data_s* ew_cnn_data;

/* New network on the current device; the weights of the two hidden layers
 * drawn He-uniform from the SplitMix64 stream `seed` (parameter i uses draw i:
 * W = u sqrt(6/fan_in), fan_in = 9 x input channels); the last layer and the
 * biases start at 0, so that the untrained network returns the base guess.
 * Work is ordered on hip_stream.  Host-blocking. */
ew_status ew_cnn_create(uint64_t seed, void* hip_stream, ew_cnn* out);
void ew_cnn_destroy(ew_cnn cnn);
/* Copy EW_CNN_PARAMS FP32 parameters in or out (host arrays); set_params also
 * resets the optimiser state.  Host-blocking. */
ew_status ew_cnn_set_params(ew_cnn cnn, const float* params_host);
ew_status ew_cnn_get_params(ew_cnn cnn, float* params_host);

/* Crop store with room for `capacity` crops of crop x crop outputs, for steps
 * whose L_h has stencil order `order` (2 or 4). */
ew_status ew_cnn_data_create(int capacity, int crop, int order, ew_cnn_data* out);
void ew_cnn_data_destroy(ew_cnn_data d);
ew_status ew_cnn_data_count(ew_cnn_data d, int* count);
/* Append n caller-made crops: fields_dev [n][2][crop+6][crop+6] FP32
 * (r/s then b/s_b), target_dev [n][crop][crop] FP32, planes_host [n][4]
 * (c2, c3, a/h_x^2, a/h_y^2) and rect_host [n][4] (row0, row1, col0, col1: the
 * half-open rectangle of the padded window inside the grid; a window edge on
 * the grid's boundary is a wall).  Host-blocking. */
ew_status ew_cnn_data_append(ew_cnn_data d, int n, const float* fields_dev, const float* target_dev,
                             const float* planes_host, const int* rect_host);
/* Copy crops first..first+count-1 out, in the layout of ew_cnn_data_append
 * (any of the four outputs may be NULL).  Host-blocking. */
ew_status ew_cnn_data_read(ew_cnn_data d, int first, int count, float* fields_dev, float* target_dev,
                           float* planes_host, int* rect_host);
/* out_dev = S v_dev computed by the implicit FP64 2D operator `op` (as
 * ew_op_apply_filter), recording crops_per_step crops at each step n >= 1
 * from the solve of M S = 2 W^n, at the operator's base guess x0 (the guess of
 * its predictor; for EW_PRED_CNN the projection guess before the correction)
 * until the store is full.  Window origins are drawn from the SplitMix64
 * stream `seed` (successive calls continue it); one eighth of the origin range
 * on each side is clamped to the walls so that walls are sampled.  The grid
 * needs n[0], n[1] >= crop and the store's order.  Host-blocking. */
ew_status ew_cnn_data_collect(ew_cnn_data d, ew_op op, const double* v_dev, double* out_dev, int crops_per_step,
                              uint64_t seed);

/* y_dev [count][crop][crop] FP32 = network output on crops first..first+count-1. */
ew_status ew_cnn_forward(ew_cnn cnn, ew_cnn_data d, int first, int count, float* y_dev);
/* Loss over crops first..first+count-1 (host, may be NULL) and its gradient
 * with respect to the parameters (grad_dev, EW_CNN_PARAMS FP32, device).
 * Host-blocking. */
ew_status ew_cnn_loss_grad(ew_cnn cnn, ew_cnn_data d, int first, int count, double* loss_host, float* grad_dev);

typedef struct {
    int steps;        /* Adam steps */
    int batch;        /* crops per step */
    double lr;        /* step size */
    double beta1, beta2, eps;
    uint64_t seed;    /* SplitMix64 stream of the minibatch draws */
} ew_cnn_train_desc;

typedef struct {
    int steps;
    double first_loss, last_loss;  /* minibatch loss of the first and last step */
    double seconds;
} ew_cnn_train_stats;

/* steps Adam updates (step t uses m_t/(1-beta1^t) and v_t/(1-beta2^t)),
 * continuing the optimiser state of earlier calls.  Host-blocking. */
ew_status ew_cnn_train(ew_cnn cnn, ew_cnn_data d, const ew_cnn_train_desc* desc, ew_cnn_train_stats* stats);

/* Attach (cnn != NULL) or detach the network used by EW_PRED_CNN (implicit
 * FP64 2D operators; EW_ERR_UNSUPPORTED for mixed precision).  The network is
 * not owned and must outlive its use by op.  Attaching allocates one vector
 * of the operator's size. */
ew_status ew_op_set_cnn(ew_op op, ew_cnn cnn);
/* guess_dev = the learned guess for M x = b_dev (implicit 2D FP64 operator
 * with a network attached): the base guess x0 (the projection on the
 * operator's window of earlier solves for EW_PRED_PROJ and EW_PRED_CNN, else
 * zero; nothing is added to the window) corrected by the network.  base_dev
 * (may be NULL) receives x0.  Vectors n_active FP64, device, not aliased.
 * Host-blocking. */
ew_status ew_op_cnn_guess(ew_op op, const double* b_dev, double* base_dev, double* guess_dev);

/* Fill x_dev (n FP64, device) with SplitMix64 uniform[-1,1) values of stream
 * `seed`: element i is 2*((z_i >> 11) * 2^-53) - 1 with z_i the SplitMix64
 * output for counter i+1.  Stream-ordered on `hip_stream`. */
ew_status ew_fill_uniform(double* x_dev, int64_t n, uint64_t seed, void* hip_stream);

/* Message for the last failing call on this thread ("" if none). */
const char* ew_last_error(void);

/* Library version string. */
const char* ew_version(void);

/* Device memory of the library's own buffers (operator workspaces,
 * multigrid levels, Krylov bases, batch and network state): hipMalloc and
 * hipFree by default.  alloc(bytes, device, stream, ctx) returns a device
 * pointer (NULL on failure) to be used on `stream` (the owning object's
 * stream, NULL for the default stream); free(ptr, ctx) releases a pointer
 * that alloc returned, and is called only after the device has finished
 * all queued work (as hipFree would wait).  Pass both or neither (NULL, NULL restores the
 * default); ctx is handed back unchanged.  Process-wide, to be set while no
 * library buffer exists: EW_ERR_INVALID_ARG while buffers from the current
 * allocator are live.  Lets a caller route the workspace through a caching
 * allocator such as PyTorch's.  (Pinned host staging buffers stay with
 * hipHostMalloc.) */
typedef void* (*ew_alloc_fn)(size_t bytes, int device, void* stream, void* ctx);
typedef void (*ew_free_fn)(void* ptr, void* ctx);
ew_status ew_set_allocator(ew_alloc_fn alloc, ew_free_fn free_fn, void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* EIGENWAVE_H */
