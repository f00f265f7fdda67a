/*
 * bemfft.h -- C ABI of the grid-embedded FFT boundary-element operator for
 * AMD Instinct MI355X (gfx950).
 *
 * Method (Benad, "Acceleration of the Boundary Element Method for arbitrary
 * shapes with the Fast Fourier Transformation"):
 *   The boundary integral equation of Laplace's equation (eq. 4) and of
 *   Navier's equation (eq. 8),
 *       c u(x0) = int q u*(x - x0) dS - int u q*(x - x0) dS,
 *   is not a convolution over the boundary, but it is one over the space one
 *   dimension higher that encloses it (Sec. 3).  The boundary data are put on
 *   a uniform grid, zero wherever there is no boundary (Fig. 4), the kernels
 *   are sampled on the padded grid (Fig. 5), and each integral becomes
 *   IFFT(FFT(field) * FFT(kernel)) (eq. 16), read back at the boundary nodes.
 *   The unknown half of the boundary data is found by an iterative solve in
 *   which this convolution is the matrix-vector product (end of Sec. 4).
 *
 * Discrete operator (one row per boundary node j, p_j its grid point):
 *     r_j = c_j u_j + D[u]_j - S[q]_j
 *     S[q]_j = sum_k G(p_k - p_j) w_k q_k,   D[u]_j = sum_k H(p_k - p_j; n_k) w_k u_k
 *   G: single-layer kernel (u* of eq. 3 in 2D, 1/(4 pi r) in 3D, Kelvin's
 *   tensor of eq. 7); H: double-layer kernel (q* of eq. 12 / its 3D analogue,
 *   Kelvin's traction kernel).  w_k: boundary measure of node k (Sec. 4
 *   scales the grid sums by the discretisation length; here that factor is
 *   folded into a per-node weight).  Pairs in
 *   one grid cell: single layer uses the grid value at offset 0 (flat-panel
 *   integral over h^(d-1), divided by it; Navier: orientation average), the
 *   node itself uses the flat-panel integral over its own w_j; double layer 0.
 *
 * Conventions for every call:
 *   - All functions return an int status: 0 = success, < 0 = error (the
 *     object is left unchanged), > 0 = a non-fatal condition (see below).
 *     bemfft_last_error() gives a thread-local message for the last failure.
 *   - Device vectors are component-major ("SoA"): [ncomp][m] doubles, with
 *     ncomp = 1 for Laplace and 3 for Navier, in the caller's node order.
 *   - Host arrays are copied before the call returns; the library never
 *     keeps a caller pointer.
 *   - A plan is used by one stream at a time (it owns one workspace); create
 *     one plan per concurrent stream.
 *   - stream: a hipStream_t (NULL = the legacy default stream).
 */
#ifndef BEMFFT_H
#define BEMFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- statuses */
#define BEMFFT_OK 0
#define BEMFFT_EINVAL (-1)     /* bad argument: sizes, nodes off the grid, ...   */
#define BEMFFT_ENOMEM (-2)     /* device or host allocation failed               */
#define BEMFFT_EDEVICE (-3)    /* a HIP runtime call failed                      */
#define BEMFFT_EUNSUPPORTED (-4) /* a padded size with no compiled FFT plan      */
#define BEMFFT_EBREAKDOWN (-5) /* non-finite values in a solve                   */
#define BEMFFT_ENOCONV 1       /* solve stopped at maxit; result still written   */

typedef struct bemfft_plan bemfft_plan; /* opaque; owns all device state */

/* Kernel families: eq. (3) Laplace 2D, its 3D analogue, eq. (7) Kelvin, and
 * the elastic half-space of eq. (9).
 *
 * BEMFFT_HALFSPACE: the surface convolution of contact mechanics that the
 * paper starts from (eq. 9, Fig. 1).  The grid is 2D and is the half-space
 * surface; nodes are surface points (normals are ignored and may be NULL;
 * weights default to the cell area h^2).  Per node, q holds the surface
 * traction sigma = (sigma_x, sigma_y, sigma_z) and u the surface
 * displacement, both [3][m] with z pointing into the solid (a compressive
 * pressure is sigma_z > 0).  K is the Boussinesq-Cerruti tensor of the
 * surface displacement due to a surface point load (the paper cites it and
 * does not print it; nu = Poisson ratio, mu = shear modulus):
 *   K_xx = g ((1 - nu)/r + nu x^2/r^3),  K_yy likewise with y,  K_xy = g nu x y / r^3,
 *   K_zz = g (1 - nu)/r,  K_xz = -K_zx = -g (1 - 2 nu) x / (2 r^2),
 *   K_yz = -K_zy = -g (1 - 2 nu) y / (2 r^2),  g = 1 / (2 pi mu),
 * at the offset (x, y) = target - source, with the mean over the node's own
 * cell at offset 0 (constant load per cell).  bemfft_apply returns
 *   r = K[sigma] - u   (the free term is c = -1 whatever the c_mode),
 * so K[sigma] is apply(sigma, 0), and bemfft_solve with bc = 0 finds the
 * traction for a given displacement (a punch of known shape on a known
 * contact area), bc = 1 the displacement for a given traction.  The 2D grid
 * box of bemfft_eval_grid holds K[sigma] at every surface grid point. */
typedef enum { BEMFFT_LAPLACE2D = 0, BEMFFT_LAPLACE3D = 1, BEMFFT_NAVIER3D = 2, BEMFFT_HALFSPACE = 3 } bemfft_kernel;

/* Arithmetic of the transforms and the spectral product.  Kernel spectra are
 * always computed in FP64 and rounded to the working precision.
 *   BEMFFT_FP64, BEMFFT_FP32: every transform and product in that precision.
 *   BEMFFT_BF16_MFMA (3D plans only): the arrays that carry the apply's HBM
 *     traffic -- the field transforms after the y pass, the results of the
 *     inverse z pass and the kernel spectra -- are stored in BF16; the z
 *     transforms run as two stages of dense 16 x 16 DFT matrix products on
 *     the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation); the x
 *     and y transforms, the spectral products and the gather are FP32, node
 *     data and results FP64.  Stated error of an apply against the FP64
 *     operator: <= 2e-3 of the term magnitudes (one BF16 unit round-off;
 *     measured 1e-4 to 5e-4); use it for the inner solves of an
 *     FP64-refined solve (bemfft_solve refine = 1).  Batches of 16-bit plans
 *     are not supported. */
typedef enum { BEMFFT_FP64 = 0, BEMFFT_FP32 = 1, BEMFFT_BF16_MFMA = 2 } bemfft_precision;

/* Free term c of eq. (4)/(8): 1/2 (smooth boundary), user values, or the
 * implicit c_j = -D[1]_j (Navier: C_j = -[D e_1, D e_2, D e_3]_j). */
typedef enum { BEMFFT_C_HALF = 0, BEMFFT_C_USER = 1, BEMFFT_C_IMPLICIT = 2 } bemfft_cmode;

/* Uniform grid: n[a] points per axis at origin + h * g, g in [0, n[a]).
 * dim = 2 uses n[0], n[1] (n[2] ignored).  pad[a] = padded FFT length per
 * axis; 0 picks the smallest supported even length >= 2 n[a] (Sec. 4 pads the
 * space for the FFT without fixing the size).  Supported lengths: 32, 64,
 * 96, 128, 192, 256, 320, 384, 512, and 1024 on 2D grids; so n[a] <= 512 in
 * 2D and <= 256 in 3D (EINVAL beyond, EUNSUPPORTED for other pad values). */
typedef struct {
    int dim;
    int64_t n[3];
    double h;
    double origin[3];
    int64_t pad[3];
} bemfft_grid;

typedef struct {
    bemfft_precision precision; /* default BEMFFT_FP64                        */
    bemfft_cmode c_mode;        /* default BEMFFT_C_IMPLICIT                  */
    const double *c_user;       /* host; m values (Laplace) or m*9 row-major
                                   3x3 blocks (Navier); read if C_USER         */
    void *stream;               /* stream used by plan_create's device work   */
    int keep_fp64;              /* 1: also keep the FP64 operator of this plan
                                   (needed by FP64-refined solves of a lower-
                                   precision plan); default 0                */
    int autotune;               /* radix schedule of the z transform: 0 the
                                   default one for the family, precision and
                                   length, 1 time every compiled schedule on
                                   this plan and keep the fastest, then time
                                   1 and 2 kx per thread in the forward
                                   direct DFT and keep the faster (both
                                   cached per kernel/precision/padded size in
                                   the file named by BEMFFT_TUNE_CACHE, if
                                   set),
                                   2 + s schedule s: 0 and 1 (16 or 32 lanes
                                   per pencil, by length) always exist; 2,
                                   the wide one with 64 lanes per pencil,
                                   only for Navier plans with padded z length
                                   256, 384 or 512 (else the default is
                                   kept).  Other values: EINVAL.            */
    int cell_quad;              /* kernel values at grid offsets m != 0
                                   (Sec. 4 / Fig. 5 discretises the kernels
                                   as constants per element): 0 or 1 the
                                   kernel at the offset itself (default);
                                   2..8 its mean over the grid cell of side h
                                   centred on the offset, by a tensor
                                   Gauss-Legendre rule of cell_quad points per
                                   grid axis (cell_quad^dim kernel values per
                                   offset; plan time grows accordingly).  The
                                   offset-0 values (self and same-cell terms)
                                   do not change.  Other values: EINVAL.     */
} bemfft_plan_opts;

/*
 * Create a plan for one boundary (eq. 4 / eq. 8 on the grid of Sec. 3).
 *   out      receives the plan (set to NULL on failure).
 *   grid     see bemfft_grid.
 *   m        number of boundary nodes (>= 1).
 *   nodes    host, m*dim doubles, row-major positions; each is snapped to the
 *            grid point floor((x - origin)/h + 1/2), which must lie in [0, n).
 *   normals  host, m*dim: mean outward normal of the node's boundary piece.
 *   weights  host, m: arc length (2D) / area (3D) of the piece, > 0; NULL
 *            means h^(dim-1) for every node (the paper's grid-aligned case).
 *   kernel   bemfft_kernel (must match grid->dim).
 *   nu, mu   Poisson ratio in (-1, 1/2) and shear modulus > 0 (Navier only).
 *   opts     NULL for defaults.
 * The plan samples the kernels on the padded grid, transforms them in FP64,
 * keeps one octant of each real (or imaginary) spectrum, and for C_IMPLICIT
 * runs the FP64 operator once per rigid mode.  Errors: EINVAL, ENOMEM,
 * EDEVICE, EUNSUPPORTED.
 */
int bemfft_plan_create(bemfft_plan **out, const bemfft_grid *grid, int64_t m,
                       const double *nodes, const double *normals, const double *weights,
                       int kernel, double nu, double mu, const bemfft_plan_opts *opts);

/*
 * r = c u + D[u] - S[q] (the residual of eq. 4 / eq. 8 at every node),
 * evaluated as the zero-padded FFT convolution of eq. (16).
 *   q, u   device, [ncomp][m] doubles (q is the flux, Navier: traction t).
 *   r      device, [ncomp][m] doubles, written; may not alias q or u.
 *   stream hipStream_t; asynchronous, no host synchronisation.
 * Errors: EINVAL (NULL pointers), EDEVICE.
 */
int bemfft_apply(bemfft_plan *p, const double *q, const double *u, double *r, void *stream);

/*
 * Same as bemfft_apply, repeated 'reps' times with HIP events recorded on
 * 'stream' between the four stages (scatter + x/y transforms, z transform +
 * spectral products, inverse y transform, gather at the nodes); stage_ms[4]
 * receives the mean duration of each stage in milliseconds.  Synchronises
 * the stream.  For measurement only.  Errors: EINVAL, EDEVICE.
 */
int bemfft_apply_profile(bemfft_plan *p, const double *q, const double *u, double *r, int reps,
                         double *stage_ms, void *stream);

/* Options of the iterative solve (GMRES, restarted, right Jacobi). */
typedef struct {
    double tol;     /* stop when ||b - A x||_2 <= tol ||b||_2 (default 1e-6) */
    int restart;    /* Krylov basis size (default 100, max 400)               */
    int maxit;      /* total iterations (default 1000)                        */
    int precond;    /* right preconditioner: 0 none, 1 Jacobi (default), 2
                       block Jacobi: the inverse of each node's 3x3 diagonal
                       block of the mixed operator (-S_jj columns where q is
                       unknown, C_j columns where u is unknown) for Navier
                       plans, Jacobi for the others.  Batches: 0 or 1.   */
    int use_x0;     /* 0: start from x = 0; 1: 'unknown' holds the initial
                       guess on entry; 2: as 1, but the guess is kept only
                       if ||b - A x0|| < ||b|| (else x = 0: plain GMRES)  */
    int refine;     /* 1: iterative refinement -- residuals r = b - A x with
                       the plan's FP64 operator (plan made with keep_fp64),
                       corrections from GMRES with the plan's working
                       precision; 0: plain GMRES in the working precision   */
    double inner_tol; /* refine: relative tolerance of each inner solve
                         (default 1e-4)                                     */
    int max_outer;  /* refine: maximum refinement steps (default 20)          */
} bemfft_solve_opts;

typedef struct {
    int iters;          /* GMRES iterations (working-precision applications)  */
    int restarts;
    double true_relres; /* ||b - A x|| / ||b|| recomputed with a fresh apply  */
    int status;         /* same as the return value                          */
    double seconds;     /* wall time of the call                              */
    int outer;          /* refinement steps (0 without refine)                */
    int applies64;      /* FP64 applications made by the refinement            */
    int x0_used;        /* 1 if the solve started from the caller's guess      */
    double x0_relres;   /* use_x0 = 2: ||b - A x0|| / ||b|| of the guess, else -1 */
} bemfft_solve_info;

/*
 * Solve the mixed boundary-value problem (Sec. 4: u given, q sought; the
 * general case mixes both per node):
 *   bc       device, [ncomp][m] uint8: 0 = u known (Dirichlet), 1 = q known.
 *   known    device, [ncomp][m]: the given value per slot.
 *   unknown  device, [ncomp][m]: the other value per slot (q where bc = 0,
 *            u where bc = 1); on entry the initial guess if use_x0.
 * Unknowns x satisfy A x = b with A x = apply(x in the unknown slots) and
 * b = -apply(known values).  Arnoldi, Givens rotations and the true residual
 * are FP64.  With opts->refine, b and every residual b - A x use the FP64
 * operator while the corrections come from GMRES on the working precision
 * (iterative refinement); the returned true_relres is then the FP64 one.
 * Returns 0, ENOCONV (maxit reached; x and info still written), EBREAKDOWN
 * (non-finite values), EINVAL (also: refine on a plan without the FP64
 * operator), EDEVICE.  The host waits once per iteration for that
 * iteration's Hessenberg column (the next iteration is already queued on
 * 'stream', so the GPU does not idle meanwhile); the stream is synchronised
 * before the call returns.
 */
int bemfft_solve(bemfft_plan *p, const uint8_t *bc, const double *known, double *unknown,
                 const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream);

/* Size of the fixed device workspace of bemfft_solve_noalloc: 32 MiB. */
#define BEMFFT_NOALLOC_SCRATCH_BYTES (32LL << 20)

/*
 * bemfft_solve without any allocation, for callers that cannot allocate
 * memory once they run: tight serving loops and harnesses that forbid
 * hipMalloc after set-up.  Arguments, options, results and statuses are
 * those of bemfft_solve (same kernels, same arithmetic: the same solution
 * bit for bit), except:
 *   - the Krylov basis, work vectors and reduction partials live in one
 *     file-scope device array of BEMFFT_NOALLOC_SCRATCH_BYTES per GPU, held
 *     until the process ends; its address is looked up once per device, on
 *     the first call there;
 *   - limit: (restart + 10) * ncomp * m + 132096 doubles must fit in it
 *     (restart + 13 with block Jacobi on a Navier plan), else
 *     EINVAL before any device work (the message names the largest restart
 *     for the plan): e.g. restart 100 for up to 36,929 unknowns, restart 30
 *     for up to 101,555;
 *   - every call on one GPU shares that array and keeps what the last call
 *     left in it: calls that overlap on one GPU (several host threads or
 *     streams) race and give wrong results;
 *   - no hipMalloc, hipFree, hipHostMalloc or event creation: the host
 *     waits for each GMRES step before queueing the next and copies its
 *     Hessenberg column to pageable host memory, so an iteration costs a
 *     little more host latency than in bemfft_solve.
 * The plan must exist already (bemfft_plan_create allocates).
 */
int bemfft_solve_noalloc(bemfft_plan *p, const uint8_t *bc, const double *known, double *unknown,
                         const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream);

/*
 * Dirichlet Laplace problem by conjugate gradients, the paper's own solver
 * (end of Sec. 4): u given at every node, find q with
 *     S[q] = c u + D[u]                      (eq. 4 with r = 0).
 * S = G W, where G (the single-layer kernel on the grid, with the exact
 * self terms on its diagonal) is symmetric and W = diag(w), so CG runs on
 * the symmetrised system
 *     W^1/2 G W^1/2 y = W^1/2 (c u + D[u]),  q = W^-1/2 y,
 * which is positive definite for the 3D kernel and for the 2D kernel when
 * the boundary's logarithmic capacity is below 1 (any boundary inside a
 * disc of radius 1).  Each iteration is one apply in the plan's working
 * precision; vectors and dot products are FP64.
 *   u  device, [m]: the Dirichlet data.
 *   q  device, [m]: on entry the initial guess if opts->use_x0 = 1; on
 *      return the solution.
 *   opts: tol (on ||r|| / ||b|| of the symmetrised system), maxit, precond
 *      (0 none, 1 Jacobi with the exact self terms), use_x0 (0 or 1);
 *      restart and the refinement fields are ignored.  NULL = defaults.
 *   info: iters, true_relres (recomputed with a fresh apply), status,
 *      seconds; the other fields are 0 (x0_relres -1).
 * Returns 0, ENOCONV (maxit reached; q and info written), EBREAKDOWN (a
 * direction with p.Ap <= 0: the system is not positive definite, q is not
 * meaningful), EINVAL (Navier or half-space plan, null pointer, bad options), ENOMEM,
 * EDEVICE.  Synchronises `stream`; not concurrent with other calls on the
 * same plan.
 */
int bemfft_solve_cg(bemfft_plan *p, const double *u, double *q, const bemfft_solve_opts *opts,
                    bemfft_solve_info *info, void *stream);

/* ------------------------------------------------------------- batches
 * Many boundaries and right-hand sides at once (the operator of eq. 4 / 8
 * for each; nothing couples the members).  A member is (plan i, right-hand
 * side j); all plans of a batch share the kernel family and working
 * precision.  Device vectors of a batch concatenate the members' [ncomp][m_i]
 * blocks in member order: plan 0 rhs 0, plan 0 rhs 1, ..., plan 1 rhs 0, ...
 * (bemfft_batch_members gives each block's offset and length in doubles).
 * The batch refers to its plans, which must outlive it, and owns one set of
 * intermediates per member.
 */
typedef struct bemfft_batch bemfft_batch;

/* Build a batch of nplans plans x nrhs right-hand sides.  Members of plans
 * with equal padded sizes and z schedule share one launch per stage.  With
 * use_graph = 1 the launch sequence is captured once into a HIP graph that
 * every batched apply replays.  Errors: EINVAL (mixed families/precisions),
 * ENOMEM, EDEVICE. */
int bemfft_batch_create(bemfft_batch **out, bemfft_plan *const *plans, int nplans, int nrhs, int use_graph,
                        void *stream);

/* r = c u + D[u] - S[q] for every member (concatenated device vectors). */
int bemfft_batch_apply(bemfft_batch *b, const double *q, const double *u, double *r, void *stream);

/* The mixed problem of bemfft_solve for every member (bc, known, unknown
 * concatenated), by restarted GMRES run for all members in lockstep: one
 * batched apply per iteration; members leave when their own relative true
 * residual meets tol.  info: NULL or one entry per member.  refine is not
 * supported (EINVAL).  Returns 0, ENOCONV if any member stopped at maxit,
 * EBREAKDOWN, EINVAL, EDEVICE. */
int bemfft_batch_solve(bemfft_batch *b, const uint8_t *bc, const double *known, double *unknown,
                       const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream);

/* Member count; offsets/lengths (may be NULL) receive each member's block. */
int bemfft_batch_members(const bemfft_batch *b, int64_t *offsets, int64_t *lengths);

int bemfft_batch_destroy(bemfft_batch *b);

/* The field over the grid box: the representation formula of eq. (4) /
 * eq. (8) with the free term c = 1 inside the boundary and c = 0 outside
 * (Sec. 2), evaluated through the same convolution as bemfft_apply, whose
 * inverse transform holds it at every grid point (Sec. 4):
 *
 *     out[o][z - z_lo][y][x] = S[q](p) - D[u](p),  p = origin + h (x, y, z),
 *
 * for 0 <= x < n[0], 0 <= y < n[1] and the planes z_lo <= z < z_lo + z_count
 * that hold nodes (bemfft_plan_get_info; 2D: one plane).  Every point
 * inside the boundary lies in this box.  Inside, for a pair (u, q) that
 * solves the boundary problem, the value is the solution u(p); outside it
 * is 0 up to discretisation error.  At grid points that hold nodes it is
 * the plain grid sum (no free term, the grid's own value at offset 0 for
 * the single layer): use bemfft_apply for values on the boundary.
 * For BEMFFT_HALFSPACE plans the box is the surface grid and out holds the
 * surface displacement K[q] at every grid point (u is not used).
 *
 * q, u: device, [ncomp][m] as in bemfft_apply.  out: device, ncomp *
 * z_count * n[1] * n[0] doubles, x fastest.  Computed in the plan's working
 * precision; async on `stream`; uses the plan's workspace, so it must not
 * overlap other calls on the same plan.  Errors: EINVAL (null pointer),
 * EDEVICE. */
int bemfft_eval_grid(bemfft_plan *p, const double *q, const double *u, double *out, void *stream);

/* Facts about a plan (host copies). */
typedef struct {
    int dim, kernel, precision, c_mode;
    int64_t m, ncomp;
    int64_t n[3], pad[3];
    int64_t z_lo, z_count;       /* occupied grid planes along the last axis   */
    int64_t nfields, nspectra, noutputs;
    int64_t workspace_bytes, spectra_bytes;
    double spectrum_parity_residual; /* max discarded (imag or real) part of
                                        the kernel spectra / max |spectrum|     */
    double plan_seconds;
    int zsched;                  /* radix schedule in use for the z transform
                                    (0, 1 or 2)                               */
    double tune_us[3];           /* autotune: mean apply time per schedule, us
                                    (0 for schedules not timed)               */
    int fwd_xg;                  /* kx per thread in the forward direct DFT
                                    (1 or 2): from the row lengths, or timed
                                    by autotune = 1                           */
    double fwd_tune_us[2];       /* autotune = 1: mean apply time with 1 and 2
                                    kx per thread, us (0 if not timed)        */
} bemfft_plan_info;

int bemfft_plan_get_info(const bemfft_plan *p, bemfft_plan_info *info);

/* Copy the free-term values c_j in use (host; m or m*9 doubles). */
int bemfft_plan_get_c(const bemfft_plan *p, double *c_host);

/* Release all device state of the plan.  NULL is accepted. */
int bemfft_plan_destroy(bemfft_plan *p);

/* ------------------------------------------------------ learned start
 * A small 3D convolutional network that maps a Dirichlet problem (Sec. 4:
 * u given on the boundary, q sought) to an initial guess of q for
 * bemfft_solve (use_x0 = 2 keeps the guess only if it beats x = 0).  This
 * is an addition to the method, not part of the paper.
 *   Input channels on the plan's n^3 grid (zero off the boundary), summed
 *   over the nodes of a voxel: a = w/h^2; a n_x; a n_y; a n_z; a s u; a s b
 *   (u the Dirichlet value, s = 1/rms(u) over the Dirichlet slots, b the
 *   right-hand side of bemfft_solve: minus the operator applied to the
 *   known values, computed with one application of the plan).
 *   Layers: 3x3x3 convolutions with per-layer dilation (zero padding),
 *   6 -> 16 -> ... -> 16 -> 1 channels, bias, ReLU on all but the last.
 *   Output y: one channel; the guess is q_j = y(voxel of node j) / (s h)
 *   (training targets are s h q_j: a flux per voxel length).
 * Parameters are FP32, laid out per layer as W[cout][cin][27] (tap index
 * (dz+1)*9 + (dy+1)*3 + (dx+1)) followed by b[cout].  Arithmetic and
 * activations are FP32.  Training minimises sum_i wt_i (y(vox_i) - t_i)^2
 * with Adam (beta 0.9 / 0.999, eps 1e-8).  A network owns its activations
 * (2 * layers * 16 * n^3 floats) and is used by one stream at a time.
 */
typedef struct bemfft_net bemfft_net;

/* grid in [4, 256], width 16, layers in [2, 8], dilations[layers] >= 1.
 * Weights: He-normal from a 64-bit Mersenne twister with 'seed' (the last
 * layer scaled by 0.1), biases 0.  Errors: EINVAL, ENOMEM. */
int bemfft_net_create(bemfft_net **out, int grid, int width, int layers, const int *dilations,
                      uint64_t seed, void *stream);
int bemfft_net_destroy(bemfft_net *n);
int64_t bemfft_net_num_params(const bemfft_net *n);
/* host <-> device copies of the parameter vector (num_params floats) */
int bemfft_net_get_params(const bemfft_net *n, float *params_host);
int bemfft_net_set_params(bemfft_net *n, const float *params_host);

/* Input channels of a problem: x device [6][n^3] floats (overwritten).  The
 * plan must be LAPLACE3D on the network's grid; bc/known as for
 * bemfft_solve (bc may be NULL: all Dirichlet); scale is s.  Runs one
 * apply of the plan on 'stream' (network-owned scratch of 3m doubles,
 * grown on demand).  Errors: EINVAL, ENOMEM, EDEVICE. */
int bemfft_net_input(bemfft_net *n, bemfft_plan *p, const uint8_t *bc, const double *known,
                     double scale, float *x, void *stream);

/* y device [n^3] = network(x), FP32 storage and arithmetic (the training
 * path). */
int bemfft_net_forward(bemfft_net *n, const float *x, float *y, void *stream);

/* y device [n^3] = network(x) for inference: activations and weights in
 * FP16 (channel-last), products on the matrix cores with FP32 accumulation,
 * bias and ReLU in FP32 before the FP16 rounding; y is FP32.  Used by
 * bemfft_net_guess.  Relative error against the FP32 path ~1e-3. */
int bemfft_net_infer(bemfft_net *n, const float *x, float *y, void *stream);

/* Loss sum_i wt_i (y(vox_i) - tgt_i)^2 of input x (all device arrays, nt
 * targets, 1 <= nt <= 2^24, vox = z*n*n + y*n + x; a target whose voxel lies
 * outside [0, n^3) is ignored) and its gradient with respect to every
 * parameter (written to grad_host if not NULL, num_params floats).
 * Deterministic except for voxels that hold several targets.  Synchronises
 * the stream.  Errors: EINVAL, EDEVICE. */
int bemfft_net_gradients(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt,
                         const float *wt, double *loss, float *grad_host, void *stream);

/* One Adam step (learning rate lr) on the loss above; the loss before the
 * step goes to *loss.  Synchronises the stream. */
int bemfft_net_train_step(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt,
                          const float *wt, float lr, double *loss, void *stream);

/* Initial guess for bemfft_solve: x0 device [m] doubles, q_j at Dirichlet
 * slots, 0 elsewhere; xbuf device [6][n^3] floats is scratch.  s is computed
 * on the device; one apply of the plan, the FP16 inference and the gather
 * are queued on 'stream' (no host synchronisation).  Errors: as
 * bemfft_net_input. */
int bemfft_net_guess(bemfft_net *n, bemfft_plan *p, const uint8_t *bc, const double *known,
                     float *xbuf, double *x0, void *stream);

/* Voxel index (z*n*n + y*n + x) and weight w_j of each node, in the
 * caller's node order (host arrays of m; either may be NULL). */
int bemfft_plan_node_voxels(const bemfft_plan *p, int *vox_host, double *w_host);

/* In-place FP64 complex 3D FFT of a device array [pz][py][px] of interleaved
 * (re, im) doubles with the library's own transform kernels (the transform
 * used for the kernel spectra); direction -1 forward, +1 inverse (unscaled).
 * Lengths must be supported FFT sizes or 1.  Provided for testing. */
int bemfft_fft3d_c2c_f64(double *data, int64_t px, int64_t py, int64_t pz, int direction,
                         void *stream);

/* Human-readable name of a status; thread-local detail of the last error. */
const char *bemfft_strerror(int status);
const char *bemfft_last_error(void);

/* Supported padded FFT lengths (fills up to cap entries; returns the count);
 * the last one, 1024, is for 2D grids only. */
int bemfft_supported_sizes(int64_t *sizes, int cap);

#ifdef __cplusplus
}
#endif
#endif /* BEMFFT_H */
