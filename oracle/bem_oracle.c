/*
 * bem_oracle.c -- plain CPU FP64 oracle for the grid-embedded BEM operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (Benad, "Acceleration of the BEM for arbitrary shapes with
 * the FFT", Secs. 2-4):
 *
 *   The boundary integral equation (eq. 4 for Laplace, eq. 8 for Navier)
 *       c u(x0) = int q u*(x - x0) dS - int u q*(x - x0) dS
 *   is evaluated at every node x0 = p_j.  Following Sec. 3 and eqs. (14)-(16),
 *   the boundary data live on the points of a uniform grid (zero elsewhere)
 *   and the kernels are sampled on the same grid, so the FFT convolution of
 *   eq. (16) equals, exactly up to rounding, the direct double sum below.  The
 *   oracle is that direct sum, O(M^2), with no transform at all:
 *
 *     S[q]_j = sum_k  G(p_k - p_j) w_k q_k         (single layer)
 *     D[u]_j = sum_k  H(p_k - p_j; n_k) w_k u_k    (double layer)
 *     r_j    = c_j u_j + D[u]_j - S[q]_j           (residual of eq. 4 / 8)
 *
 *   with p_j = origin + h g_j the node's grid point, g_j = floor((x_j -
 *   origin)/h + 1/2), w_k the boundary measure carried by node k (Sec. 4
 *   scales the grid sums by the discretisation length; that factor is folded
 *   into the weight),
 *   and n_k the node's mean outward normal.
 *
 * Readings of points the paper leaves open (each one is listed with its
 * reason in the design notes):
 *   - k == j: the single layer uses the flat-panel integral of the kernel over
 *     the node's own measure; the double-layer kernels are odd and give 0.
 *   - k != j but g_k == g_j (two nodes in one cell): the single layer uses the
 *     grid's value at offset 0, the flat-panel integral for the reference
 *     measure h^(d-1) divided by that measure (Navier: orientation average).
 *   - kernel values at offsets m != 0: the kernel at the offset itself, or,
 *     with a cell rule, its mean over the grid cell centred on the offset
 *     (the constant-element reading of Sec. 4 / Fig. 5, taken literally);
 *     the rule is a tensor product of q given points per axis on
 *     [-1/2, 1/2] with weights summing to 1 (the callers pass Gauss-Legendre
 *     points).  Offset 0 keeps the values above.
 *   - c_j: 1/2 (smooth boundary, eq. 4), user supplied, or implicit
 *     c_j = -D[1]_j (Navier: C_j = -[D e_1, D e_2, D e_3]_j), the rigid-mode
 *     identity of eq. (4)/(8) applied to the discrete operator.
 *
 * Kernels (xi = field point - target point, r = |xi|):
 *   Laplace 2D, eq. (3)/(11)/(12):  u* = -ln r / (2 pi),  grad_i u* = -xi_i / (2 pi r^2)
 *   Laplace 3D (textbook; the paper writes Laplace out in 2D only):
 *                                   u* = 1 / (4 pi r),    grad_i u* = -xi_i / (4 pi r^3)
 *   Kelvin, eq. (7):  U_kj = [(3-4nu) d_kj / r + xi_k xi_j / r^3] / (16 pi mu (1-nu))
 *   Kelvin traction (the t* "known from u* with the material law" after eq. 8):
 *     T_kj(xi; n) = -[ dr/dn ((1-2nu) d_kj + 3 e_k e_j) - (1-2nu)(e_k n_j - e_j n_k) ]
 *                   / (8 pi (1-nu) r^2),     e = xi / r,  dr/dn = e . n
 *   (k = direction of the point force = equation index, j = component.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define ORC_PI 3.14159265358979323846264338327950288

enum { ORC_LAPLACE2D = 0, ORC_LAPLACE3D = 1, ORC_NAVIER3D = 2, ORC_HALFSPACE = 3 };
enum { ORC_C_HALF = 0, ORC_C_USER = 1, ORC_C_IMPLICIT = 2 };

/* ------------------------------------------------------------------ kernels */

/* Laplace 2D, eqs. (3), (11), (12): out = {u*, d_x u*, d_y u*}. */
void orc_laplace2d(const double xi[2], double out[3])
{
    double r2 = xi[0] * xi[0] + xi[1] * xi[1];
    double r = sqrt(r2);
    out[0] = -log(r) / (2.0 * ORC_PI);
    out[1] = -xi[0] / (2.0 * ORC_PI * r2);
    out[2] = -xi[1] / (2.0 * ORC_PI * r2);
}

/* Laplace 3D: out = {u*, d_x u*, d_y u*, d_z u*}. */
void orc_laplace3d(const double xi[3], double out[4])
{
    double r2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    double r = sqrt(r2);
    out[0] = 1.0 / (4.0 * ORC_PI * r);
    out[1] = -xi[0] / (4.0 * ORC_PI * r2 * r);
    out[2] = -xi[1] / (4.0 * ORC_PI * r2 * r);
    out[3] = -xi[2] / (4.0 * ORC_PI * r2 * r);
}

/* Kelvin displacement tensor, eq. (7): U[3k + j]. */
void orc_kelvin_u(const double xi[3], double nu, double mu, double U[9])
{
    double r2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    double r = sqrt(r2);
    double pre = 1.0 / (16.0 * ORC_PI * mu * (1.0 - nu));
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j)
            U[3 * k + j] = pre * ((k == j ? (3.0 - 4.0 * nu) / r : 0.0) + xi[k] * xi[j] / (r2 * r));
}

/* Kelvin traction kernel at a field point with normal n: T[3k + j]. */
void orc_kelvin_t(const double xi[3], const double n[3], double nu, double T[9])
{
    double r2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    double r = sqrt(r2);
    double e[3] = {xi[0] / r, xi[1] / r, xi[2] / r};
    double drdn = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
    double a = 1.0 - 2.0 * nu;
    double pre = -1.0 / (8.0 * ORC_PI * (1.0 - nu) * r2);
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j)
            T[3 * k + j] = pre * (drdn * ((k == j ? a : 0.0) + 3.0 * e[k] * e[j]) - a * (e[k] * n[j] - e[j] * n[k]));
}

/* ------------------------------------------------------------- self terms */

/* Integral of u* over a straight segment of length w centred on the target:
 * int_{-w/2}^{w/2} -ln|s| / (2 pi) ds. */
double orc_self_laplace2d(double w)
{
    return w * (1.0 - log(0.5 * w)) / (2.0 * ORC_PI);
}

/* Integral of 1/(4 pi r) over a flat square of area w centred on the target. */
double orc_self_laplace3d(double w)
{
    double s = sqrt(w);
    return s * log(1.0 + sqrt(2.0)) / ORC_PI;
}

/* Integral of U over a flat square of area w with unit normal n, centred on
 * the target.  In-plane: int xi_k xi_j / r^3 = (d_kj - n_k n_j) * (1/2) int 1/r. */
void orc_self_kelvin(double w, const double n[3], double nu, double mu, double out[9])
{
    double s = sqrt(w);
    double i1 = 4.0 * s * log(1.0 + sqrt(2.0)); /* int 1/r over the square */
    double pre = 1.0 / (16.0 * ORC_PI * mu * (1.0 - nu));
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
            double d = (k == j) ? 1.0 : 0.0;
            out[3 * k + j] = pre * i1 * ((3.0 - 4.0 * nu) * d + 0.5 * (d - n[k] * n[j]));
        }
}

/* Elastic half-space, eq. (9): surface displacement component a at the
 * surface offset d = (target - source) due to a unit surface point load in
 * direction b, z pointing into the solid (Boussinesq's solution for the
 * normal load, Cerruti's for the tangential ones; Johnson, Contact
 * Mechanics, Sec. 2.2, written with E = 2 mu (1 + nu)).  out[3 a + b]. */
void orc_halfspace(const double d[2], double nu, double mu, double out[9])
{
    double x = d[0], y = d[1];
    double r2 = x * x + y * y, r = sqrt(r2);
    double e = 1.0 / (2.0 * ORC_PI * mu);
    double t = 0.5 * (1.0 - 2.0 * nu) / r2; /* normal-tangential coupling */
    out[0] = e * ((1.0 - nu) / r + nu * x * x / (r2 * r));
    out[1] = e * nu * x * y / (r2 * r);
    out[2] = -e * t * x; /* u_x from a normal load: towards the load */
    out[3] = out[1];
    out[4] = e * ((1.0 - nu) / r + nu * y * y / (r2 * r));
    out[5] = -e * t * y;
    out[6] = e * t * x;  /* u_z from a tangential load (reciprocity) */
    out[7] = e * t * y;
    out[8] = e * (1.0 - nu) / r;
}

/* The half-space tensor integrated over a square of area w centred on the
 * load (constant traction on the node's own cell): the square of side s
 * gives int 1/r = 4 s ln(1 + sqrt 2), int x^2/r^3 = int y^2/r^3 = half of
 * that, and the odd components vanish.  out[3 a + b]. */
void orc_self_halfspace(double w, double nu, double mu, double out[9])
{
    double i1 = 4.0 * sqrt(w) * log(1.0 + sqrt(2.0));
    double e = 1.0 / (2.0 * ORC_PI * mu);
    for (int i = 0; i < 9; ++i) out[i] = 0.0;
    out[0] = out[4] = e * i1 * (1.0 - 0.5 * nu);
    out[8] = e * i1 * (1.0 - nu);
}

/* Single-layer kernel value at grid offset 0, per unit weight: the flat-panel
 * integral for the reference measure h^(d-1), divided by that measure.  For
 * Navier the panel orientation is averaged: <n n> = I/3. */
void orc_grid_k0(int kernel, double h, double nu, double mu, double out[9])
{
    for (int i = 0; i < 9; ++i) out[i] = 0.0;
    if (kernel == ORC_LAPLACE2D) {
        out[0] = orc_self_laplace2d(h) / h;
    } else if (kernel == ORC_LAPLACE3D) {
        out[0] = orc_self_laplace3d(h * h) / (h * h);
    } else if (kernel == ORC_HALFSPACE) {
        /* r = K[sigma] - u: the "single layer" of the generic loop is -K */
        orc_self_halfspace(h * h, nu, mu, out);
        for (int i = 0; i < 9; ++i) out[i] = -out[i] / (h * h);
    } else {
        double s = h;
        double i1 = 4.0 * s * log(1.0 + sqrt(2.0));
        double pre = 1.0 / (16.0 * ORC_PI * mu * (1.0 - nu));
        for (int k = 0; k < 3; ++k)
            out[4 * k] = pre * i1 * ((3.0 - 4.0 * nu) + 1.0 / 3.0) / (h * h);
    }
}

/* ------------------------------------------------------------- snapping */

/* g = floor((x - origin)/h + 1/2) per axis; returns the index of the first
 * node outside [0, n) or -1 when all are inside. */
long orc_snap(int dim, long m, const double *nodes, double h, const double *origin,
              const long *n, long *g)
{
    long bad = -1;
    for (long j = 0; j < m; ++j)
        for (int a = 0; a < dim; ++a) {
            long v = (long)floor((nodes[j * dim + a] - origin[a]) / h + 0.5);
            g[j * dim + a] = v;
            if ((v < 0 || v >= n[a]) && bad < 0) bad = j;
        }
    return bad;
}

/* ------------------------------------------------------- pair contributions */

/* Single-layer block G (ncomp x ncomp) between target j and source k. */
static void single_block(int kernel, double nu, double mu, double h, const double *xi,
                         int same_cell, int same_node, double wk, const double *nk, double G[9])
{
    int nc = (kernel == ORC_NAVIER3D || kernel == ORC_HALFSPACE) ? 3 : 1;
    if (same_node) {
        if (kernel == ORC_LAPLACE2D) G[0] = orc_self_laplace2d(wk);
        else if (kernel == ORC_LAPLACE3D) G[0] = orc_self_laplace3d(wk);
        else if (kernel == ORC_HALFSPACE) {
            orc_self_halfspace(wk, nu, mu, G);
            for (int i = 0; i < 9; ++i) G[i] = -G[i];
        } else orc_self_kelvin(wk, nk, nu, mu, G);
        return;
    }
    if (same_cell) {
        double k0[9];
        orc_grid_k0(kernel, h, nu, mu, k0);
        for (int i = 0; i < nc * nc; ++i) G[i] = k0[i] * wk;
        return;
    }
    if (kernel == ORC_LAPLACE2D) {
        double o[3];
        orc_laplace2d(xi, o);
        G[0] = o[0] * wk;
    } else if (kernel == ORC_LAPLACE3D) {
        double o[4];
        orc_laplace3d(xi, o);
        G[0] = o[0] * wk;
    } else if (kernel == ORC_HALFSPACE) {
        /* u_j = sum_k K(p_j - p_k) w_k sigma_k; xi = p_k - p_j; "S" = -K */
        double d[2] = {-xi[0], -xi[1]};
        orc_halfspace(d, nu, mu, G);
        for (int i = 0; i < 9; ++i) G[i] *= -wk;
    } else {
        orc_kelvin_u(xi, nu, mu, G);
        for (int i = 0; i < 9; ++i) G[i] *= wk;
    }
}

/* Double-layer block H (ncomp x ncomp) between target j and source k;
 * zero when both sit in one cell (odd kernel at offset 0). */
static void double_block(int kernel, double nu, const double *xi, int same_cell, double wk,
                         const double *nk, double H[9])
{
    int nc = (kernel == ORC_NAVIER3D || kernel == ORC_HALFSPACE) ? 3 : 1;
    if (same_cell || kernel == ORC_HALFSPACE) { /* the half-space has no double layer */
        for (int i = 0; i < nc * nc; ++i) H[i] = 0.0;
        return;
    }
    if (kernel == ORC_LAPLACE2D) {
        double o[3];
        orc_laplace2d(xi, o);
        H[0] = (o[1] * nk[0] + o[2] * nk[1]) * wk; /* q* = n . grad u*, eq. (12) */
    } else if (kernel == ORC_LAPLACE3D) {
        double o[4];
        orc_laplace3d(xi, o);
        H[0] = (o[1] * nk[0] + o[2] * nk[1] + o[3] * nk[2]) * wk;
    } else {
        orc_kelvin_t(xi, nk, nu, H);
        for (int i = 0; i < 9; ++i) H[i] *= wk;
    }
}

/* Cell rule for the kernel values at offsets m != 0 (see the header): q
 * points x[] per axis on [-1/2, 1/2] with weights w[]; q = 0 samples the
 * kernel at the offset itself. */
typedef struct {
    int q;
    const double *x;
    const double *w;
} cell_rule;

static int ncomp_of(int kernel);
static int dim_of(int kernel);

/* G and H of one pair: the point value at offset 0 and without a rule,
 * else the weighted sum over the q^dim points of the cell around xi. */
static void pair_blocks(int kernel, double nu, double mu, double h, const double *xi, int same_cell,
                        int same_node, double wk, const double *nk, const cell_rule *cr, double G[9],
                        double H[9])
{
    if (same_cell || cr->q <= 0) {
        single_block(kernel, nu, mu, h, xi, same_cell, same_node, wk, nk, G);
        double_block(kernel, nu, xi, same_cell, wk, nk, H);
        return;
    }
    int dim = dim_of(kernel);
    int nc = ncomp_of(kernel);
    int q = cr->q;
    for (int i = 0; i < nc * nc; ++i) G[i] = H[i] = 0.0;
    int qz = (dim == 3) ? q : 1;
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
            for (int c = 0; c < qz; ++c) {
                double wt = cr->w[a] * cr->w[b] * (dim == 3 ? cr->w[c] : 1.0);
                double pt[3] = {xi[0] + h * cr->x[a], xi[1] + h * cr->x[b],
                                dim == 3 ? xi[2] + h * cr->x[c] : 0.0};
                double g[9], hh[9];
                single_block(kernel, nu, mu, h, pt, 0, 0, wk, nk, g);
                double_block(kernel, nu, pt, 0, wk, nk, hh);
                for (int i = 0; i < nc * nc; ++i) {
                    G[i] += wt * g[i];
                    H[i] += wt * hh[i];
                }
            }
}

static int ncomp_of(int kernel) { return (kernel == ORC_NAVIER3D || kernel == ORC_HALFSPACE) ? 3 : 1; }
static int dim_of(int kernel) { return (kernel == ORC_LAPLACE2D || kernel == ORC_HALFSPACE) ? 2 : 3; }

/* ---------------------------------------------------------------- the apply */

/*
 * r = c u + D[u] - S[q] for the targets t0 <= j < t1 (eq. 4 / eq. 8, in the
 * convolution reading of eqs. 14-16).
 *
 * q, u: [ncomp][m] component-major.  r, scale: [ncomp][t1 - t0].
 * c: C_HALF (1/2 I), C_USER (cuser: m values, or m*9 row-major 3x3 blocks for
 * Navier), C_IMPLICIT (c_j = -D[1]_j, computed here).
 * scale[k][j] = |c u|_k + sum |D||u| + sum |S||q|, the magnitude of the terms
 * that cancel in r, used for normwise tolerances.
 * grid_index: [m][dim] snapped grid indices (from orc_snap).
 * cq, cx, cw: the cell rule (cq = 0: point values; cx, cw unused).
 * Returns 0.
 */
int orc_apply(int kernel, double nu, double mu, double h, long m, const long *grid_index,
              const double *normals, const double *weights, int cmode, const double *cuser,
              const double *q, const double *u, long t0, long t1, double *r, double *scale,
              double *c_out, int cq, const double *cx, const double *cw)
{
    cell_rule cr = {cq, cx, cw};
    int dim = dim_of(kernel);
    int nc = ncomp_of(kernel);
    long nt = t1 - t0;
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = t0; j < t1; ++j) {
        double acc[3] = {0, 0, 0}, mag[3] = {0, 0, 0};
        double dsum[9] = {0};          /* sum_k H_jk: gives D[1] / D[e_l] */
        const long *gj = grid_index + j * dim;
        for (long k = 0; k < m; ++k) {
            const long *gk = grid_index + k * dim;
            double xi[3] = {0, 0, 0};
            int same_cell = 1;
            for (int a = 0; a < dim; ++a) {
                long d = gk[a] - gj[a];
                xi[a] = h * (double)d;
                if (d != 0) same_cell = 0;
            }
            double G[9], H[9];
            pair_blocks(kernel, nu, mu, h, xi, same_cell, k == j, weights[k], normals + k * dim, &cr, G, H);
            for (int a = 0; a < nc; ++a)
                for (int b = 0; b < nc; ++b) {
                    double uk = u[b * m + k], qk = q[b * m + k];
                    acc[a] += H[a * nc + b] * uk - G[a * nc + b] * qk;
                    mag[a] += fabs(H[a * nc + b] * uk) + fabs(G[a * nc + b] * qk);
                    dsum[a * nc + b] += H[a * nc + b];
                }
        }
        double C[9] = {0};
        if (kernel == ORC_HALFSPACE) { /* r = K[sigma] - u */
            for (int a = 0; a < nc; ++a) C[a * nc + a] = -1.0;
        } else if (cmode == ORC_C_HALF) {
            for (int a = 0; a < nc; ++a) C[a * nc + a] = 0.5;
        } else if (cmode == ORC_C_USER) {
            for (int i = 0; i < nc * nc; ++i) C[i] = cuser[j * nc * nc + i];
        } else {
            for (int i = 0; i < nc * nc; ++i) C[i] = -dsum[i];
        }
        for (int a = 0; a < nc; ++a) {
            double cu = 0.0;
            for (int b = 0; b < nc; ++b) cu += C[a * nc + b] * u[b * m + j];
            r[a * nt + (j - t0)] = cu + acc[a];
            if (scale) scale[a * nt + (j - t0)] = fabs(cu) + mag[a];
        }
        if (c_out)
            for (int i = 0; i < nc * nc; ++i) c_out[(j - t0) * nc * nc + i] = C[i];
    }
    return 0;
}

/*
 * The representation formula away from the nodes (eq. 4 / eq. 8 with the
 * free term c = 1 for points inside the boundary and c = 0 outside, Sec. 2):
 *
 *     v(p) = S[q](p) - D[u](p) = sum_k G(p_k - p) w_k q_k - H(p_k - p; n_k) w_k u_k
 *
 * at arbitrary grid points p = origin + h g (Sec. 4: the inverse transform
 * gives the convolution on the whole grid, not only at the nodes).  Inside
 * a closed boundary carrying a consistent pair (u, q) this is the field u(p);
 * outside it is 0.  A node k whose grid point coincides with p enters with
 * the grid's value at offset 0 (single layer) and 0 (double layer) -- the
 * plain grid sum, without the free term or the exact self term of the apply.
 *
 * pts: [npts][dim] grid indices of the targets.  out, scale (optional):
 * [ncomp][npts]; scale = sum |G w q| + |H w u|, the magnitude of the terms
 * that cancel in v, for normwise tolerances.
 */
int orc_volume(int kernel, double nu, double mu, double h, long m, const long *grid_index,
               const double *normals, const double *weights, const double *q, const double *u,
               long npts, const long *pts, double *out, double *scale, int cq, const double *cx,
               const double *cw)
{
    cell_rule cr = {cq, cx, cw};
    int dim = dim_of(kernel);
    int nc = ncomp_of(kernel);
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < npts; ++t) {
        double acc[3] = {0, 0, 0}, mag[3] = {0, 0, 0};
        const long *gt = pts + t * dim;
        for (long k = 0; k < m; ++k) {
            const long *gk = grid_index + k * dim;
            double xi[3] = {0, 0, 0};
            int same_cell = 1;
            for (int a = 0; a < dim; ++a) {
                long d = gk[a] - gt[a];
                xi[a] = h * (double)d;
                if (d != 0) same_cell = 0;
            }
            double G[9], H[9];
            pair_blocks(kernel, nu, mu, h, xi, same_cell, 0, weights[k], normals + k * dim, &cr, G, H);
            for (int a = 0; a < nc; ++a)
                for (int b = 0; b < nc; ++b) {
                    acc[a] += G[a * nc + b] * q[b * m + k] - H[a * nc + b] * u[b * m + k];
                    mag[a] += fabs(G[a * nc + b] * q[b * m + k]) + fabs(H[a * nc + b] * u[b * m + k]);
                }
        }
        for (int a = 0; a < nc; ++a) {
            out[a * npts + t] = acc[a];
            if (scale) scale[a * npts + t] = mag[a];
        }
    }
    return 0;
}

/*
 * Dense matrices of the discrete operator for small problems:
 * S and D are (nc*m) x (nc*m), row/column index = component * m + node, so
 * that r = C u + D u - S q with SoA vectors.  C (implicit) is returned in
 * c_out as m * nc * nc blocks.
 */
int orc_assemble(int kernel, double nu, double mu, double h, long m, const long *grid_index,
                 const double *normals, const double *weights, double *S, double *D, double *c_implicit,
                 int cq, const double *cx, const double *cw)
{
    cell_rule cr = {cq, cx, cw};
    int dim = dim_of(kernel);
    int nc = ncomp_of(kernel);
    long ld = nc * m;
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < m; ++j) {
        double dsum[9] = {0};
        const long *gj = grid_index + j * dim;
        for (long k = 0; k < m; ++k) {
            const long *gk = grid_index + k * dim;
            double xi[3] = {0, 0, 0};
            int same_cell = 1;
            for (int a = 0; a < dim; ++a) {
                long d = gk[a] - gj[a];
                xi[a] = h * (double)d;
                if (d != 0) same_cell = 0;
            }
            double G[9], H[9];
            pair_blocks(kernel, nu, mu, h, xi, same_cell, k == j, weights[k], normals + k * dim, &cr, G, H);
            for (int a = 0; a < nc; ++a)
                for (int b = 0; b < nc; ++b) {
                    S[(a * m + j) * ld + b * m + k] = G[a * nc + b];
                    D[(a * m + j) * ld + b * m + k] = H[a * nc + b];
                    dsum[a * nc + b] += H[a * nc + b];
                }
        }
        if (c_implicit)
            for (int i = 0; i < nc * nc; ++i) c_implicit[j * nc * nc + i] = -dsum[i];
    }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
