// api.hip -- plan creation, the apply entry point and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "volume_impl.hpp"
#include "fft_device.hpp"
#include "internal.hpp"
#include "kinds.hpp"

namespace bemfft {

namespace {
thread_local std::string g_last_error;
constexpr double kPi = 3.141592653589793238462643383279502884;
const int64_t kSizes[] = {32, 64, 96, 128, 192, 256, 320, 384, 512, 1024};  // 1024: 2D only
// A grid row holding this many nodes is x-transformed by FFT.
constexpr int kDenseRow = 24;
// When no other row holds more than this many nodes, the forward direct DFT
// takes two kx per thread (each node load serves both; measured on the
// 128^3 cube: 42 -> 38 us).  Plans with busier short rows keep one kx per
// thread, whose work per thread is then balanced better (the sphere).
constexpr int kFewNodesRow = 4;
// The long rows' inverse x transform goes through a row FFT (one more launch,
// a few microseconds) when the per-node sums it replaces exceed this many
// complex products: the nodes of long rows x Hx x outputs.  Measured: the
// 128^3 cube (3e6) is faster without it, the 256^2 half-space surface (5e7)
// 1.4x faster with it.
constexpr double kRowInvWork = 8.0e6;

template <typename T>
int dev_upload(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    if (src.empty()) return 0;
    if (hipMalloc(dst, src.size() * sizeof(T)) != hipSuccess) {
        set_error("hipMalloc failed");
        return BEMFFT_ENOMEM;
    }
    BF_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return 0;
}

void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

// Flat-panel self integrals of the single-layer kernel over a node's own
// measure w (straight segment in 2D, square in 3D), and the grid value at
// offset 0 (the same integral for the reference measure h^(d-1), per unit
// measure; Navier: orientation averaged).  O x O blocks, row-major.
void self_blocks(int kernel, double w, const double n[3], double h, double nu, double mu, double *self,
                 double *k0w) {
    const double l = std::log(1.0 + std::sqrt(2.0));
    if (kernel == BEMFFT_LAPLACE2D) {
        self[0] = w * (1.0 - std::log(0.5 * w)) / (2.0 * kPi);
        k0w[0] = w * (1.0 - std::log(0.5 * h)) / (2.0 * kPi);
        return;
    }
    if (kernel == BEMFFT_LAPLACE3D) {
        self[0] = std::sqrt(w) * l / kPi;
        k0w[0] = w * l / (kPi * h);
        return;
    }
    if (kernel == BEMFFT_HALFSPACE) {
        // the apply is r = K[sigma] - u, i.e. "S" = -K: blocks of -K over the
        // node's own square of area w (int 1/r = 4 s ln(1 + sqrt 2) for side s,
        // int x^2/r^3 = half of it) and over the reference cell h x h
        const double g = 1.0 / (2.0 * kPi * mu);
        const double a = 4.0 * std::sqrt(w) * l * g, aref = 4.0 * l / h * w * g;
        const double dg[3] = {1.0 - 0.5 * nu, 1.0 - 0.5 * nu, 1.0 - nu};
        for (int i = 0; i < 9; ++i) self[i] = k0w[i] = 0.0;
        for (int k = 0; k < 3; ++k) {
            self[4 * k] = -a * dg[k];
            k0w[4 * k] = -aref * dg[k];
        }
        return;
    }
    const double pre = 1.0 / (16.0 * kPi * mu * (1.0 - nu));
    const double i1 = 4.0 * std::sqrt(w) * l;
    const double i1ref = 4.0 * l / h;  // per unit measure
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
            const double d = (k == j) ? 1.0 : 0.0;
            self[3 * k + j] = pre * i1 * ((3.0 - 4.0 * nu) * d + 0.5 * (d - n[k] * n[j]));
            k0w[3 * k + j] = pre * i1ref * w * ((3.0 - 4.0 * nu) + 1.0 / 3.0) * d;
        }
}

template <typename R>
std::vector<cx<R>> twiddle_table(int64_t p) {
    std::vector<cx<R>> t(p);
    for (int64_t i = 0; i < p; ++i) {
        ctrig::CS w = ctrig::cs2pi(i, p);
        t[i] = {(R)w.c, (R)(-w.s)};
    }
    return t;
}

int64_t auto_pad(int64_t n) {
    for (int64_t s : kSizes)
        if (s >= 2 * n) return s;
    return -1;
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

void free_engine(Engine *e) {
    dev_free(e->spec);
    dev_free(e->twx);
    dev_free(e->twy);
    dev_free(e->twz);
    dev_free(e->Y);
    dev_free(e->Z);
    dev_free(e->vf);
    dev_free(e->Xd);
    *e = Engine{};
}

template <typename R>
static int upload_tw(Engine *e, const bemfft_plan *p) {
    cx<R> *d = nullptr;
    BF_CHECK(dev_upload(&d, twiddle_table<R>(p->P[0])));
    e->twx = d;
    BF_CHECK(dev_upload(&d, twiddle_table<R>(p->P[1])));
    e->twy = d;
    BF_CHECK(dev_upload(&d, twiddle_table<R>(p->P[2])));
    e->twz = d;
    return 0;
}

int upload_twiddles(Engine *e, const bemfft_plan *p) {
    return e->precision == BEMFFT_FP64 ? upload_tw<double>(e, p) : upload_tw<float>(e, p);
}

int alloc_workspace(bemfft_plan *p, Engine *e) {
    BF_CHECK(alloc_intermediates(p, e->precision, e));
    // 16-bit spectra: kz rows padded to a multiple of 8 values (16-byte runs)
    e->hzs = e->precision == BEMFFT_BF16_MFMA ? (p->H[2] + 7) / 8 * 8 : p->H[2];
    const size_t spec = (size_t)p->K * p->H[0] * p->H[1] * e->hzs * e->sreal;
    if (hipMalloc(&e->spec, spec) != hipSuccess) {
        set_error("hipMalloc of the spectra failed");
        return BEMFFT_ENOMEM;
    }
    e->bytes += spec;
    return 0;
}

void fill_apply_args(const bemfft_plan *p, const Engine &e, const Engine &ws, ApplyArgs *out) {
    ApplyArgs a{};
    a.nx = (int)p->n[0];
    a.ny = (int)p->n[1];
    a.nz = (int)p->n[2];
    a.px = (int)p->P[0];
    a.py = (int)p->P[1];
    a.pz = (int)p->P[2];
    a.hx = (int)p->H[0];
    a.hy = (int)p->H[1];
    a.hz = (int)p->H[2];
    a.hzs = (int)e.hzs;
    a.z0 = (int)p->z0;
    a.nzo = (int)p->nzo;
    a.m = (int)p->m;
    a.gx = p->d_gx;
    a.gy = p->d_gy;
    a.gz = p->d_gz;
    a.rowptr = p->d_rowptr;
    a.perm = p->d_perm;
    a.w = p->d_w;
    a.nrm = p->d_nrm;
    a.C = p->d_C;
    a.SC = p->d_SC;
    a.spec = e.spec;
    a.twx = e.twx;
    a.twy = e.twy;
    a.twz = e.twz;
    a.Y = ws.Y;
    a.Z = ws.Z;
    a.vf = ws.vf;
    a.Xd = ws.Xd;
    a.row_dense = p->d_row_dense;
    a.dense_rows = p->d_dense_rows;
    a.nd = (int)p->nd;
    a.row_inv = p->row_inv;
    a.fwd_xg = p->fwd_xg;
    a.zsched = p->zsched;
    a.off = 0;
    a.gid = 0;
    *out = a;
}

int alloc_intermediates(const bemfft_plan *p, int precision, Engine *e) {
    e->precision = precision;
    e->creal = precision == BEMFFT_FP64 ? 8 : 4;
    e->sreal = precision == BEMFFT_FP64 ? 8 : (precision == BEMFFT_FP32 ? 4 : 2);
    const size_t cb = 2 * e->creal, sb = 2 * e->sreal;
    const size_t rows = (size_t)p->H[0] * p->nzo * p->P[1];
    // Y also holds the inverse y pass's rows in the arithmetic precision:
    // O nzo ny Hx complex values, never more than F Hx nzo Py stored ones
    const size_t ysz = std::max((size_t)p->F * rows * sb, (size_t)p->O * p->nzo * p->n[1] * p->H[0] * cb);
    const size_t zsz = (size_t)p->O * rows * sb;
    const size_t vsz = (size_t)p->F * p->m * e->creal;
    const size_t xsz = std::max<size_t>(1, (size_t)p->nd * p->F * p->H[0] * cb);
    if (hipMalloc(&e->Y, ysz) != hipSuccess || hipMalloc(&e->Z, zsz) != hipSuccess ||
        hipMalloc(&e->vf, vsz) != hipSuccess || hipMalloc(&e->Xd, xsz) != hipSuccess) {
        set_error("hipMalloc of the intermediates failed");
        return BEMFFT_ENOMEM;
    }
    e->bytes = ysz + zsz + vsz + xsz;
    return 0;
}

int launch_apply(bemfft_plan *p, const Engine &e, const double *q, const double *u, double *r, hipStream_t st,
                 hipEvent_t *ev) {
    ApplyArgs a;
    fill_apply_args(p, e, e, &a);
    a.q = q;
    a.u = u;
    a.r = r;
    if (p->kernel == 0) return apply_kind<0>(e.precision, a, st, ev);
    if (p->kernel == 1) return apply_kind<1>(e.precision, a, st, ev);
    if (p->kernel == 3) return apply_kind<3>(e.precision, a, st, ev);
    return apply_kind<2>(e.precision, a, st, ev);
}

}  // namespace bemfft

using namespace bemfft;

namespace {

void destroy_plan_state(bemfft_plan *p) {
    free_engine(&p->eng);
    free_engine(&p->eng64);
    dev_free(p->d_gx);
    dev_free(p->d_gy);
    dev_free(p->d_gz);
    dev_free(p->d_perm);
    dev_free(p->d_rowptr);
    dev_free(p->d_w);
    dev_free(p->d_nrm);
    dev_free(p->d_C);
    dev_free(p->d_SC);
    dev_free(p->d_row_dense);
    dev_free(p->d_dense_rows);
    dev_free(p->s_V);
    dev_free(p->s_vec);
    dev_free(p->s_red);
    dev_free(p->s_hbuf);
    if (p->h_pinned) (void)hipHostFree(p->h_pinned);
}

// Implicit free term: c_j = -D[1]_j (Laplace), C_j = -[D e_1, D e_2, D e_3]_j
// (Navier), from the FP64 operator with c = 0 and q = 0.
int implicit_free_term(bemfft_plan *p, const Engine &e64, hipStream_t st, std::vector<double> &Cs) {
    const int64_t m = p->m;
    const int nc = p->ncomp;
    double *q = nullptr, *u = nullptr, *r = nullptr;
    const size_t bytes = (size_t)nc * m * sizeof(double);
    if (hipMalloc(&q, bytes) != hipSuccess || hipMalloc(&u, bytes) != hipSuccess || hipMalloc(&r, bytes) != hipSuccess) {
        dev_free(q);
        dev_free(u);
        dev_free(r);
        set_error("hipMalloc failed");
        return BEMFFT_ENOMEM;
    }
    std::vector<int> perm(m);
    int status = 0;
    std::vector<double> hu((size_t)nc * m), hr((size_t)nc * m);
    Cs.assign((size_t)m * nc * nc, 0.0);
    if (hipMemcpy(perm.data(), p->d_perm, m * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemsetAsync(q, 0, bytes, st) != hipSuccess)
        status = BEMFFT_EDEVICE;
    for (int l = 0; l < nc && status == 0; ++l) {
        std::fill(hu.begin(), hu.end(), 0.0);
        std::fill(hu.begin() + (size_t)l * m, hu.begin() + (size_t)(l + 1) * m, 1.0);
        if (hipMemcpyAsync(u, hu.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess) { status = BEMFFT_EDEVICE; break; }
        status = launch_apply(p, e64, q, u, r, st);
        if (status) break;
        if (hipMemcpyAsync(hr.data(), r, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) { status = BEMFFT_EDEVICE; break; }
        for (int64_t s = 0; s < m; ++s)
            for (int k = 0; k < nc; ++k) Cs[((size_t)s * nc + k) * nc + l] = -hr[(size_t)k * m + perm[s]];
    }
    dev_free(q);
    dev_free(u);
    dev_free(r);
    if (status == BEMFFT_EDEVICE) set_error("implicit free term: HIP failure");
    return status;
}

int autotune_zsched(bemfft_plan *p, hipStream_t st);
int num_zsched(const bemfft_plan *p);
int default_zsched(const bemfft_plan *p);

int plan_create_impl(bemfft_plan *p, const bemfft_grid *grid, int64_t m, const double *nodes,
                     const double *normals, const double *weights, int kernel, double nu, double mu,
                     const bemfft_plan_opts *opts) {
    auto t0 = std::chrono::steady_clock::now();
    if (kernel < 0 || kernel > 3) { set_error("unknown kernel"); return BEMFFT_EINVAL; }
    const bool halfspace = kernel == BEMFFT_HALFSPACE;
    KindInfo ki = kind_info(kernel);
    if (grid->dim != ki.dim) { set_error("grid dimension does not match the kernel"); return BEMFFT_EINVAL; }
    // kernels index the [F][m] field and [O][m] node arrays with 32-bit products
    // (f * m + s, with F up to 9), and the plan sorts with 32-bit node indices
    const int64_t m_max = (int64_t)INT32_MAX / std::max(ki.F, 3);
    if (m < 1 || m > m_max) {
        set_error("node count out of range [1, " + std::to_string(m_max) + "]");
        return BEMFFT_EINVAL;
    }
    if (!nodes || (!normals && !halfspace)) { set_error("nodes and normals are required"); return BEMFFT_EINVAL; }
    if (!(grid->h > 0.0) || !std::isfinite(grid->h)) { set_error("grid spacing must be positive"); return BEMFFT_EINVAL; }
    if ((kernel == BEMFFT_NAVIER3D || halfspace) && (!(nu > -1.0 && nu < 0.5) || !(mu > 0.0))) {
        set_error("elasticity needs nu in (-1, 1/2) and mu > 0");
        return BEMFFT_EINVAL;
    }
    const int prec = opts ? (int)opts->precision : BEMFFT_FP64;
    const int cmode = opts ? (int)opts->c_mode : BEMFFT_C_IMPLICIT;
    if (prec != BEMFFT_FP64 && prec != BEMFFT_FP32 && prec != BEMFFT_BF16_MFMA) {
        set_error("unknown precision");
        return BEMFFT_EINVAL;
    }
    if (prec == BEMFFT_BF16_MFMA && ki.dim != 3) {
        set_error("the 16-bit form runs the z transforms on the matrix cores: 3D plans only");
        return BEMFFT_EINVAL;
    }
    if (cmode < 0 || cmode > 2) { set_error("unknown c_mode"); return BEMFFT_EINVAL; }
    if (cmode == BEMFFT_C_USER && !(opts && opts->c_user)) { set_error("C_USER needs c_user"); return BEMFFT_EINVAL; }
    if (opts && (opts->autotune < 0 || opts->autotune > 4)) { set_error("autotune must be in [0, 4]"); return BEMFFT_EINVAL; }
    const int cell_quad = opts ? opts->cell_quad : 0;
    if (cell_quad < 0 || cell_quad > 8) { set_error("cell_quad must be in [0, 8]"); return BEMFFT_EINVAL; }
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    const int d = ki.dim;
    p->dim = d;
    p->kernel = kernel;
    p->cmode = cmode;
    p->ncomp = ki.ncomp;
    p->F = ki.F;
    p->K = ki.K;
    p->O = ki.O;
    p->m = m;
    p->h = grid->h;
    p->nu = nu;
    p->mu = mu;
    p->cell_quad = cell_quad;
    for (int a = 0; a < 3; ++a) {
        p->origin[a] = a < d ? grid->origin[a] : 0.0;
        p->n[a] = a < d ? grid->n[a] : 1;
        const int64_t nmax = d == 2 ? 512 : 256;  // padded lengths up to 1024 (2D) / 512 (3D)
        if (p->n[a] < 1 || p->n[a] > nmax) {
            set_error("grid size per axis must be in [1, " + std::to_string(nmax) + "]");
            return BEMFFT_EINVAL;
        }
        if (a < d) {
            int64_t pad = grid->pad[a] ? grid->pad[a] : auto_pad(p->n[a]);
            if (pad < 2 * p->n[a] - 1 || !fft_size_supported(pad) || pad == 1 || (d == 3 && pad > 512)) {
                set_error("padded length " + std::to_string(pad) + " on axis " + std::to_string(a) +
                          " is unsupported or shorter than 2n-1");
                return BEMFFT_EUNSUPPORTED;
            }
            p->P[a] = pad;
            p->H[a] = pad / 2 + 1;
        } else {
            p->P[a] = 1;
            p->H[a] = 1;
        }
    }
    // snap, validate
    std::vector<int> g((size_t)m * 3, 0);
    std::vector<double> w(m), nr((size_t)m * 3, 0.0);
    for (int64_t j = 0; j < m; ++j) {
        for (int a = 0; a < d; ++a) {
            const double x = nodes[j * d + a];
            const double nv = normals ? normals[j * d + a] : 0.0;
            if (!std::isfinite(x) || !std::isfinite(nv)) { set_error("non-finite node or normal"); return BEMFFT_EINVAL; }
            const double gi = std::floor((x - p->origin[a]) / p->h + 0.5);
            if (gi < 0.0 || gi >= (double)p->n[a]) {
                set_error("node " + std::to_string(j) + " lies outside the grid");
                return BEMFFT_EINVAL;
            }
            g[j * 3 + a] = (int)gi;
            nr[j * 3 + a] = nv;
        }
        // default measure: the grid's line or surface element (the half-space
        // grid is the surface itself: h^2)
        w[j] = weights ? weights[j] : (halfspace ? p->h * p->h : std::pow(p->h, d - 1));
        if (!(w[j] > 0.0) || !std::isfinite(w[j])) { set_error("weights must be positive and finite"); return BEMFFT_EINVAL; }
    }
    // sort by (z, y, x): rows of the grid become contiguous runs
    std::vector<int> perm(m);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
        if (g[a * 3 + 2] != g[b * 3 + 2]) return g[a * 3 + 2] < g[b * 3 + 2];
        if (g[a * 3 + 1] != g[b * 3 + 1]) return g[a * 3 + 1] < g[b * 3 + 1];
        return g[a * 3] < g[b * 3];
    });
    const int zlo = g[perm[0] * 3 + 2], zhi = g[perm[m - 1] * 3 + 2];
    p->z0 = zlo;
    p->nzo = zhi - zlo + 1;
    const int64_t ny = p->n[1];
    std::vector<int> rowptr((size_t)p->nzo * ny + 1, 0);
    std::vector<int> sgx(m), sgy(m), sgz(m);
    std::vector<double> sw(m), snr((size_t)3 * m);
    for (int64_t s = 0; s < m; ++s) {
        const int j = perm[s];
        sgx[s] = g[j * 3];
        sgy[s] = g[j * 3 + 1];
        sgz[s] = g[j * 3 + 2];
        sw[s] = w[j];
        for (int a = 0; a < 3; ++a) snr[a * m + s] = nr[j * 3 + a];
        rowptr[(size_t)(sgz[s] - zlo) * ny + sgy[s] + 1] += 1;
    }
    for (size_t i = 1; i < rowptr.size(); ++i) rowptr[i] += rowptr[i - 1];
    // long rows get their x-transform from a row FFT
    std::vector<int> row_dense((size_t)p->nzo * ny, -1), dense_rows;
    for (int64_t z = 0; z < p->nzo; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            const int64_t row = z * ny + y;
            if (rowptr[row + 1] - rowptr[row] >= kDenseRow) {
                row_dense[row] = (int)dense_rows.size();
                dense_rows.push_back((int)row);
            }
        }
    }
    p->nd = (int64_t)dense_rows.size();
    {
        int64_t busiest = 0;  // nodes of the busiest row that is not a long row
        for (size_t row = 0; row + 1 < rowptr.size(); ++row) {
            const int64_t c = rowptr[row + 1] - rowptr[row];
            if (c < kDenseRow) busiest = std::max(busiest, c);
        }
        p->fwd_xg = busiest <= kFewNodesRow ? 2 : 1;
    }
    {
        int64_t long_nodes = 0;
        for (int r : dense_rows) long_nodes += rowptr[r + 1] - rowptr[r];
        p->row_inv = (double)long_nodes * (double)p->H[0] * p->O > kRowInvWork ? 1 : 0;
    }
    // per-node free term and self correction blocks (sorted order)
    const int O = p->O;
    std::vector<double> C((size_t)m * O * O, 0.0), SC((size_t)m * O * O, 0.0);
    p->h_diag_dir.assign((size_t)O * m, 0.0);
    p->h_self.assign((size_t)O * O * m, 0.0);
    for (int64_t s = 0; s < m; ++s) {
        double self[9], k0w[9], n3[3] = {snr[s], snr[m + s], snr[2 * m + s]};
        self_blocks(kernel, sw[s], n3, p->h, nu, mu, self, k0w);
        for (int i = 0; i < O * O; ++i) SC[(size_t)s * O * O + i] = self[i] - k0w[i];
        for (int i = 0; i < O * O; ++i) p->h_self[(size_t)perm[s] * O * O + i] = self[i];
        for (int k = 0; k < O; ++k) p->h_diag_dir[(size_t)k * m + perm[s]] = -self[k * O + k];
    }
    int st_ = 0;
    st_ = dev_upload(&p->d_gx, sgx);
    if (!st_) st_ = dev_upload(&p->d_gy, sgy);
    if (!st_) st_ = dev_upload(&p->d_gz, sgz);
    if (!st_) st_ = dev_upload(&p->d_perm, perm);
    if (!st_) st_ = dev_upload(&p->d_rowptr, rowptr);
    if (!st_) st_ = dev_upload(&p->d_w, sw);
    if (!st_) st_ = dev_upload(&p->d_nrm, snr);
    if (!st_) st_ = dev_upload(&p->d_SC, SC);
    if (!st_) st_ = dev_upload(&p->d_C, C);  // zero until set below
    if (!st_) st_ = dev_upload(&p->d_row_dense, row_dense);
    if (!st_ && !dense_rows.empty()) st_ = dev_upload(&p->d_dense_rows, dense_rows);
    BF_CHECK(st_);
    // spectra in FP64, and the working-precision engine
    Engine e64;
    e64.precision = BEMFFT_FP64;
    e64.creal = 8;
    e64.sreal = 8;
    int status = alloc_workspace(p, &e64);
    if (!status) status = upload_twiddles(&e64, p);
    if (!status) status = build_spectra(p, &e64, nullptr, st);
    if (status) { free_engine(&e64); return status; }
    // free term
    std::vector<double> Cs;
    if (halfspace) {  // r = K[sigma] - u for every mode
        Cs.assign((size_t)m * O * O, 0.0);
        for (int64_t s = 0; s < m; ++s)
            for (int k = 0; k < O; ++k) Cs[((size_t)s * O + k) * O + k] = -1.0;
    } else if (cmode == BEMFFT_C_IMPLICIT) {
        status = implicit_free_term(p, e64, st, Cs);
        if (status) { free_engine(&e64); return status; }
    } else {
        Cs.assign((size_t)m * O * O, 0.0);
        for (int64_t s = 0; s < m; ++s)
            for (int k = 0; k < O; ++k)
                for (int l = 0; l < O; ++l) {
                    double v;
                    if (cmode == BEMFFT_C_HALF) v = (k == l) ? 0.5 : 0.0;
                    else v = opts->c_user[(size_t)perm[s] * O * O + k * O + l];
                    if (!std::isfinite(v)) { free_engine(&e64); set_error("non-finite c_user"); return BEMFFT_EINVAL; }
                    Cs[((size_t)s * O + k) * O + l] = v;
                }
    }
    if (hipMemcpy(p->d_C, Cs.data(), Cs.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        free_engine(&e64);
        set_error("upload of c failed");
        return BEMFFT_EDEVICE;
    }
    p->h_c.assign((size_t)m * O * O, 0.0);
    p->h_diag_neu.assign((size_t)O * m, 0.0);
    for (int64_t s = 0; s < m; ++s) {
        for (int i = 0; i < O * O; ++i) p->h_c[(size_t)perm[s] * O * O + i] = Cs[(size_t)s * O * O + i];
        for (int k = 0; k < O; ++k) p->h_diag_neu[(size_t)k * m + perm[s]] = Cs[((size_t)s * O + k) * O + k];
    }
    if (prec == BEMFFT_FP64) {
        p->eng = e64;
        p->has64 = true;
    } else {
        Engine e32;  // FP32 or 16-bit working engine
        e32.precision = prec;
        status = alloc_workspace(p, &e32);  // sets the element sizes
        if (!status) status = upload_twiddles(&e32, p);
        if (!status) {
            // the FP64 spectra rounded once to the stored precision, on the device
            const int64_t hz = p->H[2], rows = (int64_t)p->K * p->H[0] * p->H[1];
            status = convert_spectra(static_cast<const double *>(e64.spec), &e32, rows, hz, st);
            if (!status && hipStreamSynchronize(st) != hipSuccess) {
                set_error("spectrum conversion failed");
                status = BEMFFT_EDEVICE;
            }
        }
        if (status == 0 && opts && opts->keep_fp64) {
            p->eng64 = e64;  // the refinement's FP64 operator
            p->has64 = true;
        } else {
            free_engine(&e64);
        }
        if (status) { free_engine(&e32); free_engine(&p->eng64); p->has64 = false; return status; }
        p->eng = e32;
    }
    if (hipStreamSynchronize(st) != hipSuccess) { set_error("plan: stream sync failed"); return BEMFFT_EDEVICE; }
    const int tune = opts ? opts->autotune : 0;
    // the 16-bit z pass has one schedule (its transforms are matrix products)
    if (p->dim == 3 && prec != BEMFFT_BF16_MFMA) {
        p->zsched = default_zsched(p);
        if (tune >= 2 && tune - 2 < num_zsched(p)) p->zsched = tune - 2;
        else if (tune == 1) BF_CHECK(autotune_zsched(p, st));
    }
    p->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

// Cache entries hold zsched + 4 (fwd_xg - 1); the "2:" prefix keeps entries
// written before the forward width was tuned (z schedule only) from being read.
std::string tune_key(const bemfft_plan *p) {
    return "2:" + std::to_string(p->kernel) + ":" + std::to_string(p->eng.precision) + ":" + std::to_string(p->P[0]) +
           "x" + std::to_string(p->P[1]) + "x" + std::to_string(p->P[2]);
}

// Compiled z schedules of a plan: the default and the alternative one, and
// for the Navier family the wide one where the length has it.
int num_zsched(const bemfft_plan *p) {
    return (p->kernel == BEMFFT_NAVIER3D && has_wide_sched((int)p->P[2])) ? 3 : 2;
}

// Schedule used without autotuning, from z-pass times measured on MI355X
// (Navier spheres and stars, median of single applies).  Navier keeps three
// output transforms live per pencil, so its fastest schedule depends on the
// precision and the length:
//   P = 256: FP32 16-lane 196 us (wide 240, 32-lane 347), FP64 32-lane 343 us
//            (wide 499, 16-lane 933);
//   P = 384: FP32 32-lane 0.76 ms (wide 1.06, 16-lane 2.64),
//            FP64 wide 1.86 ms (32-lane 3.67, 16-lane 3.69);
//   P = 512: FP32 32-lane 1.50 ms (wide 2.57), FP64 wide 2.87 ms (32-lane 10.55).
// Other Navier lengths take the 32-lane schedule; Laplace keeps schedule 0.
int default_zsched(const bemfft_plan *p) {
    if (p->kernel != BEMFFT_NAVIER3D) return 0;
    const bool fp64 = p->eng.precision == BEMFFT_FP64;
    switch (p->P[2]) {
        case 256: return fp64 ? 1 : 0;
        case 384:
        case 512: return fp64 ? 2 : 1;
        default: return 1;
    }
}

int tune_cache_lookup(const std::string &key) {
    const char *path = std::getenv("BEMFFT_TUNE_CACHE");
    if (!path || !*path) return -1;
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char k[128];
    int v = -1, found = -1;
    while (std::fscanf(f, "%127s %d", k, &v) == 2)
        if (key == k) found = v;
    std::fclose(f);
    return (found >= 0 && found <= 2) ? found : -1;
}

void tune_cache_store(const std::string &key, int v) {
    const char *path = std::getenv("BEMFFT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", key.c_str(), v);
    std::fclose(f);
}

// Time the working-precision apply with each compiled z schedule and keep
// the fastest, then, with that schedule, the other number of kx per thread
// in the forward direct DFT (1 or 2) and keep the faster.
int autotune_zsched(bemfft_plan *p, hipStream_t st) {
    const std::string key = tune_key(p);
    const int nsched = num_zsched(p);
    const int cached = tune_cache_lookup(key);
    if (cached >= 0 && cached % 4 < nsched && cached / 4 < 2) {
        p->zsched = cached % 4;
        p->fwd_xg = cached / 4 + 1;
        return 0;
    }
    const size_t bytes = (size_t)p->ncomp * p->m * sizeof(double);
    double *q = nullptr, *u = nullptr, *r = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc(&q, bytes) != hipSuccess || hipMalloc(&u, bytes) != hipSuccess || hipMalloc(&r, bytes) != hipSuccess) {
        dev_free(q);
        dev_free(u);
        dev_free(r);
        set_error("autotune: allocation failed");
        return BEMFFT_ENOMEM;
    }
    std::vector<double> ones((size_t)p->ncomp * p->m, 1.0);
    int status = 0;
    if (hipMemcpy(q, ones.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(u, ones.data(), bytes, hipMemcpyHostToDevice) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        status = BEMFFT_EDEVICE;
    const int reps = 20;
    // mean apply time in us with the plan's current settings
    auto time_apply = [&](double *us) {
        for (int i = 0; i < 3 && status == 0; ++i) status = launch_apply(p, p->eng, q, u, r, st);
        if (status) return;
        if (hipEventRecord(e0, st) != hipSuccess) { status = BEMFFT_EDEVICE; return; }
        for (int i = 0; i < reps && status == 0; ++i) status = launch_apply(p, p->eng, q, u, r, st);
        float ms = 0.f;
        if (status == 0 && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            status = BEMFFT_EDEVICE;
        *us = 1e3 * ms / reps;
    };
    for (int sched = 0; sched < nsched && status == 0; ++sched) {
        p->zsched = sched;
        time_apply(&p->tune_us[sched]);
    }
    if (status == 0) {
        p->zsched = 0;
        for (int sched = 1; sched < nsched; ++sched)
            if (p->tune_us[sched] < p->tune_us[p->zsched]) p->zsched = sched;
    }
    // the width in use was timed with every schedule above; only the other one
    // needs applies of its own
    if (status == 0) {
        const int xg0 = p->fwd_xg, xg1 = 3 - xg0;
        p->fwd_tune_us[xg0 - 1] = p->tune_us[p->zsched];
        p->fwd_xg = xg1;
        time_apply(&p->fwd_tune_us[xg1 - 1]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free(q);
    dev_free(u);
    dev_free(r);
    if (status) {
        if (status == BEMFFT_EDEVICE) set_error("autotune: HIP failure");
        return status;
    }
    p->fwd_xg = p->fwd_tune_us[1] < p->fwd_tune_us[0] ? 2 : 1;
    tune_cache_store(key, p->zsched + 4 * (p->fwd_xg - 1));
    return 0;
}

}  // namespace

extern "C" {

int bemfft_plan_create(bemfft_plan **out, const bemfft_grid *grid, int64_t m, const double *nodes,
                       const double *normals, const double *weights, int kernel, double nu, double mu,
                       const bemfft_plan_opts *opts) {
    if (!out || !grid) {
        set_error("out and grid must be non-null");
        return BEMFFT_EINVAL;
    }
    *out = nullptr;
    bemfft_plan *p = new (std::nothrow) bemfft_plan();
    if (!p) {
        set_error("host allocation failed");
        return BEMFFT_ENOMEM;
    }
    int st = plan_create_impl(p, grid, m, nodes, normals, weights, kernel, nu, mu, opts);
    if (st) {
        destroy_plan_state(p);
        delete p;
        return st;
    }
    *out = p;
    return 0;
}

int bemfft_apply(bemfft_plan *p, const double *q, const double *u, double *r, void *stream) {
    if (!p || !q || !u || !r) {
        set_error("apply: null argument");
        return BEMFFT_EINVAL;
    }
    return launch_apply(p, p->eng, q, u, r, (hipStream_t)stream);
}

int bemfft_apply_profile(bemfft_plan *p, const double *q, const double *u, double *r, int reps,
                         double *stage_ms, void *stream) {
    if (!p || !q || !u || !r || !stage_ms || reps < 1) {
        set_error("apply_profile: bad argument");
        return BEMFFT_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[5];
    for (int i = 0; i < 5; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
            set_error("hipEventCreate failed");
            return BEMFFT_EDEVICE;
        }
    double acc[4] = {0, 0, 0, 0};
    int status = 0;
    for (int it = 0; it < reps && status == 0; ++it) {
        status = launch_apply(p, p->eng, q, u, r, st, ev);
        if (status) break;
        if (hipEventSynchronize(ev[4]) != hipSuccess) { status = BEMFFT_EDEVICE; break; }
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) { status = BEMFFT_EDEVICE; break; }
            acc[k] += ms;
        }
    }
    for (int i = 0; i < 5; ++i) (void)hipEventDestroy(ev[i]);
    if (status == BEMFFT_EDEVICE) set_error("apply_profile: HIP failure");
    for (int k = 0; k < 4; ++k) stage_ms[k] = acc[k] / reps;
    return status;
}

int bemfft_eval_grid(bemfft_plan *p, const double *q, const double *u, double *out, void *stream) {
    if (!p || !q || !u || !out) {
        set_error("eval_grid: null argument");
        return BEMFFT_EINVAL;
    }
    ApplyArgs a;
    fill_apply_args(p, p->eng, p->eng, &a);
    a.q = q;
    a.u = u;
    hipStream_t st = (hipStream_t)stream;
    if (p->kernel == 0) return volume_kind<0>(p->eng.precision, a, out, st, nullptr);
    if (p->kernel == 1) return volume_kind<1>(p->eng.precision, a, out, st, nullptr);
    if (p->kernel == 3) return volume_kind<3>(p->eng.precision, a, out, st, nullptr);
    return volume_kind<2>(p->eng.precision, a, out, st, nullptr);
}

int bemfft_plan_get_info(const bemfft_plan *p, bemfft_plan_info *info) {
    if (!p || !info) {
        set_error("null argument");
        return BEMFFT_EINVAL;
    }
    std::memset(info, 0, sizeof(*info));
    info->dim = p->dim;
    info->kernel = p->kernel;
    info->precision = p->eng.precision;
    info->c_mode = p->cmode;
    info->m = p->m;
    info->ncomp = p->ncomp;
    for (int a = 0; a < 3; ++a) {
        info->n[a] = p->n[a];
        info->pad[a] = p->P[a];
    }
    info->z_lo = p->z0;
    info->z_count = p->nzo;
    info->nfields = p->F;
    info->nspectra = p->K;
    info->noutputs = p->O;
    info->workspace_bytes = (int64_t)(p->eng.bytes + p->eng64.bytes);
    info->spectra_bytes = (int64_t)p->K * p->H[0] * p->H[1] * p->eng.hzs * (int64_t)p->eng.sreal;
    info->spectrum_parity_residual = p->parity_resid;
    info->plan_seconds = p->plan_seconds;
    info->zsched = p->zsched;
    for (int i = 0; i < 3; ++i) info->tune_us[i] = p->tune_us[i];
    info->fwd_xg = p->fwd_xg;
    for (int i = 0; i < 2; ++i) info->fwd_tune_us[i] = p->fwd_tune_us[i];
    return 0;
}

int bemfft_plan_get_c(const bemfft_plan *p, double *c_host) {
    if (!p || !c_host) {
        set_error("null argument");
        return BEMFFT_EINVAL;
    }
    std::memcpy(c_host, p->h_c.data(), p->h_c.size() * sizeof(double));
    return 0;
}

int bemfft_plan_destroy(bemfft_plan *p) {
    if (!p) return 0;
    destroy_plan_state(p);
    delete p;
    return 0;
}

int bemfft_fft3d_c2c_f64(double *data, int64_t px, int64_t py, int64_t pz, int direction, void *stream) {
    if (!data || (direction != 1 && direction != -1)) {
        set_error("fft3d: bad argument");
        return BEMFFT_EINVAL;
    }
    return fft3d_c2c_f64(data, px, py, pz, direction, (hipStream_t)stream);
}

const char *bemfft_strerror(int status) {
    switch (status) {
        case BEMFFT_OK: return "ok";
        case BEMFFT_EINVAL: return "invalid argument";
        case BEMFFT_ENOMEM: return "out of memory";
        case BEMFFT_EDEVICE: return "HIP runtime error";
        case BEMFFT_EUNSUPPORTED: return "unsupported size";
        case BEMFFT_EBREAKDOWN: return "breakdown (non-finite values)";
        case BEMFFT_ENOCONV: return "not converged within maxit";
        default: return "unknown status";
    }
}

const char *bemfft_last_error(void) { return g_last_error.c_str(); }

int bemfft_supported_sizes(int64_t *sizes, int cap) {
    int n = (int)(sizeof(kSizes) / sizeof(kSizes[0]));
    for (int i = 0; i < n && i < cap; ++i) sizes[i] = kSizes[i];
    return n;
}

}  // extern "C"
