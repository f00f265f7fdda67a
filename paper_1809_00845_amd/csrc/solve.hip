// solve.hip -- restarted GMRES for the mixed boundary-value problem.
//
// The paper obtains the unknown q "with a conjugate gradient method" in which
// the first integral is evaluated by the FFT like the others, iterating until
// the residual norm falls below a preset value (end of Sec. 4).  The operator
// of a mixed problem is not symmetric, so the iteration used here is GMRES
// with right Jacobi scaling; every matrix-vector product is one apply.
// Arnoldi uses classical Gram-Schmidt applied twice (two block reductions
// per step), all in FP64; the small Hessenberg problem is solved on the host
// with Givens rotations.  The true residual ||b - A x|| is recomputed with a
// fresh apply at every restart and at the end.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace bemfft {
namespace {

constexpr int kRedBlocks = 240;
constexpr int kRedThreads = 256;

// x_in -> (q, u) split by the flags: slot with bc = 0 has u known, so its
// unknown is q; bc = 1 has q known, unknown u.  scale (optional) multiplies x.
__global__ void k_split(const uint8_t *bc, const double *x, const double *scale, double *q, double *u,
                        int64_t n, int unknown_side) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = x[i] * (scale ? scale[i] : 1.0);
        bool qslot = (bc[i] == 0) == (unknown_side != 0);  // unknown: q where bc = 0
        q[i] = qslot ? v : 0.0;
        u[i] = qslot ? 0.0 : v;
    }
}

__global__ void k_axpby(double *y, const double *x, double a, double b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

__global__ void k_diag(const uint8_t *bc, const double *ddir, const double *dneu, double *dinv, int64_t n, int on) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d = bc[i] == 0 ? ddir[i] : dneu[i];
        dinv[i] = (on && d != 0.0 && isfinite(d)) ? 1.0 / d : 1.0;
    }
}

// partial[blk][j] = sum over this block's rows of V[j][i] w[i], j < nvec.
__global__ __launch_bounds__(kRedThreads) void k_mdot_partial(const double *V, int64_t ld, int nvec,
                                                              const double *w, int64_t n, double *partial) {
    __shared__ double sm[kRedThreads];
    for (int j0 = 0; j0 < nvec; j0 += 4) {
        double acc[4] = {0, 0, 0, 0};
        for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
            double wi = w[i];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j0 + k < nvec) acc[k] += V[(int64_t)(j0 + k) * ld + i] * wi;
        }
        for (int k = 0; k < 4 && j0 + k < nvec; ++k) {
            sm[threadIdx.x] = acc[k];
            __syncthreads();
            for (int s = kRedThreads / 2; s > 0; s >>= 1) {
                if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nvec + j0 + k] = sm[0];
            __syncthreads();
        }
    }
}

__global__ void k_mdot_final(const double *partial, int nblk, int nvec, double *out, int sqrt_last) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nvec) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * nvec + j];
    out[j] = (sqrt_last && j == nvec - 1) ? sqrt(s) : s;
}

// w[i] += sign * sum_j V[j][i] h[j]
__global__ void k_gemv(const double *V, int64_t ld, int nvec, const double *h, double *w, int64_t n, double sign) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < nvec; ++j) s += V[(int64_t)j * ld + i] * h[j];
        w[i] += sign * s;
    }
}

// v = w / norm, norm read from device memory
__global__ void k_normalize(const double *w, const double *norm, double *v, int64_t n) {
    double a = *norm;
    double inv = a > 0.0 ? 1.0 / a : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = w[i] * inv;
}

__global__ void k_mul(double *y, const double *a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] *= a[i];
}

int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

struct Ws {
    double *V, *b, *x, *w, *q, *u, *r, *dinv, *red, *hd;
    int cap;
};

int ensure_workspace(bemfft_plan *p, int restart, Ws &ws) {
    const int64_t n = (int64_t)p->ncomp * p->m;
    if (p->s_cap < restart + 1) {
        if (p->s_V) (void)hipFree(p->s_V);
        p->s_V = nullptr;
        if (hipMalloc(&p->s_V, (size_t)(restart + 1) * n * sizeof(double)) != hipSuccess) {
            p->s_cap = 0;
            set_error("GMRES basis allocation failed");
            return BEMFFT_ENOMEM;
        }
        p->s_cap = restart + 1;
    }
    if (!p->s_vec) {
        if (hipMalloc(&p->s_vec, 7 * (size_t)n * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->s_red, (size_t)kRedBlocks * 512 * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->s_hbuf, 2 * 512 * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&p->h_pinned, 2 * 512 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            set_error("GMRES workspace allocation failed");
            return BEMFFT_ENOMEM;
        }
    }
    ws.V = p->s_V;
    ws.cap = p->s_cap;
    ws.b = p->s_vec;
    ws.x = ws.b + n;
    ws.w = ws.x + n;
    ws.q = ws.w + n;
    ws.u = ws.q + n;
    ws.r = ws.u + n;
    ws.dinv = ws.r + n;
    ws.red = p->s_red;
    ws.hd = p->s_hbuf;
    return 0;
}

// out[0..nvec) = V[0..nvec)^T w  (and sqrt of the last if sqrt_last)
int mdot(const double *V, int64_t ld, int nvec, const double *w, int64_t n, double *red, double *out, int sqrt_last,
         hipStream_t st) {
    hipLaunchKernelGGL(k_mdot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, ld, nvec, w, n, red);
    hipLaunchKernelGGL(k_mdot_final, dim3((nvec + 63) / 64), dim3(64), 0, st, red, kRedBlocks, nvec, out, sqrt_last);
    BF_HIP(hipGetLastError());
    return 0;
}

// r = A x = apply(x in the unknown slots, scaled by 'scale' if given)
int apply_unknown(bemfft_plan *p, const uint8_t *bc, const double *x, const double *scale, Ws &ws, double *out,
                  hipStream_t st) {
    const int64_t n = (int64_t)p->ncomp * p->m;
    hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(256), 0, st, bc, x, scale, ws.q, ws.u, n, 1);
    BF_HIP(hipGetLastError());
    return launch_apply(p, p->eng, ws.q, ws.u, out, st);
}

double read_scalar(const double *d, double *pinned, hipStream_t st, int *status) {
    if (hipMemcpyAsync(pinned, d, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        *status = BEMFFT_EDEVICE;
        return NAN;
    }
    return pinned[0];
}

}  // namespace
}  // namespace bemfft

using namespace bemfft;

extern "C" int bemfft_solve(bemfft_plan *p, const uint8_t *bc, const double *known, double *unknown,
                            const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!p || !bc || !known || !unknown) {
        set_error("solve: null argument");
        return BEMFFT_EINVAL;
    }
    bemfft_solve_opts o{1e-6, 100, 1000, 1, 0};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.restart < 1 || o.restart > 400 || o.maxit < 1) {
        set_error("solve: bad options");
        return BEMFFT_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)p->ncomp * p->m;
    Ws ws{};
    BF_CHECK(ensure_workspace(p, o.restart, ws));
    double *hp = p->h_pinned;
    int status = 0;
    // b = -apply(known values in their slots)
    hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(256), 0, st, bc, known, (const double *)nullptr, ws.q, ws.u,
                       n, 0);
    BF_HIP(hipGetLastError());
    BF_CHECK(launch_apply(p, p->eng, ws.q, ws.u, ws.b, st));
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.b, ws.b, -1.0, 0.0, n);
    // Jacobi scaling
    {
        double *dd = ws.w, *dn = ws.r;
        BF_HIP(hipMemcpyAsync(dd, p->h_diag_dir.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
        BF_HIP(hipMemcpyAsync(dn, p->h_diag_neu.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_diag, dim3(grid_for(n)), dim3(256), 0, st, bc, dd, dn, ws.dinv, n, o.precond);
        BF_HIP(hipGetLastError());
    }
    if (o.use_x0) BF_HIP(hipMemcpyAsync(ws.x, unknown, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else BF_HIP(hipMemsetAsync(ws.x, 0, n * sizeof(double), st));
    BF_CHECK(mdot(ws.b, n, 1, ws.b, n, ws.red, ws.hd, 1, st));
    const double bnorm = read_scalar(ws.hd, hp, st, &status);
    BF_CHECK(status);
    int iters = 0, restarts = 0;
    double true_rel = 0.0;
    const int mcap = o.restart;
    std::vector<double> H((size_t)(mcap + 1) * mcap), cs(mcap), sn(mcap), g(mcap + 1), y(mcap);
    if (!std::isfinite(bnorm)) {
        status = BEMFFT_EBREAKDOWN;
        set_error("right-hand side is not finite");
    } else if (bnorm == 0.0) {
        BF_HIP(hipMemsetAsync(ws.x, 0, n * sizeof(double), st));
        true_rel = 0.0;
    } else {
        bool done = false;
        bool x_zero = !o.use_x0;
        while (!done) {
            // r0 = b - A x
            if (x_zero) {
                BF_HIP(hipMemcpyAsync(ws.w, ws.b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            } else {
                BF_CHECK(apply_unknown(p, bc, ws.x, nullptr, ws, ws.w, st));
                hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.w, ws.b, 1.0, -1.0, n);
            }
            BF_CHECK(mdot(ws.w, n, 1, ws.w, n, ws.red, ws.hd, 1, st));
            const double beta = read_scalar(ws.hd, hp, st, &status);
            BF_CHECK(status);
            true_rel = beta / bnorm;
            if (!std::isfinite(beta)) {
                status = BEMFFT_EBREAKDOWN;
                set_error("GMRES: non-finite residual");
                break;
            }
            if (true_rel <= o.tol) {
                status = 0;
                break;
            }
            if (iters >= o.maxit) {
                status = BEMFFT_ENOCONV;
                break;
            }
            if (restarts > 0 || !x_zero) {
                // keep going from the current x
            }
            hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(256), 0, st, ws.w, ws.hd, ws.V, n);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int k = 0;
            bool breakdown = false;
            for (; k < mcap && iters < o.maxit; ++k) {
                double *vk = ws.V + (int64_t)k * n;
                // w = A Dinv v_k
                BF_CHECK(apply_unknown(p, bc, vk, ws.dinv, ws, ws.w, st));
                // classical Gram-Schmidt, twice
                double *h1 = ws.hd, *h2 = ws.hd + 512;
                BF_CHECK(mdot(ws.V, n, k + 1, ws.w, n, ws.red, h1, 0, st));
                hipLaunchKernelGGL(k_gemv, dim3(grid_for(n)), dim3(256), 0, st, ws.V, n, k + 1, h1, ws.w, n, -1.0);
                BF_CHECK(mdot(ws.V, n, k + 1, ws.w, n, ws.red, h2, 0, st));
                hipLaunchKernelGGL(k_gemv, dim3(grid_for(n)), dim3(256), 0, st, ws.V, n, k + 1, h2, ws.w, n, -1.0);
                BF_CHECK(mdot(ws.w, n, 1, ws.w, n, ws.red, h2 + k + 1, 1, st));
                hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(256), 0, st, ws.w, h2 + k + 1,
                                   ws.V + (int64_t)(k + 1) * n, n);
                BF_HIP(hipGetLastError());
                BF_HIP(hipMemcpyAsync(hp, ws.hd, 1024 * sizeof(double), hipMemcpyDeviceToHost, st));
                BF_HIP(hipStreamSynchronize(st));
                ++iters;
                double *col = &H[(size_t)k * (mcap + 1)];
                for (int i = 0; i <= k; ++i) col[i] = hp[i] + hp[512 + i];
                col[k + 1] = hp[512 + k + 1];
                for (int i = 0; i <= k + 1; ++i)
                    if (!std::isfinite(col[i])) breakdown = true;
                if (breakdown) break;
                for (int i = 0; i < k; ++i) {
                    double t = cs[i] * col[i] + sn[i] * col[i + 1];
                    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                    col[i] = t;
                }
                double a = col[k], bb = col[k + 1];
                double rr = std::hypot(a, bb);
                cs[k] = rr > 0.0 ? a / rr : 1.0;
                sn[k] = rr > 0.0 ? bb / rr : 0.0;
                col[k] = rr;
                col[k + 1] = 0.0;
                g[k + 1] = -sn[k] * g[k];
                g[k] = cs[k] * g[k];
                const double est = std::fabs(g[k + 1]) / bnorm;
                if (est <= o.tol || hp[512 + k + 1] == 0.0) {
                    ++k;
                    break;
                }
            }
            if (breakdown) {
                status = BEMFFT_EBREAKDOWN;
                set_error("GMRES: non-finite Hessenberg entry");
                break;
            }
            // y = H^{-1} g (upper triangular, k x k)
            for (int i = k - 1; i >= 0; --i) {
                double s = g[i];
                for (int j = i + 1; j < k; ++j) s -= H[(size_t)j * (mcap + 1) + i] * y[j];
                double d = H[(size_t)i * (mcap + 1) + i];
                y[i] = d != 0.0 ? s / d : 0.0;
            }
            // x += Dinv V y
            BF_HIP(hipMemcpyAsync(ws.hd, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
            BF_HIP(hipMemsetAsync(ws.r, 0, n * sizeof(double), st));
            hipLaunchKernelGGL(k_gemv, dim3(grid_for(n)), dim3(256), 0, st, ws.V, n, k, ws.hd, ws.r, n, 1.0);
            hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(256), 0, st, ws.r, ws.dinv, n);
            hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.x, ws.r, 1.0, 1.0, n);
            BF_HIP(hipGetLastError());
            x_zero = false;
            ++restarts;
        }
        if (restarts > 0) --restarts;  // the first cycle is not a restart
    }
    BF_HIP(hipMemcpyAsync(unknown, ws.x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    BF_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iters = iters;
        info->restarts = restarts;
        info->true_relres = true_rel;
        info->status = status;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}
