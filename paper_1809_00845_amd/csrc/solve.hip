// solve.hip -- restarted GMRES for the mixed boundary-value problem.
//
// At the end of Sec. 4 the paper finds the unknown q by conjugate gradients,
// with the first integral also evaluated through the FFT, and stops once the
// residual norm is below a chosen bound.  The operator
// of a mixed problem is not symmetric, so the iteration used here is GMRES
// with right Jacobi scaling; every matrix-vector product is one apply.
// Arnoldi uses classical Gram-Schmidt applied twice (two block reductions
// per step), all in FP64; the small Hessenberg problem is solved on the host
// with Givens rotations.  The true residual ||b - A x|| is recomputed with a
// fresh apply at every restart and at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace bemfft {
namespace {

constexpr int kRedBlocks = 256;
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

// The next Krylov vector and the split of its scaled copy in one pass:
// v = w / norm (norm read from device memory) is stored as the basis column,
// and v * scale goes into the unknown slots of (q, u) for the apply.
__global__ void k_split_norm(const uint8_t *bc, const double *w, const double *norm, const double *scale, double *v_out,
                             double *q, double *u, int64_t n) {
    const double a = *norm;
    const double inv = a > 0.0 ? 1.0 / a : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = w[i] * inv;
        v_out[i] = v;
        const double vs = v * scale[i];
        const bool qslot = bc[i] == 0;  // unknown: q where u is known
        q[i] = qslot ? vs : 0.0;
        u[i] = qslot ? 0.0 : vs;
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

// Block Jacobi for three components per node: the diagonal block of the
// mixed operator at node j has column b = -S_jj e_b where component b's q is
// unknown (bc = 0) and C_j e_b where its u is unknown (the double-layer self
// term is zero).  blk[j] receives the inverse of that 3x3 block (row-major),
// from the adjugate; a block that is singular or not finite falls back to
// the inverse of its diagonal (1 where that is 0).  selfb, cb: [m][9] in
// caller order; blk may alias cb (each node reads its own entries first).
__global__ void k_blk_build(const uint8_t *bc, const double *selfb, const double *cb, double *blk, int64_t m) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        double a[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                a[r * 3 + c] = bc[c * m + j] == 0 ? -selfb[j * 9 + r * 3 + c] : cb[j * 9 + r * 3 + c];
        double inv[9];
        inv[0] = a[4] * a[8] - a[5] * a[7];
        inv[1] = a[2] * a[7] - a[1] * a[8];
        inv[2] = a[1] * a[5] - a[2] * a[4];
        inv[3] = a[5] * a[6] - a[3] * a[8];
        inv[4] = a[0] * a[8] - a[2] * a[6];
        inv[5] = a[2] * a[3] - a[0] * a[5];
        inv[6] = a[3] * a[7] - a[4] * a[6];
        inv[7] = a[1] * a[6] - a[0] * a[7];
        inv[8] = a[0] * a[4] - a[1] * a[3];
        const double det = a[0] * inv[0] + a[1] * inv[3] + a[2] * inv[6];
        const double scale = fabs(a[0]) + fabs(a[4]) + fabs(a[8]);
        const bool ok = isfinite(det) && fabs(det) > 1e-12 * scale * scale * scale;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            double v;
            if (ok) v = inv[i] / det;
            else v = (i % 4 == 0 && a[i] != 0.0 && isfinite(a[i])) ? 1.0 / a[i] : (i % 4 == 0 ? 1.0 : 0.0);
            blk[j * 9 + i] = v;
        }
    }
}

// z_j = blk[j] x_j per node (x, z: [3][m]) and the split of z into the
// unknown slots of (q, u): q where bc = 0, u where bc = 1.
__device__ __forceinline__ void blk_split_node(const uint8_t *bc, const double *blk, const double x[3], double *q,
                                               double *u, int64_t m, int64_t j) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double *b = blk + j * 9 + a * 3;
        const double z = b[0] * x[0] + b[1] * x[1] + b[2] * x[2];
        const bool qslot = bc[a * m + j] == 0;
        q[a * m + j] = qslot ? z : 0.0;
        u[a * m + j] = qslot ? 0.0 : z;
    }
}

__global__ void k_split_blk(const uint8_t *bc, const double *x, const double *blk, double *q, double *u, int64_t m) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const double xv[3] = {x[j], x[m + j], x[2 * m + j]};
        blk_split_node(bc, blk, xv, q, u, m, j);
    }
}

// y_j = blk[j] y_j in place (y: [3][m]).
__global__ void k_mul_blk(double *y, const double *blk, int64_t m) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const double x0 = y[j], x1 = y[m + j], x2 = y[2 * m + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double *b = blk + j * 9 + a * 3;
            y[a * m + j] = b[0] * x0 + b[1] * x1 + b[2] * x2;
        }
    }
}

// partial[blk][j] = sum over this block's rows of V[j][i] w[i], j < nvec.
// blockIdx.y picks a group of eight vectors, so every group's loads are in
// flight at once; wavefront sums by lane shuffles, then one LDS step across
// the block's four wavefronts (fixed order: bitwise reproducible).
__global__ __launch_bounds__(kRedThreads) void k_mdot_partial(const double *V, int64_t ld, int nvec,
                                                              const double *w, int64_t n, double *partial) {
    constexpr int G = 8;
    constexpr int NW = kRedThreads / 64;
    __shared__ double sm[NW][G];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int j0 = blockIdx.y * G;
    double acc[G];
#pragma unroll
    for (int k = 0; k < G; ++k) acc[k] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
        const double wi = w[i];
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (j0 + k < nvec) acc[k] += V[(int64_t)(j0 + k) * ld + i] * wi;
    }
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < G; ++k) sm[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < G && j0 + threadIdx.x < nvec) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) s += sm[q][threadIdx.x];
        partial[(int64_t)blockIdx.x * nvec + j0 + threadIdx.x] = s;
    }
}

// out[j] = sum over blocks of partial[b][j]: one wavefront per j, each lane
// a fixed stride of blocks, then a fixed shuffle tree (deterministic)
__global__ __launch_bounds__(64) void k_mdot_final(const double *partial, int nblk, int nvec, double *out,
                                                   int sqrt_last) {
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += partial[(int64_t)b * nvec + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[j] = (sqrt_last && j == nvec - 1) ? sqrt(s) : s;
}

// w[i] += sign * sum_j V[j][i] h[j]; eight independent partial sums keep
// eight loads of V in flight per row.
__global__ void k_gemv(const double *V, int64_t ld, int nvec, const double *h, double *w, int64_t n, double sign) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        }
        for (int k = 0; j + k < nvec; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        w[i] += sign * s;
    }
}

// w[i] -= sum_j V[j][i] h[j] as k_gemv, and each block's sum of the updated
// w[i]^2 into partial[block] (fixed-order reduction: reproducible)
__global__ __launch_bounds__(256) void k_gemv_norm(const double *V, int64_t ld, int nvec, const double *h, double *w,
                                                   int64_t n, double *partial) {
    __shared__ double sm[4];
    double ss = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        }
        for (int k = 0; j + k < nvec; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        const double wi = w[i] - s;
        w[i] = wi;
        ss += wi * wi;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (threadIdx.x % 64 == 0) sm[threadIdx.x / 64] = ss;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

// ---- Arnoldi kernels that reduce the inner-product partials themselves.
// Every block forms the same sums from the block partials in the fixed order
// of k_mdot_final (lane-strided, then a fixed shuffle tree), so no separate
// reduction launch sits between the partials and their consumer.
constexpr int kRedPart = 128;   // blocks of the partial inner products
constexpr int kConsumer = 128;  // blocks of the consumers (each re-reduces the partials)

// h[j] = sum over the kRedPart block partials of column j: wave q of the
// four sums partials 32 q .. 32 q + 31 of 64 columns at a time (sixteen
// loads in flight at once), then the four are added in a fixed order.
__device__ __forceinline__ void reduce_partials(const double *partial, int nvec, double *h) {
    static_assert(kRedPart == 128, "four waves of thirty-two partials");
    __shared__ double part[4][64];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    for (int j0 = 0; j0 < nvec; j0 += 64) {
        const int j = j0 + lane;
        double s = 0.0;
#pragma unroll
        for (int b0 = 0; b0 < 32; b0 += 16) {
            double v[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) v[b] = j < nvec ? partial[(int64_t)(32 * wave + b0 + b) * nvec + j] : 0.0;
#pragma unroll
            for (int b = 0; b < 16; ++b) s += v[b];
        }
        part[wave][lane] = s;
        __syncthreads();
        if (wave == 0 && j < nvec) h[j] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
        __syncthreads();
    }
}

// h = sum of the partials of V^T w; block 0 writes h to hout; w += sign V h
__global__ __launch_bounds__(256) void k_gemv_r(const double *V, int64_t ld, int nvec, const double *partial,
                                                double *w, int64_t n, double sign, double *hout) {
    __shared__ double h[512];
    reduce_partials(partial, nvec, h);
    if (blockIdx.x == 0) {  // hout may be pinned host memory
        for (int j = threadIdx.x; j < nvec; j += blockDim.x) hout[j] = h[j];
        __threadfence_system();
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        }
        for (int k = 0; j + k < nvec; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        const double sm = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        w[i] += sign * sm;
    }
}

// As k_gemv_r with sign -1, and each block's sum of the updated w[i]^2 into
// pout[block]
__global__ __launch_bounds__(256) void k_gemv_norm_r(const double *V, int64_t ld, int nvec, const double *partial,
                                                     double *w, int64_t n, double *hout, double *pout) {
    __shared__ double h[512];
    __shared__ double sm4[4];
    reduce_partials(partial, nvec, h);
    if (blockIdx.x == 0) {  // hout may be pinned host memory
        for (int j = threadIdx.x; j < nvec; j += blockDim.x) hout[j] = h[j];
        __threadfence_system();
    }
    double ss = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        }
        for (int k = 0; j + k < nvec; ++k) acc[k] += V[(int64_t)(j + k) * ld + i] * h[j + k];
        const double sm = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        const double wi = w[i] - sm;
        w[i] = wi;
        ss += wi * wi;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (threadIdx.x % 64 == 0) sm4[threadIdx.x / 64] = ss;
    __syncthreads();
    if (threadIdx.x == 0) pout[blockIdx.x] = (sm4[0] + sm4[1]) + (sm4[2] + sm4[3]);
}

// A step's last result for the host: the norm, then (if flag is given) the
// step's sequence number with system-scope release -- everything the step
// wrote for the host is visible once the host reads the flag.
__device__ __forceinline__ void post_step(double *nout, double a, uint64_t *flag, uint64_t seq) {
    *nout = a;
    __threadfence_system();
    if (flag) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ||w|| = sqrt(sum of the norm partials), then v = w / ||w|| stored as the
// basis column and v * scale split into the unknown slots of (q, u).  Block
// 0 posts the previous step's result if nout is given (pinned host memory):
// ||w|| to nout, then seq to flag with system-scope release, as k_norm_r
// does (the same sum in the same order).
__global__ __launch_bounds__(256) void k_split_norm_r(const uint8_t *bc, const double *w, const double *pnorm, int nblk,
                                                      const double *scale, double *v_out, double *q, double *u,
                                                      int64_t n, double *nout, uint64_t *flag, uint64_t seq) {
    __shared__ double nrm[1];
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) s += pnorm[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (threadIdx.x == 0) nrm[0] = sqrt(s);
    }
    __syncthreads();
    const double a = nrm[0];
    if (blockIdx.x == 0 && threadIdx.x == 0 && nout) post_step(nout, a, flag, seq);
    const double inv = a > 0.0 ? 1.0 / a : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = w[i] * inv;
        v_out[i] = v;
        const double vs = v * scale[i];
        const bool qslot = bc[i] == 0;  // unknown: q where u is known
        q[i] = qslot ? vs : 0.0;
        u[i] = qslot ? 0.0 : vs;
    }
}

// As k_split_norm_r, with the block-Jacobi scaling: one thread per node.
// The basis column v = w / ||w|| is the same, bit for bit.
__global__ __launch_bounds__(256) void k_split_norm_blk(const uint8_t *bc, const double *w, const double *pnorm,
                                                        int nblk, const double *blk, double *v_out, double *q,
                                                        double *u, int64_t m, double *nout, uint64_t *flag,
                                                        uint64_t seq) {
    __shared__ double nrm[1];
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) s += pnorm[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (threadIdx.x == 0) nrm[0] = sqrt(s);
    }
    __syncthreads();
    const double a = nrm[0];
    if (blockIdx.x == 0 && threadIdx.x == 0 && nout) post_step(nout, a, flag, seq);
    const double inv = a > 0.0 ? 1.0 / a : 0.0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        double v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = w[c * m + j] * inv;
            v_out[c * m + j] = v[c];
        }
        blk_split_node(bc, blk, v, q, u, m, j);
    }
}

// out = sqrt(sum of the norm partials) (same order as k_split_norm_r); then,
// if flag is given (pinned host memory), the step's sequence number is
// stored there with system-scope release: everything the step wrote for the
// host is visible once the host reads it
__global__ __launch_bounds__(64) void k_norm_r(const double *pnorm, int nblk, double *out, uint64_t *flag,
                                               uint64_t seq) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += pnorm[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) post_step(out, sqrt(s), flag, seq);  // out may be pinned host memory
}

// Host side: wait until the device has stored seq at flag (pinned memory).
// Spins (the answer comes within one step of the solve); checks the stream
// for errors every few milliseconds and gives up after 120 s.
int wait_step_flag(const uint64_t *flag, uint64_t seq, hipStream_t st) {
    auto t0 = std::chrono::steady_clock::now();
    for (uint64_t spins = 1;; ++spins) {
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) return 0;
        if ((spins & 0x3fff) == 0) {
            const hipError_t q = hipStreamQuery(st);
            if (q != hipSuccess && q != hipErrorNotReady) {
                set_error(std::string("GMRES: stream error while waiting: ") + hipGetErrorString(q));
                return BEMFFT_EDEVICE;
            }
            if (q == hipSuccess && __atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq) {
                set_error("GMRES: the stream drained without the step's completion flag");
                return BEMFFT_EDEVICE;
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) {
                set_error("GMRES: timed out waiting for a step");
                return BEMFFT_EDEVICE;
            }
        }
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
    double *V, *b, *x, *w, *q, *u, *r, *dinv, *ro, *d, *red, *hd;
    double *blk;  // block-Jacobi inverses, [m][9] (three components per node)
    bool blkmode;
    int cap;
};

// Block Jacobi in use: asked for, on a plan with three components per node.
bool block_mode(const bemfft_plan *p, int precond) { return precond == 2 && p->ncomp == 3; }

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
        if (hipMalloc(&p->s_vec, 12 * (size_t)n * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->s_red, (size_t)kRedBlocks * 512 * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->s_hbuf, 2 * 512 * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&p->h_pinned, 4 * 512 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
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
    ws.ro = ws.dinv + n;
    ws.d = ws.ro + n;
    ws.blk = ws.d + n;  // 3 n doubles
    ws.red = p->s_red;
    ws.hd = p->s_hbuf;
    return 0;
}

// out[0..nvec) = V[0..nvec)^T w  (and sqrt of the last if sqrt_last)
int mdot(const double *V, int64_t ld, int nvec, const double *w, int64_t n, double *red, double *out, int sqrt_last,
         hipStream_t st) {
    hipLaunchKernelGGL(k_mdot_partial, dim3(kRedBlocks, (nvec + 7) / 8), dim3(kRedThreads), 0, st, V, ld, nvec, w, n,
                       red);
    hipLaunchKernelGGL(k_mdot_final, dim3(nvec), dim3(64), 0, st, red, kRedBlocks, nvec, out, sqrt_last);
    BF_HIP(hipGetLastError());
    return 0;
}

// out = A x = apply(x in the unknown slots, scaled by 'scale' if given)
int apply_unknown(bemfft_plan *p, const Engine &e, const uint8_t *bc, const double *x, const double *scale, Ws &ws,
                  double *out, hipStream_t st) {
    const int64_t n = (int64_t)p->ncomp * p->m;
    hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(256), 0, st, bc, x, scale, ws.q, ws.u, n, 1);
    BF_HIP(hipGetLastError());
    return launch_apply(p, e, ws.q, ws.u, out, st);
}

// ||v||_2 (one host round trip)
double norm2(const double *v, int64_t n, Ws &ws, double *pinned, hipStream_t st, int *status) {
    *status = mdot(v, n, 1, v, n, ws.red, ws.hd, 1, st);
    if (*status) return NAN;
    if (hipMemcpyAsync(pinned, ws.hd, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        *status = BEMFFT_EDEVICE;
        set_error("GMRES: device-to-host copy failed");
        return NAN;
    }
    return pinned[0];
}

// Restarted GMRES with right scaling Dinv on the operator of engine e:
// solves A x = rhs, x in/out (x_zero: x is zero on entry), relative true
// residual tolerance tol, at most maxit iterations.  Uses ws.w, ws.r, ws.q,
// ws.u, ws.V.  Returns the status; iters and the final true relative
// residual (w.r.t. ||rhs||) through the pointers.
// pipelined = true: hp is pinned host memory that the step kernels write
// into, and the host polls each step's completion flag there.  pipelined =
// false (the allocation-free entry point): each step is waited for with a
// stream synchronisation before the next one is queued and its column is
// copied (hp may then be ordinary pageable host memory).
int gmres_core(bemfft_plan *p, const Engine &e, const uint8_t *bc, const double *rhs, double *x, bool x_zero,
               double tol, int mcap, int maxit, Ws &ws, double *hp, hipStream_t st, int *iters_out, int *restarts_out,
               double *relres_out, const double *r0_given, bool pipelined) {
    const int64_t n = (int64_t)p->ncomp * p->m;
    int status = 0;
    const double bnorm = norm2(rhs, n, ws, hp, st, &status);
    BF_CHECK(status);
    int iters = 0, cycles = 0;
    double true_rel = 0.0;
    std::vector<double> H((size_t)(mcap + 1) * mcap), cs(mcap), sn(mcap), g(mcap + 1), y(mcap);
    if (!std::isfinite(bnorm)) {
        set_error("GMRES: right-hand side is not finite");
        return BEMFFT_EBREAKDOWN;
    }
    if (bnorm == 0.0) {
        BF_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
        *iters_out = 0;
        *restarts_out = 0;
        *relres_out = 0.0;
        return 0;
    }
    for (;;) {
        // r0 = rhs - A x (on the first cycle the caller may already hold it)
        if (x_zero) {
            BF_HIP(hipMemcpyAsync(ws.w, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        } else if (r0_given && cycles == 0) {
            BF_HIP(hipMemcpyAsync(ws.w, r0_given, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        } else {
            BF_CHECK(apply_unknown(p, e, bc, x, nullptr, ws, ws.w, st));
            hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.w, rhs, 1.0, -1.0, n);
        }
        const double beta = norm2(ws.w, n, ws, hp, st, &status);
        BF_CHECK(status);
        true_rel = beta / bnorm;
        if (!std::isfinite(beta)) {
            status = BEMFFT_EBREAKDOWN;
            set_error("GMRES: non-finite residual");
            break;
        }
        if (true_rel <= tol) break;
        if (iters >= maxit) {
            status = BEMFFT_ENOCONV;
            break;
        }
        hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(256), 0, st, ws.w, ws.hd, ws.V, n);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool breakdown = false;
        // Step kk is queued one step ahead: step k + 1 goes to the GPU before
        // the host waits for step k's Hessenberg column (its inputs are all on
        // the device), so the GPU keeps working while the host applies the
        // rotations.  The column of step kk -- h1 at [0, kk], h2 at [512,
        // 512 + kk], ||w|| at 512 + kk + 1 -- is written by the kernels
        // themselves into half kk & 1 of the pinned host buffer (unpipelined:
        // into the device buffer, copied after the step).  The next step's
        // first kernel reduces ||w|| again from the same partials, in the same
        // order, to normalise w.  A step queued past convergence only fills
        // scratch.
        double *red1 = ws.red, *red2 = ws.red + 65536, *red3 = ws.red + 131072 - 256;
        // completion flags carry a number never used before on this plan
        const uint64_t seq0 = p->s_seq;
        p->s_seq += (uint64_t)mcap + 1;
        auto step_seq = [&](int kk) { return seq0 + (uint64_t)kk + 1; };
        const int gc = std::min(kConsumer, grid_for(n));
        auto col_of = [&](int kk) { return pipelined ? hp + 1024 * (kk & 1) : ws.hd; };
        const int kmax = std::min(mcap, maxit - iters);
        // Pipelined, every step but the last of the cycle has its norm and
        // completion flag posted by the next step's first kernel, which sums
        // the same norm partials in the same order (one kernel less per step);
        // the last step, and every step when unpipelined, posts its own.
        auto queue_step = [&](int kk) -> int {
            double *vk = ws.V + (int64_t)kk * n;
            double *hc = col_of(kk);
            // w = A Dinv v_k; for k > 0, v_k = w / ||w|| of the previous step
            const int64_t m = p->m;
            if (kk == 0) {
                if (ws.blkmode) {
                    hipLaunchKernelGGL(k_split_blk, dim3(grid_for(m)), dim3(256), 0, st, bc, vk, ws.blk, ws.q, ws.u, m);
                    BF_HIP(hipGetLastError());
                    BF_CHECK(launch_apply(p, e, ws.q, ws.u, ws.w, st));
                } else {
                    BF_CHECK(apply_unknown(p, e, bc, vk, ws.dinv, ws, ws.w, st));
                }
            } else {
                double *pn = pipelined ? col_of(kk - 1) + 512 + kk : nullptr;  // step kk - 1's ||w||
                uint64_t *pf = pipelined ? reinterpret_cast<uint64_t *>(col_of(kk - 1) + 1023) : nullptr;
                if (ws.blkmode)
                    hipLaunchKernelGGL(k_split_norm_blk, dim3(grid_for(m)), dim3(256), 0, st, bc, ws.w, red3, gc,
                                       ws.blk, vk, ws.q, ws.u, m, pn, pf, step_seq(kk - 1));
                else
                    hipLaunchKernelGGL(k_split_norm_r, dim3(grid_for(n)), dim3(256), 0, st, bc, ws.w, red3, gc, ws.dinv,
                                       vk, ws.q, ws.u, n, pn, pf, step_seq(kk - 1));
                BF_HIP(hipGetLastError());
                BF_CHECK(launch_apply(p, e, ws.q, ws.u, ws.w, st));
            }
            // classical Gram-Schmidt, twice; the second update also sums ||w||^2
            hipLaunchKernelGGL(k_mdot_partial, dim3(kRedPart, (kk + 1 + 7) / 8), dim3(kRedThreads), 0, st, ws.V, n, kk + 1,
                               ws.w, n, red1);
            hipLaunchKernelGGL(k_gemv_r, dim3(gc), dim3(256), 0, st, ws.V, n, kk + 1, red1, ws.w, n, -1.0, hc);
            hipLaunchKernelGGL(k_mdot_partial, dim3(kRedPart, (kk + 1 + 7) / 8), dim3(kRedThreads), 0, st, ws.V, n, kk + 1,
                               ws.w, n, red2);
            hipLaunchKernelGGL(k_gemv_norm_r, dim3(gc), dim3(256), 0, st, ws.V, n, kk + 1, red2, ws.w, n, hc + 512,
                               red3);
            if (!pipelined || kk + 1 >= kmax) {
                uint64_t *flag = pipelined ? reinterpret_cast<uint64_t *>(hc + 1023) : nullptr;
                hipLaunchKernelGGL(k_norm_r, dim3(1), dim3(64), 0, st, red3, gc, hc + 512 + kk + 1, flag, step_seq(kk));
            }
            BF_HIP(hipGetLastError());
            if (!pipelined) BF_HIP(hipMemcpyAsync(hp, ws.hd, 1024 * sizeof(double), hipMemcpyDeviceToHost, st));
            return 0;
        };
        if (pipelined) BF_CHECK(queue_step(0));
        for (; k < kmax; ++k) {
            if (pipelined) {
                if (k + 1 < kmax) BF_CHECK(queue_step(k + 1));
                BF_CHECK(wait_step_flag(reinterpret_cast<const uint64_t *>(col_of(k) + 1023), step_seq(k), st));
            } else {
                BF_CHECK(queue_step(k));
                BF_HIP(hipStreamSynchronize(st));
            }
            const double *hk = pipelined ? col_of(k) : hp;
            ++iters;
            double *col = &H[(size_t)k * (mcap + 1)];
            for (int i = 0; i <= k; ++i) col[i] = hk[i] + hk[512 + i];
            col[k + 1] = hk[512 + k + 1];
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
            if (est <= tol || hk[512 + k + 1] == 0.0) {
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
        if (ws.blkmode) hipLaunchKernelGGL(k_mul_blk, dim3(grid_for(p->m)), dim3(256), 0, st, ws.r, ws.blk, p->m);
        else hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(256), 0, st, ws.r, ws.dinv, n);
        hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, x, ws.r, 1.0, 1.0, n);
        BF_HIP(hipGetLastError());
        x_zero = false;
        ++cycles;
    }
    *iters_out = iters;
    *restarts_out = cycles > 0 ? cycles - 1 : 0;
    *relres_out = true_rel;
    return status;
}

// ------------------------------------------------------------------ CG
// Conjugate gradients on the symmetrised Dirichlet single-layer system.
// S = G W with G symmetric (the single-layer kernel is even, and the self
// and same-cell values are symmetric), so A = W^1/2 S W^-1/2 = W^1/2 G W^1/2
// is symmetric; it is positive definite for the 3D kernel and for the 2D
// one when the boundary's logarithmic capacity is below 1.  Scalars stay on
// the device: sc[4 c + 0] = r.z and sc[4 c + 1] = r.r of slot c (two slots,
// alternating per iteration), sc[4 c + 2] = p.Ap of the step that read slot c.

// sw[perm[s]] = sqrt(w[s]): the weights in the caller's node order
__global__ void k_cg_sqrtw(const int *perm, const double *w, double *sw, int64_t m) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x)
        sw[perm[s]] = sqrt(w[s]);
}

// apply inputs for S W^-1/2 v: q = v / sw, u = 0
__global__ void k_cg_in(const double *v, const double *sw, double *q, double *u, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        q[i] = v[i] / sw[i];
        u[i] = 0.0;
    }
}

// y = a sw y (a = -1 turns apply(q, 0) = -S q into W^1/2 S q; a = 1 scales b)
__global__ void k_cg_scale(double *y, const double *sw, double a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * sw[i] * y[i];
}

// dinv = 1 / d with d = -dneg (the positive diagonal of S); 1 where off or
// where d is not positive and finite
__global__ void k_cg_diag(const double *dneg, double *dinv, int64_t n, int on) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = -dneg[i];
        dinv[i] = (on && d > 0.0 && isfinite(d)) ? 1.0 / d : 1.0;
    }
}

// r = b - Av (or b if Av is null); z = dinv r; p = z; per-block partial
// sums of r.z and r.r into partial[blk][2]
__global__ __launch_bounds__(256) void k_cg_init(const double *b, const double *av, const double *dinv, double *r,
                                                 double *z, double *pv, int64_t n, double *partial) {
    __shared__ double sm[4][2];
    double rz = 0.0, rr = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = av ? b[i] - av[i] : b[i];
        const double zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        pv[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rz += __shfl_xor(rz, off, 64);
        rr += __shfl_xor(rr, off, 64);
    }
    if (threadIdx.x % 64 == 0) {
        sm[threadIdx.x / 64][0] = rz;
        sm[threadIdx.x / 64][1] = rr;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        partial[(int64_t)blockIdx.x * 2 + threadIdx.x] =
            (sm[0][threadIdx.x] + sm[1][threadIdx.x]) + (sm[2][threadIdx.x] + sm[3][threadIdx.x]);
}

// alpha = r.z / p.Ap of slot cur; x += alpha p; r -= alpha Ap; z = dinv r;
// partial sums of the new r.z and r.r (fixed order: reproducible)
__global__ __launch_bounds__(256) void k_cg_step(const double *sc, int cur, double *x, double *r, double *z,
                                                 const double *pv, const double *ap, const double *dinv, int64_t n,
                                                 double *partial) {
    __shared__ double sm[4][2];
    const double alpha = sc[4 * cur] / sc[4 * cur + 2];
    double rz = 0.0, rr = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * pv[i];
        const double ri = r[i] - alpha * ap[i];
        const double zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rz += __shfl_xor(rz, off, 64);
        rr += __shfl_xor(rr, off, 64);
    }
    if (threadIdx.x % 64 == 0) {
        sm[threadIdx.x / 64][0] = rz;
        sm[threadIdx.x / 64][1] = rr;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        partial[(int64_t)blockIdx.x * 2 + threadIdx.x] =
            (sm[0][threadIdx.x] + sm[1][threadIdx.x]) + (sm[2][threadIdx.x] + sm[3][threadIdx.x]);
}

// p = z + beta p with beta = (r.z of slot nxt) / (r.z of slot cur)
__global__ void k_cg_dir(const double *sc, int cur, double *pv, const double *z, int64_t n) {
    const double beta = sc[4 * (cur ^ 1)] / sc[4 * cur];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pv[i] = z[i] + beta * pv[i];
}

// Av = W^1/2 S W^-1/2 v through one apply of the plan's working precision
int cg_op(bemfft_plan *p, const double *v, const double *sw, Ws &ws, double *av, hipStream_t st) {
    const int64_t n = p->m;
    hipLaunchKernelGGL(k_cg_in, dim3(grid_for(n)), dim3(256), 0, st, v, sw, ws.q, ws.u, n);
    BF_HIP(hipGetLastError());
    BF_CHECK(launch_apply(p, p->eng, ws.q, ws.u, av, st));
    hipLaunchKernelGGL(k_cg_scale, dim3(grid_for(n)), dim3(256), 0, st, av, sw, -1.0, n);
    BF_HIP(hipGetLastError());
    return 0;
}

}  // namespace
}  // namespace bemfft

using namespace bemfft;

namespace bemfft {
namespace {

// Arguments and options of bemfft_solve, checked; o receives the options
// with defaults filled in.
int solve_check(const bemfft_plan *p, const uint8_t *bc, const double *known, const double *unknown,
                const bemfft_solve_opts *opts, bemfft_solve_opts &o) {
    if (!p || !bc || !known || !unknown) {
        set_error("solve: null argument");
        return BEMFFT_EINVAL;
    }
    o = bemfft_solve_opts{1e-6, 100, 1000, 1, 0, 0, 1e-4, 20};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.restart < 1 || o.restart > 400 || o.maxit < 1 || o.use_x0 < 0 || o.use_x0 > 2 ||
        o.precond < 0 || o.precond > 2) {
        set_error("solve: bad options");
        return BEMFFT_EINVAL;
    }
    if (o.refine && (!p->has64 || !(o.inner_tol > 0.0) || o.max_outer < 1)) {
        set_error("solve: refinement needs a plan created with keep_fp64 (or FP64), inner_tol > 0, max_outer >= 1");
        return BEMFFT_EINVAL;
    }
    return 0;
}

// The mixed problem of bemfft_solve with the given workspace (device
// vectors ws, host buffer hp of 4 * 512 doubles); pipelined as gmres_core.
int solve_impl(bemfft_plan *p, const uint8_t *bc, const double *known, double *unknown, const bemfft_solve_opts &o,
               bemfft_solve_info *info, hipStream_t st, Ws &ws, double *hp, bool pipelined,
               std::chrono::steady_clock::time_point t0) {
    const int64_t n = (int64_t)p->ncomp * p->m;
    const Engine &e64 = (p->eng.precision == BEMFFT_FP64) ? p->eng : p->eng64;
    const Engine &eo = o.refine ? e64 : p->eng;  // operator of b and of the true residual
    int status = 0;
    // b = -apply(known values in their slots)
    hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(256), 0, st, bc, known, (const double *)nullptr, ws.q, ws.u,
                       n, 0);
    BF_HIP(hipGetLastError());
    BF_CHECK(launch_apply(p, eo, ws.q, ws.u, ws.b, st));
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.b, ws.b, -1.0, 0.0, n);
    // Jacobi scaling
    {
        double *dd = ws.w, *dn = ws.r;
        BF_HIP(hipMemcpyAsync(dd, p->h_diag_dir.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
        BF_HIP(hipMemcpyAsync(dn, p->h_diag_neu.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_diag, dim3(grid_for(n)), dim3(256), 0, st, bc, dd, dn, ws.dinv, n, o.precond);
        BF_HIP(hipGetLastError());
    }
    ws.blkmode = block_mode(p, o.precond);
    if (ws.blkmode) {
        // self blocks into w, q, u (3 n contiguous doubles), c blocks into blk
        const int64_t m = p->m;
        if (ws.q != ws.w + n || ws.u != ws.q + n) {
            set_error("solve: workspace layout");
            return BEMFFT_EDEVICE;
        }
        BF_HIP(hipMemcpyAsync(ws.w, p->h_self.data(), 9 * m * sizeof(double), hipMemcpyHostToDevice, st));
        BF_HIP(hipMemcpyAsync(ws.blk, p->h_c.data(), 9 * m * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_blk_build, dim3(grid_for(m)), dim3(256), 0, st, bc, ws.w, ws.blk, ws.blk, m);
        BF_HIP(hipGetLastError());
    }
    if (o.use_x0) BF_HIP(hipMemcpyAsync(ws.x, unknown, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else BF_HIP(hipMemsetAsync(ws.x, 0, n * sizeof(double), st));
    int iters = 0, restarts = 0, outer = 0, applies64 = 1;
    double rel = 0.0, rel0 = 1.0;
    bool use_x0 = o.use_x0 != 0;
    if (o.use_x0 == 2) {
        // keep the guess only if its true residual is below that of x = 0
        int s2 = 0;
        BF_CHECK(apply_unknown(p, eo, bc, ws.x, nullptr, ws, ws.ro, st));
        hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.ro, ws.b, 1.0, -1.0, n);
        BF_HIP(hipGetLastError());
        const double rn = norm2(ws.ro, n, ws, hp, st, &s2);
        BF_CHECK(s2);
        const double bn = norm2(ws.b, n, ws, hp, st, &s2);
        BF_CHECK(s2);
        rel0 = bn > 0.0 ? rn / bn : 0.0;
        if (!(rn < bn)) {
            use_x0 = false;
            BF_HIP(hipMemsetAsync(ws.x, 0, n * sizeof(double), st));
        }
    }
    if (!o.refine) {
        status = gmres_core(p, p->eng, bc, ws.b, ws.x, !use_x0, o.tol, o.restart, o.maxit, ws, hp, st, &iters,
                            &restarts, &rel, o.use_x0 == 2 ? ws.ro : nullptr, pipelined);
    } else {
        // iterative refinement: r = b - A64 x in FP64, d ~ A^-1 r in the
        // working precision, x += d
        int st2 = 0;
        const double bnorm = norm2(ws.b, n, ws, hp, st, &st2);
        BF_CHECK(st2);
        bool x_zero = !use_x0;
        for (;;) {
            if (x_zero) {
                BF_HIP(hipMemcpyAsync(ws.ro, ws.b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            } else {
                BF_CHECK(apply_unknown(p, e64, bc, ws.x, nullptr, ws, ws.ro, st));
                ++applies64;
                hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.ro, ws.b, 1.0, -1.0, n);
            }
            const double rn = norm2(ws.ro, n, ws, hp, st, &st2);
            BF_CHECK(st2);
            rel = bnorm > 0.0 ? rn / bnorm : 0.0;
            if (!std::isfinite(rn)) {
                status = BEMFFT_EBREAKDOWN;
                set_error("refinement: non-finite residual");
                break;
            }
            if (rel <= o.tol || bnorm == 0.0) { status = 0; break; }
            if (outer >= o.max_outer || iters >= o.maxit) { status = BEMFFT_ENOCONV; break; }
            // inner solve: no need to go below what the outer target still needs
            const double itol = std::max(o.inner_tol, 0.5 * o.tol / rel);
            int it = 0, rs = 0;
            double irel = 0.0;
            BF_HIP(hipMemsetAsync(ws.d, 0, n * sizeof(double), st));
            int s3 = gmres_core(p, p->eng, bc, ws.ro, ws.d, true, itol, o.restart, o.maxit - iters, ws, hp, st, &it,
                                &rs, &irel, nullptr, pipelined);
            iters += it;
            restarts += rs;
            if (s3 < 0) { status = s3; break; }
            hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ws.x, ws.d, 1.0, 1.0, n);
            BF_HIP(hipGetLastError());
            x_zero = false;
            ++outer;
        }
    }
    BF_HIP(hipMemcpyAsync(unknown, ws.x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    BF_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iters = iters;
        info->restarts = restarts;
        info->true_relres = rel;
        info->status = status;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->outer = outer;
        info->applies64 = o.refine ? applies64 : 0;
        info->x0_used = use_x0 ? 1 : 0;
        info->x0_relres = o.use_x0 == 2 ? rel0 : -1.0;
    }
    return status;
}

// ------------------------------------------------------------------ no allocation
// Workspace of bemfft_solve_noalloc: one file-scope device array per GPU,
// held until the process ends.  Its host-side name is not a device address:
// host code uses only the per-device pointer from hipGetSymbolAddress.
constexpr int64_t kScratchDoubles = BEMFFT_NOALLOC_SCRATCH_BYTES / 8;
constexpr int64_t kRedDoubles = (int64_t)kRedBlocks * 512;  // reduction partials
constexpr int64_t kHdDoubles = 2 * 512;                     // Hessenberg column buffer
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
// host side of the per-step Hessenberg copies (pageable; one per device)
double g_noalloc_host[kMaxDevices][4 * 512];

// Largest restart whose basis fits the workspace for n unknowns.
int64_t noalloc_max_restart(int64_t n) {
    const int64_t avail = kScratchDoubles - kRedDoubles - kHdDoubles;
    return std::min<int64_t>(400, avail / n - 10);
}

int scratch_for_current_device(double **out, int *dev_out) {
    int dev = -1;
    BF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("solve_noalloc: device index out of range");
        return BEMFFT_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        BF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    *dev_out = dev;
    return 0;
}

}  // namespace
}  // namespace bemfft

extern "C" int bemfft_solve(bemfft_plan *p, const uint8_t *bc, const double *known, double *unknown,
                            const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    bemfft_solve_opts o;
    BF_CHECK(solve_check(p, bc, known, unknown, opts, o));
    Ws ws{};
    BF_CHECK(ensure_workspace(p, o.restart, ws));
    return solve_impl(p, bc, known, unknown, o, info, (hipStream_t)stream, ws, p->h_pinned, true, t0);
}

extern "C" int bemfft_solve_noalloc(bemfft_plan *p, const uint8_t *bc, const double *known, double *unknown,
                                    const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    bemfft_solve_opts o;
    BF_CHECK(solve_check(p, bc, known, unknown, opts, o));
    const int64_t n = (int64_t)p->ncomp * p->m;
    const int64_t extra = block_mode(p, o.precond) ? 3 * n : 0;  // block-Jacobi inverses
    const int64_t need = (int64_t)(o.restart + 1) * n + 9 * n + extra + kRedDoubles + kHdDoubles;
    if (need > kScratchDoubles) {
        set_error("solve_noalloc: (restart + " + std::to_string(10 + extra / n) + ") * ncomp * m = " +
                  std::to_string((int64_t)(o.restart + 10) * n + extra) +
                  " doubles exceeds the fixed workspace; largest restart for this plan: " +
                  std::to_string(noalloc_max_restart(n) - extra / n));
        return BEMFFT_EINVAL;
    }
    double *base = nullptr;
    int dev = 0;
    BF_CHECK(scratch_for_current_device(&base, &dev));
    Ws ws{};
    ws.red = base;
    ws.hd = ws.red + kRedDoubles;
    ws.b = ws.hd + kHdDoubles;
    ws.x = ws.b + n;
    ws.w = ws.x + n;
    ws.q = ws.w + n;
    ws.u = ws.q + n;
    ws.r = ws.u + n;
    ws.dinv = ws.r + n;
    ws.ro = ws.dinv + n;
    ws.d = ws.ro + n;
    ws.V = ws.d + n;
    ws.cap = o.restart + 1;
    ws.blk = ws.V + (int64_t)ws.cap * n;  // 3 n doubles when used
    return solve_impl(p, bc, known, unknown, o, info, (hipStream_t)stream, ws, g_noalloc_host[dev], false, t0);
}

extern "C" int bemfft_solve_cg(bemfft_plan *p, const double *u, double *q, const bemfft_solve_opts *opts,
                               bemfft_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!p || !u || !q) {
        set_error("solve_cg: null argument");
        return BEMFFT_EINVAL;
    }
    if (p->kernel != BEMFFT_LAPLACE2D && p->kernel != BEMFFT_LAPLACE3D) {
        set_error("solve_cg: Laplace plans only");
        return BEMFFT_EINVAL;
    }
    bemfft_solve_opts o{1e-6, 100, 1000, 1, 0, 0, 1e-4, 20};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.maxit < 1 || o.use_x0 < 0 || o.use_x0 > 1 || o.precond < 0 || o.precond > 1) {
        set_error("solve_cg: bad options");
        return BEMFFT_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = p->m;
    Ws ws{};
    BF_CHECK(ensure_workspace(p, 1, ws));
    double *hp = p->h_pinned;
    double *sc = ws.hd;  // device scalars
    double *sw = ws.V, *b = ws.b, *x = ws.x, *r = ws.r, *z = ws.ro, *pv = ws.d, *ap = ws.w, *dinv = ws.dinv;
    hipLaunchKernelGGL(k_cg_sqrtw, dim3(grid_for(n)), dim3(256), 0, st, p->d_perm, p->d_w, sw, n);
    BF_HIP(hipGetLastError());
    // b = W^1/2 (c u + D[u]) = W^1/2 apply(0, u)
    BF_HIP(hipMemsetAsync(ws.q, 0, n * sizeof(double), st));
    BF_CHECK(launch_apply(p, p->eng, ws.q, u, b, st));
    hipLaunchKernelGGL(k_cg_scale, dim3(grid_for(n)), dim3(256), 0, st, b, sw, 1.0, n);
    // Jacobi: diag(A) = diag(S), the exact self terms (the negated Dirichlet
    // diagonal of the mixed operator)
    BF_HIP(hipMemcpyAsync(ap, p->h_diag_dir.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_cg_diag, dim3(grid_for(n)), dim3(256), 0, st, ap, dinv, n, o.precond);
    BF_HIP(hipGetLastError());
    int status = 0, iters = 0;
    double bn = 0.0, rel = 0.0;
    {
        int s2 = 0;
        bn = norm2(b, n, ws, hp, st, &s2);
        BF_CHECK(s2);
    }
    // r0 = b - A x0, z0 = dinv r0, p0 = z0 (slot 0)
    if (o.use_x0) {
        BF_HIP(hipMemcpyAsync(x, q, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_cg_scale, dim3(grid_for(n)), dim3(256), 0, st, x, sw, 1.0, n);
        BF_CHECK(cg_op(p, x, sw, ws, ap, st));
    } else {
        BF_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
    }
    hipLaunchKernelGGL(k_cg_init, dim3(kRedBlocks), dim3(256), 0, st, b, o.use_x0 ? ap : (const double *)nullptr,
                       dinv, r, z, pv, n, ws.red);
    hipLaunchKernelGGL(k_mdot_final, dim3(2), dim3(64), 0, st, ws.red, kRedBlocks, 2, sc, 0);
    BF_HIP(hipGetLastError());
    int cur = 0;
    for (;;) {
        BF_HIP(hipMemcpyAsync(hp, sc, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        BF_HIP(hipStreamSynchronize(st));
        const double rr = hp[4 * cur + 1];
        if (iters > 0 && !(hp[4 * (cur ^ 1) + 2] > 0.0)) {
            status = BEMFFT_EBREAKDOWN;
            set_error("solve_cg: p.Ap <= 0 (the symmetrised operator is not positive definite)");
            break;
        }
        if (!std::isfinite(rr)) {
            status = BEMFFT_EBREAKDOWN;
            set_error("solve_cg: non-finite residual");
            break;
        }
        rel = bn > 0.0 ? std::sqrt(rr) / bn : 0.0;
        if (rel <= o.tol || bn == 0.0) break;
        if (iters >= o.maxit) {
            status = BEMFFT_ENOCONV;
            break;
        }
        // one iteration: Ap, p.Ap into slot cur, the step into slot cur^1, the new direction
        BF_CHECK(cg_op(p, pv, sw, ws, ap, st));
        BF_CHECK(mdot(pv, n, 1, ap, n, ws.red, sc + 4 * cur + 2, 0, st));
        hipLaunchKernelGGL(k_cg_step, dim3(kRedBlocks), dim3(256), 0, st, sc, cur, x, r, z, pv, ap, dinv, n, ws.red);
        hipLaunchKernelGGL(k_mdot_final, dim3(2), dim3(64), 0, st, ws.red, kRedBlocks, 2, sc + 4 * (cur ^ 1), 0);
        hipLaunchKernelGGL(k_cg_dir, dim3(grid_for(n)), dim3(256), 0, st, sc, cur, pv, z, n);
        BF_HIP(hipGetLastError());
        cur ^= 1;
        ++iters;
    }
    // q = W^-1/2 x; true residual ||b - A x|| / ||b|| with a fresh apply
    if (status >= 0) {
        BF_CHECK(cg_op(p, x, sw, ws, ap, st));
        hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, ap, b, 1.0, -1.0, n);
        BF_HIP(hipGetLastError());
        int s2 = 0;
        const double tn = norm2(ap, n, ws, hp, st, &s2);
        BF_CHECK(s2);
        rel = bn > 0.0 ? tn / bn : 0.0;
    }
    hipLaunchKernelGGL(k_cg_in, dim3(grid_for(n)), dim3(256), 0, st, x, sw, q, ws.u, n);
    BF_HIP(hipGetLastError());
    BF_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iters = iters;
        info->restarts = 0;
        info->true_relres = rel;
        info->status = status;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->outer = 0;
        info->applies64 = 0;
        info->x0_used = o.use_x0;
        info->x0_relres = -1.0;
    }
    return status;
}
