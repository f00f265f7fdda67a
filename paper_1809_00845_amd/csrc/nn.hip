// nn.hip -- a small convolutional network that proposes the initial guess
// of the iterative solve (the unknown flux q of a Dirichlet problem, Sec. 4),
// with its own forward, backward and optimiser kernels.
//
// Input: voxel channels on the plan's grid, nonzero only at boundary nodes:
// a = w/h^2, a n_x, a n_y, a n_z, a s u and a s b, with s = 1/rms(u) over
// the Dirichlet nodes and b the right-hand side of the solve (minus the
// operator applied to the known values, one application of eq. 16).
// Layers: 3x3x3 convolutions with dilations d_l (zero padding), ReLU between
// layers, one output channel read back at the node voxels as s h q.
// Training (FP32 storage and arithmetic) minimises the weighted squared error
// sum_j wt_j (y(v_j) - s h q_j)^2 against solved problems, with Adam.
// Inference (the guess) runs in FP16 on the matrix cores with FP32
// accumulation.  The solve keeps the guess only when its residual is smaller
// than ||b|| (plain GMRES from zero otherwise).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "internal.hpp"

struct bemfft_net {
    int G = 0, cin = 0, width = 0, nl = 0;
    int64_t V = 0;  // G^3
    std::vector<int> dil, ci, co;
    std::vector<int64_t> woff, boff;
    int64_t nparam = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // params, grads, Adam moments
    float *pre = nullptr, *post = nullptr;  // per layer [co][V] (post = relu(pre) for hidden layers)
    float *ga = nullptr, *gb = nullptr;     // gradient ping-pong [width][V]
    float *part = nullptr;                  // weight-gradient partial sums
    float *red = nullptr;                   // loss partial sums
    float *y = nullptr;                     // output of the last forward [V]
    int64_t t = 0;                          // Adam step
    double *dq = nullptr, *du = nullptr, *db = nullptr;  // right-hand side scratch [cap]
    int64_t cap = 0;
    // inference in FP16: channel-last activations [V][16] (ping-pong), packed
    // weights [layer][27][16][16], biases [layer][16], scale s on the device
    _Float16 *ha = nullptr, *hb = nullptr, *wp = nullptr;
    float *bp = nullptr;
    double *sdev = nullptr;
    int64_t *d_woff = nullptr, *d_boff = nullptr;
    int *d_ci = nullptr, *d_co = nullptr;
};

namespace bemfft {
namespace {

constexpr int kChunk = 8192;  // voxels per weight-gradient block
constexpr int64_t kMaxTargets = 65536LL * 256;  // loss partial sums: one per 256 targets

__device__ __forceinline__ void vox_xyz(int64_t v, int G, int &x, int &y, int &z) {
    x = (int)(v % G);
    y = (int)((v / G) % G);
    z = (int)(v / ((int64_t)G * G));
}

__device__ __forceinline__ bool inside(int x, int y, int z, int G) {
    return x >= 0 && x < G && y >= 0 && y < G && z >= 0 && z < G;
}

__global__ void k_fill(float *a, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// known values into their slots: u where bc = 0 (or bc absent), q where bc = 1
__global__ void k_nn_split(const uint8_t *bc, const double *known, double *q, double *u, int64_t m) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= m) return;
    const bool qk = bc != nullptr && bc[j] != 0;
    q[j] = qk ? known[j] : 0.0;
    u[j] = qk ? 0.0 : known[j];
}

// input channels at the node voxels (the buffer was cleared before); r is
// the operator applied to the known values (b = -r).  Nodes that share a
// voxel add up; atomics keep that correct whatever the node order.
__global__ void k_nn_input(const int *gx, const int *gy, const int *gz, const int *perm, const double *w,
                           const double *nrm, const double *known, const double *r, const uint8_t *bc, int64_t m,
                           int G, double inv_h2, double s_host, const double *s_dev, float *x, int64_t V) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    const double s = s_dev ? *s_dev : s_host;
    const int j = perm[k];
    const int64_t v = ((int64_t)gz[k] * G + gy[k]) * G + gx[k];
    const double ww = w[k] * inv_h2;
    const double u = (bc == nullptr || bc[j] == 0) ? known[j] : 0.0;
    atomicAdd(&x[v], (float)ww);
    atomicAdd(&x[V + v], (float)(ww * nrm[k]));
    atomicAdd(&x[2 * V + v], (float)(ww * nrm[m + k]));
    atomicAdd(&x[3 * V + v], (float)(ww * nrm[2 * m + k]));
    atomicAdd(&x[4 * V + v], (float)(ww * s * u));
    atomicAdd(&x[5 * V + v], (float)(-ww * s * r[j]));
}

// out[c][v] = b[c] + sum_{ci, tap} W[c][ci][tap] in[ci][v + d tap]
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_fwd(const float *in, const float *W, const float *bias, float *pre,
                                                  float *post, int G, int d, int relu) {
    __shared__ float sW[COUT * CIN * 27];
    __shared__ float sb[COUT];
    for (int i = threadIdx.x; i < COUT * CIN * 27; i += 256) sW[i] = W[i];
    for (int i = threadIdx.x; i < COUT; i += 256) sb[i] = bias[i];
    __syncthreads();
    const int64_t V = (int64_t)G * G * G;
    const int64_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
    int x, y, z;
    vox_xyz(v, G, x, y, z);
    float acc[COUT];
#pragma unroll
    for (int c = 0; c < COUT; ++c) acc[c] = sb[c];
    for (int ci = 0; ci < CIN; ++ci) {
        const float *src = in + (int64_t)ci * V;
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            const int xx = x + d * dx, yy = y + d * dy, zz = z + d * dz;
            const float val = inside(xx, yy, zz, G) ? src[((int64_t)zz * G + yy) * G + xx] : 0.f;
#pragma unroll
            for (int c = 0; c < COUT; ++c) acc[c] += sW[(c * CIN + ci) * 27 + t] * val;
        }
    }
#pragma unroll
    for (int c = 0; c < COUT; ++c) {
        pre[(int64_t)c * V + v] = acc[c];
        if (post) post[(int64_t)c * V + v] = relu ? fmaxf(acc[c], 0.f) : acc[c];
    }
}

// gin[ci][v] = (sum_{c, tap} W[c][ci][tap] g[c][v - d tap]) * (prev_pre[ci][v] > 0)
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float *g, const float *W, const float *prev_pre,
                                                       float *gin, int G, int d) {
    __shared__ float sW[COUT * CIN * 27];
    for (int i = threadIdx.x; i < COUT * CIN * 27; i += 256) sW[i] = W[i];
    __syncthreads();
    const int64_t V = (int64_t)G * G * G;
    const int64_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
    int x, y, z;
    vox_xyz(v, G, x, y, z);
    float acc[CIN];
#pragma unroll
    for (int c = 0; c < CIN; ++c) acc[c] = 0.f;
    for (int c = 0; c < COUT; ++c) {
        const float *src = g + (int64_t)c * V;
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            const int xx = x - d * dx, yy = y - d * dy, zz = z - d * dz;
            const float val = inside(xx, yy, zz, G) ? src[((int64_t)zz * G + yy) * G + xx] : 0.f;
#pragma unroll
            for (int k = 0; k < CIN; ++k) acc[k] += sW[(c * CIN + k) * 27 + t] * val;
        }
    }
#pragma unroll
    for (int k = 0; k < CIN; ++k) {
        const int64_t idx = (int64_t)k * V + v;
        gin[idx] = prev_pre[idx] > 0.f ? acc[k] : 0.f;
    }
}

// Weight gradients of one layer, one chunk of voxels per block:
// part[chunk][c][ci][tap] for the 9 taps of the block's dz plane, and the
// bias gradient on the dz = 0 blocks (slot 27).  Wavefront shuffles, then a
// fixed-order sum across the block: deterministic.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float *g, const float *in, float *part, int G, int d) {
    constexpr int NA = COUT * 9;
    __shared__ float sm[4][NA + COUT];
    const int64_t V = (int64_t)G * G * G;
    const int chunk = blockIdx.x, ci = blockIdx.y, dzi = blockIdx.z;  // dz = dzi - 1
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    float acc[NA];
    float accb[COUT];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.f;
#pragma unroll
    for (int c = 0; c < COUT; ++c) accb[c] = 0.f;
    const int64_t v0 = (int64_t)chunk * kChunk;
    const int64_t v1 = (v0 + kChunk < V) ? v0 + kChunk : V;
    const float *src = in + (int64_t)ci * V;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
        int x, y, z;
        vox_xyz(v, G, x, y, z);
        float gv[COUT];
#pragma unroll
        for (int c = 0; c < COUT; ++c) gv[c] = g[(int64_t)c * V + v];
#pragma unroll
        for (int t9 = 0; t9 < 9; ++t9) {
            const int dx = t9 % 3 - 1, dy = t9 / 3 - 1, dz = dzi - 1;
            const int xx = x + d * dx, yy = y + d * dy, zz = z + d * dz;
            const float val = inside(xx, yy, zz, G) ? src[((int64_t)zz * G + yy) * G + xx] : 0.f;
#pragma unroll
            for (int c = 0; c < COUT; ++c) acc[c * 9 + t9] += gv[c] * val;
        }
        if (dzi == 1 && ci == 0) {
#pragma unroll
            for (int c = 0; c < COUT; ++c) accb[c] += gv[c];
        }
    }
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[i] += __shfl_xor(acc[i], o, 64);
#pragma unroll
    for (int c = 0; c < COUT; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) accb[c] += __shfl_xor(accb[c], o, 64);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) sm[wave][i] = acc[i];
#pragma unroll
        for (int c = 0; c < COUT; ++c) sm[wave][NA + c] = accb[c];
    }
    __syncthreads();
    // part layout: [chunk][COUT][CIN][28]  (tap 0..26, bias in slot 27 of ci 0)
    for (int i = threadIdx.x; i < NA; i += 256) {
        const int c = i / 9, t9 = i % 9;
        const float sum = (sm[0][i] + sm[1][i]) + (sm[2][i] + sm[3][i]);
        part[(((int64_t)chunk * COUT + c) * CIN + ci) * 28 + dzi * 9 + t9] = sum;
    }
    if (dzi == 1 && ci == 0)
        for (int c = threadIdx.x; c < COUT; c += 256)
            part[(((int64_t)chunk * COUT + c) * CIN + 0) * 28 + 27] =
                (sm[0][NA + c] + sm[1][NA + c]) + (sm[2][NA + c] + sm[3][NA + c]);
}

// gW[c][ci][t] = sum_chunks part; gb[c] likewise (fixed order)
__global__ void k_conv_w_reduce(const float *part, int nchunk, int cin, int cout, float *gW, float *gb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * 27;
    if (i < nw) {
        const int c = i / (cin * 27), r = i % (cin * 27), k = r / 27, t = r % 27;
        float s = 0.f;
        for (int ch = 0; ch < nchunk; ++ch) s += part[(((int64_t)ch * cout + c) * cin + k) * 28 + t];
        gW[i] = s;
    } else if (i < nw + cout) {
        const int c = i - nw;
        float s = 0.f;
        for (int ch = 0; ch < nchunk; ++ch) s += part[(((int64_t)ch * cout + c) * cin + 0) * 28 + 27];
        gb[c] = s;
    }
}

// weighted squared error at the node voxels; dL/dy scattered into gy
// (targets whose voxel lies outside [0, V) are skipped: no access is made)
__global__ void k_nn_loss(const float *y, const int *vox, const float *tgt, const float *wt, int64_t nt, int64_t V,
                          float *gy, float *red) {
    __shared__ float sm[4];
    const int64_t i = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < nt) {
        const int v = vox[i];
        if (v >= 0 && v < V) {
            const float e = y[v] - tgt[i];
            l = wt[i] * e * e;
            atomicAdd(&gy[v], 2.f * wt[i] * e);
        }
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if (threadIdx.x % 64 == 0) sm[threadIdx.x / 64] = l;
    __syncthreads();
    if (threadIdx.x == 0) red[blockIdx.x] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// x0 at the Dirichlet slots: y(v_j) / (s h)
__global__ void k_nn_gather(const float *y, const int *gx, const int *gy, const int *gz, const int *perm,
                            const uint8_t *bc, int64_t m, int G, const double *s_dev, double h, double *x0) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int j = perm[k];
    const int64_t v = ((int64_t)gz[k] * G + gy[k]) * G + gx[k];
    x0[j] = (bc == nullptr || bc[j] == 0) ? (double)y[v] / (*s_dev * h) : 0.0;
}

// s = 1/rms(u) over the Dirichlet slots (1 if there are none or u = 0):
// one block, fixed-order reduction
__global__ __launch_bounds__(256) void k_nn_scale(const double *known, const uint8_t *bc, int64_t m, double *s_out) {
    __shared__ double ss[256], sc[256];
    double a = 0.0, c = 0.0;
    for (int64_t j = threadIdx.x; j < m; j += 256)
        if (bc == nullptr || bc[j] == 0) {
            a += known[j] * known[j];
            c += 1.0;
        }
    ss[threadIdx.x] = a;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ss[threadIdx.x] += ss[threadIdx.x + o];
            sc[threadIdx.x] += sc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *s_out = (ss[0] > 0.0 && sc[0] > 0.0) ? 1.0 / sqrt(ss[0] / sc[0]) : 1.0;
}

// ---------------------------------------------------------------- FP16 inference
// Implicit-GEMM convolution on the matrix cores: for each tap t, the 16 x 16
// weight block W[c][ci][t] (rows c) times the 16 x 16 block of activations
// act[v_j + d o_t][ci] of 16 consecutive voxels (columns j), accumulated in
// FP32 over the 27 taps.  Activations are FP16, channel-last [V][16], so one
// lane's four B values are one 8-byte load.  Operand layout of the 16x16x16
// MFMA (wave of 64): A[i][k] at lane i + 16 (k / 4), element k % 4; B[k][j] at
// lane j + 16 (k / 4), element k % 4; D[i][j] at lane j + 16 (i / 4),
// element i % 4.
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// planar FP32 [cin][V] -> channel-last FP16 [V][16], channels >= cin zero
__global__ void k_to_cl16(const float *x, int cin, int64_t V, _Float16 *o) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    h4 w[4];
#pragma unroll
    for (int c = 0; c < 16; ++c) w[c / 4][c % 4] = (_Float16)(c < cin ? x[(int64_t)c * V + v] : 0.f);
    h4 *dst = reinterpret_cast<h4 *>(o + v * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = w[q];
}

// FP32 parameters W[co][ci][27], b[co] of every layer -> FP16 Wp[l][27][16][16]
// (zero-padded to 16 x 16) and FP32 bp[l][16]
__global__ void k_pack16(const float *p, const int64_t *woff, const int64_t *boff, const int *ci, const int *co,
                         _Float16 *wp, float *bp) {
    const int l = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // t*256 + c*16 + k
    if (i >= 27 * 256) return;
    const int t = i / 256, c = (i / 16) % 16, k = i % 16;
    const float w = (c < co[l] && k < ci[l]) ? p[woff[l] + ((int64_t)c * ci[l] + k) * 27 + t] : 0.f;
    wp[(int64_t)l * 27 * 256 + i] = (_Float16)w;
    if (i < 16) bp[l * 16 + i] = i < co[l] ? p[boff[l] + i] : 0.f;
}

// Tiles of 16 consecutive voxels; each wave keeps its weight operands in
// registers and walks many tiles.  gfx950's 16x16x32 FP16 product takes two
// taps per instruction (K = 2 x 16 input channels): for each (dy, dz) row the
// dx = -1 and 0 taps share one product and dx = +1 takes one with a zero
// second half, so a tile needs 18 products instead of 27.  Lane (j, kq) holds
// voxel j's channels 8 (kq % 2) .. + 7 of the first tap (kq < 2) or of the
// second (kq >= 2), loaded as one 16-byte word; neighbours outside the grid
// are zero padding.  Blocks are mapped so that the 8 XCDs (blocks go round-
// robin to them) each sweep one contiguous range of tiles: the dilated taps
// then re-read planes that the same XCD's L2 just fetched.  Three
// accumulators (one per dz) keep three independent MFMA chains.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

template <bool LAST>
__global__ __launch_bounds__(256) void k_conv16(const _Float16 *__restrict__ in, const _Float16 *__restrict__ Wp,
                                                const float *__restrict__ bias, _Float16 *__restrict__ out,
                                                float *__restrict__ y, int G, int d, int64_t ntiles) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, kq = lane >> 4;
    const int half = 8 * (kq & 1);  // this lane's eight channels of its tap
    const bool first = kq < 2;      // first tap of the pair (else the second)
    const h8 zero8 = {};
    // A operands: per (dz, dy) row, the pair (dx = -1, dx = 0) and (dx = +1, none)
    h8 A[9][2];
#pragma unroll
    for (int rq = 0; rq < 9; ++rq) {
        const int t0 = rq * 3;  // tap index q * 9 + r * 3 + (dx + 1), rq = q * 3 + r
        const int ta = first ? t0 : t0 + 1;
        A[rq][0] = *reinterpret_cast<const h8 *>(Wp + (ta * 16 + j) * 16 + half);
        A[rq][1] = first ? *reinterpret_cast<const h8 *>(Wp + ((t0 + 2) * 16 + j) * 16 + half) : zero8;
    }
    float br[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) br[r] = bias[4 * kq + r];
    const int64_t V = (int64_t)G * G * G;
    const int xcd = blockIdx.x % 8, lb = blockIdx.x / 8, nlb = gridDim.x / 8;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t t_lo = xcd * per, t_hi = (t_lo + per < ntiles) ? t_lo + per : ntiles;
    for (int64_t tile = t_lo + (int64_t)lb * 4 + wave; tile < t_hi; tile += (int64_t)nlb * 4) {
        const int64_t v = tile * 16 + j;
        const bool valid = v < V;
        int x, yy, z;
        vox_xyz(valid ? v : 0, G, x, yy, z);
        f4 acc[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
        // pair 0: x - d (first) and x (second); pair 1: x + d (first), zero
        const int xa = first ? x - d : x;
        const int xb = x + d;
#pragma unroll
        for (int q = 0; q < 3; ++q) {  // dz = q - 1
            const int zz = z + d * (q - 1);
#pragma unroll
            for (int r = 0; r < 3; ++r) {  // dy = r - 1
                const int y2 = yy + d * (r - 1);
                const bool row_ok = valid && y2 >= 0 && y2 < G && zz >= 0 && zz < G;
                const _Float16 *rowp = in + (((int64_t)zz * G + y2) * G) * 16 + half;
                h8 b0 = zero8, b1 = zero8;
                if (row_ok && xa >= 0) b0 = *reinterpret_cast<const h8 *>(rowp + (int64_t)xa * 16);
                if (row_ok && first && xb < G) b1 = *reinterpret_cast<const h8 *>(rowp + (int64_t)xb * 16);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[q * 3 + r][0], b0, acc[q], 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[q * 3 + r][1], b1, acc[q], 0, 0, 0);
            }
        }
        if (valid) {
            const f4 s = (acc[0] + acc[1]) + acc[2];
            if (!LAST) {
                h4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = (_Float16)fmaxf(s[r] + br[r], 0.f);
                *reinterpret_cast<h4 *>(out + v * 16 + 4 * kq) = o;
            } else if (kq == 0) {
                y[v] = s[0] + br[0];
            }
        }
    }
}

int grid1(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 65535); }

template <int CIN, int COUT>
int conv_fwd(const float *in, const float *W, const float *b, float *pre, float *post, int G, int d, int relu,
             hipStream_t st) {
    const int64_t V = (int64_t)G * G * G;
    hipLaunchKernelGGL((k_conv_fwd<CIN, COUT>), dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, in, W, b, pre, post,
                       G, d, relu);
    BF_HIP(hipGetLastError());
    return 0;
}

int layer_fwd(bemfft_net *n, int l, const float *in, hipStream_t st) {
    const float *W = n->p + n->woff[l], *b = n->p + n->boff[l];
    float *pre = n->pre + (int64_t)l * n->width * n->V;
    float *post = n->post + (int64_t)l * n->width * n->V;
    const int relu = l < n->nl - 1;
    const int ci = n->ci[l], co = n->co[l];
    if (ci == 6 && co == 16) return conv_fwd<6, 16>(in, W, b, pre, post, n->G, n->dil[l], relu, st);
    if (ci == 16 && co == 16) return conv_fwd<16, 16>(in, W, b, pre, post, n->G, n->dil[l], relu, st);
    if (ci == 16 && co == 1) return conv_fwd<16, 1>(in, W, b, pre, post, n->G, n->dil[l], relu, st);
    set_error("network: unsupported layer shape");
    return BEMFFT_EUNSUPPORTED;
}

int forward(bemfft_net *n, const float *x, hipStream_t st) {
    const float *in = x;
    for (int l = 0; l < n->nl; ++l) {
        BF_CHECK(layer_fwd(n, l, in, st));
        in = n->post + (int64_t)l * n->width * n->V;
    }
    n->y = n->post + (int64_t)(n->nl - 1) * n->width * n->V;
    return 0;
}

template <int CIN, int COUT>
int bwd_w(const float *g, const float *in, float *part, int G, int d, float *gW, float *gb, hipStream_t st) {
    const int64_t V = (int64_t)G * G * G;
    const int nch = (int)((V + kChunk - 1) / kChunk);
    hipLaunchKernelGGL((k_conv_bwd_w<CIN, COUT>), dim3(nch, CIN, 3), dim3(256), 0, st, g, in, part, G, d);
    const int tot = COUT * CIN * 27 + COUT;
    hipLaunchKernelGGL(k_conv_w_reduce, dim3((tot + 255) / 256), dim3(256), 0, st, part, nch, CIN, COUT, gW, gb);
    BF_HIP(hipGetLastError());
    return 0;
}

template <int CIN, int COUT>
int bwd_d(const float *g, const float *W, const float *prev_pre, float *gin, int G, int d, hipStream_t st) {
    const int64_t V = (int64_t)G * G * G;
    hipLaunchKernelGGL((k_conv_bwd_data<CIN, COUT>), dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, g, W,
                       prev_pre, gin, G, d);
    BF_HIP(hipGetLastError());
    return 0;
}

// gradients of all parameters for the loss at the given node voxels
int gradients(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt, const float *wt,
              double *loss, hipStream_t st) {
    BF_CHECK(forward(n, x, st));
    float *gcur = n->ga, *gnext = n->gb;
    hipLaunchKernelGGL(k_fill, dim3(grid1(n->V)), dim3(256), 0, st, gcur, n->V, 0.f);
    const int nb = (int)((nt + 255) / 256);
    hipLaunchKernelGGL(k_nn_loss, dim3(nb), dim3(256), 0, st, n->y, vox, tgt, wt, nt, n->V, gcur, n->red);
    BF_HIP(hipGetLastError());
    std::vector<float> hred(nb);
    BF_HIP(hipMemcpyAsync(hred.data(), n->red, nb * sizeof(float), hipMemcpyDeviceToHost, st));
    for (int l = n->nl - 1; l >= 0; --l) {
        const float *in = l == 0 ? x : n->post + (int64_t)(l - 1) * n->width * n->V;
        float *gW = n->g + n->woff[l], *gb = n->g + n->boff[l];
        const int ci = n->ci[l], co = n->co[l], d = n->dil[l];
        int s;
        if (ci == 6 && co == 16) s = bwd_w<6, 16>(gcur, in, n->part, n->G, d, gW, gb, st);
        else if (ci == 16 && co == 16) s = bwd_w<16, 16>(gcur, in, n->part, n->G, d, gW, gb, st);
        else s = bwd_w<16, 1>(gcur, in, n->part, n->G, d, gW, gb, st);
        BF_CHECK(s);
        if (l > 0) {
            const float *W = n->p + n->woff[l];
            const float *prev_pre = n->pre + (int64_t)(l - 1) * n->width * n->V;
            if (co == 16) s = bwd_d<16, 16>(gcur, W, prev_pre, gnext, n->G, d, st);
            else s = bwd_d<16, 1>(gcur, W, prev_pre, gnext, n->G, d, st);
            BF_CHECK(s);
            std::swap(gcur, gnext);
        }
    }
    BF_HIP(hipStreamSynchronize(st));
    double L = 0.0;
    for (float v : hred) L += v;
    if (loss) *loss = L;
    return 0;
}

int input_impl(bemfft_net *n, bemfft_plan *p, const uint8_t *bc, const double *known, double s_host,
               const double *s_dev, float *x, hipStream_t st) {
    if (p->dim != 3 || p->kernel != BEMFFT_LAPLACE3D || p->n[0] != n->G || p->n[1] != n->G || p->n[2] != n->G) {
        set_error("net_input: needs a Laplace 3D plan on the network's grid");
        return BEMFFT_EINVAL;
    }
    if (p->m > n->cap) {
        BF_HIP(hipStreamSynchronize(st));
        for (double **q : {&n->dq, &n->du, &n->db}) {
            if (*q) (void)hipFree(*q);
            *q = nullptr;
        }
        n->cap = 0;
        if (hipMalloc(&n->dq, p->m * 8) != hipSuccess || hipMalloc(&n->du, p->m * 8) != hipSuccess ||
            hipMalloc(&n->db, p->m * 8) != hipSuccess) {
            set_error("net_input: allocation failed");
            return BEMFFT_ENOMEM;
        }
        n->cap = p->m;
    }
    const unsigned gm = (unsigned)((p->m + 255) / 256);
    hipLaunchKernelGGL(k_nn_split, dim3(gm), dim3(256), 0, st, bc, known, n->dq, n->du, p->m);
    BF_HIP(hipGetLastError());
    BF_CHECK(launch_apply(p, p->eng, n->dq, n->du, n->db, st));
    hipLaunchKernelGGL(k_fill, dim3(grid1(n->cin * n->V)), dim3(256), 0, st, x, n->cin * n->V, 0.f);
    hipLaunchKernelGGL(k_nn_input, dim3(gm), dim3(256), 0, st, p->d_gx, p->d_gy, p->d_gz, p->d_perm, p->d_w, p->d_nrm,
                       known, n->db, bc, p->m, n->G, 1.0 / (p->h * p->h), s_host, s_dev, x, n->V);
    BF_HIP(hipGetLastError());
    return 0;
}

// FP16 inference: x planar FP32 [6][V] -> n->y (FP32 [V])
int infer(bemfft_net *n, const float *x, hipStream_t st) {
    const int64_t V = n->V;
    hipLaunchKernelGGL(k_to_cl16, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, x, n->cin, V, n->ha);
    hipLaunchKernelGGL(k_pack16, dim3(27, n->nl), dim3(256), 0, st, n->p, n->d_woff, n->d_boff, n->d_ci, n->d_co,
                       n->wp, n->bp);
    BF_HIP(hipGetLastError());
    const int64_t ntiles = (V + 15) / 16;
    // a multiple of 8 blocks (one share per XCD), at most 8 per CU
    const int64_t per_xcd = ((ntiles + 7) / 8 + 3) / 4;
    const unsigned blocks = 8u * (unsigned)std::max<int64_t>(1, std::min<int64_t>(per_xcd, 256));
    float *y = n->post + (int64_t)(n->nl - 1) * n->width * V;
    _Float16 *in = n->ha, *out = n->hb;
    for (int l = 0; l < n->nl; ++l) {
        const _Float16 *W = n->wp + (int64_t)l * 27 * 256;
        const float *b = n->bp + l * 16;
        if (l == n->nl - 1)
            hipLaunchKernelGGL(k_conv16<true>, dim3(blocks), dim3(256), 0, st, in, W, b, out, y, n->G, n->dil[l], ntiles);
        else
            hipLaunchKernelGGL(k_conv16<false>, dim3(blocks), dim3(256), 0, st, in, W, b, out, y, n->G, n->dil[l],
                               ntiles);
        BF_HIP(hipGetLastError());
        std::swap(in, out);
    }
    n->y = y;
    return 0;
}

}  // namespace
}  // namespace bemfft

using namespace bemfft;

extern "C" {

int bemfft_net_create(bemfft_net **out, int grid, int width, int nlayers, const int *dilations, uint64_t seed,
                      void *stream) {
    (void)stream;
    if (!out || grid < 4 || grid > 256 || width != 16 || nlayers < 2 || nlayers > 8 || !dilations) {
        set_error("net_create: grid in [4, 256], width 16, 2..8 layers, dilations required");
        return BEMFFT_EINVAL;
    }
    *out = nullptr;
    bemfft_net *n = new (std::nothrow) bemfft_net();
    if (!n) return BEMFFT_ENOMEM;
    n->G = grid;
    n->cin = 6;
    n->width = width;
    n->nl = nlayers;
    n->V = (int64_t)grid * grid * grid;
    for (int l = 0; l < nlayers; ++l) {
        if (dilations[l] < 1 || dilations[l] > grid) {
            delete n;
            set_error("net_create: bad dilation");
            return BEMFFT_EINVAL;
        }
        n->dil.push_back(dilations[l]);
        n->ci.push_back(l == 0 ? n->cin : width);
        n->co.push_back(l == nlayers - 1 ? 1 : width);
    }
    std::vector<float> hp;
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int l = 0; l < nlayers; ++l) {
        n->woff.push_back((int64_t)hp.size());
        const int fan = n->ci[l] * 27;
        const double sd = std::sqrt(2.0 / fan) * (l == nlayers - 1 ? 0.1 : 1.0);
        for (int i = 0; i < n->co[l] * fan; ++i) hp.push_back((float)(sd * nd(rng)));
        n->boff.push_back((int64_t)hp.size());
        for (int i = 0; i < n->co[l]; ++i) hp.push_back(0.f);
    }
    n->nparam = (int64_t)hp.size();
    const int nch = (int)((n->V + kChunk - 1) / kChunk);
    const size_t act = (size_t)nlayers * width * n->V * sizeof(float);
    if (hipMalloc(&n->p, n->nparam * 4) != hipSuccess || hipMalloc(&n->g, n->nparam * 4) != hipSuccess ||
        hipMalloc(&n->m, n->nparam * 4) != hipSuccess || hipMalloc(&n->v, n->nparam * 4) != hipSuccess ||
        hipMalloc(&n->pre, act) != hipSuccess || hipMalloc(&n->post, act) != hipSuccess ||
        hipMalloc(&n->ga, (size_t)width * n->V * 4) != hipSuccess ||
        hipMalloc(&n->gb, (size_t)width * n->V * 4) != hipSuccess ||
        hipMalloc(&n->part, (size_t)nch * width * width * 28 * 4) != hipSuccess ||
        hipMalloc(&n->red, (size_t)65536 * 4) != hipSuccess ||
        hipMalloc(&n->ha, (size_t)n->V * 16 * 2) != hipSuccess || hipMalloc(&n->hb, (size_t)n->V * 16 * 2) != hipSuccess ||
        hipMalloc(&n->wp, (size_t)nlayers * 27 * 256 * 2) != hipSuccess ||
        hipMalloc(&n->bp, (size_t)nlayers * 16 * 4) != hipSuccess || hipMalloc(&n->sdev, 8) != hipSuccess ||
        hipMalloc(&n->d_woff, nlayers * 8) != hipSuccess || hipMalloc(&n->d_boff, nlayers * 8) != hipSuccess ||
        hipMalloc(&n->d_ci, nlayers * 4) != hipSuccess || hipMalloc(&n->d_co, nlayers * 4) != hipSuccess ||
        hipMemcpy(n->d_woff, n->woff.data(), nlayers * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->d_boff, n->boff.data(), nlayers * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->d_ci, n->ci.data(), nlayers * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->d_co, n->co.data(), nlayers * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->p, hp.data(), n->nparam * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, n->nparam * 4) != hipSuccess || hipMemset(n->v, 0, n->nparam * 4) != hipSuccess) {
        bemfft_net_destroy(n);
        set_error("net_create: allocation failed");
        return BEMFFT_ENOMEM;
    }
    *out = n;
    return 0;
}

int bemfft_net_destroy(bemfft_net *n) {
    if (!n) return 0;
    for (float *q : {n->p, n->g, n->m, n->v, n->pre, n->post, n->ga, n->gb, n->part, n->red})
        if (q) (void)hipFree(q);
    for (double *q : {n->dq, n->du, n->db, n->sdev})
        if (q) (void)hipFree(q);
    for (void *q : {(void *)n->ha, (void *)n->hb, (void *)n->wp, (void *)n->bp, (void *)n->d_woff, (void *)n->d_boff,
                    (void *)n->d_ci, (void *)n->d_co})
        if (q) (void)hipFree(q);
    delete n;
    return 0;
}

int64_t bemfft_net_num_params(const bemfft_net *n) { return n ? n->nparam : 0; }

int bemfft_net_get_params(const bemfft_net *n, float *host) {
    if (!n || !host) return BEMFFT_EINVAL;
    BF_HIP(hipMemcpy(host, n->p, n->nparam * 4, hipMemcpyDeviceToHost));
    return 0;
}

int bemfft_net_set_params(bemfft_net *n, const float *host) {
    if (!n || !host) return BEMFFT_EINVAL;
    BF_HIP(hipMemcpy(n->p, host, n->nparam * 4, hipMemcpyHostToDevice));
    return 0;
}

int bemfft_net_input(bemfft_net *n, bemfft_plan *p, const uint8_t *bc, const double *known, double scale, float *x,
                     void *stream) {
    if (!n || !p || !known || !x) {
        set_error("net_input: null argument");
        return BEMFFT_EINVAL;
    }
    return input_impl(n, p, bc, known, scale, nullptr, x, (hipStream_t)stream);
}

int bemfft_net_forward(bemfft_net *n, const float *x, float *y, void *stream) {
    if (!n || !x || !y) return BEMFFT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    BF_CHECK(forward(n, x, st));
    BF_HIP(hipMemcpyAsync(y, n->y, n->V * 4, hipMemcpyDeviceToDevice, st));
    return 0;
}

int bemfft_net_infer(bemfft_net *n, const float *x, float *y, void *stream) {
    if (!n || !x || !y) return BEMFFT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    BF_CHECK(infer(n, x, st));
    BF_HIP(hipMemcpyAsync(y, n->y, n->V * 4, hipMemcpyDeviceToDevice, st));
    return 0;
}

int bemfft_net_gradients(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt, const float *wt,
                         double *loss, float *grad_host, void *stream) {
    if (!n || !x || nt < 1 || nt > kMaxTargets || !vox || !tgt || !wt) {
        set_error("net_gradients: null argument or target count outside [1, 2^24]");
        return BEMFFT_EINVAL;
    }
    BF_CHECK(gradients(n, x, nt, vox, tgt, wt, loss, (hipStream_t)stream));
    if (grad_host) BF_HIP(hipMemcpy(grad_host, n->g, n->nparam * 4, hipMemcpyDeviceToHost));
    return 0;
}

int bemfft_net_train_step(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt, const float *wt,
                          float lr, double *loss, void *stream) {
    if (!n || !x || nt < 1 || nt > kMaxTargets || !vox || !tgt || !wt || !(lr > 0.f)) {
        set_error("net_train_step: null argument, target count outside [1, 2^24] or lr <= 0");
        return BEMFFT_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    BF_CHECK(gradients(n, x, nt, vox, tgt, wt, loss, st));
    n->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - (float)std::pow(b1, (double)n->t), c2 = 1.f - (float)std::pow(b2, (double)n->t);
    hipLaunchKernelGGL(k_adam, dim3(grid1(n->nparam)), dim3(256), 0, st, n->p, n->g, n->m, n->v, n->nparam, lr, b1, b2,
                       c1, c2, 1e-8f);
    BF_HIP(hipGetLastError());
    return 0;
}

int bemfft_net_guess(bemfft_net *n, bemfft_plan *p, const uint8_t *bc, const double *known, float *xbuf,
                     double *x0, void *stream) {
    if (!n || !p || !known || !xbuf || !x0) return BEMFFT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_nn_scale, dim3(1), dim3(256), 0, st, known, bc, p->m, n->sdev);
    BF_HIP(hipGetLastError());
    BF_CHECK(input_impl(n, p, bc, known, 1.0, n->sdev, xbuf, st));
    BF_CHECK(infer(n, xbuf, st));
    hipLaunchKernelGGL(k_nn_gather, dim3((unsigned)((p->m + 255) / 256)), dim3(256), 0, st, n->y, p->d_gx, p->d_gy,
                       p->d_gz, p->d_perm, bc, p->m, n->G, n->sdev, p->h, x0);
    BF_HIP(hipGetLastError());
    return 0;
}

// Node voxel index and weight of each node in the caller's order (for the
// training targets).
int bemfft_plan_node_voxels(const bemfft_plan *p, int *vox_host, double *w_host) {
    if (!p) return BEMFFT_EINVAL;
    const int64_t m = p->m;
    std::vector<int> gx(m), gy(m), gz(m), perm(m);
    std::vector<double> w(m);
    BF_HIP(hipMemcpy(gx.data(), p->d_gx, m * 4, hipMemcpyDeviceToHost));
    BF_HIP(hipMemcpy(gy.data(), p->d_gy, m * 4, hipMemcpyDeviceToHost));
    BF_HIP(hipMemcpy(gz.data(), p->d_gz, m * 4, hipMemcpyDeviceToHost));
    BF_HIP(hipMemcpy(perm.data(), p->d_perm, m * 4, hipMemcpyDeviceToHost));
    BF_HIP(hipMemcpy(w.data(), p->d_w, m * 8, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < m; ++k) {
        const int j = perm[k];
        if (vox_host) vox_host[j] = (int)(((int64_t)gz[k] * p->n[1] + gy[k]) * p->n[0] + gx[k]);
        if (w_host) w_host[j] = w[k];
    }
    return 0;
}

}  // extern "C"
