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
// Training (FP32 storage and arithmetic, the convolutions on the matrix
// cores) minimises the weighted squared error sum_j wt_j (y(v_j) - s h q_j)^2
// against solved problems, with Adam.
// Inference (the guess) runs in FP16 on the matrix cores with FP32
// accumulation.  The solve keeps the guess only when its residual is smaller
// than ||b|| (plain GMRES from zero otherwise).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <type_traits>
#include <vector>

#include "internal.hpp"

struct bemfft_net {
    int G = 0, cin = 0, width = 0, nl = 0;
    int64_t V = 0;  // G^3
    std::vector<int> dil, ci, co;
    std::vector<int64_t> woff, boff;
    int64_t nparam = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // params, grads, Adam moments
    float *xcl = nullptr;                   // training input, channel-last [V][8]
    float *pre = nullptr, *post = nullptr;  // per layer [V][co] (post = relu(pre) for hidden layers)
    float *ga = nullptr, *gb = nullptr;     // gradient ping-pong [V][width]
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

constexpr int kWgBlocks = 512;  // most weight-gradient blocks (partial sums) of a layer
constexpr int64_t kMaxTargets = 65536LL * 256;  // loss partial sums: one per 256 targets

__device__ __forceinline__ void vox_xyz(int64_t v, int G, int &x, int &y, int &z) {
    x = (int)(v % G);
    y = (int)((v / G) % G);
    z = (int)(v / ((int64_t)G * G));
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

// gW[c][ci][t] = sum over the chunks of part; gb[c] likewise.  A block
// takes 32 outputs; eight groups of 32 threads sum eight contiguous slices
// of the chunks, added in a fixed order: deterministic.
__global__ __launch_bounds__(256) void k_conv_w_reduce(const float *part, int nchunk, int cin, int cout, float *gW,
                                                       float *gb) {
    __shared__ float sm[8][32];
    const int o = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + o;
    const int nw = cout * cin * 27;
    int off = -1;
    if (i < nw) {
        const int c = i / (cin * 27), r = i % (cin * 27), k = r / 27, t = r % 27;
        off = (c * cin + k) * 28 + t;
    } else if (i < nw + cout) {
        off = ((i - nw) * cin + 0) * 28 + 27;
    }
    const int per = (nchunk + 7) / 8, c0 = sl * per, c1 = c0 + per < nchunk ? c0 + per : nchunk;
    const int64_t stride = (int64_t)cout * cin * 28;
    float s = 0.f;
    if (off >= 0)
        for (int ch = c0; ch < c1; ++ch) s += part[ch * stride + off];
    sm[sl][o] = s;
    __syncthreads();
    if (sl == 0 && off >= 0) {
        const float tot = ((sm[0][o] + sm[1][o]) + (sm[2][o] + sm[3][o])) + ((sm[4][o] + sm[5][o]) + (sm[6][o] + sm[7][o]));
        if (i < nw) gW[i] = tot;
        else gb[i - nw] = tot;
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

// ---------------------------------------------------------------- FP32 training on the matrix cores
// Every layer trains as an implicit GEMM on gfx950's FP32 16x16x4 matrix
// product: FP32 operands, FP32 accumulation.  Activations and their
// gradients are channel-last: [V][16] for the hidden layers, [V][8] for the
// input (channels 6 and 7 zero), [V] for the one-channel output; so a lane
// fetches the channels of its products with one 8- or 16-byte load.
// Operand layout (wave of 64): A[i][k] at lane i + 16 k, B[k][j] at lane
// j + 16 k, D[i][j] at lane j + 16 (i / 4), element i % 4.  The K index of a
// product is a summation index, so lane group k may hold any channel: with
// CP stored channels, lane (j, k) of step s (NS = CP / 4 steps) takes
// channel NS k + s.  Output rows beyond a layer's channels are zero.  Work
// is split in contiguous ranges, ranked so that each of the 8 XCDs (blocks
// go round-robin to them) sweeps one contiguous eighth of the grid: the
// dilated taps then re-read planes its own L2 fetched.
typedef float f2 __attribute__((ext_vector_type(2)));
template <int N>
using fvec = typename std::conditional<N == 4, f4, typename std::conditional<N == 2, f2, float>::type>::type;

__device__ __forceinline__ int xcd_rank(int b, int nb) { return nb % 8 == 0 ? (b % 8) * (nb / 8) + b / 8 : b; }

__device__ __forceinline__ float lane_elem(float v, int) { return v; }
template <typename T>
__device__ __forceinline__ float lane_elem(T v, int s) { return v[s]; }

// Planar input [6][V] -> channel-last [V][8], channels 6 and 7 zero.
__global__ void k_to_cl8(const float *x, int64_t V, float *o) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    f4 a, b;
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = x[c * V + v];
    b[0] = x[4 * V + v];
    b[1] = x[5 * V + v];
    b[2] = 0.f;
    b[3] = 0.f;
    reinterpret_cast<f4 *>(o + v * 8)[0] = a;
    reinterpret_cast<f4 *>(o + v * 8)[1] = b;
}

// Weight operands of one layer in LDS: sA[t][lane] holds lane (j, k)'s NS
// values of tap t, W[j][NS k + s][t] (forward) or W[NS k + s][j][t] (data
// gradient, transposed); zero beyond the layer's channels.
template <int NS, bool TRANSPOSED>
__device__ __forceinline__ void stage_weights(const float *__restrict__ W, int cin, int cout, fvec<NS> (*sA)[64]) {
    for (int i = threadIdx.x; i < 27 * 64; i += blockDim.x) {
        const int t = i / 64, ln = i % 64, jj = ln & 15, k = ln >> 4;
        fvec<NS> a = {};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = NS * k + s;  // the K channel of this lane group and step
            float w = 0.f;
            if (!TRANSPOSED && jj < cout && c < cin) w = W[(jj * cin + c) * 27 + t];
            if (TRANSPOSED && c < cout && jj < cin) w = W[(c * cin + jj) * 27 + t];
            if constexpr (NS == 1) a = w;
            else a[s] = w;
        }
        sA[t][ln] = a;
    }
}

// One z plane (dz = q - 1, times SIGN) of a tile's taps: B[r * 3 + s3] holds
// lane (j, k)'s NS channels of voxel (x + SIGN d dx, y + SIGN d dy, z + SIGN
// d dz) of the channel-last array src (CP channels per voxel), zero outside
// the grid or for lane groups beyond KMAX channels.
template <int CP, int NS, int SIGN>
__device__ __forceinline__ void load_plane(const float *__restrict__ src, int x, int y, int z, bool valid, int q, int G,
                                           int d, int kq, fvec<NS> *B) {
    const int zz = z + SIGN * d * (q - 1);
    const bool zok = valid && NS * kq < CP && zz >= 0 && zz < G;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int y2 = y + SIGN * d * (r - 1);
        const bool rok = zok && y2 >= 0 && y2 < G;
        const int row = (zz * G + y2) * G;
#pragma unroll
        for (int s3 = 0; s3 < 3; ++s3) {
            const int xx = x + SIGN * d * (s3 - 1);
            const bool ok = rok && xx >= 0 && xx < G;
            // branch-free: an in-bounds load, then zero where the tap leaves the grid
            // (keeps the loads in one block, so waits count only the loads needed)
            const fvec<NS> val = *reinterpret_cast<const fvec<NS> *>(src + (ok ? (int64_t)(row + xx) * CP + NS * kq : 0));
            B[r * 3 + s3] = ok ? val : fvec<NS>{};
        }
    }
}

// Forward of one layer, out[v][c] = b[c] + sum_{ci, t} W[c][ci][t] in[v + d o_t][ci]:
// per tap t, D (16 output channels x 16 consecutive voxels) += W_t (16 x CP)
// in(. + d o_t) (CP x 16), NS products of four channels.
template <int CIN, int CP, int COUT>
__global__ __launch_bounds__(256) void k_conv_fwd_mx(const float *__restrict__ in, const float *__restrict__ W,
                                                     const float *__restrict__ bias, float *__restrict__ pre,
                                                     float *__restrict__ post, int G, int d, int relu, int ntiles) {
    constexpr int NS = CP / 4;
    typedef fvec<NS> VT;
    __shared__ VT sA[27][64];
    stage_weights<NS, false>(W, CIN, COUT, sA);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, kq = lane >> 4;
    f4 br;
#pragma unroll
    for (int r = 0; r < 4; ++r) br[r] = 4 * kq + r < COUT ? bias[4 * kq + r] : 0.f;
    const int V = G * G * G;
    const int nb = gridDim.x, per = (ntiles + nb - 1) / nb;
    const int t_lo = xcd_rank(blockIdx.x, nb) * per;
    const int t_hi = t_lo + per < ntiles ? t_lo + per : ntiles;
    int tile = t_lo + wave;
    VT Bc[9], Bn[9];
    int x = 0, y = 0, z = 0, v = 0;
    bool valid = false;
    auto coords = [&](int tl, int &cx, int &cy, int &cz, int &cv, bool &cval) {
        cv = tl * 16 + j;
        cval = cv < V;
        const int vv = cval ? cv : 0;
        cx = vv % G;
        cy = (vv / G) % G;
        cz = vv / (G * G);
    };
    if (tile < t_hi) {
        coords(tile, x, y, z, v, valid);
        load_plane<CP, NS, 1>(in, x, y, z, valid, 0, G, d, kq, Bc);
    }
    for (; tile < t_hi; tile += 4) {
        int xn = 0, yn = 0, zn = 0, vn = 0;
        bool validn = false;
        const bool more = tile + 4 < t_hi;
        if (more) coords(tile + 4, xn, yn, zn, vn, validn);
        f4 acc[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[r] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            __builtin_amdgcn_sched_barrier(0);  // one plane's weight words live at a time
            if (q < 2) load_plane<CP, NS, 1>(in, x, y, z, valid, q + 1, G, d, kq, Bn);
            else if (more) load_plane<CP, NS, 1>(in, xn, yn, zn, validn, 0, G, d, kq, Bn);
#pragma unroll
            for (int s3 = 0; s3 < 3; ++s3)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const VT a = sA[q * 9 + r * 3 + s3][lane];
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(lane_elem(a, s), lane_elem(Bc[r * 3 + s3], s),
                                                                      acc[r], 0, 0, 0);
                }
#pragma unroll
            for (int e = 0; e < 9; ++e) Bc[e] = Bn[e];
        }
        if (valid) {
            const f4 o = ((acc[0] + acc[1]) + acc[2]) + br;
            if constexpr (COUT == 16) {
                *reinterpret_cast<f4 *>(pre + (int64_t)v * 16 + 4 * kq) = o;
                if (post) {
                    f4 p;
#pragma unroll
                    for (int r = 0; r < 4; ++r) p[r] = relu ? fmaxf(o[r], 0.f) : o[r];
                    *reinterpret_cast<f4 *>(post + (int64_t)v * 16 + 4 * kq) = p;
                }
            } else if (kq == 0) {
                pre[v] = o[0];
                if (post) post[v] = relu ? fmaxf(o[0], 0.f) : o[0];
            }
        }
        x = xn;
        y = yn;
        z = zn;
        v = vn;
        valid = validn;
    }
}

// Data gradient into a 16-channel layer, gin[v][ci] = (prev_pre[v][ci] > 0)
// sum_{c, t} W[c][ci][t] g[v - d o_t][c]: per tap t, D (16 input channels x
// 16 voxels) += W_t^T (16 x COUT) g(. - d o_t) (COUT x 16); the same plane
// pipeline as the forward.
template <int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_data_mx(const float *__restrict__ g, const float *__restrict__ W,
                                                          const float *__restrict__ prev_pre, float *__restrict__ gin,
                                                          int G, int d, int ntiles) {
    constexpr int NS = COUT == 16 ? 4 : 1;
    typedef fvec<NS> VT;
    __shared__ VT sA[27][64];
    stage_weights<NS, true>(W, 16, COUT, sA);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, kq = lane >> 4;
    const int V = G * G * G;
    const int nb = gridDim.x, per = (ntiles + nb - 1) / nb;
    const int t_lo = xcd_rank(blockIdx.x, nb) * per;
    const int t_hi = t_lo + per < ntiles ? t_lo + per : ntiles;
    int tile = t_lo + wave;
    VT Bc[9], Bn[9];
    int x = 0, y = 0, z = 0, v = 0;
    bool valid = false;
    auto coords = [&](int tl, int &cx, int &cy, int &cz, int &cv, bool &cval) {
        cv = tl * 16 + j;
        cval = cv < V;
        const int vv = cval ? cv : 0;
        cx = vv % G;
        cy = (vv / G) % G;
        cz = vv / (G * G);
    };
    if (tile < t_hi) {
        coords(tile, x, y, z, v, valid);
        load_plane<COUT, NS, -1>(g, x, y, z, valid, 0, G, d, kq, Bc);
    }
    for (; tile < t_hi; tile += 4) {
        int xn = 0, yn = 0, zn = 0, vn = 0;
        bool validn = false;
        const bool more = tile + 4 < t_hi;
        if (more) coords(tile + 4, xn, yn, zn, vn, validn);
        f4 acc[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[r] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            __builtin_amdgcn_sched_barrier(0);  // one plane's weight words live at a time
            if (q < 2) load_plane<COUT, NS, -1>(g, x, y, z, valid, q + 1, G, d, kq, Bn);
            else if (more) load_plane<COUT, NS, -1>(g, xn, yn, zn, validn, 0, G, d, kq, Bn);
#pragma unroll
            for (int s3 = 0; s3 < 3; ++s3)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const VT a = sA[q * 9 + r * 3 + s3][lane];
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(lane_elem(a, s), lane_elem(Bc[r * 3 + s3], s),
                                                                      acc[r], 0, 0, 0);
                }
#pragma unroll
            for (int e = 0; e < 9; ++e) Bc[e] = Bn[e];
        }
        if (valid) {
            const f4 o = (acc[0] + acc[1]) + acc[2];
            const f4 pp = *reinterpret_cast<const f4 *>(prev_pre + (int64_t)v * 16 + 4 * kq);
            f4 w;
#pragma unroll
            for (int r = 0; r < 4; ++r) w[r] = pp[r] > 0.f ? o[r] : 0.f;
            *reinterpret_cast<f4 *>(gin + (int64_t)v * 16 + 4 * kq) = w;
        }
        x = xn;
        y = yn;
        z = zn;
        v = vn;
        valid = validn;
    }
}

// Weight and bias gradients of one layer, gW[c][ci][t] = sum_v g[v][c]
// in[v + d o_t][ci]: per tap t, D (16 output channels x 16 input channels)
// += g (16 x 4 voxels) in(. + d o_t)^T (4 x 16), four voxels per product,
// one accumulator per tap.  blockIdx.y picks the z offset of the taps (9
// taps per block).  A block walks slabs of kSlab voxels; lane (j, k) of wave
// w keeps g of voxels 64 k + 16 w + i (i < 16, the K index of product i) in
// registers for the whole slab.  Tap by tap, the slab's shifted input (zero
// where the tap leaves the grid) is fetched with coalesced 16-byte loads --
// the next two taps' into registers while the current one is multiplied --
// and stored transposed in LDS, [ci][u] with padded rows, so that a lane
// reads the B values of four products with one 16-byte LDS load (two
// buffers, one barrier per tap).  The four wavefronts' sums are added
// through LDS in a fixed order into the partial part[blockIdx.x][c][ci][28]
// (taps 0..26, bias in slot 27 of ci 0), which k_conv_w_reduce adds up in a
// fixed order: deterministic.
constexpr int kSlab = 256;

template <int CIN, int CP, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w_mx(const float *__restrict__ g, const float *__restrict__ in,
                                                       float *__restrict__ part, int G, int d, int nslabs) {
    constexpr int QV = CP / 4;            // 16-byte words per voxel of the input
    constexpr int NF = kSlab * QV / 256;  // of them staged per thread and tap
    constexpr int LD = kSlab + 4;         // padded row of the transposed slab
    __shared__ __align__(16) float sT[2][CP * LD];
    __shared__ float sR[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, kq = lane >> 4;
    const int qz = blockIdx.y;  // taps 9 qz .. 9 qz + 8 (dz = qz - 1)
    const int V = G * G * G, GG = G * G;
    const int ubase = 64 * kq + 16 * wave;  // this lane's product voxels: ubase + i
    f4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    float accb = 0.f;  // bias of channel j from this lane's voxels
    const int nb = gridDim.x, per = (nslabs + nb - 1) / nb;
    const int s_lo = xcd_rank(blockIdx.x, nb) * per;
    const int s_hi = s_lo + per < nslabs ? s_lo + per : nslabs;
    for (int slab = s_lo; slab < s_hi; ++slab) {
        const int v0 = slab * kSlab;
        // staged words: f = tid + 256 i is voxel f / QV, channels 4 (f % QV) .. + 3
        int ux[NF], uy[NF], uz[NF];
        bool uval[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int vs = v0 + (tid + 256 * i) / QV;
            uval[i] = vs < V;
            const int vv = uval[i] ? vs : 0;
            ux[i] = vv % G;
            uy[i] = (vv / G) % G;
            uz[i] = vv / GG;
        }
        auto fetch = [&](int t9, f4 *R) {
            const int dx = d * (t9 % 3 - 1), dy = d * (t9 / 3 - 1), dz = d * (qz - 1);
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const int f = tid + 256 * i;
                const int xx = ux[i] + dx, yy = uy[i] + dy, zz = uz[i] + dz;
                const bool ok = uval[i] && xx >= 0 && xx < G && yy >= 0 && yy < G && zz >= 0 && zz < G;
                const f4 val =
                    *reinterpret_cast<const f4 *>(in + (ok ? ((int64_t)(zz * G + yy) * G + xx) * CP + 4 * (f % QV) : 0));
                R[i] = ok ? val : f4{0.f, 0.f, 0.f, 0.f};
            }
        };
        f4 R0[NF], R1[NF];  // taps t and t + 1 in flight
        fetch(0, R0);
        fetch(1, R1);
        float a[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int vg = v0 + ubase + i;
            const bool ok = j < COUT && vg < V;
            const float val = g[ok ? (int64_t)vg * COUT + (COUT == 16 ? j : 0) : 0];
            a[i] = ok ? val : 0.f;
            accb += a[i];
        }
        __syncthreads();  // the previous slab's products have read both buffers
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            float *T = sT[t & 1];
            f4 *R = (t & 1) ? R1 : R0;
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const int f = tid + 256 * i, u = f / QV, c0 = 4 * (f % QV);
#pragma unroll
                for (int e = 0; e < 4; ++e) T[(c0 + e) * LD + u] = R[i][e];
            }
            __syncthreads();
            if (t + 2 < 9) fetch(t + 2, R);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                f4 b = f4{0.f, 0.f, 0.f, 0.f};
                if (j < CP) b = *reinterpret_cast<const f4 *>(T + j * LD + ubase + 4 * h);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * h + e], b[e], acc[t], 0, 0, 0);
            }
        }
    }
    // block sums in a fixed order
    float *pb = part + (int64_t)blockIdx.x * COUT * CIN * 28;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sR[wave][lane * 4 + r] = acc[t][r];
        __syncthreads();
        {
            const int i = tid, ln = i >> 2, c = 4 * (ln >> 4) + (i & 3), ci = ln & 15;
            const float s = (sR[0][i] + sR[1][i]) + (sR[2][i] + sR[3][i]);
            if (c < COUT && ci < CIN) pb[(c * CIN + ci) * 28 + 9 * qz + t] = s;
        }
        __syncthreads();
    }
    if (qz == 0) {  // the bias once per chunk
        accb += __shfl_xor(accb, 16, 64);
        accb += __shfl_xor(accb, 32, 64);
        if (kq == 0) sR[wave][j] = accb;
        __syncthreads();
        if (tid < COUT) pb[(tid * CIN + 0) * 28 + 27] = (sR[0][tid] + sR[1][tid]) + (sR[2][tid] + sR[3][tid]);
    }
}

int grid1(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 65535); }

// Blocks for a sweep of n work items, about 'each' per block; above 8, a
// multiple of 8 (one equal share per XCD).  cap is a multiple of 8.
int mx_blocks(int64_t n, int64_t each, int cap) {
    int64_t b = std::max<int64_t>(1, std::min<int64_t>((n + each - 1) / each, cap));
    if (b > 8) b = (b + 7) / 8 * 8;
    return (int)b;
}

template <int CIN, int CP, int COUT>
int conv_fwd(const float *in, const float *W, const float *b, float *pre, float *post, int G, int d, int relu,
             hipStream_t st) {
    const int64_t V = (int64_t)G * G * G;
    const int ntiles = (int)((V + 15) / 16);
    hipLaunchKernelGGL((k_conv_fwd_mx<CIN, CP, COUT>), dim3(mx_blocks(ntiles, 32, 2048)), dim3(256), 0, st, in, W, b,
                       pre, post, G, d, relu, ntiles);
    BF_HIP(hipGetLastError());
    return 0;
}

int layer_fwd(bemfft_net *n, int l, const float *in, hipStream_t st) {
    const float *W = n->p + n->woff[l], *b = n->p + n->boff[l];
    float *pre = n->pre + (int64_t)l * n->width * n->V;
    float *post = n->post + (int64_t)l * n->width * n->V;
    const int relu = l < n->nl - 1;
    const int ci = n->ci[l], co = n->co[l];
    if (ci == 6 && co == 16) return conv_fwd<6, 8, 16>(in, W, b, pre, post, n->G, n->dil[l], relu, st);
    if (ci == 16 && co == 16) return conv_fwd<16, 16, 16>(in, W, b, pre, post, n->G, n->dil[l], relu, st);
    if (ci == 16 && co == 1) return conv_fwd<16, 16, 1>(in, W, b, pre, post, n->G, n->dil[l], relu, st);
    set_error("network: unsupported layer shape");
    return BEMFFT_EUNSUPPORTED;
}

// x: planar [6][V]; converted to the channel-last n->xcl first
int forward(bemfft_net *n, const float *x, hipStream_t st) {
    hipLaunchKernelGGL(k_to_cl8, dim3((unsigned)((n->V + 255) / 256)), dim3(256), 0, st, x, n->V, n->xcl);
    const float *in = n->xcl;
    for (int l = 0; l < n->nl; ++l) {
        BF_CHECK(layer_fwd(n, l, in, st));
        in = n->post + (int64_t)l * n->width * n->V;
    }
    n->y = n->post + (int64_t)(n->nl - 1) * n->width * n->V;
    return 0;
}

template <int CIN, int CP, int COUT>
int bwd_w(const float *g, const float *in, float *part, int G, int d, float *gW, float *gb, hipStream_t st) {
    const int64_t V = (int64_t)G * G * G;
    const int nslabs = (int)((V + kSlab - 1) / kSlab);
    const int nch = mx_blocks(nslabs, 2, kWgBlocks);
    hipLaunchKernelGGL((k_conv_bwd_w_mx<CIN, CP, COUT>), dim3(nch, 3), dim3(256), 0, st, g, in, part, G, d, nslabs);
    const int tot = COUT * CIN * 27 + COUT;
    hipLaunchKernelGGL(k_conv_w_reduce, dim3((tot + 31) / 32), dim3(256), 0, st, part, nch, CIN, COUT, gW, gb);
    BF_HIP(hipGetLastError());
    return 0;
}

template <int COUT>
int bwd_d(const float *g, const float *W, const float *prev_pre, float *gin, int G, int d, hipStream_t st) {
    const int64_t V = (int64_t)G * G * G;
    const int ntiles = (int)((V + 15) / 16);
    hipLaunchKernelGGL((k_conv_bwd_data_mx<COUT>), dim3(mx_blocks(ntiles, 32, 2048)), dim3(256), 0, st, g, W, prev_pre,
                       gin, G, d, ntiles);
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
        const float *in = l == 0 ? n->xcl : n->post + (int64_t)(l - 1) * n->width * n->V;
        float *gW = n->g + n->woff[l], *gb = n->g + n->boff[l];
        const int ci = n->ci[l], co = n->co[l], d = n->dil[l];
        int s;
        if (ci == 6 && co == 16) s = bwd_w<6, 8, 16>(gcur, in, n->part, n->G, d, gW, gb, st);
        else if (ci == 16 && co == 16) s = bwd_w<16, 16, 16>(gcur, in, n->part, n->G, d, gW, gb, st);
        else s = bwd_w<16, 16, 1>(gcur, in, n->part, n->G, d, gW, gb, st);
        BF_CHECK(s);
        if (l > 0) {
            const float *W = n->p + n->woff[l];
            const float *prev_pre = n->pre + (int64_t)(l - 1) * n->width * n->V;
            if (co == 16) s = bwd_d<16>(gcur, W, prev_pre, gnext, n->G, d, st);
            else s = bwd_d<1>(gcur, W, prev_pre, gnext, n->G, d, st);
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
    const int nch = kWgBlocks;
    const size_t act = (size_t)nlayers * width * n->V * sizeof(float);
    if (hipMalloc(&n->p, n->nparam * 4) != hipSuccess || hipMalloc(&n->g, n->nparam * 4) != hipSuccess ||
        hipMalloc(&n->m, n->nparam * 4) != hipSuccess || hipMalloc(&n->v, n->nparam * 4) != hipSuccess ||
        hipMalloc(&n->pre, act) != hipSuccess || hipMalloc(&n->post, act) != hipSuccess ||
        hipMalloc(&n->xcl, (size_t)8 * n->V * 4) != hipSuccess ||
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
    for (float *q : {n->p, n->g, n->m, n->v, n->xcl, n->pre, n->post, n->ga, n->gb, n->part, n->red})
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
