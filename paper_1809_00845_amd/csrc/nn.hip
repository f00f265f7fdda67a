// nn.hip -- a small convolutional network that proposes the initial guess
// of the iterative solve (the unknown flux q of a Dirichlet problem, Sec. 4),
// with its own forward, backward and optimiser kernels.
//
// Input: voxel channels on the plan's grid, nonzero only at boundary nodes:
// a = w/h^2, a n_x, a n_y, a n_z, a s u and a s b, with s = 1/rms(u) over
// the Dirichlet nodes and b the right-hand side of the solve (minus the
// operator applied to the known values, one application of eq. 16).  Layers: 3x3x3 convolutions with dilations d_l (zero
// padding), ReLU between layers, one output channel read back at the node
// voxels as s h q.  Storage and arithmetic are FP32.  Training minimises the
// weighted squared error sum_j w_j (y(v_j) - s q_j)^2 / sum_j w_j against
// solved problems (targets s h q_j), with Adam.  The solve keeps the guess only when its
// residual is smaller than ||b|| (plain GMRES from zero otherwise).
#include <hip/hip_runtime.h>

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
};

namespace bemfft {
namespace {

constexpr int kChunk = 8192;  // voxels per weight-gradient block

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
                           int G, double inv_h2, double s, float *x, int64_t V) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
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
__global__ void k_nn_loss(const float *y, const int *vox, const float *tgt, const float *wt, int64_t nt, float *gy,
                          float *red) {
    __shared__ float sm[4];
    const int64_t i = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < nt) {
        const float e = y[vox[i]] - tgt[i];
        l = wt[i] * e * e;
        atomicAdd(&gy[vox[i]], 2.f * wt[i] * e);
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
                            const uint8_t *bc, int64_t m, int G, double inv_s, double *x0) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int j = perm[k];
    const int64_t v = ((int64_t)gz[k] * G + gy[k]) * G + gx[k];
    x0[j] = (bc == nullptr || bc[j] == 0) ? (double)y[v] * inv_s : 0.0;
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
    hipLaunchKernelGGL(k_nn_loss, dim3(nb), dim3(256), 0, st, n->y, vox, tgt, wt, nt, gcur, n->red);
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

double rms_known(const bemfft_plan *p, const double *known, const uint8_t *bc, hipStream_t st, int *status) {
    const int64_t m = p->m;
    std::vector<double> hk(m);
    std::vector<uint8_t> hb(m, 0);
    if (hipMemcpyAsync(hk.data(), known, m * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        (bc && hipMemcpyAsync(hb.data(), bc, m, hipMemcpyDeviceToHost, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess) {
        *status = BEMFFT_EDEVICE;
        return 0.0;
    }
    double s = 0.0;
    int64_t c = 0;
    for (int64_t j = 0; j < m; ++j)
        if (hb[j] == 0) {
            s += hk[j] * hk[j];
            ++c;
        }
    return c ? std::sqrt(s / c) : 0.0;
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
    for (double *q : {n->dq, n->du, n->db})
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
    if (p->dim != 3 || p->kernel != BEMFFT_LAPLACE3D || p->n[0] != n->G || p->n[1] != n->G || p->n[2] != n->G) {
        set_error("net_input: needs a Laplace 3D plan on the network's grid");
        return BEMFFT_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
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
                       known, n->db, bc, p->m, n->G, 1.0 / (p->h * p->h), scale, x, n->V);
    BF_HIP(hipGetLastError());
    return 0;
}

int bemfft_net_forward(bemfft_net *n, const float *x, float *y, void *stream) {
    if (!n || !x || !y) return BEMFFT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    BF_CHECK(forward(n, x, st));
    BF_HIP(hipMemcpyAsync(y, n->y, n->V * 4, hipMemcpyDeviceToDevice, st));
    return 0;
}

int bemfft_net_gradients(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt, const float *wt,
                         double *loss, float *grad_host, void *stream) {
    if (!n || !x || nt < 1 || !vox || !tgt || !wt) return BEMFFT_EINVAL;
    BF_CHECK(gradients(n, x, nt, vox, tgt, wt, loss, (hipStream_t)stream));
    if (grad_host) BF_HIP(hipMemcpy(grad_host, n->g, n->nparam * 4, hipMemcpyDeviceToHost));
    return 0;
}

int bemfft_net_train_step(bemfft_net *n, const float *x, int64_t nt, const int *vox, const float *tgt, const float *wt,
                          float lr, double *loss, void *stream) {
    if (!n || !x || nt < 1 || !vox || !tgt || !wt || !(lr > 0.f)) return BEMFFT_EINVAL;
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
    int status = 0;
    const double rms = rms_known(p, known, bc, st, &status);
    BF_CHECK(status);
    const double s = rms > 0.0 ? 1.0 / rms : 1.0;
    BF_CHECK(bemfft_net_input(n, p, bc, known, s, xbuf, stream));
    BF_CHECK(forward(n, xbuf, st));
    hipLaunchKernelGGL(k_nn_gather, dim3((unsigned)((p->m + 255) / 256)), dim3(256), 0, st, n->y, p->d_gx, p->d_gy,
                       p->d_gz, p->d_perm, bc, p->m, n->G, 1.0 / (s * p->h), x0);
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
