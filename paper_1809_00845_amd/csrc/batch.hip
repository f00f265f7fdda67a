// batch.hip -- many boundaries and right-hand sides in one launch sequence.
//
// A batch holds members (plan, right-hand side).  Plans with the same kernel
// family, working precision, padded sizes and z schedule form a group; every
// stage of the apply is one launch per group with the member in blockIdx.z.
// Spectra, tables and node data are the plans' own (shared by the right-hand
// sides of a plan); each member has its own intermediate buffers.  The base
// pointers of q, u, r and the mask of members still iterating live in device
// memory, so the whole launch sequence is captured once into a HIP graph and
// replayed for every batched apply.  The batched solve runs restarted GMRES
// for all members in lockstep (one batched apply per iteration, per-member
// Arnoldi reductions, one host round trip per iteration for all members).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "apply_impl.hpp"
#include "internal.hpp"

namespace bemfft {
namespace {

constexpr int kBpm = 64;       // reduction blocks per member
constexpr int kHs = 1024;      // per-member slots of the Hessenberg column buffer

struct Group {
    int kernel, precision;
    GroupDims dims;
    std::vector<int> members;
    ApplyArgs *d_args = nullptr;
};

}  // namespace
}  // namespace bemfft

struct bemfft_batch {
    int nplans = 0, nrhs = 0, kernel = 0, precision = 0, ncomp = 1;
    std::vector<bemfft_plan *> plans;
    std::vector<int> mem_plan;        // member -> plan index
    std::vector<int64_t> mem_off;     // member -> offset of its [ncomp][m] block
    std::vector<int64_t> mem_len;     // member -> ncomp * m
    int64_t total = 0;
    std::vector<bemfft::Group> groups;
    std::vector<bemfft::Engine> ws;   // member intermediates
    bemfft::BatchIO *d_io = nullptr;
    int *d_active = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // solve workspace
    int s_cap = 0;
    double *s_V = nullptr, *s_vec = nullptr, *s_red = nullptr, *s_hb = nullptr, *s_hc = nullptr;
    double *h_hc = nullptr;           // pinned copy of the compact Hessenberg columns
    int64_t *d_off = nullptr, *d_len = nullptr, *d_voff = nullptr;
    int *d_kc = nullptr;              // basis columns used by each member's update
    int *h_active = nullptr;          // pinned
};

namespace bemfft {
namespace {

void bfree(void *p) {
    if (p) (void)hipFree(p);
}

int launch_groups(bemfft_batch *b, hipStream_t st) {
    for (auto &g : b->groups) {
        int s;
        if (g.kernel == 0) s = apply_batch_kind<0>(g.precision, g.d_args, b->d_io, g.dims, st);
        else if (g.kernel == 1) s = apply_batch_kind<1>(g.precision, g.d_args, b->d_io, g.dims, st);
        else if (g.kernel == 3) s = apply_batch_kind<3>(g.precision, g.d_args, b->d_io, g.dims, st);
        else s = apply_batch_kind<2>(g.precision, g.d_args, b->d_io, g.dims, st);
        BF_CHECK(s);
    }
    return 0;
}

// The pointers travel as kernel arguments (copied at launch), so successive
// calls on a stream never race on a staging buffer.
__global__ void k_set_io(BatchIO *io, const double *q, const double *u, double *r, const int *active) {
    io->q = q;
    io->u = u;
    io->r = r;
    io->active = active;
}

// one batched apply of every active member: q, u -> r (concatenated layout)
int batch_apply_impl(bemfft_batch *b, const double *q, const double *u, double *r, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(k_set_io, dim3(1), dim3(1), 0, st, b->d_io, q, u, r, active);
    BF_HIP(hipGetLastError());
    if (b->exec) {
        BF_HIP(hipGraphLaunch(b->exec, st));
        return 0;
    }
    return launch_groups(b, st);
}

// ------------------------------------------------------------------ solve kernels
// Member k owns rows [off[k], off[k] + len[k]) of every concatenated vector
// and the basis V_k = V + voff[k] (vector j at V_k + j len[k]).

__global__ void kbs_split(const uint8_t *bc, const double *x, const double *scale, double *q, double *u, int64_t n,
                          int unknown_side) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i] * (scale ? scale[i] : 1.0);
        const bool qslot = (bc[i] == 0) == (unknown_side != 0);
        q[i] = qslot ? v : 0.0;
        u[i] = qslot ? 0.0 : v;
    }
}

__global__ void kbs_axpby(double *y, const double *x, double a, double bb, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + bb * y[i];
}

// partial[k][blk][j] = sum over the block's rows of V_k[j][i] w[off_k + i]
__global__ __launch_bounds__(256) void kbs_mdot_partial(const double *V, const int64_t *voff, const int64_t *off,
                                                        const int64_t *len, int nvec, const double *w,
                                                        double *partial, const int *active, int self) {
    constexpr int G = 8;
    __shared__ double sm[4][G];
    const int k = blockIdx.y;
    if (!active[k]) return;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t n = len[k];
    const double *Vk = self ? (w + off[k]) : (V + voff[k]);  // self: dot of w with itself
    const double *wk = w + off[k];
    for (int j0 = 0; j0 < nvec; j0 += G) {
        double acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q) acc[q] = 0.0;
        for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
            const double wi = wk[i];
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (j0 + q < nvec) acc[q] += Vk[(int64_t)(j0 + q) * n + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < G; ++q) sm[wave][q] = acc[q];
        __syncthreads();
        if (threadIdx.x < G && j0 + threadIdx.x < nvec)
            partial[((int64_t)k * gridDim.x + blockIdx.x) * nvec + j0 + threadIdx.x] =
                (sm[0][threadIdx.x] + sm[1][threadIdx.x]) + (sm[2][threadIdx.x] + sm[3][threadIdx.x]);
        __syncthreads();
    }
}

// hb[k * kHs + base + j] = sum_blk partial[k][blk][j] (sqrt if sqrt_out)
// hb[k][base + j] = sum over blocks of partial[k][b][j]: one wavefront per
// (member, j), fixed-order lane sums and shuffle tree (deterministic)
__global__ __launch_bounds__(64) void kbs_mdot_final(const double *partial, int nblk, int nvec, double *hb, int base,
                                                     int sqrt_out, const int *active) {
    const int k = blockIdx.x, j = blockIdx.y;
    if (!active[k]) return;
    double s = 0.0;
    for (int bl = threadIdx.x; bl < nblk; bl += 64) s += partial[((int64_t)k * nblk + bl) * nvec + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) hb[(int64_t)k * kHs + base + j] = sqrt_out ? sqrt(s) : s;
}

// w_k += sign * V_k h_k, h_k = hb[k * kHs + base ...]
// kcount (optional): member k uses only its first kcount[k] <= nvec columns
// (a member that stopped early has no coefficients, and possibly never-written
// basis columns, beyond them).
__global__ void kbs_gemv(const double *V, const int64_t *voff, const int64_t *off, const int64_t *len, int nvec,
                         const double *hb, int base, double *w, double sign, const int *active, const int *kcount) {
    const int k = blockIdx.y;
    if (!active[k]) return;
    if (kcount) nvec = min(nvec, kcount[k]);
    const int64_t n = len[k];
    const double *Vk = V + voff[k];
    const double *h = hb + (int64_t)k * kHs + base;
    double *wk = w + off[k];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += Vk[(int64_t)(j + q) * n + i] * h[j + q];
        }
        for (int q = 0; j + q < nvec; ++q) acc[q] += Vk[(int64_t)(j + q) * n + i] * h[j + q];
        wk[i] += sign * (((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
    }
}

// V_k[col] = w_k / hb[k * kHs + idx]
__global__ void kbs_normalize(const double *w, const double *hb, int idx, double *V, const int64_t *voff,
                              const int64_t *off, const int64_t *len, int col, const int *active) {
    const int k = blockIdx.y;
    if (!active[k]) return;
    const int64_t n = len[k];
    const double a = hb[(int64_t)k * kHs + idx];
    const double inv = a > 0.0 ? 1.0 / a : 0.0;
    double *v = V + voff[k] + (int64_t)col * n;
    const double *wk = w + off[k];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = wk[i] * inv;
}

// hc[k * stride + i] = h1 + h2 (i <= it), the new norm at i = it + 1
__global__ void kbs_combine(const double *hb, int it, double *hc, int stride, const int *active) {
    const int k = blockIdx.x;
    for (int i = threadIdx.x; i <= it + 1; i += blockDim.x) {
        double v = 0.0;
        if (active[k]) v = (i <= it) ? hb[(int64_t)k * kHs + i] + hb[(int64_t)k * kHs + 512 + i]
                                     : hb[(int64_t)k * kHs + 512 + it + 1];
        hc[(int64_t)k * stride + i] = v;
    }
}

// out[off_k + i] = V_k[col][i]: column col of every active member's basis
// gathered into the concatenated layout
__global__ void kbs_column(const double *V, const int64_t *voff, const int64_t *off, const int64_t *len, int col,
                           double *out, const int *active) {
    const int k = blockIdx.y;
    if (!active[k]) return;
    const int64_t n = len[k];
    const double *v = V + voff[k] + (int64_t)col * n;
    double *o = out + off[k];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = v[i];
}

// x += d .* r
__global__ void kbs_axpy_scaled(double *x, const double *d, const double *r, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += d[i] * r[i];
}

int gridn(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 2048); }

int ensure_solve_ws(bemfft_batch *b, int restart) {
    const int nm = (int)b->mem_plan.size();
    if (b->s_cap < restart + 1) {
        bfree(b->s_V);
        b->s_V = nullptr;
        if (hipMalloc(&b->s_V, (size_t)(restart + 1) * b->total * sizeof(double)) != hipSuccess) {
            b->s_cap = 0;
            set_error("batched GMRES basis allocation failed");
            return BEMFFT_ENOMEM;
        }
        // columns a member never reaches stay finite (zero) whatever the memory held
        BF_HIP(hipMemset(b->s_V, 0, (size_t)(restart + 1) * b->total * sizeof(double)));
        b->s_cap = restart + 1;
        std::vector<int64_t> voff(nm);
        for (int k = 0; k < nm; ++k) voff[k] = (int64_t)(restart + 1) * b->mem_off[k];
        bfree(b->d_voff);
        b->d_voff = nullptr;
        BF_HIP(hipMalloc(&b->d_voff, nm * sizeof(int64_t)));
        BF_HIP(hipMemcpy(b->d_voff, voff.data(), nm * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    if (!b->s_vec) {
        if (hipMalloc(&b->s_vec, 9 * (size_t)b->total * sizeof(double)) != hipSuccess ||
            hipMalloc(&b->s_red, (size_t)nm * kBpm * 512 * sizeof(double)) != hipSuccess ||
            hipMalloc(&b->s_hb, (size_t)nm * kHs * sizeof(double)) != hipSuccess ||
            hipMalloc(&b->s_hc, (size_t)nm * 512 * sizeof(double)) != hipSuccess ||
            hipMalloc(&b->d_kc, (size_t)nm * sizeof(int)) != hipSuccess ||
            hipHostMalloc(&b->h_hc, (size_t)nm * 512 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            set_error("batched GMRES workspace allocation failed");
            return BEMFFT_ENOMEM;
        }
    }
    return 0;
}

}  // namespace
}  // namespace bemfft

using namespace bemfft;

extern "C" {

int bemfft_batch_destroy(bemfft_batch *b) {
    if (!b) return 0;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto &g : b->groups) bfree(g.d_args);
    for (auto &e : b->ws) free_engine(&e);
    bfree(b->d_io);
    bfree(b->d_active);
    bfree(b->s_V);
    bfree(b->s_vec);
    bfree(b->s_red);
    bfree(b->s_hb);
    bfree(b->s_hc);
    if (b->h_hc) (void)hipHostFree(b->h_hc);
    if (b->h_active) (void)hipHostFree(b->h_active);
    bfree(b->d_off);
    bfree(b->d_len);
    bfree(b->d_voff);
    bfree(b->d_kc);
    delete b;
    return 0;
}

int bemfft_batch_create(bemfft_batch **out, bemfft_plan *const *plans, int nplans, int nrhs, int use_graph,
                        void *stream) {
    if (!out || !plans || nplans < 1 || nrhs < 1) {
        set_error("batch_create: bad argument");
        return BEMFFT_EINVAL;
    }
    *out = nullptr;
    for (int i = 0; i < nplans; ++i) {
        if (!plans[i]) {
            set_error("batch_create: null plan");
            return BEMFFT_EINVAL;
        }
        if (plans[i]->eng.precision == BEMFFT_BF16_MFMA) {
            set_error("batch_create: batches of 16-bit plans are not supported");
            return BEMFFT_EINVAL;
        }
        if (plans[i]->kernel != plans[0]->kernel || plans[i]->eng.precision != plans[0]->eng.precision) {
            set_error("batch_create: plans must share the kernel family and the working precision");
            return BEMFFT_EINVAL;
        }
    }
    bemfft_batch *b = new (std::nothrow) bemfft_batch();
    if (!b) {
        set_error("host allocation failed");
        return BEMFFT_ENOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    b->nplans = nplans;
    b->nrhs = nrhs;
    b->kernel = plans[0]->kernel;
    b->precision = plans[0]->eng.precision;
    b->ncomp = plans[0]->ncomp;
    b->plans.assign(plans, plans + nplans);
    int status = 0;
    // members in plan order, right-hand sides of a plan adjacent
    for (int i = 0; i < nplans; ++i)
        for (int j = 0; j < nrhs; ++j) {
            b->mem_plan.push_back(i);
            b->mem_off.push_back(b->total);
            b->mem_len.push_back((int64_t)plans[i]->ncomp * plans[i]->m);
            b->total += (int64_t)plans[i]->ncomp * plans[i]->m;
        }
    const int nm = (int)b->mem_plan.size();
    b->ws.resize(nm);
    for (int k = 0; k < nm && status == 0; ++k)
        status = alloc_intermediates(plans[b->mem_plan[k]], b->precision, &b->ws[k]);
    // groups
    std::map<std::tuple<int64_t, int64_t, int64_t, int>, int> gidx;
    for (int k = 0; k < nm && status == 0; ++k) {
        bemfft_plan *p = plans[b->mem_plan[k]];
        auto key = std::make_tuple(p->P[0], p->P[1], p->P[2], p->zsched);
        auto it = gidx.find(key);
        if (it == gidx.end()) {
            Group g;
            g.kernel = b->kernel;
            g.precision = b->precision;
            g.dims = GroupDims{0, 0, 0, 0, (int)p->H[0], (int)p->P[0], (int)p->P[1], (int)p->P[2], p->zsched, 0};
            gidx[key] = (int)b->groups.size();
            b->groups.push_back(g);
            it = gidx.find(key);
        }
        Group &g = b->groups[it->second];
        g.members.push_back(k);
        g.dims.nmem += 1;
        g.dims.max_m = std::max<int>(g.dims.max_m, (int)p->m);
        g.dims.max_nd = std::max<int>(g.dims.max_nd, (int)p->nd);
        g.dims.max_nzo = std::max<int>(g.dims.max_nzo, (int)p->nzo);
        g.dims.row_inv = std::max(g.dims.row_inv, p->row_inv);
    }
    for (auto &g : b->groups) {
        if (status) break;
        std::vector<ApplyArgs> args(g.members.size());
        for (size_t i = 0; i < g.members.size(); ++i) {
            const int k = g.members[i];
            bemfft_plan *p = plans[b->mem_plan[k]];
            fill_apply_args(p, p->eng, b->ws[k], &args[i]);
            args[i].off = b->mem_off[k];
            args[i].gid = k;
        }
        if (hipMalloc(&g.d_args, args.size() * sizeof(ApplyArgs)) != hipSuccess ||
            hipMemcpy(g.d_args, args.data(), args.size() * sizeof(ApplyArgs), hipMemcpyHostToDevice) != hipSuccess) {
            status = BEMFFT_ENOMEM;
            set_error("batch_create: member table upload failed");
        }
    }
    std::vector<int64_t> off(b->mem_off), len(b->mem_len);
    if (status == 0 &&
        (hipMalloc(&b->d_io, sizeof(BatchIO)) != hipSuccess ||
         hipMalloc(&b->d_active, nm * sizeof(int)) != hipSuccess ||
         hipHostMalloc(&b->h_active, nm * sizeof(int), hipHostMallocDefault) != hipSuccess ||
         hipMalloc(&b->d_off, nm * sizeof(int64_t)) != hipSuccess || hipMalloc(&b->d_len, nm * sizeof(int64_t)) != hipSuccess ||
         hipMemcpy(b->d_off, off.data(), nm * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(b->d_len, len.data(), nm * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)) {
        status = BEMFFT_ENOMEM;
        set_error("batch_create: allocation failed");
    }
    // capture the launch sequence once (the inputs are read through d_io)
    if (status == 0 && use_graph) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            status = BEMFFT_EDEVICE;
        } else {
            if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) status = BEMFFT_EDEVICE;
            if (status == 0) {
                int ls = launch_groups(b, cs);
                hipGraph_t g = nullptr;
                hipError_t ee = hipStreamEndCapture(cs, &g);
                if (ls || ee != hipSuccess) {
                    status = ls ? ls : BEMFFT_EDEVICE;
                    if (g) (void)hipGraphDestroy(g);
                } else {
                    b->graph = g;
                    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) status = BEMFFT_EDEVICE;
                }
            }
            (void)hipStreamDestroy(cs);
        }
        if (status == BEMFFT_EDEVICE) set_error("batch_create: graph capture failed");
    }
    (void)st;
    if (status) {
        bemfft_batch_destroy(b);
        return status;
    }
    *out = b;
    return 0;
}

int bemfft_batch_apply(bemfft_batch *b, const double *q, const double *u, double *r, void *stream) {
    if (!b || !q || !u || !r) {
        set_error("batch_apply: null argument");
        return BEMFFT_EINVAL;
    }
    return batch_apply_impl(b, q, u, r, nullptr, (hipStream_t)stream);
}

int bemfft_batch_solve(bemfft_batch *b, const uint8_t *bc, const double *known, double *unknown,
                       const bemfft_solve_opts *opts, bemfft_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!b || !bc || !known || !unknown) {
        set_error("batch_solve: null argument");
        return BEMFFT_EINVAL;
    }
    bemfft_solve_opts o{1e-6, 100, 1000, 1, 0, 0, 1e-4, 20};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.restart < 1 || o.restart > 400 || o.maxit < 1 || o.refine || o.use_x0 < 0 ||
        o.use_x0 > 1 || o.precond < 0 || o.precond > 1) {
        set_error("batch_solve: bad options (refine, use_x0 = 2 and block Jacobi are not supported for batches)");
        return BEMFFT_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    BF_CHECK(ensure_solve_ws(b, o.restart));
    const int nm = (int)b->mem_plan.size();
    const int64_t n = b->total;
    double *bv = b->s_vec, *x = bv + n, *w = x + n, *q = w + n, *u = q + n, *r = u + n, *dinv = r + n;
    double *V = b->s_V;
    const int mcap = o.restart;
    int *act = b->h_active;
    // b = -apply(known)
    hipLaunchKernelGGL(kbs_split, dim3(gridn(n)), dim3(256), 0, st, bc, known, (const double *)nullptr, q, u, n, 0);
    BF_HIP(hipGetLastError());
    BF_CHECK(batch_apply_impl(b, q, u, bv, nullptr, st));
    hipLaunchKernelGGL(kbs_axpby, dim3(gridn(n)), dim3(256), 0, st, bv, bv, -1.0, 0.0, n);
    // Jacobi scaling from the plans' diagonal entries, chosen per slot on the host
    {
        std::vector<uint8_t> hbc(n);
        std::vector<double> hd(n);
        BF_HIP(hipMemcpyAsync(hbc.data(), bc, n, hipMemcpyDeviceToHost, st));
        BF_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < nm; ++k) {
            const bemfft_plan *p = b->plans[b->mem_plan[k]];
            for (int64_t i = 0; i < b->mem_len[k]; ++i) {
                const int64_t gi = b->mem_off[k] + i;
                const double d = hbc[gi] == 0 ? p->h_diag_dir[i] : p->h_diag_neu[i];
                hd[gi] = (o.precond && d != 0.0 && std::isfinite(d)) ? 1.0 / d : 1.0;
            }
        }
        BF_HIP(hipMemcpyAsync(dinv, hd.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    }
    if (o.use_x0) BF_HIP(hipMemcpyAsync(x, unknown, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else BF_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
    // per-member 2-norms of a concatenated vector (one host round trip)
    const dim3 gm(gridn(n / nm + 1), nm);
    auto norms = [&](const double *vec, std::vector<double> &outn) -> int {
        hipLaunchKernelGGL(kbs_mdot_partial, dim3(kBpm, nm), dim3(256), 0, st, V, b->d_voff, b->d_off, b->d_len, 1,
                           vec, b->s_red, b->d_active, 1);
        hipLaunchKernelGGL(kbs_mdot_final, dim3(nm, 1), dim3(64), 0, st, b->s_red, kBpm, 1, b->s_hb, 512, 1, b->d_active);
        hipLaunchKernelGGL(kbs_combine, dim3(nm), dim3(64), 0, st, b->s_hb, -1, b->s_hc, 512, b->d_active);
        BF_HIP(hipGetLastError());
        BF_HIP(hipMemcpy2DAsync(b->h_hc, sizeof(double), b->s_hc, 512 * sizeof(double), sizeof(double), nm,
                                hipMemcpyDeviceToHost, st));
        BF_HIP(hipStreamSynchronize(st));
        outn.resize(nm);
        for (int k = 0; k < nm; ++k) outn[k] = b->h_hc[(size_t)k];
        return 0;
    };
    // the mask is read by kernels queued later; the host rewrites 'act'
    // soon after, so each upload completes before returning
    auto upload_active = [&]() -> int {
        BF_HIP(hipMemcpyAsync(b->d_active, act, nm * sizeof(int), hipMemcpyHostToDevice, st));
        BF_HIP(hipStreamSynchronize(st));
        return 0;
    };
    for (int k = 0; k < nm; ++k) act[k] = 1;
    BF_CHECK(upload_active());
    std::vector<double> bnorm(nm), beta(nm), rel(nm, 0.0);
    std::vector<int> iters(nm, 0), cycles(nm, 0), conv(nm, 0), status_m(nm, 0);
    BF_CHECK(norms(bv, bnorm));
    int status = 0;
    std::vector<double> H((size_t)nm * (mcap + 1) * mcap), cs((size_t)nm * mcap), sn((size_t)nm * mcap),
        g((size_t)nm * (mcap + 1));
    bool x_zero = !o.use_x0;
    for (int k = 0; k < nm; ++k) {
        if (!std::isfinite(bnorm[k])) {  // non-finite data: breakdown, not "zero data"
            status_m[k] = BEMFFT_EBREAKDOWN;
            conv[k] = 1;
        } else if (!(bnorm[k] > 0.0)) {
            conv[k] = 1;  // zero data: x = 0
        }
    }
    for (;;) {
        // true residuals of the members not yet converged
        for (int k = 0; k < nm; ++k) act[k] = conv[k] ? 0 : 1;
        BF_CHECK(upload_active());
        if (x_zero) {
            BF_HIP(hipMemcpyAsync(w, bv, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        } else {
            hipLaunchKernelGGL(kbs_split, dim3(gridn(n)), dim3(256), 0, st, bc, x, (const double *)nullptr, q, u, n, 1);
            BF_CHECK(batch_apply_impl(b, q, u, w, b->d_active, st));
            hipLaunchKernelGGL(kbs_axpby, dim3(gridn(n)), dim3(256), 0, st, w, bv, 1.0, -1.0, n);
        }
        BF_CHECK(norms(w, beta));
        bool any = false;
        for (int k = 0; k < nm; ++k) {
            if (!act[k]) continue;
            rel[k] = beta[k] / bnorm[k];
            if (!std::isfinite(beta[k])) {
                status_m[k] = BEMFFT_EBREAKDOWN;
                conv[k] = 1;
            } else if (rel[k] <= o.tol) {
                conv[k] = 1;
            } else if (iters[k] >= o.maxit) {
                status_m[k] = BEMFFT_ENOCONV;
                conv[k] = 1;
            }
            act[k] = conv[k] ? 0 : 1;
            any = any || act[k];
        }
        if (!any) break;
        BF_CHECK(upload_active());
        // v_0 = r / beta (the norm sits at hb[k][512])
        hipLaunchKernelGGL(kbs_normalize, gm, dim3(256), 0, st, w, b->s_hb, 512, V, b->d_voff, b->d_off, b->d_len, 0,
                           b->d_active);
        std::vector<int> kk(nm, 0);
        for (int k = 0; k < nm; ++k) {
            std::fill(g.begin() + (size_t)k * (mcap + 1), g.begin() + (size_t)(k + 1) * (mcap + 1), 0.0);
            g[(size_t)k * (mcap + 1)] = beta[k];
        }
        std::vector<int> inner(act, act + nm);  // members still in this Arnoldi cycle
        for (int it = 0; it < mcap; ++it) {
            bool anyin = false;
            for (int k = 0; k < nm; ++k) anyin = anyin || inner[k];
            if (!anyin) break;
            for (int k = 0; k < nm; ++k) act[k] = inner[k];
            BF_CHECK(upload_active());
            // w = A Dinv v_it for the members still iterating
            hipLaunchKernelGGL(kbs_column, gm, dim3(256), 0, st, V, b->d_voff, b->d_off, b->d_len, it, r, b->d_active);
            hipLaunchKernelGGL(kbs_split, dim3(gridn(n)), dim3(256), 0, st, bc, r, dinv, q, u, n, 1);
            BF_HIP(hipGetLastError());
            BF_CHECK(batch_apply_impl(b, q, u, w, b->d_active, st));
            // classical Gram-Schmidt twice, then the new norm
            for (int pass = 0; pass < 2; ++pass) {
                const int base = pass * 512;
                hipLaunchKernelGGL(kbs_mdot_partial, dim3(kBpm, nm), dim3(256), 0, st, V, b->d_voff, b->d_off, b->d_len,
                                   it + 1, w, b->s_red, b->d_active, 0);
                hipLaunchKernelGGL(kbs_mdot_final, dim3(nm, it + 1), dim3(64), 0, st, b->s_red, kBpm, it + 1, b->s_hb, base, 0,
                                   b->d_active);
                hipLaunchKernelGGL(kbs_gemv, gm, dim3(256), 0, st, V, b->d_voff, b->d_off, b->d_len, it + 1, b->s_hb,
                                   base, w, -1.0, b->d_active, (const int *)nullptr);
            }
            hipLaunchKernelGGL(kbs_mdot_partial, dim3(kBpm, nm), dim3(256), 0, st, V, b->d_voff, b->d_off, b->d_len, 1,
                               w, b->s_red, b->d_active, 1);
            hipLaunchKernelGGL(kbs_mdot_final, dim3(nm, 1), dim3(64), 0, st, b->s_red, kBpm, 1, b->s_hb, 512 + it + 1, 1,
                               b->d_active);
            hipLaunchKernelGGL(kbs_normalize, gm, dim3(256), 0, st, w, b->s_hb, 512 + it + 1, V, b->d_voff, b->d_off,
                               b->d_len, it + 1, b->d_active);
            hipLaunchKernelGGL(kbs_combine, dim3(nm), dim3(64), 0, st, b->s_hb, it, b->s_hc, 512, b->d_active);
            BF_HIP(hipGetLastError());
            BF_HIP(hipMemcpy2DAsync(b->h_hc, (it + 2) * sizeof(double), b->s_hc, 512 * sizeof(double),
                                    (it + 2) * sizeof(double), nm, hipMemcpyDeviceToHost, st));
            BF_HIP(hipStreamSynchronize(st));
            for (int k = 0; k < nm; ++k) {
                if (!inner[k]) continue;
                ++iters[k];
                double *col = &H[((size_t)k * mcap + it) * (mcap + 1)];
                const double *hc = b->h_hc + (size_t)k * (it + 2);
                bool bad = false;
                for (int i = 0; i <= it + 1; ++i) {
                    col[i] = hc[i];
                    if (!std::isfinite(col[i])) bad = true;
                }
                if (bad) {
                    status_m[k] = BEMFFT_EBREAKDOWN;
                    conv[k] = 1;
                    inner[k] = 0;
                    kk[k] = 0;
                    continue;
                }
                double *csk = &cs[(size_t)k * mcap], *snk = &sn[(size_t)k * mcap], *gk = &g[(size_t)k * (mcap + 1)];
                for (int i = 0; i < it; ++i) {
                    const double t = csk[i] * col[i] + snk[i] * col[i + 1];
                    col[i + 1] = -snk[i] * col[i] + csk[i] * col[i + 1];
                    col[i] = t;
                }
                const double a = col[it], bb = col[it + 1];
                const double rr = std::hypot(a, bb);
                csk[it] = rr > 0.0 ? a / rr : 1.0;
                snk[it] = rr > 0.0 ? bb / rr : 0.0;
                const double hnext = hc[it + 1];
                col[it] = rr;
                col[it + 1] = 0.0;
                gk[it + 1] = -snk[it] * gk[it];
                gk[it] = csk[it] * gk[it];
                kk[k] = it + 1;
                if (std::fabs(gk[it + 1]) / bnorm[k] <= o.tol || hnext == 0.0 || iters[k] >= o.maxit) inner[k] = 0;
            }
        }
        // x_k += Dinv V_k y_k with H_k y_k = g_k (upper triangular)
        std::vector<double> yh((size_t)nm * kHs, 0.0);
        int maxk = 0;
        for (int k = 0; k < nm; ++k) {
            const int kc = kk[k];
            const double *gk = &g[(size_t)k * (mcap + 1)];
            double *yk = &yh[(size_t)k * kHs];
            for (int i = kc - 1; i >= 0; --i) {
                double s2 = gk[i];
                for (int j = i + 1; j < kc; ++j) s2 -= H[((size_t)k * mcap + j) * (mcap + 1) + i] * yk[j];
                const double d = H[((size_t)k * mcap + i) * (mcap + 1) + i];
                yk[i] = d != 0.0 ? s2 / d : 0.0;
            }
            act[k] = kc > 0 ? 1 : 0;
            if (kc > 0) ++cycles[k];
            maxk = std::max(maxk, kc);
        }
        BF_CHECK(upload_active());
        BF_HIP(hipMemcpyAsync(b->s_hb, yh.data(), yh.size() * sizeof(double), hipMemcpyHostToDevice, st));
        BF_HIP(hipMemcpyAsync(b->d_kc, kk.data(), nm * sizeof(int), hipMemcpyHostToDevice, st));
        BF_HIP(hipMemsetAsync(r, 0, n * sizeof(double), st));
        hipLaunchKernelGGL(kbs_gemv, gm, dim3(256), 0, st, V, b->d_voff, b->d_off, b->d_len, maxk, b->s_hb, 0, r, 1.0,
                           b->d_active, (const int *)b->d_kc);
        hipLaunchKernelGGL(kbs_axpy_scaled, dim3(gridn(n)), dim3(256), 0, st, x, dinv, r, n);
        BF_HIP(hipGetLastError());
        x_zero = false;
    }
    BF_HIP(hipMemcpyAsync(unknown, x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    BF_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < nm; ++k) {
        if (status_m[k] < 0) status = status_m[k];
        else if (status_m[k] > 0 && status == 0) status = status_m[k];
        if (info) {
            info[k].iters = iters[k];
            info[k].restarts = cycles[k] > 0 ? cycles[k] - 1 : 0;
            info[k].true_relres = rel[k];
            info[k].status = status_m[k];
            info[k].seconds = secs;
            info[k].outer = 0;
            info[k].applies64 = 0;
            info[k].x0_used = o.use_x0 ? 1 : 0;
            info[k].x0_relres = -1.0;
        }
    }
    return status;
}

int bemfft_batch_members(const bemfft_batch *b, int64_t *offsets, int64_t *lengths) {
    if (!b) {
        set_error("null batch");
        return BEMFFT_EINVAL;
    }
    const int nm = (int)b->mem_plan.size();
    for (int k = 0; k < nm; ++k) {
        if (offsets) offsets[k] = b->mem_off[k];
        if (lengths) lengths[k] = b->mem_len[k];
    }
    return nm;
}

}  // extern "C"
