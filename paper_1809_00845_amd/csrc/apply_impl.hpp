// apply_impl.hpp -- the hot path: r = c u + D[u] - S[q] as the zero-padded
// FFT convolution of eq. (16), in four kernels.
//
//   k_fwd_xy   per occupied z-plane and chunk of kx: scatter of the boundary
//              fields (Fig. 4) fused with their x-transform, done as a direct
//              DFT over the few nodes of each grid row (the field is zero
//              elsewhere), then the y-FFT in LDS.   -> Y[f][kx][z][ky]
//   k_zpass    per (kx, tile of ky): forward z-FFT of every field (input zero
//              outside the occupied planes), products with the compact kernel
//              spectra summed into each output (eqs. 15-16), inverse z-FFT,
//              keep the occupied planes.              -> Z[o][kx][z][ky]
//   k_inv_y    per occupied z-plane and chunk of kx: inverse y-FFT in
//              registers/LDS, rows y < ny stored with kx contiguous
//                                                      -> W[o][z][y][kx] (in Y)
//   k_gather   eight lanes per node: the inverse x-transform of its row
//              evaluated only at its own x (Sec. 4: only the boundary
//              values are needed), plus c u and the self-term
//              correction                              -> r
//              (nodes of long rows read their row's inverse FFT, made by
//              k_rows_inv, instead)
//
// Layout: complex intermediates are interleaved (re, im) in the working
// precision R with ky contiguous, so every global access is a run of whole
// rows; kernel spectra are [c][kx][ky][kz] reals over one octant.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_device.hpp"
#include "internal.hpp"
#include "kinds.hpp"

namespace bemfft {

struct ApplyArgs {
    int nx, ny, nz;
    int px, py, pz;
    int hx, hy, hz;
    int hzs;          // stored kz row length of the spectra (hz, or padded)
    int z0, nzo;
    int m;
    int zsched;       // radix schedule of the z pass (0, 1, or 2 where a wide one exists)
    int64_t off;      // batched apply: offset of this member's q, u, r
    int gid;          // batched apply: member index in the whole batch
    const int *gx, *gy, *gz, *rowptr, *perm;
    const double *w, *nrm, *C, *SC;
    const double *q, *u;
    double *r;
    const void *spec, *twx, *twy, *twz;
    void *vf;  // [F][m] boundary fields in sorted order, working precision
    void *Xd;  // [nd][F][hx] transforms of the long rows
    const int *row_dense;   // [nzo * ny]: index into dense_rows, or -1
    const int *dense_rows;  // [nd]: row index (zz * ny + y) of each long row
    int nd;
    int row_inv;            // 1: the long rows' inverse x transform is an FFT (k_rows_inv)
    int fwd_xg;             // kx per thread in the forward direct DFT (1 or 2)
    void *Y, *Z;
};

// Launch extents of one group of batch members (same family, precision,
// padded sizes and schedule): the largest per-member extents.
struct GroupDims {
    int nmem;
    int max_m, max_nd, max_nzo;
    int hx, px, py, pz, zsched;
    int row_inv;  // some member takes the row FFT for its long rows
};

// Base pointers of a batched apply (device memory, so that a captured graph
// of the launches serves any call) and the members still iterating.
struct BatchIO {
    const double *q, *u;
    double *r;
    const int *active;  // null: all members
};

constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
constexpr int mini(int a, int b) { return a < b ? a : b; }
constexpr int kMaxPx = 1024;         // largest padded length along x (2D plans; 3D stop at 512)

// Complex value stored in 16 bits per part (the intermediates Y and Z of the
// 16-bit form); arithmetic stays FP32.
struct alignas(4) cbf16 {
    __bf16 x, y;
};
// Storage conversions: identity for cx<R>, FP32 <-> BF16 (round to nearest
// even) for cbf16.
template <typename S, typename R>
__device__ __forceinline__ S to_store(cx<R> v) {
    if constexpr (std::is_same<S, cbf16>::value) return cbf16{(__bf16)(float)v.x, (__bf16)(float)v.y};
    else return v;
}
template <typename R, typename S>
__device__ __forceinline__ cx<R> from_store(S v) {
    if constexpr (std::is_same<S, cbf16>::value) return cx<R>{(R)(float)v.x, (R)(float)v.y};
    else return v;
}

// (k x) mod p for 0 <= k x < 2^24, with a float estimate of the quotient.
__device__ __forceinline__ int mod_small(int kx, int x, int p, float inv_p) {
    const int prod = kx * x;
    int r = prod - (int)((float)prod * inv_p) * p;
    if (r < 0) r += p;
    if (r >= p) r -= p;
    return r;
}

// ------------------------------------------------------------------ k_fields
// Boundary fields of every node in sorted order (the zero-extended data of
// Fig. 4 before it is placed on the grid): Laplace q w and u n_i w;
// Navier t_j w and the symmetrised u (x) n w; half-space sigma_b w.
template <typename R, int KIND>
__device__ __forceinline__ void fields_body(const ApplyArgs &a, const int bx, const int by, const int bz) {
    const int s = bx * 256 + threadIdx.x;
    if (s >= a.m) return;
    R *vf = static_cast<R *>(a.vf);
    const int j = a.perm[s];
    const double wt = a.w[s];
    const double n[3] = {a.nrm[s], a.nrm[a.m + s], a.nrm[2 * a.m + s]};
    if constexpr (KIND == 3) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vf[c * a.m + s] = (R)(a.q[c * a.m + j] * wt);
    } else if constexpr (KIND == 0 || KIND == 1) {
        const double uw = a.u[j] * wt;
        vf[s] = (R)(a.q[j] * wt);
#pragma unroll
        for (int i = 0; i < (KIND == 0 ? 2 : 3); ++i) vf[(1 + i) * a.m + s] = (R)(uw * n[i]);
    } else {
        double uu[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vf[c * a.m + s] = (R)(a.q[c * a.m + j] * wt);
            uu[c] = a.u[c * a.m + j];
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = pair_i(p), k = pair_j(p);
            const double v = (i == k ? uu[i] * n[i] : uu[i] * n[k] + uu[k] * n[i]) * wt;
            vf[(3 + p) * a.m + s] = (R)v;
        }
    }
}

template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_fields(ApplyArgs a) {
    fields_body<R, KIND>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Batched form: blockIdx.z = member * zdiv + the kernel's own z index.
template <typename R, int KIND>
__global__ __launch_bounds__(256) void kb_fields(const ApplyArgs *members, const BatchIO *io, int zdiv) {
    ApplyArgs a = members[blockIdx.z / zdiv];
    if (io->active && !io->active[a.gid]) return;
    a.q = io->q + a.off;
    a.u = io->u + a.off;
    a.r = io->r + a.off;
    fields_body<R, KIND>(a, blockIdx.x, blockIdx.y, blockIdx.z % zdiv);
}

// All F field values of sorted node s at once (one set of loads), computed
// from q and u exactly as fields_body stores them (same operations, same
// rounding), for the long-row transforms, which do not wait for k_fields.
template <typename R, int KIND>
__device__ __forceinline__ void node_fields(const ApplyArgs &a, const int s, R *v) {
    constexpr int F = Terms<KIND>::F;
    const int j = a.perm[s];
    const double wt = a.w[s];
    if constexpr (KIND == 3) {  // half-space: the three traction components
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = (R)(a.q[c * a.m + j] * wt);
    } else if constexpr (KIND == 0 || KIND == 1) {
        v[0] = (R)(a.q[j] * wt);
        const double uw = a.u[j] * wt;
#pragma unroll
        for (int f = 1; f < F; ++f) v[f] = (R)(uw * a.nrm[(f - 1) * a.m + s]);
    } else {
        static_assert(F == 9, "Navier: three tractions and six symmetrised u n products");
        double uu[3], nn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = (R)(a.q[c * a.m + j] * wt);
            uu[c] = a.u[c * a.m + j];
            nn[c] = a.nrm[c * a.m + s];
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = pair_i(p), k = pair_j(p);
            v[3 + p] = (R)((i == k ? uu[i] * nn[i] : uu[i] * nn[k] + uu[k] * nn[i]) * wt);
        }
    }
}

// ------------------------------------------------------------------ long rows
// Long grid rows (e.g. rows of a box face lying in a grid plane) are
// x-transformed with an FFT instead of the direct sum: the row's nodes are
// placed on a zero pencil (nodes sharing a cell are summed in order) and
// transformed; kx < Hx is kept.                          -> Xd[d][f][kx]
template <typename R, int PX, int KIND>
struct RowCfg {
    static constexpr int TPP = PencilShape<PX>::TPP;
    static constexpr int PPB = 256 / TPP;  // pencils per block
};

template <typename R, int PX, int KIND>
__device__ __forceinline__ void rows_fft_body(const ApplyArgs &a, const int bx, const int by, const int bz) {
    // one block per long row: every thread places whole cells (all fields of
    // a node at once, one round of gathers), then each wavefront transforms
    // its pencils; fields beyond one block's pencils take further passes
    using Cfg = RowCfg<R, PX, KIND>;
    constexpr int TPP = Cfg::TPP, NPEN = Cfg::PPB, E = PX / TPP, PS = pstride<PX>();
    constexpr int F = Terms<KIND>::F;
    const int d = bx;
    if (d >= a.nd) return;  // block-uniform: batched members with fewer long rows
    __shared__ cx<R> buf[NPEN * PS];
    __shared__ cx<R> tw[PX];
    const int tid = threadIdx.x;
    const cx<R> *gtwx = static_cast<const cx<R> *>(a.twx);
    for (int i = tid; i < PX; i += 256) tw[i] = gtwx[i];
    const int row = a.dense_rows[d];
    const int s0 = a.rowptr[row], s1 = a.rowptr[row + 1];
    const int pen = tid / TPP, t = tid % TPP;
    cx<R> *pb = buf + pen * PS;
    cx<R> *Xd = static_cast<cx<R> *>(a.Xd);
#pragma unroll
    for (int f0 = 0; f0 < F; f0 += NPEN) {
#pragma unroll
        for (int e = 0; e < E; ++e) pb[pslot(t + e * TPP)] = {R(0), R(0)};
        __syncthreads();
        for (int s = s0 + tid; s < s1; s += 256) {
            const int x = a.gx[s];
            if (s > s0 && a.gx[s - 1] == x) continue;  // summed by the first node of the cell
            R v[F];
            node_fields<R, KIND>(a, s, v);  // all fields of the node from one set of loads
            for (int s2 = s + 1; s2 < s1 && a.gx[s2] == x; ++s2) {
                R v2[F];
                node_fields<R, KIND>(a, s2, v2);
#pragma unroll
                for (int f = 0; f < F; ++f) v[f] += v2[f];
            }
#pragma unroll
            for (int fl = 0; fl < NPEN; ++fl)
                if (f0 + fl < F) buf[fl * PS + pslot(x)] = {v[f0 + fl], R(0)};
        }
        __syncthreads();
        const int f = f0 + pen;
        cx<R> xr[E];
#pragma unroll
        for (int e = 0; e < E; ++e) xr[e] = pb[pslot(t + e * TPP)];
        fft_regs<R, PX, -1>(xr, pb, tw, t);
        if (f < F) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int kx = t + e * TPP;
                if (kx < a.hx) Xd[((size_t)d * F + f) * a.hx + kx] = xr[e];
            }
        }
        __syncthreads();  // the next pass rewrites the pencils
    }
}

// Field scatter and long-row transforms in one launch (they do not depend on each
// other): the first nfb blocks scatter the fields, the rest transform rows.
template <typename R, int PX, int KIND>
__global__ __launch_bounds__(256) void k_fields_rows(ApplyArgs a, int nfb) {
    if ((int)blockIdx.x < nfb) fields_body<R, KIND>(a, blockIdx.x, 0, 0);
    else rows_fft_body<R, PX, KIND>(a, blockIdx.x - nfb, 0, 0);
}

// Batched form: blockIdx.z = member * zdiv + the kernel's own z index.
template <typename R, int PX, int KIND>
__global__ __launch_bounds__(256) void kb_rows_fft(const ApplyArgs *members, const BatchIO *io, int zdiv) {
    ApplyArgs a = members[blockIdx.z / zdiv];
    if (io->active && !io->active[a.gid]) return;
    a.q = io->q + a.off;
    a.u = io->u + a.off;
    a.r = io->r + a.off;
    rows_fft_body<R, PX, KIND>(a, blockIdx.x, blockIdx.y, blockIdx.z % zdiv);
}

// ------------------------------------------------------------------ k_fwd_xy
template <typename R, int PY, int KIND>
struct FwdCfg {
    static constexpr int F = Terms<KIND>::F;
    static constexpr int TPP = PencilShape<PY>::TPP;
    static constexpr int CB = (int)sizeof(cx<R>);
    static constexpr int PS = pstride<PY>();
    static constexpr int FIXED = PY * CB;
    // kx per block: 4 in FP32; 2 in FP64, where more, smaller blocks hide the
    // node loads of the direct DFT better (the 128^3 cube: 82 -> 72 us)
    static constexpr int KXC = clampi(mini(256 / (F * TPP), (64 * 1024 - FIXED) / (F * PS * CB)), 1, CB == 16 ? 2 : 4);
    static constexpr int NT = F * KXC * TPP;
};

// XG: kx per thread in the direct DFT (1, or 2 on plans whose short rows
// hold few nodes, where one node load then serves two kx).
template <typename R, int PY, int KIND, int XG_, typename YS = cx<R>>
__device__ __forceinline__ void fwd_xy_body(const ApplyArgs &a, const int bx, const int by, const int bz) {
    if (by >= a.nzo) return;  // batched: a member with fewer occupied planes
    using Cfg = FwdCfg<R, PY, KIND>;
    constexpr int F = Cfg::F, KXC = Cfg::KXC, NT = Cfg::NT, TPP = Cfg::TPP, PS = Cfg::PS, E = PY / TPP;
    __shared__ cx<R> buf[F * KXC * PS];
    __shared__ cx<R> tw[PY];
    const int tid = threadIdx.x;
    const int kx0 = bx * KXC;
    const int zz = by;
    const cx<R> *gtwx = static_cast<const cx<R> *>(a.twx);
    const cx<R> *gtwy = static_cast<const cx<R> *>(a.twy);
    const R *vf = static_cast<const R *>(a.vf);
    const cx<R> *Xd = static_cast<const cx<R> *>(a.Xd);
    for (int i = tid; i < PY; i += NT) tw[i] = gtwy[i];
    __syncthreads();
    const float inv_px = 1.0f / (float)a.px;
    // x-transform of the zero-extended fields for rows y < ny: a direct DFT
    // over the row's few nodes, or the row FFT of a long row.  A thread takes
    // one row and XG consecutive kx: each node's data is loaded once for the
    // XG kx and its twiddles are stepped from (kx x) mod px.
    constexpr int XG = clampi(XG_, 1, KXC);
    constexpr int NG = (KXC + XG - 1) / XG;
    for (int it = tid; it < NG * a.ny; it += NT) {
        const int gk = it % NG, y = it / NG;
        const int kxa = kx0 + gk * XG;
        const int row = zz * a.ny + y;
        const int dense = a.row_dense[row];
        const int r0 = a.rowptr[row], r1 = a.rowptr[row + 1];
        cx<R> acc[XG][F];
        if (dense >= 0) {
#pragma unroll
            for (int k = 0; k < XG; ++k)
#pragma unroll
                for (int f = 0; f < F; ++f)
                    acc[k][f] = (kxa + k < a.hx) ? Xd[((size_t)dense * F + f) * a.hx + kxa + k] : cx<R>{R(0), R(0)};
        } else {
#pragma unroll
            for (int k = 0; k < XG; ++k)
#pragma unroll
                for (int f = 0; f < F; ++f) acc[k][f] = {R(0), R(0)};
            // the x twiddles come from the block's LDS table when Px = Py
            // (the same table), else through the caches
            auto row_sum = [&](const cx<R> *twt) {
#pragma unroll 4
                for (int s = r0; s < r1; ++s) {
                    const int xg = a.gx[s];
                    R vv[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) vv[f] = vf[f * a.m + s];
                    int idx = mod_small(kxa, xg, a.px, inv_px);
#pragma unroll
                    for (int k = 0; k < XG; ++k) {
                        const cx<R> w = twt[idx];
#pragma unroll
                        for (int f = 0; f < F; ++f) {
                            acc[k][f].x += vv[f] * w.x;
                            acc[k][f].y += vv[f] * w.y;
                        }
                        idx += xg;
                        if (idx >= a.px) idx -= a.px;
                    }
                }
            };
            if (a.px == PY) row_sum(tw);
            else row_sum(gtwx);
        }
#pragma unroll
        for (int k = 0; k < XG; ++k)
            if (gk * XG + k < KXC)
#pragma unroll
                for (int f = 0; f < F; ++f) buf[(f * KXC + gk * XG + k) * PS + pslot(y)] = acc[k][f];
    }
    __syncthreads();
    // y-FFT in registers (rows y >= ny are zero), stored straight from them
    const int pen = tid / TPP, t = tid % TPP;
    const int f = pen / KXC, kx = kx0 + pen % KXC;
    cx<R> *pb = buf + pen * PS;
    cx<R> x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        // rows y >= P/2 lie beyond the grid (ny <= P/2): zero at compile time
        const int y = t + e * TPP;
        x[e] = (e < E / 2 && y < a.ny) ? pb[pslot(y)] : cx<R>{R(0), R(0)};
    }
    fft_regs<R, PY, -1>(x, pb, tw, t);
    if (kx < a.hx) {
        YS *Y = static_cast<YS *>(a.Y) + ((size_t)(f * a.hx + kx) * a.nzo + zz) * PY;
#pragma unroll
        for (int e = 0; e < E; ++e) Y[t + e * TPP] = to_store<YS>(x[e]);
    }
}

template <typename R, int PY, int KIND, int XG, typename YS = cx<R>>
// Grid (nzo, kx groups): consecutive blocks take consecutive planes of the
// same kx group, so blocks in flight write neighbouring rows of Y.
__global__ __launch_bounds__((FwdCfg<R, PY, KIND>::NT)) void k_fwd_xy(ApplyArgs a) {
    fwd_xy_body<R, PY, KIND, XG, YS>(a, blockIdx.y, blockIdx.x, blockIdx.z);
}

// Batched form: blockIdx.z = member * zdiv + the kernel's own z index.
template <typename R, int PY, int KIND>
__global__ __launch_bounds__((FwdCfg<R, PY, KIND>::NT)) void kb_fwd_xy(const ApplyArgs *members, const BatchIO *io, int zdiv) {
    ApplyArgs a = members[blockIdx.z / zdiv];
    if (io->active && !io->active[a.gid]) return;
    a.q = io->q + a.off;
    a.u = io->u + a.off;
    a.r = io->r + a.off;
    fwd_xy_body<R, PY, KIND, 1>(a, blockIdx.x, blockIdx.y, blockIdx.z % zdiv);
}

// ------------------------------------------------------------------ k_zpass
// One wavefront owns PPW = 64/TPP pencils (consecutive ky at one kx) from
// load to store; waves never wait for each other, so the loads of one wave
// overlap the transforms of the others.  Lane t of a pencil loads the rows
// its first FFT stage needs straight into registers, multiplies the
// transformed values in registers, and stores the inverse transform's rows
// from registers: LDS only carries the exchange between FFT stages.
template <typename R, typename SH, int KIND>
struct ZCfg {
    static constexpr int PZ = SH::P;
    static constexpr int TPP = SH::TPP;
    static constexpr int PPW = 64 / TPP;
    static constexpr int CB = (int)sizeof(cx<R>);
    static constexpr int PS = pstride<PZ>();
    static constexpr int WAVES = clampi((64 * 1024) / (PPW * PS * CB), 1, 4);
    static constexpr int TY = PPW * WAVES;
    static constexpr int NT = 64 * WAVES;
    static constexpr int E = PZ / TPP;
};

// Kernel spectrum value for component c at (kx, ky, kz) from the octant
// store, with the reflection sign of each odd axis.
template <typename R, int KIND>
__device__ __forceinline__ R spec_at(const R *spec, const ApplyArgs &a, int c, int kx, int ky, int kz) {
    const int mask = comp_oddmask(KIND, c);
    const int kyp = ky < a.hy ? ky : a.py - ky;
    const int kzp = kz < a.hz ? kz : a.pz - kz;
    R s = spec[(((size_t)c * a.hx + kx) * a.hy + kyp) * a.hz + kzp];
    const bool flip = ((ky >= a.hy) && (mask & 2)) != ((kz >= a.hz) && (mask & 4));
    return flip ? -s : s;
}

template <typename R>
__device__ __forceinline__ void mac(cx<R> &acc, cx<R> v, R s, bool imag) {
    if (imag) {  // (i s) v
        acc.x -= s * v.y;
        acc.y += s * v.x;
    } else {
        acc.x += s * v.x;
        acc.y += s * v.y;
    }
}

template <typename R, typename SH, int KIND>
__device__ __forceinline__ void zpass_body(const ApplyArgs &a, const int bx, const int by, const int bz) {
    using Cfg = ZCfg<R, SH, KIND>;
    constexpr int PZ = SH::P;
    using T = Terms<KIND>;
    constexpr int PPW = Cfg::PPW, TY = Cfg::TY, NT = Cfg::NT, TPP = Cfg::TPP, E = Cfg::E, PS = Cfg::PS;
    constexpr int F = T::F, O = T::O;
    __shared__ cx<R> buf[TY * PS];
    __shared__ cx<R> tw[PZ];
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int kx = bx;
    const int b = lane / TPP, t = lane % TPP;
    const int ky = by * TY + wave * PPW + b;
    const bool live = ky < a.py;
    cx<R> *pb = buf + (wave * PPW + b) * PS;
    const cx<R> *twz = static_cast<const cx<R> *>(a.twz);
    const R *spec = static_cast<const R *>(a.spec);
    for (int i = tid; i < PZ; i += NT) tw[i] = twz[i];
    __syncthreads();
    cx<R> acc[O][E];
#pragma unroll
    for (int o = 0; o < O; ++o)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[o][e] = {R(0), R(0)};

    // Row and spectrum addressing, hoisted out of the element loops: lane t
    // holds z = t + e*TPP; elements e < E/2 lie in the lower half (kz < P/2,
    // read straight from the octant), e >= E/2 in the upper half (kz >= P/2,
    // read at P - kz with the z-reflection sign; kz = P/2 reads the Nyquist
    // plane, where every z-odd spectrum is zero, so its sign is immaterial).
    const int zoff = t - a.z0;
    const int64_t estride = (int64_t)TPP * a.py;
    const size_t fstride = (size_t)a.hx * a.nzo * a.py;
    const cx<R> *Yl = static_cast<const cx<R> *>(a.Y) + (size_t)kx * a.nzo * a.py + (int64_t)zoff * a.py + ky;
    const int kyp = ky < a.hy ? ky : a.py - ky;
    const bool fy = ky >= a.hy;
    const R *srow = spec + ((size_t)kx * a.hy + kyp) * a.hz;
    const size_t cstride = (size_t)a.hx * a.hy * a.hz;

    // Field f's rows into registers: occupied planes only (planes z >= P/2 are
    // padding, the grid spans at most P/2 planes).  With nine fields (Navier)
    // the next field's loads are issued before this field's transform.  They
    // are branch-free -- a load from a valid address (Y's first element,
    // written by the forward pass), times zero where the plane is not occupied
    // -- so one field's loads sit in one block and the wait before a transform
    // counts only that field's loads, not the next field's, in flight.  The
    // four-field kinds, and FP64 below 384 points (registers near the limit),
    // keep the plain conditional loads: there the extra registers cost more
    // occupancy than the overlap gains (measured on the 128^3 Navier sphere:
    // FP64 at 256 points 342 -> 541 us with it; FP32 195 -> 185 us).
    constexpr bool kPrefetch = KIND == 2 && (sizeof(R) == 4 || PZ >= 384);
    const cx<R> *Ybase = static_cast<const cx<R> *>(a.Y);
    auto load_field = [&](int f, cx<R> *x) {
        const cx<R> *Yf = Yl + f * fstride;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int zz = zoff + e * TPP;  // occupied plane index; others are zero
            if (e >= E / 2) {
                x[e] = cx<R>{R(0), R(0)};
            } else if constexpr (kPrefetch) {
                const bool ok = live && zz >= 0 && zz < a.nzo;
                const cx<R> v = *(ok ? Yf + e * estride : Ybase);
                const R mk = ok ? R(1) : R(0);  // a product, not a select: the load stays unconditional
                x[e] = cx<R>{v.x * mk, v.y * mk};
            } else {
                x[e] = (live && zz >= 0 && zz < a.nzo) ? Yf[e * estride] : cx<R>{R(0), R(0)};
            }
        }
    };
    [[maybe_unused]] cx<R> xn[kPrefetch ? E : 1];
    if constexpr (kPrefetch) load_field(0, xn);
    static_for<0, F>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        cx<R> x[E];
        if constexpr (kPrefetch) {
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = xn[e];
            if constexpr (f + 1 < F) load_field(f + 1, xn);  // next field in flight during this one
        } else {
            load_field(f, x);
        }
        fft_regs_s<R, SH, -1>(x, pb, tw, t);
        if (live) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int kz = t + e * TPP;
                const int kzp = e < E / 2 ? kz : PZ - kz;
                static_for<0, T::N>([&](auto tc) {
                    constexpr int term = decltype(tc)::value;
                    if constexpr (T::f(term) == f) {
                        constexpr int c = T::c(term);
                        constexpr int mask = comp_oddmask(KIND, c);
                        const R sv = srow[c * cstride + kzp];
                        const bool flip = (fy && (mask & 2)) != ((e >= E / 2) && (mask & 4));
                        mac<R>(acc[T::o(term)][e], x[e], flip ? -sv : sv, comp_imag(KIND, c));
                    }
                });
            }
        }
    });

#pragma unroll
    for (int o = 0; o < O; ++o) {
        fft_regs_s<R, SH, 1>(acc[o], pb, tw, t);
        if (live) {
            cx<R> *Zl = static_cast<cx<R> *>(a.Z) + (size_t)(o * a.hx + kx) * a.nzo * a.py + (int64_t)zoff * a.py + ky;
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {  // outputs z >= P/2 are never needed
                const int zz = zoff + e * TPP;
                if (zz >= 0 && zz < a.nzo) Zl[e * estride] = acc[o][e];
            }
        }
    }
}

// One-dimensional grid of 8 * ceil(hx * nby / 8) blocks.  Blocks go to the
// 8 XCDs round-robin, so block b runs on XCD b % 8; each XCD is given one
// contiguous run of (kx, ky-block) work items, ordered so that the blocks of
// one kx and their mirrored ky blocks (which read the same octant rows of
// the spectra) follow each other on the same L2.
template <typename R, typename SH, int KIND>
__global__ __launch_bounds__((ZCfg<R, SH, KIND>::NT)) void k_zpass(ApplyArgs a, int nby) {
    const int total = a.hx * nby;
    const int per = (total + 7) / 8;
    const int lam = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (lam >= total) return;
    const int kx = lam / nby, j = lam % nby;
    const int by = (j & 1) ? nby - 1 - (j >> 1) : (j >> 1);
    zpass_body<R, SH, KIND>(a, kx, by, 0);
}

// Batched form: blockIdx.z = member * zdiv + the kernel's own z index.
template <typename R, typename SH, int KIND>
__global__ __launch_bounds__((ZCfg<R, SH, KIND>::NT)) void kb_zpass(const ApplyArgs *members, const BatchIO *io, int zdiv) {
    ApplyArgs a = members[blockIdx.z / zdiv];
    if (io->active && !io->active[a.gid]) return;
    a.q = io->q + a.off;
    a.u = io->u + a.off;
    a.r = io->r + a.off;
    zpass_body<R, SH, KIND>(a, blockIdx.x, blockIdx.y, blockIdx.z % zdiv);
}

// 2D: the third axis has length 1, so the "z pass" is the spectral product.
template <typename R, int KIND>
__device__ __forceinline__ void mac2d_body(const ApplyArgs &a, const int bx, const int by, const int bz) {
    using T = Terms<KIND>;
    constexpr int O = T::O;
    const int kx = bx;
    const int ky = by * 256 + threadIdx.x;
    if (ky >= a.py) return;
    const cx<R> *Y = static_cast<const cx<R> *>(a.Y);
    cx<R> *Z = static_cast<cx<R> *>(a.Z);
    const R *spec = static_cast<const R *>(a.spec);
    cx<R> acc[O];
#pragma unroll
    for (int o = 0; o < O; ++o) acc[o] = {R(0), R(0)};
    static_for<0, T::N>([&](auto tc) {
        constexpr int term = decltype(tc)::value;
        constexpr int c = T::c(term), o = T::o(term), f = T::f(term);
        const cx<R> v = Y[(size_t)(f * a.hx + kx) * a.py + ky];
        mac<R>(acc[o], v, spec_at<R, KIND>(spec, a, c, kx, ky, 0), comp_imag(KIND, c));
    });
#pragma unroll
    for (int o = 0; o < O; ++o) Z[(size_t)(o * a.hx + kx) * a.py + ky] = acc[o];
}

template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_mac2d(ApplyArgs a) {
    mac2d_body<R, KIND>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Batched form: blockIdx.z = member * zdiv + the kernel's own z index.
template <typename R, int KIND>
__global__ __launch_bounds__(256) void kb_mac2d(const ApplyArgs *members, const BatchIO *io, int zdiv) {
    ApplyArgs a = members[blockIdx.z / zdiv];
    if (io->active && !io->active[a.gid]) return;
    a.q = io->q + a.off;
    a.u = io->u + a.off;
    a.r = io->r + a.off;
    mac2d_body<R, KIND>(a, blockIdx.x, blockIdx.y, blockIdx.z % zdiv);
}

// ------------------------------------------------------------------ k_inv_y
template <typename R, int PY, int KIND>
struct InvYCfg {
    static constexpr int O = Terms<KIND>::O;
    static constexpr int TPP = PencilShape<PY>::TPP;
    static constexpr int CB = (int)sizeof(cx<R>);
    static constexpr int PS = pstride<PY>();
    static constexpr int KXC = clampi(mini(256 / (O * TPP), (64 * 1024 - PY * CB) / (O * PS * CB)), 1, 16);
    static constexpr int NT = O * KXC * TPP;
};

// all_rows = 0 (the apply): only rows that hold nodes are stored, the
// gather reads nothing else; all_rows = 1 (the grid evaluation): every row.
template <typename R, int PY, int KIND, typename ZS = cx<R>>
__device__ __forceinline__ void inv_y_body(const ApplyArgs &a, const int bx, const int by, const int all_rows) {
    if (by >= a.nzo) return;  // batched: a member with fewer occupied planes
    using Cfg = InvYCfg<R, PY, KIND>;
    constexpr int O = Cfg::O, KXC = Cfg::KXC, NT = Cfg::NT, TPP = Cfg::TPP, PS = Cfg::PS, E = PY / TPP;
    __shared__ cx<R> buf[O * KXC * PS];
    __shared__ cx<R> tw[PY];
    __shared__ unsigned char keep[PY / 2];
    const int tid = threadIdx.x;
    const int kx0 = bx * KXC;
    const int zz = by;
    const cx<R> *gtwy = static_cast<const cx<R> *>(a.twy);
    for (int i = tid; i < PY; i += NT) tw[i] = gtwy[i];
    for (int y = tid; y < a.ny; y += NT)
        keep[y] = all_rows || a.rowptr[zz * a.ny + y + 1] > a.rowptr[zz * a.ny + y];
    const int pen = tid / TPP, t = tid % TPP;
    const int o = pen / KXC, kx = kx0 + pen % KXC;
    cx<R> x[E];
    if (kx < a.hx) {
        const ZS *Zr = static_cast<const ZS *>(a.Z) + ((size_t)(o * a.hx + kx) * a.nzo + zz) * PY;
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = from_store<R>(Zr[t + e * TPP]);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = {R(0), R(0)};
    }
    __syncthreads();  // twiddle table, row flags
    cx<R> *pb = buf + pen * PS;
    fft_regs<R, PY, 1>(x, pb, tw, t);
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {  // ny <= Py/2: rows y >= Py/2 hold no node
        const int y = t + e * TPP;
        if (y < a.ny) pb[pslot(y)] = x[e];
    }
    __syncthreads();  // the transposed store reads every pencil
    const int nk = min(KXC, a.hx - kx0);
    cx<R> *W = static_cast<cx<R> *>(a.Y);
    for (int i = tid; i < O * a.ny * KXC; i += NT) {
        const int kl = i % KXC, rest = i / KXC;
        const int y = rest % a.ny, oo = rest / a.ny;
        if (kl < nk && keep[y])
            W[((size_t)(oo * a.nzo + zz) * a.ny + y) * a.hx + kx0 + kl] = buf[(oo * KXC + kl) * PS + pslot(y)];
    }
}

template <typename R, int PY, int KIND, typename ZS = cx<R>>
__global__ __launch_bounds__((InvYCfg<R, PY, KIND>::NT)) void k_inv_y(ApplyArgs a, int all_rows) {
    inv_y_body<R, PY, KIND, ZS>(a, blockIdx.x, blockIdx.y, all_rows);
}

// Batched form: blockIdx.z = member * zdiv + the kernel's own z index.
template <typename R, int PY, int KIND>
__global__ __launch_bounds__((InvYCfg<R, PY, KIND>::NT)) void kb_inv_y(const ApplyArgs *members, const BatchIO *io, int zdiv) {
    const ApplyArgs &a = members[blockIdx.z / zdiv];
    if (io->active && !io->active[a.gid]) return;
    inv_y_body<R, PY, KIND>(a, blockIdx.x, blockIdx.y, 0);
}

// ------------------------------------------------------------------ whole rows, inverse x
template <typename R, int PX>
struct RowInvCfg {
    static constexpr int TPP = PencilShape<PX>::TPP;
    static constexpr int CB = (int)sizeof(cx<R>);
    static constexpr int PS = pstride<PX>();
    static constexpr int PPB = clampi(mini(256 / TPP, (64 * 1024 - PX * CB) / (PS * CB)), 1, 64);
    static constexpr int NT = PPB * TPP;
};

// Inverse x transform of two real rows from their half spectra Wa, Wb (Hx =
// PX/2 + 1 coefficients; a missing row is zero): the spectra are extended to
// Hermitian sequences A, B (imaginary parts at kx = 0 and PX/2 dropped, as
// the node gather does) and packed as A + iB, so one complex inverse FFT of
// length PX holds row a in its real and row b in its imaginary part.  Lane t
// of the pencil ends with x[e] = value at t + e TPP.  tw: the LDS twiddle
// table, already synchronised.
template <typename R, int PX>
__device__ __forceinline__ void inv_x_pair(const cx<R> *Wa, const cx<R> *Wb, bool va, bool vb, cx<R> *pen,
                                           const cx<R> *tw, int t, cx<R> (&x)[PX / PencilShape<PX>::TPP]) {
    constexpr int TPP = PencilShape<PX>::TPP, E = PX / TPP;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TPP;
        const bool lo = 2 * k <= PX;
        const int kk = lo ? k : PX - k;  // kk < Hx
        cx<R> A = va ? Wa[kk] : cx<R>{R(0), R(0)};
        cx<R> B = vb ? Wb[kk] : cx<R>{R(0), R(0)};
        if (kk == 0 || 2 * kk == PX) {
            A.y = R(0);
            B.y = R(0);
        }
        if (!lo) {  // Hermitian extension: conj of the mirrored coefficient
            A.y = -A.y;
            B.y = -B.y;
        }
        x[e] = {A.x - B.y, A.y + B.x};  // A + iB
    }
    fft_regs<R, PX, 1>(x, pen, tw, t);
}

// Long rows (those whose forward x transform was an FFT) get their inverse x
// transform by FFT too: row (d, o) of W -> Xr[d][o][x], x < nx, in the
// buffer of the forward row transforms (free after the forward pass).  The
// gather then reads their nodes' values instead of summing the row's
// spectrum once per node.
template <typename R, int PX, int KIND>
__device__ __forceinline__ void rows_inv_body(const ApplyArgs &a, const int bx) {
    using Cfg = RowInvCfg<R, PX>;
    constexpr int O = Terms<KIND>::O, TPP = Cfg::TPP, PS = Cfg::PS, PPB = Cfg::PPB, NT = Cfg::NT, E = PX / TPP;
    __shared__ cx<R> buf[PPB * PS];
    __shared__ cx<R> tw[PX];
    const int nrows = a.row_inv ? a.nd * O : 0;
    if (bx * PPB * 2 >= nrows) return;  // block-uniform: batched members with fewer long rows
    const int tid = threadIdx.x;
    const cx<R> *gtwx = static_cast<const cx<R> *>(a.twx);
    for (int i = tid; i < PX; i += NT) tw[i] = gtwx[i];
    __syncthreads();
    const int pen = tid / TPP, t = tid % TPP;
    const int ra = (bx * PPB + pen) * 2, rb = ra + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    const cx<R> *W = static_cast<const cx<R> *>(a.Y);
    const size_t ostride = (size_t)a.nzo * a.ny;  // rows of W per output
    const cx<R> *Wa = W + ((size_t)(ra % O) * ostride + (va ? a.dense_rows[ra / O] : 0)) * a.hx;
    const cx<R> *Wb = W + ((size_t)(rb % O) * ostride + (vb ? a.dense_rows[rb / O] : 0)) * a.hx;
    cx<R> x[E];
    inv_x_pair<R, PX>(Wa, Wb, va, vb, buf + pen * PS, tw, t, x);
    R *Xr = static_cast<R *>(a.Xd);
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {  // nx <= Px/2
        const int xg = t + e * TPP;
        if (xg < a.nx) {
            if (va) Xr[(size_t)ra * a.nx + xg] = x[e].x;
            if (vb) Xr[(size_t)rb * a.nx + xg] = x[e].y;
        }
    }
}

template <typename R, int PX, int KIND>
__global__ __launch_bounds__((RowInvCfg<R, PX>::NT)) void k_rows_inv(ApplyArgs a) {
    rows_inv_body<R, PX, KIND>(a, blockIdx.x);
}

// Batched form: blockIdx.z = member.
template <typename R, int PX, int KIND>
__global__ __launch_bounds__((RowInvCfg<R, PX>::NT)) void kb_rows_inv(const ApplyArgs *members, const BatchIO *io) {
    const ApplyArgs &a = members[blockIdx.z];
    if (io->active && !io->active[a.gid]) return;
    rows_inv_body<R, PX, KIND>(a, blockIdx.x);
}

// ------------------------------------------------------------------ k_gather
// Eight lanes per node: the inverse x transform of the node's row in W,
//   sum_kx cf Re(W[kx] exp(+2 pi i kx x / Px)),  cf = 1 at kx = 0 and Px/2,
//   2 between (the real field from its half spectrum),
// evaluated at the node's x only.  Lane l of a node takes kx = 1 + l, 9 + l,
// ... (the eight lanes read consecutive coefficients), accumulates in FP64,
// and a fixed shuffle tree sums the lanes (reproducible); the first lane
// adds kx = 0, Px/2 and r = c u - (exact - grid) self term q.
constexpr int kGatherLanes = 8;

template <typename R, int KIND>
__device__ __forceinline__ void gather_body(const ApplyArgs &a, const int bx) {
    constexpr int O = Terms<KIND>::O, L = kGatherLanes;
    __shared__ cx<R> twx[(KIND == 0 || KIND == 3) ? kMaxPx : kMaxPx / 2];  // 3D: px <= 512
    const cx<R> *gtwx = static_cast<const cx<R> *>(a.twx);
    for (int i = threadIdx.x; i < a.px; i += 256) twx[i] = gtwx[i];
    __syncthreads();
    const int sub = threadIdx.x % L;
    const int s = bx * (256 / L) + threadIdx.x / L;
    if (s >= a.m) return;  // the node's eight lanes leave together
    const int zz = a.gz[s] - a.z0, y = a.gy[s], xg = a.gx[s];
    const int dr = a.row_inv ? a.row_dense[zz * a.ny + y] : -1;
    if (dr >= 0) {  // a long row: its values come from the row FFT
        if (sub != 0) return;
        const R *Xr = static_cast<const R *>(a.Xd);
        const int j = a.perm[s];
#pragma unroll
        for (int o = 0; o < O; ++o) {
            double v = (double)Xr[((size_t)dr * O + o) * a.nx + xg];
#pragma unroll
            for (int l = 0; l < O; ++l) {
                v += a.C[((size_t)s * O + o) * O + l] * a.u[l * a.m + j];
                v -= a.SC[((size_t)s * O + o) * O + l] * a.q[l * a.m + j];
            }
            a.r[o * a.m + j] = v;
        }
        return;
    }
    const int hx = a.hx, px = a.px;
    const size_t rstride = (size_t)a.nzo * a.ny * hx;  // between outputs
    const cx<R> *row = static_cast<const cx<R> *>(a.Y) + ((size_t)zz * a.ny + y) * hx;
    double acc[O];
#pragma unroll
    for (int o = 0; o < O; ++o) acc[o] = 0.0;
    const int step = (L * xg) % px;
    int idx = ((1 + sub) * xg) % px;  // (kx x) mod px
    int kx = 1 + sub;
    // eight coefficients per output in flight before they are used.  Past
    // the row's end a lane loads kx = 1 (in bounds: the loop runs only when
    // hx >= 3) and weighs it by zero -- a product, so the load stays
    // unconditional and the chunk's loads are waited for together.
    for (; kx < hx - 1; kx += 8 * L) {
        cx<R> v[8][O];
        R mk[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool in = kx + k * L < hx - 1;
            const int kc = in ? kx + k * L : 1;
            mk[k] = in ? R(1) : R(0);
#pragma unroll
            for (int o = 0; o < O; ++o) v[k][o] = row[o * rstride + kc];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const cx<R> w = twx[idx];
#pragma unroll
            for (int o = 0; o < O; ++o) acc[o] += (double)((v[k][o].x * w.x + v[k][o].y * w.y) * mk[k]);
            idx += step;
            if (idx >= px) idx -= px;
        }
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1)
#pragma unroll
        for (int o = 0; o < O; ++o) acc[o] += __shfl_xor(acc[o], off, 64);
    if (sub != 0) return;
    const R wn = (xg & 1) ? R(-1) : R(1);  // exp(i pi x)
    const int j = a.perm[s];
#pragma unroll
    for (int o = 0; o < O; ++o) {
        const cx<R> v0 = row[o * rstride];
        const cx<R> vn = row[o * rstride + hx - 1];
        double v = (double)v0.x + (double)(vn.x * wn) + 2.0 * acc[o];
#pragma unroll
        for (int l = 0; l < O; ++l) {
            v += a.C[((size_t)s * O + o) * O + l] * a.u[l * a.m + j];
            v -= a.SC[((size_t)s * O + o) * O + l] * a.q[l * a.m + j];
        }
        a.r[o * a.m + j] = v;
    }
}

template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_gather(ApplyArgs a) {
    gather_body<R, KIND>(a, blockIdx.x);
}

// Batched form: blockIdx.z = member.
template <typename R, int KIND>
__global__ __launch_bounds__(256) void kb_gather(const ApplyArgs *members, const BatchIO *io) {
    ApplyArgs a = members[blockIdx.z];
    if (io->active && !io->active[a.gid]) return;
    a.q = io->q + a.off;
    a.u = io->u + a.off;
    a.r = io->r + a.off;
    gather_body<R, KIND>(a, blockIdx.x);
}

// ------------------------------------------------------------------ launchers
template <typename R, int PY, int KIND, typename YS = cx<R>>
int launch_fwd(const ApplyArgs &a, hipStream_t st) {
    using Cfg = FwdCfg<R, PY, KIND>;
    dim3 grid(a.nzo, (a.hx + Cfg::KXC - 1) / Cfg::KXC);
    if (a.fwd_xg == 2) hipLaunchKernelGGL((k_fwd_xy<R, PY, KIND, 2, YS>), grid, dim3(Cfg::NT), 0, st, a);
    else hipLaunchKernelGGL((k_fwd_xy<R, PY, KIND, 1, YS>), grid, dim3(Cfg::NT), 0, st, a);
    BF_HIP(hipGetLastError());
    return 0;
}
template <typename R, int PY, int KIND, typename ZS = cx<R>>
int launch_inv_y(const ApplyArgs &a, int all_rows, hipStream_t st) {
    using Cfg = InvYCfg<R, PY, KIND>;
    dim3 grid((a.hx + Cfg::KXC - 1) / Cfg::KXC, a.nzo);
    hipLaunchKernelGGL((k_inv_y<R, PY, KIND, ZS>), grid, dim3(Cfg::NT), 0, st, a, all_rows);
    BF_HIP(hipGetLastError());
    return 0;
}
template <typename R, int PZ, int KIND, int SCHED>
int launch_z(const ApplyArgs &a, hipStream_t st) {
    if constexpr (PZ == 1) {
        dim3 grid(a.hx, (a.py + 255) / 256);
        hipLaunchKernelGGL((k_mac2d<R, KIND>), grid, dim3(256), 0, st, a);
    } else {
        using SH = Sched<PZ, SCHED>;
        using Cfg = ZCfg<R, SH, KIND>;
        const int nby = (a.py + Cfg::TY - 1) / Cfg::TY;
        const int per = (a.hx * nby + 7) / 8;
        hipLaunchKernelGGL((k_zpass<R, SH, KIND>), dim3(8 * per), dim3(Cfg::NT), 0, st, a, nby);
    }
    BF_HIP(hipGetLastError());
    return 0;
}

#define BF_SIZE_SWITCH(len, FN, ...)                        \
    switch (len) {                                          \
        case 32: return FN<32>(__VA_ARGS__);                \
        case 64: return FN<64>(__VA_ARGS__);                \
        case 96: return FN<96>(__VA_ARGS__);                \
        case 128: return FN<128>(__VA_ARGS__);              \
        case 192: return FN<192>(__VA_ARGS__);              \
        case 256: return FN<256>(__VA_ARGS__);              \
        case 320: return FN<320>(__VA_ARGS__);              \
        case 384: return FN<384>(__VA_ARGS__);              \
        case 512: return FN<512>(__VA_ARGS__);              \
        default: break;                                     \
    }

// As BF_SIZE_SWITCH, plus length 1024 for the 2D families (grids of up to
// 512 points per axis); 3D plans never reach it and do not compile it.
#define BF_SIZE_SWITCH_K(KIND_, len, FN, ...)                              \
    if constexpr (KIND_ == 0 || KIND_ == 3) {                              \
        if ((len) == 1024) return FN<1024>(__VA_ARGS__);                   \
    }                                                                      \
    BF_SIZE_SWITCH(len, FN, __VA_ARGS__)

template <typename R, int KIND>
struct Launch {
    template <int P> static int fwd(const ApplyArgs &a, hipStream_t st) { return launch_fwd<R, P, KIND>(a, st); }
    template <int P> static int rows(const ApplyArgs &a, hipStream_t st) {
        using Cfg = RowCfg<R, P, KIND>;
        const int nfb = (a.m + 255) / 256;
        const int nrb = a.nd;  // one block per long row
        hipLaunchKernelGGL((k_fields_rows<R, P, KIND>), dim3(nfb + nrb), dim3(256), 0, st, a, nfb);
        BF_HIP(hipGetLastError());
        return 0;
    }
    template <int P> static int rows_inv(const ApplyArgs &a, hipStream_t st) {
        using Cfg = RowInvCfg<R, P>;
        const int nb = (a.nd * Terms<KIND>::O + 2 * Cfg::PPB - 1) / (2 * Cfg::PPB);
        hipLaunchKernelGGL((k_rows_inv<R, P, KIND>), dim3(nb), dim3(Cfg::NT), 0, st, a);
        BF_HIP(hipGetLastError());
        return 0;
    }
    template <int P> static int brows_inv(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        using Cfg = RowInvCfg<R, P>;
        const int nb = (g.max_nd * Terms<KIND>::O + 2 * Cfg::PPB - 1) / (2 * Cfg::PPB);
        hipLaunchKernelGGL((kb_rows_inv<R, P, KIND>), dim3(nb, 1, g.nmem), dim3(Cfg::NT), 0, st, dm, io);
        BF_HIP(hipGetLastError());
        return 0;
    }
    static int dispatch_rows_inv(const ApplyArgs &a, hipStream_t st) {
        BF_SIZE_SWITCH_K(KIND, a.px, rows_inv, a, st);
        set_error("unsupported x length");
        return BEMFFT_EUNSUPPORTED;
    }
    template <int P> static int inv_y(const ApplyArgs &a, int all_rows, hipStream_t st) {
        return launch_inv_y<R, P, KIND>(a, all_rows, st);
    }
    template <int P> static int z(const ApplyArgs &a, hipStream_t st) {
        if constexpr (KIND == 2 && has_wide_sched(P)) {
            if (a.zsched == 2) return launch_z<R, P, KIND, 2>(a, st);
        }
        return a.zsched == 1 ? launch_z<R, P, KIND, 1>(a, st) : launch_z<R, P, KIND, 0>(a, st);
    }

    // Fields, forward x/y and the z pass: everything up to Z.  ev (optional):
    // events 0-2 recorded around the two stages.
    static int front(const ApplyArgs &a, hipStream_t st, hipEvent_t *ev = nullptr) {
        if (ev) BF_HIP(hipEventRecord(ev[0], st));
        if (a.nd > 0) {
            BF_CHECK(dispatch_rows(a, st));  // fields and long-row transforms, one launch
        } else {
            hipLaunchKernelGGL((k_fields<R, KIND>), dim3((a.m + 255) / 256), dim3(256), 0, st, a);
        }
        BF_CHECK(dispatch_fwd(a, st));
        if (ev) BF_HIP(hipEventRecord(ev[1], st));
        BF_CHECK(dispatch_z(a, st));
        if (ev) BF_HIP(hipEventRecord(ev[2], st));
        return 0;
    }

    // ev (optional): five events recorded around the four stages.
    static int run(const ApplyArgs &a, hipStream_t st, hipEvent_t *ev = nullptr) {
        BF_CHECK(front(a, st, ev));
        BF_CHECK(dispatch_inv_y(a, 0, st));
        if (ev) BF_HIP(hipEventRecord(ev[3], st));
        if (a.nd > 0 && a.row_inv) BF_CHECK(dispatch_rows_inv(a, st));
        constexpr int NPB = 256 / kGatherLanes;  // nodes per block
        hipLaunchKernelGGL((k_gather<R, KIND>), dim3((a.m + NPB - 1) / NPB), dim3(256), 0, st, a);
        BF_HIP(hipGetLastError());
        if (ev) BF_HIP(hipEventRecord(ev[4], st));
        return 0;
    }
    static int dispatch_fwd(const ApplyArgs &a, hipStream_t st) {
        BF_SIZE_SWITCH_K(KIND, a.py, fwd, a, st);
        set_error("unsupported y length");
        return BEMFFT_EUNSUPPORTED;
    }
    // ---- batched: one launch per stage for all members of a group
    template <int P> static int bfwd(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        using Cfg = FwdCfg<R, P, KIND>;
        dim3 grid((g.hx + Cfg::KXC - 1) / Cfg::KXC, g.max_nzo, g.nmem);
        hipLaunchKernelGGL((kb_fwd_xy<R, P, KIND>), grid, dim3(Cfg::NT), 0, st, dm, io, 1);
        BF_HIP(hipGetLastError());
        return 0;
    }
    template <int P> static int brows(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        using Cfg = RowCfg<R, P, KIND>;
        dim3 grid(g.max_nd, 1, g.nmem);  // one block per long row
        hipLaunchKernelGGL((kb_rows_fft<R, P, KIND>), grid, dim3(256), 0, st, dm, io, 1);
        BF_HIP(hipGetLastError());
        return 0;
    }
    template <int P> static int binv(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        using Cfg = InvYCfg<R, P, KIND>;
        dim3 grid((g.hx + Cfg::KXC - 1) / Cfg::KXC, g.max_nzo, g.nmem);
        hipLaunchKernelGGL((kb_inv_y<R, P, KIND>), grid, dim3(Cfg::NT), 0, st, dm, io, 1);
        BF_HIP(hipGetLastError());
        return 0;
    }
    template <int PZ, int SCHED>
    static int bz_s(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        if constexpr (PZ == 1) {
            dim3 grid(g.hx, (g.py + 255) / 256, g.nmem);
            hipLaunchKernelGGL((kb_mac2d<R, KIND>), grid, dim3(256), 0, st, dm, io, 1);
        } else {
            using SH = Sched<PZ, SCHED>;
            using Cfg = ZCfg<R, SH, KIND>;
            dim3 grid(g.hx, (g.py + Cfg::TY - 1) / Cfg::TY, g.nmem);
            hipLaunchKernelGGL((kb_zpass<R, SH, KIND>), grid, dim3(Cfg::NT), 0, st, dm, io, 1);
        }
        BF_HIP(hipGetLastError());
        return 0;
    }
    template <int P> static int bz(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        if constexpr (KIND == 2 && has_wide_sched(P)) {
            if (g.zsched == 2) return bz_s<P, 2>(dm, io, g, st);
        }
        return g.zsched == 1 ? bz_s<P, 1>(dm, io, g, st) : bz_s<P, 0>(dm, io, g, st);
    }
    static int run_batch(const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
        hipLaunchKernelGGL((kb_fields<R, KIND>), dim3((g.max_m + 255) / 256, 1, g.nmem), dim3(256), 0, st, dm, io, 1);
        BF_HIP(hipGetLastError());
        if (g.max_nd > 0) {
            int s2 = BEMFFT_EUNSUPPORTED;
            if constexpr (KIND == 0 || KIND == 3) {
                if (g.px == 1024) s2 = brows<1024>(dm, io, g, st);
            }
            switch (g.px) {
                case 32: s2 = brows<32>(dm, io, g, st); break;
                case 64: s2 = brows<64>(dm, io, g, st); break;
                case 96: s2 = brows<96>(dm, io, g, st); break;
                case 128: s2 = brows<128>(dm, io, g, st); break;
                case 192: s2 = brows<192>(dm, io, g, st); break;
                case 256: s2 = brows<256>(dm, io, g, st); break;
                case 320: s2 = brows<320>(dm, io, g, st); break;
                case 384: s2 = brows<384>(dm, io, g, st); break;
                case 512: s2 = brows<512>(dm, io, g, st); break;
                default: break;
            }
            BF_CHECK(s2);
        }
        int s3 = BEMFFT_EUNSUPPORTED;
        if constexpr (KIND == 0 || KIND == 3) {
            if (g.py == 1024) s3 = bfwd<1024>(dm, io, g, st);
        }
        switch (g.py) {
            case 32: s3 = bfwd<32>(dm, io, g, st); break;
            case 64: s3 = bfwd<64>(dm, io, g, st); break;
            case 96: s3 = bfwd<96>(dm, io, g, st); break;
            case 128: s3 = bfwd<128>(dm, io, g, st); break;
            case 192: s3 = bfwd<192>(dm, io, g, st); break;
            case 256: s3 = bfwd<256>(dm, io, g, st); break;
            case 320: s3 = bfwd<320>(dm, io, g, st); break;
            case 384: s3 = bfwd<384>(dm, io, g, st); break;
            case 512: s3 = bfwd<512>(dm, io, g, st); break;
            default: break;
        }
        BF_CHECK(s3);
        int s4 = BEMFFT_EUNSUPPORTED;
        if constexpr (KIND == 0 || KIND == 3) {
            if (g.pz == 1) s4 = bz_s<1, 0>(dm, io, g, st);
        } else {
            switch (g.pz) {
                case 32: s4 = bz<32>(dm, io, g, st); break;
                case 64: s4 = bz<64>(dm, io, g, st); break;
                case 96: s4 = bz<96>(dm, io, g, st); break;
                case 128: s4 = bz<128>(dm, io, g, st); break;
                case 192: s4 = bz<192>(dm, io, g, st); break;
                case 256: s4 = bz<256>(dm, io, g, st); break;
                case 320: s4 = bz<320>(dm, io, g, st); break;
                case 384: s4 = bz<384>(dm, io, g, st); break;
                case 512: s4 = bz<512>(dm, io, g, st); break;
                default: break;
            }
        }
        BF_CHECK(s4);
        int s5 = BEMFFT_EUNSUPPORTED;
        if constexpr (KIND == 0 || KIND == 3) {
            if (g.py == 1024) s5 = binv<1024>(dm, io, g, st);
        }
        switch (g.py) {
            case 32: s5 = binv<32>(dm, io, g, st); break;
            case 64: s5 = binv<64>(dm, io, g, st); break;
            case 96: s5 = binv<96>(dm, io, g, st); break;
            case 128: s5 = binv<128>(dm, io, g, st); break;
            case 192: s5 = binv<192>(dm, io, g, st); break;
            case 256: s5 = binv<256>(dm, io, g, st); break;
            case 320: s5 = binv<320>(dm, io, g, st); break;
            case 384: s5 = binv<384>(dm, io, g, st); break;
            case 512: s5 = binv<512>(dm, io, g, st); break;
            default: break;
        }
        BF_CHECK(s5);
        if (g.max_nd > 0 && g.row_inv) {
            int s6 = BEMFFT_EUNSUPPORTED;
            if constexpr (KIND == 0 || KIND == 3) {
                if (g.px == 1024) s6 = brows_inv<1024>(dm, io, g, st);
            }
            switch (g.px) {
                case 32: s6 = brows_inv<32>(dm, io, g, st); break;
                case 64: s6 = brows_inv<64>(dm, io, g, st); break;
                case 96: s6 = brows_inv<96>(dm, io, g, st); break;
                case 128: s6 = brows_inv<128>(dm, io, g, st); break;
                case 192: s6 = brows_inv<192>(dm, io, g, st); break;
                case 256: s6 = brows_inv<256>(dm, io, g, st); break;
                case 320: s6 = brows_inv<320>(dm, io, g, st); break;
                case 384: s6 = brows_inv<384>(dm, io, g, st); break;
                case 512: s6 = brows_inv<512>(dm, io, g, st); break;
                default: break;
            }
            BF_CHECK(s6);
        }
        constexpr int NPB = 256 / kGatherLanes;  // nodes per block
        hipLaunchKernelGGL((kb_gather<R, KIND>), dim3((g.max_m + NPB - 1) / NPB, 1, g.nmem), dim3(256), 0, st, dm, io);
        BF_HIP(hipGetLastError());
        return 0;
    }

    static int dispatch_rows(const ApplyArgs &a, hipStream_t st) {
        BF_SIZE_SWITCH_K(KIND, a.px, rows, a, st);
        set_error("unsupported x length");
        return BEMFFT_EUNSUPPORTED;
    }
    // all_rows: store every row y < ny (the grid evaluation), not only those
    // that hold nodes (the apply)
    static int dispatch_inv_y(const ApplyArgs &a, int all_rows, hipStream_t st) {
        BF_SIZE_SWITCH_K(KIND, a.py, inv_y, a, all_rows, st);
        set_error("unsupported y length");
        return BEMFFT_EUNSUPPORTED;
    }
    static int dispatch_z(const ApplyArgs &a, hipStream_t st) {
        if constexpr (KIND == 0 || KIND == 3) {
            if (a.pz == 1) return launch_z<R, 1, KIND, 0>(a, st);
            set_error("2D plans need pz == 1");
            return BEMFFT_EUNSUPPORTED;
        } else {
            BF_SIZE_SWITCH(a.pz, z, a, st);
            set_error("unsupported z length");
            return BEMFFT_EUNSUPPORTED;
        }
    }
};

// Per-family entry points, instantiated in one source file per family.
template <int KIND>
int apply_kind(int precision, const ApplyArgs &a, hipStream_t st, hipEvent_t *ev);
template <int KIND>
int apply_batch_kind(int precision, const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st);

// Apply arguments of plan p with the spectra/tables of 'shared' and the
// intermediate buffers of 'ws' (q, u, r left null).
void fill_apply_args(const bemfft_plan *p, const Engine &shared, const Engine &ws, ApplyArgs *a);
// Intermediate buffers of one apply of plan p (Y, Z, fields, long rows),
// without spectra or tables.
int alloc_intermediates(const bemfft_plan *p, int precision, Engine *e);

}  // namespace bemfft
