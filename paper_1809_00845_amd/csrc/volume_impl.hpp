// volume_impl.hpp -- the field over the whole grid box instead of at the
// nodes only.  The representation formula (eq. 4 / eq. 8 with c = 1 for
// points inside the boundary and c = 0 outside, Sec. 2) reads
//     v(p) = S[q](p) - D[u](p),
// and the inverse transform of the convolution gives it at every grid
// point (Sec. 4), so the forward passes, the z pass and the inverse y pass
// of the apply are reused unchanged and only the last stage differs:
//
//   k_inv_y  (the apply's own) inverse y-FFT of every output, rows y < ny
//            written with kx contiguous            -> W[o][z][y][kx]  (in Y)
//   k_vol_x  two grid rows per pencil through inv_x_pair (the half spectra
//            of rows a and b packed as A + iB of their Hermitian extensions;
//            one inverse complex FFT of length Px holds row a in its real and
//            row b in its imaginary part).  x < nx is kept,
//            negated (the grid holds D[u] - S[q]; for the half-space it
//            holds K[sigma], kept as it is).
//                                                -> out[o][z][y][x] (FP64)
//
// W reuses the forward intermediate Y, free once the z pass has run:
// O nzo ny Hx <= F Hx nzo Py complex values.
#pragma once

#include "apply_impl.hpp"

namespace bemfft {

// ------------------------------------------------------------------ k_vol_x
// W: [nrows][hx] half spectra; out: [nrows][nx].  Two rows per pencil
// (inv_x_pair), times sign.
template <typename R, int PX>
__global__ __launch_bounds__((RowInvCfg<R, PX>::NT)) void k_vol_x(const cx<R> *__restrict__ W, const cx<R> *twx,
                                                                   int hx, int nx, int64_t nrows, double sign,
                                                                   double *__restrict__ out) {
    using Cfg = RowInvCfg<R, PX>;
    constexpr int TPP = Cfg::TPP, PS = Cfg::PS, PPB = Cfg::PPB, NT = Cfg::NT, E = PX / TPP;
    __shared__ cx<R> buf[PPB * PS];
    __shared__ cx<R> tw[PX];
    const int tid = threadIdx.x;
    for (int i = tid; i < PX; i += NT) tw[i] = twx[i];
    __syncthreads();  // twiddle table
    const int pen = tid / TPP, t = tid % TPP;
    const int64_t ra = ((int64_t)blockIdx.x * PPB + pen) * 2, rb = ra + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    cx<R> x[E];
    inv_x_pair<R, PX>(W + ra * hx, W + rb * hx, va, vb, buf + pen * PS, tw, t, x);
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {  // nx <= Px/2
        const int xg = t + e * TPP;
        if (xg < nx) {
            if (va) out[ra * nx + xg] = sign * (double)x[e].x;
            if (vb) out[rb * nx + xg] = sign * (double)x[e].y;
        }
    }
}

// ------------------------------------------------------------------ launcher
template <typename R, int KIND>
struct VolumeLaunch {
    template <int P> static int x(const ApplyArgs &a, double *out, hipStream_t st) {
        using Cfg = RowInvCfg<R, P>;
        const int64_t nrows = (int64_t)Terms<KIND>::O * a.nzo * a.ny;
        const int64_t nb = (nrows + 2 * Cfg::PPB - 1) / (2 * Cfg::PPB);
        hipLaunchKernelGGL((k_vol_x<R, P>), dim3((unsigned)nb), dim3(Cfg::NT), 0, st,
                           static_cast<const cx<R> *>(a.Y), static_cast<const cx<R> *>(a.twx), a.hx, a.nx, nrows,
                           KIND == 3 ? 1.0 : -1.0, out);
        BF_HIP(hipGetLastError());
        return 0;
    }
    static int dispatch_x(const ApplyArgs &a, double *out, hipStream_t st) {
        BF_SIZE_SWITCH_K(KIND, a.px, x, a, out, st);
        set_error("unsupported x length");
        return BEMFFT_EUNSUPPORTED;
    }
    // ev (optional): four events recorded around the three stages (front,
    // inverse y, inverse x).
    static int run(const ApplyArgs &a, double *out, hipStream_t st, hipEvent_t *ev) {
        if (ev) BF_HIP(hipEventRecord(ev[0], st));
        BF_CHECK((Launch<R, KIND>::front(a, st, nullptr)));
        if (ev) BF_HIP(hipEventRecord(ev[1], st));
        BF_CHECK((Launch<R, KIND>::dispatch_inv_y(a, 1, st)));
        if (ev) BF_HIP(hipEventRecord(ev[2], st));
        BF_CHECK(dispatch_x(a, out, st));
        if (ev) BF_HIP(hipEventRecord(ev[3], st));
        return 0;
    }
};

// Per-family entry point, instantiated beside apply_kind.
template <int KIND>
int volume_kind(int precision, const ApplyArgs &a, double *out, hipStream_t st, hipEvent_t *ev);

}  // namespace bemfft
