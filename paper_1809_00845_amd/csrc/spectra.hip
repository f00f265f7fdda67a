// spectra.hip -- kernel sampling on the padded grid and its FP64 transform.
//
// Sec. 4 (Fig. 5) discretises the kernel functions coarsely, as constant
// values per element, over the whole zero-padded space that the FFT acts
// on.  Reading used here: the kernel
// is point-sampled at every padded-grid offset m (m_a in [-P_a/2, P_a/2)),
// with the flat-panel value at m = 0 for the single layer (0 for the odd
// double-layer kernels) and 0 on the planes m_a = -P_a/2, which no pair of
// nodes reaches and whose zeroing keeps odd kernels exactly odd.  As a plan
// option the values at m != 0 are instead the kernel's mean over the grid
// cell centred on h m (the constant element taken literally), by a tensor
// Gauss-Legendre rule; m = 0 and the zero planes are unchanged.  The
// transform is FP64 always; one octant of the real (or imaginary) spectrum is
// kept, because each kernel is even or odd along every axis.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "fft_device.hpp"
#include "internal.hpp"
#include "kinds.hpp"

namespace bemfft {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Kernel component c of family 'kernel' at offset xi (physical units), FP64.
__device__ double kernel_value(int kernel, int c, double x, double y, double z, double nu, double mu) {
    double r2 = x * x + y * y + z * z;
    double r = sqrt(r2);
    if (kernel == BEMFFT_LAPLACE2D) {
        if (c == 0) return -log(r) / (2.0 * kPi);         // eq. (3)
        double a = (c == 1) ? x : y;
        return -a / (2.0 * kPi * r2);                      // eq. (12), gradient of u*
    }
    if (kernel == BEMFFT_LAPLACE3D) {
        if (c == 0) return 1.0 / (4.0 * kPi * r);
        double a = (c == 1) ? x : ((c == 2) ? y : z);
        return -a / (4.0 * kPi * r2 * r);
    }
    if (kernel == BEMFFT_HALFSPACE) {
        // surface displacement a at offset (x, y) from a unit surface point
        // load b (Boussinesq for b = z, Cerruti for b = x, y), z into the solid
        const double g = 1.0 / (2.0 * kPi * mu);
        switch (c) {
            case 0: return g * ((1.0 - nu) / r + nu * x * x / (r2 * r));  // xx
            case 1: return g * ((1.0 - nu) / r + nu * y * y / (r2 * r));  // yy
            case 2: return g * nu * x * y / (r2 * r);                     // xy
            case 3: return g * (1.0 - nu) / r;                            // zz
            case 4: return -g * 0.5 * (1.0 - 2.0 * nu) * x / r2;          // xz
            case 5: return -g * 0.5 * (1.0 - 2.0 * nu) * y / r2;          // yz
            case 6: return g * 0.5 * (1.0 - 2.0 * nu) * x / r2;           // zx
            default: return g * 0.5 * (1.0 - 2.0 * nu) * y / r2;          // zy
        }
    }
    double xi[3] = {x, y, z};
    if (c < 6) {  // Kelvin displacement tensor, eq. (7)
        int k = pair_i(c), j = pair_j(c);
        double v = xi[k] * xi[j] / (r2 * r);
        if (k == j) v += (3.0 - 4.0 * nu) / r;
        return v / (16.0 * kPi * mu * (1.0 - nu));
    }
    // Kelvin stress tensor: the stress of the fundamental displacement
    int k = (c - 6) / 6, p = (c - 6) % 6;
    int i = pair_i(p), j = pair_j(p);
    double e[3] = {x / r, y / r, z / r};
    double a = 1.0 - 2.0 * nu;
    double v = a * ((k == i ? e[j] : 0.0) + (k == j ? e[i] : 0.0) - (i == j ? e[k] : 0.0)) + 3.0 * e[i] * e[j] * e[k];
    return -v / (8.0 * kPi * (1.0 - nu) * r2);
}

// Grid value at offset 0: flat-panel integral over the reference measure
// h^(d-1), per unit measure.  Navier: panel orientation averaged (<n n> = I/3).
double kernel_k0(int kernel, int c, double h, double nu, double mu) {
    const double l = std::log(1.0 + std::sqrt(2.0));
    if (kernel == BEMFFT_LAPLACE2D) return c == 0 ? (1.0 - std::log(0.5 * h)) / (2.0 * kPi) : 0.0;
    if (kernel == BEMFFT_LAPLACE3D) return c == 0 ? l / (kPi * h) : 0.0;
    if (kernel == BEMFFT_HALFSPACE) {
        // mean over the h x h cell: <1/r> = 4 ln(1 + sqrt 2) / h, <x^2/r^3> = <1/r> / 2
        const double a0 = 4.0 * l / h / (2.0 * kPi * mu);
        if (c == 0 || c == 1) return a0 * (1.0 - 0.5 * nu);
        if (c == 3) return a0 * (1.0 - nu);
        return 0.0;
    }
    if (c < 3) return (4.0 * l / h) * ((3.0 - 4.0 * nu) + 1.0 / 3.0) / (16.0 * kPi * mu * (1.0 - nu));
    return 0.0;
}

// Gauss-Legendre rule on [-1/2, 1/2] with weights summing to 1 (q points;
// q <= 1: the midpoint, i.e. point sampling).
struct CellRule {
    int q;
    double x[8];
    double w[8];
};

// Nodes by Newton's method on the Legendre polynomial P_q (three-term
// recurrence), started from the asymptotic guesses cos(pi (i + 3/4) / (q + 1/2)).
CellRule gauss_legendre_cell(int q) {
    CellRule r{};
    if (q <= 1) {
        r.q = 1;
        r.x[0] = 0.0;
        r.w[0] = 1.0;
        return r;
    }
    r.q = q;
    for (int i = 0; i < q; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        r.x[i] = 0.5 * t;
        r.w[i] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2 / ((1 - t^2) P_q'(t)^2), halved
    }
    return r;
}

__global__ void k_sample(cx<double> *out, int64_t px, int64_t py, int64_t pz, int kernel, int c,
                         double h, double nu, double mu, double k0, double scale, CellRule rule, int dim) {
    int64_t total = px * py * pz;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t ix = idx % px, iy = (idx / px) % py, iz = idx / (px * py);
        bool nyq = (px > 1 && 2 * ix == px) || (py > 1 && 2 * iy == py) || (pz > 1 && 2 * iz == pz);
        int64_t mx = (2 * ix < px) ? ix : ix - px;
        int64_t my = (2 * iy < py) ? iy : iy - py;
        int64_t mz = (2 * iz < pz) ? iz : iz - pz;
        double v;
        if (nyq) v = 0.0;
        else if (mx == 0 && my == 0 && mz == 0) v = k0;
        else if (rule.q <= 1) v = kernel_value(kernel, c, h * (double)mx, h * (double)my, h * (double)mz, nu, mu);
        else {
            // mean over the cell around h m
            const int qz = dim == 3 ? rule.q : 1;
            v = 0.0;
            for (int a = 0; a < rule.q; ++a)
                for (int b = 0; b < rule.q; ++b) {
                    double s = 0.0;
                    for (int e = 0; e < qz; ++e) {
                        const double z = dim == 3 ? h * ((double)mz + rule.x[e]) : 0.0;
                        const double we = dim == 3 ? rule.w[e] : 1.0;
                        s += we * kernel_value(kernel, c, h * ((double)mx + rule.x[a]), h * ((double)my + rule.x[b]),
                                               z, nu, mu);
                    }
                    v += rule.w[a] * rule.w[b] * s;
                }
        }
        out[idx] = {scale * v, 0.0};
    }
}

// Pencils per block of the FP64 axis pass: at most 16, 256 threads and 64 KB of LDS.
template <int P>
constexpr int axis_batch() {
    int b = 16;
    if (256 / PencilShape<P>::TPP < b) b = 256 / PencilShape<P>::TPP;
    int lds = (64 * 1024 - P * 16) / (pstride<P>() * 16);
    if (lds < b) b = lds;
    return b < 1 ? 1 : b;
}

// Batched FFT along one axis of a [pz][py][px] complex FP64 array.  A block
// takes B pencils adjacent in memory along the fastest other axis, so that
// global loads and stores are coalesced; the pencils are transformed in LDS.
template <int P, int DIR>
__global__ void k_fft_axis(cx<double> *data, int axis, int64_t px, int64_t py, int64_t pz) {
    using S = PencilShape<P>;
    constexpr int B = axis_batch<P>();
    constexpr int NT = B * S::TPP;
    constexpr int PS = pstride<P>();
    __shared__ cx<double> buf[B * PS];
    __shared__ cx<double> tw[P];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += NT) {
        ctrig::CS w = ctrig::cs2pi(i, P);  // exact quadrant reduction
        tw[i] = {w.c, -w.s};
    }
    int64_t npen, stride;
    if (axis == 0) { npen = py * pz; stride = 1; }
    else if (axis == 1) { npen = px * pz; stride = px; }
    else { npen = px * py; stride = px * py; }
    const int64_t pid0 = (int64_t)blockIdx.x * B;
    auto base_of = [&](int64_t pid) -> int64_t {
        if (axis == 0) return pid * px;
        if (axis == 1) return (pid / px) * py * px + (pid % px);
        return pid;  // (y * px + x)
    };
    for (int i = tid; i < B * P; i += NT) {
        int b, e;
        if (axis == 0) { b = i / P; e = i % P; } else { e = i / B; b = i % B; }
        int64_t pid = pid0 + b;
        buf[b * PS + pslot(e)] = (pid < npen) ? data[base_of(pid) + e * stride] : cx<double>{0.0, 0.0};
    }
    __syncthreads();
    pencil_fft<double, P, DIR>(buf + (tid / S::TPP) * PS, tw, tid % S::TPP);
    __syncthreads();
    for (int i = tid; i < B * P; i += NT) {
        int b, e;
        if (axis == 0) { b = i / P; e = i % P; } else { e = i / B; b = i % B; }
        int64_t pid = pid0 + b;
        if (pid < npen) data[base_of(pid) + e * stride] = buf[b * PS + pslot(e)];
    }
}

template <int P>
int launch_axis(cx<double> *d, int axis, int64_t px, int64_t py, int64_t pz, int dir, hipStream_t st) {
    using S = PencilShape<P>;
    constexpr int B = axis_batch<P>();
    int64_t npen = (axis == 0) ? py * pz : (axis == 1 ? px * pz : px * py);
    dim3 grid((unsigned)((npen + B - 1) / B)), block(B * S::TPP);
    if (dir < 0) hipLaunchKernelGGL((k_fft_axis<P, -1>), grid, block, 0, st, d, axis, px, py, pz);
    else hipLaunchKernelGGL((k_fft_axis<P, 1>), grid, block, 0, st, d, axis, px, py, pz);
    BF_HIP(hipGetLastError());
    return 0;
}

int axis_pass(cx<double> *d, int axis, int64_t len, int64_t px, int64_t py, int64_t pz, int dir, hipStream_t st) {
    switch (len) {
        case 1: return 0;
        case 32: return launch_axis<32>(d, axis, px, py, pz, dir, st);
        case 64: return launch_axis<64>(d, axis, px, py, pz, dir, st);
        case 96: return launch_axis<96>(d, axis, px, py, pz, dir, st);
        case 128: return launch_axis<128>(d, axis, px, py, pz, dir, st);
        case 192: return launch_axis<192>(d, axis, px, py, pz, dir, st);
        case 256: return launch_axis<256>(d, axis, px, py, pz, dir, st);
        case 320: return launch_axis<320>(d, axis, px, py, pz, dir, st);
        case 384: return launch_axis<384>(d, axis, px, py, pz, dir, st);
        case 512: return launch_axis<512>(d, axis, px, py, pz, dir, st);
        case 1024: return launch_axis<1024>(d, axis, px, py, pz, dir, st);
        default:
            set_error("FFT length " + std::to_string(len) + " is not supported");
            return BEMFFT_EUNSUPPORTED;
    }
}

// Positive doubles order like their bit patterns: max via 64-bit atomics.
__device__ void atomic_max_pos(unsigned long long *dst, double v) {
    atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

// One octant of the real (or imaginary) part: out[kx][ky][kz] from
// full[kz][ky][kx], through a 32 x 32 (kz, kx) LDS tile per block so that the
// reads run along kx and the writes along kz.  The largest kept and
// discarded magnitudes are reduced in the block and merged with one atomic
// per block.  Grid: (ceil(hx/32), ceil(hz/32), hy), 256 threads.
__global__ __launch_bounds__(256) void k_extract(const cx<double> *full, double *out, int64_t px, int64_t py,
                                                 int64_t hx, int64_t hy, int64_t hz, int imag,
                                                 unsigned long long *stats) {
    __shared__ double tile[32][33];
    __shared__ double red[2][4];
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    const int64_t kx0 = (int64_t)blockIdx.x * 32, kz0 = (int64_t)blockIdx.y * 32, ky = blockIdx.z;
    double kept = 0.0, disc = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t kz = kz0 + ty + 8 * i, kx = kx0 + tx;
        double a = 0.0;
        if (kz < hz && kx < hx) {
            const cx<double> v = full[(kz * py + ky) * px + kx];
            a = imag ? v.y : v.x;
            kept = fmax(kept, fabs(a));
            disc = fmax(disc, fabs(imag ? v.x : v.y));
        }
        tile[ty + 8 * i][tx] = a;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t kx = kx0 + ty + 8 * i, kz = kz0 + tx;
        if (kx < hx && kz < hz) out[(kx * hy + ky) * hz + kz] = tile[tx][ty + 8 * i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        kept = fmax(kept, __shfl_xor(kept, off, 64));
        disc = fmax(disc, __shfl_xor(disc, off, 64));
    }
    if (threadIdx.x % 64 == 0) {
        red[0][threadIdx.x / 64] = kept;
        red[1][threadIdx.x / 64] = disc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomic_max_pos(stats + 0, fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3])));
        atomic_max_pos(stats + 1, fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3])));
    }
}

__global__ void k_to_f32(const double *in, float *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// BF16 bit pattern of v: rounded to FP32, then to 8 significant bits, round
// to nearest, ties to even (v finite).  Rows of hz values are stored at a
// stride of hzs (>= hz), zero beyond hz.
__global__ void k_to_bf16_rows(const double *in, uint16_t *out, int64_t rows, int64_t hz, int64_t hzs) {
    const int64_t n = rows * hzs;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / hzs, k = i % hzs;
        uint16_t b = 0;
        if (k < hz) {
            unsigned u = __float_as_uint((float)in[r * hz + k]);
            u += 0x7fffu + ((u >> 16) & 1u);
            b = (uint16_t)(u >> 16);
        }
        out[i] = b;
    }
}

}  // namespace

bool fft_size_supported(int64_t n) {
    switch (n) {
        case 1: case 32: case 64: case 96: case 128: case 192: case 256: case 320: case 384: case 512: case 1024:
            return true;
        default:
            return false;
    }
}

int fft3d_c2c_f64(double *data, int64_t px, int64_t py, int64_t pz, int dir, hipStream_t st) {
    if (!fft_size_supported(px) || !fft_size_supported(py) || !fft_size_supported(pz)) {
        set_error("fft3d: unsupported length");
        return BEMFFT_EUNSUPPORTED;
    }
    cx<double> *d = reinterpret_cast<cx<double> *>(data);
    BF_CHECK(axis_pass(d, 0, px, px, py, pz, dir, st));
    BF_CHECK(axis_pass(d, 1, py, px, py, pz, dir, st));
    BF_CHECK(axis_pass(d, 2, pz, px, py, pz, dir, st));
    return 0;
}

// The FP64 spectra rounded once to the working engine's stored precision,
// on the device: FP32 contiguous, or BF16 rows of hz values at stride hzs.
int convert_spectra(const double *in, Engine *e, int64_t rows, int64_t hz, hipStream_t st) {
    const int64_t n = rows * (e->precision == BEMFFT_BF16_MFMA ? e->hzs : hz);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    if (e->precision == BEMFFT_FP32)
        hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, st, in, static_cast<float *>(e->spec), n);
    else
        hipLaunchKernelGGL(k_to_bf16_rows, dim3(blocks), dim3(256), 0, st, in, static_cast<uint16_t *>(e->spec), rows,
                           hz, e->hzs);
    if (hipGetLastError() != hipSuccess) {
        set_error("spectrum conversion failed");
        return BEMFFT_EDEVICE;
    }
    return 0;
}

int build_spectra(bemfft_plan *p, Engine *e64, Engine *e32, hipStream_t st) {
    const int64_t px = p->P[0], py = p->P[1], pz = p->P[2];
    const int64_t hx = p->H[0], hy = p->H[1], hz = p->H[2];
    const int64_t full_n = px * py * pz;
    const int64_t oct = hx * hy * hz;
    cx<double> *full = nullptr;
    unsigned long long *stats = nullptr;
    BF_HIP(hipMalloc(&full, full_n * sizeof(cx<double>)));
    if (hipMalloc(&stats, 2 * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipFree(full);
        set_error("hipMalloc(stats) failed");
        return BEMFFT_ENOMEM;
    }
    double worst = 0.0;
    int status = 0;
    const double scale = (p->kernel == BEMFFT_HALFSPACE ? 1.0 : -1.0) / (double)full_n;
    const CellRule rule = gauss_legendre_cell(p->cell_quad);
    for (int c = 0; c < p->K && status == 0; ++c) {
        double k0 = kernel_k0(p->kernel, c, p->h, p->nu, p->mu);
        int blocks = (int)std::min<int64_t>((full_n + 255) / 256, 65536);
        hipLaunchKernelGGL(k_sample, dim3(blocks), dim3(256), 0, st, full, px, py, pz, p->kernel, c, p->h,
                           p->nu, p->mu, k0, scale, rule, p->dim);
        if (hipGetLastError() != hipSuccess) { status = BEMFFT_EDEVICE; break; }
        status = fft3d_c2c_f64(reinterpret_cast<double *>(full), px, py, pz, -1, st);
        if (status) break;
        if (hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), st) != hipSuccess) { status = BEMFFT_EDEVICE; break; }
        double *dst = static_cast<double *>(e64->spec) + (int64_t)c * oct;
        const dim3 eg((unsigned)((hx + 31) / 32), (unsigned)((hz + 31) / 32), (unsigned)hy);
        hipLaunchKernelGGL(k_extract, eg, dim3(256), 0, st, full, dst, px, py, hx, hy, hz,
                           comp_imag(p->kernel, c) ? 1 : 0, stats);
        unsigned long long hs[2];
        if (hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) { status = BEMFFT_EDEVICE; break; }
        double kept, disc;
        std::memcpy(&kept, &hs[0], 8);
        std::memcpy(&disc, &hs[1], 8);
        if (kept > 0.0) worst = std::max(worst, disc / kept);
    }
    if (status == 0 && e32) {
        int64_t n = (int64_t)p->K * oct;
        int eb = (int)std::min<int64_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(k_to_f32, dim3(eb), dim3(256), 0, st, static_cast<const double *>(e64->spec),
                           static_cast<float *>(e32->spec), n);
        if (hipGetLastError() != hipSuccess) status = BEMFFT_EDEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess && status == 0) status = BEMFFT_EDEVICE;
    (void)hipFree(full);
    (void)hipFree(stats);
    if (status == BEMFFT_EDEVICE) set_error("spectrum precompute: HIP failure");
    p->parity_resid = worst;
    return status;
}

}  // namespace bemfft
