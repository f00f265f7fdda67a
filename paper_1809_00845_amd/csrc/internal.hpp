// internal.hpp -- plan layout and launchers shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bemfft.h"

namespace bemfft {

// Thread-local error message (bemfft_last_error).
void set_error(const std::string &msg);

#define BF_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::bemfft::set_error(std::string(#call) + ": " + hipGetErrorString(e_));  \
            return BEMFFT_EDEVICE;                                                    \
        }                                                                             \
    } while (0)

#define BF_CHECK(st)                \
    do {                            \
        int s_ = (st);              \
        if (s_ < 0) return s_;      \
    } while (0)

// Fields, spectra and outputs of each kernel family (the integrals of
// eqs. 14-15 for Laplace; eq. 8 written with Kelvin's tensors for Navier).
//   Laplace 2D: fields q w, u n_x w, u n_y w; spectra u*, d_x u*, d_y u*.
//   Laplace 3D: fields q w, u n_i w (3);      spectra u*, d_i u* (3).
//   Navier:     fields t_j w (3), s_(ij) w (6, symmetric u (x) n);
//               spectra U_(kj) (6), Sigma_k,(ij) (18).
//   Half-space: fields sigma_b w (3); spectra K_xx, K_yy, K_xy, K_zz, K_xz,
//               K_yz, K_zx, K_zy (Boussinesq-Cerruti, eq. 9).
struct KindInfo {
    int dim, ncomp, F, K, O;
};
inline KindInfo kind_info(int kernel) {
    switch (kernel) {
        case BEMFFT_LAPLACE2D: return {2, 1, 3, 3, 1};
        case BEMFFT_LAPLACE3D: return {3, 1, 4, 4, 1};
        case BEMFFT_HALFSPACE: return {2, 3, 3, 8, 3};
        default: return {3, 3, 9, 24, 3};
    }
}

// Device state of one working precision.
struct Engine {
    int precision = BEMFFT_FP64;  // BEMFFT_FP64, BEMFFT_FP32 or BEMFFT_BF16_MFMA
    size_t creal = 8;             // bytes per real of the arithmetic (twiddles, fields, rows)
    size_t sreal = 8;             // bytes per real of the stored Y, Z and spectra
    int64_t hzs = 1;              // stored length of a spectrum's kz row (>= Hz)
    void *spec = nullptr;         // [K][Hx][Hy][hzs] reals (sreal bytes each)
    void *twx = nullptr;          // [Px] complex, exp(-2 pi i t / Px)
    void *twy = nullptr;          // [Py]
    void *twz = nullptr;          // [Pz]
    void *Y = nullptr;            // [F][Hx][nzo][Py] complex
    void *Z = nullptr;            // [O][Hx][nzo][Py] complex
    void *vf = nullptr;           // [F][m] sorted boundary fields
    void *Xd = nullptr;           // [nd][F][Hx] transforms of the long rows
    size_t bytes = 0;
};

}  // namespace bemfft

struct bemfft_plan {
    int dim = 0, kernel = 0, cmode = 0;
    int ncomp = 1, F = 0, K = 0, O = 0;
    int64_t m = 0;
    int64_t n[3] = {1, 1, 1};
    int64_t P[3] = {1, 1, 1};
    int64_t H[3] = {1, 1, 1};
    int64_t z0 = 0, nzo = 1;
    int *d_row_dense = nullptr;   // [nzo * ny] long-row index or -1
    int *d_dense_rows = nullptr;  // [nd]
    int64_t nd = 0;               // rows whose x-transform is an FFT
    int row_inv = 0;              // their inverse x transform is an FFT too
    int fwd_xg = 1;               // kx per thread in the forward direct DFT
    double h = 0.0, nu = 0.0, mu = 0.0;
    double origin[3] = {0, 0, 0};
    // node arrays in sorted order (z, y, x)
    int *d_gx = nullptr, *d_gy = nullptr, *d_gz = nullptr;
    int *d_perm = nullptr;     // sorted slot -> caller's node index
    int *d_rowptr = nullptr;   // [nzo * ny + 1] start of each (z, y) row
    double *d_w = nullptr;     // [m]
    double *d_nrm = nullptr;   // [3][m]
    double *d_C = nullptr;     // [m][O][O] free term
    double *d_SC = nullptr;    // [m][O][O] self-term correction (exact - grid)
    bemfft::Engine eng;        // working precision
    bemfft::Engine eng64;      // FP64 operator kept for refinement (if not the working one)
    bool has64 = false;        // an FP64 operator is available (eng or eng64)
    std::vector<double> h_c;   // c values in caller order (m or 9 m)
    std::vector<double> h_diag_dir, h_diag_neu;  // Jacobi entries per slot
    std::vector<double> h_self;  // exact single-layer self blocks, caller order (m or 9 m)
    double parity_resid = 0.0;
    int zsched = 0;               // radix schedule of the z transform
    int cell_quad = 0;            // kernel values at m != 0: 0 point, q >= 2 cell mean (q^dim points)
    double tune_us[3] = {0, 0, 0};
    double fwd_tune_us[2] = {0, 0};  // autotune: apply time with 1 and 2 kx per forward thread, us
    double plan_seconds = 0.0;
    // solve workspace, allocated on first use
    double *s_V = nullptr;
    int s_cap = 0;
    double *s_vec = nullptr;   // misc vectors
    double *s_red = nullptr;   // reduction scratch
    double *s_hbuf = nullptr;  // device copy of Hessenberg column / coefficients
    double *h_pinned = nullptr;
    uint64_t s_seq = 0;        // last step number handed to a GMRES completion flag
};

namespace bemfft {

// Apply-stage launchers (apply.hip).
int launch_apply(bemfft_plan *p, const Engine &e, const double *q, const double *u, double *r,
                 hipStream_t st, hipEvent_t *ev = nullptr);
// Spectrum precompute (spectra.hip): fills e64 (FP64) and, if e32 is
// non-null, its rounded FP32 copy.
int build_spectra(bemfft_plan *p, Engine *e64, Engine *e32, hipStream_t st);
int convert_spectra(const double *in, Engine *e, int64_t rows, int64_t hz, hipStream_t st);
int fft3d_c2c_f64(double *data, int64_t px, int64_t py, int64_t pz, int dir, hipStream_t st);
bool fft_size_supported(int64_t n);
int upload_twiddles(Engine *e, const bemfft_plan *p);
int alloc_workspace(bemfft_plan *p, Engine *e);
void free_engine(Engine *e);

}  // namespace bemfft
