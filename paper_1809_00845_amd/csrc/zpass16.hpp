// zpass16.hpp -- the 16-bit form of the apply (BEMFFT_BF16_MFMA).
//
// What is stored in 16 bits: the intermediates after the forward y transform
// (Y) and after the inverse z transform (Z), and the kernel spectra -- the
// arrays that carry almost all of the apply's HBM traffic.  Every transform
// accumulates in FP32 and the spectral products of eqs. (15)-(16) are FP32;
// the node fields, the x transforms, the gather and its epilogue are those of
// the FP32 path.
//
// The z pass runs its transforms on the matrix cores.  A z pencil of length
// P = 16 N2 (zero for z >= P/2 on input; only z < P/2 is kept on output) is
// transformed in two stages of dense DFT matrix products (the four-step
// factorisation n = N2 n1 + n2, k = k1 + 16 k2):
//
//   X[k1 + 16 k2] = sum_n2 W_N2^(n2 k2) W_P^(n2 k1) sum_n1 W_16^(n1 k1) x[N2 n1 + n2]
//   (W_N = exp(-2 pi i / N)), and the inverse in the mirrored order.
//
// Each stage is a 16 x 16 complex product done as two real
// v_mfma_f32_16x16x32_bf16 (K = 16 complex values = 32 reals, FP32
// accumulate).  Data tiles live in the accumulator ("D") layout: lane
// l = 16 g + c of a wavefront holds rows 4 g + r (r < 4) of column c.  The
// contraction index K of the next product is spread over lanes the same way
// (lane group g holds K entries 8 g .. 8 g + 7), so a D tile is directly the
// next product's A or B operand once its 4 complex values are packed as
// (re, im) pairs: used as B it keeps its columns and contracts over its rows;
// used as A its columns become the rows of the result.  Forward: stage 1 with
// the data as A (rows n1, columns n2 -> rows n2, columns k1), the twiddle
// W_P^(n2 k1), stage 2 with the data as B (-> rows k2, columns k1).
// Inverse: data as A (rows k2 -> rows k1, columns n2), twiddle, data as B
// (-> rows n1, columns n2): the output tile has the input's (n1, n2) layout.
// Short pencils (N2 < 16) share a tile side by side with block-diagonal
// second-stage matrices; long ones (N2 > 16) span two column tiles.
//
// A block owns PPB pencils of consecutive ky at one kx.  Rows of Y are read
// from HBM as 16-byte runs of 4 pencils into an LDS staging tile (one field
// at a time, the next field's loads in flight meanwhile), and each wavefront
// reads its pencils' tiles from there; outputs go back through the same kind
// of tile and leave as 16-byte runs.
#pragma once

#include "volume_impl.hpp"

namespace bemfft {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// One 16 x 16 complex tile in the accumulator layout.
struct MTile {
    f32x4 re, im;
};

__device__ __forceinline__ MTile mtile_zero() {
    MTile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        t.re[r] = 0.f;
        t.im[r] = 0.f;
    }
    return t;
}

// The lane's four complex values as an MFMA operand: K entry 8 g + e holds
// the real (e even) or imaginary (e odd) part of row 4 g + e / 2.
__device__ __forceinline__ bf16x8 mpack(const MTile &t) {
    bf16x8 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v[2 * r] = (__bf16)t.re[r];
        v[2 * r + 1] = (__bf16)t.im[r];
    }
    return v;
}

// Data as A (its columns become the result's rows), constant matrix as B.
__device__ __forceinline__ MTile mmul_da(bf16x8 d, const bf16x8 *bop, int lane, MTile acc) {
    MTile o;
    o.re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(d, bop[lane], acc.re, 0, 0, 0);
    o.im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(d, bop[64 + lane], acc.im, 0, 0, 0);
    return o;
}
// Constant matrix as A, data as B (columns kept).
__device__ __forceinline__ MTile mmul_db(const bf16x8 *aop, bf16x8 d, int lane, MTile acc) {
    MTile o;
    o.re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[lane], d, acc.re, 0, 0, 0);
    o.im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[64 + lane], d, acc.im, 0, 0, 0);
    return o;
}

template <int P, int KIND>
struct Z16Cfg {
    static constexpr int N2 = P / 16;
    static constexpr int CT = N2 > 16 ? 2 : 1;           // column tiles per pencil
    static constexpr int PPT = CT == 1 ? 16 / N2 : 1;    // pencils per tile
    static constexpr int O = Terms<KIND>::O;
    static constexpr int PPB = O == 1 ? 16 : 8;          // pencils per block
    static constexpr int UPB = (PPB + PPT - 1) / PPT;    // tile groups per block
    static constexpr int WAVES = 4, NT = 64 * WAVES;
    static constexpr int UPW = (UPB + WAVES - 1) / WAVES;
    static constexpr int NOPS = CT == 1 ? 4 : 10;        // constant operand matrices
    static constexpr int HALF = P / 2;                   // rows z < P/2
    static constexpr int LS = PPB + 1;                   // staging row stride (padded)
    static constexpr int QPR = PPB / 4;                  // 16-byte runs per row
    static constexpr int LMAX = (HALF * QPR + NT - 1) / NT;
    static constexpr int HZS = (P / 2 + 1 + 7) / 8 * 8;  // stored kz row of a spectrum
    static constexpr int NCF = max_field_ncomp<KIND>();  // spectra per field
    static constexpr int SRUNS = HZS / 8;                // 16-byte runs per spectrum row
    static constexpr int SMAX = (NCF * PPB * SRUNS + NT - 1) / NT;
    static_assert(N2 * 16 == P && PPB % 4 == 0, "length and block shape");
};

// Constant operand matrices, indexed by m:
//   0: F16 as B (forward stage 1), 1: conj F16 as A (inverse stage 2);
//   one tile per pencil group: 2: F_N2 block diagonal as A, 3: its conjugate as B;
//   two column tiles: 2 + 2 u + t: block (u, t) of F_N2 as A,
//                     6 + 2 u + t: block (u, t) of conj F_N2 as B.
// tw[t] = exp(-2 pi i t / P).  Returns the matrix entry at (row, col).
template <int P, int KIND>
__device__ __forceinline__ cx<float> zop_entry(int m, int row, int col, const cx<float> *tw) {
    using C = Z16Cfg<P, KIND>;
    constexpr int N2 = C::N2;
    const cx<float> zero{0.f, 0.f};
    auto w = [&](int e, bool cj) {
        cx<float> v = tw[e % P];
        if (cj) v.y = -v.y;
        return v;
    };
    if (m == 0) return w(N2 * row * col, false);
    if (m == 1) return w(N2 * row * col, true);
    if constexpr (C::CT == 1) {
        const int br = row / N2, bc = col / N2;
        if (br != bc || br >= C::PPT) return zero;
        return w(16 * (row % N2) * (col % N2), m == 3);
    } else {
        const bool cj = m >= 6;
        const int u = ((m - 2) % 4) / 2, t = (m - 2) % 2;
        const int a = 16 * u + row, b = 16 * t + col;  // k2 index (rows of F), n2 index
        if (a >= N2 || b >= N2) return zero;
        return w(16 * a * b, cj);
    }
}

template <int P, int KIND>
__device__ __forceinline__ void zop_fill(bf16x8 *ops, const cx<float> *tw) {
    using C = Z16Cfg<P, KIND>;
    for (int idx = threadIdx.x; idx < C::NOPS * 64; idx += C::NT) {
        const int m = idx / 64, l = idx % 64;
        // A operands: m = 1, 2 (one tile) or 2..5 (two tiles); B otherwise
        const bool is_a = (m == 1) || (C::CT == 1 ? m == 2 : (m >= 2 && m < 6));
        bf16x8 vre, vim;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int rho = 4 * (l / 16) + e / 2, other = l % 16;
            const cx<float> M = is_a ? zop_entry<P, KIND>(m, other, rho, tw) : zop_entry<P, KIND>(m, rho, other, tw);
            if ((e & 1) == 0) {
                vre[e] = (__bf16)M.x;
                vim[e] = (__bf16)M.y;
            } else {
                vre[e] = (__bf16)(-M.y);
                vim[e] = (__bf16)M.x;
            }
        }
        ops[(2 * m) * 64 + l] = vre;
        ops[(2 * m + 1) * 64 + l] = vim;
    }
}

__device__ __forceinline__ cx<float> cmul_f(cx<float> a, cx<float> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Per-lane element tables (built once per block): for element e = 4 t + r
// (tile t, row r of the lane) the forward twiddle after stage 1, the inverse
// twiddle after inverse stage 1, and the spectrum position of the forward
// result: kz reflected into the octant (bits 0-15), the pencil slot inside
// the tile (bits 16-23), "valid" (bit 29) and "kz in the upper half" as a
// sign bit (bit 31).
constexpr unsigned kKzValid = 1u << 29, kKzSign = 1u << 31;

template <int P, int KIND>
__device__ __forceinline__ void z16_tables(cx<float> *twf, cx<float> *twi, unsigned *kzo, const cx<float> *tw, int hz) {
    using C = Z16Cfg<P, KIND>;
    constexpr int N2 = C::N2, CT = C::CT, PPT = C::PPT, NE = 4 * C::CT;
    for (int idx = threadIdx.x; idx < NE * 64; idx += C::NT) {
        const int e = idx / 64, l = idx % 64, t = e / 4, r = e % 4;
        const int g = l / 16, c = l % 16, i = 4 * g + r;
        // forward: rows n2, column k1 = c
        const int n2f = CT == 1 ? i % N2 : 16 * t + i;
        twf[idx] = tw[(n2f * c) % P];
        // inverse: rows k1 = i, column n2
        const int n2i = CT == 1 ? c % N2 : 16 * t + c;
        cx<float> w = tw[(n2i * i) % P];
        w.y = -w.y;
        twi[idx] = w;
        // forward result: rows k2 (pencil slot s), column k1 = c
        // rows beyond the pencils of the tile hold zeros after stage 2; they
        // read the spectrum of the tile's first pencil at kz = 0 (in bounds,
        // multiplied by zero)
        const int s = CT == 1 ? i / N2 : 0;
        const int k2 = CT == 1 ? i % N2 : 16 * t + i;
        const bool ok = CT == 1 ? s < PPT : k2 < N2;
        const int kz = ok ? c + 16 * k2 : 0;
        const int kzp = kz < hz ? kz : P - kz;
        kzo[idx] = (unsigned)kzp | ((unsigned)(ok ? s : 0) << 16) | (ok ? kKzValid : 0u) | (kz >= hz ? kKzSign : 0u);
    }
}

__device__ __forceinline__ bf16x8 bf16x8_from_words(unsigned w0, unsigned w1, unsigned w2, unsigned w3) {
    union {
        unsigned u[4];
        bf16x8 v;
    } x;
    x.u[0] = w0;
    x.u[1] = w1;
    x.u[2] = w2;
    x.u[3] = w3;
    return x.v;
}

// Loads of field f into registers: its rows of Y for the block's pencils
// and the rows of the spectra that multiply it, all as 16-byte runs.
template <int P, int KIND>
__device__ __forceinline__ void z16_load_field(const int f, const ApplyArgs &a, const unsigned *Y,
                                               const uint16_t *spec, size_t fstride, int nrun, int kx, int ky0,
                                               u32x4 (&pre)[Z16Cfg<P, KIND>::LMAX],
                                               u32x4 (&spre)[Z16Cfg<P, KIND>::SMAX]) {
    using C = Z16Cfg<P, KIND>;
    constexpr int PPB = C::PPB, QPR = C::QPR, NT = C::NT;
    const int tid = threadIdx.x;
    const unsigned *Yf = Y + (size_t)f * fstride;
    // every lane loads (runs past the end repeat the last one) so that the
    // loads stay in flight in registers; only the LDS writes are conditional
#pragma unroll
    for (int k = 0; k < C::LMAX; ++k) {
        const int it = min(tid + k * NT, nrun - 1);
        const int zz = it / QPR, q = it % QPR;
        pre[k] = *reinterpret_cast<const u32x4 *>(Yf + (size_t)zz * a.py + 4 * q);
    }
    const int ncf = field_ncomp<KIND>(f);  // f is a constant once the field loop is unrolled
    static_assert(C::NCF <= 3, "at most three spectra per field");
#pragma unroll
    for (int k = 0; k < C::SMAX; ++k) {
        const int it = min(tid + k * NT, ncf * PPB * C::SRUNS - 1);
        const int slot = it / (PPB * C::SRUNS), pen = (it / C::SRUNS) % PPB, q = it % C::SRUNS;
        int comp = field_comp<KIND>(f, 0);
        if (ncf > 1) comp = slot == 1 ? field_comp<KIND>(f, 1) : comp;
        if (ncf > 2) comp = slot == 2 ? field_comp<KIND>(f, 2) : comp;
        const int ky = ky0 + pen;
        const int kyp = ky < a.hy ? ky : a.py - ky;
        spre[k] = *reinterpret_cast<const u32x4 *>(spec + ((size_t)(comp * a.hx + kx) * a.hy + kyp) * C::HZS + 8 * q);
    }
}

// One block: kx and PPB consecutive ky (ky0 = by * PPB).  One-dimensional
// grid with the XCD-aware order of k_zpass.
template <int P, int KIND>
__device__ __forceinline__ void zpass16_body(const ApplyArgs &a, const int kx, const int by) {
    using C = Z16Cfg<P, KIND>;
    using T = Terms<KIND>;
    constexpr int N2 = C::N2, CT = C::CT, PPT = C::PPT, O = C::O, F = T::F, NE = 4 * CT;
    constexpr int PPB = C::PPB, LS = C::LS, QPR = C::QPR, UPW = C::UPW, NT = C::NT, HALF = C::HALF;
    __shared__ unsigned stg[HALF * LS];  // complex BF16 values, one 32-bit word each
    __shared__ cx<float> tw[P];
    __shared__ bf16x8 ops[2 * C::NOPS * 64];
    __shared__ cx<float> twf[NE * 64], twi[NE * 64];
    __shared__ unsigned kzo[NE * 64];
    // the field's spectrum rows for the block's pencils: [slot][pencil][kz]
    __shared__ uint16_t sspec[C::NCF * PPB * C::HZS];
    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int g = lane / 16, c = lane % 16;
    const int ky0 = by * PPB;
    const cx<float> *twz = static_cast<const cx<float> *>(a.twz);
    for (int i = tid; i < P; i += NT) tw[i] = twz[i];
    for (int i = tid; i < HALF * LS; i += NT) {
        const int z = i / LS;
        if (z < a.z0 || z >= a.z0 + a.nzo) stg[i] = 0u;
    }
    __syncthreads();
    zop_fill<P, KIND>(ops, tw);
    z16_tables<P, KIND>(twf, twi, kzo, tw, a.hz);

    const size_t fstride = (size_t)a.hx * a.nzo * a.py;  // complex values per field
    const unsigned *Y = static_cast<const unsigned *>(a.Y) + (size_t)kx * a.nzo * a.py + ky0;
    const uint16_t *spec = static_cast<const uint16_t *>(a.spec);
    const int nrun = a.nzo * QPR;  // 16-byte runs of one field

    u32x4 pre[C::LMAX], spre[C::SMAX];
    z16_load_field<P, KIND>(0, a, Y, spec, fstride, nrun, kx, ky0, pre, spre);

    MTile acc[UPW][CT][O];
#pragma unroll
    for (int u = 0; u < UPW; ++u)
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int o = 0; o < O; ++o) acc[u][t][o] = mtile_zero();

    // stage-1 operand position of this lane: rows n1 = 4 g + r (g < 2; rows
    // n1 >= 8 are the zero padding), column n2 of pencil slot s.  Lanes
    // without a value read (and later write) the staging tile's pad column.
    const int s1 = CT == 1 ? c / N2 : 0;
    const bool in_ok1 = g < 2 && (CT == 1 ? s1 < PPT : true);
    auto stg_at = [&](int unit, int n2, bool ok) -> unsigned * {
        return ok ? stg + (size_t)(N2 * 4 * g + n2) * LS + unit * PPT + s1 : stg + PPB;
    };

#pragma unroll
    for (int f = 0; f < F; ++f) {
        __syncthreads();  // the previous field's tiles have been read
#pragma unroll
        for (int k = 0; k < C::LMAX; ++k) {
            const int it = tid + k * NT;
            if (it < nrun) {
                const int zz = it / QPR, q = it % QPR;
                unsigned *row = stg + (size_t)(a.z0 + zz) * LS + 4 * q;
                row[0] = pre[k][0];
                row[1] = pre[k][1];
                row[2] = pre[k][2];
                row[3] = pre[k][3];
            }
        }
#pragma unroll
        for (int k = 0; k < C::SMAX; ++k) {
            const int it = tid + k * NT;
            if (it < field_ncomp<KIND>(f) * PPB * C::SRUNS)
                *reinterpret_cast<u32x4 *>(sspec + 8 * it) = spre[k];  // [slot][pencil][kz] in run order
        }
        __syncthreads();
        if (f + 1 < F)  // in flight during the transforms
            z16_load_field<P, KIND>(f + 1, a, Y, spec, fstride, nrun, kx, ky0, pre, spre);
#pragma unroll
        for (int u = 0; u < UPW; ++u) {
            const int unit = u * C::WAVES + wave;
            if (unit >= C::UPB) continue;  // wave-uniform
            // stage 1 (data as A)
            bf16x8 b1[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int n2 = CT == 1 ? c % N2 : 16 * t + c;
                const bool ok = in_ok1 && (CT == 1 || n2 < N2);
                const unsigned *src = stg_at(unit, n2, ok);
                unsigned w[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) w[r] = ok ? src[r * N2 * LS] : 0u;
                MTile s1t = mmul_da(bf16x8_from_words(w[0], w[1], w[2], w[3]), ops + 0 * 128, lane, mtile_zero());
#pragma unroll
                for (int r = 0; r < 4; ++r) {  // twiddle W_P^(n2 k1)
                    const cx<float> v = cmul_f({s1t.re[r], s1t.im[r]}, twf[(4 * t + r) * 64 + lane]);
                    s1t.re[r] = v.x;
                    s1t.im[r] = v.y;
                }
                b1[t] = mpack(s1t);
            }
            // stage 2 (data as B): rows k2, columns k1
            MTile X[CT];
            if constexpr (CT == 1) {
                X[0] = mmul_db(ops + 2 * 128, b1[0], lane, mtile_zero());
            } else {
#pragma unroll
                for (int u2 = 0; u2 < 2; ++u2) {
                    X[u2] = mmul_db(ops + (2 + 2 * u2) * 128, b1[0], lane, mtile_zero());
                    X[u2] = mmul_db(ops + (3 + 2 * u2) * 128, b1[1], lane, X[u2]);
                }
            }
            // spectral products at kz = k1 + 16 k2 of pencil ky: the octant
            // store is read at the reflected index, with the sign of each odd axis
            const int kyu = ky0 + unit * PPT;
#pragma unroll
            for (int t2 = 0; t2 < CT; ++t2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned kd = kzo[(4 * t2 + r) * 64 + lane];
                    const int pen = unit * PPT + (PPT == 1 ? 0 : (int)((kd >> 16) & 0xffu));
                    const bool fy = ky0 + pen >= a.hy;
                    const unsigned zs = kd & kKzSign, ys = fy ? kKzSign : 0u;
                    const uint16_t *srow = sspec + pen * C::HZS + (kd & 0xffffu);
                    const float xr = X[t2].re[r], xi = X[t2].im[r];
                    static_for<0, T::N>([&](auto tc) {
                        constexpr int term = decltype(tc)::value;
                        if (T::f(term) == f) {
                            constexpr int comp = T::c(term);
                            constexpr int mask = comp_oddmask(KIND, comp);
                            unsigned bits = (unsigned)srow[term_slot<KIND>(term) * PPB * C::HZS] << 16;
                            if constexpr (mask & 4) bits ^= zs;
                            if constexpr (mask & 2) bits ^= ys;
                            const float sv = __uint_as_float(bits);
                            MTile &A = acc[u][t2][T::o(term)];
                            if constexpr (comp_imag(KIND, comp)) {  // (i s) x
                                A.re[r] -= sv * xi;
                                A.im[r] += sv * xr;
                            } else {
                                A.re[r] += sv * xr;
                                A.im[r] += sv * xi;
                            }
                        }
                    });
                }
            }
        }
    }

    // inverse transforms, one output at a time through the staging tile
    unsigned *Z = static_cast<unsigned *>(a.Z) + (size_t)kx * a.nzo * a.py + ky0;
#pragma unroll
    for (int o = 0; o < O; ++o) {
        __syncthreads();  // staging free (last field read / previous output stored)
#pragma unroll
        for (int u = 0; u < UPW; ++u) {
            const int unit = u * C::WAVES + wave;
            if (unit >= C::UPB) continue;
            bf16x8 xa[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) xa[t] = mpack(acc[u][t][o]);
#pragma unroll
            for (int tp = 0; tp < CT; ++tp) {
                // stage 1 (data as A): rows k1, columns n2
                MTile y;
                if constexpr (CT == 1) {
                    y = mmul_da(xa[0], ops + 3 * 128, lane, mtile_zero());
                } else {
                    y = mmul_da(xa[0], ops + (6 + tp) * 128, lane, mtile_zero());
                    y = mmul_da(xa[1], ops + (8 + tp) * 128, lane, y);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {  // twiddle W_P^(-n2 k1)
                    const cx<float> v = cmul_f({y.re[r], y.im[r]}, twi[(4 * tp + r) * 64 + lane]);
                    y.re[r] = v.x;
                    y.im[r] = v.y;
                }
                // stage 2 (data as B): rows n1, columns n2 -> z = N2 n1 + n2
                const MTile zt = mmul_db(ops + 1 * 128, mpack(y), lane, mtile_zero());
                const int n2 = CT == 1 ? c % N2 : 16 * tp + c;
                unsigned *dst = stg_at(unit, n2, in_ok1 && (CT == 1 || n2 < N2));  // z < P/2
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const cbf16 v{(__bf16)zt.re[r], (__bf16)zt.im[r]};
                    dst[r * N2 * LS] = *reinterpret_cast<const unsigned *>(&v);
                }
            }
        }
        __syncthreads();
        unsigned *Zo = Z + (size_t)o * fstride;
        for (int it = tid; it < nrun; it += NT) {
            const int zz = it / QPR, q = it % QPR;
            const unsigned *row = stg + (size_t)(a.z0 + zz) * LS + 4 * q;
            u32x4 v;
            v[0] = row[0];
            v[1] = row[1];
            v[2] = row[2];
            v[3] = row[3];
            *reinterpret_cast<u32x4 *>(Zo + (size_t)zz * a.py + 4 * q) = v;
        }
    }
}

template <int P, int KIND>
__global__ __launch_bounds__(256) void k_zpass16(ApplyArgs a, int nby) {
    const int total = a.hx * nby;
    const int per = (total + 7) / 8;
    const int lam = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (lam >= total) return;
    const int kx = lam / nby, j = lam % nby;
    const int by = (j & 1) ? nby - 1 - (j >> 1) : (j >> 1);
    zpass16_body<P, KIND>(a, kx, by);
}

template <int P, int KIND>
int launch_z16(const ApplyArgs &a, hipStream_t st) {
    using C = Z16Cfg<P, KIND>;
    if (a.py % C::PPB != 0 || a.hzs != C::HZS) {
        set_error("16-bit z pass: y length not a multiple of the block's pencils, or unpadded spectra");
        return BEMFFT_EUNSUPPORTED;
    }
    const int nby = a.py / C::PPB;
    const int per = (a.hx * nby + 7) / 8;
    hipLaunchKernelGGL((k_zpass16<P, KIND>), dim3(8 * per), dim3(C::NT), 0, st, a, nby);
    BF_HIP(hipGetLastError());
    return 0;
}

// The 16-bit apply: the FP32 kernels with BF16 Y/Z storage around the
// matrix-core z pass.  2D plans have no z transform: their spectral product
// reads BF16 Y and spectra and writes BF16 Z.
template <int KIND>
struct Launch16 {
    using L = Launch<float, KIND>;
    template <int P> static int fwd(const ApplyArgs &a, hipStream_t st) {
        return launch_fwd<float, P, KIND, cbf16>(a, st);
    }
    template <int P> static int inv_y(const ApplyArgs &a, int all_rows, hipStream_t st) {
        return launch_inv_y<float, P, KIND, cbf16>(a, all_rows, st);
    }
    template <int P> static int z(const ApplyArgs &a, hipStream_t st) { return launch_z16<P, KIND>(a, st); }
    static int dispatch_fwd(const ApplyArgs &a, hipStream_t st) {
        BF_SIZE_SWITCH(a.py, fwd, a, st);
        set_error("unsupported y length");
        return BEMFFT_EUNSUPPORTED;
    }
    static int dispatch_inv_y(const ApplyArgs &a, int all_rows, hipStream_t st) {
        BF_SIZE_SWITCH(a.py, inv_y, a, all_rows, st);
        set_error("unsupported y length");
        return BEMFFT_EUNSUPPORTED;
    }
    static int dispatch_z(const ApplyArgs &a, hipStream_t st) {
        if constexpr (KIND == 0 || KIND == 3) {
            set_error("the 16-bit form needs a 3D plan");
            return BEMFFT_EUNSUPPORTED;
        } else {
            BF_SIZE_SWITCH(a.pz, z, a, st);
            set_error("unsupported z length");
            return BEMFFT_EUNSUPPORTED;
        }
    }
    static int front(const ApplyArgs &a, hipStream_t st, hipEvent_t *ev = nullptr) {
        if (ev) BF_HIP(hipEventRecord(ev[0], st));
        if (a.nd > 0) {
            BF_CHECK(L::dispatch_rows(a, st));
        } else {
            hipLaunchKernelGGL((k_fields<float, KIND>), dim3((a.m + 255) / 256), dim3(256), 0, st, a);
        }
        BF_CHECK(dispatch_fwd(a, st));
        if (ev) BF_HIP(hipEventRecord(ev[1], st));
        BF_CHECK(dispatch_z(a, st));
        if (ev) BF_HIP(hipEventRecord(ev[2], st));
        return 0;
    }
    static int run(const ApplyArgs &a, hipStream_t st, hipEvent_t *ev = nullptr) {
        BF_CHECK(front(a, st, ev));
        BF_CHECK(dispatch_inv_y(a, 0, st));
        if (ev) BF_HIP(hipEventRecord(ev[3], st));
        if (a.nd > 0 && a.row_inv) BF_CHECK(L::dispatch_rows_inv(a, st));
        constexpr int NPB = 256 / kGatherLanes;
        hipLaunchKernelGGL((k_gather<float, KIND>), dim3((a.m + NPB - 1) / NPB), dim3(256), 0, st, a);
        BF_HIP(hipGetLastError());
        if (ev) BF_HIP(hipEventRecord(ev[4], st));
        return 0;
    }
};

// The field over the grid box with the 16-bit passes (see volume_impl.hpp).
template <int KIND>
struct VolumeLaunch16 {
    static int run(const ApplyArgs &a, double *out, hipStream_t st, hipEvent_t *ev) {
        if (ev) BF_HIP(hipEventRecord(ev[0], st));
        BF_CHECK(Launch16<KIND>::front(a, st, nullptr));
        if (ev) BF_HIP(hipEventRecord(ev[1], st));
        BF_CHECK(Launch16<KIND>::dispatch_inv_y(a, 1, st));
        if (ev) BF_HIP(hipEventRecord(ev[2], st));
        BF_CHECK((VolumeLaunch<float, KIND>::dispatch_x(a, out, st)));
        if (ev) BF_HIP(hipEventRecord(ev[3], st));
        return 0;
    }
};

}  // namespace bemfft
