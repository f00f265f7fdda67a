// kinds.hpp -- kernel components, their parities and the spectral products.
//
// Sign convention.  With xi = field point - target, the integrals of eq. (4)
// are correlations; eq. (15) rewrites them as convolutions
//     (K * f)(x0) = sum_x K(x0 - x) f(x).
// An even kernel is unchanged by the rewrite, an odd one changes sign.  The
// grid part of r = c u + D[u] - S[q] is then
//   Laplace:  - u* * (q w) - sum_i d_i u* * (u n_i w)
//   Navier:   - sum_j U_kj * (t_j w) - sum_(ij) Sigma_k,(ij) * s_(ij)
// so every spectrum is stored with the factor -1 (and 1/(Px Py Pz)) folded in
// and each output is a plain sum of products.
//
// The elastic half-space (eq. 9) is a convolution already: the surface
// displacement is u_a = sum_b K_ab * (sigma_b w) with the Boussinesq-Cerruti
// tensor K; its spectra carry +1/(Px Py) and the plan's free term c = -1
// turns the apply into r = K[sigma] - u.
#pragma once

#include <hip/hip_runtime.h>

namespace bemfft {

// Symmetric index pairs (ij) of Kelvin's tensors, in storage order.
__host__ __device__ constexpr int pair_i(int p) { return p < 3 ? p : (p == 5 ? 1 : 0); }
__host__ __device__ constexpr int pair_j(int p) { return p < 3 ? p : (p == 3 ? 1 : 2); }
__host__ __device__ constexpr int pair_of(int i, int j) {
    return (i == j) ? i : ((i + j == 1) ? 3 : ((i + j == 2) ? 4 : 5));
}

// Bit a set <=> component c is odd along axis a.  The spectrum of a real
// kernel that is even/odd per axis is real when the number of odd axes is
// even and imaginary when it is odd; it keeps each axis' parity in k.
__host__ __device__ constexpr int comp_oddmask(int kernel, int c) {
    if (kernel == 3) {  // xx, yy, xy, zz, xz, yz, zx, zy
        constexpr int m[8] = {0, 0, 3, 0, 1, 2, 1, 2};
        return m[c];
    }
    if (kernel == 0) return c == 0 ? 0 : (1 << (c - 1));
    if (kernel == 1) return c == 0 ? 0 : (1 << (c - 1));
    if (c < 6) return (1 << pair_i(c)) ^ (1 << pair_j(c));
    int k = (c - 6) / 6, p = (c - 6) % 6;
    return (1 << k) ^ (1 << pair_i(p)) ^ (1 << pair_j(p));
}
__host__ __device__ constexpr bool comp_imag(int kernel, int c) {
    int m = comp_oddmask(kernel, c);
    return (((m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1)) & 1) != 0;
}

// Spectral product terms (field f, output o, component c).
template <int KIND>
struct Terms;

template <>
struct Terms<0> {  // Laplace 2D
    static constexpr int F = 3, O = 1, K = 3, N = 3;
    __host__ __device__ static constexpr int f(int t) { return t; }
    __host__ __device__ static constexpr int o(int) { return 0; }
    __host__ __device__ static constexpr int c(int t) { return t; }
};
template <>
struct Terms<1> {  // Laplace 3D
    static constexpr int F = 4, O = 1, K = 4, N = 4;
    __host__ __device__ static constexpr int f(int t) { return t; }
    __host__ __device__ static constexpr int o(int) { return 0; }
    __host__ __device__ static constexpr int c(int t) { return t; }
};
template <>
struct Terms<2> {  // Navier (Kelvin): 27 terms, 3 per field, ordered by field
    static constexpr int F = 9, O = 3, K = 24, N = 27;
    __host__ __device__ static constexpr int f(int t) { return t / 3; }
    __host__ __device__ static constexpr int o(int t) { return t % 3; }
    __host__ __device__ static constexpr int c(int t) {
        return f(t) < 3 ? pair_of(o(t), f(t)) : 6 + 6 * o(t) + (f(t) - 3);
    }
};

template <>
struct Terms<3> {  // elastic half-space: u_a = sum_b K_ab * sigma_b, 9 terms
    static constexpr int F = 3, O = 3, K = 8, N = 9;
    __host__ __device__ static constexpr int f(int t) { return t % 3; }
    __host__ __device__ static constexpr int o(int t) { return t / 3; }
    __host__ __device__ static constexpr int c(int t) {
        constexpr int tab[9] = {0, 2, 4, 2, 1, 5, 6, 7, 3};  // (o, f) row-major
        return tab[t];
    }
};

// Spectral components that multiply field f, in term order.
template <int KIND>
__host__ __device__ constexpr int field_ncomp(int f) {
    int n = 0;
    for (int t = 0; t < Terms<KIND>::N; ++t)
        if (Terms<KIND>::f(t) == f) ++n;
    return n;
}
template <int KIND>
__host__ __device__ constexpr int field_comp(int f, int i) {
    int n = 0;
    for (int t = 0; t < Terms<KIND>::N; ++t)
        if (Terms<KIND>::f(t) == f) {
            if (n == i) return Terms<KIND>::c(t);
            ++n;
        }
    return -1;
}
// Position of term t among the terms of its field.
template <int KIND>
__host__ __device__ constexpr int term_slot(int t) {
    int n = 0;
    for (int u = 0; u < t; ++u)
        if (Terms<KIND>::f(u) == Terms<KIND>::f(t)) ++n;
    return n;
}
template <int KIND>
__host__ __device__ constexpr int max_field_ncomp() {
    int m = 0;
    for (int f = 0; f < Terms<KIND>::F; ++f) m = field_ncomp<KIND>(f) > m ? field_ncomp<KIND>(f) : m;
    return m;
}

}  // namespace bemfft
