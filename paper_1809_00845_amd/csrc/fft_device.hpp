// fft_device.hpp -- LDS-staged mixed-radix Stockham FFT for pencils on gfx950.
//
// One pencil of P complex points is owned by TPP consecutive lanes of one
// wavefront (TPP divides 64), each lane holding E = P/TPP points while a
// radix stage runs in registers.  Stages exchange data through LDS.  The
// stage rule is the self-sorting (Stockham) decimation in time: with Ns the
// product of the radices already applied, butterfly j reads x[j + s P/R],
// twiddles by w_{Ns R}^{s (j mod Ns)}, runs a radix-R DFT and writes
// y[(j / Ns) Ns R + (j mod Ns) + s Ns]; the result comes out in natural order.
//
// Radix-R DFTs are unrolled at compile time; composite radices use the
// two-level split R = R1 R2 with constant twiddles computed by constexpr
// code (exact integer reduction of the angle to one octant, Taylor series
// there).  Runtime stage twiddles come from a per-size table in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace bemfft {

template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// ------------------------------------------------------------ constexpr trig
namespace ctrig {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kSqrtHalf = 0.707106781186547524400844362104849039;

constexpr double poly_sin(double x) {
    double x2 = x * x, t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double poly_cos(double x) {
    double x2 = x * x, t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
struct CS {
    double c, s;
};
// (cos, sin) of 2 pi t / n.  The quadrant is taken in exact integers; the
// remaining angle is folded into [0, pi/4] before the series.
constexpr CS cs2pi(long t, long n) {
    t %= n;
    if (t < 0) t += n;
    long q = (4 * t) / n;
    long r = 4 * t - q * n;  // angle = (q + r/n) * pi/2
    double c = 1.0, s = 0.0;
    if (r == 0) {
        c = 1.0;
        s = 0.0;
    } else if (2 * r == n) {
        c = kSqrtHalf;
        s = kSqrtHalf;
    } else if (2 * r < n) {
        double phi = (kPi / 2.0) * (double)r / (double)n;
        c = poly_cos(phi);
        s = poly_sin(phi);
    } else {
        double phi = (kPi / 2.0) * (double)(n - r) / (double)n;
        c = poly_sin(phi);
        s = poly_cos(phi);
    }
    for (long i = 0; i < q; ++i) {
        double c2 = -s, s2 = c;
        c = c2;
        s = s2;
    }
    return {c, s};
}
}  // namespace ctrig

// Multiply by exp(DIR * 2 pi i T / N), a compile-time constant.
template <long T, long N, int DIR, typename R>
__device__ __forceinline__ cx<R> twc(cx<R> a) {
    constexpr ctrig::CS w = ctrig::cs2pi(T, N);
    constexpr double wr = w.c;
    constexpr double wi = DIR * w.s;
    if constexpr (wi == 0.0 && wr == 1.0) {
        return a;
    } else if constexpr (wi == 0.0 && wr == -1.0) {
        return {-a.x, -a.y};
    } else if constexpr (wr == 0.0 && wi == 1.0) {
        return {-a.y, a.x};
    } else if constexpr (wr == 0.0 && wi == -1.0) {
        return {a.y, -a.x};
    } else {
        return {R(wr) * a.x - R(wi) * a.y, R(wr) * a.y + R(wi) * a.x};
    }
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ------------------------------------------------------------ small DFTs
// In-place DFT of N points in registers: X_k = sum_s v_s exp(DIR 2 pi i s k / N).
template <int N, int DIR, typename R>
struct DFT;

template <int DIR, typename R>
struct DFT<1, DIR, R> {
    __device__ static __forceinline__ void run(cx<R> (&)[1]) {}
};

template <int DIR, typename R>
struct DFT<2, DIR, R> {
    __device__ static __forceinline__ void run(cx<R> (&v)[2]) {
        cx<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int DIR, typename R>
struct DFT<3, DIR, R> {
    __device__ static __forceinline__ void run(cx<R> (&v)[3]) {
        // w = exp(DIR 2 pi i / 3) = -1/2 + i DIR sqrt(3)/2
        constexpr R k = R(DIR * 0.866025403784438646763723170752936183);
        cx<R> s = cadd(v[1], v[2]);
        cx<R> d = csub(v[1], v[2]);
        cx<R> m = {v[0].x - R(0.5) * s.x, v[0].y - R(0.5) * s.y};
        v[0] = cadd(v[0], s);
        cx<R> id = {-k * d.y, k * d.x};  // i k d
        v[1] = cadd(m, id);
        v[2] = csub(m, id);
    }
};

template <int DIR, typename R>
struct DFT<4, DIR, R> {
    __device__ static __forceinline__ void run(cx<R> (&v)[4]) {
        cx<R> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        cx<R> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        // (DIR i) t3
        cx<R> it3 = {R(-DIR) * t3.y, R(DIR) * t3.x};
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, it3);
        v[3] = csub(t1, it3);
    }
};

// Prime 5: direct sum with constant twiddles.
template <int DIR, typename R>
struct DFT<5, DIR, R> {
    __device__ static __forceinline__ void run(cx<R> (&v)[5]) {
        cx<R> out[5];
        static_for<0, 5>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            cx<R> acc = v[0];
            static_for<1, 5>([&](auto ss) {
                constexpr int s = decltype(ss)::value;
                acc = cadd(acc, twc<(long)s * k, 5, DIR, R>(v[s]));
            });
            out[k] = acc;
        });
#pragma unroll
        for (int k = 0; k < 5; ++k) v[k] = out[k];
    }
};

// N = N1 * N2: inner DFTs of length N1 over v[N2 s1 + s2], twiddle
// exp(DIR 2 pi i s2 k1 / N), outer DFTs of length N2 -> X[k1 + N1 k2].
template <int N, int N1, int N2, int DIR, typename R>
struct DFTSplit {
    __device__ static __forceinline__ void run(cx<R> (&v)[N]) {
        cx<R> a[N2][N1];
        static_for<0, N2>([&](auto s2c) {
            constexpr int s2 = decltype(s2c)::value;
            cx<R> t[N1];
#pragma unroll
            for (int s1 = 0; s1 < N1; ++s1) t[s1] = v[N2 * s1 + s2];
            DFT<N1, DIR, R>::run(t);
            static_for<0, N1>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                a[s2][k1] = twc<(long)s2 * k1, N, DIR, R>(t[k1]);
            });
        });
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
            cx<R> t[N2];
#pragma unroll
            for (int s2 = 0; s2 < N2; ++s2) t[s2] = a[s2][k1];
            DFT<N2, DIR, R>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) v[k1 + N1 * k2] = t[k2];
        }
    }
};

template <int DIR, typename R> struct DFT<6, DIR, R> : DFTSplit<6, 2, 3, DIR, R> {};
template <int DIR, typename R> struct DFT<8, DIR, R> : DFTSplit<8, 2, 4, DIR, R> {};
template <int DIR, typename R> struct DFT<12, DIR, R> : DFTSplit<12, 3, 4, DIR, R> {};
template <int DIR, typename R> struct DFT<16, DIR, R> : DFTSplit<16, 4, 4, DIR, R> {};
template <int DIR, typename R> struct DFT<20, DIR, R> : DFTSplit<20, 4, 5, DIR, R> {};

// ------------------------------------------------------------ pencil plans
// Radix schedules: every radix divides E = P / TPP, so each lane runs E/R
// whole butterflies in every stage.
template <int... Rs>
struct Radices {};

// A radix schedule: P points per pencil, TPP lanes per pencil, radices Rs.
template <int P_, int TPP_, int... Rs>
struct FFTShape {
    static constexpr int P = P_;
    static constexpr int TPP = TPP_;
    static constexpr int E = P_ / TPP_;
    using rad = Radices<Rs...>;
};

// Two compiled schedules per length (S = 0 default, S = 1 alternative), and
// for three lengths a wide one (S = 2: one pencil per wavefront, 64 lanes,
// so a lane holds P/64 values -- for the z pass of the Navier family, whose
// three FP64 output accumulators do not fit in registers at 16 or 32 lanes
// per pencil); the plan's autotuner picks one for the z pass by timing them.
template <int P, int S>
struct Sched;
template <> struct Sched<1, 0> : FFTShape<1, 1> {};
template <> struct Sched<32, 0> : FFTShape<32, 4, 4, 8> {};
template <> struct Sched<32, 1> : FFTShape<32, 4, 8, 4> {};
template <> struct Sched<64, 0> : FFTShape<64, 8, 8, 8> {};
template <> struct Sched<64, 1> : FFTShape<64, 4, 16, 4> {};
template <> struct Sched<96, 0> : FFTShape<96, 8, 4, 4, 6> {};
template <> struct Sched<96, 1> : FFTShape<96, 8, 6, 4, 4> {};
template <> struct Sched<128, 0> : FFTShape<128, 8, 16, 8> {};
template <> struct Sched<128, 1> : FFTShape<128, 16, 8, 4, 4> {};
template <> struct Sched<192, 0> : FFTShape<192, 16, 4, 4, 12> {};
template <> struct Sched<192, 1> : FFTShape<192, 16, 12, 4, 4> {};
template <> struct Sched<256, 0> : FFTShape<256, 16, 16, 16> {};
template <> struct Sched<256, 1> : FFTShape<256, 32, 8, 8, 4> {};
template <> struct Sched<320, 0> : FFTShape<320, 16, 4, 4, 20> {};
template <> struct Sched<320, 1> : FFTShape<320, 16, 20, 4, 4> {};
template <> struct Sched<384, 0> : FFTShape<384, 16, 8, 6, 8> {};
template <> struct Sched<384, 1> : FFTShape<384, 32, 4, 4, 4, 6> {};
template <> struct Sched<512, 0> : FFTShape<512, 32, 8, 8, 8> {};
template <> struct Sched<512, 1> : FFTShape<512, 32, 16, 4, 8> {};
// 1024 points: 2D plans only (grids of up to 512 points per axis)
template <> struct Sched<1024, 0> : FFTShape<1024, 64, 16, 16, 4> {};
template <> struct Sched<1024, 1> : FFTShape<1024, 64, 4, 16, 16> {};
template <> struct Sched<256, 2> : FFTShape<256, 64, 4, 4, 4, 4> {};
template <> struct Sched<384, 2> : FFTShape<384, 64, 6, 2, 2, 2, 2, 2, 2> {};
template <> struct Sched<512, 2> : FFTShape<512, 64, 8, 8, 8> {};

// Lengths with a wide schedule.
__host__ __device__ constexpr bool has_wide_sched(int p) { return p == 256 || p == 384 || p == 512; }

template <int P>
using PencilShape = Sched<P, 0>;

// Lanes of one pencil always sit in one wavefront, so the exchanges inside a
// transform only need the wave's LDS accesses to stay in program order (LDS
// executes one wave's instructions in order); this barrier stops the compiler
// from moving them.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS slot of pencil element i: one pad slot after every 16 elements keeps
// the stride-R writes of a radix-R stage off a single bank.
__host__ __device__ constexpr int pslot(int i) { return i + (i >> 4); }
// LDS elements reserved per pencil.
template <int P>
__host__ __device__ constexpr int pstride() { return P + P / 16 + 1; }

// Register layout of a pencil: lane t (0 <= t < TPP) holds x[t + e TPP],
// e in [0, E).  With the stage rule above this is exactly what the first
// stage reads and what the last stage writes, for every radix schedule, so a
// transform starts and ends in registers and only the exchanges between
// stages pass through the pencil's LDS slots.
template <typename R, int P, int TPP, int RAD, int NS, int DIR>
__device__ __forceinline__ void reg_stage(cx<R> (&x)[P / TPP], cx<R> *pen, const cx<R> *tw, int t) {
    constexpr int E = P / TPP;
    constexpr int NB = E / RAD;
    constexpr int STRIDE = P / RAD;
    constexpr bool FIRST = (NS == 1);
    constexpr bool LAST = (NS * RAD == P);
    static_assert(E % RAD == 0, "radix must divide the points per lane");
    cx<R> v[NB][RAD];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int s = 0; s < RAD; ++s) {
            if constexpr (FIRST) v[b][s] = x[b + s * NB];
            else v[b][s] = pen[pslot(t + b * TPP + s * STRIDE)];
        }
    if constexpr (!FIRST) wave_lds_sync();  // all reads of this stage precede its writes
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * TPP;
        const int k = j % NS;
        if constexpr (NS > 1) {
            constexpr int TWSTEP = P / (NS * RAD);
#pragma unroll
            for (int s = 1; s < RAD; ++s) {
                const cx<R> w = tw[s * k * TWSTEP];
                v[b][s] = (DIR < 0) ? cmul(v[b][s], w) : cmulc(v[b][s], w);
            }
        }
        DFT<RAD, DIR, R>::run(v[b]);
        if constexpr (LAST) {
#pragma unroll
            for (int s = 0; s < RAD; ++s) x[b + s * NB] = v[b][s];
        } else {
            const int base = (j / NS) * NS * RAD + k;
#pragma unroll
            for (int s = 0; s < RAD; ++s) pen[pslot(base + s * NS)] = v[b][s];
        }
    }
    if constexpr (!LAST) wave_lds_sync();  // writes visible to the next stage
}

template <typename R, int P, int TPP, int DIR, int NS>
__device__ __forceinline__ void reg_stages(cx<R> (&)[P / TPP], cx<R> *, const cx<R> *, int, Radices<>) {}

template <typename R, int P, int TPP, int DIR, int NS, int RAD, int... REST>
__device__ __forceinline__ void reg_stages(cx<R> (&x)[P / TPP], cx<R> *pen, const cx<R> *tw, int t,
                                           Radices<RAD, REST...>) {
    reg_stage<R, P, TPP, RAD, NS, DIR>(x, pen, tw, t);
    reg_stages<R, P, TPP, DIR, NS * RAD>(x, pen, tw, t, Radices<REST...>{});
}

// In-register FFT of one pencil (unscaled; DIR = -1 forward, +1 inverse)
// with schedule SH.  x: the lane's E = P/TPP points in the layout above,
// replaced by the transform in the same layout.  pen: the pencil's
// pstride<P>() LDS slots (scratch).  tw: LDS table tw[i] = exp(-2 pi i i / P).
// Synchronises only the pencil's wavefront.
template <typename R, typename SH, int DIR>
__device__ __forceinline__ void fft_regs_s(cx<R> (&x)[SH::E], cx<R> *pen, const cx<R> *tw, int t) {
    static_assert(64 % SH::TPP == 0, "a pencil must not straddle wavefronts");
    wave_lds_sync();  // earlier users of the pencil's slots are done
    reg_stages<R, SH::P, SH::TPP, DIR, 1>(x, pen, tw, t, typename SH::rad{});
}

template <typename R, int P, int DIR>
__device__ __forceinline__ void fft_regs(cx<R> (&x)[P / PencilShape<P>::TPP], cx<R> *pen, const cx<R> *tw, int t) {
    fft_regs_s<R, PencilShape<P>, DIR>(x, pen, tw, t);
}

// FFT of a pencil held in LDS slots (pslot layout), in place.
template <typename R, int P, int DIR>
__device__ __forceinline__ void pencil_fft(cx<R> *pen, const cx<R> *tw, int t) {
    using S = PencilShape<P>;
    constexpr int E = P / S::TPP;
    cx<R> x[E];
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = pen[pslot(t + e * S::TPP)];
    fft_regs<R, P, DIR>(x, pen, tw, t);
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) pen[pslot(t + e * S::TPP)] = x[e];
    wave_lds_sync();
}

}  // namespace bemfft
