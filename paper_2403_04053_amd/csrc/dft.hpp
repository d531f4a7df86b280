// Register-resident small DFTs for gfx950 wavefronts.
//
// dft<R, S>(v) replaces v[0..R) by X_k = sum_n v_n exp(S 2 pi i n k / R)
// (S = -1 forward, +1 inverse, unnormalised).  Every index is a compile-time
// constant after unrolling, so the arrays live in VGPRs and every twiddle is a
// literal folded into the FMAs.  Twiddle values come from a constexpr FP64
// series rounded once to FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace pstd {

namespace cx {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double sin_series(double x) {
    double t = x, s = x;
    for (int k = 1; k < 40; ++k) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double cos_series(double x) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 40; ++k) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
// 2 pi J / R folded into [-pi, pi]
constexpr double angle(int R, int J) {
    int j = ((J % R) + R) % R;
    if (2 * j > R) j -= R;
    return 2.0 * kPi * j / R;
}
constexpr double cosr(int R, int J) { return cos_series(angle(R, J)); }
constexpr double sinr(int R, int J) { return sin_series(angle(R, J)); }
}  // namespace cx

template <int... I, class F>
__device__ __forceinline__ void unroll_impl(std::integer_sequence<int, I...>, F&& f) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F&& f) {
    unroll_impl(std::make_integer_sequence<int, N>{}, f);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// S * i * a
template <int S>
__device__ __forceinline__ float2 muli(float2 a) {
    if constexpr (S > 0) return make_float2(-a.y, a.x);
    else return make_float2(a.y, -a.x);
}

// x * exp(S 2 pi i J / R)
template <int R, int J, int S>
__device__ __forceinline__ float2 twmul(float2 x) {
    constexpr int j = ((J % R) + R) % R;
    if constexpr (j == 0) {
        return x;
    } else if constexpr (2 * j == R) {
        return make_float2(-x.x, -x.y);
    } else if constexpr (4 * j == R) {
        return muli<S>(x);
    } else if constexpr (4 * j == 3 * R) {
        return muli<-S>(x);
    } else {
        constexpr float c = (float)cx::cosr(R, j);
        constexpr float s = (float)(S * cx::sinr(R, j));
        return make_float2(x.x * c - x.y * s, x.x * s + x.y * c);
    }
}

constexpr int first_factor(int R) {
    return (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3
         : (R % 5 == 0 && R != 5) ? 5 : R;
}

template <int R, int S>
__device__ __forceinline__ void dft(float2 (&v)[R]);

// odd R, direct sum with the symmetric pairs (n, R - n)
template <int R, int S>
__device__ __forceinline__ void dft_odd(float2 (&v)[R]) {
    constexpr int H = (R - 1) / 2;
    float2 sp[H + 1], sm[H + 1];
    unroll<H>([&](auto i) {
        constexpr int n = decltype(i)::value + 1;
        sp[n] = cadd(v[n], v[R - n]);
        sm[n] = csub(v[n], v[R - n]);
    });
    float2 out[R];
    float2 x0 = v[0];
    unroll<H>([&](auto i) {
        constexpr int n = decltype(i)::value + 1;
        x0 = cadd(x0, sp[n]);
    });
    out[0] = x0;
    unroll<H>([&](auto ik) {
        constexpr int k = decltype(ik)::value + 1;
        float2 a = v[0];
        float2 b = make_float2(0.f, 0.f);
        unroll<H>([&](auto i) {
            constexpr int n = decltype(i)::value + 1;
            constexpr float c = (float)cx::cosr(R, n * k);
            constexpr float s = (float)cx::sinr(R, n * k);
            a.x += sp[n].x * c;
            a.y += sp[n].y * c;
            b.x += sm[n].x * s;
            b.y += sm[n].y * s;
        });
        const float2 ib = muli<S>(b);
        out[k] = cadd(a, ib);
        out[R - k] = csub(a, ib);
    });
    unroll<R>([&](auto i) { v[decltype(i)::value] = out[decltype(i)::value]; });
}

template <int R, int S>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const float2 s13 = cadd(v[1], v[3]), d13 = muli<S>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if constexpr (first_factor(R) == R) {
        static_assert(R % 2 == 1, "odd prime-like radix expected");
        dft_odd<R, S>(v);
    } else {
        // R = A B; n = B a + b, k = ka + A kb
        constexpr int A = first_factor(R);
        constexpr int B = R / A;
        float2 t[R];
        unroll<B>([&](auto ib) {
            constexpr int b = decltype(ib)::value;
            float2 u[A];
            unroll<A>([&](auto ia) { u[decltype(ia)::value] = v[B * decltype(ia)::value + b]; });
            dft<A, S>(u);
            unroll<A>([&](auto ika) {
                constexpr int ka = decltype(ika)::value;
                t[ka * B + b] = twmul<R, b * ka, S>(u[ka]);
            });
        });
        unroll<A>([&](auto ika) {
            constexpr int ka = decltype(ika)::value;
            float2 u[B];
            unroll<B>([&](auto ib) { u[decltype(ib)::value] = t[ka * B + decltype(ib)::value]; });
            dft<B, S>(u);
            unroll<B>([&](auto ikb) { v[ka + A * decltype(ikb)::value] = u[decltype(ikb)::value]; });
        });
    }
}

}  // namespace pstd
