// md.hpp -- device multiple-double arithmetic for gfx950.
//
// An m-double is M binary64 limbs, limb 0 most significant, denoting the
// exact sum of its limbs.  The operations follow the project's fixed
// specification (error-free transformations, level sums, renormalisation);
// they are fully unrolled at compile time, branch-free and data-independent,
// so a wavefront never diverges inside an operation.  Build with
// -ffp-contract=off and without fast-math: every + - * below is one IEEE
// round-to-nearest operation and __builtin_fma is the fused one.
//
//   two_sum(a, b)   s = a+b, e = (a-(s-bb)) + (b-bb), bb = s-a   (Knuth)
//   two_prod(a, b)  p = a*b, e = fma(a, b, -p)
//   deposit<LO>     add t into the level sums S[LO..M-1]; exact until the
//                   last level, which adds plainly
//   renorm          bottom-up two_sum pass, then top-down two_sum pass
//   md_add(x, y)    S = x; deposit y_k at level k; renorm
//   md_mul(x, y)    exact products of levels 0..M-2, plain FMAs for levels
//                   M-1 and M, exact low parts pushed one level down; renorm
//
// Complex m-doubles (real and imaginary parts kept apart, Sections 2 and 5)
// are 2M doubles, the real limbs then the imaginary ones:
//   cmd_mul(x, y)   re = md_add(xr*yr, -(xi*yi)), im = md_add(xr*yi, xi*yr),
//                   each product an md_mul, the negation exact
//   cmd_add(x, y)   md_add of the real parts and of the imaginary parts
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mdpe {

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    double ss = a + b;
    double bb = ss - a;
    e = (a - (ss - bb)) + (b - bb);
    s = ss;
}

__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
    double pp = a * b;
    e = __builtin_fma(a, b, -pp);
    p = pp;
}

template <int M, int LO>
__device__ __forceinline__ void deposit(double (&S)[M], double t) {
    if constexpr (LO < M - 1) {
        two_sum(S[LO], t, S[LO], t);
        deposit<M, LO + 1>(S, t);
    } else {
        S[M - 1] = S[M - 1] + t;
    }
}

template <int M>
__device__ __forceinline__ void renorm(const double (&S)[M], double (&r)[M]) {
    if constexpr (M == 1) {
        r[0] = S[0];
    } else {
        double u[M];
        double s = S[M - 1];
        sfor<0, M - 1>([&](auto q) {
            constexpr int j = M - 2 - decltype(q)::value;
            two_sum(S[j], s, s, u[j + 1]);
        });
        u[0] = s;
        r[0] = u[0];
        double e = u[1];
        sfor<1, M - 1>([&](auto q) {
            constexpr int j = decltype(q)::value;
            two_sum(e, u[j + 1], r[j], e);
        });
        r[M - 1] = e;
    }
}

template <int M>
__device__ __forceinline__ void md_add(const double (&x)[M], const double (&y)[M], double (&z)[M]) {
    double S[M];
    sfor<0, M>([&](auto k) { S[decltype(k)::value] = x[decltype(k)::value]; });
    sfor<0, M>([&](auto k) {
        constexpr int K = decltype(k)::value;
        deposit<M, K>(S, y[K]);
    });
    renorm<M>(S, z);
}

template <int M>
__device__ __forceinline__ void md_mul(const double (&x)[M], const double (&y)[M], double (&z)[M]) {
    double S[M];
    double E[M > 1 ? M - 1 : 1];
    sfor<0, M - 1>([&](auto k) {
        constexpr int K = decltype(k)::value;
        two_prod(x[0], y[K], S[K], E[K]);
    });
    S[M - 1] = x[0] * y[M - 1];
    sfor<1, M>([&](auto i) {
        constexpr int I = decltype(i)::value;
        S[M - 1] = __builtin_fma(x[I], y[M - 1 - I], S[M - 1]);
    });
    sfor<1, M>([&](auto i) {
        constexpr int I = decltype(i)::value;
        S[M - 1] = __builtin_fma(x[I], y[M - I], S[M - 1]);
    });
    sfor<0, M - 1>([&](auto k) {
        constexpr int K = decltype(k)::value;
        deposit<M, K + 1>(S, E[K]);
    });
    sfor<1, M - 1>([&](auto k) {
        constexpr int K = decltype(k)::value;
        sfor<1, K + 1>([&](auto i) {
            constexpr int I = decltype(i)::value;
            double p, e;
            two_prod(x[I], y[K - I], p, e);
            deposit<M, K>(S, p);
            deposit<M, K + 1>(S, e);
        });
    });
    renorm<M>(S, z);
}

// Doubles per coefficient: M limbs, or 2M for complex series.
template <int M, bool CX>
constexpr int kCoef = CX ? 2 * M : M;

template <int M>
__device__ __forceinline__ void cmd_mul(const double (&x)[2 * M], const double (&y)[2 * M], double (&z)[2 * M]) {
    double xr[M], xi[M], yr[M], yi[M];
    sfor<0, M>([&](auto l) {
        constexpr int L = decltype(l)::value;
        xr[L] = x[L];
        xi[L] = x[M + L];
        yr[L] = y[L];
        yi[L] = y[M + L];
    });
    double rr[M], ii[M], ri[M], ir[M], zr[M], zi[M];
    md_mul<M>(xr, yr, rr);
    md_mul<M>(xi, yi, ii);
    md_mul<M>(xr, yi, ri);
    md_mul<M>(xi, yr, ir);
    sfor<0, M>([&](auto l) { ii[decltype(l)::value] = -ii[decltype(l)::value]; });
    md_add<M>(rr, ii, zr);
    md_add<M>(ri, ir, zi);
    sfor<0, M>([&](auto l) {
        constexpr int L = decltype(l)::value;
        z[L] = zr[L];
        z[M + L] = zi[L];
    });
}

template <int M>
__device__ __forceinline__ void cmd_add(const double (&x)[2 * M], const double (&y)[2 * M], double (&z)[2 * M]) {
    double xr[M], xi[M], yr[M], yi[M], zr[M], zi[M];
    sfor<0, M>([&](auto l) {
        constexpr int L = decltype(l)::value;
        xr[L] = x[L];
        xi[L] = x[M + L];
        yr[L] = y[L];
        yi[L] = y[M + L];
    });
    md_add<M>(xr, yr, zr);
    md_add<M>(xi, yi, zi);
    sfor<0, M>([&](auto l) {
        constexpr int L = decltype(l)::value;
        z[L] = zr[L];
        z[M + L] = zi[L];
    });
}

// One coefficient operation of the series' number field.
template <int M, bool CX>
__device__ __forceinline__ void coef_mul(const double (&x)[kCoef<M, CX>], const double (&y)[kCoef<M, CX>],
                                         double (&z)[kCoef<M, CX>]) {
    if constexpr (CX)
        cmd_mul<M>(x, y, z);
    else
        md_mul<M>(x, y, z);
}

template <int M, bool CX>
__device__ __forceinline__ void coef_add(const double (&x)[kCoef<M, CX>], const double (&y)[kCoef<M, CX>],
                                         double (&z)[kCoef<M, CX>]) {
    if constexpr (CX)
        cmd_add<M>(x, y, z);
    else
        md_add<M>(x, y, z);
}

}  // namespace mdpe
