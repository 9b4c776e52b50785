// Small forward DFTs held in registers:  y[k] = sum_q v[q] exp(-2 pi i q k / R).
// Radices 2, 3, 4, 5, 7, 8 and 16, for float and double.  Used as the
// butterflies of the Stockham passes in fft_engines.hpp.
#pragma once

#include "common.hpp"

namespace ca {

template <typename T> __device__ __forceinline__ void dft2(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
}

// Generic in-place radix-4 on four named values.
template <typename T>
__device__ __forceinline__ void dft4(cpx<T>& a, cpx<T>& b, cpx<T>& c, cpx<T>& d) {
    cpx<T> s0 = add(a, c), s1 = sub(a, c), s2 = add(b, d), s3 = sub(b, d);
    a = add(s0, s2);
    c = sub(s0, s2);
    b = add(s1, mul_mi(s3));   // s1 - i s3
    d = sub(s1, mul_mi(s3));   // s1 + i s3
}
template <typename T> __device__ __forceinline__ void dft4(cpx<T>* v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename T> __device__ __forceinline__ void dft3(cpx<T>* v) {
    const T h = T(0.86602540378443864676);   // sin(2 pi / 3)
    cpx<T> a = v[0], b = v[1], c = v[2];
    cpx<T> t1 = add(b, c);
    cpx<T> t2 = sub(a, scale(t1, T(0.5)));
    cpx<T> m = scale(sub(b, c), h);
    v[0] = add(a, t1);
    v[1] = add(t2, mul_mi(m));
    v[2] = sub(t2, mul_mi(m));
}

// Odd prime radix through the symmetric pairs (q, R - q).
template <int R> struct odd_tab;
template <> struct odd_tab<5> {
    static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                    -0.80901699437494742410, 0.30901699437494742410};
    static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                    -0.58778525229247312917, -0.95105651629515357212};
};
template <> struct odd_tab<7> {
    static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                    -0.90096886790241912624, -0.90096886790241912624,
                                    -0.22252093395631440429, 0.62348980185873353053};
    static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                    0.43388373911755812048, -0.43388373911755812048,
                                    -0.97492791218182360702, -0.78183148246802980871};
};

template <int R, typename T> __device__ __forceinline__ void dft_odd(cpx<T>* v) {
    constexpr int H = (R - 1) / 2;
    cpx<T> a[H + 1], b[H + 1];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        a[q] = add(v[q], v[R - q]);
        b[q] = sub(v[q], v[R - q]);
    }
    cpx<T> y[R];
    cpx<T> s0 = v[0];
#pragma unroll
    for (int q = 1; q <= H; ++q) s0 = add(s0, a[q]);
    y[0] = s0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        cpx<T> A = v[0];
        cpx<T> B = {T(0), T(0)};
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            const int e = (q * k) % R;
            const T cc = T(odd_tab<R>::c[e]);
            const T ss = T(odd_tab<R>::s[e]);
            A.x += cc * a[q].x; A.y += cc * a[q].y;
            B.x += ss * b[q].x; B.y += ss * b[q].y;
        }
        // y[k] = A - i B, y[R-k] = A + i B
        y[k] = {A.x + B.y, A.y - B.x};
        y[R - k] = {A.x - B.y, A.y + B.x};
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = y[k];
}

// Multiply by exp(-2 pi i M / 16) with M known at compile time.
template <int M, typename T> __device__ __forceinline__ cpx<T> w16(cpx<T> z) {
    constexpr int m = M & 15;
    const T r = T(0.70710678118654752440);
    const T c = T(0.92387953251128675613);   // cos(pi/8)
    const T s = T(0.38268343236508977173);   // sin(pi/8)
    if constexpr (m == 0) return z;
    else if constexpr (m == 4) return mul_mi(z);
    else if constexpr (m == 8) return cpx<T>{-z.x, -z.y};
    else if constexpr (m == 12) return mul_pi(z);
    else if constexpr (m == 2) return cpx<T>{r * (z.x + z.y), r * (z.y - z.x)};
    else if constexpr (m == 6) return cpx<T>{r * (z.y - z.x), -r * (z.x + z.y)};
    else if constexpr (m == 10) return cpx<T>{-r * (z.x + z.y), r * (z.x - z.y)};
    else if constexpr (m == 14) return cpx<T>{r * (z.x - z.y), r * (z.x + z.y)};
    else {
        // general: (cos t, -sin t) with t = 2 pi m / 16
        constexpr int q = m & 3;          // position inside the quadrant
        const T cq = (q == 1) ? c : s;    // cos of the in-quadrant angle (pi/8 or 3pi/8)
        const T sq = (q == 1) ? s : c;
        cpx<T> w = {cq * z.x + sq * z.y, cq * z.y - sq * z.x};   // z * exp(-i q pi/8)
        if constexpr (m < 4) return w;
        else if constexpr (m < 8) return mul_mi(w);
        else if constexpr (m < 12) return cpx<T>{-w.x, -w.y};
        else return mul_pi(w);
    }
}

template <typename T> __device__ __forceinline__ void dft8(cpx<T>* v) {
    cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = w16<2>(o1);
    o2 = w16<4>(o2);
    o3 = w16<6>(o3);
    v[0] = add(e0, o0); v[4] = sub(e0, o0);
    v[1] = add(e1, o1); v[5] = sub(e1, o1);
    v[2] = add(e2, o2); v[6] = sub(e2, o2);
    v[3] = add(e3, o3); v[7] = sub(e3, o3);
}

// 16 = 4 x 4: inputs x[4 n1 + n2], outputs y[k1 + 4 k2].
template <typename T> __device__ __forceinline__ void dft16(cpx<T>* v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // a[n2][k1] sits at v[n2 + 4 k1]; twiddle by w16^(n2 k1)
    v[5] = w16<1>(v[5]);  v[9] = w16<2>(v[9]);   v[13] = w16<3>(v[13]);
    v[6] = w16<2>(v[6]);  v[10] = w16<4>(v[10]); v[14] = w16<6>(v[14]);
    v[7] = w16<3>(v[7]);  v[11] = w16<6>(v[11]); v[15] = w16<9>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // y[k1 + 4 k2] is at v[4 k1 + k2]: transpose the 4 x 4 register block
    cpx<T> t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
}

template <int R, typename T> __device__ __forceinline__ void dft(cpx<T>* v) {
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 3) dft3(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 5) dft_odd<5>(v);
    else if constexpr (R == 7) dft_odd<7>(v);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 16) dft16(v);
    else static_assert(R == 2, "unsupported radix");
}

}  // namespace ca
