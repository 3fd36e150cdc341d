// Batched 1-D FFT of length N = 2^a or 3 2^a for one line held by T = N/16
// threads.
//
// Stockham autosort: radix-16 passes in registers with the exchanges between
// passes through an LDS line buffer, a radix-2/4/8 pass when log2 of the
// power-of-two part is not a multiple of 4, and for N = 3 2^a a last radix-3
// pass done in place in the LDS buffer (N/3 butterflies shared out over the T
// threads).  On entry thread j holds x[j + T k] (k = 0..15); on exit it holds
// X[j + T k], where X[f] = sum_n x[n] exp(DIR i 2 pi n f / N), unnormalised.
// Twiddles come from a float64-derived table tw[k] = exp(+i 2 pi k / N).
#pragma once
#include "common.hpp"

namespace wsg {

// LDS index with one pad element per 16 (spreads the radix-16 scatter over banks).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
template <int N>
struct LinePad {
    static constexpr int size = N + N / 16;
};

// multiply by exp(DIR i 2 pi m / 16) for a compile-time m
template <typename R, int DIR, int M>
__device__ __forceinline__ cpx<R> w16(cpx<R> a) {
    constexpr int m = M & 15;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 4) {          // DIR * i
        return DIR > 0 ? cpx<R>{-a.y, a.x} : cpx<R>{a.y, -a.x};
    } else if constexpr (m == 8) {
        return {-a.x, -a.y};
    } else if constexpr (m == 12) {
        return DIR > 0 ? cpx<R>{a.y, -a.x} : cpx<R>{-a.y, a.x};
    } else {
        constexpr double c[16] = {
            1.0, 0.92387953251128673848, 0.70710678118654752440, 0.38268343236508977173,
            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128673848,
            -1.0, -0.92387953251128673848, -0.70710678118654752440, -0.38268343236508977173,
            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128673848};
        constexpr double s[16] = {
            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128673848,
            1.0, 0.92387953251128673848, 0.70710678118654752440, 0.38268343236508977173,
            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128673848,
            -1.0, -0.92387953251128673848, -0.70710678118654752440, -0.38268343236508977173};
        const R wc = R(c[m]), ws = R(DIR * s[m]);
        return {a.x * wc - a.y * ws, a.x * ws + a.y * wc};
    }
}

template <typename R, int DIR>
__device__ __forceinline__ void dft2(cpx<R>& a, cpx<R>& b) {
    cpx<R> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// natural order in and out: v[k] <- sum_n v[n] exp(DIR i 2 pi n k / 4)
template <typename R, int DIR>
__device__ __forceinline__ void dft4(cpx<R>& v0, cpx<R>& v1, cpx<R>& v2, cpx<R>& v3) {
    cpx<R> a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = csub(v1, v3);
    d = w16<R, DIR, 4>(d);
    v0 = cadd(a, c);
    v2 = csub(a, c);
    v1 = cadd(b, d);
    v3 = csub(b, d);
}

// 8-point DFT as 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2
template <typename R, int DIR>
__device__ __forceinline__ void dft8(cpx<R>* v) {
    dft4<R, DIR>(v[0], v[2], v[4], v[6]);
    dft4<R, DIR>(v[1], v[3], v[5], v[7]);
    cpx<R> y[8];
    y[0] = v[0]; y[1] = v[2]; y[2] = v[4]; y[3] = v[6];
    y[4] = v[1];
    y[5] = w16<R, DIR, 2>(v[3]);
    y[6] = w16<R, DIR, 4>(v[5]);
    y[7] = w16<R, DIR, 6>(v[7]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        v[k1] = cadd(y[k1], y[4 + k1]);
        v[k1 + 4] = csub(y[k1], y[4 + k1]);
    }
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <typename R, int DIR>
__device__ __forceinline__ void dft16(cpx<R>* v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<R, DIR>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[4 k1 + n2] now holds y[n2][k1]; twiddle by W16^(n2 k1)
    v[5] = w16<R, DIR, 1>(v[5]);
    v[6] = w16<R, DIR, 2>(v[6]);
    v[7] = w16<R, DIR, 3>(v[7]);
    v[9] = w16<R, DIR, 2>(v[9]);
    v[10] = w16<R, DIR, 4>(v[10]);
    v[11] = w16<R, DIR, 6>(v[11]);
    v[13] = w16<R, DIR, 3>(v[13]);
    v[14] = w16<R, DIR, 6>(v[14]);
    v[15] = w16<R, DIR, 9>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<R, DIR>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]; transpose to natural order
    cpx<R> t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
}

template <typename R, int DIR>
__device__ __forceinline__ cpx<R> twiddle(const cpx<R>* __restrict__ tw, int k) {
    cpx<R> w = tw[k];
    if (DIR < 0) w.y = -w.y;
    return w;
}

// log2 of a power of two
template <int N>
constexpr int log2_of() {
    int l = 0;
    while ((1 << l) < N) ++l;
    return l;
}

// In-place FFT of one line; `buf` is this line's LDS buffer of LinePad<N>::size
// elements.  Every thread of the block must call this the same number of times
// (it contains __syncthreads).
template <typename R, int N, int DIR>
__device__ __forceinline__ void fft_line(cpx<R> (&v)[16], cpx<R>* buf, const cpx<R>* __restrict__ tw, int j) {
    constexpr bool R3 = N % 3 == 0;
    constexpr int NP2 = R3 ? N / 3 : N;               // power-of-two part
    constexpr int LOG2 = log2_of<NP2>();
    static_assert((1 << LOG2) == NP2 && N % 16 == 0, "N = 2^a or 3 2^a, a multiple of 16");
    constexpr int T = N / 16;
    constexpr int P16 = LOG2 / 4;
    constexpr int REM = LOG2 % 4;
    int Ns = 1;
#pragma unroll
    for (int p = 0; p < P16; ++p) {
        if (p > 0) {
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m] = buf[lpad(j + m * T)];
            const int k = j & (Ns - 1);
            const int stride = N / (Ns * 16);
#pragma unroll
            for (int m = 1; m < 16; ++m) v[m] = cmul(v[m], twiddle<R, DIR>(tw, k * m * stride));
        }
        dft16<R, DIR>(v);
        if (!R3 && REM == 0 && p == P16 - 1) return;   // natural order: v[m] = X[j + m T]
        __syncthreads();
        const int base = (j / Ns) * Ns * 16 + (j & (Ns - 1));
#pragma unroll
        for (int m = 0; m < 16; ++m) buf[lpad(base + m * Ns)] = v[m];
        __syncthreads();
        Ns *= 16;
    }
    if constexpr (REM > 0) {
        constexpr int RR = 1 << REM;      // radix of this pass
        constexpr int B = 16 / RR;        // butterflies per thread
        constexpr int NR = N / RR;        // butterfly stride (= Ns when this is the last pass)
        constexpr int TWS = R3 ? 3 : 1;   // N / (Ns RR)
        cpx<R> u[16];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int m = 0; m < RR; ++m) u[b * RR + m] = buf[lpad(j + b * T + m * NR)];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = (j + b * T) & (Ns - 1);
#pragma unroll
            for (int m = 1; m < RR; ++m) u[b * RR + m] = cmul(u[b * RR + m], twiddle<R, DIR>(tw, k * m * TWS));
            if constexpr (RR == 2) dft2<R, DIR>(u[b * RR], u[b * RR + 1]);
            if constexpr (RR == 4) dft4<R, DIR>(u[b * RR], u[b * RR + 1], u[b * RR + 2], u[b * RR + 3]);
            if constexpr (RR == 8) dft8<R, DIR>(&u[b * RR]);
        }
        if constexpr (!R3) {
            // output X[j + b T + m' NR] = X[j + T (b + m' B)]
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int m = 0; m < RR; ++m) v[b + m * B] = u[b * RR + m];
            return;
        } else {
            __syncthreads();
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int jb = j + b * T;
                const int base = (jb / Ns) * Ns * RR + (jb & (Ns - 1));
#pragma unroll
                for (int m = 0; m < RR; ++m) buf[lpad(base + m * Ns)] = u[b * RR + m];
            }
            __syncthreads();
            Ns *= RR;
        }
    }
    if constexpr (R3) {
        // last pass, radix 3 with Ns = N / 3: butterfly i reads and writes
        // positions i, i + N/3, i + 2N/3 (natural order out), twiddles exp(DIR i 2 pi i m / N)
        constexpr int N3 = N / 3;
        const R hs = R(DIR) * R(0.86602540378443864676);      // DIR sin(2 pi / 3)
        for (int i = j; i < N3; i += T) {
            cpx<R> a = buf[lpad(i)], b = buf[lpad(i + N3)], c = buf[lpad(i + 2 * N3)];
            b = cmul(b, twiddle<R, DIR>(tw, i));
            c = cmul(c, twiddle<R, DIR>(tw, 2 * i));
            const cpx<R> s1 = cadd(b, c), d1 = csub(b, c);
            const cpx<R> m1 = {a.x - R(0.5) * s1.x, a.y - R(0.5) * s1.y};
            const cpx<R> rot = {-hs * d1.y, hs * d1.x};         // DIR i sin(2 pi/3) (b - c)
            buf[lpad(i)] = cadd(a, s1);
            buf[lpad(i + N3)] = cadd(m1, rot);
            buf[lpad(i + 2 * N3)] = csub(m1, rot);
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = buf[lpad(j + m * T)];
    }
}

}  // namespace wsg
