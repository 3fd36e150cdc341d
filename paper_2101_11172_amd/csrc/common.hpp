// Device-side types shared by the wsgrid kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsg {

template <typename R>
struct cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }

// exp(i 2 pi f) for a phase f given in turns, reduced to [-1/2, 1/2] in float64
// first so that the float32 sine/cosine see a small argument.
__device__ __forceinline__ void phase_turns(double f, float* s, float* c) {
    double r = f - rint(f);
    sincospif(2.0f * float(r), s, c);
}
__device__ __forceinline__ void phase_turns(double f, double* s, double* c) {
    double r = f - rint(f);
    sincospi(2.0 * r, s, c);
}

// One binned visibility.  ruv packs the first support index along u (low 16
// bits) and v (high 16 bits), both taken modulo N'; rt is the first support
// layer counted from t_lo.  nu are the fractional offsets in [-1/2, 1/2).
// grid:   v = V exp(+i 2 pi w (n0 - 1)), conjugated first if folded; idx unused.
// degrid: v = exp(-i 2 pi w (n0 - 1)); idx = k | (folded << 31).
template <typename R>
struct Rec {
    uint32_t ruv;
    uint32_t rt;
    R nu[3];
    R v[2];
    uint32_t idx;
};

// Scalars every kernel needs, passed by value.
struct DevParams {
    int N, Np, W, n_layers, t_lo;
    int nbr, nbs, nbt;      // bins (= tiles) along r (u), s (v), t (w)
    int degree;             // kernel polynomial degree
    double umul;            // l_max / x0: u -> u'
    double nscale;          // w -> w'
    double z0;
    double wmax;
    double dl;              // pixel size L / N
};

constexpr int kTileR = 16, kTileS = 16, kTileT = 16;

// blockIdx -> logical block so that each XCD (blocks are dealt round-robin to
// the 8 XCDs) walks a contiguous range of logical blocks: neighbouring tiles
// share their visibility bins in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    int per = n >> 3, rem = n & 7;
    int x = b & 7, i = b >> 3;
    return x * per + min(x, rem) + i;
}

}  // namespace wsg
