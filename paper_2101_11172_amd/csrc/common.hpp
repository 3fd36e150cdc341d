// Device-side types shared by the wsgrid kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsg {

template <typename R>
struct cpx {
    R x, y;
};

// Store of a complex value that is read back only by a later kernel (the FFT
// intermediates): non-temporal, so it streams through the caches.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream(cpx<float>* p, cpx<float> v) {
    __builtin_nontemporal_store(nt_f2{v.x, v.y}, reinterpret_cast<nt_f2*>(p));
}
__device__ __forceinline__ void store_stream(cpx<double>* p, cpx<double> v) {
    __builtin_nontemporal_store(nt_d2{v.x, v.y}, reinterpret_cast<nt_d2*>(p));
}

template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }

// exp(i 2 pi f) for a phase f given in turns, reduced to [-1/2, 1/2] in float64
// first.  Float32: the hardware sine and cosine, which take their argument in
// turns (one instruction each; absolute error <= 1.2e-7, RMS 4.9e-8 and no
// bias over [-1/2, 1/2], measured against float64 on 2^24 points).
__device__ __forceinline__ void phase_turns(double f, float* s, float* c) {
    const float r = float(f - rint(f));
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
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
    int Wz;                 // width of the w-axis gridding function (W: the same on all axes)
    int tclamp;             // original W-stacking: the last w bin is closed at wmax
    double wshift;          // w' = n_scale w + wshift (original W-stacking: -1/2)
    double tphase;          // layer t's w-screen uses t + tphase (original W-stacking: bin midpoints, 1/2)
    int nbr, nbs, nbt;      // bins (= tiles) along r (u), s (v), t (w) of one channel
    // Channels of a batched call: channel c's layers are the virtual layers
    // [c chl, c chl + n_layers) with chl = nbt kTileT (its tile layers follow
    // the previous channel's); virtual layers beyond n_layers in a channel are
    // padding that nothing reads or writes.  One channel: virtual = plain.
    int nch;
    // layer pass: virtual layers [pl0, pl0 + pln) (pl0 a multiple of kTileT)
    // sit in the stack and FFT buffers, local layer index t - pl0
    int pl0, pln;
    double umul;            // l_max / x0: u -> u'
    double nscale;          // w -> w'
    double zshift;          // (1 - n0) / n_scale: z = (n - 1) / n_scale + zshift
    double wmax;
    double dl;              // pixel size L / N
};

constexpr int kTileR = 16, kTileS = 16, kTileT = 16;

// blockIdx -> logical block so that each XCD (blocks are dealt round-robin to
// the 8 XCDs) walks a contiguous range of logical blocks.  For uniform work
// (the FFT passes): neighbouring lines share cache lines in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    int per = n >> 3, rem = n & 7;
    int x = b & 7, i = b >> 3;
    return x * per + min(x, rem) + i;
}

// blockIdx -> logical block dealing groups of G consecutive logical blocks to
// the XCDs in turn.  For the tile kernels, whose work is concentrated in the
// dense centre of the uv plane: the load spreads over all XCDs while runs of G
// neighbouring tiles (which share visibility bins) stay on one L2.  The last
// partial round keeps the identity mapping so the result is a permutation.
template <int G>
__device__ __forceinline__ int xcd_interleave(int b, int n) {
    const int full = (n / (8 * G)) * (8 * G);
    if (b >= full) return b;
    const int x = b & 7, i = b >> 3;
    return (i / G) * (8 * G) + x * G + (i % G);
}

}  // namespace wsg
