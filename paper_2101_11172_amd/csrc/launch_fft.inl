// FFT-pass launchers for one precision (included by fft_f32.hip and
// fft_f64.hip, which instantiate them).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "launch.hpp"

namespace wsg {

// r_in: the stack frequency r is the input row index (grid), else the output's.
// 512 threads per 64 x 64 tile (8 elements each) measured fastest (256: 1.45 ms,
// 512: 1.04 ms, 1024: 1.18 ms per wide-field transpose).
template <typename R>
void transpose(const DevParams& P, const cpx<R>* in, cpx<R>* out, int A, int B, bool r_in, const uint8_t* rows,
               hipStream_t s) {
    constexpr int TH = 512;
    const unsigned blocks = unsigned(P.pln) * unsigned((A + 63) / 64) * unsigned((B + 63) / 64);
    const int chl = P.nch > 1 ? P.nbt * kTileT : 0;     // 0: one channel, no padding layers to skip
    if (r_in)
        hipLaunchKernelGGL((k_transpose<R, TH, true>), dim3(blocks), dim3(TH), 0, s, in, out, A, B, rows, P.nbr,
                           P.pl0, chl, P.n_layers);
    else
        hipLaunchKernelGGL((k_transpose<R, TH, false>), dim3(blocks), dim3(TH), 0, s, in, out, A, B, rows, P.nbr,
                           P.pl0, chl, P.n_layers);
}

// One layer pass of the FFT stages.  Pass B (along u / p, with the w-screen)
// runs once per channel segment of the pass: the virtual layers of channel c
// in the pass, whose map is dirty + c N^2 (grid, written by the channel's first
// segment and added to by later ones) or image + c N^2 (degrid).
template <typename R, int NP>
void launch_fft_n(bool grid, const DevParams& P, const uint8_t* occ, const uint8_t* rows, cpx<R>* stack, cpx<R>* inter,
                  cpx<R>* inter2, const cpx<R>* tw, const R* corr, const R* image, R* dirty, hipStream_t s) {
    using C = FftCfg<R, NP>;
    const unsigned grid_a = unsigned(P.pln) * unsigned(C::N / kTileR);
    const unsigned grid_b = unsigned((P.N + C::kNLr - 1) / C::kNLr);
    const int chl = P.nbt * kTileT;
    const size_t map = size_t(P.N) * size_t(P.N);
    auto segments = [&](auto&& fn) {
        for (int c = P.pl0 / chl; c < P.nch && c * chl < P.pl0 + P.pln; ++c) {
            const int lo = std::max(P.pl0, c * chl), hi = std::min(P.pl0 + P.pln, c * chl + P.n_layers);
            if (hi > lo) fn(c, lo, hi);
        }
    };
    if (grid) {
        {
            StageMark mark(s, 2);
            hipLaunchKernelGGL((k_grid_fft_a<R, NP>), dim3(grid_a), dim3(C::kNLt * C::T), 0, s,
                               (const cpx<R>*)stack, occ, inter, tw, P.N, P.n_layers, P.nch > 1 ? chl : 0, P.nbr,
                               P.pl0);
        }
        {
            StageMark mark(s, 8);
            transpose<R>(P, inter, inter2, P.Np, P.N, true, rows, s);     // [t][r][q] -> [t][q][r]
        }
        StageMark mark(s, 3);
        segments([&](int c, int lo, int hi) {
            DevParams Q = P;
            Q.pln = hi - lo;
            hipLaunchKernelGGL((k_grid_fft_b<R, NP>), dim3(grid_b), dim3(C::kNLr * C::T), 0, s,
                               (const cpx<R>*)inter2, rows, tw, corr, dirty + size_t(c) * map, Q, lo - P.pl0,
                               lo - c * chl, lo > c * chl ? 1 : 0);
        });
    } else {
        {
            StageMark mark(s, 5);
            segments([&](int c, int lo, int hi) {
                DevParams Q = P;
                Q.pln = hi - lo;
                hipLaunchKernelGGL((k_degrid_fft_b<R, NP>), dim3(grid_b), dim3(C::kNLr * C::T), 0, s,
                                   image + size_t(c) * map, corr, tw, rows, inter, Q, lo - P.pl0, lo - c * chl);
            });
        }
        {
            StageMark mark(s, 9);
            transpose<R>(P, inter, inter2, P.N, P.Np, false, rows, s);    // [t][q][r] -> [t][r][q]
        }
        StageMark mark(s, 6);
        hipLaunchKernelGGL((k_degrid_fft_a<R, NP>), dim3(grid_a), dim3(C::kNLt * C::T), 0, s,
                           (const cpx<R>*)inter2, occ, tw, stack, P.N, P.n_layers, P.nch > 1 ? chl : 0, P.nbr,
                           P.pl0);
    }
}

#define WSG_FFT_SIZES(X) \
    X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096) X(6144) X(8192)

template <typename R>
bool launch_fft(bool grid, const DevParams& P, const uint8_t* occ, const uint8_t* rows, cpx<R>* stack, cpx<R>* inter,
                cpx<R>* inter2, const cpx<R>* tw, const R* corr, const R* image, R* dirty, hipStream_t s) {
    switch (P.Np) {
#define WSG_N(n) \
    case n: launch_fft_n<R, n>(grid, P, occ, rows, stack, inter, inter2, tw, corr, image, dirty, s); return true;
        WSG_FFT_SIZES(WSG_N)
#undef WSG_N
        default: return false;
    }
}

}  // namespace wsg
