// Tile-kernel launchers for one precision (included by tiles_f32.hip and
// tiles_f64.hip, which instantiate them).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"

namespace wsg {

// The (W, Wz) pairs with a w-axis design of their own: W = 7 with every
// narrower or equal w width (the accuracy trade-off of Sec. 6.1 and the
// original W-stacking's W_z = 1 of Table 2 rows a-c), and W_z = 1 beside
// W = 3 .. 8.  One design on all axes is compiled for every W in 1 .. 16.
#define WSG_OWN_Z_PAIRS(X) \
    X(7, 1) X(7, 2) X(7, 3) X(7, 4) X(7, 5) X(7, 6) X(7, 7) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(8, 1)
#define WSG_SAME_WIDTHS(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <typename R, int W, int WZ, bool SAME>
void launch_tiles_w(bool grid, int nblocks, const Rec<R>* rec, const uint32_t* start, const uint32_t* cls,
                    const uint32_t* tlist, const uint32_t* tpos, const DevParams& P, const R* coef, const R* coefz,
                    const cpx<R>* vis, cpx<R>* stack, cpx<R>* part, size_t part_stride, hipStream_t s) {
    if (grid && vis)
        hipLaunchKernelGGL((k_grid_tiles<R, W, WZ, SAME, true>), dim3(nblocks), dim3(ScatterCfg<R, W, WZ>::kThreads),
                           0, s, rec, start, cls, tlist, tpos, P, coef, coefz, vis, stack);
    else if (grid)
        hipLaunchKernelGGL((k_grid_tiles<R, W, WZ, SAME, false>), dim3(nblocks), dim3(ScatterCfg<R, W, WZ>::kThreads),
                           0, s, rec, start, cls, tlist, tpos, P, coef, coefz, (const cpx<R>*)nullptr, stack);
    else
        hipLaunchKernelGGL((k_degrid_tiles<R, W, WZ, SAME>), dim3(nblocks), dim3(256), 0, s, rec, start, cls, tlist,
                           tpos, P, coef, coefz, (const cpx<R>*)stack, part, part_stride);
}

template <typename R>
bool launch_tiles(bool grid, int W, int Wz, bool same, int nblocks, const Rec<R>* rec, const uint32_t* start,
                  const uint32_t* cls, const uint32_t* tlist, const uint32_t* tpos, const DevParams& P,
                  const R* coef, const R* coefz, const cpx<R>* vis, cpx<R>* stack, cpx<R>* part, size_t part_stride,
                  hipStream_t s) {
    if (same) {
        if (Wz != W) return false;
        switch (W) {
#define WSG_SAME(w)                                                                                          \
    case w:                                                                                                   \
        launch_tiles_w<R, w, w, true>(grid, nblocks, rec, start, cls, tlist, tpos, P, coef, coefz, vis, stack,  \
                                      part, part_stride, s);                                                  \
        return true;
            WSG_SAME_WIDTHS(WSG_SAME)
#undef WSG_SAME
            default: return false;
        }
    }
#define WSG_OWN(w, wz)                                                                                          \
    if (W == w && Wz == wz) {                                                                                 \
        launch_tiles_w<R, w, wz, false>(grid, nblocks, rec, start, cls, tlist, tpos, P, coef, coefz, vis, stack, \
                                        part, part_stride, s);                                                  \
        return true;                                                                                           \
    }
    WSG_OWN_Z_PAIRS(WSG_OWN)
#undef WSG_OWN
    return false;
}

}  // namespace wsg
