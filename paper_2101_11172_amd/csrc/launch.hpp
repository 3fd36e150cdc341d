// Host-side launchers of the tile and FFT kernels, compiled in their own units
// (one per stage family and precision, built in parallel) and called by the
// launch sequences in wsgrid.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace wsg {

// HIP events around a stage while stage timing is enabled on this thread
// (wsg_stage_timing); defined in wsgrid.hip.
struct StageMark {
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    StageMark(hipStream_t s_, int st);
    ~StageMark();
};

// Whether the tile kernels are compiled for widths (W on u, v; Wz on w) and
// one design on all axes (same) or a w-axis design of its own.
bool tiles_supported(int W, int Wz, bool same);

// One launch of the 3-D scatter (grid) or gather over the occupied tiles of a
// layer pass; false when (W, Wz, same) is not compiled.  vis (grid only):
// non-null when rec holds a shared binning's degridding records, whose values
// the scatter then takes from vis.
template <typename R>
bool launch_tiles(bool grid, int W, int Wz, bool same, int nblocks, const Rec<R>* rec, const uint32_t* start,
                  const uint32_t* cls, const uint32_t* tlist, const uint32_t* tpos, const DevParams& P,
                  const R* coef, const R* coefz, const cpx<R>* vis, cpx<R>* stack, cpx<R>* part, size_t part_stride,
                  hipStream_t s);

// FFT lengths N' the passes are compiled for: 2^a and 3 2^a from 64 to 8192.
bool fft_supported(int Np);

// One layer pass of the FFT stages (pass A, transpose, pass B with the
// w-screen; or their adjoints); false when N' is not compiled.
template <typename R>
bool launch_fft(bool grid, const DevParams& P, const uint8_t* occ, const uint8_t* rows, cpx<R>* stack, cpx<R>* inter,
                cpx<R>* inter2, const cpx<R>* tw, const R* corr, const R* image, R* dirty, hipStream_t s);

}  // namespace wsg
