// Tile-kernel launchers, float64.
#include "launch_tiles.inl"

namespace wsg {

template bool launch_tiles<double>(bool, int, int, bool, int, const Rec<double>*, const uint32_t*, const uint32_t*,
                                   const uint32_t*, const uint32_t*, const DevParams&, const double*, const double*,
                                   const cpx<double>*, cpx<double>*, cpx<double>*, size_t, hipStream_t);

}  // namespace wsg
