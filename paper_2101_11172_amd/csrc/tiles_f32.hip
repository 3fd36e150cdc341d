// Tile-kernel launchers, float32.
#include "launch_tiles.inl"

namespace wsg {

bool tiles_supported(int W, int Wz, bool same) {
    if (same) return Wz == W && W >= 1 && W <= 16;
#define WSG_OWN_Q(w, wz) \
    if (W == w && Wz == wz) return true;
    WSG_OWN_Z_PAIRS(WSG_OWN_Q)
#undef WSG_OWN_Q
    return false;
}

template bool launch_tiles<float>(bool, int, int, bool, int, const Rec<float>*, const uint32_t*, const uint32_t*,
                                  const uint32_t*, const uint32_t*, const DevParams&, const float*, const float*,
                                  const cpx<float>*, cpx<float>*, cpx<float>*, size_t, hipStream_t);

}  // namespace wsg
