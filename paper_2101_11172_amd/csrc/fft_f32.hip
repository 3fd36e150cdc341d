// FFT-pass launchers, float32.
#include "launch_fft.inl"

namespace wsg {

bool fft_supported(int Np) {
    switch (Np) {
#define WSG_N(n) \
    case n: return true;
        WSG_FFT_SIZES(WSG_N)
#undef WSG_N
        default: return false;
    }
}

template bool launch_fft<float>(bool, const DevParams&, const uint8_t*, const uint8_t*, cpx<float>*, cpx<float>*,
                                cpx<float>*, const cpx<float>*, const float*, const float*, float*, hipStream_t);

}  // namespace wsg
