// FFT-pass launchers, float64.
#include "launch_fft.inl"

namespace wsg {

template bool launch_fft<double>(bool, const DevParams&, const uint8_t*, const uint8_t*, cpx<double>*, cpx<double>*,
                                 cpx<double>*, const cpx<double>*, const double*, const double*, double*, hipStream_t);

}  // namespace wsg
