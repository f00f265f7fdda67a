// apply_hs.hip -- instantiation of the hot path for kernel family 3 (the
// elastic half-space of eq. 9).
#include "volume_impl.hpp"

namespace bemfft {

template <>
int apply_kind<3>(int precision, const ApplyArgs &a, hipStream_t st, hipEvent_t *ev) {
    if (precision == BEMFFT_FP32) return Launch<float, 3>::run(a, st, ev);
    return Launch<double, 3>::run(a, st, ev);
}

template <>
int apply_batch_kind<3>(int precision, const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
    if (precision == BEMFFT_FP32) return Launch<float, 3>::run_batch(dm, io, g, st);
    return Launch<double, 3>::run_batch(dm, io, g, st);
}

template <>
int volume_kind<3>(int precision, const ApplyArgs &a, double *out, hipStream_t st, hipEvent_t *ev) {
    if (precision == BEMFFT_FP32) return VolumeLaunch<float, 3>::run(a, out, st, ev);
    return VolumeLaunch<double, 3>::run(a, out, st, ev);
}

}  // namespace bemfft
