// apply_l3d.hip -- instantiation of the hot path for kernel family 1.
#include "volume_impl.hpp"
#include "zpass16.hpp"

namespace bemfft {

template <>
int apply_kind<1>(int precision, const ApplyArgs &a, hipStream_t st, hipEvent_t *ev) {
    if (precision == BEMFFT_BF16_MFMA) return Launch16<1>::run(a, st, ev);
    if (precision == BEMFFT_FP32) return Launch<float, 1>::run(a, st, ev);
    return Launch<double, 1>::run(a, st, ev);
}

template <>
int apply_batch_kind<1>(int precision, const ApplyArgs *dm, const BatchIO *io, const GroupDims &g, hipStream_t st) {
    if (precision == BEMFFT_BF16_MFMA) {
        set_error("batches of 16-bit plans are not supported");
        return BEMFFT_EINVAL;
    }
    if (precision == BEMFFT_FP32) return Launch<float, 1>::run_batch(dm, io, g, st);
    return Launch<double, 1>::run_batch(dm, io, g, st);
}

template <>
int volume_kind<1>(int precision, const ApplyArgs &a, double *out, hipStream_t st, hipEvent_t *ev) {
    if (precision == BEMFFT_BF16_MFMA) return VolumeLaunch16<1>::run(a, out, st, ev);
    if (precision == BEMFFT_FP32) return VolumeLaunch<float, 1>::run(a, out, st, ev);
    return VolumeLaunch<double, 1>::run(a, out, st, ev);
}

}  // namespace bemfft
