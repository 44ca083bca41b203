// fdas_spectrum_noalloc: the spectra and median normalisations of
// fdas_spectrum without a plan and without any allocation.
//
// The FFT ping-pong buffers, the per-series scales and norms and the
// median-select histograms live in one file-scope device array of fixed size
// (FDAS_NOALLOC_SCRATCH_BYTES, held by every GPU the library runs on until the process
// ends). Its device address is looked up once per device with
// hipGetSymbolAddress while that device is current; host code passes only
// that address to kernels (the array's name is a host-side stand-in).
//
// Every call on one GPU shares that GPU's array and leaves its contents
// behind: the kernels overwrite the FFT buffers completely and the median
// kernels clear their histograms before counting, so nothing has to start at
// zero, but calls that overlap on one GPU (other streams or host threads)
// race.
#include "fdas_internal.h"

#include <mutex>

namespace fdas {
namespace {

constexpr size_t kScratchBytes = (size_t)FDAS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device address of this device's scratch array (looked up once per device).
hipError_t scratch_of(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace fdas

using namespace fdas;

extern "C" fdas_status fdas_spectrum_noalloc(const float *series_dev, int64_t nsamp, int32_t nseries,
                                             float *spec_dev, double *norm_host, void *stream) {
    if (!series_dev || ((uintptr_t)series_dev & 7) || !spec_dev || ((uintptr_t)spec_dev & 7))
        return FDAS_E_INVAL;
    if (nseries < 1 || nseries > 65535 || nsamp < 8 || (nsamp & 1)) return FDAS_E_INVAL;
    if (!fft_length_supported(nsamp)) return FDAS_E_UNSUPPORTED;
    const int64_t half = nsamp / 2;
    // scratch layout: FFT buffer w0 [nseries][half], scales, norms, median scratch
    const size_t fft_bytes = align256((size_t)nseries * (size_t)half * sizeof(float2));
    const size_t scale_bytes = align256((size_t)nseries * sizeof(float));
    const size_t norm_bytes = align256((size_t)nseries * sizeof(double));
    const size_t med_bytes = align256(median_scratch_bytes(nseries));
    if ((size_t)half > kScratchBytes / sizeof(float2) ||
        fft_bytes + scale_bytes + norm_bytes + med_bytes > kScratchBytes)
        return FDAS_E_INVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return FDAS_E_DEVICE;
    }
    void *base = nullptr;
    if (scratch_of(dev, &base) != hipSuccess) {
        (void)hipGetLastError();
        return FDAS_E_DEVICE;
    }
    unsigned char *b = static_cast<unsigned char *>(base);
    float2 *w0 = reinterpret_cast<float2 *>(b);
    float *scale = reinterpret_cast<float *>(b + fft_bytes);
    double *norm = reinterpret_cast<double *>(b + fft_bytes + scale_bytes);
    void *med = b + fft_bytes + scale_bytes + norm_bytes;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float2 *spec = reinterpret_cast<float2 *>(spec_dev);
    if (launch_rfft(series_dev, nsamp, nseries, w0, spec, half + 1, st) != hipSuccess ||
        launch_median_scale(spec, half + 1, half, nseries, scale, norm, med, st) != hipSuccess) {
        (void)hipGetLastError();
        return FDAS_E_DEVICE;
    }
    if (norm_host &&
        hipMemcpyAsync(norm_host, norm, (size_t)nseries * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) {
        (void)hipGetLastError();
        return FDAS_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return FDAS_E_DEVICE;
    }
    return FDAS_OK;
}
