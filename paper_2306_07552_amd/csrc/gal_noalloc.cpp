// Allocation-free surrogate inference (declared in include/gal.h): the same
// launches as gal_mlp_forward, with their scratch (the first layer's partial
// sums) in a fixed device array of the library instead of the MLP object, for
// callers that cannot allocate device memory.
#include "gal.h"
#include "gal_mlp.h"

#include <mutex>

namespace gal {
int api_fail(int code, const char *fmt, ...);
}

namespace {

// Every row count needs at most 512 slabs of 32 x 256 FP32 partial sums (the
// split rule of the inference launch).
constexpr size_t kPartFloats = (size_t)512 * 32 * gal::kMlpHidden;   // 16 MiB

// The scratch, one copy per GPU, held until the process ends.  Its name is a
// host-side stand-in in host code: the device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) float scratch[kPartFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

int scratch_for_current_device(float **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gal::api_fail(GAL_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return gal::api_fail(GAL_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gal::api_fail(GAL_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = static_cast<float *>(g_scratch[dev]);
    return GAL_OK;
}

}  // namespace

extern "C" int gal_mlp_forward_static(gal_mlp *m, const uint16_t *x_dev, int32_t rows, float *logits_dev,
                                      void *stream)
{
    if (!m || !x_dev || !logits_dev) return gal::api_fail(GAL_EINVAL, "null argument");
    if (rows < 0 || rows > GAL_MLP_STATIC_MAX_ROWS)
        return gal::api_fail(GAL_EINVAL, "rows must be in [0, %d], got %d", GAL_MLP_STATIC_MAX_ROWS, rows);
    if ((uintptr_t)x_dev % 16) return gal::api_fail(GAL_EINVAL, "x_dev must be 16-byte aligned");
    if (gal::sur_infer_part_floats(rows) > kPartFloats)
        return gal::api_fail(GAL_EINVAL, "%d rows need more than the fixed scratch", rows);
    if (rows == 0) return GAL_OK;
    float *base = nullptr;
    int rc = scratch_for_current_device(&base);
    if (rc) return rc;
    // every partial sum the launch reads is written by the same call first,
    // so nothing has to start at zero
    return gal::mlp_infer_rows(m, x_dev, nullptr, rows, logits_dev, nullptr, (hipStream_t)stream, base);
}
