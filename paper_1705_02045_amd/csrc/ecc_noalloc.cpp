// The stream-ordered integer curve without any allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops
// that forbid it).  Its scratch is one statically sized device array per GPU:
// the status block, the 16-bit changes vector, the changes vector, the merge
// stage rows and the per-workgroup count rows, in that order.  The launch's
// workgroups are capped at kMaxRows so that its count rows always fit (a
// larger image gives each workgroup more tiles), so no image the integer
// path takes needs more than the array holds.
#include <mutex>

#include "ecc_internal.h"

namespace ecc {
namespace {

constexpr int kMaxRows = 1024;           // workgroups of one launch
constexpr size_t kMaxBins = 16384;       // bins of one launch's histograms (u8: 256)
constexpr size_t kAlign = 256;
constexpr size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kOffStatus = 0;
constexpr size_t kOffVcec16 = kOffStatus + up(kStatusBytes);
constexpr size_t kOffVcec = kOffVcec16 + up(65536 * sizeof(int64_t));
constexpr size_t kOffStage = kOffVcec + up(kMaxBins * sizeof(int64_t));
constexpr size_t kStageRows = 32;        // merge_stage_rows(kMaxRows)
constexpr size_t kOffPartial = kOffStage + up(kStageRows * kMaxBins * sizeof(int64_t));
constexpr size_t kScratchBytes = kOffPartial + up((size_t)kMaxRows * kMaxBins * sizeof(int32_t));  // 68.6 MiB

// Each GPU holds its own copy until the process ends.  Host code never uses
// this name as an address: the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t *g_scratch[kMaxDevices] = {};

int scratch_for_current_device(uint8_t **out) {
    int dev = -1;
    ECC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("ecc_compute_async_noalloc: device %d beyond the %d this library tracks", dev, kMaxDevices);
        return ECC_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch[dev] = (uint8_t *)p;
    }
    *out = g_scratch[dev];
    return ECC_OK;
}

}  // namespace
}  // namespace ecc

using namespace ecc;

extern "C" int ecc_compute_async_noalloc(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype,
                                         int64_t *chi_dev, uint32_t *status_dev, void *stream) {
    g_err_clear();
    static_assert(kStageRows >= 32, "stage rows of the merge for kMaxRows rows");
    uint8_t *base = nullptr;
    int rc = scratch_for_current_device(&base);
    if (rc) return rc;
    Workspace ws;
    ws.fixed = true;
    ws.max_grid = kMaxRows;
    ws.status = (uint32_t *)(base + kOffStatus);
    ws.vcec16 = (int64_t *)(base + kOffVcec16);
    ws.vcec16_bytes = 65536 * sizeof(int64_t);
    ws.vcec = (int64_t *)(base + kOffVcec);
    ws.vcec_bytes = kMaxBins * sizeof(int64_t);
    ws.stage = (int64_t *)(base + kOffStage);
    ws.stage_bytes = kStageRows * kMaxBins * sizeof(int64_t);
    ws.partial = (int32_t *)(base + kOffPartial);
    ws.partial_bytes = (size_t)kMaxRows * kMaxBins * sizeof(int32_t);
    // The array keeps the last call's contents: the status words start at
    // zero here (a fill kernel; the kernels set bits in them).  Every other
    // region is overwritten before it is read (the count rows by their
    // workgroups, the stage rows and changes vector by the merge, the 16-bit
    // changes vector cleared by its own pass).
    rc = launch_zero(ws.status, 16, (hipStream_t)stream);
    if (rc) return rc;
    return compute_async_ws(image_dev, dims, dtype, chi_dev, status_dev, (hipStream_t)stream, &ws);
}
