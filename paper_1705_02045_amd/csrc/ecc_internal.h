// Internal declarations of libecc (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "ecc.h"

namespace ecc {

constexpr int kWave = 64;
constexpr uint32_t kStatusRange = ECC_STATUS_RANGE_BIT;

void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define ECC_HIP(call)                                  \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

// Source of axis-0 planes for one launch: planes [0, seg0_planes) live at
// seg0, the following planes at seg1.  Lets a chunk be read together with the
// collar planes kept from the previous chunk without copying either.
struct PlaneSrc {
    const uint8_t *seg0;
    const uint8_t *seg1;
    int64_t seg0_planes;
    int64_t plane_bytes;
};

// Integer-path view of an image: axis 0 is the walking axis, the remaining
// axes (at most two here) are the in-plane axes; nin = number of in-plane axes.
struct IntView {
    int nin;        // 1: plane is one row of n2 values; 2: plane is n1 rows of n2 values
    int64_t n0;     // planes in the whole image
    int32_t n1, n2; // in-plane extents (n1 = 1 when nin == 1)
};

// One launch of the integer kernel over planes [e0, e1) of a buffer.
struct IntJob {
    PlaneSrc src;
    IntView view;
    int32_t e0, e1;       // emitted planes, buffer coordinates
    int32_t lo_inf;       // plane e0-1 lies outside the image
    int32_t hi_inf;       // plane e1 lies outside the image
    int dtype;            // ECC_U8 or ECC_U14
};

// Tiling of the integer kernel (chosen by the tuner in ecc_tune.cpp).
struct IntTiling {
    int rows;      // rows (nin == 2) or 64-wide x segments (nin == 1) per wave
    int dbl;       // per-item update form of the four-item blocks (see ecc_int.hip)
    int wx, wy;    // waves per workgroup along x and along y
    int zc;        // planes per tile
    int grid;      // workgroups (persistent)
};

// Device scratch of one (device, stream) pair.
struct Workspace {
    int device = -1;
    void *stream = nullptr;
    int32_t *partial = nullptr;  // [grid][m] per-workgroup counts
    size_t partial_bytes = 0;
    int64_t *vcec = nullptr;     // [m] changes vector
    size_t vcec_bytes = 0;
    uint32_t *status = nullptr;  // device status word
    int64_t *chi_tmp = nullptr;  // [m] curve staging for host outputs
    size_t chi_tmp_bytes = 0;
    void *img_tmp = nullptr;     // device copy of a host image
    size_t img_tmp_bytes = 0;
};

int get_workspace(void *stream, Workspace **out);
int ensure_bytes(void **ptr, size_t *cap, size_t need);

int64_t threshold_count(int dtype);
int device_cu_count();

IntTiling choose_int_tiling(const IntView &v, int dtype, int64_t planes);

// Kernels (ecc_int.hip / ecc_scan.hip).  All enqueue on `stream`.
int launch_int_partial(const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status,
                       hipStream_t stream);
int launch_zero(void *p, size_t bytes, hipStream_t stream);
int launch_reduce_rows(const int32_t *partial, int rows, int m, int64_t *vcec, bool accumulate,
                       hipStream_t stream);
int launch_scan(const int64_t *vcec, int m, int64_t *chi, const uint32_t *status, uint32_t *status_out,
                hipStream_t stream);

bool normalize_int_view(const ecc_dims *dims, IntView *v, int *err_ndim_dropped);

// Optional event timing of the per-voxel kernels (ecc_profile.cpp).
int profile_begin(hipStream_t s, void **token);
int profile_end(hipStream_t s, void *token);

}  // namespace ecc
