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
constexpr uint32_t kStatusNaN = 2u;  // a float image holds a NaN
// Device status block (1024 bytes per workspace or stream): word 0 status,
// word 1 its copy taken by the scan, word 2 the copy handed to the host,
// words 8-9 a value range, bytes [kStatusTotalsOffset, +512) the scan's
// group totals.
constexpr size_t kStatusBytes = 1024;
constexpr size_t kStatusTotalsOffset = 128;
constexpr size_t kStatusMinMaxOffset = 32;  // two words: minimum and maximum of a 16-bit image

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Logical index of workgroup b of a grid of G: the workgroups of one XCD
// take one contiguous range of indices (a bijection of [0, G)), so that
// neighbouring work shares an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
    const uint32_t q = G / 8, rem = G % 8, x = b % 8;
    return x * q + (x < rem ? x : rem) + b / 8;
}

void set_error(const char *fmt, ...);
void g_err_clear();
int hip_fail(hipError_t e, const char *what);

#define ECC_HIP(call)                                  \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

// Source of axis-0 planes for one launch.  Plane p of a launch (buffer coordinates) is read at base + p * plane_bytes
// for p >= 0 and at lo_base + p * plane_bytes for p < 0: a launch can start in
// a second buffer that holds the planes just before `base` (the carried
// planes of a stream).  lo_base = base when there is no such buffer.
struct PlaneSrc {
    const uint8_t *base;
    const uint8_t *lo_base;
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
    int invert;           // values read as M-1-v (largest-value convention)
    int32_t win_shift;    // ECC_U16: the launch counts bin = clamp(v - win_shift, 0, 16383)
    // ECC_U16 in 32768-bin passes: 1 = every value lies in [win_shift,
    // win_shift + 32768) and the launch counts bin = v - win_shift; 2 = the
    // same for the values in that range, the others skipped; 0 = a window
    // as above
    int range_pass;
    uint32_t *high_flag;  // range passes: set to 1 when a value >= 32768 is loaded (may be null)
};

// Tiling of the integer kernel (chosen by choose_int_tiling in ecc_api.cpp).
struct IntTiling {
    int rows;      // rows (nin == 2) or 64-wide x segments (nin == 1) per wave
    int mode;      // update form of the four-item groups (0..3, see ecc_int.hip)
    int pd;        // planes of raw loads in flight ahead of the compared plane
    int wx, wy;    // waves per workgroup along x and along y
    int zc;        // planes per tile
    int per_wg;    // tiles walked by one workgroup into one histogram (at most)
    int tile_stride;  // 0: a workgroup walks per_wg consecutive tiles; 1: tiles strided by the grid
    int grid;      // workgroups = ceil(tiles / per_wg)
    int pair = 1;  // row-pair layout allowed (used where the shape and alignment permit)
};

// Device scratch of one (device, stream) pair.
struct Workspace {
    int device = -1;
    void *stream = nullptr;
    int32_t *partial = nullptr;  // [grid][m] per-workgroup counts
    size_t partial_bytes = 0;
    int64_t *vcec = nullptr;     // [m] changes vector
    size_t vcec_bytes = 0;
    uint32_t *status = nullptr;  // device status block (kStatusBytes)
    // A pinned, coherent host block of 16 words: word 0, the status that the
    // scan writes (read after the stream is synchronized, without a
    // device-to-host copy); word 1, the 16-bit path's high-value flag; words
    // 2-3, the float path's record count; words 4-11, the float key sort's
    // top-byte mask.  With its device-side address.
    volatile uint32_t *host_status = nullptr;
    uint32_t *host_status_dev = nullptr;
    int64_t *stage = nullptr;    // merge stage rows
    size_t stage_bytes = 0;
    int64_t *chi_tmp = nullptr;  // [m] curve staging for host outputs
    size_t chi_tmp_bytes = 0;
    void *img_tmp = nullptr;     // device copy of a host image
    size_t img_tmp_bytes = 0;
    void *fbuf = nullptr;        // float path: keys, record regions, sort scratch, curve staging
    size_t fbuf_bytes = 0;
    void *frec = nullptr;        // float path: the dense records (two buffers) and their prefix
    size_t frec_bytes = 0;
    void *dual_buf = nullptr;    // dual complex: gathered faces of the box, per-face curves
    size_t dual_buf_bytes = 0;
    void *i2f_buf = nullptr;     // integer images through the float path: float copy, float curve, expanded curve
    size_t i2f_buf_bytes = 0;
    int64_t *vcec16 = nullptr;   // [65536] changes vector of a 16-bit image (window passes)
    size_t vcec16_bytes = 0;
    // Fixed scratch (the entry point that allocates nothing): the buffers
    // above point into memory the library does not own and never grow;
    // ws_ensure fails instead of allocating.  max_grid caps the workgroup
    // count of a launch (0: no cap) so the count rows fit.
    bool fixed = false;
    int max_grid = 0;
};

// hipMalloc / hipHostMalloc through the allocation-failure injection hook
// (ECC_FAIL_ALLOC, ecc_api.cpp); every allocation of the library uses them.
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t host_malloc(void **p, size_t bytes, unsigned flags);

int get_workspace(void *stream, Workspace **out);
int ensure_bytes(void **ptr, size_t *cap, size_t need);
// ensure_bytes for a buffer of ws: grows it, or on a fixed workspace fails
// with ECC_E_NOMEM when the buffer is smaller than need.
int ws_ensure(Workspace *ws, void **ptr, size_t *cap, size_t need);
// The stream-ordered integer curve of a device image (ecc_compute_async's
// work) with the scratch of ws.
int compute_async_ws(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, int64_t *chi_dev,
                     uint32_t *status_dev, hipStream_t stream, Workspace *ws);

int64_t threshold_count(int dtype);
int device_cu_count();

IntTiling choose_int_tiling(const IntView &v, int dtype, int64_t planes, int max_grid = 0);
// The tiling of a 16-bit launch in 32768-bin passes (IntJob::range_pass).
IntTiling range_pass_tiling(const IntView &v, int64_t planes);

// Kernels (ecc_int.hip / ecc_scan.hip).  All enqueue on `stream`.
// zero_vcec: when not null, workgroup 0 clears m int64 entries there first.
int launch_int_partial(const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status,
                       int64_t *zero_vcec, hipStream_t stream);
int launch_zero(void *p, size_t bytes, hipStream_t stream);
// 16-bit images (m = 65536): one launch counts one window of 16384 bins,
// bin = clamp(v - shift, 0, 16383); bins [klo, khi] are values
// [shift + klo, shift + khi] (bin 0 / 16383 are guards where values lie
// below / above the window).  Windows for values [vmin, vmax], at most
// kU16MaxWindows; returns their number.
struct U16Window {
    int32_t shift;
    int klo, khi;
};
constexpr int kU16MaxWindows = 5;  // 16383 + 3 * 16382 + 16383 >= 65536
int plan_u16_windows(uint32_t vmin, uint32_t vmax, U16Window *w);
// The whole curve of a device-resident 16-bit image on stream (windows over
// the whole value range), the status copied to status_out (may be null).
int u16_curve_async(const void *image_dev, const IntView &v, int64_t *chi_dev, uint32_t *status_out,
                    hipStream_t stream);
// Column sums of the per-workgroup rows into vcec through int64 stage rows
// ([merge_stage_rows(rows)][m]) and, with do_scan, the prefix sum of vcec into
// chi (ecc_scan.hip).  The scan copies the status word to status_out (when
// not null) and clears it.
int merge_stage_rows(int rows);
int launch_merge(const int32_t *partial, int rows, int m, int64_t *stage, int64_t *vcec, bool accumulate,
                 bool do_scan, int64_t *chi, uint32_t *status, uint32_t *status_out, hipStream_t stream,
                 bool reverse = false);

// Copies the n0 x n1 x n2 sub-array of src starting at element `base` with
// element strides s0, s1, s2 into dst (contiguous, C order).
int launch_gather(const void *src, int elem, int64_t base, int64_t s0, int64_t s1, int64_t s2, int64_t n0,
                  int64_t n1, int64_t n2, void *dst, hipStream_t stream);
// Minimum and maximum of n uint16 values into out[0], out[1].
int launch_minmax_u16(const uint16_t *img, int64_t n, uint32_t *out, hipStream_t stream);
// out[t] = sign * sum_f (-1)^((neg_mask >> f) & 1) * curves[f * m + t], t < m.
// (faces f < 128: bit f of the pair {mask[0], mask[1]})
int launch_signed_sum(const int64_t *curves, int nf, const uint64_t neg_mask[2], const uint64_t skip_mask[2],
                      int sign, int m, int64_t *out, hipStream_t stream);
// A face of the box of at most one dimension: elements base + i * stride,
// i < len (len = 0: a corner, the single element at base), added with sign.
struct LowFace {
    int64_t base, stride, len;
    int64_t sign;
};
// Largest-value changes vectors of such faces, added into out (ecc_scan.hip).
int launch_low_faces(const void *img, int elem, const LowFace *faces_dev, int nfaces, int m, int64_t *out,
                     hipStream_t stream);

bool normalize_int_view(const ecc_dims *dims, IntView *v, int *err_ndim_dropped);
int check_dims(const ecc_dims *dims, int64_t *total);
size_t elem_bytes(int dtype);

// Batched integer path (ecc_int.hip, ecc_scan.hip, ecc_batch.cpp).  The
// per-image kernel parameters are opaque to the host code: kparams_bytes()
// bytes each, filled by fill_kparams().
size_t kparams_bytes();
void fill_kparams(void *dst, const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status);
// Table of one batched run, built on the host and copied to the device as a
// whole (offsets in bytes from the table start).  The copy also resets the
// tile kernel's work counter.
struct BatchHeader {
    int32_t njobs;
    int32_t ntiles;           // workgroup-tiles over all images
    int32_t nitems;           // (image, 1024-column group) items of the merge
    uint32_t next_tile;       // work counter of the tile kernel (0 in the copied table)
    uint32_t off_kparams;     // KParams[njobs], kparams_bytes() each
    uint32_t off_tile_begin;  // int32[njobs + 1]: prefix of the images' tiles
    uint32_t off_kind;        // int32[njobs]: (dtype == U14) * 2 + (nin == 2)
    uint32_t off_merge;       // MergeJob[njobs]
    uint32_t off_item_begin;  // int32[njobs + 1]: prefix of the images' column groups
    uint32_t pad[7];
};
// One persistent launch over the tiles of every image of the table: `grid`
// workgroups take tiles from the work counter until none are left.
int launch_int_persistent(const void *table_dev, int grid, hipStream_t stream);
struct MergeJob {
    const int32_t *partial;  // [rows][m]
    int32_t rows;
    int32_t m;
    int64_t *vcec;           // [m] scratch
    int64_t *chi;            // [m] output
    uint32_t *status;        // device status word of the image (cleared here)
    uint32_t *status_out;    // optional copy for the caller
};
// Batched merge of the table's images: column sums into each image's vcec,
// then each image's scan into its curve (fixed grids, loops over the work).
int launch_batch_merge(const void *table_dev, int colsum_grid, int scan_grid, hipStream_t stream);

// Float path (ecc_float.hip, ecc_sort.hip).
// The change kernel writes every voxel's order-preserving 32-bit key and,
// for the voxels whose change is not zero, (key, change) records into its
// workgroup's region: region b holds slots [b * R, (b+1) * R) of nz_key and
// nz_chg, R = slots / regions (float_regions); nz_cnt[b] and nz_off[b]
// receive the region's record count.
int64_t float_regions(const ecc_dims *dims, int64_t *slots);  // regions, or -1 with the error set
// keys may be null (not written).  [e0, e1): the axis-0 planes whose voxels
// are emitted, for an image with four axes longer than 1 (the default: all);
// the other planes are neighbours only and their regions stay empty.
int launch_float_change(const float *img_dev, const ecc_dims *dims, uint32_t *keys, uint32_t *nz_key,
                        int32_t *nz_chg, uint32_t *nz_cnt, uint32_t *nz_off, uint32_t *status, hipStream_t stream,
                        int32_t e0 = 0, int32_t e1 = INT32_MAX);
// Integer images through the change kernel: the regions' records added to
// vcec (m int64) at the records' values.
int launch_records_to_vcec(const uint32_t *nz_key, const int32_t *nz_chg, const uint32_t *nz_cnt, int64_t regions,
                           int64_t region_slots, int m, int64_t *vcec, hipStream_t stream);
// Exclusive scan of nz_off (regions entries; sums: radix_scan_tiles(regions)),
// then the record count into *total_dev and *total_host (host-mapped).
int launch_nz_total(const uint32_t *nz_cnt, uint32_t *nz_off, int64_t regions, uint32_t *sums, int64_t *total_dev,
                    int64_t *total_host, hipStream_t stream);
// The regions' records, densely, as key << 32 | (uint32) change.
int launch_nz_compact(const uint32_t *nz_key, const int32_t *nz_chg, const uint32_t *nz_cnt, const uint32_t *nz_off,
                      int64_t regions, int64_t region_slots, uint64_t *rec, hipStream_t stream);
// Tiles of the radix sort for n words of elem (4 or 8) bytes.
int64_t radix_tiles(int64_t n, int elem);
int64_t radix_scan_tiles(int64_t entries);
// Digit-table entries of a sort of n words of elem bytes (digits of up to
// 10 bits for keys, 8 for records); sums: radix_scan_tiles of that.
int64_t radix_count_entries(int64_t n, int elem);
// Sorts key[0]; on return key[0] is the sorted buffer and key[1] the other
// (the two may be swapped).  mask_dev: 8 device words; mask_host /
// mask_host_dev: 8 words of host-mapped memory, host and device views.
// Synchronizes on an event recorded early in the sort (the host reads which
// top bytes occur to choose the last passes).
int radix_sort_keys(uint32_t *key[2], int64_t n, uint32_t *counts, uint32_t *sums, uint32_t *mask_dev,
                    volatile uint32_t *mask_host, uint32_t *mask_host_dev, hipStream_t stream);
// Sorts rec[0] in place (an even number of passes).
int radix_sort_records(uint64_t *rec[2], int64_t n, uint32_t *counts, uint32_t *sums, hipStream_t stream);
int64_t float_tiles(int64_t n);
// From the sorted keys and the sorted records: the K distinct keys as
// float32 (out_keys) and the curve (out_chi), K written to *kcount.
// tile_cnt: float_tiles(n) uint32; sums: radix_scan_tiles(float_tiles(n));
// tile_sum: float_tiles(n) int64; bound: float_tiles(n) + 1 int64; prefix:
// nnz int64.
int launch_float_curve(const uint32_t *key, int64_t n, const uint64_t *rec, int64_t nnz, int64_t *prefix,
                       uint32_t *tile_cnt, uint32_t *sums, int64_t *tile_sum, int64_t *bound, int64_t *kcount,
                       float *out_keys, int64_t *out_chi, hipStream_t stream);
// Exclusive scan of n uint32 in place; sums: radix_scan_tiles(n) entries.
int exclusive_scan_u32(uint32_t *a, int64_t n, uint32_t *sums, hipStream_t stream);
// Keys where chi changes, compacted (count written on the device).
int launch_change_points(const float *keys, const int64_t *chi, int64_t K, uint32_t *pos, uint32_t *sums,
                         float *out_keys, int64_t *out_chi, int64_t *count, hipStream_t stream);
// Integer image (elem = 1 or 2 bytes) to float32 (invert: limit - 1 - v);
// values >= limit set kStatusRange.
int launch_int_to_f32(const void *img, int elem, int64_t n, uint32_t limit, int invert, float *out,
                      uint32_t *status, hipStream_t stream);
// Largest-value curve (changes = 0) or changes vector (changes = 1) from the
// smallest-value curve g of the inverted image, m entries.
int launch_reflect_curve(const int64_t *g, int m, int changes, int64_t *out, hipStream_t stream);
// out[t] = chi at the largest key <= t (0 below keys[0]), t < m.
int launch_expand_steps(const float *keys, const int64_t *chi, int64_t K, int m, int64_t *out,
                        hipStream_t stream);
// Float image to integer bins (elem = 1 or 2 bytes), NaN -> kStatusNaN.
int launch_quantize(const float *img, int64_t n, float lo, float scale, int m, int elem, void *out,
                    uint32_t *status, hipStream_t stream);

// Streaming internals for the serving loop (ecc_stream.cpp).
int stream_finish_async(ecc_stream *st, int64_t *chi_dev, uint32_t *status_dev);
int64_t stream_plane_bytes(const ecc_stream *st);

// Optional event timing of the per-voxel kernels (ecc_profile.cpp).
int profile_begin(hipStream_t s, void **token);
int profile_end(hipStream_t s, void *token);

}  // namespace ecc
