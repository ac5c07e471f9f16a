// Streaming interface (Sec. 3, "Streaming", "Parallel Computations" and
// "Processing one Chunk"): the image arrives as consecutive chunks of whole
// axis-0 planes.  Each chunk's last plane waits for the next chunk, which
// holds its upper collar.  The changes of a plane need the planes on either
// side of it, so the launch of a chunk [f, f+n) covers planes [f-1, f+n-1)
// (to the end of the image on the last chunk) and reads planes f-2 and f-1
// from a two-plane carry buffer (the previous push's last planes), the rest
// from the chunk itself.
// Counts accumulate on the device; the prefix sum is taken once.  16-bit
// images (m = 65536) run every launch as two 32768-bin passes (Sec. 3,
// "Range of Values"), over the whole value range, since a stream does not
// know its values in advance; each pass adds the values of its half of
// 0..65535 to that half of the changes vector.
//
// Planes with three axes longer than 1 (4-D images) go through the float
// path's change kernel instead (Sec. 3, "Other Ranges of Gray Values": the
// same owner rule on any ordered values): a launch's planes and its collars
// are converted to float32 into one window buffer, the kernel emits the
// changes of the launch's planes only (the collars are neighbours), and the
// non-zero changes are added to the changes vector at their voxels' values.
//
// Host chunks go through two device staging buffers filled on a copy stream
// (hipMemcpyAsync), so the copy of chunk k+1 overlaps the kernels of chunk k.
// Device chunks are read in place.
#include <cstring>

#include "ecc_internal.h"

struct ecc_stream {
    ecc_dims dims{};  // as given to ecc_stream_begin
    int device = -1;
    hipStream_t compute = nullptr;  // caller's stream
    hipStream_t copy = nullptr;     // owned
    ecc::IntView view{};
    int dtype = 0;
    int m = 0;
    int64_t plane_bytes = 0;
    int64_t pushed = 0;   // image planes received
    int64_t emitted = 0;  // image planes whose changes were added
    // carry buffers of two planes: [0, ncarry) hold image planes
    // [pushed - ncarry, pushed)
    uint8_t *carry_buf[2] = {nullptr, nullptr};
    int cur = 0;
    int ncarry = 0;
    // staging for host chunks
    uint8_t *stage[2] = {nullptr, nullptr};
    size_t stage_cap = 0;
    hipEvent_t ready[2] = {nullptr, nullptr};
    hipEvent_t released[2] = {nullptr, nullptr};
    bool released_recorded[2] = {false, false};
    int nstaged = 0;
    // device change vector and per-workgroup rows
    int32_t *partial = nullptr;
    size_t partial_bytes = 0;
    int64_t *mstage = nullptr;  // merge stage rows
    size_t mstage_bytes = 0;
    int64_t *vcec = nullptr;
    uint32_t *status = nullptr;
    // 4-D images: extents, the float window of a launch and its change records
    bool four_d = false;
    int64_t n4[4] = {0, 0, 0, 0};
    float *wbuf = nullptr;
    size_t wbuf_bytes = 0;
    uint8_t *nzbuf = nullptr;
    size_t nzbuf_bytes = 0;
};

namespace {

using namespace ecc;

void destroy(ecc_stream *st) {
    if (!st) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (st->device >= 0) (void)hipSetDevice(st->device);
    if (st->compute) (void)hipStreamSynchronize(st->compute);
    if (st->copy) (void)hipStreamSynchronize(st->copy);
    for (int i = 0; i < 2; ++i) {
        if (st->carry_buf[i]) (void)hipFree(st->carry_buf[i]);
        if (st->stage[i]) (void)hipFree(st->stage[i]);
        if (st->ready[i]) (void)hipEventDestroy(st->ready[i]);
        if (st->released[i]) (void)hipEventDestroy(st->released[i]);
    }
    if (st->partial) (void)hipFree(st->partial);
    if (st->mstage) (void)hipFree(st->mstage);
    if (st->vcec) (void)hipFree(st->vcec);
    if (st->wbuf) (void)hipFree(st->wbuf);
    if (st->nzbuf) (void)hipFree(st->nzbuf);
    if (st->status) (void)hipFree(st->status);
    if (st->copy) (void)hipStreamDestroy(st->copy);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete st;
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

// 4-D images: the changes of image planes [lo, hi) of a push whose chunk
// holds image planes [f, f + n), the carry holding planes [f - a, f).  A
// launch covers planes [b0, b1) with the window [b0 - 1, b1 + 1) within the
// image, as many planes at a time as the float kernel takes (below 2^30
// values).
int run_chunk_4d(ecc_stream *st, const uint8_t *chunk, int64_t f, int64_t lo, int64_t hi) {
    const int64_t n0 = st->view.n0;
    const int64_t pe = st->n4[1] * st->n4[2] * st->n4[3];  // elements per plane
    const int eb = st->dtype == ECC_U8 ? 1 : 2;
    const int64_t step = (((int64_t)1 << 30) - 1) / pe - 2;  // (>= 1: planes hold at most 2^28 values)
    const uint8_t *carry = st->carry_buf[st->cur];
    // every buffer at its largest size first: a push that fails to allocate
    // has added nothing, so it can be pushed again
    {
        ecc_dims w{};
        w.ndim = 4;
        w.n[0] = min64(step, hi - lo) + 2;
        for (int k = 1; k < 4; ++k) w.n[k] = st->n4[k];
        int64_t slots = 0;
        const int64_t regions = float_regions(&w, &slots);
        if (regions < 0) return ECC_E_UNSUPPORTED;
        int rc = ensure_bytes((void **)&st->wbuf, &st->wbuf_bytes, (size_t)(w.n[0] * pe) * 4);
        if (!rc) rc = ensure_bytes((void **)&st->nzbuf, &st->nzbuf_bytes, (size_t)slots * 8 + (size_t)regions * 8);
        if (rc) return rc;
    }
    for (int64_t b0 = lo; b0 < hi; b0 += step) {
        const int64_t b1 = min64(b0 + step, hi);
        const int64_t wlo = b0 > 0 ? b0 - 1 : 0, whi = b1 < n0 ? b1 + 1 : n0;
        const int64_t p = whi - wlo;
        const int64_t ncar = wlo < f ? f - wlo : 0;  // window planes from the carry (0..2)
        if (ncar > st->ncarry) {
            set_error("internal error: 4-D stream window");
            return ECC_E_STATE;
        }
        int rc = ensure_bytes((void **)&st->wbuf, &st->wbuf_bytes, (size_t)(p * pe) * 4);
        if (rc) return rc;
        if (ncar > 0) {
            rc = launch_int_to_f32(carry + (st->ncarry - ncar) * st->plane_bytes, eb, ncar * pe, (uint32_t)st->m, 0,
                                   st->wbuf, st->status, st->compute);
            if (rc) return rc;
        }
        const int64_t c0 = wlo + ncar;  // first window plane from the chunk
        rc = launch_int_to_f32(chunk + (c0 - f) * st->plane_bytes, eb, (whi - c0) * pe, (uint32_t)st->m, 0,
                               st->wbuf + ncar * pe, st->status, st->compute);
        if (rc) return rc;
        ecc_dims w{};
        w.ndim = 4;
        w.n[0] = p;
        for (int k = 1; k < 4; ++k) w.n[k] = st->n4[k];
        int64_t slots = 0;
        const int64_t regions = float_regions(&w, &slots);
        if (regions < 0) return ECC_E_UNSUPPORTED;
        const size_t off_cnt = (size_t)slots * 8, off_off = off_cnt + (size_t)regions * 4;
        rc = ensure_bytes((void **)&st->nzbuf, &st->nzbuf_bytes, off_off + (size_t)regions * 4);
        if (rc) return rc;
        uint32_t *nz_key = (uint32_t *)st->nzbuf;
        int32_t *nz_chg = (int32_t *)(nz_key + slots);
        uint32_t *nz_cnt = (uint32_t *)(st->nzbuf + off_cnt), *nz_off = (uint32_t *)(st->nzbuf + off_off);
        // (a one-plane image: its plane is emitted, and the kernel sees three axes)
        rc = launch_float_change(st->wbuf, &w, nullptr, nz_key, nz_chg, nz_cnt, nz_off, st->status, st->compute,
                                 p > 1 ? (int32_t)(b0 - wlo) : 0, p > 1 ? (int32_t)(b1 - wlo) : INT32_MAX);
        if (rc) return rc;
        rc = launch_records_to_vcec(nz_key, nz_chg, nz_cnt, regions, slots / regions, st->m, st->vcec, st->compute);
        if (rc) return rc;
    }
    return ECC_OK;
}

// Adds the changes of image planes [emitted, hi) of a push whose chunk holds
// image planes [f, f + n), in one launch: buffer plane p is image plane f + p,
// read from the chunk for p >= 0 and from the carry buffer (the previous
// image planes [f - a, f)) for p < 0.  Then keeps the last two image planes
// for the next push.
int run_chunk(ecc_stream *st, const uint8_t *chunk, int64_t f, int64_t n, int64_t hi) {
    const int64_t pb = st->plane_bytes;
    const int64_t n0 = st->view.n0;
    const int a = st->ncarry;
    uint8_t *carry = st->carry_buf[st->cur];
    const int64_t lo = st->emitted;  // f - 1, or 0 on the first push
    if (lo < hi && st->four_d) {
        int rc = run_chunk_4d(st, chunk, f, lo, hi);
        if (rc) return rc;
    } else if (lo < hi) {
        IntJob j{};
        j.src.base = chunk;
        j.src.lo_base = carry + a * pb;
        j.src.plane_bytes = pb;
        j.view = st->view;
        j.dtype = st->dtype;
        j.e0 = (int32_t)(lo - f);
        j.e1 = (int32_t)(hi - f);
        j.lo_inf = lo == 0;  // else plane lo - 1 = f - 2 is carry plane a - 2 (a == 2)
        j.hi_inf = hi == n0;  // else plane hi = f + n - 1 is the chunk's last plane
        const bool u16 = st->dtype == ECC_U16;
        const IntTiling tl = u16 ? range_pass_tiling(st->view, hi - lo) : choose_int_tiling(st->view, st->dtype, hi - lo);
        const int mloc = u16 ? 32768 : st->m;  // bins of one launch
        int rc = ensure_bytes((void **)&st->partial, &st->partial_bytes, (size_t)tl.grid * mloc * sizeof(int32_t));
        if (rc) return rc;
        rc = ensure_bytes((void **)&st->mstage, &st->mstage_bytes,
                          (size_t)merge_stage_rows(tl.grid) * mloc * sizeof(int64_t));
        if (rc) return rc;
        if (u16) {
            // two 32768-bin passes, each adding the values of its half of
            // 0..65535 into that half of the changes vector
            j.range_pass = 2;
            for (int i = 0; i < 2; ++i) {
                j.win_shift = i * 32768;
                rc = launch_int_partial(j, tl, st->partial, st->status, nullptr, st->compute);
                if (rc) return rc;
                rc = launch_merge(st->partial, tl.grid, mloc, st->mstage, st->vcec + i * 32768, true, false, nullptr,
                                  st->status, nullptr, st->compute);
                if (rc) return rc;
            }
        } else {
            rc = launch_int_partial(j, tl, st->partial, st->status, nullptr, st->compute);
            if (rc) return rc;
            rc = launch_merge(st->partial, tl.grid, st->m, st->mstage, st->vcec, true, false, nullptr, st->status,
                              nullptr, st->compute);
            if (rc) return rc;
        }
    }

    // next carry: image planes [f + n - keep, f + n), keep = min(a + n, 2)
    const int nxt = st->cur ^ 1;
    const int keep = (int)min64(a + n, 2);
    uint8_t *dst = st->carry_buf[nxt];
    if (n >= 2) {
        ECC_HIP(hipMemcpyAsync(dst, chunk + (n - 2) * pb, (size_t)(2 * pb), hipMemcpyDeviceToDevice, st->compute));
    } else {  // n == 1: the last carried plane (if any), then the chunk's plane
        if (keep == 2)
            ECC_HIP(hipMemcpyAsync(dst, carry + (a - 1) * pb, (size_t)pb, hipMemcpyDeviceToDevice, st->compute));
        ECC_HIP(hipMemcpyAsync(dst + (keep - 1) * pb, chunk, (size_t)pb, hipMemcpyDeviceToDevice, st->compute));
    }
    st->cur = nxt;
    st->ncarry = keep;
    return ECC_OK;
}

// Snapshot (a resume state, Sec. 3 "Streaming": the changes vector, the
// planes a later chunk still needs and the count of planes pushed): a
// header, the changes vector (m int64), the carried planes.
constexpr uint32_t kSnapMagic = 0x53434345u;  // "ECCS"
struct SnapHeader {
    uint32_t magic, version;
    ecc_dims dims;
    int32_t dtype, m;
    int64_t pushed, emitted, plane_bytes;
    int32_t ncarry;
    uint32_t status;
};
int64_t snap_bytes(const ecc_stream *st) {
    return (int64_t)sizeof(SnapHeader) + (int64_t)st->m * 8 + (int64_t)st->ncarry * st->plane_bytes;
}

}  // namespace

extern "C" {

int ecc_stream_begin(const ecc_dims *full_dims, ecc_dtype dtype, void *stream, ecc_stream **out) {
    if (!full_dims || !out) {
        set_error("ecc_stream_begin: NULL argument");
        return ECC_E_ARG;
    }
    *out = nullptr;
    if (full_dims->ndim < 1 || full_dims->ndim > 4) {
        set_error("ndim %d outside 1..4", (int)full_dims->ndim);
        return ECC_E_ARG;
    }
    for (int k = 0; k < full_dims->ndim; ++k)
        if (full_dims->n[k] < 1) {
            set_error("n[%d] < 1", k);
            return ECC_E_ARG;
        }
    if (dtype != ECC_U8 && dtype != ECC_U14 && dtype != ECC_U16) {
        if (dtype == ECC_F32) {
            set_error("streaming: dtype %d not available in this library", (int)dtype);
            return ECC_E_UNSUPPORTED;
        }
        set_error("unknown dtype %d", (int)dtype);
        return ECC_E_ARG;
    }
    // Streaming cuts along axis 0 of the image as given, which stays the
    // walking axis; in-plane axes of length 1 are dropped (their complex is a
    // product with a unit interval).
    IntView v{};
    int64_t ins[3];
    int k = 0;
    for (int i = 1; i < full_dims->ndim; ++i)
        if (full_dims->n[i] > 1) ins[k++] = full_dims->n[i];
    if (k == 0) {
        v.nin = 1; v.n1 = 1; v.n2 = 1;
    } else if (k == 1 && ins[0] <= INT32_MAX) {
        v.nin = 1; v.n1 = 1; v.n2 = (int32_t)ins[0];
    } else if (k == 2 && ins[0] * ins[1] <= INT32_MAX) {
        v.nin = 2; v.n1 = (int32_t)ins[0]; v.n2 = (int32_t)ins[1];
    } else if (k == 3 && ins[0] * ins[1] * ins[2] <= ((int64_t)1 << 28)) {
        v.nin = 3;  // 4-D: the float change kernel on a window of planes
        v.n1 = 1;
        v.n2 = 1;
    } else {
        set_error("streaming: plane shape not supported (a plane beyond 2^31 elements, or 2^28 with three axes)");
        return ECC_E_UNSUPPORTED;
    }
    v.n0 = full_dims->n[0];
    if (v.n0 > INT32_MAX - 4) {
        set_error("streaming: too many planes");
        return ECC_E_UNSUPPORTED;
    }
    ecc_stream *st = new ecc_stream();
    st->dims = *full_dims;
    st->compute = (hipStream_t)stream;
    st->view = v;
    st->dtype = dtype;
    st->m = (int)threshold_count(dtype);
    st->plane_bytes = (int64_t)v.n1 * v.n2 * (dtype == ECC_U8 ? 1 : 2);
    if (v.nin == 3) {
        st->four_d = true;
        st->n4[0] = full_dims->n[0];
        for (int i = 0; i < 3; ++i) st->n4[i + 1] = ins[i];
        st->plane_bytes = ins[0] * ins[1] * ins[2] * (dtype == ECC_U8 ? 1 : 2);
    }
    int rc = ECC_OK;
    auto fail = [&](int code) {
        destroy(st);
        return code;
    };
    if (hipGetDevice(&st->device) != hipSuccess) return fail(hip_fail(hipErrorInvalidDevice, "hipGetDevice"));
    hipError_t e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
    for (int i = 0; i < 2; ++i) {
        if ((e = dev_malloc((void **)&st->carry_buf[i], (size_t)st->plane_bytes * 2)) != hipSuccess)
            return fail(hip_fail(e, "hipMalloc(carry)"));
        if ((e = hipEventCreateWithFlags(&st->ready[i], hipEventDisableTiming)) != hipSuccess)
            return fail(hip_fail(e, "hipEventCreate"));
        if ((e = hipEventCreateWithFlags(&st->released[i], hipEventDisableTiming)) != hipSuccess)
            return fail(hip_fail(e, "hipEventCreate"));
    }
    if ((e = dev_malloc((void **)&st->vcec, (size_t)st->m * sizeof(int64_t))) != hipSuccess)
        return fail(hip_fail(e, "hipMalloc(vcec)"));
    if ((e = dev_malloc((void **)&st->status, kStatusBytes)) != hipSuccess) return fail(hip_fail(e, "hipMalloc(status)"));
    if ((rc = launch_zero(st->vcec, (size_t)st->m * sizeof(int64_t), st->compute))) return fail(rc);
    if ((rc = launch_zero(st->status, kStatusBytes, st->compute))) return fail(rc);
    *out = st;
    return ECC_OK;
}

int ecc_stream_push_chunk(ecc_stream *st, const void *planes, int64_t n_planes) {
    if (!st || !planes || n_planes < 1) {
        set_error("ecc_stream_push_chunk: bad argument");
        return ECC_E_ARG;
    }
    if (st->pushed + n_planes > st->view.n0) {
        set_error("ecc_stream_push_chunk: %lld planes pushed, image has %lld",
                  (long long)(st->pushed + n_planes), (long long)st->view.n0);
        return ECC_E_STATE;
    }
    if (n_planes > INT32_MAX / 2) {
        set_error("ecc_stream_push_chunk: chunk too large");
        return ECC_E_ARG;
    }
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != st->device) ECC_HIP(hipSetDevice(st->device));
    const size_t bytes = (size_t)n_planes * (size_t)st->plane_bytes;
    const uint8_t *chunk = (const uint8_t *)planes;
    int rc = ECC_OK;
    if (!is_device_ptr(planes)) {
        // Host chunk: copy into staging buffer k % 2 on the copy stream, after
        // the kernels that last read that buffer are done.
        const int k = st->nstaged & 1;
        if (bytes > st->stage_cap) {
            ECC_HIP(hipStreamSynchronize(st->compute));
            ECC_HIP(hipStreamSynchronize(st->copy));
            for (int i = 0; i < 2; ++i) {
                if (st->stage[i]) ECC_HIP(hipFree(st->stage[i]));
                st->stage[i] = nullptr;
                st->released_recorded[i] = false;
            }
            st->stage_cap = 0;
            for (int i = 0; i < 2; ++i) ECC_HIP(dev_malloc((void **)&st->stage[i], bytes));
            st->stage_cap = bytes;
        }
        if (st->released_recorded[k]) ECC_HIP(hipStreamWaitEvent(st->copy, st->released[k], 0));
        ECC_HIP(hipMemcpyAsync(st->stage[k], planes, bytes, hipMemcpyHostToDevice, st->copy));
        ECC_HIP(hipEventRecord(st->ready[k], st->copy));
        ECC_HIP(hipStreamWaitEvent(st->compute, st->ready[k], 0));
        chunk = st->stage[k];
        st->nstaged++;
        const int64_t first = st->pushed;
        const int64_t hi = (first + n_planes == st->view.n0) ? st->view.n0 : first + n_planes - 1;
        rc = run_chunk(st, chunk, first, n_planes, hi);
        if (!rc) {
            ECC_HIP(hipEventRecord(st->released[k], st->compute));
            st->released_recorded[k] = true;
            // the caller's buffer may be reused once its copy is done
            ECC_HIP(hipEventSynchronize(st->ready[k]));
            st->emitted = hi;
            st->pushed = first + n_planes;
        }
    } else {
        const int64_t first = st->pushed;
        const int64_t hi = (first + n_planes == st->view.n0) ? st->view.n0 : first + n_planes - 1;
        rc = run_chunk(st, chunk, first, n_planes, hi);
        if (!rc) {
            st->emitted = hi;
            st->pushed = first + n_planes;
        }
    }
    if (prev != st->device) (void)hipSetDevice(prev);
    return rc;
}

int ecc_stream_finish(ecc_stream *st, ecc_curve *curve) {
    if (!st) {
        set_error("ecc_stream_finish: NULL stream");
        return ECC_E_ARG;
    }
    int rc = ECC_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(st->device);
    do {
        if (!curve || !curve->chi) {
            set_error("ecc_stream_finish: NULL curve");
            rc = ECC_E_ARG;
            break;
        }
        if (st->pushed != st->view.n0) {
            set_error("ecc_stream_finish: %lld of %lld planes pushed", (long long)st->pushed,
                      (long long)st->view.n0);
            rc = ECC_E_STATE;
            break;
        }
        if (curve->capacity < st->m) {
            curve->count = st->m;
            set_error("curve capacity %lld < %d", (long long)curve->capacity, st->m);
            rc = ECC_E_BUFFER_TOO_SMALL;
            break;
        }
        int64_t *tmp = nullptr;
        hipError_t e = dev_malloc((void **)&tmp, (size_t)st->m * sizeof(int64_t));
        if (e != hipSuccess) {
            rc = hip_fail(e, "hipMalloc(curve)");
            break;
        }
        rc = launch_merge(nullptr, 0, st->m, nullptr, st->vcec, true, true, tmp, st->status, st->status + 2,
                          st->compute);
        uint32_t stv = 0;
        if (!rc) {
            e = hipMemcpyAsync(&stv, st->status + 2, 4, hipMemcpyDeviceToHost, st->compute);
            if (e == hipSuccess) e = hipStreamSynchronize(st->compute);
            if (e != hipSuccess) rc = hip_fail(e, "status read");
        }
        if (!rc && (stv & kStatusRange)) {
            set_error("a 14-bit image holds a value >= 16384");
            rc = ECC_E_RANGE;
        } else if (!rc && stv != 0) {
            set_error("internal error: device status 0x%08x", stv);
            rc = ECC_E_HIP;
        }
        if (!rc) {
            e = hipMemcpyAsync(curve->chi, tmp, (size_t)st->m * sizeof(int64_t), hipMemcpyDefault, st->compute);
            if (e == hipSuccess) e = hipStreamSynchronize(st->compute);
            if (e != hipSuccess) rc = hip_fail(e, "curve copy");
            else curve->count = st->m;
        }
        (void)hipFree(tmp);
    } while (0);
    destroy(st);
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
}

void ecc_stream_abort(ecc_stream *st) { destroy(st); }

int ecc_stream_snapshot_size(const ecc_stream *st, int64_t *bytes) {
    if (!st || !bytes) {
        set_error("ecc_stream_snapshot_size: NULL argument");
        return ECC_E_ARG;
    }
    *bytes = snap_bytes(st);
    return ECC_OK;
}

int ecc_stream_snapshot(ecc_stream *st, void *host_buf, int64_t capacity) {
    if (!st || !host_buf) {
        set_error("ecc_stream_snapshot: NULL argument");
        return ECC_E_ARG;
    }
    const int64_t need = snap_bytes(st);
    if (capacity < need) {
        set_error("ecc_stream_snapshot: %lld bytes needed, %lld given", (long long)need, (long long)capacity);
        return ECC_E_BUFFER_TOO_SMALL;
    }
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != st->device) ECC_HIP(hipSetDevice(st->device));
    SnapHeader h{};
    h.magic = kSnapMagic;
    h.version = 1;
    h.dims = st->dims;
    h.dtype = st->dtype;
    h.m = st->m;
    h.pushed = st->pushed;
    h.emitted = st->emitted;
    h.plane_bytes = st->plane_bytes;
    h.ncarry = st->ncarry;
    uint8_t *out = (uint8_t *)host_buf;
    hipError_t e = hipStreamSynchronize(st->copy);
    if (e == hipSuccess) e = hipMemcpyAsync(out + sizeof h, st->vcec, (size_t)st->m * 8, hipMemcpyDeviceToHost, st->compute);
    if (e == hipSuccess && st->ncarry > 0)
        e = hipMemcpyAsync(out + sizeof h + (size_t)st->m * 8, st->carry_buf[st->cur],
                           (size_t)(st->ncarry * st->plane_bytes), hipMemcpyDeviceToHost, st->compute);
    if (e == hipSuccess) e = hipMemcpyAsync(&h.status, st->status, 4, hipMemcpyDeviceToHost, st->compute);
    if (e == hipSuccess) e = hipStreamSynchronize(st->compute);
    if (prev != st->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "ecc_stream_snapshot");
    memcpy(out, &h, sizeof h);
    return ECC_OK;
}

int ecc_stream_restore(const void *host_buf, int64_t bytes, void *stream, ecc_stream **out) {
    if (!host_buf || !out) {
        set_error("ecc_stream_restore: NULL argument");
        return ECC_E_ARG;
    }
    *out = nullptr;
    SnapHeader h;
    if (bytes < (int64_t)sizeof h) {
        set_error("ecc_stream_restore: %lld bytes is not a snapshot", (long long)bytes);
        return ECC_E_ARG;
    }
    memcpy(&h, host_buf, sizeof h);
    if (h.magic != kSnapMagic || h.version != 1) {
        set_error("ecc_stream_restore: not a stream snapshot (magic or version)");
        return ECC_E_ARG;
    }
    ecc_stream *st = nullptr;
    int rc = ecc_stream_begin(&h.dims, (ecc_dtype)h.dtype, stream, &st);
    if (rc) return rc;
    // the snapshot must describe a state of a stream of these dims: every
    // field in range, and the size exact
    const bool ok = h.m == st->m && h.plane_bytes == st->plane_bytes && h.pushed >= 0 && h.pushed <= st->view.n0 &&
                    h.ncarry == (int32_t)min64(h.pushed, 2) &&
                    h.emitted == (h.pushed == 0 ? 0 : (h.pushed == st->view.n0 ? st->view.n0 : h.pushed - 1)) &&
                    (h.status & ~kStatusRange) == 0 &&
                    bytes == (int64_t)sizeof h + (int64_t)h.m * 8 + (int64_t)h.ncarry * h.plane_bytes;
    if (!ok) {
        destroy(st);
        set_error("ecc_stream_restore: the snapshot's state does not match its dims");
        return ECC_E_ARG;
    }
    const uint8_t *in = (const uint8_t *)host_buf;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != st->device) (void)hipSetDevice(st->device);
    hipError_t e = hipMemcpyAsync(st->vcec, in + sizeof h, (size_t)h.m * 8, hipMemcpyHostToDevice, st->compute);
    if (e == hipSuccess && h.ncarry > 0)
        e = hipMemcpyAsync(st->carry_buf[st->cur], in + sizeof h + (size_t)h.m * 8, (size_t)(h.ncarry * h.plane_bytes),
                           hipMemcpyHostToDevice, st->compute);
    if (e == hipSuccess) e = hipMemcpyAsync(st->status, &h.status, 4, hipMemcpyHostToDevice, st->compute);
    if (e == hipSuccess) e = hipStreamSynchronize(st->compute);
    if (prev != st->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        destroy(st);
        return hip_fail(e, "ecc_stream_restore");
    }
    st->pushed = h.pushed;
    st->emitted = h.emitted;
    st->ncarry = h.ncarry;
    *out = st;
    return ECC_OK;
}

}  // extern "C"

namespace ecc {

// The end of ecc_stream_finish without waiting (the serving loop): after
// the last plane was pushed, the prefix sum of the changes vector is
// enqueued on the handle's stream into chi_dev (device memory, m entries,
// written only if no range error was seen) and the status word is copied to
// status_dev.  The handle stays valid until ecc_stream_abort.
int stream_finish_async(ecc_stream *st, int64_t *chi_dev, uint32_t *status_dev) {
    if (!st || !chi_dev) {
        set_error("stream_finish_async: NULL argument");
        return ECC_E_ARG;
    }
    if (st->pushed != st->view.n0) {
        set_error("stream_finish_async: %lld of %lld planes pushed", (long long)st->pushed, (long long)st->view.n0);
        return ECC_E_STATE;
    }
    return launch_merge(nullptr, 0, st->m, nullptr, st->vcec, true, true, chi_dev, st->status, status_dev,
                        st->compute);
}

int64_t stream_plane_bytes(const ecc_stream *st) { return st->plane_bytes; }

}  // namespace ecc
