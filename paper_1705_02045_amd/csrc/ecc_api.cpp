// C ABI of libecc: argument checks, views, workspaces and the resident path.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <mutex>
#include <utility>
#include <vector>

#include "ecc_internal.h"

#include <algorithm>

namespace ecc {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void g_err_clear() { g_err[0] = 0; }

int hip_fail(hipError_t e, const char *what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ECC_E_NOMEM : ECC_E_HIP;
}

int64_t threshold_count(int dtype) {
    switch (dtype) {
    case ECC_U8: return 256;
    case ECC_U14: return 16384;
    case ECC_U16: return 65536;
    default: return -1;
    }
}

size_t elem_bytes(int dtype) {
    switch (dtype) {
    case ECC_U8: return 1;
    case ECC_U14:
    case ECC_U16: return 2;
    case ECC_F32: return 4;
    default: return 0;
    }
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// Allocation-failure injection (testing the error paths): with
// ECC_FAIL_ALLOC=k set, the k-th and every later device or pinned-host
// allocation the library attempts fails as out of memory; the count restarts
// whenever the variable's value changes.
static std::mutex g_fail_mu;
static std::string g_fail_val;
static int64_t g_fail_count = 0;

static bool injected_failure() {
    const char *v = getenv("ECC_FAIL_ALLOC");
    std::lock_guard<std::mutex> lk(g_fail_mu);
    const std::string cur = v ? v : "";
    if (cur != g_fail_val) {
        g_fail_val = cur;
        g_fail_count = 0;
    }
    if (cur.empty()) return false;
    const int64_t k = atoll(cur.c_str());
    return k > 0 && ++g_fail_count >= k;
}

hipError_t dev_malloc(void **p, size_t bytes) {
    if (injected_failure()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t host_malloc(void **p, size_t bytes, unsigned flags) {
    if (injected_failure()) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, flags);
}

int ensure_bytes(void **ptr, size_t *cap, size_t need) {
    if (*cap >= need && *ptr) return ECC_OK;
    if (*ptr) {
        ECC_HIP(hipFree(*ptr));
        *ptr = nullptr;
        *cap = 0;
    }
    size_t sz = need < 256 ? 256 : need;
    ECC_HIP(dev_malloc((void **)ptr, sz));
    *cap = sz;
    return ECC_OK;
}

int ws_ensure(Workspace *ws, void **ptr, size_t *cap, size_t need) {
    if (!ws->fixed) return ensure_bytes(ptr, cap, need);
    if (*ptr && *cap >= need) return ECC_OK;
    set_error("fixed scratch too small: %zu bytes needed, %zu held", need, *cap);
    return ECC_E_NOMEM;
}

static std::mutex g_ws_mu;
static std::map<std::pair<int, void *>, Workspace *> g_ws;

int get_workspace(void *stream, Workspace **out) {
    int dev = 0;
    ECC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it == g_ws.end()) {
        Workspace *w = new Workspace();
        w->device = dev;
        w->stream = stream;
        void *p = nullptr;
        hipError_t e = dev_malloc((void **)&p, kStatusBytes);
        if (e != hipSuccess) {
            delete w;
            return hip_fail(e, "hipMalloc(status)");
        }
        w->status = (uint32_t *)p;
        void *hp = nullptr, *hd = nullptr;
        e = host_malloc((void **)&hp, 64, hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer(&hd, hp, 0);
        if (e != hipSuccess) {
            if (hp) (void)hipHostFree(hp);
            (void)hipFree(p);
            delete w;
            return hip_fail(e, "hipHostMalloc(status word)");
        }
        w->host_status = (volatile uint32_t *)hp;
        w->host_status_dev = (uint32_t *)hd;
        int rc = launch_zero(p, kStatusBytes, (hipStream_t)stream);
        if (rc) {
            (void)hipHostFree(hp);
            (void)hipFree(p);
            delete w;
            return rc;
        }
        it = g_ws.emplace(key, w).first;
    }
    *out = it->second;
    return ECC_OK;
}

// Side streams of a caller's stream: the box faces of the dual complex run
// on them, concurrently with the full box on the caller's stream (a fork at
// the call's start, a join before the faces' changes are summed).  Created
// on first use per (device, caller's stream) with the default priority,
// non-blocking, and kept for the process; each has its own workspace.
struct SideStreams {
    static constexpr int kCount = 4;
    hipStream_t s[kCount] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kCount] = {};
};
static std::mutex g_side_mu;
static std::map<std::pair<int, void *>, SideStreams *> g_side;

static int get_side_streams(void *stream, SideStreams **out) {
    int dev = 0;
    ECC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_side.find(key);
    if (it == g_side.end()) {
        SideStreams *p = new SideStreams();
        hipError_t e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        for (int k = 0; e == hipSuccess && k < SideStreams::kCount; ++k) {
            e = hipStreamCreateWithFlags(&p->s[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[k], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            for (int k = 0; k < SideStreams::kCount; ++k) {
                if (p->join[k]) (void)hipEventDestroy(p->join[k]);
                if (p->s[k]) (void)hipStreamDestroy(p->s[k]);
            }
            if (p->fork) (void)hipEventDestroy(p->fork);
            delete p;
            return hip_fail(e, "side streams");
        }
        it = g_side.emplace(key, p).first;
    }
    *out = it->second;
    return ECC_OK;
}

int check_dims(const ecc_dims *dims, int64_t *total) {
    if (!dims) {
        set_error("dims is NULL");
        return ECC_E_ARG;
    }
    if (dims->ndim < 1 || dims->ndim > 4) {
        set_error("ndim %d outside 1..4", (int)dims->ndim);
        return ECC_E_ARG;
    }
    int64_t t = 1;
    for (int k = 0; k < dims->ndim; ++k) {
        if (dims->n[k] < 1) {
            set_error("n[%d] = %lld < 1", k, (long long)dims->n[k]);
            return ECC_E_ARG;
        }
        if (t > ((int64_t)1 << 62) / dims->n[k]) {
            set_error("image size overflows");
            return ECC_E_ARG;
        }
        t *= dims->n[k];
    }
    *total = t;
    return ECC_OK;
}

// Axes of length 1 are dropped: the complex of such an image is the product of
// the complex of the remaining axes with a closed unit interval, and taking
// that product changes no Euler characteristic of any threshold.
bool normalize_int_view(const ecc_dims *dims, IntView *v, int *unsupported) {
    int64_t ns[4];
    int k = 0;
    for (int i = 0; i < dims->ndim; ++i)
        if (dims->n[i] > 1) ns[k++] = dims->n[i];
    *unsupported = 0;
    if (k == 0) ns[k++] = 1;
    if (k == 1) {
        v->nin = 1; v->n0 = 1; v->n1 = 1;
        if (ns[0] > INT32_MAX) { *unsupported = 1; return false; }
        v->n2 = (int32_t)ns[0];
    } else if (k == 2) {
        v->nin = 1; v->n0 = ns[0]; v->n1 = 1;
        if (ns[1] > INT32_MAX) { *unsupported = 1; return false; }
        v->n2 = (int32_t)ns[1];
    } else if (k == 3) {
        v->nin = 2; v->n0 = ns[0];
        if (ns[1] > INT32_MAX || ns[2] > INT32_MAX || ns[1] * ns[2] > INT32_MAX) { *unsupported = 1; return false; }
        v->n1 = (int32_t)ns[1]; v->n2 = (int32_t)ns[2];
    } else {
        *unsupported = 1;
        return false;
    }
    if (v->n0 > INT32_MAX - 4) { *unsupported = 1; return false; }
    return true;
}

static int env_int(const char *name, int dflt) {
    const char *s = getenv(name);
    return (s && *s) ? atoi(s) : dflt;
}

// Tuning overrides (measurement only): ECC_INT_ROWS, ECC_INT_MODE, ECC_INT_PD, ECC_INT_WX, ECC_U16_TILES_PER_CU,
// ECC_U16_WINDOWS (1: 16-bit images in the window form),
// ECC_INT_WAVES, ECC_INT_TILES_PER_CU, ECC_INT_TILE_STRIDE, ECC_INT_PAIR (0: no row pairs).
// The tiling for given parameters: R rows per wave, up to wx_cap waves
// along x (16-wave workgroups), about tiles_per_cu workgroups per CU.
IntTiling make_int_tiling(const IntView &v, int64_t planes, int rows, int tiles_per_cu, int wx_cap,
                          int max_grid = 0) {
    IntTiling t{};
    t.rows = rows;
    t.mode = env_int("ECC_INT_MODE", 0);
    const int cus = device_cu_count();
    const int max_waves = env_int("ECC_INT_WAVES", 16);
    int64_t tiles_xy;
    if (v.nin == 1) {
        const int64_t segs = (v.n2 + (int64_t)kWave * t.rows - 1) / ((int64_t)kWave * t.rows);
        t.wx = (int)(segs < max_waves ? segs : max_waves);
        t.wy = 1;
        tiles_xy = (segs + t.wx - 1) / t.wx;
    } else {
        const int64_t xs = (v.n2 + kWave - 1) / kWave;
        t.wx = (int)(xs < wx_cap ? xs : wx_cap);
        const int64_t ys = (v.n1 + t.rows - 1) / t.rows;
        const int64_t wy = max_waves / t.wx;
        t.wy = (int)(ys < wy ? ys : wy);
        tiles_xy = ((xs + t.wx - 1) / t.wx) * ((ys + t.wy - 1) / t.wy);
    }
    // split axis 0 until there are about tiles_per_cu tiles per CU; planes
    // with more tiles than that get several tiles per workgroup, so the
    // per-workgroup rows stay about tiles_per_cu per CU
    const int64_t target = (int64_t)cus * tiles_per_cu;
    int64_t tz = (target + tiles_xy - 1) / tiles_xy;
    if (tz < 1) tz = 1;
    if (tz > planes) tz = planes;
    int64_t zc = (planes + tz - 1) / tz;
    if (zc < 8 && planes >= 8) zc = 8;
    t.zc = (int)zc;
    // planes of loads in flight: two on walks of 128 planes and more (1024^3:
    // 2 % faster, 512 x 4096^2: 7 %), one on shorter walks, where the longer
    // prologue costs more than it hides (14 x 8192^2: 20 % slower with two);
    // two with four rows per wave, whose register budget (one workgroup per
    // CU) holds them without spills (64-plane slabs of 14450^2: 2 % faster)
    t.pd = env_int("ECC_INT_PD", (zc >= 128 || rows >= 4) ? 2 : 1);
    const int64_t tiles = tiles_xy * ((planes + zc - 1) / zc);
    int64_t per = tiles > target ? (tiles + target - 1) / target : 1;
    // a cap on the workgroups (fixed scratch): more tiles per workgroup
    if (max_grid > 0 && (tiles + per - 1) / per > max_grid) per = (tiles + max_grid - 1) / max_grid;
    t.per_wg = (int)per;
    t.tile_stride = env_int("ECC_INT_TILE_STRIDE", 0);
    t.pair = env_int("ECC_INT_PAIR", 1);
    t.grid = (int)((tiles + per - 1) / per);
    return t;
}

// Tilings chosen by ecc_autotune, per (dtype, rank, n1, n2, planes).
struct TuneKey {
    int dtype, nin;
    int32_t n1, n2;
    int64_t planes;
    bool operator<(const TuneKey &o) const {
        return std::tie(dtype, nin, n1, n2, planes) < std::tie(o.dtype, o.nin, o.n1, o.n2, o.planes);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, ecc_tiling> g_tuned;

static bool tuned_tiling(const IntView &v, int dtype, int64_t planes, ecc_tiling *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(TuneKey{dtype, v.nin, v.n1, v.n2, planes});
    if (it == g_tuned.end()) return false;
    *out = it->second;
    return true;
}

// Launch-size rule (measured on MI355X): below 256 MiB four tiles per CU are
// fastest, above it eight.  From 4 GiB on (e.g. 62 planes of 8192^2 or of
// 14450^2) four rows per wave run at about 2.8 TB/s where two rows reach
// 2.0-2.4; below 2 GiB two rows are faster.  Likely cause: four rows keep
// half as many workgroups in flight, so fewer distinct 2 MiB pages per plane
// step need translating once a plane spans many pages.
// Between 256 MiB and 4 GiB, four tiles per CU when that gives walks of 256
// planes or more (1024^3: 512-plane walks, the same kernel time as eight
// tiles per CU and half the count rows to merge: 0.770 vs 0.781 ms per
// curve), else eight (62 x 4096^2: 0.735 vs 0.831 ms).
static ecc_tiling rule_tiling(const IntView &v, int dtype, int64_t planes) {
    const int64_t launch_bytes = planes * (int64_t)v.n1 * v.n2 * (dtype == ECC_U8 ? 1 : 2);
    ecc_tiling c{};
    c.rows = launch_bytes >= ((int64_t)4 << 30) ? 4 : 2;
    // four rows: workgroups two waves tall (64-plane slabs of 14450^2: 2 %
    // faster than one row of 16 waves)
    c.waves_x = c.rows == 4 ? 8 : 16;
    if (launch_bytes < ((int64_t)256 << 20)) c.tiles_per_cu = 4;
    else if (c.rows == 4) c.tiles_per_cu = 16;
    else c.tiles_per_cu = make_int_tiling(v, planes, c.rows, 4, c.waves_x).zc >= 256 ? 4 : 8;
    return c;
}

// Parameters: ECC_INT_* environment overrides (measurement), else a tiling
// ecc_autotune stored for this shape, else the launch-size rule.
static ecc_tiling tiling_params(const IntView &v, int dtype, int64_t planes) {
    ecc_tiling c{};
    if (!tuned_tiling(v, dtype, planes, &c)) c = rule_tiling(v, dtype, planes);
    c.rows = env_int("ECC_INT_ROWS", c.rows);
    c.tiles_per_cu = env_int("ECC_INT_TILES_PER_CU", c.tiles_per_cu);
    c.waves_x = env_int("ECC_INT_WX", c.waves_x);
    return c;
}

IntTiling choose_int_tiling(const IntView &v, int dtype, int64_t planes, int max_grid) {
    const ecc_tiling c = tiling_params(v, dtype, planes);
    return make_int_tiling(v, planes, c.rows, c.tiles_per_cu, c.waves_x, max_grid);
}

// Enqueue the whole integer computation for a device-resident image.
static int enqueue_int(const void *image_dev, const IntView &v, int dtype, int64_t *chi_dev,
                       uint32_t *status_out, hipStream_t stream, Workspace *ws, bool max_entry = false) {
    const int m = (int)threshold_count(dtype);
    const size_t eb = elem_bytes(dtype);
    IntTiling tl = choose_int_tiling(v, dtype, v.n0, ws->max_grid);
    int rc = ws_ensure(ws, (void **)&ws->partial, &ws->partial_bytes, (size_t)tl.grid * m * sizeof(int32_t));
    if (rc) return rc;
    rc = ws_ensure(ws, (void **)&ws->vcec, &ws->vcec_bytes, (size_t)m * sizeof(int64_t));
    if (rc) return rc;
    IntJob job{};
    job.src.base = (const uint8_t *)image_dev;
    job.src.lo_base = job.src.base;
    job.src.plane_bytes = (int64_t)v.n1 * v.n2 * (int64_t)eb;
    job.view = v;
    job.e0 = 0;
    job.e1 = (int32_t)v.n0;
    job.lo_inf = 1;
    job.hi_inf = 1;
    job.dtype = dtype;
    job.invert = max_entry ? 1 : 0;
    rc = ws_ensure(ws, (void **)&ws->stage, &ws->stage_bytes, (size_t)merge_stage_rows(tl.grid) * m * sizeof(int64_t));
    if (rc) return rc;
    rc = launch_int_partial(job, tl, ws->partial, ws->status, nullptr, stream);
    if (rc) return rc;
    return launch_merge(ws->partial, tl.grid, m, ws->stage, ws->vcec, false, true, chi_dev, ws->status, status_out,
                        stream, max_entry);
}

// 16-bit images (m = 65536): the workgroup histograms hold 16384 bins, so
// one launch counts one window of values.  The kernel reads
// bin = clamp(v - shift, 0, 16383); bins [klo, khi] are values
// [shift + klo, shift + khi].  A window needs a guard bin only on a side
// where the image has values outside it: bin 0 when values below exist
// (klo = 1), bin 16383 when values above exist (khi = 16382).  The guard
// bins are dropped; the monotone clamp keeps every comparison that decides a
// kept bin (each involves the counted value itself).  Each pass's column
// sums go to their place in the 65536-bin changes vector, scanned once.
int plan_u16_windows(uint32_t vmin, uint32_t vmax, U16Window *w) {
    int n = 0;
    int64_t v = vmin;
    while (v <= (int64_t)vmax) {
        U16Window x;
        x.klo = v > (int64_t)vmin ? 1 : 0;
        x.shift = (int32_t)(v - x.klo);
        x.khi = (int64_t)x.shift + 16383 >= (int64_t)vmax ? (int)((int64_t)vmax - x.shift) : 16382;
        w[n++] = x;
        v = (int64_t)x.shift + x.khi + 1;
    }
    return n;
}

// Tiling of a 32768-bin pass: two rows per wave, two planes of look-ahead,
// about two workgroups per CU (one resident at a time: 1024^3, 2.21 ms for
// the full range; one per CU 2.21, four 2.28, eight 2.43).
IntTiling range_pass_tiling(const IntView &v, int64_t planes) {
    IntTiling tl = make_int_tiling(v, planes, 2, env_int("ECC_U16_TILES_PER_CU", 2), 16);
    tl.pd = 2;
    tl.mode = 0;
    return tl;
}

// 16-bit images in 32768-bin passes (a 128 KiB workgroup histogram, one
// workgroup per CU): the fields and comparisons take the raw values and each
// pass adds the changes at values [lo, lo + 32768) exactly, with no guard
// bins: one pass from min(vmin, 32768) when the image's values span fewer
// than 32768, else the passes [0, 32768) and [32768, 65536), each skipping
// the adds of values outside its range.  Each pass's column sums go to their
// place in the 65536-bin changes vector, scanned once.
static int enqueue_u16_passes(const void *image_dev, const IntView &v, int64_t *chi_dev, uint32_t *status_out,
                              hipStream_t stream, Workspace *ws, uint32_t vmin, uint32_t vmax) {
    constexpr int mpass = 32768, mtot = 65536;
    int32_t lo[2] = {0, mpass};
    int npass = 2, mode = 2;
    if (vmax - vmin < (uint32_t)mpass) {
        npass = 1;
        mode = 1;
        lo[0] = (int32_t)(vmin < (uint32_t)mpass ? vmin : (uint32_t)mpass);
    }
    const IntTiling tl = range_pass_tiling(v, v.n0);
    int rc = ensure_bytes((void **)&ws->partial, &ws->partial_bytes, (size_t)tl.grid * mpass * sizeof(int32_t));
    if (rc) return rc;
    rc = ensure_bytes((void **)&ws->stage, &ws->stage_bytes,
                      (size_t)merge_stage_rows(tl.grid) * mpass * sizeof(int64_t));
    if (rc) return rc;
    rc = ensure_bytes((void **)&ws->vcec16, &ws->vcec16_bytes, (size_t)mtot * sizeof(int64_t));
    if (rc) return rc;
    if (npass == 1) {  // the bins outside the pass stay zero
        rc = launch_zero(ws->vcec16, (size_t)mtot * sizeof(int64_t), stream);
        if (rc) return rc;
    }
    IntJob job{};
    job.src.base = (const uint8_t *)image_dev;
    job.src.lo_base = job.src.base;
    job.src.plane_bytes = (int64_t)v.n1 * v.n2 * 2;
    job.view = v;
    job.e0 = 0;
    job.e1 = (int32_t)v.n0;
    job.lo_inf = 1;
    job.hi_inf = 1;
    job.dtype = ECC_U16;
    job.range_pass = mode;
    for (int i = 0; i < npass; ++i) {
        job.win_shift = lo[i];
        rc = launch_int_partial(job, tl, ws->partial, ws->status, nullptr, stream);
        if (rc) return rc;
        rc = launch_merge(ws->partial, tl.grid, mpass, ws->stage, ws->vcec16 + lo[i], false, false, nullptr,
                          ws->status, nullptr, stream);
        if (rc) return rc;
    }
    return launch_merge(nullptr, 0, mtot, nullptr, ws->vcec16, true, true, chi_dev, ws->status, status_out, stream);
}

// The synchronous call's 16-bit path: the pass over [0, 32768) first, which
// notes whether any value lies above it (a word of host memory, read after
// the pass), and the pass over [32768, 65536) only then.  No separate read
// for the image's range: images below 32768 take one pass (1024^3 14-bit
// and 15-bit data: 0.92 ms, against 1.15 and 2.54 ms for the range read and
// one or two windows), full ranges two (1.80 ms, against 3.94 ms in five
// windows); an image whose values all lie above 32768 reads it once in vain.
static int enqueue_u16_adaptive(const void *image_dev, const IntView &v, int64_t *chi_dev, uint32_t *status_out,
                                hipStream_t stream, Workspace *ws) {
    constexpr int mpass = 32768, mtot = 65536;
    const IntTiling tl = range_pass_tiling(v, v.n0);
    int rc = ensure_bytes((void **)&ws->partial, &ws->partial_bytes, (size_t)tl.grid * mpass * sizeof(int32_t));
    if (rc) return rc;
    rc = ensure_bytes((void **)&ws->stage, &ws->stage_bytes,
                      (size_t)merge_stage_rows(tl.grid) * mpass * sizeof(int64_t));
    if (rc) return rc;
    rc = ensure_bytes((void **)&ws->vcec16, &ws->vcec16_bytes, (size_t)mtot * sizeof(int64_t));
    if (rc) return rc;
    rc = launch_zero(ws->vcec16 + mpass, (size_t)mpass * sizeof(int64_t), stream);  // if the second pass is skipped
    if (rc) return rc;
    volatile uint32_t *high = ws->host_status + 1;
    *high = 0u;
    IntJob job{};
    job.src.base = (const uint8_t *)image_dev;
    job.src.lo_base = job.src.base;
    job.src.plane_bytes = (int64_t)v.n1 * v.n2 * 2;
    job.view = v;
    job.e0 = 0;
    job.e1 = (int32_t)v.n0;
    job.lo_inf = 1;
    job.hi_inf = 1;
    job.dtype = ECC_U16;
    job.range_pass = 2;
    for (int i = 0; i < 2; ++i) {
        job.win_shift = i * mpass;
        job.high_flag = i == 0 ? ws->host_status_dev + 1 : nullptr;
        rc = launch_int_partial(job, tl, ws->partial, ws->status, nullptr, stream);
        if (rc) return rc;
        rc = launch_merge(ws->partial, tl.grid, mpass, ws->stage, ws->vcec16 + i * mpass, false, false, nullptr,
                          ws->status, nullptr, stream);
        if (rc) return rc;
        if (i == 0) {
            ECC_HIP(hipStreamSynchronize(stream));
            if (*high == 0u) break;
        }
    }
    return launch_merge(nullptr, 0, mtot, nullptr, ws->vcec16, true, true, chi_dev, ws->status, status_out, stream);
}

// Planned from a known range (the entry point that allocates nothing, whose
// fixed scratch holds count rows of 16384 bins, and the asynchronous calls,
// which plan for 0..65535): values that fit one window take the window form
// (16384-bin passes, eight waves per SIMD; 1024^3: 1.15 ms against 1.25 ms in
// a 32768-bin pass), wider ranges the 32768-bin passes (full range: 2.2 ms
// against 4.0 ms in five windows).
static int enqueue_u16(const void *image_dev, const IntView &v, int64_t *chi_dev, uint32_t *status_out,
                       hipStream_t stream, Workspace *ws, uint32_t vmin, uint32_t vmax) {
    constexpr int mloc = 16384, mtot = 65536;
    U16Window win[kU16MaxWindows + 1];
    const int nwin = plan_u16_windows(vmin, vmax, win);
    if (nwin > 1 && !ws->fixed && env_int("ECC_U16_WINDOWS", 0) == 0)
        return enqueue_u16_passes(image_dev, v, chi_dev, status_out, stream, ws, vmin, vmax);
    IntTiling tl = choose_int_tiling(v, ECC_U16, v.n0, ws->max_grid);
    int rc = ws_ensure(ws, (void **)&ws->partial, &ws->partial_bytes, (size_t)tl.grid * mloc * sizeof(int32_t));
    if (rc) return rc;
    rc = ws_ensure(ws, (void **)&ws->vcec, &ws->vcec_bytes, (size_t)mloc * sizeof(int64_t));
    if (rc) return rc;
    rc = ws_ensure(ws, (void **)&ws->stage, &ws->stage_bytes,
                   (size_t)merge_stage_rows(tl.grid) * mloc * sizeof(int64_t));
    if (rc) return rc;
    rc = ws_ensure(ws, (void **)&ws->vcec16, &ws->vcec16_bytes, (size_t)mtot * sizeof(int64_t));
    if (rc) return rc;
    rc = launch_zero(ws->vcec16, (size_t)mtot * sizeof(int64_t), stream);
    if (rc) return rc;
    IntJob job{};
    job.src.base = (const uint8_t *)image_dev;
    job.src.lo_base = job.src.base;
    job.src.plane_bytes = (int64_t)v.n1 * v.n2 * 2;
    job.view = v;
    job.e0 = 0;
    job.e1 = (int32_t)v.n0;
    job.lo_inf = 1;
    job.hi_inf = 1;
    job.dtype = ECC_U16;
    for (int i = 0; i < nwin; ++i) {
        job.win_shift = win[i].shift;
        rc = launch_int_partial(job, tl, ws->partial, ws->status, nullptr, stream);
        if (rc) return rc;
        rc = launch_merge(ws->partial, tl.grid, mloc, ws->stage, ws->vcec, false, false, nullptr, ws->status,
                          nullptr, stream);
        if (rc) return rc;
        ECC_HIP(hipMemcpyAsync(ws->vcec16 + win[i].shift + win[i].klo, ws->vcec + win[i].klo,
                               (size_t)(win[i].khi - win[i].klo + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                               stream));
    }
    return launch_merge(nullptr, 0, mtot, nullptr, ws->vcec16, true, true, chi_dev, ws->status, status_out, stream);
}

int u16_curve_async(const void *image_dev, const IntView &v, int64_t *chi_dev, uint32_t *status_out,
                    hipStream_t stream) {
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, &ws);
    if (rc) return rc;
    return enqueue_u16(image_dev, v, chi_dev, status_out, stream, ws, 0, 65535);
}

// Changes vector only (no scan) of a device image into vcec_out; a range
// error stays set in ws->status for a later scan to report.
// plane_stride: elements between consecutive planes of a view with one
// in-plane axis (0: the planes are contiguous rows); the kernel reads only
// the first n2 elements of each plane.
static int enqueue_int_changes(const void *image_dev, const IntView &v, int dtype, int64_t *vcec_out,
                               hipStream_t stream, Workspace *ws, bool max_entry, int64_t plane_stride = 0) {
    const int m = (int)threshold_count(dtype);
    if (plane_stride != 0 && (v.nin != 1 || plane_stride < v.n2 || plane_stride * (int64_t)elem_bytes(dtype) > INT32_MAX)) {
        set_error("internal error: plane stride %lld for a view of %d in-plane axes", (long long)plane_stride, v.nin);
        return ECC_E_ARG;
    }
    IntTiling tl = choose_int_tiling(v, dtype, v.n0);
    int rc = ensure_bytes((void **)&ws->partial, &ws->partial_bytes, (size_t)tl.grid * m * sizeof(int32_t));
    if (rc) return rc;
    rc = ensure_bytes((void **)&ws->stage, &ws->stage_bytes,
                      (size_t)merge_stage_rows(tl.grid) * m * sizeof(int64_t));
    if (rc) return rc;
    IntJob job{};
    job.src.base = (const uint8_t *)image_dev;
    job.src.lo_base = job.src.base;
    job.src.plane_bytes = (plane_stride ? plane_stride : (int64_t)v.n1 * v.n2) * (int64_t)elem_bytes(dtype);
    job.view = v;
    job.e0 = 0;
    job.e1 = (int32_t)v.n0;
    job.lo_inf = 1;
    job.hi_inf = 1;
    job.dtype = dtype;
    job.invert = max_entry ? 1 : 0;
    rc = launch_int_partial(job, tl, ws->partial, ws->status, nullptr, stream);
    if (rc) return rc;
    return launch_merge(ws->partial, tl.grid, m, ws->stage, vcec_out, false, false, nullptr, ws->status, nullptr,
                        stream, max_entry);
}

static bool is_device_ptr(const void *p) {
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Float images: records -> sort -> per-key running sums (ecc_float.hip,
// ecc_sort.hip).  Synchronous: the number of distinct values is only known
// at the end.
static int compute_float(const void *image, const ecc_dims *dims, int64_t n, ecc_curve *curve, hipStream_t s,
                         bool steps_only);

// Integer images the integer kernel does not take (four axes longer than 1):
// exact through the float path, whose curve is a step function over the
// image's distinct values; chi(T_t) is its value at the largest distinct
// value <= t.  max_entry: the float path runs on the inverted image (values
// m - 1 - v) and the result is reflected (launch_reflect_curve).  out_dev
// receives m int64: the curve, or with changes (max_entry only) the changes
// vector.  img_dev is device memory.
static int int_via_float_dev(const void *img_dev, const ecc_dims *dims, int64_t total, ecc_dtype dtype,
                             bool max_entry, bool changes, int64_t *out_dev, hipStream_t s, Workspace *ws) {
    const int64_t m = threshold_count(dtype);
    if (total > (int64_t)UINT32_MAX) {
        set_error("integer path: image too large for the float path");
        return ECC_E_UNSUPPORTED;
    }
    const size_t eb = elem_bytes(dtype);
    // i2f_buf: the float image, the float curve (keys, chi), the expanded curve
    const size_t o_keys = align256((size_t)total * 4), o_chi = o_keys + align256((size_t)total * 4);
    const size_t o_out = o_chi + align256((size_t)total * 8);
    int rc = ensure_bytes(&ws->i2f_buf, &ws->i2f_buf_bytes, o_out + (size_t)m * 8);
    if (rc) return rc;
    uint8_t *buf = (uint8_t *)ws->i2f_buf;
    uint32_t *flag = ws->status + kStatusMinMaxOffset / 4 + 3;
    rc = launch_zero(flag, 4, s);
    if (rc) return rc;
    rc = launch_int_to_f32(img_dev, (int)eb, total, (uint32_t)m, max_entry ? 1 : 0, (float *)buf, flag, s);
    if (rc) return rc;
    uint32_t bad = 0;
    ECC_HIP(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, s));
    ECC_HIP(hipStreamSynchronize(s));
    if (bad) {
        set_error("a 14-bit image holds a value >= 16384");
        return ECC_E_RANGE;
    }
    ecc_curve fc{};
    fc.capacity = total;
    fc.keys = (float *)(buf + o_keys);
    fc.chi = (int64_t *)(buf + o_chi);
    rc = compute_float(buf, dims, total, &fc, s, false);
    if (rc) return rc;
    int64_t *g = max_entry ? (int64_t *)(buf + o_out) : out_dev;
    rc = launch_expand_steps(fc.keys, fc.chi, fc.count, (int)m, g, s);
    if (rc) return rc;
    if (max_entry) return launch_reflect_curve(g, (int)m, changes ? 1 : 0, out_dev, s);
    return ECC_OK;
}

static int compute_int_via_float(const void *image, const ecc_dims *dims, int64_t total, ecc_dtype dtype,
                                 ecc_curve *curve, hipStream_t s, bool max_entry) {
    const int64_t m = threshold_count(dtype);
    Workspace *ws = nullptr;
    int rc = get_workspace(s, &ws);
    if (rc) return rc;
    const size_t eb = elem_bytes(dtype);
    const void *img_dev = image;
    if (!is_device_ptr(image)) {
        rc = ensure_bytes(&ws->img_tmp, &ws->img_tmp_bytes, (size_t)total * eb);
        if (rc) return rc;
        ECC_HIP(hipMemcpyAsync(ws->img_tmp, image, (size_t)total * eb, hipMemcpyHostToDevice, s));
        img_dev = ws->img_tmp;
    }
    rc = ensure_bytes((void **)&ws->chi_tmp, &ws->chi_tmp_bytes, (size_t)m * 8);
    if (rc) return rc;
    rc = int_via_float_dev(img_dev, dims, total, dtype, max_entry, false, ws->chi_tmp, s, ws);
    if (rc) return rc;
    ECC_HIP(hipMemcpyAsync(curve->chi, ws->chi_tmp, (size_t)m * 8, hipMemcpyDefault, s));
    ECC_HIP(hipStreamSynchronize(s));
    curve->count = m;
    return ECC_OK;
}

// Synchronous integer curve: host or device image and curve.  max_entry:
// each cell's value is the maximum over its voxels (the kernel reads M-1-v
// and the merge writes the rows reversed).
static int compute_int(const void *image, const ecc_dims *dims, int64_t total, ecc_dtype dtype, ecc_curve *curve,
                       hipStream_t s, bool max_entry) {
    if (dtype == ECC_U16 && max_entry) {
        set_error("the largest-value convention is available for u8 and u14");
        return ECC_E_UNSUPPORTED;
    }
    const int64_t m = threshold_count(dtype);
    if (m < 0) {
        set_error("unknown dtype %d", (int)dtype);
        return ECC_E_ARG;
    }
    if (curve->capacity < m) {
        curve->count = m;
        set_error("curve capacity %lld < %lld", (long long)curve->capacity, (long long)m);
        return ECC_E_BUFFER_TOO_SMALL;
    }
    IntView v{};
    int unsup = 0;
    if (!normalize_int_view(dims, &v, &unsup)) {
        if (total <= (int64_t)UINT32_MAX) return compute_int_via_float(image, dims, total, dtype, curve, s, max_entry);
        set_error("integer path: shape not supported (4 axes longer than 1, or an extent beyond 2^31)");
        return ECC_E_UNSUPPORTED;
    }
    Workspace *ws = nullptr;
    int rc = get_workspace(s, &ws);
    if (rc) return rc;
    const void *img_dev = image;
    if (!is_device_ptr(image)) {
        const size_t bytes = (size_t)total * elem_bytes(dtype);
        rc = ensure_bytes(&ws->img_tmp, &ws->img_tmp_bytes, bytes);
        if (rc) return rc;
        ECC_HIP(hipMemcpyAsync(ws->img_tmp, image, bytes, hipMemcpyHostToDevice, s));
        img_dev = ws->img_tmp;
    }
    const bool chi_dev = is_device_ptr(curve->chi);
    int64_t *chi_target = curve->chi;
    if (!chi_dev) {
        rc = ensure_bytes((void **)&ws->chi_tmp, &ws->chi_tmp_bytes, (size_t)m * sizeof(int64_t));
        if (rc) return rc;
        chi_target = ws->chi_tmp;
    }
    if (dtype == ECC_U16 && !ws->fixed && env_int("ECC_U16_WINDOWS", 0) == 0) {
        *ws->host_status = 0xFFFFFFFFu;  // overwritten by the scan
        rc = enqueue_u16_adaptive(img_dev, v, chi_target, ws->host_status_dev, s, ws);
    } else if (dtype == ECC_U16) {  // only the windows between the image's minimum and maximum
        uint32_t *mm = ws->status + kStatusMinMaxOffset / 4;
        rc = launch_minmax_u16((const uint16_t *)img_dev, total, mm, s);
        if (rc) return rc;
        uint32_t range[2] = {0, 0};
        ECC_HIP(hipMemcpyAsync(range, mm, sizeof range, hipMemcpyDeviceToHost, s));
        ECC_HIP(hipStreamSynchronize(s));
        *ws->host_status = 0xFFFFFFFFu;  // overwritten by the scan
        rc = enqueue_u16(img_dev, v, chi_target, ws->host_status_dev, s, ws, range[0], range[1]);
    } else {
        *ws->host_status = 0xFFFFFFFFu;
        rc = enqueue_int(img_dev, v, dtype, chi_target, ws->host_status_dev, s, ws, max_entry);
    }
    if (rc) {
        (void)hipStreamSynchronize(s);  // the scan may still write the host word
        return rc;
    }
    ECC_HIP(hipStreamSynchronize(s));
    const uint32_t st = *ws->host_status;
    if (st == 0xFFFFFFFFu) {
        set_error("internal error: the scan did not report a status");
        return ECC_E_HIP;
    }
    if (st & kStatusRange) {
        set_error("a 14-bit image holds a value >= 16384");
        return ECC_E_RANGE;
    }
    if (st != 0) {
        set_error("internal error: device status 0x%08x", st);
        return ECC_E_HIP;
    }
    if (!chi_dev) {
        ECC_HIP(hipMemcpyAsync(curve->chi, ws->chi_tmp, (size_t)m * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        ECC_HIP(hipStreamSynchronize(s));
    }
    curve->count = m;
    return ECC_OK;
}

// steps_only: the output keeps the keys where chi changes (chi = 0 before
// the first key), compacted after the full curve is built.
static int compute_float(const void *image, const ecc_dims *dims, int64_t n, ecc_curve *curve, hipStream_t s,
                         bool steps_only) {
    if (!curve->keys) {
        set_error("ECC_F32 needs curve->keys");
        return ECC_E_ARG;
    }
    Workspace *ws = nullptr;
    int rc = get_workspace(s, &ws);
    if (rc) return rc;
    const float *img_dev = (const float *)image;
    if (!is_device_ptr(image)) {
        const size_t bytes = (size_t)n * 4;
        rc = ensure_bytes(&ws->img_tmp, &ws->img_tmp_bytes, bytes);
        if (rc) return rc;
        ECC_HIP(hipMemcpyAsync(ws->img_tmp, image, bytes, hipMemcpyHostToDevice, s));
        img_dev = (const float *)ws->img_tmp;
    }
    // carve the float scratch: two key buffers (sort), the record regions
    // (keys then changes; after the records are compacted, the change-point
    // output's chi), the region counts and offsets, the digit table and its
    // scan sums, the curve's tile sums, the counts
    int64_t slots = 0;
    const int64_t regions = float_regions(dims, &slots);
    if (regions < 0) return ECC_E_UNSUPPORTED;
    const int64_t digit_entries = std::max(radix_count_entries(n, 4), radix_count_entries(n, 8));
    const int64_t ft = float_tiles(n);
    enum { kKey0, kKey1, kNz, kNzCnt, kNzOff, kCounts, kSums, kTileA, kTileB, kBound, kCnt, kSteps, kNbuf };
    size_t off[kNbuf], total = 0;
    const int64_t scan_entries = std::max(std::max(digit_entries, regions), steps_only ? n : 0);
    const size_t sz[kNbuf] = {(size_t)n * 4, (size_t)n * 4, (size_t)slots * 8, (size_t)regions * 4,
                              (size_t)regions * 4, (size_t)digit_entries * 4,
                              (size_t)radix_scan_tiles(scan_entries) * 4, (size_t)ft * 8, (size_t)ft * 8,
                              (size_t)(ft + 1) * 8, 64,
                              steps_only ? (size_t)n * 4 : 0};
    for (int i = 0; i < kNbuf; ++i) {
        off[i] = total;
        total += align256(sz[i]);
    }
    // curve staging unless the caller's buffers are device memory that holds
    // any possible count (n entries)
    const bool direct = !steps_only && curve->capacity >= n && is_device_ptr(curve->chi) &&
                        is_device_ptr(curve->keys);
    const size_t out_k = total, out_c = out_k + align256((size_t)n * 4);
    if (!direct) total = out_c + align256((size_t)n * 8);
    rc = ensure_bytes(&ws->fbuf, &ws->fbuf_bytes, total);
    if (rc) return rc;
    uint8_t *b = (uint8_t *)ws->fbuf;
    uint32_t *key[2] = {(uint32_t *)(b + off[kKey0]), (uint32_t *)(b + off[kKey1])};
    uint32_t *nz_key = (uint32_t *)(b + off[kNz]);
    int32_t *nz_chg = (int32_t *)(nz_key + slots);
    uint32_t *nz_cnt = (uint32_t *)(b + off[kNzCnt]);
    uint32_t *nz_off = (uint32_t *)(b + off[kNzOff]);
    uint32_t *counts = (uint32_t *)(b + off[kCounts]);
    uint32_t *sums = (uint32_t *)(b + off[kSums]);
    int64_t *tile_a = (int64_t *)(b + off[kTileA]);
    int64_t *tile_b = (int64_t *)(b + off[kTileB]);
    int64_t *bound = (int64_t *)(b + off[kBound]);
    int64_t *nnz_dev = (int64_t *)(b + off[kCnt]);
    int64_t *count_dev = (int64_t *)(b + off[kCnt] + 8);
    int64_t *count2_dev = (int64_t *)(b + off[kCnt] + 16);
    uint32_t *mask_dev = (uint32_t *)(b + off[kCnt] + 32);  // the key sort's top-byte mask (8 words)
    float *out_keys = direct ? curve->keys : (float *)(b + out_k);
    int64_t *out_chi = direct ? curve->chi : (int64_t *)(b + out_c);
    // the record count, read on the host while the keys are sorted: a word of
    // the host-mapped status block
    volatile int64_t *nnz_host = (volatile int64_t *)(ws->host_status + 2);
    int64_t *nnz_host_dev = (int64_t *)(ws->host_status_dev + 2);
    *nnz_host = -1;

    rc = launch_float_change(img_dev, dims, key[0], nz_key, nz_chg, nz_cnt, nz_off, ws->status, s);
    if (rc) return rc;
    rc = launch_nz_total(nz_cnt, nz_off, regions, sums, nnz_dev, nnz_host_dev, s);
    if (rc) return rc;
    hipEvent_t counted = nullptr;
    ECC_HIP(hipEventCreateWithFlags(&counted, hipEventDisableTiming));
    hipError_t e = hipEventRecord(counted, s);
    if (e == hipSuccess) {
        rc = radix_sort_keys(key, n, counts, sums, mask_dev, ws->host_status + 4, ws->host_status_dev + 4, s);
        e = hipEventSynchronize(counted);
    }
    (void)hipEventDestroy(counted);
    ECC_HIP(e);
    if (rc) return rc;
    const int64_t nnz = *nnz_host;
    if (nnz < 0 || nnz > n) {
        set_error("internal error: %lld change records for %lld voxels", (long long)nnz, (long long)n);
        return ECC_E_HIP;
    }
    // the dense records (two sort buffers) and their prefix
    const size_t rb = align256((size_t)nnz * 8);
    rc = ensure_bytes(&ws->frec, &ws->frec_bytes, 3 * rb + 256);
    if (rc) return rc;
    uint64_t *rec[2] = {(uint64_t *)ws->frec, (uint64_t *)((uint8_t *)ws->frec + rb)};
    int64_t *prefix = (int64_t *)((uint8_t *)ws->frec + 2 * rb);
    if (nnz > 0) {
        rc = launch_nz_compact(nz_key, nz_chg, nz_cnt, nz_off, regions, slots / regions, rec[0], s);
        if (rc) return rc;
        rc = radix_sort_records(rec, nnz, counts, sums, s);
        if (rc) return rc;
    }
    rc = launch_float_curve(key[0], n, rec[0], nnz, prefix, (uint32_t *)tile_b, sums, tile_a, bound, count_dev, out_keys,
                            out_chi, s);
    if (rc) return rc;
    uint32_t st = 0;
    int64_t kcount = 0;
    ECC_HIP(hipMemcpyAsync(&st, ws->status, 4, hipMemcpyDeviceToHost, s));
    ECC_HIP(hipMemcpyAsync(&kcount, count_dev, 8, hipMemcpyDeviceToHost, s));
    ECC_HIP(hipStreamSynchronize(s));
    if (st != 0) {
        rc = launch_zero(ws->status, 4, s);
        if (rc) return rc;
        ECC_HIP(hipStreamSynchronize(s));
        if (st & kStatusNaN) {
            set_error("a float image holds a NaN");
            return ECC_E_NAN;
        }
        set_error("internal error: device status 0x%08x", st);
        return ECC_E_HIP;
    }
    if (steps_only) {  // compact into buffers free after the curve: the second key buffer, the regions
        float *step_keys = (float *)key[1];
        int64_t *step_chi = (int64_t *)nz_key;
        rc = launch_change_points(out_keys, out_chi, kcount, (uint32_t *)(b + off[kSteps]), sums, step_keys,
                                  step_chi, count2_dev, s);
        if (rc) return rc;
        ECC_HIP(hipMemcpyAsync(&kcount, count2_dev, 8, hipMemcpyDeviceToHost, s));
        ECC_HIP(hipStreamSynchronize(s));
        out_keys = step_keys;
        out_chi = step_chi;
    }
    if (kcount > curve->capacity) {
        curve->count = kcount;
        set_error("curve capacity %lld < %lld output entries", (long long)curve->capacity, (long long)kcount);
        return ECC_E_BUFFER_TOO_SMALL;
    }
    if (!direct) {
        ECC_HIP(hipMemcpyAsync(curve->keys, out_keys, (size_t)kcount * 4, hipMemcpyDefault, s));
        ECC_HIP(hipMemcpyAsync(curve->chi, out_chi, (size_t)kcount * 8, hipMemcpyDefault, s));
        ECC_HIP(hipStreamSynchronize(s));
    }
    curve->count = kcount;
    return ECC_OK;
}

// ws == nullptr: the per-(device, stream) workspace.
int compute_async_ws(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, int64_t *chi_dev,
                     uint32_t *status_dev, hipStream_t stream, Workspace *ws) {
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image_dev || !chi_dev) {
        set_error("NULL image or chi");
        return ECC_E_ARG;
    }
    if (dtype != ECC_U8 && dtype != ECC_U14 && dtype != ECC_U16) {
        if (dtype == ECC_F32) {
            set_error("ecc_compute_async: dtype %d not available in this library", (int)dtype);
            return ECC_E_UNSUPPORTED;
        }
        set_error("unknown dtype %d", (int)dtype);
        return ECC_E_ARG;
    }
    IntView v{};
    int unsup = 0;
    if (!normalize_int_view(dims, &v, &unsup)) {
        set_error("integer path: shape not supported (4 axes longer than 1, or an extent beyond 2^31)");
        return ECC_E_UNSUPPORTED;
    }
    if (!ws) {
        rc = get_workspace(stream, &ws);
        if (rc) return rc;
    }
    if (dtype == ECC_U16)  // stream-ordered: windows over all values (no host read of the value range)
        return enqueue_u16(image_dev, v, chi_dev, status_dev, stream, ws, 0, 65535);
    return enqueue_int(image_dev, v, dtype, chi_dev, status_dev, stream, ws);
}

}  // namespace ecc

using namespace ecc;

extern "C" {

const char *ecc_last_error(void) { return g_err; }

const char *ecc_version(void) { return "libecc 0.1 (gfx950)"; }

int ecc_threshold_count(ecc_dtype dtype, int64_t *m_out) {
    const int64_t m = threshold_count(dtype);
    if (m < 0 || !m_out) {
        set_error("not an integer dtype or NULL output");
        return ECC_E_ARG;
    }
    *m_out = m;
    return ECC_OK;
}

int ecc_compute_async(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, int64_t *chi_dev,
                      uint32_t *status_dev, void *stream) {
    g_err[0] = 0;
    return compute_async_ws(image_dev, dims, dtype, chi_dev, status_dev, (hipStream_t)stream, nullptr);
}

int ecc_compute(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve, void *stream) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image || !curve || !curve->chi) {
        set_error("NULL image, curve or curve->chi");
        return ECC_E_ARG;
    }
    if (dtype == ECC_F32) return compute_float(image, dims, total, curve, (hipStream_t)stream, false);
    return compute_int(image, dims, total, dtype, curve, (hipStream_t)stream, false);
}

int ecc_compute_max_entry(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve,
                          void *stream) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image || !curve || !curve->chi) {
        set_error("NULL image, curve or curve->chi");
        return ECC_E_ARG;
    }
    if (dtype == ECC_F32) {
        set_error("ecc_compute_max_entry: integer dtypes only");
        return ECC_E_UNSUPPORTED;
    }
    return compute_int(image, dims, total, dtype, curve, (hipStream_t)stream, true);
}

int ecc_compute_change_points(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve,
                              void *stream) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image || !curve || !curve->chi) {
        set_error("NULL image, curve or curve->chi");
        return ECC_E_ARG;
    }
    if (dtype != ECC_F32) {
        set_error("ecc_compute_change_points: ECC_F32 only");
        return dtype >= ECC_U8 && dtype <= ECC_U16 ? ECC_E_UNSUPPORTED : ECC_E_ARG;
    }
    return compute_float(image, dims, total, curve, (hipStream_t)stream, true);
}

int ecc_compute_quantized(const float *image, const ecc_dims *dims, float lo, float hi, ecc_dtype bins,
                          ecc_curve *curve, void *stream) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image || !curve || !curve->chi) {
        set_error("NULL image, curve or curve->chi");
        return ECC_E_ARG;
    }
    if (bins != ECC_U8 && bins != ECC_U14 && bins != ECC_U16) {
        set_error("ecc_compute_quantized: bins must be ECC_U8, ECC_U14 or ECC_U16");
        return ECC_E_ARG;
    }
    const float width = hi - lo;
    if (!(width > 0.0f) || !(width <= 3.0e38f)) {
        set_error("ecc_compute_quantized: need lo < hi, both finite");
        return ECC_E_ARG;
    }
    const int64_t m = threshold_count(bins);
    if (curve->capacity < m) {
        curve->count = m;
        set_error("curve capacity %lld < %lld", (long long)curve->capacity, (long long)m);
        return ECC_E_BUFFER_TOO_SMALL;
    }
    hipStream_t s = (hipStream_t)stream;
    Workspace *ws = nullptr;
    rc = get_workspace(s, &ws);
    if (rc) return rc;
    const float *img_dev = image;
    const size_t qbytes = (size_t)total * elem_bytes(bins);
    const size_t qoff = is_device_ptr(image) ? 0 : align256((size_t)total * 4);
    rc = ensure_bytes(&ws->img_tmp, &ws->img_tmp_bytes, qoff + qbytes);
    if (rc) return rc;
    if (qoff) {
        ECC_HIP(hipMemcpyAsync(ws->img_tmp, image, (size_t)total * 4, hipMemcpyHostToDevice, s));
        img_dev = (const float *)ws->img_tmp;
    }
    void *q = (uint8_t *)ws->img_tmp + qoff;
    const float scale = (float)m / width;
    uint32_t *flag = ws->status + kStatusMinMaxOffset / 4 + 2;  // NaN flag word
    rc = launch_zero(flag, 4, s);
    if (rc) return rc;
    rc = launch_quantize(img_dev, total, lo, scale, (int)m, (int)elem_bytes(bins), q, flag, s);
    if (rc) return rc;
    uint32_t nan = 0;
    ECC_HIP(hipMemcpyAsync(&nan, flag, 4, hipMemcpyDeviceToHost, s));
    ECC_HIP(hipStreamSynchronize(s));
    if (nan) {
        set_error("a float image holds a NaN");
        return ECC_E_NAN;
    }
    return compute_int(q, dims, total, bins, curve, s, false);
}

int ecc_autotune(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, void *stream, ecc_tiling *best) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image_dev || !best) {
        set_error("NULL image or output");
        return ECC_E_ARG;
    }
    if (dtype != ECC_U8 && dtype != ECC_U14) {
        set_error("ecc_autotune: U8 or U14 images");
        return (dtype == ECC_U16 || dtype == ECC_F32) ? ECC_E_UNSUPPORTED : ECC_E_ARG;
    }
    if (!is_device_ptr(image_dev)) {
        set_error("ecc_autotune: the image must be device memory");
        return ECC_E_ARG;
    }
    IntView v{};
    int unsup = 0;
    if (!normalize_int_view(dims, &v, &unsup)) {
        set_error("integer path: shape not supported (4 axes longer than 1, or an extent beyond 2^31)");
        return ECC_E_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    Workspace *ws = nullptr;
    rc = get_workspace(s, &ws);
    if (rc) return rc;
    const int m = (int)threshold_count(dtype);
    rc = ensure_bytes((void **)&ws->vcec, &ws->vcec_bytes, (size_t)m * sizeof(int64_t));
    if (rc) return rc;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return hip_fail(e, "ecc_autotune: events");
    }
    ecc_tiling win{};
    win.ms = 1e30f;
    const ecc_tiling rule = rule_tiling(v, dtype, v.n0);
    float rule_ms = 1e30f;
    IntJob job{};
    job.src.base = (const uint8_t *)image_dev;
    job.src.lo_base = job.src.base;
    job.src.plane_bytes = (int64_t)v.n1 * v.n2 * (int64_t)elem_bytes(dtype);
    job.view = v;
    job.e0 = 0;
    job.e1 = (int32_t)v.n0;
    job.lo_inf = 1;
    job.hi_inf = 1;
    job.dtype = dtype;
    // candidates, timed in rounds over all of them (one warm-up round, then
    // three; each keeps its fastest) so that clock ramps and drift do not
    // favour the ones timed last
    const int rows_c[2] = {2, 4}, tpc_c[3] = {4, 8, 16}, wx_c[2] = {8, 16};
    struct Cand {
        ecc_tiling p;
        IntTiling tl;
        float best;
    };
    std::vector<Cand> cands;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < (v.nin == 2 ? 2 : 1); ++c) {
                Cand x{};
                x.p.rows = rows_c[a];
                x.p.tiles_per_cu = tpc_c[b];
                x.p.waves_x = wx_c[c + (v.nin == 2 ? 0 : 1)];
                x.tl = make_int_tiling(v, v.n0, x.p.rows, x.p.tiles_per_cu, x.p.waves_x);
                x.best = 1e30f;
                cands.push_back(x);
                if (!rc) rc = ensure_bytes((void **)&ws->partial, &ws->partial_bytes,
                                           (size_t)x.tl.grid * m * sizeof(int32_t));
                if (!rc)
                    rc = ensure_bytes((void **)&ws->stage, &ws->stage_bytes,
                                      (size_t)merge_stage_rows(x.tl.grid) * m * sizeof(int64_t));
            }
    for (int round = 0; round < 4 && !rc; ++round)
        for (Cand &x : cands) {
            if ((e = hipEventRecord(ev[0], s)) != hipSuccess) rc = hip_fail(e, "ecc_autotune: event");
            if (!rc) rc = launch_int_partial(job, x.tl, ws->partial, ws->status, nullptr, s);
            if (!rc)
                rc = launch_merge(ws->partial, x.tl.grid, m, ws->stage, ws->vcec, false, false, nullptr, ws->status,
                                  nullptr, s);
            if (!rc && (e = hipEventRecord(ev[1], s)) != hipSuccess) rc = hip_fail(e, "ecc_autotune: event");
            if (!rc && (e = hipEventSynchronize(ev[1])) != hipSuccess) rc = hip_fail(e, "ecc_autotune: sync");
            float ms = 0.0f;
            if (!rc && (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) rc = hip_fail(e, "ecc_autotune");
            if (!rc && round > 0 && ms < x.best) x.best = ms;
            if (rc) break;
        }
    for (const Cand &x : cands) {
        if (x.p.rows == rule.rows && x.p.tiles_per_cu == rule.tiles_per_cu && x.p.waves_x == rule.waves_x)
            rule_ms = x.best;
        if (x.best < win.ms) {
            win = x.p;
            win.ms = x.best;
        }
    }
    // the rule stays unless a candidate beats it by 2 % (timing noise would
    // otherwise flip between near-equal tilings from run to run)
    if (!rc && win.ms > 0.98f * rule_ms) {
        win = rule;
        win.ms = rule_ms;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc) return rc;
    // the status word collects range errors of the timed runs; read and clear it
    uint32_t st = 0;
    ECC_HIP(hipMemcpyAsync(&st, ws->status, 4, hipMemcpyDeviceToHost, s));
    ECC_HIP(hipStreamSynchronize(s));
    rc = launch_zero(ws->status, 8, s);
    if (rc) return rc;
    ECC_HIP(hipStreamSynchronize(s));
    if (st & kStatusRange) {
        set_error("a 14-bit image holds a value >= 16384");
        return ECC_E_RANGE;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[TuneKey{dtype, v.nin, v.n1, v.n2, v.n0}] = win;
    }
    *best = win;
    return ECC_OK;
}

int ecc_tiling_for(const ecc_dims *dims, ecc_dtype dtype, ecc_tiling *out) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!out) {
        set_error("NULL output");
        return ECC_E_ARG;
    }
    if (dtype != ECC_U8 && dtype != ECC_U14 && dtype != ECC_U16) {
        set_error("ecc_tiling_for: integer dtypes");
        return dtype == ECC_F32 ? ECC_E_UNSUPPORTED : ECC_E_ARG;
    }
    IntView v{};
    int unsup = 0;
    if (!normalize_int_view(dims, &v, &unsup)) {
        set_error("integer path: shape not supported");
        return ECC_E_UNSUPPORTED;
    }
    *out = tiling_params(v, dtype, v.n0);
    out->ms = 0.0f;
    return ECC_OK;
}

void ecc_autotune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

// The growable scratch of every workspace of the current device is freed
// (the small status block and host word stay, so the workspaces remain
// valid); the next call on a stream grows its buffers again.  Work still in
// flight on the device may use them: it is waited for first.
int ecc_release_workspaces(void) {
    int dev = 0;
    ECC_HIP(hipGetDevice(&dev));
    ECC_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(g_ws_mu);
    hipError_t first = hipSuccess;
    auto drop = [&](void *p, size_t *cap) {
        if (p) {
            const hipError_t e = hipFree(p);
            if (e != hipSuccess && first == hipSuccess) first = e;
        }
        *cap = 0;
    };
    for (auto &kv : g_ws) {
        Workspace *w = kv.second;
        if (w->device != dev || w->fixed) continue;
        drop(w->partial, &w->partial_bytes);
        w->partial = nullptr;
        drop(w->vcec, &w->vcec_bytes);
        w->vcec = nullptr;
        drop(w->stage, &w->stage_bytes);
        w->stage = nullptr;
        drop(w->chi_tmp, &w->chi_tmp_bytes);
        w->chi_tmp = nullptr;
        drop(w->img_tmp, &w->img_tmp_bytes);
        w->img_tmp = nullptr;
        drop(w->fbuf, &w->fbuf_bytes);
        w->fbuf = nullptr;
        drop(w->frec, &w->frec_bytes);
        w->frec = nullptr;
        drop(w->dual_buf, &w->dual_buf_bytes);
        w->dual_buf = nullptr;
        drop(w->i2f_buf, &w->i2f_buf_bytes);
        w->i2f_buf = nullptr;
        drop(w->vcec16, &w->vcec16_bytes);
        w->vcec16 = nullptr;
    }
    if (first != hipSuccess) return hip_fail(first, "hipFree(workspace)");
    return ECC_OK;
}

static const char kTuneTag[] = "ecc-tiling-v1";

int ecc_autotune_save(const char *path) {
    g_err[0] = 0;
    if (!path) {
        set_error("ecc_autotune_save: NULL path");
        return ECC_E_ARG;
    }
    std::vector<std::pair<TuneKey, ecc_tiling>> rows;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        rows.assign(g_tuned.begin(), g_tuned.end());
    }
    FILE *f = fopen(path, "w");
    if (!f) {
        set_error("ecc_autotune_save: cannot open %s for writing", path);
        return ECC_E_ARG;
    }
    bool ok = true;
    for (const auto &r : rows)
        ok = ok && fprintf(f, "%s %d %d %d %d %lld %d %d %d %.6g\n", kTuneTag, r.first.dtype, r.first.nin,
                           (int)r.first.n1, (int)r.first.n2, (long long)r.first.planes, (int)r.second.rows,
                           (int)r.second.tiles_per_cu, (int)r.second.waves_x, (double)r.second.ms) > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok) {
        set_error("ecc_autotune_save: write to %s failed", path);
        return ECC_E_ARG;
    }
    return (int)rows.size();
}

int ecc_autotune_load(const char *path) {
    g_err[0] = 0;
    if (!path) {
        set_error("ecc_autotune_load: NULL path");
        return ECC_E_ARG;
    }
    FILE *f = fopen(path, "r");
    if (!f) {
        set_error("ecc_autotune_load: cannot open %s", path);
        return ECC_E_ARG;
    }
    std::vector<std::pair<TuneKey, ecc_tiling>> rows;
    char line[512];
    int lineno = 0;
    bool ok = true;
    while (ok && fgets(line, sizeof line, f)) {
        ++lineno;
        char tag[32] = {0}, extra[2] = {0};
        int dtype = 0, nin = 0, n1 = 0, n2 = 0, r = 0, tpc = 0, wx = 0;
        long long planes = 0;
        double ms = 0;
        const int got = sscanf(line, "%31s %d %d %d %d %lld %d %d %d %lf %1s", tag, &dtype, &nin, &n1, &n2, &planes, &r,
                               &tpc, &wx, &ms, extra);
        if (got == EOF || (got == 1 && tag[0] == '#')) continue;  // blank line or comment
        ok = got == 10 && strcmp(tag, kTuneTag) == 0 && threshold_count((ecc_dtype)dtype) > 0 &&
             dtype != ECC_F32 && (nin == 1 || nin == 2) && n1 >= 1 && n2 >= 1 && planes >= 1 &&
             (r == 2 || r == 4) && (tpc == 4 || tpc == 8 || tpc == 16) && (wx == 8 || wx == 16) && ms >= 0;
        if (ok) {
            ecc_tiling t{};
            t.rows = r;
            t.tiles_per_cu = tpc;
            t.waves_x = wx;
            t.ms = (float)ms;
            rows.push_back({TuneKey{dtype, nin, n1, n2, (int64_t)planes}, t});
        }
    }
    const bool read_ok = !ferror(f);
    fclose(f);
    if (!ok || !read_ok) {
        if (!ok) set_error("ecc_autotune_load: %s line %d is not a tiling entry", path, lineno);
        else set_error("ecc_autotune_load: reading %s failed", path);
        return ECC_E_ARG;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &e : rows) g_tuned[e.first] = e.second;
    return (int)rows.size();
}

// Dual complex (voxels as vertices, lower-star filtration).  Its cells are
// the cells of the voxel complex away from the box's outer boundary, with
// dimension d - dim and value the maximum over their voxels, so by
// inclusion-exclusion over the faces F of the box (every axis free, or fixed
// at its first or last index):
//   dual(f)(t) = (-1)^d sum_F (-1)^codim(F) max_entry(f|F)(t).
// The sum is linear, so it is taken over the faces' changes vectors and the
// result is scanned once.  Axes of length 1 are dropped first (a product
// with a point).
int ecc_compute_dual(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve, void *stream) {
    g_err[0] = 0;
    int64_t total = 0;
    int rc = check_dims(dims, &total);
    if (rc) return rc;
    if (!image || !curve || !curve->chi) {
        set_error("NULL image, curve or curve->chi");
        return ECC_E_ARG;
    }
    if (dtype != ECC_U8 && dtype != ECC_U14) {
        if (dtype == ECC_F32 || dtype == ECC_U16) {
            set_error("ecc_compute_dual: integer dtypes u8 and u14 only");
            return ECC_E_UNSUPPORTED;
        }
        set_error("unknown dtype %d", (int)dtype);
        return ECC_E_ARG;
    }
    const int64_t m = threshold_count(dtype);
    if (curve->capacity < m) {
        curve->count = m;
        set_error("curve capacity %lld < %lld", (long long)curve->capacity, (long long)m);
        return ECC_E_BUFFER_TOO_SMALL;
    }
    int64_t n[4];
    int d = 0;
    for (int k = 0; k < dims->ndim; ++k)
        if (dims->n[k] > 1) n[d++] = dims->n[k];
    // (d <= 4: the full box of a 4-D image goes through the float path, its
    // faces of at most three dimensions through the integer kernel)
    hipStream_t s = (hipStream_t)stream;
    Workspace *ws = nullptr;
    rc = get_workspace(s, &ws);
    if (rc) return rc;
    const size_t eb = elem_bytes(dtype);
    const void *img_dev = image;
    if (!is_device_ptr(image)) {
        rc = ensure_bytes(&ws->img_tmp, &ws->img_tmp_bytes, (size_t)total * eb);
        if (rc) return rc;
        ECC_HIP(hipMemcpyAsync(ws->img_tmp, image, (size_t)total * eb, hipMemcpyHostToDevice, s));
        img_dev = ws->img_tmp;
    }
    int nf = 1;
    for (int k = 0; k < d; ++k) nf *= 3;
    int64_t st[4] = {1, 1, 1, 1};  // element strides of the kept axes
    for (int k = d - 2; k >= 0; --k) st[k] = st[k + 1] * n[k + 1];
    int64_t face_max = 1;  // the largest face of codimension >= 1
    for (int k = 0; k < d; ++k)
        if (total / n[k] > face_max) face_max = total / n[k];
    // dual_buf: [nf][m] per-face changes vectors, [m] the changes of the
    // faces of at most one dimension (all of them, signed), [m] the signed
    // sum, the table of faces of at most one dimension
    const size_t curves_bytes = (size_t)(nf + 2) * m * sizeof(int64_t);
    const size_t low_off = (curves_bytes + 255) & ~(size_t)255;
    rc = ensure_bytes(&ws->dual_buf, &ws->dual_buf_bytes, low_off + ((nf * sizeof(LowFace) + 255) & ~(size_t)255));
    if (rc) return rc;
    int64_t *curves = (int64_t *)ws->dual_buf;
    int64_t *lowv = curves + (size_t)nf * m;
    int64_t *result = lowv + m;
    LowFace *low_dev = (LowFace *)((uint8_t *)ws->dual_buf + low_off);
    // Faces of two or more dimensions below the full box go round-robin to
    // the side streams, each with its own workspace (and gather buffer in
    // its img_tmp); the full box runs on s.
    SideStreams *side = nullptr;
    rc = get_side_streams(s, &side);
    if (rc) return rc;
    Workspace *sws[SideStreams::kCount];
    for (int k = 0; k < SideStreams::kCount; ++k) {
        rc = get_workspace(side->s[k], &sws[k]);
        if (rc) return rc;
    }
    bool used[SideStreams::kCount] = {};
    int next_side = 0;
    // after the fork, every return first waits for the side streams (their
    // work uses buffers that a later call may reallocate)
    auto sync_sides = [&]() {
        for (int k = 0; k < SideStreams::kCount; ++k)
            if (used[k]) (void)hipStreamSynchronize(side->s[k]);
    };
    ECC_HIP(hipEventRecord(side->fork, s));  // the image (and its copy, if any) is ready here
    const int gsign = (d & 1) ? -1 : 1;
    uint64_t neg[2] = {0, 0}, skip[2] = {0, 0};  // bit f of the pair: face f
    auto set_bit = [](uint64_t *mask, int f) { mask[f >> 6] |= 1ull << (f & 63); };
    // Box edges and corners (faces of at most one dimension, below the full
    // box) have a closed-form changes vector; they are added by one launch
    // after the signed sum instead of a gather, a kernel and a merge each.
    std::vector<LowFace> low;
    for (int f = 0; f < nf; ++f) {
        int code[4] = {0, 0, 0, 0};
        for (int k = 0, r = f; k < d; ++k, r /= 3) code[k] = r % 3;
        int codim = 0, nfree = 0;
        int64_t base = 0, fs[4] = {1, 1, 1, 1}, fst[4] = {0, 0, 0, 0};
        for (int k = 0; k < d; ++k) {
            if (code[k] == 0) {
                fs[nfree] = n[k];
                fst[nfree] = st[k];
                ++nfree;
            } else {
                base += (code[k] == 1 ? 0 : n[k] - 1) * st[k];
                ++codim;
            }
        }
        if (codim > 0 && nfree <= 1) {
            LowFace L{};
            L.base = base;
            L.stride = nfree ? fst[0] : 0;
            L.len = nfree ? fs[0] : 0;
            L.sign = (codim & 1) ? -gsign : gsign;
            low.push_back(L);
            set_bit(skip, f);
            continue;
        }
        if (nfree == 4) {  // the whole 4-D box
            ecc_dims bd{};
            bd.ndim = 4;
            for (int k = 0; k < 4; ++k) bd.n[k] = n[k];
            rc = int_via_float_dev(img_dev, &bd, total, dtype, true, true, curves + (size_t)f * m, s, ws);
            if (rc) {
                sync_sides();
                return rc;
            }
            continue;
        }
        // the full box on s, a face on the next side stream
        const int k = codim > 0 ? (next_side++ % SideStreams::kCount) : -1;
        hipStream_t fs_stream = k < 0 ? s : side->s[k];
        Workspace *fws = k < 0 ? ws : sws[k];
        if (k >= 0 && !used[k]) {
            hipError_t e = hipStreamWaitEvent(fs_stream, side->fork, 0);
            if (e != hipSuccess) {
                sync_sides();
                return hip_fail(e, "ecc_compute_dual: fork");
            }
            used[k] = true;
        }
        const void *src = img_dev;
        int64_t pstride = 0;
        if (codim > 0 && nfree == 2 && fst[1] == 1 && fst[0] * (int64_t)eb <= INT32_MAX) {
            // a 2-D face whose rows are contiguous in the image: walked in
            // place, one row per plane, fst[0] elements apart
            src = (const uint8_t *)img_dev + base * (int64_t)eb;
            pstride = fst[0];
        } else if (codim > 0) {
            // free axes as the trailing axes of an n0 x n1 x n2 gather, into
            // the side stream's buffer (its faces run in stream order)
            int64_t g[3] = {1, 1, 1}, gs[3] = {0, 0, 0};
            for (int i = 0; i < nfree; ++i) {
                g[3 - nfree + i] = fs[i];
                gs[3 - nfree + i] = fst[i];
            }
            rc = ensure_bytes(&fws->img_tmp, &fws->img_tmp_bytes, (size_t)face_max * eb);
            if (!rc) rc = launch_gather(img_dev, (int)eb, base, gs[0], gs[1], gs[2], g[0], g[1], g[2], fws->img_tmp, fs_stream);
            if (rc) {
                sync_sides();
                return rc;
            }
            src = fws->img_tmp;
        }
        ecc_dims fd{};
        fd.ndim = nfree > 0 ? nfree : 1;
        for (int i = 0; i < 4; ++i) fd.n[i] = 1;
        for (int i = 0; i < nfree; ++i) fd.n[i] = fs[i];
        IntView v{};
        int unsup = 0;
        if (!normalize_int_view(&fd, &v, &unsup)) {
            sync_sides();
            set_error("ecc_compute_dual: face shape not supported");
            return ECC_E_UNSUPPORTED;
        }
        rc = enqueue_int_changes(src, v, dtype, curves + (size_t)f * m, fs_stream, fws, true, pstride);
        if (rc) {
            sync_sides();
            return rc;
        }
        if (codim & 1) set_bit(neg, f);
    }
    // Box edges and corners: their table, a cleared vector and the
    // closed-form changes on the next side stream, summed as one more face
    // (slot nf, whose entries carry their signs already: the global sign
    // is cancelled by the slot's own).  The host table must outlive the
    // copy: every return below this point waits for the side streams (the
    // join and the final synchronisation of s, or sync_sides).
    if (!low.empty()) {
        const int k = next_side % SideStreams::kCount;
        hipStream_t ls = side->s[k];
        hipError_t e = hipSuccess;
        if (!used[k]) e = hipStreamWaitEvent(ls, side->fork, 0);
        used[k] = true;
        if (e == hipSuccess)
            e = hipMemcpyAsync(low_dev, low.data(), low.size() * sizeof(LowFace), hipMemcpyHostToDevice, ls);
        if (e != hipSuccess) {
            sync_sides();
            return hip_fail(e, "ecc_compute_dual: edge and corner table");
        }
        rc = launch_zero(lowv, (size_t)m * sizeof(int64_t), ls);
        if (!rc) rc = launch_low_faces(img_dev, (int)eb, low_dev, (int)low.size(), (int)m, lowv, ls);
        if (rc) {
            sync_sides();
            return rc;
        }
        if (gsign < 0) set_bit(neg, nf);
    } else {
        set_bit(skip, nf);
    }
    // join: s waits for every side stream that took work
    for (int k = 0; k < SideStreams::kCount; ++k) {
        if (!used[k]) continue;
        hipError_t e = hipEventRecord(side->join[k], side->s[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, side->join[k], 0);
        if (e != hipSuccess) {
            sync_sides();
            return hip_fail(e, "ecc_compute_dual: join");
        }
    }
    rc = launch_signed_sum(curves, nf + 1, neg, skip, gsign, (int)m, result, s);
    if (rc) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    // scan into slot 0 (its changes are summed already); the status of every
    // face launch (all read the image's values) is reported and cleared here
    int64_t *chi_dev = curves;
    *ws->host_status = 0xFFFFFFFFu;  // overwritten by the scan
    rc = launch_merge(nullptr, 0, (int)m, nullptr, result, true, true, chi_dev, ws->status, ws->host_status_dev, s);
    if (rc) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    ECC_HIP(hipStreamSynchronize(s));
    const uint32_t stv = *ws->host_status;
    if (stv == 0xFFFFFFFFu) {
        set_error("internal error: the scan did not report a status");
        return ECC_E_HIP;
    }
    if (stv & kStatusRange) {
        set_error("a 14-bit image holds a value >= 16384");
        return ECC_E_RANGE;
    }
    if (stv != 0) {
        set_error("internal error: device status 0x%08x", stv);
        return ECC_E_HIP;
    }
    ECC_HIP(hipMemcpyAsync(curve->chi, chi_dev, (size_t)m * sizeof(int64_t), hipMemcpyDefault, s));
    ECC_HIP(hipStreamSynchronize(s));
    curve->count = m;
    return ECC_OK;
}

}  // extern "C"
