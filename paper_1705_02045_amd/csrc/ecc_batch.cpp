// Batched and served computation of many independent images (integer dtypes).
//
// The curves of different images are independent (Sec. 3, "Parallel
// Computations": VCECs of disjoint parts merge by addition, and unrelated
// images simply do not merge), so one launch can hold the tiles of many
// images: a host-built descriptor table gives every image its kernel
// parameters and its range of workgroups, and a batched merge sums and scans
// each image's rows into its own curve.
//
// ecc_serve_simulate replays a stream of requests with given arrival times
// against the device, either with continuous batching (everything that has
// arrived when the device can take more work goes into the next batch) or
// one launch per image, and reports each request's latency from arrival to
// its curve being in host memory.

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <vector>

#include "ecc_internal.h"

struct ecc_batch {
    int device = -1;
    hipStream_t stream = nullptr;
    // descriptor tables: a ring of pinned host staging areas and device copies
    static constexpr int kSlots = 4;
    void *host[kSlots] = {};
    void *dev[kSlots] = {};
    size_t cap[kSlots] = {};
    hipEvent_t done[kSlots] = {};
    bool used[kSlots] = {};
    int next = 0;
    // scratch shared by consecutive runs (ordered by the stream)
    int32_t *partial8 = nullptr;
    size_t partial8_bytes = 0;
    int32_t *partial14 = nullptr;
    size_t partial14_bytes = 0;
    int64_t *vcec = nullptr;
    size_t vcec_bytes = 0;
    uint32_t *status = nullptr;  // one word per image, zero between runs
    size_t status_bytes = 0;
};

namespace {

using namespace ecc;

// Tiling of one image inside a batch: 2 rows per wave, 16-wave workgroups,
// tiles of at least 64 planes (or the whole image) so that small images take
// one workgroup and large ones a few hundred.
IntTiling batch_tiling(const IntView &v) {
    IntTiling t{};
    t.rows = 2;
    t.mode = 0;
    t.pd = 1;
    const int max_waves = 16;
    int64_t tiles_xy;
    if (v.nin == 1) {
        const int64_t segs = (v.n2 + (int64_t)kWave * t.rows - 1) / ((int64_t)kWave * t.rows);
        t.wx = (int)std::min<int64_t>(segs, max_waves);
        t.wy = 1;
        tiles_xy = (segs + t.wx - 1) / t.wx;
    } else {
        const int64_t xs = (v.n2 + kWave - 1) / kWave;
        t.wx = (int)std::min<int64_t>(xs, max_waves);
        const int64_t ys = (v.n1 + t.rows - 1) / t.rows;
        t.wy = (int)std::min<int64_t>(ys, max_waves / t.wx);
        tiles_xy = ((xs + t.wx - 1) / t.wx) * ((ys + t.wy - 1) / t.wy);
    }
    int64_t zc = std::max<int64_t>(64, (v.n0 + 3) / 4);
    if (zc > v.n0) zc = v.n0;
    t.zc = (int)zc;
    t.per_wg = 1;
    t.grid = (int)(tiles_xy * ((v.n0 + zc - 1) / zc));
    return t;
}

int grow(ecc_batch *b, void **p, size_t *cap, size_t need) {
    if (*cap >= need && *p) return ECC_OK;
    ECC_HIP(hipStreamSynchronize(b->stream));  // in-flight runs may still use it
    return ensure_bytes(p, cap, need);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Prepared {
    IntView view;
    IntTiling tl;
    int group;  // (dtype == U14) * 2 + (nin == 2)
    int m;
};

}  // namespace

extern "C" {

int ecc_batch_create(void *stream, ecc_batch **out) {
    if (!out) {
        set_error("ecc_batch_create: NULL output");
        return ECC_E_ARG;
    }
    *out = nullptr;
    ecc_batch *b = new ecc_batch();
    b->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&b->device);
    for (int i = 0; e == hipSuccess && i < ecc_batch::kSlots; ++i)
        e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "ecc_batch_create");
        for (int i = 0; i < ecc_batch::kSlots; ++i)
            if (b->done[i]) (void)hipEventDestroy(b->done[i]);
        delete b;
        return rc;
    }
    *out = b;
    return ECC_OK;
}

void ecc_batch_destroy(ecc_batch *b) {
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (int i = 0; i < ecc_batch::kSlots; ++i) {
        if (b->host[i]) (void)hipHostFree(b->host[i]);
        if (b->dev[i]) (void)hipFree(b->dev[i]);
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
    }
    if (b->partial8) (void)hipFree(b->partial8);
    if (b->partial14) (void)hipFree(b->partial14);
    if (b->vcec) (void)hipFree(b->vcec);
    if (b->status) (void)hipFree(b->status);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete b;
}

int ecc_batch_run(ecc_batch *b, int32_t n_jobs, const ecc_job *jobs, uint32_t *status_dev) {
    g_err_clear();
    if (!b || n_jobs < 0 || (n_jobs > 0 && !jobs)) {
        set_error("ecc_batch_run: bad argument");
        return ECC_E_ARG;
    }
    if (n_jobs == 0) return ECC_OK;
    std::vector<Prepared> prep(n_jobs);
    int64_t rows[4] = {0, 0, 0, 0};
    int64_t cnt[4] = {0, 0, 0, 0};
    int64_t vcec_words = 0;
    int max_m = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const ecc_job &J = jobs[j];
        int64_t total = 0;
        int rc = check_dims(&J.dims, &total);
        if (rc) return rc;
        if (!J.image || !J.chi) {
            set_error("job %d: NULL image or chi", j);
            return ECC_E_ARG;
        }
        if (J.dtype != ECC_U8 && J.dtype != ECC_U14) {
            set_error("job %d: batches take U8 or U14 images", j);
            return (J.dtype == ECC_U16 || J.dtype == ECC_F32) ? ECC_E_UNSUPPORTED : ECC_E_ARG;
        }
        Prepared &P = prep[j];
        int unsup = 0;
        if (!normalize_int_view(&J.dims, &P.view, &unsup)) {
            set_error("job %d: shape not supported", j);
            return ECC_E_UNSUPPORTED;
        }
        P.tl = batch_tiling(P.view);
        P.group = (J.dtype == ECC_U14 ? 2 : 0) + (P.view.nin == 2 ? 1 : 0);
        P.m = (int)threshold_count(J.dtype);
        rows[P.group] += P.tl.grid;
        cnt[P.group] += 1;
        vcec_words += P.m;
        max_m = std::max(max_m, P.m);
    }
    for (int g = 0; g < 4; ++g)
        if (rows[g] > INT32_MAX) {
            set_error("ecc_batch_run: too many tiles in one batch");
            return ECC_E_UNSUPPORTED;
        }
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != b->device) ECC_HIP(hipSetDevice(b->device));
    int rc = ECC_OK;
    do {
        // device scratch
        const int64_t rows8 = rows[0] + rows[1], rows14 = rows[2] + rows[3];
        if ((rc = grow(b, (void **)&b->partial8, &b->partial8_bytes, (size_t)rows8 * 256 * 4))) break;
        if ((rc = grow(b, (void **)&b->partial14, &b->partial14_bytes, (size_t)rows14 * 16384 * 4))) break;
        if ((rc = grow(b, (void **)&b->vcec, &b->vcec_bytes, (size_t)vcec_words * 8))) break;
        if (b->status_bytes < (size_t)n_jobs * 4 || !b->status) {
            if ((rc = grow(b, (void **)&b->status, &b->status_bytes, (size_t)n_jobs * 4))) break;
            if ((rc = launch_zero(b->status, b->status_bytes, b->stream))) break;
        }
        // table layout: per group KParams[cnt] and tile_begin[cnt + 1], then MergeJob[n]
        const size_t kp = kparams_bytes();
        size_t off_kp[4], off_tb[4], total = 0;
        for (int g = 0; g < 4; ++g) {
            off_kp[g] = total;
            total = align_up(total + (size_t)cnt[g] * kp, 16);
            off_tb[g] = total;
            total = align_up(total + (size_t)(cnt[g] + 1) * 4, 16);
        }
        const size_t off_mj = total;
        total = align_up(total + (size_t)n_jobs * sizeof(MergeJob), 256);
        // a free slot (its previous run's table copy has been consumed)
        const int s = b->next;
        b->next = (s + 1) % ecc_batch::kSlots;
        if (b->used[s]) {
            hipError_t e = hipEventSynchronize(b->done[s]);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_batch_run: slot wait");
                break;
            }
        }
        if (b->cap[s] < total) {
            if (b->host[s]) (void)hipHostFree(b->host[s]);
            if (b->dev[s]) (void)hipFree(b->dev[s]);
            b->host[s] = b->dev[s] = nullptr;
            b->cap[s] = 0;
            hipError_t e = hipHostMalloc(&b->host[s], total, hipHostMallocDefault);
            if (e == hipSuccess) e = hipMalloc(&b->dev[s], total);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_batch_run: table allocation");
                break;
            }
            b->cap[s] = total;
        }
        uint8_t *h = (uint8_t *)b->host[s];
        uint8_t *d = (uint8_t *)b->dev[s];
        int64_t idx[4] = {0, 0, 0, 0}, row_in_group[4] = {0, 0, 0, 0};
        int64_t row8 = 0, row14 = 0, vw = 0;
        for (int g = 0; g < 4; ++g) ((int32_t *)(h + off_tb[g]))[0] = 0;
        MergeJob *mj = (MergeJob *)(h + off_mj);
        for (int j = 0; j < n_jobs; ++j) {
            const Prepared &P = prep[j];
            const int g = P.group;
            int32_t *part;
            if (P.m == 256) {
                part = b->partial8 + row8 * 256;
                row8 += P.tl.grid;
            } else {
                part = b->partial14 + row14 * 16384;
                row14 += P.tl.grid;
            }
            IntJob job{};
            job.src.base = (const uint8_t *)jobs[j].image;
            job.src.lo_base = job.src.base;
            job.src.plane_bytes = (int64_t)P.view.n1 * P.view.n2 * (int64_t)elem_bytes(jobs[j].dtype);
            job.view = P.view;
            job.e0 = 0;
            job.e1 = (int32_t)P.view.n0;
            job.lo_inf = 1;
            job.hi_inf = 1;
            job.dtype = jobs[j].dtype;
            fill_kparams(h + off_kp[g] + (size_t)idx[g] * kp, job, P.tl, part, b->status + j);
            row_in_group[g] += P.tl.grid;
            ((int32_t *)(h + off_tb[g]))[idx[g] + 1] = (int32_t)row_in_group[g];
            idx[g] += 1;
            mj[j].partial = part;
            mj[j].rows = P.tl.grid;
            mj[j].m = P.m;
            mj[j].vcec = b->vcec + vw;
            mj[j].chi = jobs[j].chi;
            mj[j].status = b->status + j;
            mj[j].status_out = status_dev ? status_dev + j : nullptr;
            vw += P.m;
        }
        hipError_t e = hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, b->stream);
        if (e != hipSuccess) {
            rc = hip_fail(e, "ecc_batch_run: table copy");
            break;
        }
        for (int g = 0; g < 4 && !rc; ++g)
            if (cnt[g] > 0)
                rc = launch_int_batch(g >= 2 ? ECC_U14 : ECC_U8, (g & 1) ? 2 : 1, d + off_kp[g],
                                      (const int32_t *)(d + off_tb[g]), (int)cnt[g], (int)rows[g], b->stream);
        if (rc) break;
        rc = launch_batch_merge((const MergeJob *)(d + off_mj), n_jobs, max_m, b->stream);
        if (rc) break;
        e = hipEventRecord(b->done[s], b->stream);
        if (e != hipSuccess) {
            rc = hip_fail(e, "ecc_batch_run: event");
            break;
        }
        b->used[s] = true;
    } while (0);
    if (prev != b->device) (void)hipSetDevice(prev);
    return rc;
}

int ecc_serve_simulate(ecc_batch *b, int32_t n, const ecc_job *jobs, const double *arrival_s, int32_t max_batch,
                       int32_t one_launch_per_image, int64_t *chi_host, double *latency_s) {
    g_err_clear();
    if (!b || n < 1 || !jobs || !arrival_s || !chi_host || !latency_s || max_batch < 1) {
        set_error("ecc_serve_simulate: bad argument");
        return ECC_E_ARG;
    }
    for (int i = 1; i < n; ++i)
        if (arrival_s[i] < arrival_s[i - 1]) {
            set_error("ecc_serve_simulate: arrivals must be sorted");
            return ECC_E_ARG;
        }
    // every request writes its curve to a device staging area laid out in
    // request order, so a batch's curves go to the host in one copy
    std::vector<int64_t> off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const int64_t m = threshold_count(jobs[i].dtype);
        if (m < 0) {
            set_error("request %d: bad dtype", i);
            return ECC_E_ARG;
        }
        off[i + 1] = off[i] + m;
    }
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != b->device) ECC_HIP(hipSetDevice(b->device));
    // curves land in pinned host memory (a copy into pageable memory would
    // block the host thread until the stream drains) and are copied to
    // chi_host at the end
    int64_t *chi_dev = nullptr, *chi_pin = nullptr;
    hipError_t e = hipMalloc(&chi_dev, (size_t)off[n] * 8);
    if (e == hipSuccess) e = hipHostMalloc(&chi_pin, (size_t)off[n] * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
        if (chi_dev) (void)hipFree(chi_dev);
        if (prev != b->device) (void)hipSetDevice(prev);
        return hip_fail(e, "ecc_serve_simulate: curve staging");
    }
    std::vector<ecc_job> js(jobs, jobs + n);
    for (int i = 0; i < n; ++i) js[i].chi = chi_dev + off[i];
    struct Flight {
        hipEvent_t ev;
        int first, last;
    };
    std::deque<Flight> flight;
    std::vector<hipEvent_t> pool;
    int rc = ECC_OK;
    const int max_inflight = one_launch_per_image ? (1 << 30) : 2;
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    int next = 0, arrived = 0, done = 0;
    while (done < n && !rc) {
        const double t = now();
        while (arrived < n && arrival_s[arrived] <= t) ++arrived;
        while (next < arrived && (int)flight.size() < max_inflight && !rc) {
            const int k = one_launch_per_image ? 1 : std::min(arrived - next, (int)max_batch);
            if (one_launch_per_image) {
                rc = ecc_compute_async(js[next].image, &js[next].dims, (ecc_dtype)js[next].dtype, js[next].chi,
                                       nullptr, b->stream);
            } else {
                rc = ecc_batch_run(b, k, js.data() + next, nullptr);
            }
            if (rc) break;
            e = hipMemcpyAsync(chi_pin + off[next], chi_dev + off[next], (size_t)(off[next + k] - off[next]) * 8,
                               hipMemcpyDeviceToHost, b->stream);
            hipEvent_t ev = nullptr;
            if (e == hipSuccess) {
                if (!pool.empty()) {
                    ev = pool.back();
                    pool.pop_back();
                } else {
                    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(ev, b->stream);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_serve_simulate: launch");
                break;
            }
            flight.push_back({ev, next, next + k});
            next += k;
        }
        while (!flight.empty() && !rc) {
            e = hipEventQuery(flight.front().ev);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_serve_simulate: completion");
                break;
            }
            const double tc = now();
            for (int i = flight.front().first; i < flight.front().last; ++i) latency_s[i] = tc - arrival_s[i];
            done += flight.front().last - flight.front().first;
            pool.push_back(flight.front().ev);
            flight.pop_front();
        }
    }
    (void)hipStreamSynchronize(b->stream);
    for (auto &f : flight) (void)hipEventDestroy(f.ev);
    for (auto ev : pool) (void)hipEventDestroy(ev);
    if (!rc) memcpy(chi_host, chi_pin, (size_t)off[n] * 8);
    (void)hipHostFree(chi_pin);
    (void)hipFree(chi_dev);
    if (prev != b->device) (void)hipSetDevice(prev);
    return rc;
}

}  // extern "C"
