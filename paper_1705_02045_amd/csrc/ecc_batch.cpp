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
#include <cstdlib>
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
    // per slot, the graph of one run: table copy, persistent tile kernel,
    // batched merge (captured once for the slot's buffers; each run only
    // sets the copy's size)
    bool use_graph = true;
    hipStream_t capture = nullptr;
    hipGraph_t graph[kSlots] = {};
    hipGraphExec_t exec[kSlots] = {};
    hipGraphNode_t copy_node[kSlots] = {};
    int tile_grid = 0, colsum_grid = 0, scan_grid = 0;
    // batch tile depth (ecc_batch_autotune)
    int min_planes = 64, split = 4;
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
// tiles of max(min_planes, planes / split) planes (or the whole image), so
// that small images take one workgroup and large ones a few hundred.  The
// defaults (64, 4) hold until ecc_batch_autotune picks others.
constexpr int kBatchMinPlanes = 64, kBatchSplit = 4;

IntTiling batch_tiling(const IntView &v, int min_planes = kBatchMinPlanes, int split = kBatchSplit) {
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
    int64_t zc = std::max<int64_t>(min_planes, (v.n0 + split - 1) / split);
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
    int64_t voxels;
};

void drop_graph(ecc_batch *b, int s) {
    if (b->exec[s]) (void)hipGraphExecDestroy(b->exec[s]);
    if (b->graph[s]) (void)hipGraphDestroy(b->graph[s]);
    b->exec[s] = nullptr;
    b->graph[s] = nullptr;
    b->copy_node[s] = nullptr;
}

// Captures slot s's run: the copy of the whole table capacity (its size is
// set per run), the persistent tile kernel, the batched merge.
int build_graph(ecc_batch *b, int s) {
    drop_graph(b, s);
    hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "ecc_batch: begin capture");
    int rc = ECC_OK;
    e = hipMemcpyAsync(b->dev[s], b->host[s], b->cap[s], hipMemcpyHostToDevice, b->capture);
    if (e != hipSuccess) rc = hip_fail(e, "ecc_batch: captured copy");
    if (!rc) rc = launch_int_persistent(b->dev[s], b->tile_grid, b->capture);
    if (!rc) rc = launch_batch_merge(b->dev[s], b->colsum_grid, b->scan_grid, b->capture);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture, &g);
    if (!rc && e != hipSuccess) rc = hip_fail(e, "ecc_batch: end capture");
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    b->graph[s] = g;
    size_t n = 0;
    e = hipGraphGetNodes(g, nullptr, &n);
    std::vector<hipGraphNode_t> nodes(n);
    if (e == hipSuccess) e = hipGraphGetNodes(g, nodes.data(), &n);
    for (size_t i = 0; e == hipSuccess && i < n; ++i) {
        hipGraphNodeType t;
        e = hipGraphNodeGetType(nodes[i], &t);
        if (e == hipSuccess && t == hipGraphNodeTypeMemcpy) b->copy_node[s] = nodes[i];
    }
    if (e == hipSuccess && !b->copy_node[s]) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[s], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b, s);
        return hip_fail(e, "ecc_batch: graph");
    }
    return ECC_OK;
}

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
    const int cus = device_cu_count();
    b->tile_grid = 2 * cus;    // two 1024-thread workgroups per CU (64 KiB histograms)
    b->colsum_grid = 4 * cus;
    b->scan_grid = cus;
    const char *g = getenv("ECC_BATCH_GRAPH");
    b->use_graph = !(g && g[0] == '0');
    for (int i = 0; e == hipSuccess && i < ecc_batch::kSlots; ++i)
        e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    if (e == hipSuccess && b->use_graph) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "ecc_batch_create");
        for (int i = 0; i < ecc_batch::kSlots; ++i)
            if (b->done[i]) (void)hipEventDestroy(b->done[i]);
        if (b->capture) (void)hipStreamDestroy(b->capture);
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
        drop_graph(b, i);
        if (b->host[i]) (void)hipHostFree(b->host[i]);
        if (b->dev[i]) (void)hipFree(b->dev[i]);
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
    }
    if (b->capture) (void)hipStreamDestroy(b->capture);
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
    int64_t rows8 = 0, rows14 = 0, ntiles = 0, nitems = 0, vcec_words = 0;
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
        P.tl = batch_tiling(P.view, b->min_planes, b->split);
        P.group = (J.dtype == ECC_U14 ? 2 : 0) + (P.view.nin == 2 ? 1 : 0);
        P.m = (int)threshold_count(J.dtype);
        P.voxels = total;
        (P.m == 256 ? rows8 : rows14) += P.tl.grid;
        ntiles += P.tl.grid;
        nitems += (P.m + 1023) / 1024;
        vcec_words += P.m;
    }
    if (ntiles > INT32_MAX) {
        set_error("ecc_batch_run: too many tiles in one batch");
        return ECC_E_UNSUPPORTED;
    }
    // tiles of the largest images first, so the persistent workgroups end
    // on small tiles
    std::vector<int> order(n_jobs);
    for (int j = 0; j < n_jobs; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return prep[a].voxels > prep[c].voxels; });
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != b->device) ECC_HIP(hipSetDevice(b->device));
    int rc = ECC_OK;
    do {
        // device scratch
        if ((rc = grow(b, (void **)&b->partial8, &b->partial8_bytes, (size_t)rows8 * 256 * 4))) break;
        if ((rc = grow(b, (void **)&b->partial14, &b->partial14_bytes, (size_t)rows14 * 16384 * 4))) break;
        if ((rc = grow(b, (void **)&b->vcec, &b->vcec_bytes, (size_t)vcec_words * 8))) break;
        if (b->status_bytes < (size_t)n_jobs * 4 || !b->status) {
            if ((rc = grow(b, (void **)&b->status, &b->status_bytes, (size_t)n_jobs * 4))) break;
            if ((rc = launch_zero(b->status, b->status_bytes, b->stream))) break;
        }
        // table: header, KParams[n], tile_begin[n+1], kind[n], MergeJob[n], item_begin[n+1]
        const size_t kp = kparams_bytes();
        BatchHeader hd{};
        size_t total = align_up(sizeof(BatchHeader), 16);
        hd.off_kparams = (uint32_t)total;
        total = align_up(total + (size_t)n_jobs * kp, 16);
        hd.off_tile_begin = (uint32_t)total;
        total = align_up(total + (size_t)(n_jobs + 1) * 4, 16);
        hd.off_kind = (uint32_t)total;
        total = align_up(total + (size_t)n_jobs * 4, 16);
        hd.off_merge = (uint32_t)total;
        total = align_up(total + (size_t)n_jobs * sizeof(MergeJob), 16);
        hd.off_item_begin = (uint32_t)total;
        total = align_up(total + (size_t)(n_jobs + 1) * 4, 256);
        if (total > UINT32_MAX) {
            set_error("ecc_batch_run: batch table too large");
            rc = ECC_E_UNSUPPORTED;
            break;
        }
        hd.njobs = n_jobs;
        hd.ntiles = (int32_t)ntiles;
        hd.nitems = (int32_t)nitems;
        hd.next_tile = 0;
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
            drop_graph(b, s);
            if (b->host[s]) (void)hipHostFree(b->host[s]);
            if (b->dev[s]) (void)hipFree(b->dev[s]);
            b->host[s] = b->dev[s] = nullptr;
            b->cap[s] = 0;
            const size_t want = std::max(total, (size_t)64 << 10);  // room for later, larger batches
            hipError_t e = hipHostMalloc(&b->host[s], want, hipHostMallocDefault);
            if (e == hipSuccess) e = hipMalloc(&b->dev[s], want);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_batch_run: table allocation");
                break;
            }
            b->cap[s] = want;
        }
        uint8_t *h = (uint8_t *)b->host[s];
        uint8_t *d = (uint8_t *)b->dev[s];
        memcpy(h, &hd, sizeof hd);
        int32_t *tile_begin = (int32_t *)(h + hd.off_tile_begin);
        int32_t *kind = (int32_t *)(h + hd.off_kind);
        MergeJob *mj = (MergeJob *)(h + hd.off_merge);
        int32_t *item_begin = (int32_t *)(h + hd.off_item_begin);
        tile_begin[0] = 0;
        item_begin[0] = 0;
        int64_t row8 = 0, row14 = 0, vw = 0;
        for (int p = 0; p < n_jobs; ++p) {
            const int j = order[p];
            const Prepared &P = prep[j];
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
            fill_kparams(h + hd.off_kparams + (size_t)p * kp, job, P.tl, part, b->status + j);
            tile_begin[p + 1] = tile_begin[p] + P.tl.grid;
            kind[p] = P.group;
            mj[p].partial = part;
            mj[p].rows = P.tl.grid;
            mj[p].m = P.m;
            mj[p].vcec = b->vcec + vw;
            mj[p].chi = jobs[j].chi;
            mj[p].status = b->status + j;
            mj[p].status_out = status_dev ? status_dev + j : nullptr;
            item_begin[p + 1] = item_begin[p] + (P.m + 1023) / 1024;
            vw += P.m;
        }
        if (b->use_graph) {
            if (!b->exec[s] && (rc = build_graph(b, s))) break;
            hipError_t e = hipGraphExecMemcpyNodeSetParams1D(b->exec[s], b->copy_node[s], d, h, total,
                                                             hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipGraphLaunch(b->exec[s], b->stream);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_batch_run: graph launch");
                break;
            }
        } else {
            hipError_t e = hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, b->stream);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ecc_batch_run: table copy");
                break;
            }
            if ((rc = launch_int_persistent(d, b->tile_grid, b->stream))) break;
            if ((rc = launch_batch_merge(d, b->colsum_grid, b->scan_grid, b->stream))) break;
        }
        hipError_t e = hipEventRecord(b->done[s], b->stream);
        if (e != hipSuccess) {
            rc = hip_fail(e, "ecc_batch_run: event");
            break;
        }
        b->used[s] = true;
    } while (0);
    if (prev != b->device) (void)hipSetDevice(prev);
    return rc;
}

int ecc_batch_autotune(ecc_batch *b, int32_t n_jobs, const ecc_job *jobs, int32_t *min_planes, int32_t *split,
                       float *ms) {
    g_err_clear();
    if (!b || n_jobs < 1 || !jobs) {
        set_error("ecc_batch_autotune: bad argument");
        return ECC_E_ARG;
    }
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != b->device) ECC_HIP(hipSetDevice(b->device));
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    int rc = e == hipSuccess ? ECC_OK : hip_fail(e, "ecc_batch_autotune: events");
    const int mp_c[4] = {16, 32, 64, 128}, sp_c[3] = {2, 4, 8};
    int best_mp = b->min_planes, best_sp = b->split;
    float best = 1e30f;
    for (int i = 0; i < 4 && !rc; ++i)
        for (int k = 0; k < 3 && !rc; ++k) {
            b->min_planes = mp_c[i];
            b->split = sp_c[k];
            float tmin = 1e30f;
            for (int rep = 0; rep < 4 && !rc; ++rep) {  // one warm-up, three timed
                if ((e = hipEventRecord(ev[0], b->stream)) != hipSuccess) rc = hip_fail(e, "ecc_batch_autotune");
                if (!rc) rc = ecc_batch_run(b, n_jobs, jobs, nullptr);
                if (!rc && (e = hipEventRecord(ev[1], b->stream)) != hipSuccess) rc = hip_fail(e, "ecc_batch_autotune");
                if (!rc && (e = hipEventSynchronize(ev[1])) != hipSuccess) rc = hip_fail(e, "ecc_batch_autotune");
                float t = 0.0f;
                if (!rc && (e = hipEventElapsedTime(&t, ev[0], ev[1])) != hipSuccess)
                    rc = hip_fail(e, "ecc_batch_autotune");
                if (!rc && rep > 0 && t < tmin) tmin = t;
            }
            if (!rc && tmin < best) {
                best = tmin;
                best_mp = mp_c[i];
                best_sp = sp_c[k];
            }
        }
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    b->min_planes = best_mp;
    b->split = best_sp;
    if (!rc) {
        if (min_planes) *min_planes = best_mp;
        if (split) *split = best_sp;
        if (ms) *ms = best;
    }
    if (prev != b->device) (void)hipSetDevice(prev);
    return rc;
}

int ecc_job_footprint(const ecc_job *job, int64_t *bytes) {
    g_err_clear();
    if (!job || !bytes) {
        set_error("ecc_job_footprint: NULL argument");
        return ECC_E_ARG;
    }
    int64_t total = 0;
    int rc = check_dims(&job->dims, &total);
    if (rc) return rc;
    if (job->dtype != ECC_U8 && job->dtype != ECC_U14) {
        set_error("ecc_job_footprint: U8 or U14 images");
        return (job->dtype == ECC_U16 || job->dtype == ECC_F32) ? ECC_E_UNSUPPORTED : ECC_E_ARG;
    }
    IntView v{};
    int unsup = 0;
    if (!normalize_int_view(&job->dims, &v, &unsup)) {
        set_error("ecc_job_footprint: shape not supported");
        return ECC_E_UNSUPPORTED;
    }
    const int64_t m = threshold_count(job->dtype);
    *bytes = total * (int64_t)elem_bytes(job->dtype) + (int64_t)batch_tiling(v).grid * m * 4 + 2 * m * 8;
    return ECC_OK;
}

int ecc_serve_simulate(ecc_batch *b, int32_t n, const ecc_job *jobs, const double *arrival_s, int32_t max_batch,
                       int64_t max_batch_bytes, int32_t one_launch_per_image, int64_t *chi_host, double *latency_s,
                       int32_t *batch_id) {
    g_err_clear();
    if (!b || n < 1 || !jobs || !arrival_s || !chi_host || !latency_s || max_batch < 1 || max_batch_bytes < 0) {
        set_error("ecc_serve_simulate: bad argument");
        return ECC_E_ARG;
    }
    std::vector<int64_t> foot(n, 0);
    for (int i = 0; i < n && max_batch_bytes > 0; ++i) {
        const int rc = ecc_job_footprint(&jobs[i], &foot[i]);
        if (rc) return rc;
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
    // The curves go to the host on a second stream (default priority), each
    // copy ordered after its launch by an event, so the copy of one batch
    // overlaps the kernels of the next.
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipHostFree(chi_pin);
        (void)hipFree(chi_dev);
        if (prev != b->device) (void)hipSetDevice(prev);
        return hip_fail(e, "ecc_serve_simulate: copy stream");
    }
    struct Flight {
        hipEvent_t ev, kev;  // copy done, kernels done
        int first, last;
    };
    std::deque<Flight> flight;
    std::vector<hipEvent_t> pool;
    int rc = ECC_OK;
    const int max_inflight = one_launch_per_image ? (1 << 30) : 3;
    auto take_event = [&](hipEvent_t *ev) -> hipError_t {
        if (!pool.empty()) {
            *ev = pool.back();
            pool.pop_back();
            return hipSuccess;
        }
        return hipEventCreateWithFlags(ev, hipEventDisableTiming);
    };
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    int next = 0, arrived = 0, done = 0, batches = 0;
    while (done < n && !rc) {
        const double t = now();
        while (arrived < n && arrival_s[arrived] <= t) ++arrived;
        while (next < arrived && (int)flight.size() < max_inflight && !rc) {
            // admission: in arrival order, up to max_batch requests and
            // max_batch_bytes of footprint (the first request always fits)
            int k = 1;
            if (!one_launch_per_image) {
                int64_t bytes = foot[next];
                while (next + k < arrived && k < max_batch &&
                       (max_batch_bytes == 0 || bytes + foot[next + k] <= max_batch_bytes))
                    bytes += foot[next + k++];
            }
            if (batch_id)
                for (int i = next; i < next + k; ++i) batch_id[i] = batches;
            ++batches;
            if (one_launch_per_image) {
                rc = ecc_compute_async(js[next].image, &js[next].dims, (ecc_dtype)js[next].dtype, js[next].chi,
                                       nullptr, b->stream);
            } else {
                rc = ecc_batch_run(b, k, js.data() + next, nullptr);
            }
            if (rc) break;
            hipEvent_t ev = nullptr, kev = nullptr;
            e = take_event(&kev);
            if (e == hipSuccess) e = take_event(&ev);
            if (e == hipSuccess) e = hipEventRecord(kev, b->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs, kev, 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(chi_pin + off[next], chi_dev + off[next],
                                   (size_t)(off[next + k] - off[next]) * 8, hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess) e = hipEventRecord(ev, cs);
            if (e != hipSuccess) {
                if (kev) pool.push_back(kev);
                if (ev) pool.push_back(ev);
                rc = hip_fail(e, "ecc_serve_simulate: launch");
                break;
            }
            flight.push_back({ev, kev, next, next + k});
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
            pool.push_back(flight.front().kev);
            flight.pop_front();
        }
    }
    (void)hipStreamSynchronize(b->stream);
    (void)hipStreamSynchronize(cs);
    for (auto &f : flight) {
        (void)hipEventDestroy(f.ev);
        (void)hipEventDestroy(f.kev);
    }
    for (auto ev : pool) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cs);
    if (!rc) memcpy(chi_host, chi_pin, (size_t)off[n] * 8);
    (void)hipHostFree(chi_pin);
    (void)hipFree(chi_dev);
    if (prev != b->device) (void)hipSetDevice(prev);
    return rc;
}

}  // extern "C"
