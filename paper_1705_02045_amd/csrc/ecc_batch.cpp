// Batched and served computation of many independent images (integer dtypes).
//
// The curves of different images are independent (Sec. 3, "Parallel
// Computations": VCECs of disjoint parts merge by addition, and unrelated
// images simply do not merge), so one launch can hold the tiles of many
// images: a host-built descriptor table gives every image its kernel
// parameters and its range of workgroups, and a batched merge sums and scans
// each image's rows into its own curve.
//
// ecc_serve replays a stream of requests with given arrival times against
// the device, either with continuous batching (everything that has arrived
// when the device can take more work goes into the next batch) or one launch
// per image, and reports each request's latency from arrival to its curve
// being in host memory.  Requests may start in device memory or in pinned
// host memory; host-origin images are copied into an arena of device memory
// as they are admitted (pinned images by one gather kernel per 32 requests,
// which reads them through their device-mapped addresses: many small DMA
// copies, one per request, reach about 48 GB/s over PCIe where the kernel
// reaches 56), and requests above a size are pushed chunk by chunk
// through the streaming path (Sec. 3, "Streaming") while batches of the
// others keep running.

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
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

// ------------------------------------------------------------------ serving
// One request of a serving run, as the loop sees it.
struct Req {
    int m = 0;
    int64_t bytes = 0;         // image bytes
    int64_t foot = 0;          // ecc_job_footprint (batched requests)
    bool streamed = false;     // pushed chunk by chunk through the streaming path
    int64_t plane_bytes = 0;   // streamed: bytes of one axis-0 plane
    int64_t chunk_planes = 0;  // streamed: planes per pushed chunk
};

// Host-origin images to the arena in one launch: block b copies chunk
// b - first[r] (kGatherChunk bytes, the last one shorter) of request r,
// first[r] <= b < first[r + 1].  Sources are device-mapped addresses of
// pinned host memory; sources and destinations are 16-byte aligned.
constexpr int kGatherMax = 32;
constexpr int64_t kGatherChunk = 65536;
struct GatherArgs {
    const uint8_t *src[kGatherMax];
    uint8_t *dst[kGatherMax];
    int64_t bytes[kGatherMax];
    uint32_t first[kGatherMax + 1];
    int n;
};

__global__ void __launch_bounds__(256) gather_images_kernel(GatherArgs a) {
    const uint32_t b = blockIdx.x;
    int r = 0;
    while (r + 1 < a.n && a.first[r + 1] <= b) ++r;
    const int64_t off = (int64_t)(b - a.first[r]) * kGatherChunk;
    const int64_t len = std::min(kGatherChunk, a.bytes[r] - off);
    const uint8_t *src = a.src[r] + off;
    uint8_t *dst = a.dst[r] + off;
    const int64_t n16 = len / 16;
    for (int64_t i = threadIdx.x; i < n16; i += 256)
        reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
    for (int64_t i = n16 * 16 + threadIdx.x; i < len; i += 256) dst[i] = src[i];
}

// First-fit allocator over one device buffer in 256-byte granules: the
// images (and streamed chunks) of host-origin requests while they are in
// flight.  Admission takes blocks from it and completion returns them, so
// the device memory held by requests never exceeds the arena.
class Arena {
  public:
    void reset(uint8_t *base, int64_t cap) {
        base_ = base;
        free_.clear();
        if (cap > 0) free_[0] = cap;
    }
    int64_t alloc(int64_t bytes) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, size = it->second;
            free_.erase(it);
            if (size > bytes) free_[off + bytes] = size - bytes;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = round(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint8_t *at(int64_t off) const { return base_ + off; }

  private:
    static int64_t round(int64_t b) { return (b + 255) & ~(int64_t)255; }
    uint8_t *base_ = nullptr;
    std::map<int64_t, int64_t> free_;  // offset -> bytes
};

class Serve {
  public:
    Serve(ecc_batch *b, int n) : b_(b), n_(n) {}

    int setup(const std::vector<Req> &req, int64_t arena_bytes) {
        int64_t words = 0;
        for (const Req &R : req) words += R.m;
        slot_req_.assign(n_, -1);
        slot_off_.assign(n_ + 1, 0);
        js_.assign(n_, ecc_job{});
        hipError_t e = dev_malloc((void **)&chi_dev_, (size_t)words * 8);
        if (e == hipSuccess) e = host_malloc((void **)&chi_pin_, (size_t)words * 8, hipHostMallocDefault);
        if (e == hipSuccess) e = dev_malloc((void **)&status_dev_, (size_t)n_ * 4);
        if (e == hipSuccess && arena_bytes > 0) e = dev_malloc((void **)&arena_buf_, (size_t)arena_bytes);
        for (hipStream_t *s : {&h2d_, &d2h_, &os_})
            if (e == hipSuccess) e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "ecc_serve: set-up");
        arena_.reset((uint8_t *)arena_buf_, arena_bytes);
        return launch_zero(status_dev_, (size_t)n_ * 4, b_->stream);
    }

    int run(const ecc_job *jobs, const std::vector<Req> &req, const double *arrival, const ecc_serve_config &c,
            bool single, bool host_origin, double *latency, int32_t *batch_id) {
        jobs_ = jobs;
        req_ = &req;
        host_origin_ = host_origin;
        latency_ = latency;
        batch_id_ = batch_id;
        arrival_ = arrival;
        const int max_inflight = c.max_inflight > 0 ? c.max_inflight : (single ? (1 << 30) : 3);
        // host-origin images that the gather kernel may read: pinned host
        // memory with a device-mapped address, 16-byte aligned (the others,
        // pageable or device memory, are copied one by one)
        mapped_.assign(n_, nullptr);
        if (host_origin)
            for (int i = 0; i < n_; ++i) {
                void *d = nullptr;
                if (hipHostGetDevicePointer(&d, const_cast<void *>(jobs[i].image), 0) != hipSuccess) {
                    (void)hipGetLastError();
                    continue;
                }
                if (((uintptr_t)d & 15u) == 0u) mapped_[i] = (const uint8_t *)d;
            }
        ECC_HIP(hipStreamSynchronize(b_->stream));  // the status clear
        t0_ = std::chrono::steady_clock::now();
        int arrived = 0, rc = ECC_OK;
        while (done_ < n_ && !rc) {
            const double t = now();
            for (; arrived < n_ && arrival[arrived] <= t; ++arrived)
                (req[arrived].streamed ? sq_ : bq_).push_back(arrived);
            rc = pump_stream();
            while (!rc && !bq_.empty() && (int)flights_.size() < max_inflight) {
                bool formed = false;
                rc = dispatch(c, single, &formed);
                if (!formed) break;
            }
            if (!rc) rc = poll_flights();
        }
        return rc;
    }

    // Status and curves to the caller, in request order.
    int collect(const std::vector<Req> &req, int64_t *chi_host, int32_t *status) {
        std::vector<uint32_t> st(n_, 0);
        ECC_HIP(hipMemcpy(st.data(), status_dev_, (size_t)n_ * 4, hipMemcpyDeviceToHost));
        std::vector<int64_t> roff(n_ + 1, 0);
        for (int i = 0; i < n_; ++i) roff[i + 1] = roff[i] + req[i].m;
        int rc = ECC_OK;
        for (int s = 0; s < nslots_; ++s) {
            const int r = slot_req_[s];
            const int m = req[r].m;
            int code = ECC_OK;
            if (st[s] & kStatusRange) code = ECC_E_RANGE;
            else if (st[s] != 0) code = ECC_E_HIP;
            if (status) status[r] = code;
            if (code == ECC_OK) {
                memcpy(chi_host + roff[r], chi_pin_ + slot_off_[s], (size_t)m * 8);
            } else {
                memset(chi_host + roff[r], 0, (size_t)m * 8);
                if (!rc) {
                    rc = code;
                    if (code == ECC_E_RANGE) set_error("ecc_serve: request %d holds a 14-bit value >= 16384", r);
                    else set_error("ecc_serve: request %d: device status 0x%08x", r, st[s]);
                }
            }
        }
        return rc;
    }

    void teardown() {
        (void)hipStreamSynchronize(b_->stream);
        for (hipStream_t s : {os_, h2d_, d2h_})
            if (s) (void)hipStreamSynchronize(s);
        if (cur_.st) ecc_stream_abort(cur_.st);
        for (auto &f : flights_) {
            pool_.push_back(f.kev);
            pool_.push_back(f.cev);
        }
        for (auto &ch : cur_.chunks) pool_.push_back(ch.ev);
        if (cur_.cev) pool_.push_back(cur_.cev);
        for (hipEvent_t ev : pool_)
            if (ev) (void)hipEventDestroy(ev);
        for (hipStream_t s : {h2d_, d2h_, os_})
            if (s) (void)hipStreamDestroy(s);
        if (arena_buf_) (void)hipFree(arena_buf_);
        if (status_dev_) (void)hipFree(status_dev_);
        if (chi_pin_) (void)hipHostFree(chi_pin_);
        if (chi_dev_) (void)hipFree(chi_dev_);
    }

  private:
    struct Flight {  // one batch, or one launch of a single image
        hipEvent_t kev = nullptr;  // its kernels are done: its arena blocks return
        hipEvent_t cev = nullptr;  // its curves are in host memory
        int s0 = 0, s1 = 0;        // its dispatch slots
        std::vector<std::pair<int64_t, int64_t>> held;
        bool released = false;
    };
    struct Chunk {
        hipEvent_t ev;  // the kernels reading it are done
        int64_t off, bytes;
    };
    struct Streamed {  // the request being pushed chunk by chunk
        int r = -1, slot = -1;
        ecc_stream *st = nullptr;
        int64_t pushed = 0;
        std::deque<Chunk> chunks;
        bool finishing = false;
        hipEvent_t cev = nullptr;
    };

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count(); }

    int event(hipEvent_t *ev) {
        if (!pool_.empty()) {
            *ev = pool_.back();
            pool_.pop_back();
            return ECC_OK;
        }
        ECC_HIP(hipEventCreateWithFlags(ev, hipEventDisableTiming));
        return ECC_OK;
    }

    // Curve slot s for request r (dispatch order, so a batch's curves are contiguous).
    int new_slot(int r) {
        const int s = nslots_++;
        slot_req_[s] = r;
        slot_off_[s + 1] = slot_off_[s] + (*req_)[r].m;
        return s;
    }

    // Copy of the curves of slots [s0, s1) to pinned host memory after the
    // work recorded by kev, on the copy-out stream; records cev.
    int copy_out(hipEvent_t kev, int s0, int s1, hipEvent_t *cev) {
        int rc = event(cev);
        if (rc) return rc;
        ECC_HIP(hipStreamWaitEvent(d2h_, kev, 0));
        ECC_HIP(hipMemcpyAsync(chi_pin_ + slot_off_[s0], chi_dev_ + slot_off_[s0],
                               (size_t)(slot_off_[s1] - slot_off_[s0]) * 8, hipMemcpyDeviceToHost, d2h_));
        ECC_HIP(hipEventRecord(*cev, d2h_));
        return ECC_OK;
    }

    // The next batch from the queue, in arrival order: at most max_batch
    // requests (one in the per-image mode) and max_batch_bytes of footprint
    // (the first request always counts), each host-origin image in an arena
    // block, copied in on the copy-in stream.
    int dispatch(const ecc_serve_config &c, bool single, bool *formed) {
        const std::vector<Req> &req = *req_;
        const int cap = single ? 1 : c.max_batch;
        int k = 0;
        int64_t foot = 0;
        Flight f;
        while (k < cap && k < (int)bq_.size()) {
            const int r = bq_[k];
            if (k > 0 && c.max_batch_bytes > 0 && foot + req[r].foot > c.max_batch_bytes) break;
            if (host_origin_) {
                const int64_t off = arena_.alloc(req[r].bytes);
                if (off < 0) break;
                f.held.emplace_back(off, req[r].bytes);
            }
            foot += req[r].foot;
            ++k;
        }
        *formed = k > 0;
        if (!k) return ECC_OK;
        f.s0 = nslots_;
        GatherArgs ga{};
        int rc = ECC_OK;
        for (int i = 0; i < k; ++i) {
            const int r = bq_.front();
            bq_.pop_front();
            const int s = new_slot(r);
            js_[s] = jobs_[r];
            js_[s].chi = chi_dev_ + slot_off_[s];
            if (batch_id_) batch_id_[r] = groups_;
            if (host_origin_) {
                js_[s].image = arena_.at(f.held[i].first);
                if (mapped_[r] && req[r].bytes > 0) {
                    ga.src[ga.n] = mapped_[r];
                    ga.dst[ga.n] = (uint8_t *)js_[s].image;
                    ga.bytes[ga.n] = req[r].bytes;
                    ga.first[ga.n + 1] = ga.first[ga.n] + (uint32_t)((req[r].bytes + kGatherChunk - 1) / kGatherChunk);
                    if (++ga.n == kGatherMax && (rc = gather(&ga))) return rc;
                } else {
                    ECC_HIP(hipMemcpyAsync((void *)js_[s].image, jobs_[r].image, (size_t)req[r].bytes,
                                           hipMemcpyHostToDevice, h2d_));
                }
            }
        }
        if (ga.n > 0 && (rc = gather(&ga))) return rc;
        f.s1 = nslots_;
        ++groups_;
        if (host_origin_) {
            hipEvent_t in = nullptr;
            if ((rc = event(&in))) return rc;
            ECC_HIP(hipEventRecord(in, h2d_));
            ECC_HIP(hipStreamWaitEvent(b_->stream, in, 0));
            pool_.push_back(in);  // reusable: the wait has taken its record
        }
        if (single) {
            const ecc_job &J = js_[f.s0];
            rc = ecc_compute_async(J.image, &J.dims, (ecc_dtype)J.dtype, J.chi, status_dev_ + f.s0, b_->stream);
        } else {
            rc = ecc_batch_run(b_, k, js_.data() + f.s0, status_dev_ + f.s0);
        }
        if (rc) return rc;
        if ((rc = event(&f.kev))) return rc;
        ECC_HIP(hipEventRecord(f.kev, b_->stream));
        if ((rc = copy_out(f.kev, f.s0, f.s1, &f.cev))) return rc;
        flights_.push_back(std::move(f));
        return ECC_OK;
    }

    // One gather launch on the copy-in stream for the requests in *a; *a is
    // emptied.
    int gather(GatherArgs *a) {
        const uint32_t blocks = a->first[a->n];
        if (blocks > 0) {
            hipLaunchKernelGGL(gather_images_kernel, dim3(blocks), dim3(256), 0, h2d_, *a);
            ECC_HIP(hipGetLastError());
        }
        *a = GatherArgs{};
        return ECC_OK;
    }

    // Oversized requests, one at a time: chunks of whole planes pushed through
    // the streaming path on a stream of their own (two chunks in flight, each
    // in an arena block for host-origin requests); the partial changes vector
    // stays on the device between chunks; the curve is scanned and copied out
    // after the last chunk.
    int pump_stream() {
        int rc = ECC_OK;
        if (!cur_.st && !sq_.empty()) {
            cur_ = Streamed{};
            cur_.r = sq_.front();
            sq_.pop_front();
            cur_.slot = new_slot(cur_.r);
            if (batch_id_) batch_id_[cur_.r] = groups_;
            ++groups_;
            const ecc_job &J = jobs_[cur_.r];
            if ((rc = ecc_stream_begin(&J.dims, (ecc_dtype)J.dtype, os_, &cur_.st))) return rc;
        }
        if (!cur_.st) return ECC_OK;
        const Req &R = (*req_)[cur_.r];
        const ecc_job &J = jobs_[cur_.r];
        const int64_t planes = J.dims.n[0];
        while (!cur_.chunks.empty()) {
            const hipError_t e = hipEventQuery(cur_.chunks.front().ev);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return hip_fail(e, "ecc_serve: chunk");
            if (cur_.chunks.front().off >= 0) arena_.release(cur_.chunks.front().off, cur_.chunks.front().bytes);
            pool_.push_back(cur_.chunks.front().ev);
            cur_.chunks.pop_front();
        }
        while (cur_.pushed < planes && cur_.chunks.size() < 2) {
            const int64_t np = std::min(R.chunk_planes, planes - cur_.pushed);
            const int64_t bytes = np * R.plane_bytes;
            const uint8_t *src = (const uint8_t *)J.image + cur_.pushed * R.plane_bytes;
            const uint8_t *dst = src;
            int64_t off = -1;
            if (host_origin_) {
                off = arena_.alloc(bytes);
                if (off < 0) break;
                dst = arena_.at(off);
                hipEvent_t in = nullptr;
                if ((rc = event(&in))) return rc;
                ECC_HIP(hipMemcpyAsync((void *)dst, src, (size_t)bytes, hipMemcpyHostToDevice, h2d_));
                ECC_HIP(hipEventRecord(in, h2d_));
                ECC_HIP(hipStreamWaitEvent(os_, in, 0));
                pool_.push_back(in);
            }
            if ((rc = ecc_stream_push_chunk(cur_.st, dst, np))) return rc;
            Chunk ch{nullptr, off, bytes};
            if ((rc = event(&ch.ev))) return rc;
            ECC_HIP(hipEventRecord(ch.ev, os_));
            cur_.chunks.push_back(ch);
            cur_.pushed += np;
        }
        if (cur_.pushed == planes && !cur_.finishing) {
            if ((rc = stream_finish_async(cur_.st, chi_dev_ + slot_off_[cur_.slot], status_dev_ + cur_.slot)))
                return rc;
            hipEvent_t k = nullptr;
            if ((rc = event(&k))) return rc;
            ECC_HIP(hipEventRecord(k, os_));
            if ((rc = copy_out(k, cur_.slot, cur_.slot + 1, &cur_.cev))) return rc;
            pool_.push_back(k);
            cur_.finishing = true;
        }
        if (cur_.finishing) {
            const hipError_t e = hipEventQuery(cur_.cev);
            if (e == hipErrorNotReady) return ECC_OK;
            if (e != hipSuccess) return hip_fail(e, "ecc_serve: streamed request");
            latency_[cur_.r] = now() - arrival_[cur_.r];
            ++done_;
            for (auto &ch : cur_.chunks) {  // done: recorded before the scan
                if (ch.off >= 0) arena_.release(ch.off, ch.bytes);
                pool_.push_back(ch.ev);
            }
            pool_.push_back(cur_.cev);
            ecc_stream_abort(cur_.st);
            cur_ = Streamed{};
        }
        return ECC_OK;
    }

    int poll_flights() {
        for (auto &f : flights_) {  // arena blocks return as soon as a batch's kernels are done
            if (f.released) continue;
            const hipError_t e = hipEventQuery(f.kev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return hip_fail(e, "ecc_serve: kernels");
            for (auto &h : f.held) arena_.release(h.first, h.second);
            f.released = true;
        }
        while (!flights_.empty()) {
            Flight &f = flights_.front();
            const hipError_t e = hipEventQuery(f.cev);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return hip_fail(e, "ecc_serve: completion");
            if (!f.released) {  // (the copy waited for the kernels)
                for (auto &h : f.held) arena_.release(h.first, h.second);
            }
            const double tc = now();
            for (int s = f.s0; s < f.s1; ++s) latency_[slot_req_[s]] = tc - arrival_[slot_req_[s]];
            done_ += f.s1 - f.s0;
            pool_.push_back(f.kev);
            pool_.push_back(f.cev);
            flights_.pop_front();
        }
        return ECC_OK;
    }

    ecc_batch *b_;
    int n_;
    const ecc_job *jobs_ = nullptr;
    std::vector<const uint8_t *> mapped_;  // per request: device-mapped image address, or null
    const std::vector<Req> *req_ = nullptr;
    const double *arrival_ = nullptr;
    double *latency_ = nullptr;
    int32_t *batch_id_ = nullptr;
    bool host_origin_ = false;
    std::chrono::steady_clock::time_point t0_;
    int64_t *chi_dev_ = nullptr, *chi_pin_ = nullptr;
    uint32_t *status_dev_ = nullptr;
    void *arena_buf_ = nullptr;
    Arena arena_;
    hipStream_t h2d_ = nullptr, d2h_ = nullptr, os_ = nullptr;
    std::vector<int> slot_req_;
    std::vector<int64_t> slot_off_;
    std::vector<ecc_job> js_;
    int nslots_ = 0, groups_ = 0, done_ = 0;
    std::deque<int> bq_, sq_;
    std::deque<Flight> flights_;
    Streamed cur_;
    std::vector<hipEvent_t> pool_;
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
    std::vector<int> wide;  // ECC_U16 jobs: windowed launches of their own, after the batch
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
        if (J.dtype != ECC_U8 && J.dtype != ECC_U14 && J.dtype != ECC_U16) {
            set_error("job %d: batches take U8, U14 or U16 images", j);
            return J.dtype == ECC_F32 ? ECC_E_UNSUPPORTED : ECC_E_ARG;
        }
        Prepared &P = prep[j];
        int unsup = 0;
        if (!normalize_int_view(&J.dims, &P.view, &unsup)) {
            set_error("job %d: shape not supported", j);
            return ECC_E_UNSUPPORTED;
        }
        if (J.dtype == ECC_U16) {
            wide.push_back(j);
            continue;
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
    std::vector<int> order;
    for (int j = 0; j < n_jobs; ++j)
        if (jobs[j].dtype != ECC_U16) order.push_back(j);
    const int nb = (int)order.size();  // jobs in the persistent launch
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return prep[a].voxels > prep[c].voxels; });
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != b->device) ECC_HIP(hipSetDevice(b->device));
    int rc = ECC_OK;
    do {
        if (nb == 0) break;
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
        total = align_up(total + (size_t)nb * kp, 16);
        hd.off_tile_begin = (uint32_t)total;
        total = align_up(total + (size_t)(nb + 1) * 4, 16);
        hd.off_kind = (uint32_t)total;
        total = align_up(total + (size_t)nb * 4, 16);
        hd.off_merge = (uint32_t)total;
        total = align_up(total + (size_t)nb * sizeof(MergeJob), 16);
        hd.off_item_begin = (uint32_t)total;
        total = align_up(total + (size_t)(nb + 1) * 4, 256);
        if (total > UINT32_MAX) {
            set_error("ecc_batch_run: batch table too large");
            rc = ECC_E_UNSUPPORTED;
            break;
        }
        hd.njobs = nb;
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
            hipError_t e = host_malloc((void **)&b->host[s], want, hipHostMallocDefault);
            if (e == hipSuccess) e = dev_malloc((void **)&b->dev[s], want);
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
        for (int p = 0; p < nb; ++p) {
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
    // 16-bit images: one launch per window of 16384 values each (the
    // persistent kernel's histograms hold 16384 bins), on the same stream
    for (size_t w = 0; !rc && w < wide.size(); ++w) {
        const int j = wide[w];
        rc = u16_curve_async(jobs[j].image, prep[j].view, jobs[j].chi, status_dev ? status_dev + j : nullptr,
                             b->stream);
    }
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
    if (job->dtype != ECC_U8 && job->dtype != ECC_U14 && job->dtype != ECC_U16) {
        set_error("ecc_job_footprint: U8, U14 or U16 images");
        return job->dtype == ECC_F32 ? ECC_E_UNSUPPORTED : ECC_E_ARG;
    }
    IntView v{};
    int unsup = 0;
    if (!normalize_int_view(&job->dims, &v, &unsup)) {
        set_error("ecc_job_footprint: shape not supported");
        return ECC_E_UNSUPPORTED;
    }
    const int64_t m = threshold_count(job->dtype), mrow = m < 16384 ? m : 16384;  // bins of a count row
    *bytes = total * (int64_t)elem_bytes(job->dtype) + (int64_t)batch_tiling(v).grid * mrow * 4 + 2 * m * 8;
    return ECC_OK;
}

int ecc_serve_simulate(ecc_batch *b, int32_t n, const ecc_job *jobs, const double *arrival_s, int32_t max_batch,
                       int64_t max_batch_bytes, int32_t one_launch_per_image, int64_t *chi_host, double *latency_s,
                       int32_t *batch_id) {
    ecc_serve_config c{};
    c.max_batch = max_batch;
    c.one_launch_per_image = one_launch_per_image;
    c.max_batch_bytes = max_batch_bytes;
    return ecc_serve(b, n, jobs, arrival_s, &c, chi_host, latency_s, batch_id, nullptr);
}

int ecc_serve(ecc_batch *b, int32_t n, const ecc_job *jobs, const double *arrival_s, const ecc_serve_config *cfg,
              int64_t *chi_host, double *latency_s, int32_t *batch_id, int32_t *status) {
    g_err_clear();
    if (!b || n < 1 || !jobs || !arrival_s || !cfg || !chi_host || !latency_s || cfg->max_batch < 1 ||
        cfg->max_batch_bytes < 0 || cfg->arena_bytes < 0 || cfg->stream_above_bytes < 0 || cfg->chunk_bytes < 0 ||
        cfg->max_inflight < 0) {
        set_error("ecc_serve: bad argument");
        return ECC_E_ARG;
    }
    for (int i = 1; i < n; ++i)
        if (arrival_s[i] < arrival_s[i - 1]) {
            set_error("ecc_serve: arrivals must be sorted");
            return ECC_E_ARG;
        }
    const bool host_origin = cfg->arena_bytes > 0;
    const bool single = cfg->one_launch_per_image != 0;
    const int64_t stream_above =
        cfg->stream_above_bytes > 0 ? cfg->stream_above_bytes : (host_origin ? cfg->arena_bytes / 4 : 0);
    if (host_origin && stream_above > cfg->arena_bytes / 2) {
        set_error("ecc_serve: stream_above_bytes must be at most half of arena_bytes");
        return ECC_E_ARG;
    }
    const int64_t chunk_target = cfg->chunk_bytes > 0 ? cfg->chunk_bytes : ((int64_t)64 << 20);
    std::vector<Req> req(n);
    for (int i = 0; i < n; ++i) {
        int64_t total = 0;
        int rc = check_dims(&jobs[i].dims, &total);
        if (rc) return rc;
        const int64_t m = threshold_count(jobs[i].dtype);
        if (!jobs[i].image || (jobs[i].dtype != ECC_U8 && jobs[i].dtype != ECC_U14 && jobs[i].dtype != ECC_U16)) {
            set_error("request %d: NULL image, or a dtype other than U8/U14/U16", i);
            return jobs[i].image ? ECC_E_UNSUPPORTED : ECC_E_ARG;
        }
        Req &R = req[i];
        R.m = (int)m;
        R.bytes = total * (int64_t)elem_bytes(jobs[i].dtype);
        R.streamed = stream_above > 0 && R.bytes > stream_above;
        if (!R.streamed && (rc = ecc_job_footprint(&jobs[i], &R.foot))) return rc;
        if (R.streamed) {
            const int64_t planes = jobs[i].dims.n[0];
            R.plane_bytes = R.bytes / planes;
            if (host_origin && R.plane_bytes > cfg->arena_bytes / 4) {
                set_error("request %d: one axis-0 plane (%lld bytes) exceeds a quarter of the arena", i,
                          (long long)R.plane_bytes);
                return ECC_E_UNSUPPORTED;
            }
            const int64_t cap = host_origin ? cfg->arena_bytes / 4 : chunk_target;
            R.chunk_planes = std::max<int64_t>(1, std::min(chunk_target, cap) / R.plane_bytes);
        }
    }
    int prev = -1;
    ECC_HIP(hipGetDevice(&prev));
    if (prev != b->device) ECC_HIP(hipSetDevice(b->device));
    Serve S(b, n);
    int rc = S.setup(req, host_origin ? cfg->arena_bytes : 0);
    if (!rc) rc = S.run(jobs, req, arrival_s, *cfg, single, host_origin, latency_s, batch_id);
    if (!rc) rc = S.collect(req, chi_host, status);
    S.teardown();
    if (prev != b->device) (void)hipSetDevice(prev);
    return rc;
}

}  // extern "C"
