// Merging the per-workgroup change vectors and the prefix sum (Sec. 3,
// "Post-Processing": the VCECs of all workers are summed and the curve is
// their running sum).
#include "ecc_internal.h"

namespace ecc {

__global__ void zero_kernel(uint32_t *p, size_t words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

int launch_zero(void *p, size_t bytes, hipStream_t stream) {
    if (bytes % 4) {
        set_error("launch_zero: size %zu not a multiple of 4", bytes);
        return ECC_E_ARG;
    }
    const size_t words = bytes / 4;
    const int threads = 256;
    int blocks = (int)((words + threads - 1) / threads);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(threads), 0, stream, (uint32_t *)p, words);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// Merge of the per-workgroup rows [rows][m] (int32) into the int64 change
// vector, in kernels that follow each other on the stream (the kernel
// boundary orders their memory; no fences or counters):
//  1. colsum_kernel, block (bx, by): rows by, by+BY, ... of columns
//     bx*1024 .. +1023 (256 threads x 4 columns, 16-byte loads), written to
//     stage[by][column], or, with BY == 1, straight into vcec;
//  2. fold_scan_kernel: the BY stage rows of each column into vcec (BY > 1)
//     and, with do_scan, the prefix sums of column groups of 1024;
//  3. scan_offsets_kernel (do_scan): adds the totals of the preceding groups;
//     the curve is written only if the status word is clear, and the status
//     is copied out and cleared.
// With `reverse`, colsum_kernel writes column c of the rows at m-1-c (the
// largest-value convention: the kernel counted at m-1-value).
// vcec is overwritten, or added to with `accumulate`.
__global__ void __launch_bounds__(256) colsum_kernel(const int32_t *__restrict__ partial, int rows, int m,
                                                     int64_t *__restrict__ dst, int accumulate, int reverse) {
    const int BY = gridDim.y;
    const int c0 = blockIdx.x * 1024 + threadIdx.x * 4;
    if (c0 >= m) return;
    int64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    const int4 *p = reinterpret_cast<const int4 *>(partial);
    const size_t stride4 = (size_t)m / 4;
    int r = blockIdx.y;
    for (; r + 3 * BY < rows; r += 4 * BY) {
        int4 a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = p[(size_t)(r + j * BY) * stride4 + c0 / 4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s0 += a[j].x;
            s1 += a[j].y;
            s2 += a[j].z;
            s3 += a[j].w;
        }
    }
    for (; r < rows; r += BY) {
        const int4 a = p[(size_t)r * stride4 + c0 / 4];
        s0 += a.x;
        s1 += a.y;
        s2 += a.z;
        s3 += a.w;
    }
    int64_t *row = dst + (size_t)blockIdx.y * m;
    if (reverse) {  // column c lands at m-1-c
        int64_t *d = row + (m - 1 - c0);
        if (accumulate) {
            s0 += d[0];
            s1 += d[-1];
            s2 += d[-2];
            s3 += d[-3];
        }
        d[0] = s0;
        d[-1] = s1;
        d[-2] = s2;
        d[-3] = s3;
        return;
    }
    int64_t *d = row + c0;
    if (accumulate) {
        s0 += d[0];
        s1 += d[1];
        s2 += d[2];
        s3 += d[3];
    }
    d[0] = s0;
    d[1] = s1;
    d[2] = s2;
    d[3] = s3;
}

// Column group bx (1024 columns, 4 per thread): the BY stage rows are folded
// into vcec (when stage is not null) and, with do_scan and a clear status
// word, the group's inclusive prefix sum is written to chi and its total to
// totals[bx].  Block 0 copies the status word to status[1] for the offsets
// kernel.
__global__ void __launch_bounds__(256) fold_scan_kernel(const int64_t *__restrict__ stage, int by, int m,
                                                        int64_t *__restrict__ vcec, int accumulate, int do_scan,
                                                        int64_t *__restrict__ chi, uint32_t *status,
                                                        int64_t *__restrict__ totals) {
    __shared__ int64_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = blockIdx.x * 1024 + tid * 4;
    int64_t v[4] = {0, 0, 0, 0};
    if (c0 < m) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (stage == nullptr || accumulate) ? vcec[c0 + j] : 0;
        if (stage != nullptr) {
            // eight rows of loads in flight (by is a power of two, 2..32)
            int y = 0;
            for (; y + 8 <= by; y += 8) {
                int64_t a[8][4];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int j = 0; j < 4; ++j) a[u][j] = stage[(size_t)(y + u) * m + c0 + j];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] += a[u][j];
            }
            for (; y < by; ++y) {
                const int64_t *st = stage + (size_t)y * m + c0;
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] += st[j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) vcec[c0 + j] = v[j];
        }
    }
    if (!do_scan) return;
    const uint32_t stv = *status;
    if (blockIdx.x == 0 && tid == 0) status[1] = stv;
    if (stv != 0) return;
    // inclusive scan: within the thread, across the wave, across the 4 waves
    v[1] += v[0];
    v[2] += v[1];
    v[3] += v[2];
    int64_t x = v[3];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t u = __shfl_up(x, off, 64);
        if (lane >= off) x += u;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t base = x - v[3];
    for (int w = 0; w < wave; ++w) base += wsum[w];
    if (c0 < m) {
#pragma unroll
        for (int j = 0; j < 4; ++j) chi[c0 + j] = base + v[j];
    }
    if (tid == 0) totals[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Adds the totals of the preceding column groups to chi (when the status
// copied by fold_scan_kernel is clear); block 0 copies the status out and
// clears the status word.
__global__ void __launch_bounds__(256) scan_offsets_kernel(int m, int64_t *__restrict__ chi, uint32_t *status,
                                                           uint32_t *status_out, const int64_t *__restrict__ totals) {
    const uint32_t stv = status[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (status_out) *status_out = stv;
        status[0] = 0u;
    }
    if (stv != 0 || blockIdx.x == 0) return;
    int64_t off = 0;
    for (int j = 0; j < (int)blockIdx.x; ++j) off += totals[j];
    const int c0 = blockIdx.x * 1024 + threadIdx.x * 4;
    if (c0 < m) {
#pragma unroll
        for (int j = 0; j < 4; ++j) chi[c0 + j] += off;
    }
}

// ----------------------------------------------------------------------------
// Batched merge over the images of a batch table (fixed grids: the graph of
// a batched run does not change with its contents).
// batch_colsum_kernel: item i = (image j, 1024-column group g), j found in
// the table's item prefix: sums image j's rows over those columns into its
// vcec.  batch_scan_kernel: image j (blocks loop over images) writes its
// curve if its status word is clear, copies the status out and clears it.

__device__ __forceinline__ int find_prefix(const int32_t *begin, int n, int v) {
    int lo = 0, hi = n - 1;  // last j with begin[j] <= v
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) batch_colsum_kernel(const uint8_t *__restrict__ table) {
    const BatchHeader *H = (const BatchHeader *)table;
    const MergeJob *jobs = (const MergeJob *)(table + H->off_merge);
    const int32_t *item_begin = (const int32_t *)(table + H->off_item_begin);
    for (int i = blockIdx.x; i < H->nitems; i += gridDim.x) {
        const int j = __builtin_amdgcn_readfirstlane(find_prefix(item_begin, H->njobs, i));
        const MergeJob J = jobs[j];
        const int c0 = (i - item_begin[j]) * 1024 + threadIdx.x * 4;
        if (c0 >= J.m) continue;
        const int4 *p = reinterpret_cast<const int4 *>(J.partial);
        const size_t stride4 = (size_t)J.m / 4;
        int64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        int r = 0;
        for (; r + 8 <= J.rows; r += 8) {  // eight rows of loads in flight
            int4 a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = p[(size_t)(r + u) * stride4 + c0 / 4];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s0 += a[u].x;
                s1 += a[u].y;
                s2 += a[u].z;
                s3 += a[u].w;
            }
        }
        for (; r < J.rows; ++r) {
            const int4 a = p[(size_t)r * stride4 + c0 / 4];
            s0 += a.x;
            s1 += a.y;
            s2 += a.z;
            s3 += a.w;
        }
        J.vcec[c0] = s0;
        J.vcec[c0 + 1] = s1;
        J.vcec[c0 + 2] = s2;
        J.vcec[c0 + 3] = s3;
    }
}

// One image per workgroup of 1024 threads, chunks of 16384 entries: thread t
// holds entries c0 + k * 1024 + t (k < 16: sixteen rows, every load and
// store coalesced).  Each row is scanned across the wave with shuffles; the
// wave totals per row go to LDS, where 16 threads turn them into per-wave
// prefixes and row totals; every thread then adds the rows before its row and
// the waves before its wave.  The running carry is the same in all threads.
__global__ void __launch_bounds__(1024) batch_scan_kernel(const uint8_t *__restrict__ table) {
    __shared__ int64_t ws[16][17];   // [row][wave]: wave totals, then exclusive prefixes over the waves
    __shared__ int64_t rowtot[16];
    const BatchHeader *H = (const BatchHeader *)table;
    const MergeJob *jobs = (const MergeJob *)(table + H->off_merge);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int jb = blockIdx.x; jb < H->njobs; jb += gridDim.x) {
        const MergeJob J = jobs[jb];
        const uint32_t stv = *J.status;
        __syncthreads();  // every wave holds the status before thread 0 clears it below
        if (stv == 0) {
            int64_t carry = 0;
            for (int c0 = 0; c0 < J.m; c0 += 1024 * 16) {
                int64_t v[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int i = c0 + k * 1024 + tid;
                    v[k] = i < J.m ? J.vcec[i] : 0;
                }
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int64_t u = __shfl_up(v[k], off, 64);
                        if (lane >= off) v[k] += u;
                    }
                }
                if (lane == 63) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) ws[k][wave] = v[k];
                }
                __syncthreads();
                if (tid < 16) {  // row tid: exclusive prefix over the waves, and the row total
                    int64_t run = 0;
                    for (int w = 0; w < 16; ++w) {
                        const int64_t x = ws[tid][w];
                        ws[tid][w] = run;
                        run += x;
                    }
                    rowtot[tid] = run;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int i = c0 + k * 1024 + tid;
                    if (i < J.m) J.chi[i] = carry + ws[k][wave] + v[k];
                    carry += rowtot[k];
                }
                __syncthreads();  // ws and rowtot are rewritten by the next chunk
            }
        }
        if (tid == 0) {
            if (J.status_out) *J.status_out = stv;
            *J.status = 0u;
        }
        __syncthreads();  // the status of the next image of this workgroup
    }
}

int launch_batch_merge(const void *table_dev, int colsum_grid, int scan_grid, hipStream_t stream) {
    hipLaunchKernelGGL(batch_colsum_kernel, dim3(colsum_grid), dim3(256), 0, stream, (const uint8_t *)table_dev);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(batch_scan_kernel, dim3(scan_grid), dim3(1024), 0, stream, (const uint8_t *)table_dev);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// ----------------------------------------------------------------------------
// Dual complex helpers: strided gather of a face of the box, signed sum of
// the faces' curves.

template <typename T>
__global__ void __launch_bounds__(256) gather_kernel(const T *__restrict__ src, int64_t base, int64_t s0, int64_t s1,
                                                     int64_t s2, int64_t n1, int64_t n2, int64_t total,
                                                     T *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t i2 = i % n2, r = i / n2;
        const int64_t i1 = r % n1, i0 = r / n1;
        dst[i] = src[base + i0 * s0 + i1 * s1 + i2 * s2];
    }
}

int launch_gather(const void *src, int elem, int64_t base, int64_t s0, int64_t s1, int64_t s2, int64_t n0,
                  int64_t n1, int64_t n2, void *dst, hipStream_t stream) {
    const int64_t total = n0 * n1 * n2;
    if (total <= 0) return ECC_OK;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (elem == 1)
        hipLaunchKernelGGL(gather_kernel<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint8_t *)src,
                           base, s0, s1, s2, n1, n2, total, (uint8_t *)dst);
    else
        hipLaunchKernelGGL(gather_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const uint16_t *)src, base, s0, s1, s2, n1, n2, total, (uint16_t *)dst);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

__global__ void __launch_bounds__(256) signed_sum_kernel(const int64_t *__restrict__ curves, int nf, uint64_t neg0,
                                                         uint64_t neg1, uint64_t skip0, uint64_t skip1, int sign,
                                                         int m, int64_t *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    int64_t acc = 0;
    for (int f = 0; f < nf; ++f) {
        const uint64_t skip = f < 64 ? skip0 >> f : skip1 >> (f - 64);
        const uint64_t neg = f < 64 ? neg0 >> f : neg1 >> (f - 64);
        if (skip & 1) continue;
        const int64_t v = curves[(size_t)f * m + t];
        acc += (neg & 1) ? -v : v;
    }
    out[t] = sign < 0 ? -acc : acc;
}

int launch_signed_sum(const int64_t *curves, int nf, const uint64_t neg_mask[2], const uint64_t skip_mask[2],
                      int sign, int m, int64_t *out, hipStream_t stream) {
    if (nf > 128) {
        set_error("internal error: %d faces", nf);
        return ECC_E_ARG;
    }
    hipLaunchKernelGGL(signed_sum_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, curves, nf, neg_mask[0],
                       neg_mask[1], skip_mask[0], skip_mask[1], sign, m, out);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// Faces of at most one dimension (box edges and corners), largest-value
// convention, added with their signs straight into a changes vector.  A
// line of n voxels is the 1-D complex of n intervals (value: the voxel's)
// and n + 1 vertices (value: the larger of the voxels they touch); its
// changes vector adds +1 at each vertex's value and -1 at each interval's.
// A corner is one vertex.  Values >= m are skipped (the volume's own launch
// reports them as range errors).  One workgroup of 1024 threads per face
// (an edge of up to 1023 voxels in one round of loads).
template <typename T>
__global__ void __launch_bounds__(1024) low_faces_kernel(const T *__restrict__ img, const LowFace *__restrict__ faces,
                                                        int m, int64_t *__restrict__ out) {
    const LowFace F = faces[blockIdx.x];
    auto val = [&](int64_t i) -> uint32_t { return (uint32_t)img[F.base + i * F.stride]; };
    auto add = [&](uint32_t v, int64_t c) {
        if (v < (uint32_t)m) atomicAdd((unsigned long long *)&out[v], (unsigned long long)c);
    };
    const int64_t s = F.sign;
    for (int64_t i = threadIdx.x; i <= F.len; i += blockDim.x) {
        if (F.len == 0) {  // a corner: one vertex
            if (i == 0) add(val(0), s);
            continue;
        }
        // vertex i: between voxels i-1 and i (one voxel at either end)
        const uint32_t a = i > 0 ? val(i - 1) : 0u, b = i < F.len ? val(i) : 0u;
        add(i == 0 ? b : i == F.len ? a : (a > b ? a : b), s);
        if (i < F.len) add(b, -s);  // interval i
    }
}

int launch_low_faces(const void *img, int elem, const LowFace *faces_dev, int nfaces, int m, int64_t *out,
                     hipStream_t stream) {
    if (nfaces <= 0) return ECC_OK;
    if (elem == 1)
        hipLaunchKernelGGL(low_faces_kernel<uint8_t>, dim3(nfaces), dim3(1024), 0, stream, (const uint8_t *)img,
                           faces_dev, m, out);
    else
        hipLaunchKernelGGL(low_faces_kernel<uint16_t>, dim3(nfaces), dim3(1024), 0, stream, (const uint16_t *)img,
                           faces_dev, m, out);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

__global__ void minmax_init_kernel(uint32_t *out) {
    out[0] = 0xFFFFFFFFu;
    out[1] = 0u;
}

__global__ void __launch_bounds__(256) minmax_u16_kernel(const uint16_t *__restrict__ img, int64_t n, int vec,
                                                         uint32_t *out) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n8 = vec ? n / 8 : 0;  // 16-byte groups when the image is 16-byte aligned
    const uint4 *v8 = reinterpret_cast<const uint4 *>(img);
    auto fold = [&](const uint4 q) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t a = w[j] & 0xFFFFu, b = w[j] >> 16;
            lo = min(lo, min(a, b));
            hi = max(hi, max(a, b));
        }
    };
    // each workgroup streams one contiguous chunk, four independent 16-byte
    // loads in flight per thread
    const int64_t chunk = (n8 + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n8 ? beg + chunk : n8;
    const int64_t bd = blockDim.x;
    int64_t i = beg + threadIdx.x;
    for (; i + 3 * bd < end; i += 4 * bd) {
        uint4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = v8[i + u * bd];
#pragma unroll
        for (int u = 0; u < 4; ++u) fold(q[u]);
    }
    for (; i < end; i += bd) fold(v8[i]);
    for (int64_t i = n8 * 8 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        lo = min(lo, (uint32_t)img[i]);
        hi = max(hi, (uint32_t)img[i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&out[0], lo);
        atomicMax(&out[1], hi);
    }
}

int launch_minmax_u16(const uint16_t *img, int64_t n, uint32_t *out, hipStream_t stream) {
    hipLaunchKernelGGL(minmax_init_kernel, dim3(1), dim3(1), 0, stream, out);
    ECC_HIP(hipGetLastError());
    int64_t blocks = (n / 8 + 255) / 256;
    const int64_t cap = 8 * (int64_t)device_cu_count();  // eight workgroups of 4 waves per CU
    if (blocks < 1) blocks = 1;
    if (blocks > cap) blocks = cap;
    const int vec = ((uintptr_t)img % 16) == 0;
    hipLaunchKernelGGL(minmax_u16_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, img, n, vec, out);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// Curves of at most 1024 thresholds from at most kSmallMergeRows rows: the
// three merge kernels above in one workgroup (256 threads x 4 columns), for
// the latency of small images.  The column sums are placed through LDS
// (with `reverse`, column c lands at m-1-c, in another thread's columns);
// then vcec, the scan into chi (only with a clear status word), and the
// status copy and clear, as in the three-kernel form.
constexpr int kSmallMergeRows = 64;
__global__ void __launch_bounds__(256) merge_scan_small_kernel(const int32_t *__restrict__ partial, int rows, int m,
                                                               int64_t *__restrict__ vcec, int accumulate, int reverse,
                                                               int64_t *__restrict__ chi, uint32_t *status,
                                                               uint32_t *status_out) {
    __shared__ int64_t col[1024];
    __shared__ int64_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = tid * 4;
    const bool own = c0 < m;
    const uint32_t stv = *status;  // cleared below, after a barrier
    if (rows > 0) {
        if (own) {
            int64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
            const int4 *p = reinterpret_cast<const int4 *>(partial) + c0 / 4;
            const size_t stride4 = (size_t)m / 4;
            int r = 0;
            for (; r + 8 <= rows; r += 8) {
                int4 a[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) a[j] = p[(size_t)(r + j) * stride4];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    s0 += a[j].x;
                    s1 += a[j].y;
                    s2 += a[j].z;
                    s3 += a[j].w;
                }
            }
            for (; r < rows; ++r) {
                const int4 a = p[(size_t)r * stride4];
                s0 += a.x;
                s1 += a.y;
                s2 += a.z;
                s3 += a.w;
            }
            if (reverse) {
                col[m - 1 - c0] = s0;
                col[m - 2 - c0] = s1;
                col[m - 3 - c0] = s2;
                col[m - 4 - c0] = s3;
            } else {
                col[c0] = s0;
                col[c0 + 1] = s1;
                col[c0 + 2] = s2;
                col[c0 + 3] = s3;
            }
        }
        __syncthreads();
    }
    int64_t v[4] = {0, 0, 0, 0};
    if (own) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t x = (rows == 0 || accumulate) ? vcec[c0 + j] : 0;
            if (rows > 0) x += col[c0 + j];
            v[j] = x;
        }
        if (rows > 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) vcec[c0 + j] = v[j];
        }
    }
    // inclusive scan: within the thread, across the wave, across the 4 waves
    v[1] += v[0];
    v[2] += v[1];
    v[3] += v[2];
    int64_t x = v[3];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t u = __shfl_up(x, off, 64);
        if (lane >= off) x += u;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t base = x - v[3];
    for (int w = 0; w < wave; ++w) base += wsum[w];
    if (own && stv == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) chi[c0 + j] = base + v[j];
    }
    if (tid == 0) {
        status[1] = stv;
        if (status_out) *status_out = stv;
        status[0] = 0u;
    }
}

int merge_stage_rows(int rows) {
    int by = 1;
    while (by < 32 && by * 8 <= rows) by *= 2;
    return by;
}

int launch_merge(const int32_t *partial, int rows, int m, int64_t *stage, int64_t *vcec, bool accumulate,
                 bool do_scan, int64_t *chi, uint32_t *status, uint32_t *status_out, hipStream_t stream,
                 bool reverse) {
    if (m % 4 != 0 || m > 65536) {
        set_error("launch_merge: m = %d not supported", m);
        return ECC_E_ARG;
    }
    const int groups = (m + 1023) / 1024;
    if (do_scan && groups == 1 && rows <= kSmallMergeRows) {
        hipLaunchKernelGGL(merge_scan_small_kernel, dim3(1), dim3(256), 0, stream, partial, rows, m, vcec,
                           accumulate ? 1 : 0, reverse ? 1 : 0, chi, status, status_out);
        ECC_HIP(hipGetLastError());
        return ECC_OK;
    }
    int by = 0;
    if (rows > 0) {
        by = merge_stage_rows(rows);
        hipLaunchKernelGGL(colsum_kernel, dim3(groups, by), dim3(256), 0, stream, partial, rows, m,
                           by == 1 ? vcec : stage, (by == 1 && accumulate) ? 1 : 0, reverse ? 1 : 0);
        ECC_HIP(hipGetLastError());
    }
    if (by > 1 || do_scan) {
        int64_t *totals = reinterpret_cast<int64_t *>(status) + kStatusTotalsOffset / 8;
        hipLaunchKernelGGL(fold_scan_kernel, dim3(groups), dim3(256), 0, stream, by > 1 ? (const int64_t *)stage : nullptr,
                           by, m, vcec, accumulate ? 1 : 0, do_scan ? 1 : 0, chi, status, totals);
        ECC_HIP(hipGetLastError());
        if (do_scan) {
            hipLaunchKernelGGL(scan_offsets_kernel, dim3(groups), dim3(256), 0, stream, m, chi, status, status_out,
                               (const int64_t *)totals);
            ECC_HIP(hipGetLastError());
        }
    }
    return ECC_OK;
}

}  // namespace ecc
