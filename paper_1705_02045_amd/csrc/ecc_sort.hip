// Stable LSD radix sort of float records (32-bit key, 8-bit change), 8-bit
// digits, four passes (Sec. 3, "Floating Point Values": the values are
// sorted before the running sum).
//
// Each wave owns a segment of kSegRecords consecutive records.  A pass:
//  1. digit counts per (digit, segment), digit-major, from a per-wave LDS
//     histogram;
//  2. exclusive scan of that table: the output position of the first record
//     of each digit in each segment;
//  3. the wave walks its segment in order, 64 records at a time; the lanes
//     with equal digits find each other with eight ballots, take ranks by
//     lane order, and the leader advances the digit's running position.
// Records keep their order within a digit, so every pass is stable.

#include "ecc_internal.h"

namespace ecc {

constexpr int kSortThreads = 256;  // four waves
constexpr int kSegRounds = 256;
constexpr int64_t kSegRecords = (int64_t)kSegRounds * kWave;

__global__ void __launch_bounds__(kSortThreads) radix_count_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                                   int shift, int64_t segs,
                                                                   uint32_t *__restrict__ counts) {
    __shared__ uint32_t cnt[kSortThreads / kWave][256];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    for (int d = lane; d < 256; d += kWave) cnt[wave][d] = 0;
    __syncthreads();
    const int64_t seg = (int64_t)blockIdx.x * (kSortThreads / kWave) + wave;
    if (seg < segs) {
        const int64_t i0 = seg * kSegRecords;
        for (int r = 0; r < kSegRounds; ++r) {
            const int64_t i = i0 + (int64_t)r * kWave + lane;
            if (i < n) atomicAdd(&cnt[wave][(keys[i] >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    if (seg < segs)
        for (int d = lane; d < 256; d += kWave) counts[(int64_t)d * segs + seg] = cnt[wave][d];
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(const uint32_t *__restrict__ keys_in,
                                                                     const int8_t *__restrict__ vals_in, int64_t n,
                                                                     int shift, int64_t segs,
                                                                     const uint32_t *__restrict__ offsets,
                                                                     uint32_t *__restrict__ keys_out,
                                                                     int8_t *__restrict__ vals_out) {
    __shared__ uint32_t pos[kSortThreads / kWave][256];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    const int64_t seg = (int64_t)blockIdx.x * (kSortThreads / kWave) + wave;
    if (seg >= segs) return;  // whole wave (no block barriers below)
    for (int d = lane; d < 256; d += kWave) pos[wave][d] = offsets[(int64_t)d * segs + seg];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t i0 = seg * kSegRecords;
    for (int r = 0; r < kSegRounds; ++r) {
        const int64_t i = i0 + (int64_t)r * kWave + lane;
        if (i0 + (int64_t)r * kWave >= n) break;  // uniform
        const bool in = i < n;
        const uint32_t k = in ? keys_in[i] : 0u;
        const int8_t v = in ? vals_in[i] : (int8_t)0;
        const uint32_t d = (k >> shift) & 255u;
        uint64_t peers = __builtin_amdgcn_ballot_w64(in);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __builtin_amdgcn_ballot_w64((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__builtin_popcountll(peers & lt);
        const uint32_t p = pos[wave][d] + rank;
        if (in) {
            keys_out[p] = k;
            vals_out[p] = v;
        }
        // the lowest lane of each digit group advances the group's position
        // (every lane has read it above: one wave, program order)
        if (in && rank == 0) pos[wave][d] += (uint32_t)__builtin_popcountll(peers);
    }
}

// ----------------------------------------------------------------------------
// Exclusive scan of a uint32 array in place (totals below 2^32): tile sums,
// one workgroup scanning the tile sums, then the tiles with their offsets.

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads) scan_tile_sums_kernel(const uint32_t *__restrict__ a, int64_t n,
                                                                      uint32_t *__restrict__ sums) {
    __shared__ uint32_t sh[kScanThreads / kWave];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = t0 + (int64_t)j * kScanThreads + threadIdx.x;
        if (i < n) s += a[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) t += sh[w];
        sums[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(1024) scan_sums_kernel(uint32_t *sums, int64_t nt) {
    __shared__ uint32_t ws[16];
    __shared__ uint32_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nt; c0 += 1024) {
        const int64_t i = c0 + tid;
        const uint32_t v = i < nt ? sums[i] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t u = __shfl_up(x, off, 64);
            if (lane >= off) x += u;
        }
        if (lane == 63) ws[wave] = x;
        __syncthreads();
        uint32_t p = carry;
        for (int w = 0; w < wave; ++w) p += ws[w];
        if (i < nt) sums[i] = p + x - v;
        __syncthreads();
        if (tid == 0)
            for (int w = 0; w < 16; ++w) carry += ws[w];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) scan_tiles_kernel(uint32_t *__restrict__ a, int64_t n,
                                                                  const uint32_t *__restrict__ sums) {
    __shared__ uint32_t ws[kScanThreads / kWave];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (i0 + j < n) ? a[i0 + j] : 0u;
        s += v[j];
    }
    uint32_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(x, off, 64);
        if (lane >= off) x += u;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    uint32_t p = sums[blockIdx.x] + x - s;
    for (int w = 0; w < wave; ++w) p += ws[w];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (i0 + j < n) a[i0 + j] = p;
        p += v[j];
    }
}

static int exclusive_scan_u32(uint32_t *a, int64_t n, uint32_t *sums, hipStream_t stream) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)nt), dim3(kScanThreads), 0, stream, (const uint32_t *)a, n,
                       sums);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, stream, sums, nt);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)nt), dim3(kScanThreads), 0, stream, a, n,
                       (const uint32_t *)sums);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

int64_t radix_segments(int64_t n) { return (n + kSegRecords - 1) / kSegRecords; }
int64_t radix_scan_tiles(int64_t entries) { return (entries + kScanTile - 1) / kScanTile; }

// Sorts (k[0], v[0]) into (k[0], v[0]) using (k[1], v[1]) as the other buffer
// (four passes: the result ends where it started).  counts: 256 * segs
// entries; sums: radix_scan_tiles(256 * segs) entries.
int radix_sort_records(uint32_t *k[2], int8_t *v[2], int64_t n, uint32_t *counts, uint32_t *sums,
                       hipStream_t stream) {
    if (n <= 1) return ECC_OK;
    if (n > (int64_t)UINT32_MAX) {
        set_error("radix sort: too many records");
        return ECC_E_UNSUPPORTED;
    }
    const int64_t segs = radix_segments(n);
    const int64_t blocks = (segs + (kSortThreads / kWave) - 1) / (kSortThreads / kWave);
    int cur = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(radix_count_kernel, dim3((unsigned)blocks), dim3(kSortThreads), 0, stream,
                           (const uint32_t *)k[cur], n, shift, segs, counts);
        ECC_HIP(hipGetLastError());
        int rc = exclusive_scan_u32(counts, 256 * segs, sums, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)blocks), dim3(kSortThreads), 0, stream,
                           (const uint32_t *)k[cur], (const int8_t *)v[cur], n, shift, segs,
                           (const uint32_t *)counts, k[cur ^ 1], v[cur ^ 1]);
        ECC_HIP(hipGetLastError());
        cur ^= 1;
    }
    return ECC_OK;
}

}  // namespace ecc
