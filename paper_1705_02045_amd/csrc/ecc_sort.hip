// Stable LSD radix sort (Sec. 3, "Other Ranges of Gray Values": the distinct
// values are found by sorting) of the order-preserving 32-bit keys of a
// float image, and of the voxels' non-zero (key, change) records, 64-bit
// words with the key in the high half, sorted on that half.  Four passes of
// 8-bit digits.
//
// A workgroup owns a tile of kTile consecutive keys.  A pass:
//  1. radix_count_kernel: digit counts per (digit, tile), digit-major;
//  2. exclusive scan of that table: the output position of the first key
//     of each digit of each tile;
//  3. radix_scatter_kernel: the tile is ranked stably in LDS (each wave
//     ranks its kItems * 64 consecutive keys: lanes with equal digits find each
//     other with eight ballots and the wave keeps its digit counts in its
//     own LDS row; then one prefix over the waves per digit), reordered by
//     digit in LDS, and written out: keys of one digit leave a tile as one
//     contiguous run, so the stores coalesce.

#include "ecc_internal.h"

#include <algorithm>

namespace ecc {

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / kWave;

// Items per thread: the LDS tile of the scatter kernel is kItems words.
template <typename T>
struct SortTile {
    static constexpr int kItems = sizeof(T) == 4 ? 8 : 8;
    static constexpr int64_t kTile = (int64_t)kSortThreads * kItems;
};

template <typename T>
__device__ __forceinline__ uint32_t digit_of(T r, int shift) { return (uint32_t)(r >> shift) & 255u; }

// A count workgroup takes tpw <= kCountTiles consecutive tiles, so that its
// counts leave as runs of tpw consecutive words of the digit-major table
// (whole 64-byte lines at tpw = 16, instead of 256 scattered words per tile);
// small sorts take fewer tiles per workgroup to keep the chip busy.
constexpr int kCountTiles = 16;

template <typename T, bool AGG>
__global__ void __launch_bounds__(kSortThreads) radix_count_kernel(const T *__restrict__ rec, int64_t n,
                                                                   int shift, int64_t tiles, int tpw,
                                                                   uint32_t *__restrict__ counts) {
    constexpr int kItems = SortTile<T>::kItems;
    constexpr int64_t kTile = SortTile<T>::kTile;
    __shared__ uint32_t cnt[kCountTiles][257];  // (padded: the final transpose reads a column)
    const int tid = threadIdx.x;
    for (int i = tid; i < kCountTiles * 257; i += kSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int lane = tid & (kWave - 1);
    const int64_t tb = (int64_t)blockIdx.x * tpw;
    for (int k = 0; k < tpw && tb + k < tiles; ++k) {
        const int64_t t0 = (tb + k) * kTile;
        T r[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = t0 + (int64_t)j * kSortThreads + tid;
            r[j] = i < n ? rec[i] : T(0);
        }
        // AGG (the top digit: sign and exponent, a handful of values): same-digit
        // lanes would serialize on one LDS address, so up to four rounds take the
        // digit of the lowest lane not yet counted and add all its lanes through
        // that lane; what is left (many distinct digits) adds per lane.  On the
        // low digits per-lane adds are cheaper.
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = t0 + (int64_t)j * kSortThreads + tid;
            const bool ok = i < n;
            const uint32_t d = digit_of(r[j], shift);
            if constexpr (!AGG) {
                if (ok) atomicAdd(&cnt[k][d], 1u);
                continue;
            }
            uint64_t rem = __builtin_amdgcn_ballot_w64(ok);
            for (int it = 0; it < 4 && rem != 0; ++it) {
                const int l0 = (int)__builtin_ctzll(rem);
                const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, l0);
                const uint64_t m = __builtin_amdgcn_ballot_w64(d == d0) & rem;
                if (lane == l0) atomicAdd(&cnt[k][d0], (uint32_t)__builtin_popcountll(m));
                rem &= ~m;
            }
            if ((rem >> lane) & 1ull) atomicAdd(&cnt[k][d], 1u);
        }
    }
    __syncthreads();
    for (int i = tid; i < tpw * 256; i += kSortThreads) {
        const int k = i % tpw, d = i / tpw;
        if (tb + k < tiles) counts[(int64_t)d * tiles + tb + k] = cnt[k][d];
    }
}

template <typename T>
__global__ void __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(8))) radix_scatter_kernel(const T *__restrict__ in, int64_t n,
                                                                     int shift, int64_t tiles,
                                                                     const uint32_t *__restrict__ offsets,
                                                                     T *__restrict__ out) {
    constexpr int kItems = SortTile<T>::kItems;
    constexpr int64_t kTile = SortTile<T>::kTile;
    constexpr int kChunk = kItems * kWave;       // keys of one wave, consecutive
    __shared__ T buf[kTile];                     // the tile reordered by digit
    __shared__ uint16_t wcnt[kSortWaves][256];   // per wave: digit counts, then the wave's offset per digit
    __shared__ uint32_t start[256];              // digit totals, then the first slot of each digit
    __shared__ uint32_t dest[256];               // per digit: output position minus first slot
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    // neighbouring tiles on one XCD: they read neighbouring words of the
    // offset table and write neighbouring ends of each digit's runs
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t0 = (int64_t)tile * kTile;
    // the tile's output position per digit, loaded while the tile is ranked
    const uint32_t gpos = tid < 256 ? offsets[(int64_t)tid * tiles + tile] : 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) wcnt[wave][lane * 4 + q] = 0;  // the wave's own row

    // wave w ranks keys t0 + w*kChunk + j*64 + lane (j = 0..kItems-1), in
    // that order: tile order, so the ranking is stable
    T r[kItems];
    uint32_t rank[kItems];
    const int64_t wb = t0 + (int64_t)wave * kChunk;
    // (a full tile, every tile but the last: loads and stores without bounds
    // checks)
    const bool full = t0 + kTile <= n;
    if (full) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) r[j] = in[wb + j * kWave + lane];
    } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = wb + (int64_t)j * kWave + lane;
            r[j] = i < n ? in[i] : ~T(0);  // past the end: digit 255, last in the tile, never written
        }
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t d = digit_of(r[j], shift);
        // peers: the lanes whose digit equals this lane's, as two 32-bit
        // halves: the complement of the lanes that disagree with this lane on
        // some bit.  Per bit, sb is all ones where the bit is set (kept
        // opaque, so that the ballot compares it instead of recomputing the
        // bit) and m the ballot of the lanes with the bit set; per half,
        // x = (m0 ^ sb0) | (m1 ^ sb1) | ... with one three-input op per bit
        // after the first (x | (m ^ sb): truth table 0xF6 over (x, m, sb)).
        // The ballots are VALU writes of scalar registers, which a VALU op may
        // read only two wait states later: each block starts with s_nop 1.
        uint32_t sb[8];
        uint64_t m[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            sb[b] = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
            asm("" : "+v"(sb[b]));
            m[b] = __builtin_amdgcn_ballot_w64(sb[b] != 0);
        }
        uint32_t xlo, xhi;
#define ECC_MISMATCH(X, H)                                                                                       \
    asm("s_nop 1\n\t"                                                                                           \
        "v_xor_b32 %0, %1, %9\n\t"                                                                              \
        "v_bitop3_b32 %0, %0, %2, %10 bitop3:0xf6\n\t"                                                          \
        "v_bitop3_b32 %0, %0, %3, %11 bitop3:0xf6\n\t"                                                          \
        "v_bitop3_b32 %0, %0, %4, %12 bitop3:0xf6\n\t"                                                          \
        "v_bitop3_b32 %0, %0, %5, %13 bitop3:0xf6\n\t"                                                          \
        "v_bitop3_b32 %0, %0, %6, %14 bitop3:0xf6\n\t"                                                          \
        "v_bitop3_b32 %0, %0, %7, %15 bitop3:0xf6\n\t"                                                          \
        "v_bitop3_b32 %0, %0, %8, %16 bitop3:0xf6"                                                                \
        : "=&v"(X)                                                                                                \
        : "s"(H(m[0])), "s"(H(m[1])), "s"(H(m[2])), "s"(H(m[3])), "s"(H(m[4])), "s"(H(m[5])), "s"(H(m[6])),    \
          "s"(H(m[7])), "v"(sb[0]), "v"(sb[1]), "v"(sb[2]), "v"(sb[3]), "v"(sb[4]), "v"(sb[5]), "v"(sb[6]),      \
          "v"(sb[7]))
#define ECC_LO(v) ((uint32_t)(v))
#define ECC_HI(v) ((uint32_t)((v) >> 32))
        ECC_MISMATCH(xlo, ECC_LO);
        ECC_MISMATCH(xhi, ECC_HI);
#undef ECC_HI
#undef ECC_LO
#undef ECC_MISMATCH
        const uint32_t plo = ~xlo, phi = ~xhi;
        const uint32_t rw = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));  // peers below
        // the wave's own count row: LDS operations of one wave take effect in order
        const uint32_t base = wcnt[wave][d];
        rank[j] = base + rw;
        if (rw == 0) wcnt[wave][d] = (uint16_t)(base + __builtin_popcount(plo) + __builtin_popcount(phi));
    }
    __syncthreads();
    if (tid < 256) {  // per digit: the waves' offsets and the digit's total
        uint32_t acc = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = wcnt[w][tid];
            wcnt[w][tid] = (uint16_t)acc;
            acc += c;
        }
        start[tid] = acc;
    }
    __syncthreads();
    // first slot of each digit: exclusive scan of the totals (one wave, four
    // digits per lane)
    if (tid < kWave) {
        uint32_t v[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = start[tid * 4 + q];
            s += v[q];
        }
        uint32_t x = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t u = __shfl_up(x, off, 64);
            if (lane >= off) x += u;
        }
        uint32_t p = x - s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            start[tid * 4 + q] = p;
            p += v[q];
        }
    }
    __syncthreads();
    if (tid < 256) dest[tid] = gpos - start[tid];  // (mod 2^32: positions are below 2^32)
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t d = digit_of(r[j], shift);
        buf[start[d] + wcnt[wave][d] + rank[j]] = r[j];
    }
    __syncthreads();
    if (full) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int s = j * kSortThreads + tid;
            const T v = buf[s];
            out[dest[digit_of(v, shift)] + (uint32_t)s] = v;
        }
        return;
    }
    const int64_t valid = n - t0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int s = j * kSortThreads + tid;
        if (s < valid) {
            const T v = buf[s];
            const uint32_t d = digit_of(v, shift);
            out[dest[d] + (uint32_t)s] = v;
        }
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
    // a thread's run of kScanItems counts is 64 contiguous bytes: 16-byte
    // loads and stores where the whole run is in range and aligned
    static_assert(kScanItems % 4 == 0, "runs of whole 16-byte groups");
    const bool vec = ((reinterpret_cast<uintptr_t>(a) & 15u) == 0) && i0 + kScanItems <= n;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    if (vec) {
        const uint4 *a4 = reinterpret_cast<const uint4 *>(a + i0);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const uint4 w = a4[q];
            v[4 * q] = w.x;
            v[4 * q + 1] = w.y;
            v[4 * q + 2] = w.z;
            v[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) v[j] = (i0 + j < n) ? a[i0 + j] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += v[j];
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
    uint32_t e[kScanItems];  // exclusive prefix of the run
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        e[j] = p;
        p += v[j];
    }
    if (vec) {
        uint4 *a4 = reinterpret_cast<uint4 *>(a + i0);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) a4[q] = make_uint4(e[4 * q], e[4 * q + 1], e[4 * q + 2], e[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j)
            if (i0 + j < n) a[i0 + j] = e[j];
    }
}

int exclusive_scan_u32(uint32_t *a, int64_t n, uint32_t *sums, hipStream_t stream) {
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

int64_t radix_tiles(int64_t n, int elem) {
    const int64_t t = elem == 4 ? SortTile<uint32_t>::kTile : SortTile<uint64_t>::kTile;
    return (n + t - 1) / t;
}
int64_t radix_scan_tiles(int64_t entries) { return (entries + kScanTile - 1) / kScanTile; }

// Four passes on the 32 bits from bit `low` up: v[0] ends sorted, v[1]
// being the other buffer.
template <typename T>
static int radix_sort(T *v[2], int64_t n, int low, uint32_t *counts, uint32_t *sums, hipStream_t stream) {
    if (n <= 1) return ECC_OK;
    if (n > (int64_t)UINT32_MAX) {
        set_error("radix sort: too many keys");
        return ECC_E_UNSUPPORTED;
    }
    const int64_t tiles = radix_tiles(n, (int)sizeof(T));
    const int tpw = (int)std::min<int64_t>(kCountTiles, std::max<int64_t>(1, tiles / 2048));
    const unsigned cgrid = (unsigned)((tiles + tpw - 1) / tpw);
    int cur = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = low + 8 * pass;
        if (pass == 3)
            hipLaunchKernelGGL((radix_count_kernel<T, true>), dim3(cgrid), dim3(kSortThreads), 0, stream,
                               (const T *)v[cur], n, shift, tiles, tpw, counts);
        else
            hipLaunchKernelGGL((radix_count_kernel<T, false>), dim3(cgrid), dim3(kSortThreads), 0, stream,
                               (const T *)v[cur], n, shift, tiles, tpw, counts);
        ECC_HIP(hipGetLastError());
        int rc = exclusive_scan_u32(counts, 256 * tiles, sums, stream);
        if (rc) return rc;
        hipLaunchKernelGGL((radix_scatter_kernel<T>), dim3((unsigned)tiles), dim3(kSortThreads), 0, stream,
                           (const T *)v[cur], n, shift, tiles, (const uint32_t *)counts, v[cur ^ 1]);
        ECC_HIP(hipGetLastError());
        cur ^= 1;
    }
    return ECC_OK;
}

int radix_sort_keys(uint32_t *key[2], int64_t n, uint32_t *counts, uint32_t *sums, hipStream_t stream) {
    return radix_sort<uint32_t>(key, n, 0, counts, sums, stream);
}

int radix_sort_records(uint64_t *rec[2], int64_t n, uint32_t *counts, uint32_t *sums, hipStream_t stream) {
    return radix_sort<uint64_t>(rec, n, 32, counts, sums, stream);
}

}  // namespace ecc
