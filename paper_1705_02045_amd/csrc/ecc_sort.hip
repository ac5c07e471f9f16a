// Stable LSD radix sort (Sec. 3, "Other Ranges of Gray Values": the distinct
// values are found by sorting) of the order-preserving 32-bit keys of a
// float image, and of the voxels' non-zero (key, change) records, 64-bit
// words with the key in the high half, sorted on that half.
//
// The records take four passes of 8-bit digits.  The keys take 9-bit
// digits on bits 0-8 and 9-17, then, when the keys hold at most 16 distinct
// top bytes (sign and high exponent bits: a float image whose values span a
// few dozen binades), one pass on bits 18-23 joined to the rank of the key's
// top byte among those present (3 or 4 bits; the rank is monotone in the
// byte, so the order is the keys' own), else two 7-bit passes on bits 18-24
// and 25-31.  The first count pass notes which top bytes occur; the host
// reads that note while the first two passes run and chooses the rest.
//
// A workgroup owns a tile of kTile consecutive keys.  A pass:
//  1. radix_count_kernel: digit counts per (digit, tile), digit-major;
//  2. exclusive scan of that table: the output position of the first key
//     of each digit of each tile;
//  3. radix_scatter_kernel: the tile is ranked stably in LDS (each wave
//     ranks its kItems * 64 consecutive keys: lanes with equal digits find each
//     other with one ballot per digit bit and the wave keeps its digit counts
//     in its own LDS row; then one prefix over the waves per digit),
//     reordered by digit in LDS, and written out: keys of one digit leave a
//     tile as one contiguous run, so the stores coalesce.

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

// The digit of a key: BITS bits from `shift`, or (REMAP, 32-bit keys only)
// bits 18-23 below the rank of the top byte (rank: a 256-entry LDS table;
// the host takes REMAP passes only when every rank fits in BITS - 6 bits).
constexpr int kRemapShift = 18;
constexpr int kRemapLow = 6;

template <typename T, int BITS, bool REMAP>
__device__ __forceinline__ uint32_t digit_of(T r, int shift, const uint8_t *rank) {
    if constexpr (REMAP) {
        static_assert(sizeof(T) == 4 && BITS > kRemapLow, "32-bit keys; the rank takes the digit's high bits");
        return (((uint32_t)r >> kRemapShift) & ((1u << kRemapLow) - 1u)) | ((uint32_t)rank[(uint32_t)r >> 24] << kRemapLow);
    } else {
        return (uint32_t)(r >> shift) & ((1u << BITS) - 1u);
    }
}

// The rank table of REMAP passes from the top-byte presence mask (8 words,
// bit b of word w: byte 32 w + b occurs): rank[t] = present bytes below t.
// Byte 255, when absent, takes the largest rank of a BITS-bit digit, so that
// the all-ones keys that pad the last tile take the largest digit.  Called
// by every thread; ends with a barrier.
template <int BITS>
__device__ __forceinline__ void build_rank(const uint32_t *__restrict__ mask, uint8_t *rank) {
    const int t = threadIdx.x;
    if (t < 256) {
        uint32_t c = 0;
        for (int w = 0; w < (t >> 5); ++w) c += (uint32_t)__builtin_popcount(mask[w]);
        c += (uint32_t)__builtin_popcount(mask[t >> 5] & ((1u << (t & 31)) - 1u));
        if (t == 255 && (mask[7] >> 31) == 0u) c = (1u << (BITS - kRemapLow)) - 1u;
        rank[t] = (uint8_t)c;
    }
    __syncthreads();
}

// A count workgroup takes tpw <= kCountTiles consecutive tiles, so that its
// counts leave as runs of tpw consecutive words of the digit-major table
// (whole 64-byte lines at tpw = 16, instead of 256 scattered words per tile);
// small sorts take fewer tiles per workgroup to keep the chip busy.
constexpr int kCountTiles = 16;

// MASK (the first pass over 32-bit keys): also ORs the presence of each
// key's top byte into mask (8 words, zero before the launch).
template <typename T, int BITS, bool AGG, bool REMAP, bool MASK>
__global__ void __launch_bounds__(kSortThreads) radix_count_kernel(const T *__restrict__ rec, int64_t n,
                                                                   int shift, int64_t tiles, int tpw,
                                                                   uint32_t *__restrict__ counts,
                                                                   uint32_t *__restrict__ mask) {
    constexpr int kItems = SortTile<T>::kItems;
    constexpr int64_t kTile = SortTile<T>::kTile;
    constexpr int kDig = 1 << BITS;
    static_assert(!MASK || sizeof(T) == 4, "top bytes of 32-bit keys");
    __shared__ uint32_t cnt[kCountTiles][kDig + 1];  // (padded: the final transpose reads a column)
    __shared__ uint8_t rank[REMAP ? 256 : 1];
    __shared__ uint8_t present[MASK ? 256 : 1];  // MASK: top bytes seen
    const int tid = threadIdx.x;
    for (int i = tid; i < kCountTiles * (kDig + 1); i += kSortThreads) (&cnt[0][0])[i] = 0;
    if (MASK && tid < 256) present[tid] = 0;
    if constexpr (REMAP) build_rank<BITS>(mask, rank);  // (its barrier also orders the clearing)
    else __syncthreads();
    const int lane = tid & (kWave - 1);
    const int64_t tb = (int64_t)blockIdx.x * tpw;
    uint32_t last = 256u;  // MASK: the top byte this thread noted last
    for (int k = 0; k < tpw && tb + k < tiles; ++k) {
        const int64_t t0 = (tb + k) * kTile;
        T r[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = t0 + (int64_t)j * kSortThreads + tid;
            r[j] = i < n ? rec[i] : T(0);
        }
        // AGG (a top digit: sign and exponent, a handful of values): same-digit
        // lanes would serialize on one LDS address, so up to four rounds take the
        // digit of the lowest lane not yet counted and add all its lanes through
        // that lane; what is left (many distinct digits) adds per lane.  On the
        // low digits per-lane adds are cheaper.  MASK: a thread stores a
        // presence byte only when its key's top byte differs from the last one
        // it noted (neighbouring voxels share their top bytes).
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = t0 + (int64_t)j * kSortThreads + tid;
            const bool ok = i < n;
            const uint32_t d = digit_of<T, BITS, REMAP>(r[j], shift, rank);
            if constexpr (MASK) {
                const uint32_t top = (uint32_t)r[j] >> 24;
                if (ok && top != last) {
                    present[top] = 1;
                    last = top;
                }
            }
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
    if (MASK && tid < 256) {  // wave w: bytes 64 w .. 64 w + 63, mask words 2 w and 2 w + 1
        const uint64_t b = __builtin_amdgcn_ballot_w64(present[tid] != 0);
        if (lane == 0 && (uint32_t)b != 0u) atomicOr(&mask[2 * (tid >> 6)], (uint32_t)b);
        if (lane == 0 && (uint32_t)(b >> 32) != 0u) atomicOr(&mask[2 * (tid >> 6) + 1], (uint32_t)(b >> 32));
    }
    for (int i = tid; i < tpw * kDig; i += kSortThreads) {
        const int k = i % tpw, d = i / tpw;
        if (tb + k < tiles) counts[(int64_t)d * tiles + tb + k] = cnt[k][d];
    }
}

// The presence mask, copied to host-mapped memory (read by the host after an
// event, to choose the remaining passes).
__global__ void mask_publish_kernel(const uint32_t *__restrict__ mask, uint32_t *host) {
    if (threadIdx.x < 8) host[threadIdx.x] = mask[threadIdx.x];
}

template <typename T, int BITS, bool REMAP>
__global__ void __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(8))) radix_scatter_kernel(const T *__restrict__ in, int64_t n,
                                                                     int shift, int64_t tiles,
                                                                     const uint32_t *__restrict__ offsets,
                                                                     const uint32_t *__restrict__ mask,
                                                                     T *__restrict__ out) {
    constexpr int kItems = SortTile<T>::kItems;
    constexpr int64_t kTile = SortTile<T>::kTile;
    constexpr int kChunk = kItems * kWave;       // keys of one wave, consecutive
    constexpr int kDig = 1 << BITS;
    constexpr int kPer = kDig / kWave;           // digits per lane in the scan of the totals
    static_assert(BITS >= 1 && BITS <= 10, "digits of at most 10 bits (LDS rows of 1024 counts per wave)");
    static_assert(kDig <= kSortThreads, "one thread per digit");
    __shared__ T buf[kTile];                     // the tile reordered by digit
    // per wave: digit counts, then the wave's offset per digit (16-bit: a
    // tile holds at most 8192 keys; pairs of digits read as one word)
    __shared__ __attribute__((aligned(16))) uint16_t wcnt[kSortWaves][kDig];
    __shared__ uint32_t start[kDig];             // digit totals, then the first slot of each digit
    __shared__ uint32_t dest[kDig];              // per digit: output position minus first slot
    __shared__ uint8_t rank_t[REMAP ? 256 : 1];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    // neighbouring tiles on one XCD: they read neighbouring words of the
    // offset table and write neighbouring ends of each digit's runs
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t0 = (int64_t)tile * kTile;
    // the tile's output position per digit, loaded while the tile is ranked
    const uint32_t gpos = tid < kDig ? offsets[(int64_t)tid * tiles + tile] : 0u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) wcnt[wave][lane * kPer + q] = 0;  // the wave's own row
    if constexpr (REMAP) build_rank<BITS>(mask, rank_t);

    // wave w ranks keys t0 + w*kChunk + j*64 + lane (j = 0..kItems-1), in
    // that order: tile order, so the ranking is stable
    T r[kItems];
    uint32_t rank[kItems];
    const int64_t wb = t0 + (int64_t)wave * kChunk;
    // (a full tile, every tile but the last: loads and stores without bounds
    // checks; in the last tile the keys past the end are all ones, whose
    // digit is the largest (for REMAP through the rank of byte 255), so that
    // they rank last in the tile and are never written)
    const bool full = t0 + kTile <= n;
    if (full) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) r[j] = in[wb + j * kWave + lane];
    } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = wb + (int64_t)j * kWave + lane;
            r[j] = i < n ? in[i] : ~T(0);
        }
    }
    auto digit = [&](int j) -> uint32_t { return digit_of<T, BITS, REMAP>(r[j], shift, rank_t); };
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t d = digit(j);
        // peers: the lanes whose digit equals this lane's, as two 32-bit
        // halves: the complement of the lanes that disagree with this lane on
        // some bit.  Per bit, sb is all ones where the bit is set (kept
        // opaque, so that the ballot compares it instead of recomputing the
        // bit) and m the ballot of the lanes with the bit set; per half,
        // x = (m0 ^ sb0) | (m1 ^ sb1) | ... with one three-input op per bit
        // after the first (x | (m ^ sb): truth table 0xF6 over (x, m, sb)).
        uint32_t sb[BITS];
        uint64_t m[BITS];
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            sb[b] = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
            asm("" : "+v"(sb[b]));
            m[b] = __builtin_amdgcn_ballot_w64(sb[b] != 0);
        }
        uint32_t xlo = (uint32_t)m[0] ^ sb[0], xhi = (uint32_t)(m[0] >> 32) ^ sb[0];
#pragma unroll
        for (int b = 1; b < BITS; ++b) {
            xlo = __builtin_amdgcn_bitop3_b32(xlo, (uint32_t)m[b], sb[b], 0xf6);
            xhi = __builtin_amdgcn_bitop3_b32(xhi, (uint32_t)(m[b] >> 32), sb[b], 0xf6);
        }
        const uint32_t plo = ~xlo, phi = ~xhi;
        const uint32_t rw = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));  // peers below
        // the wave's own count row: LDS operations of one wave take effect in order
        const uint32_t base = wcnt[wave][d];
        rank[j] = base + rw;
        if (rw == 0) wcnt[wave][d] = (uint16_t)(base + __builtin_popcount(plo) + __builtin_popcount(phi));
    }
    __syncthreads();
    if (tid < kDig / 2) {  // per pair of digits: the waves' offsets and the digits' totals
        // two 16-bit counts per word, added as one: a digit's total over
        // the tile is at most 8192, so the low half never carries
        uint32_t acc = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            uint32_t *cw = reinterpret_cast<uint32_t *>(&wcnt[w][0]) + tid;
            const uint32_t c = *cw;
            *cw = acc;
            acc += c;
        }
        start[2 * tid] = acc & 0xFFFFu;
        start[2 * tid + 1] = acc >> 16;
    }
    __syncthreads();
    // first slot of each digit: exclusive scan of the totals (one wave, kPer
    // digits per lane)
    if (tid < kWave) {
        uint32_t v[kPer], s = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            v[q] = start[tid * kPer + q];
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
        for (int q = 0; q < kPer; ++q) {
            start[tid * kPer + q] = p;
            p += v[q];
        }
    }
    __syncthreads();
    if (tid < kDig) dest[tid] = gpos - start[tid];  // (mod 2^32: positions are below 2^32)
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t d = digit(j);
        buf[start[d] + wcnt[wave][d] + rank[j]] = r[j];
    }
    __syncthreads();
    if (full) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int s = j * kSortThreads + tid;
            const T v = buf[s];
            out[dest[digit_of<T, BITS, REMAP>(v, shift, rank_t)] + (uint32_t)s] = v;
        }
        return;
    }
    const int64_t valid = n - t0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int s = j * kSortThreads + tid;
        if (s < valid) {
            const T v = buf[s];
            const uint32_t d = digit_of<T, BITS, REMAP>(v, shift, rank_t);
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
int64_t radix_count_entries(int64_t n, int elem) { return (elem == 4 ? 1024 : 256) * radix_tiles(n, elem); }

// One pass: counts, their scan, the scatter from v[*cur] to the other buffer.
template <typename T, int BITS, bool AGG, bool REMAP, bool MASK>
static int radix_pass(T *v[2], int *cur, int64_t n, int shift, uint32_t *counts, uint32_t *sums, uint32_t *mask,
                      hipStream_t stream) {
    const int64_t tiles = radix_tiles(n, (int)sizeof(T));
    const int tpw = (int)std::min<int64_t>(kCountTiles, std::max<int64_t>(1, tiles / 2048));
    const unsigned cgrid = (unsigned)((tiles + tpw - 1) / tpw);
    hipLaunchKernelGGL((radix_count_kernel<T, BITS, AGG, REMAP, MASK>), dim3(cgrid), dim3(kSortThreads), 0, stream,
                       (const T *)v[*cur], n, shift, tiles, tpw, counts, mask);
    ECC_HIP(hipGetLastError());
    int rc = exclusive_scan_u32(counts, ((int64_t)1 << BITS) * tiles, sums, stream);
    if (rc) return rc;
    hipLaunchKernelGGL((radix_scatter_kernel<T, BITS, REMAP>), dim3((unsigned)tiles), dim3(kSortThreads), 0, stream,
                       (const T *)v[*cur], n, shift, tiles, (const uint32_t *)counts, (const uint32_t *)mask,
                       v[*cur ^ 1]);
    ECC_HIP(hipGetLastError());
    *cur ^= 1;
    return ECC_OK;
}

static int check_count(int64_t n) {
    if (n > (int64_t)UINT32_MAX) {
        set_error("radix sort: too many keys");
        return ECC_E_UNSUPPORTED;
    }
    return ECC_OK;
}

int radix_sort_keys(uint32_t *key[2], int64_t n, uint32_t *counts, uint32_t *sums, uint32_t *mask_dev,
                    volatile uint32_t *mask_host, uint32_t *mask_host_dev, hipStream_t stream) {
    if (n <= 1) return ECC_OK;
    int rc = check_count(n);
    if (rc) return rc;
    int cur = 0;
    // pass 1 notes the top bytes; the host reads them while passes 1 and 2 run
    rc = launch_zero(mask_dev, 32, stream);
    if (rc) return rc;
    const int64_t tiles = radix_tiles(n, 4);
    const int tpw = (int)std::min<int64_t>(kCountTiles, std::max<int64_t>(1, tiles / 2048));
    hipLaunchKernelGGL((radix_count_kernel<uint32_t, 9, false, false, true>), dim3((unsigned)((tiles + tpw - 1) / tpw)),
                       dim3(kSortThreads), 0, stream, (const uint32_t *)key[0], n, 0, tiles, tpw, counts, mask_dev);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(mask_publish_kernel, dim3(1), dim3(64), 0, stream, (const uint32_t *)mask_dev, mask_host_dev);
    ECC_HIP(hipGetLastError());
    hipEvent_t noted = nullptr;
    ECC_HIP(hipEventCreateWithFlags(&noted, hipEventDisableTiming));
    hipError_t e = hipEventRecord(noted, stream);
    if (e == hipSuccess) {
        rc = exclusive_scan_u32(counts, 512 * tiles, sums, stream);
        if (!rc) {
            hipLaunchKernelGGL((radix_scatter_kernel<uint32_t, 9, false>), dim3((unsigned)tiles), dim3(kSortThreads), 0,
                               stream, (const uint32_t *)key[0], n, 0, tiles, (const uint32_t *)counts,
                               (const uint32_t *)mask_dev, key[1]);
            e = hipGetLastError();
            cur = 1;
        }
        if (!rc && e == hipSuccess) rc = radix_pass<uint32_t, 9, false, false, false>(key, &cur, n, 9, counts, sums, mask_dev, stream);
        const hipError_t w = hipEventSynchronize(noted);
        if (e == hipSuccess) e = w;
    }
    (void)hipEventDestroy(noted);
    ECC_HIP(e);
    if (rc) return rc;
    int present = 0;
    for (int w = 0; w < 8; ++w) present += __builtin_popcount(mask_host[w]);
    if (present <= 8) {  // ranks in 3 bits: a 9-bit digit
        rc = radix_pass<uint32_t, 9, false, true, false>(key, &cur, n, kRemapShift, counts, sums, mask_dev, stream);
    } else if (present <= 16) {  // ranks in 4 bits: a 10-bit digit
        rc = radix_pass<uint32_t, 10, false, true, false>(key, &cur, n, kRemapShift, counts, sums, mask_dev, stream);
    } else {  // bits 18-24 and 25-31 (sign and high exponent bits: a handful of values)
        rc = radix_pass<uint32_t, 7, false, false, false>(key, &cur, n, 18, counts, sums, mask_dev, stream);
        if (!rc) rc = radix_pass<uint32_t, 7, true, false, false>(key, &cur, n, 25, counts, sums, mask_dev, stream);
    }
    if (rc) return rc;
    if (cur == 1) std::swap(key[0], key[1]);
    return ECC_OK;
}

// Four passes of 8-bit digits on the key half.
int radix_sort_records(uint64_t *rec[2], int64_t n, uint32_t *counts, uint32_t *sums, hipStream_t stream) {
    if (n <= 1) return ECC_OK;
    int rc = check_count(n);
    int cur = 0;
    for (int pass = 0; pass < 4 && !rc; ++pass) {
        if (pass == 3)
            rc = radix_pass<uint64_t, 8, true, false, false>(rec, &cur, n, 32 + 8 * pass, counts, sums, nullptr, stream);
        else
            rc = radix_pass<uint64_t, 8, false, false, false>(rec, &cur, n, 32 + 8 * pass, counts, sums, nullptr, stream);
    }
    return rc;
}

}  // namespace ecc
