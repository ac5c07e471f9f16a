// Float32 images (Sec. 3, "Other Ranges of Gray Values"): the values are not known
// in advance, so every voxel emits a record (key, change) and the records
// are sorted by key, summed per distinct key and prefix-summed.
//
// The change of a voxel v is the signed count of the cells of the cubical
// complex that v introduces (Sec. 3, Algorithm 1: a cell enters with the
// first of its incident voxels in the order "smaller value first, ties broken
// by position").  A cell of the closed voxel v is named by a direction
// s in {-1,0,1}^D (s_i = 0: the cell spans v along axis i; s_i = +-1: it is
// the face on that side); it has dimension #{i : s_i = 0}.  Its other
// incident voxels are v + delta with delta_i in {0, s_i}, delta != 0, so v
// introduces it iff none of those precedes v.  With U_s = OR of "precedes"
// over that box, U_s = prec(s) | OR_{i : s_i != 0} U_{s with s_i = 0}, and
//     change(v) = sum_s (-1)^dim(s) [U_s = 0] = 1 - sum_{s != 0} (-1)^dim(s) U_s
// (the first sum over all s is prod_i (2 - 1) = 1).
//
// On the GPU a wave holds 64 consecutive voxels of one line of the last axis
// (their neighbourhoods staged in LDS by the workgroup);
// "precedes" for each of the 3^D - 1 neighbour directions is one ballot, the
// recursion for U_s runs on those wave-wide masks in scalar registers, and
// each U_s is accumulated per lane with one add-with-carry.
//
// Keys: the canonical float (-0 folded into +0) mapped to an unsigned integer
// with the same order (sign bit set: all bits flipped; else the sign bit set).
// A record is one 64-bit word: key in bits 8..39, change (int8) in bits 0..7.

#include "ecc_internal.h"

namespace ecc {

__device__ __forceinline__ uint32_t f32_key(uint32_t u) {
    if ((u & 0x7FFFFFFFu) == 0u) u = 0u;  // -0 -> +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_to_f32(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

constexpr int pow3(int d) { return d == 0 ? 1 : 3 * pow3(d - 1); }
// base-3 digit k of a direction code: 0 -> -1, 1 -> 0, 2 -> +1
constexpr int digit3(int t, int k) { return (t / pow3(k)) % 3; }
template <int D>
constexpr int nonzeros(int t) {
    int c = 0;
    for (int k = 0; k < D; ++k) c += digit3(t, k) != 1;
    return c;
}
// delta earlier than v in C order: its first non-zero component (axis 0 is
// the most significant, digit D-1-k holds axis k) is negative
template <int D>
constexpr bool earlier(int t) {
    for (int a = 0; a < D; ++a) {
        const int dg = digit3(t, D - 1 - a);
        if (dg != 1) return dg == 0;
    }
    return false;
}

__device__ __forceinline__ uint64_t ballot64(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// Visiting order of the 81 directions in 4-D (digit value 1 = zero offset):
// blocks (digit 3, digit 2) in the order (1,1) (2,1) (1,2) (2,2) (1,0) (2,0)
// (0,1) (0,2) (0,0), each block's nine (digit 0, digit 1) pairs by
// increasing non-zeros.  A block depends on itself and on the blocks with one
// or both outer digits set to 1, all visited before it.
struct Order4 {
    int t[81];
    constexpr Order4() : t{} {
        const int ba[9] = {1, 2, 1, 2, 1, 2, 0, 0, 0}, bb[9] = {1, 1, 2, 2, 0, 0, 1, 2, 0};
        const int w0[9] = {1, 0, 2, 1, 1, 0, 2, 0, 2}, w1[9] = {1, 1, 1, 0, 2, 0, 0, 2, 2};
        for (int k = 0; k < 81; ++k) t[k] = w0[k % 9] + 3 * w1[k % 9] + 9 * bb[k / 9] + 27 * ba[k / 9];
    }
};
constexpr Order4 kOrder4{};

// acc += lane bit of m  /  acc -= lane bit of m  (one VALU op each: the mask is
// the carry-in; the carry-out goes to a scratch scalar pair)
__device__ __forceinline__ void add_bit(int32_t &acc, uint64_t m) {
    uint64_t co;
    asm("v_addc_co_u32_e64 %0, %1, %0, 0, %2" : "+v"(acc), "=&s"(co) : "s"(m));
}
__device__ __forceinline__ void sub_bit(int32_t &acc, uint64_t m) {
    uint64_t co;
    asm("v_subb_co_u32_e64 %0, %1, %0, 0, %2" : "+v"(acc), "=&s"(co) : "s"(m));
}

struct FloatView {
    int32_t n[4];       // extents, axis 0 slowest, padded in front with 1
    uint32_t stride[4]; // element strides
    int32_t bpr;        // blocks per line of the last axis
    int32_t run;        // lines along axis 2 walked by one workgroup
    int32_t nruns;      // runs per axis-2 extent
};

// One thread per voxel.  D = number of axes after dropping axes of extent 1
// (the complex of the others times unit intervals has the same curve).
//
// A workgroup of T threads takes T consecutive voxels (x in [xs, xs+T)) of a
// run of consecutive lines along axis 2 of the padded view and walks the run
// line by line.  The values of the 3^D neighbourhood come from LDS: a ring of
// four slots, one per line position along axis 2, each holding the
// S = 3^(D-2) lines at offsets -1, 0, +1 along the axes before it, over
// x in [xs-1, xs+T].  While line y is compared, the loads for line y+2 are in
// flight; each line is loaded once per workgroup (one coalesced load per
// thread and line, plus one load for the two ends of all S lines), instead of
// 3^D - 1 scattered loads per voxel.  Absent neighbours (outside the image)
// are stored as NaN, which compares false and so never precedes.
template <int D, int T>
__global__ void __launch_bounds__(T) float_change_kernel(const float *__restrict__ img, uint32_t img_bytes,
                                                         FloatView v, uint64_t *__restrict__ rec,
                                                         uint32_t *status) {
    constexpr int P = pow3(D);
    constexpr int C = (P - 1) / 2;             // code of the zero direction
    constexpr int S = D >= 2 ? pow3(D - 2) : 1;  // lines per slot
    constexpr int PITCH = T + 2;
    __shared__ float ring[4 * S * PITCH];
    const int32_t nx = v.n[3], n2 = v.n[2];
    const int tid = (int)threadIdx.x;
    // block -> (outer line over axes 0..1, run along axis 2, x block); uniform
    int32_t r = __builtin_amdgcn_readfirstlane((int32_t)blockIdx.x);
    const int32_t xs = (r % v.bpr) * T;
    r /= v.bpr;
    const int32_t y0 = (r % v.nruns) * v.run;
    const int32_t y1 = min(y0 + v.run, n2);
    r /= v.nruns;
    const int32_t c1 = r % v.n[1];
    const int32_t c0 = r / v.n[1];
    const int32_t x = xs + tid;
    const bool act = x < nx;
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)img, (short)0, (int)img_bytes, 0x00020000);
    const float nan = __uint_as_float(0x7FC00000u);

    // slot line j: offsets (digit 0 of j -> axis 1, digit 1 -> axis 0).  Per
    // workgroup: its element offset at axis-2 position 0 (32-bit: images
    // hold fewer than 2^30 elements) and whether it exists (bit j of lmask).
    uint32_t lb0[S];
    uint32_t lmask = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int32_t a1 = c1 + (D >= 3 ? (j % 3) - 1 : 0);
        const int32_t a0 = c0 + (D >= 4 ? (j / 3) % 3 - 1 : 0);
        lb0[j] = (uint32_t)a0 * v.stride[0] + (uint32_t)a1 * v.stride[1];
        if (a1 >= 0 && a1 < v.n[1] && a0 >= 0 && a0 < v.n[0]) lmask |= 1u << j;
    }
    // the end values x = xs-1 (even lanes) and xs+T (odd lanes) of line
    // (tid >> 1), lanes 0 .. 2S-1
    const int ej = tid >> 1;
    const int32_t xe = (tid & 1) ? xs + T : xs - 1;
    uint32_t elb0 = 0;
#pragma unroll
    for (int j = 0; j < S; ++j)
        if (j == ej) elb0 = lb0[j];
    const bool eok = tid < 2 * S && ((lmask >> (ej < S ? ej : 0)) & 1u) && xe >= 0 && xe < nx;
    // Every load is issued, branch-free: offsets of absent lines or of lanes
    // past the line's end may point anywhere (wrapped 32-bit arithmetic), but a
    // raw buffer load is bounds-checked against the image (past the end it
    // returns 0 and touches nothing), and such values are replaced by NaN.
    auto fetch = [&](int32_t y, float (&val)[S], float &end) {
        const bool yok = y >= 0 && y < n2;
        const uint32_t ys = (uint32_t)y * v.stride[2];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const float w = __uint_as_float(
                __builtin_amdgcn_raw_buffer_load_b32(rs, (lb0[j] + ys + (uint32_t)x) * 4u, 0, 0));
            val[j] = (yok && ((lmask >> j) & 1u) && act) ? w : nan;
        }
        const float we = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (elb0 + ys + (uint32_t)xe) * 4u, 0, 0));
        end = (yok && eok) ? we : nan;
    };
    // element index of this thread's voxel in line (S / 2) at position y
    auto own_index = [&](int32_t y) -> uint32_t { return lb0[S / 2] + (uint32_t)y * v.stride[2] + (uint32_t)x; };
    auto store = [&](int32_t y, const float (&val)[S], float end) {
        float *slot = ring + (y & 3) * (S * PITCH);
#pragma unroll
        for (int j = 0; j < S; ++j) slot[j * PITCH + 1 + tid] = val[j];
        if (tid < 2 * S) slot[ej * PITCH + ((tid & 1) ? T + 1 : 0)] = end;
    };

    float val[S], end;
    for (int32_t y = y0 - 1; y <= y0 + 1; ++y) {
        fetch(y, val, end);
        store(y, val, end);
    }
    for (int32_t y = y0; y < y1; ++y) {
        __syncthreads();  // slots y-1 .. y+1 written; slot y+2 (= y-2) no longer read
        const bool next = y + 1 < y1;
        if (next) fetch(y + 2, val, end);
        // this voxel's column in the three slots around y
        const float *col[3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) col[dy] = ring + ((y - 1 + dy) & 3) * (S * PITCH) + 1 + tid;
        const float f0 = col[1][(S / 2) * PITCH];
        const uint32_t own_bits = __float_as_uint(f0);
        const uint32_t k0 = f32_key(own_bits);

        // "Neighbour t precedes v" is computed where the recursion first needs
        // it (level by level), so that only the U masks of two adjacent levels
        // are live in scalar registers, not all 3^D - 1 comparison masks too.
        auto prec = [&](int t) -> uint64_t {
            const int dx = digit3(t, 0) - 1;
            const int dyi = D >= 2 ? digit3(t, 1) : 1;
            const int j = D >= 3 ? t / 9 : 0;
            // IEEE comparisons: -0 == +0, infinities are ordinary values, NaN
            // (an absent neighbour) never precedes; a NaN in the image fails the call
            const float fn = col[dyi][j * PITCH + dx];
            const bool p = earlier<D>(t) ? (fn <= f0) : (fn < f0);
            return ballot64(p);
        };
        // U_s, each after the U it depends on, then the signed sum
        uint64_t U[P];
        U[C] = 0;  // the zero direction: empty box
        int32_t acc = 0;
        auto visit = [&](int t) {
            uint64_t u = prec(t);
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (digit3(t, j) != 1) u |= U[t + (1 - digit3(t, j)) * pow3(j)];
            U[t] = u;
            // (-1)^dim, dim = D - (non-zero components): subtract for even dim
            if (((D - nonzeros<D>(t)) & 1) == 0) add_bit(acc, u);
            else sub_bit(acc, u);
        };
        if constexpr (D == 4) {
            // blocks of nine by the two outer digits, in an order that lets
            // each block's masks die early (at most five blocks live)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int t = kOrder4.t[k];
                if (t != C) visit(t);
                // keep the scheduler from hoisting later blocks' compares
                // (their masks would all be live at once and spill)
                if (k % 9 == 8) __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            // increasing numbers of non-zero components
#pragma unroll
            for (int lvl = 1; lvl <= D; ++lvl)
#pragma unroll
                for (int t = 0; t < P; ++t)
                    if (nonzeros<D>(t) == lvl) visit(t);
        }
        if (ballot64(act && (own_bits & 0x7FFFFFFFu) > 0x7F800000u) != 0 && (threadIdx.x & (kWave - 1)) == 0)
            atomicOr(status, kStatusNaN);
        if (act) rec[own_index(y)] = ((uint64_t)k0 << 8) | (uint8_t)(int8_t)(1 - acc);
        if (next) store(y + 2, val, end);
    }
}

int launch_float_change(const float *img_dev, const ecc_dims *dims, uint64_t *rec, uint32_t *status,
                        hipStream_t stream) {
    // drop axes of extent 1, pad in front to four axes
    int32_t ext[4];
    int d = 0;
    int64_t total = 1;
    for (int i = 0; i < dims->ndim; ++i) {
        total *= dims->n[i];
        if (dims->n[i] > 1) ext[d++] = (int32_t)dims->n[i];
    }
    if (total * 4 > (int64_t)UINT32_MAX) {
        set_error("float images are limited to 2^30 elements in this build");
        return ECC_E_UNSUPPORTED;
    }
    FloatView v{};
    const int D = d == 0 ? 1 : d;
    if (d == 0) ext[d++] = 1;
    for (int k = 0; k < 4; ++k) v.n[k] = 1;
    for (int i = 0; i < D; ++i) v.n[4 - D + i] = ext[i];
    uint32_t s = 1;
    for (int k = 3; k >= 0; --k) {
        v.stride[k] = s;
        s *= (uint32_t)v.n[k];
    }
    const int nx = v.n[3];
    const int threads = nx >= 256 ? 256 : ((nx + 63) / 64) * 64;
    v.bpr = (nx + threads - 1) / threads;
    v.run = v.n[2] < 32 ? v.n[2] : 32;
    v.nruns = (v.n[2] + v.run - 1) / v.run;
    const int64_t grid = (int64_t)v.n[0] * v.n[1] * v.nruns * v.bpr;
    if (grid > INT32_MAX) {
        set_error("float image: too many lines");
        return ECC_E_UNSUPPORTED;
    }
    const uint32_t bytes = (uint32_t)(total * 4);
    void *tok = nullptr;
    int rc = profile_begin(stream, &tok);
    if (rc) return rc;
    const dim3 g((unsigned)grid), b(threads);
#define ECC_FCK(DD)                                                                                              \
    switch (threads) {                                                                                           \
    case 64: hipLaunchKernelGGL((float_change_kernel<DD, 64>), g, b, 0, stream, img_dev, bytes, v, rec, status); break;   \
    case 128: hipLaunchKernelGGL((float_change_kernel<DD, 128>), g, b, 0, stream, img_dev, bytes, v, rec, status); break; \
    case 192: hipLaunchKernelGGL((float_change_kernel<DD, 192>), g, b, 0, stream, img_dev, bytes, v, rec, status); break; \
    default: hipLaunchKernelGGL((float_change_kernel<DD, 256>), g, b, 0, stream, img_dev, bytes, v, rec, status); break;  \
    }
    switch (D) {
    case 1: ECC_FCK(1); break;
    case 2: ECC_FCK(2); break;
    case 3: ECC_FCK(3); break;
    default: ECC_FCK(4); break;
    }
#undef ECC_FCK
    ECC_HIP(hipGetLastError());
    return profile_end(stream, tok);
}

// ----------------------------------------------------------------------------
// After sorting: chi after each distinct key = running sum of the changes up
// to and including the last record with that key.  Records are taken in tiles
// of kFTile; pass 1 sums each tile (changes, and the number of last-of-key
// positions), pass 2 scans the tile sums in one workgroup, pass 3 writes
// (key, chi) at the rank of each last-of-key position.

constexpr int kFThreads = 256;
constexpr int kFItems = 16;
constexpr int kFTile = kFThreads * kFItems;

__device__ __forceinline__ uint32_t rec_key(uint64_t r) { return (uint32_t)(r >> 8); }
__device__ __forceinline__ int32_t rec_chg(uint64_t r) { return (int32_t)(int8_t)(uint8_t)(r & 0xFFu); }
__device__ __forceinline__ bool last_of_key(const uint64_t *rec, int64_t i, int64_t n) {
    return i == n - 1 || rec_key(rec[i]) != rec_key(rec[i + 1]);
}

template <typename T>
__device__ T block_sum(T v, T *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    T t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;
}

__global__ void __launch_bounds__(kFThreads) fsum_tiles_kernel(const uint64_t *__restrict__ rec, int64_t n,
                                                              int64_t *__restrict__ tile_chg,
                                                              int64_t *__restrict__ tile_last) {
    __shared__ int64_t sh[4];
    const int64_t t0 = (int64_t)blockIdx.x * kFTile;
    int64_t s = 0, l = 0;
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        const int64_t i = t0 + (int64_t)j * kFThreads + threadIdx.x;
        if (i < n) {
            s += rec_chg(rec[i]);
            l += last_of_key(rec, i, n);
        }
    }
    s = block_sum(s, sh);
    l = block_sum(l, sh);
    if (threadIdx.x == 0) {
        tile_chg[blockIdx.x] = s;
        tile_last[blockIdx.x] = l;
    }
}

// Exclusive scan in place of two int64 arrays of length nt by one workgroup;
// total_last receives the sum of the second (the number of distinct keys).
// Exclusive scans of both tile arrays in one workgroup of 1024 threads, in
// chunks of 16384 tiles: thread t holds tiles c0 + k * 1024 + t (k < 16:
// sixteen rows, every load and store coalesced).  Each row is scanned
// across the wave with shuffles; the wave totals per row go to LDS, where
// 32 threads turn them into per-wave prefixes and row totals.  The running
// carries are the same in all threads.  (With runs of consecutive tiles per
// thread one CU's address unit, fed 64 cache lines per load, was the limit:
// 0.14 ms for 2^16 tiles, 0.16 ms with one tile per thread.)
__global__ void __launch_bounds__(1024) fscan_tiles_kernel(int64_t *a, int64_t *b, int64_t nt, int64_t *total_last) {
    __shared__ int64_t wsa[16][17], wsb[16][17];  // [row][wave]
    __shared__ int64_t tota[16], totb[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t ca = 0, cb = 0;
    for (int64_t c0 = 0; c0 < nt; c0 += 1024 * 16) {
        int64_t xa[16], xb[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t i = c0 + k * 1024 + tid;
            xa[k] = i < nt ? a[i] : 0;
            xb[k] = i < nt ? b[i] : 0;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int64_t ua = __shfl_up(xa[k], off, 64), ub = __shfl_up(xb[k], off, 64);
                if (lane >= off) {
                    xa[k] += ua;
                    xb[k] += ub;
                }
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                wsa[k][wave] = xa[k];
                wsb[k][wave] = xb[k];
            }
        }
        __syncthreads();
        if (tid < 32) {  // row tid & 15 of array tid >> 4: exclusive prefix over the waves, row total
            int64_t(*ws)[17] = tid < 16 ? wsa : wsb;
            const int k = tid & 15;
            int64_t run = 0;
            for (int w = 0; w < 16; ++w) {
                const int64_t x = ws[k][w];
                ws[k][w] = run;
                run += x;
            }
            (tid < 16 ? tota : totb)[k] = run;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            // exclusive within the wave: the inclusive value of the lane below
            const int64_t pa = __shfl_up(xa[k], 1, 64), pb = __shfl_up(xb[k], 1, 64);
            const int64_t i = c0 + k * 1024 + tid;
            if (i < nt) {
                a[i] = ca + wsa[k][wave] + (lane > 0 ? pa : 0);
                b[i] = cb + wsb[k][wave] + (lane > 0 ? pb : 0);
            }
            ca += tota[k];
            cb += totb[k];
        }
        __syncthreads();  // the LDS rows are rewritten by the next chunk
    }
    if (tid == 0) *total_last = cb;
}

// The curve write walks the same tiles with twice the threads (8 records
// each): its LDS tile allows four workgroups per CU, so 512 threads keep 32
// waves per CU in flight instead of 16.
constexpr int kWThreads = 512;
constexpr int kWItems = kFTile / kWThreads;
constexpr int kWWaves = kWThreads / 64;
static_assert(kWItems * kWThreads == kFTile && kWThreads % 64 == 0, "curve write: whole tiles of whole waves");
__global__ void __launch_bounds__(kWThreads) fwrite_kernel(const uint64_t *__restrict__ rec, int64_t n,
                                                          const int64_t *__restrict__ tile_chg,
                                                          const int64_t *__restrict__ tile_last,
                                                          float *__restrict__ out_keys, int64_t *__restrict__ out_chi) {
    __shared__ int64_t wc[kWWaves], wl[kWWaves];
    // the tile and the record after it, loaded coalesced; slot i at i + i / 16
    // (fewer bank conflicts when threads read runs of consecutive records)
    __shared__ uint64_t tile[kFTile + kFTile / 16 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kFTile;
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
        const int q = j * kWThreads + tid;
        const int64_t i = t0 + q;
        tile[q + q / 16] = i < n ? rec[i] : 0ull;
    }
    if (tid == 0) {
        const int64_t i = t0 + kFTile;
        tile[kFTile + kFTile / 16] = i < n ? rec[i] : 0ull;
    }
    __syncthreads();
    // each thread takes kWItems consecutive records of the tile
    const int64_t i0 = t0 + (int64_t)tid * kWItems;
    uint64_t r[kWItems + 1];
#pragma unroll
    for (int j = 0; j <= kWItems; ++j) {
        const int q = tid * kWItems + j;
        r[j] = tile[q + q / 16];
    }
    int64_t c[kWItems];
    bool last[kWItems];
    int64_t sc = 0, sl = 0;
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
        const int64_t i = i0 + j;
        const bool in = i < n;
        sc += in ? rec_chg(r[j]) : 0;
        c[j] = sc;
        last[j] = in && (i == n - 1 || rec_key(r[j]) != rec_key(r[j + 1]));
        sl += last[j];
    }
    int64_t xc = sc, xl = sl;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t uc = __shfl_up(xc, off, 64), ul = __shfl_up(xl, off, 64);
        if (lane >= off) {
            xc += uc;
            xl += ul;
        }
    }
    if (lane == 63) {
        wc[wave] = xc;
        wl[wave] = xl;
    }
    __syncthreads();
    int64_t bc = tile_chg[blockIdx.x] + xc - sc, bl = tile_last[blockIdx.x] + xl - sl;
    for (int w = 0; w < wave; ++w) {
        bc += wc[w];
        bl += wl[w];
    }
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
        if (last[j]) {
            out_keys[bl] = key_to_f32(rec_key(r[j]));
            out_chi[bl] = bc + c[j];
            ++bl;
        }
    }
}

int launch_float_curve(const uint64_t *rec, int64_t n, int64_t *tile_chg, int64_t *tile_last,
                       int64_t *total_last, float *out_keys, int64_t *out_chi, hipStream_t stream) {
    const int64_t nt = (n + kFTile - 1) / kFTile;
    if (nt > INT32_MAX) {
        set_error("float curve: too many records");
        return ECC_E_UNSUPPORTED;
    }
    hipLaunchKernelGGL(fsum_tiles_kernel, dim3((unsigned)nt), dim3(kFThreads), 0, stream, rec, n, tile_chg,
                       tile_last);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(fscan_tiles_kernel, dim3(1), dim3(1024), 0, stream, tile_chg, tile_last, nt, total_last);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(fwrite_kernel, dim3((unsigned)nt), dim3(kWThreads), 0, stream, rec, n, tile_chg,
                       tile_last, out_keys, out_chi);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

int64_t float_tiles(int64_t n) { return (n + kFTile - 1) / kFTile; }

// ----------------------------------------------------------------------------
// Change points of a float curve: the keys where chi differs from the
// previous key's (chi = 0 before the first key).

__device__ __forceinline__ uint32_t is_step(const int64_t *chi, int64_t k) {
    return chi[k] != (k > 0 ? chi[k - 1] : 0) ? 1u : 0u;
}

__global__ void __launch_bounds__(256) step_flags_kernel(const int64_t *__restrict__ chi, int64_t K,
                                                         uint32_t *__restrict__ pos) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) pos[k] = is_step(chi, k);
}

__global__ void __launch_bounds__(256) step_scatter_kernel(const float *__restrict__ keys,
                                                           const int64_t *__restrict__ chi,
                                                           const uint32_t *__restrict__ pos, int64_t K,
                                                           float *__restrict__ out_keys,
                                                           int64_t *__restrict__ out_chi, int64_t *count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) {
        const uint32_t f = is_step(chi, k);
        if (f) {
            out_keys[pos[k]] = keys[k];
            out_chi[pos[k]] = chi[k];
        }
        if (k == K - 1) *count = (int64_t)pos[k] + f;
    }
}

// pos: K uint32 (positions, scratch); sums: radix_scan_tiles(K) uint32.
int launch_change_points(const float *keys, const int64_t *chi, int64_t K, uint32_t *pos, uint32_t *sums,
                         float *out_keys, int64_t *out_chi, int64_t *count, hipStream_t stream) {
    if (K <= 0) return ECC_OK;
    int64_t blocks = (K + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(step_flags_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, chi, K, pos);
    ECC_HIP(hipGetLastError());
    int rc = exclusive_scan_u32(pos, K, sums, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(step_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, keys, chi,
                       (const uint32_t *)pos, K, out_keys, out_chi, count);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// ----------------------------------------------------------------------------
// Integer images through the float path (images the integer kernel does not
// take: four axes longer than 1).  Values convert exactly to float32; the
// float curve lists chi after each distinct value, and chi(T_t) for integer
// t is its value at the largest distinct value <= t (0 below the first).

template <typename T>
__global__ void __launch_bounds__(256) int_to_f32_kernel(const T *__restrict__ img, int64_t n, uint32_t limit,
                                                         float *__restrict__ out, uint32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = img[i];
        bad |= v >= limit;
        out[i] = (float)v;
    }
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, kStatusRange);
}

int launch_int_to_f32(const void *img, int elem, int64_t n, uint32_t limit, float *out, uint32_t *status,
                      hipStream_t stream) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (elem == 1)
        hipLaunchKernelGGL(int_to_f32_kernel<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const uint8_t *)img, n, limit, out, status);
    else
        hipLaunchKernelGGL(int_to_f32_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const uint16_t *)img, n, limit, out, status);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

__global__ void __launch_bounds__(256) expand_steps_kernel(const float *__restrict__ keys,
                                                           const int64_t *__restrict__ chi, int64_t K, int m,
                                                           int64_t *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const float ft = (float)t;
    int64_t lo = 0, hi = K;  // first index with keys[idx] > t
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] <= ft) lo = mid + 1;
        else hi = mid;
    }
    out[t] = lo > 0 ? chi[lo - 1] : 0;
}

int launch_expand_steps(const float *keys, const int64_t *chi, int64_t K, int m, int64_t *out,
                        hipStream_t stream) {
    hipLaunchKernelGGL(expand_steps_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, keys, chi, K, m, out);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// ----------------------------------------------------------------------------
// Quantisation of a float image to integer bins: x = (v - lo) * scale in
// float32 (each operation rounded to nearest); bin 0 below x = 0 (and -inf),
// m-1 from x = m on (and +inf), else the integer part of x.  NaN sets the
// status bit and writes bin 0.

template <typename T>
__global__ void __launch_bounds__(256) quantize_kernel(const float *__restrict__ img, int64_t n, float lo,
                                                       float scale, int m, T *__restrict__ out,
                                                       uint32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool nan = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float v = img[i];
        nan |= v != v;
        const float x = __fmul_rn(__fsub_rn(v, lo), scale);
        int q;
        if (!(x >= 0.0f)) q = 0;
        else if (x >= (float)m) q = m - 1;
        else q = (int)x;
        out[i] = (T)q;
    }
    if (__builtin_amdgcn_ballot_w64(nan) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, kStatusNaN);
}

int launch_quantize(const float *img, int64_t n, float lo, float scale, int m, int elem, void *out,
                    uint32_t *status, hipStream_t stream) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (elem == 1)
        hipLaunchKernelGGL(quantize_kernel<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, stream, img, n, lo, scale,
                           m, (uint8_t *)out, status);
    else
        hipLaunchKernelGGL(quantize_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, stream, img, n, lo,
                           scale, m, (uint16_t *)out, status);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

}  // namespace ecc
