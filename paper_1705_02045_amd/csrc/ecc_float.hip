// Float32 images (Sec. 3, "Other Ranges of Gray Values"): the values are not known
// in advance, so every voxel's key is written and the keys are sorted to
// find the distinct values; the voxels whose change is not zero (a few in a
// hundred) are also written, as (key, change) records, and each change is
// added at its key's rank among the distinct values; a prefix sum over the
// distinct values gives the curve.
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

// m = 2 m + (lane bit of mask): one VALU op, the mask is the carry-in (the
// carry-out goes to a scratch scalar pair).
__device__ __forceinline__ void push_bit(uint32_t &m, uint64_t mask) {
    uint64_t co;
    asm("v_addc_co_u32_e64 %0, %1, %0, %0, %2" : "+v"(m), "=&s"(co) : "s"(mask));
}

// Bit layout of the direction masks: word w, bit b holds direction
// t = w * BW + b (BW = 3^min(D, 3) directions per word, NW words).
template <int D>
constexpr int kBW = D >= 3 ? 27 : pow3(D);
template <int D>
constexpr int kNW = D == 4 ? 3 : 1;
// bits of a 27-bit word whose digit k is 1 (no offset along that axis)
constexpr uint32_t mid_mask(int k) {
    uint32_t m = 0;
    for (int b = 0; b < 27; ++b)
        if (digit3(b, k) == 1) m |= 1u << b;
    return m;
}
constexpr uint32_t kMid[3] = {mid_mask(0), mid_mask(1), mid_mask(2)};
// directions whose box enters the sum with sign +1 (PLUS) or -1, zero
// direction excluded
template <int D, bool PLUS>
struct SignMasks {
    uint32_t m[3];
    constexpr SignMasks() : m{} {
        for (int t = 0; t < pow3(D); ++t) {
            if (t == (pow3(D) - 1) / 2) continue;
            const bool even = ((D - nonzeros<D>(t)) & 1) == 0;
            if (even == PLUS) m[t / kBW<D>] |= 1u << (t % kBW<D>);
        }
    }
};
template <int D>
constexpr SignMasks<D, true> kPlus{};
template <int D>
constexpr SignMasks<D, false> kMinus{};

struct FloatView {
    int32_t n[4];       // extents, axis 0 slowest, padded in front with 1
    uint32_t stride[4]; // element strides
    int32_t bpr;        // blocks per line of the last axis
    int32_t run;        // lines along axis 2 walked by one workgroup
    int32_t nruns;      // runs per axis-2 extent
    int32_t e0, e1;     // axis-0 indices whose voxels are emitted (the others are neighbours only)
};

// One thread per voxel.  D = number of axes after dropping axes of extent 1
// (the complex of the others times unit intervals has the same curve).
//
// A workgroup of T threads takes T consecutive voxels (x in [xs, xs+T)) of a
// run of consecutive lines along axis 2 of the padded view and walks the run
// line by line.  The values of the 3^D neighbourhood come from LDS: a ring of
// four slots, one per line position along axis 2, each holding the
// S = 3^(D-2) lines at offsets -1, 0, +1 along the axes before it, over
// x in [xs-1, xs+T], x-major (the S values of one x are adjacent: a thread's
// 3 S neighbours in a slot lie within 12 S bytes of one address, so one
// address per slot serves all its reads).  While line y is compared, the loads for line y+2 are in
// flight; each line is loaded once per workgroup (one coalesced load per
// thread and line, plus one load for the two ends of all S lines), instead of
// 3^D - 1 scattered loads per voxel.  Absent neighbours (outside the image)
// are stored as NaN, which compares false and so never precedes.
// Outputs: keys[i] for every voxel i; for every voxel whose change is not
// zero, one (key, change) record in the workgroup's own region of the record
// arrays (region b = records [b * T * run, (b+1) * T * run), as many slots as
// the workgroup has voxels), at a slot taken from an LDS counter (one LDS
// add per wave and line); nz_cnt[b] and nz_off[b] receive the region's
// record count.
template <int D, int T>
__global__ void __launch_bounds__(T) float_change_kernel(const float *__restrict__ img, uint32_t img_bytes,
                                                         FloatView v, uint32_t *__restrict__ keys,
                                                         uint32_t *__restrict__ nz_key, int32_t *__restrict__ nz_chg,
                                                         uint32_t *__restrict__ nz_cnt, uint32_t *__restrict__ nz_off,
                                                         uint32_t *status) {
    constexpr int P = pow3(D);
    constexpr int C = (P - 1) / 2;             // code of the zero direction
    constexpr int S = D >= 2 ? pow3(D - 2) : 1;  // lines per slot
    constexpr int PITCH = T + 2;
    constexpr int BW = kBW<D>, NW = kNW<D>;
    __shared__ float ring[4 * S * PITCH];
    __shared__ uint32_t region_count;
    const int32_t nx = v.n[3], n2 = v.n[2];
    const int tid = (int)threadIdx.x;
    if (tid == 0) region_count = 0;  // (the first barrier below orders it)
    // block -> (outer line over axes 0..1, run along axis 2, x block); uniform
    const uint32_t blk = blockIdx.x;
    const uint32_t region = blk * (uint32_t)(T * v.run);
    int32_t r = __builtin_amdgcn_readfirstlane((int32_t)blk);
    const int32_t xs = (r % v.bpr) * T;
    r /= v.bpr;
    const int32_t y0 = (r % v.nruns) * v.run;
    const int32_t y1 = min(y0 + v.run, n2);
    r /= v.nruns;
    const int32_t c1 = r % v.n[1];
    const int32_t c0 = r / v.n[1];
    if (c0 < v.e0 || c0 >= v.e1) {  // (uniform) a collar plane of a streamed chunk: nothing to emit
        if (tid == 0) {
            nz_cnt[blk] = 0;
            nz_off[blk] = 0;
        }
        return;
    }
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
        for (int j = 0; j < S; ++j) slot[(1 + tid) * S + j] = val[j];
        if (tid < 2 * S) slot[((tid & 1) ? T + 1 : 0) * S + ej] = end;
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
        for (int dy = 0; dy < 3; ++dy) col[dy] = ring + ((y - 1 + dy) & 3) * (S * PITCH) + (1 + tid) * S;
        const float f0 = col[1][S / 2];
        const uint32_t own_bits = __float_as_uint(f0);
        const uint32_t k0 = f32_key(own_bits);

        // Per lane, bit b of word w says whether neighbour t = w * BW + b
        // precedes v (IEEE comparisons: -0 == +0, infinities are ordinary
        // values, NaN (an absent neighbour) never precedes; a NaN in the image
        // fails the call).  The zero direction's bit is 0.
        uint32_t M[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t m = 0;
#pragma unroll
            for (int b = BW - 1; b >= 0; --b) {
                const int t = w * BW + b;
                if (t == C) {
                    m <<= 1;
                    continue;
                }
                const int dx = digit3(t, 0) - 1;
                const int dyi = D >= 2 ? digit3(t, 1) : 1;
                const int j = D >= 3 ? t / 9 : 0;
                const float fn = col[dyi][dx * S + j];
                push_bit(m, ballot64(earlier<D>(t) ? (fn <= f0) : (fn < f0)));
            }
            M[w] = m;
        }
        // U_t (some vertex of the box spanned by v and v + t, other than v,
        // precedes v): the OR of the bits over the box's directions, taken
        // axis by axis (the box is a product): every digit 0 or 2 receives
        // the bit of the same direction with that digit set to 1 (no offset).
#pragma unroll
        for (int k = 0; k < (D < 3 ? D : 3); ++k) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t mid = M[w] & kMid[k];
                M[w] |= (mid << pow3(k)) | (mid >> pow3(k));
            }
        }
        if constexpr (D == 4) {
            M[0] |= M[1];
            M[2] |= M[1];
        }
        // the signed sum of the boxes that v completes, (-1)^dim each,
        // dim = D - (non-zero components)
        int32_t acc = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            acc += (int32_t)__builtin_popcount(M[w] & kPlus<D>.m[w]) - (int32_t)__builtin_popcount(M[w] & kMinus<D>.m[w]);
        if (ballot64(act && (own_bits & 0x7FFFFFFFu) > 0x7F800000u) != 0 && (threadIdx.x & (kWave - 1)) == 0)
            atomicOr(status, kStatusNaN);
        const int32_t chg = 1 - acc;
        if (act && keys) keys[own_index(y)] = k0;
        const uint64_t nzm = ballot64(act && chg != 0);
        if (nzm != 0) {
            const int lane = (int)(threadIdx.x & (kWave - 1));
            const int leader = __builtin_ctzll(nzm);
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&region_count, (uint32_t)__builtin_popcountll(nzm));
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
            if (act && chg != 0) {
                const uint64_t below = lane == 0 ? 0ull : (nzm & (~0ull >> (64 - lane)));
                const uint32_t slot = region + base + (uint32_t)__builtin_popcountll(below);
                nz_key[slot] = k0;
                nz_chg[slot] = chg;
            }
        }
        if (next) store(y + 2, val, end);
    }
    __syncthreads();
    if (tid == 0) {
        nz_cnt[blk] = region_count;
        nz_off[blk] = region_count;
    }
}

// Geometry of the change kernel's launch for an image (workgroups, threads,
// lines per run), shared by the launch and by the record layout.
struct FloatGrid {
    FloatView v;
    int D, threads;
    int64_t grid;
};

static int float_grid(const ecc_dims *dims, FloatGrid *g) {
    // drop axes of extent 1, pad in front to four axes
    int32_t ext[4];
    int d = 0;
    int64_t total = 1;
    for (int i = 0; i < dims->ndim; ++i) {
        total *= dims->n[i];
        if (dims->n[i] > 1) ext[d++] = (int32_t)dims->n[i];
    }
    if (total * 4 > (int64_t)UINT32_MAX) {
        set_error("float images are limited to 2^30 elements");
        return ECC_E_UNSUPPORTED;
    }
    FloatView &v = g->v;
    v = FloatView{};
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
    if (grid > INT32_MAX || grid * threads * v.run > (int64_t)UINT32_MAX) {
        set_error("float image: too many lines");
        return ECC_E_UNSUPPORTED;
    }
    v.e0 = 0;
    v.e1 = INT32_MAX;
    g->D = D;
    g->threads = threads;
    g->grid = grid;
    return ECC_OK;
}

int64_t float_regions(const ecc_dims *dims, int64_t *slots) {
    FloatGrid g;
    if (float_grid(dims, &g)) return -1;
    *slots = g.grid * g.threads * g.v.run;
    return g.grid;
}

int launch_float_change(const float *img_dev, const ecc_dims *dims, uint32_t *keys, uint32_t *nz_key,
                        int32_t *nz_chg, uint32_t *nz_cnt, uint32_t *nz_off, uint32_t *status, hipStream_t stream,
                        int32_t e0, int32_t e1) {
    FloatGrid fg;
    int rc = float_grid(dims, &fg);
    if (rc) return rc;
    if ((e0 != 0 || e1 != INT32_MAX) && (fg.D != 4 || dims->ndim != 4)) {
        set_error("internal error: an emit range needs four axes longer than 1");
        return ECC_E_ARG;
    }
    FloatView v = fg.v;
    v.e0 = e0;
    v.e1 = e1;
    const int D = fg.D, threads = fg.threads;
    const int64_t grid = fg.grid;
    int64_t total = 1;
    for (int i = 0; i < dims->ndim; ++i) total *= dims->n[i];
    const uint32_t bytes = (uint32_t)(total * 4);
    void *tok = nullptr;
    rc = profile_begin(stream, &tok);
    if (rc) return rc;
    const dim3 g((unsigned)grid), b(threads);
#define ECC_FCK(DD)                                                                                              \
    switch (threads) {                                                                                           \
    case 64: hipLaunchKernelGGL((float_change_kernel<DD, 64>), g, b, 0, stream, img_dev, bytes, v, keys, nz_key, nz_chg, nz_cnt, nz_off, status); break;   \
    case 128: hipLaunchKernelGGL((float_change_kernel<DD, 128>), g, b, 0, stream, img_dev, bytes, v, keys, nz_key, nz_chg, nz_cnt, nz_off, status); break; \
    case 192: hipLaunchKernelGGL((float_change_kernel<DD, 192>), g, b, 0, stream, img_dev, bytes, v, keys, nz_key, nz_chg, nz_cnt, nz_off, status); break; \
    default: hipLaunchKernelGGL((float_change_kernel<DD, 256>), g, b, 0, stream, img_dev, bytes, v, keys, nz_key, nz_chg, nz_cnt, nz_off, status); break;  \
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
// The non-zero change records, from the workgroups' regions to one dense
// array of 64-bit words (key << 32 | change as uint32), sorted by key.

// After the exclusive scan of nz_off (region offsets): the record count.
// Written to device memory and to host-mapped memory (read by the host
// after an event, to size the record sort).
__global__ void nz_total_kernel(const uint32_t *nz_cnt, const uint32_t *nz_off, int64_t regions, int64_t *total_dev,
                                int64_t *total_host) {
    const int64_t t = (int64_t)nz_off[regions - 1] + nz_cnt[regions - 1];
    *total_dev = t;
    *total_host = t;
}

int launch_nz_total(const uint32_t *nz_cnt, uint32_t *nz_off, int64_t regions, uint32_t *sums, int64_t *total_dev,
                    int64_t *total_host, hipStream_t stream) {
    int rc = exclusive_scan_u32(nz_off, regions, sums, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(nz_total_kernel, dim3(1), dim3(1), 0, stream, nz_cnt, (const uint32_t *)nz_off, regions,
                       total_dev, total_host);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

__global__ void __launch_bounds__(256) nz_compact_kernel(const uint32_t *__restrict__ nz_key,
                                                         const int32_t *__restrict__ nz_chg,
                                                         const uint32_t *__restrict__ nz_cnt,
                                                         const uint32_t *__restrict__ nz_off, int64_t region_slots,
                                                         uint64_t *__restrict__ rec) {
    const uint32_t c = nz_cnt[blockIdx.x];
    const int64_t src = (int64_t)blockIdx.x * region_slots, dst = nz_off[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < c; i += blockDim.x)
        rec[dst + i] = ((uint64_t)nz_key[src + i] << 32) | (uint32_t)nz_chg[src + i];
}

int launch_nz_compact(const uint32_t *nz_key, const int32_t *nz_chg, const uint32_t *nz_cnt, const uint32_t *nz_off,
                      int64_t regions, int64_t region_slots, uint64_t *rec, hipStream_t stream) {
    if (regions > INT32_MAX) {
        set_error("float image: too many regions");
        return ECC_E_UNSUPPORTED;
    }
    hipLaunchKernelGGL(nz_compact_kernel, dim3((unsigned)regions), dim3(256), 0, stream, nz_key, nz_chg, nz_cnt, nz_off,
                       region_slots, rec);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// Integer images through the change kernel (their values as floats, exact
// below 2^24): every region's records added to the changes vector at the
// record's value (int64 atomics: exact in any order).  Values >= m were
// flagged by the conversion and are skipped here.
__global__ void __launch_bounds__(256) records_to_vcec_kernel(const uint32_t *__restrict__ nz_key,
                                                              const int32_t *__restrict__ nz_chg,
                                                              const uint32_t *__restrict__ nz_cnt,
                                                              int64_t region_slots, int m,
                                                              int64_t *__restrict__ vcec) {
    const uint32_t c = nz_cnt[blockIdx.x];
    const int64_t src = (int64_t)blockIdx.x * region_slots;
    for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
        const uint32_t v = (uint32_t)key_to_f32(nz_key[src + i]);
        if (v < (uint32_t)m) atomicAdd((unsigned long long *)&vcec[v], (unsigned long long)(int64_t)nz_chg[src + i]);
    }
}

int launch_records_to_vcec(const uint32_t *nz_key, const int32_t *nz_chg, const uint32_t *nz_cnt, int64_t regions,
                           int64_t region_slots, int m, int64_t *vcec, hipStream_t stream) {
    if (regions > INT32_MAX) {
        set_error("float image: too many regions");
        return ECC_E_UNSUPPORTED;
    }
    hipLaunchKernelGGL(records_to_vcec_kernel, dim3((unsigned)regions), dim3(256), 0, stream, nz_key, nz_chg, nz_cnt,
                       region_slots, m, vcec);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// ----------------------------------------------------------------------------
// After both sorts: the distinct keys and the curve.  chi after a distinct
// value v is the sum of the changes of the voxels with key <= v, i.e. the
// inclusive prefix P of the sorted records' changes at the last record with
// key <= v (0 if there is none).
//  1. ukey_count_kernel: per tile of kFTile sorted keys, the number of
//     last-of-key positions (a key differing from the next one), and its
//     exclusive scan: the tile's first rank;
//  2. rec_tile_sums_kernel, fscan_tiles_kernel, rec_prefix_kernel: P over
//     the records;
//  4. slice_bounds_kernel, curve_write_kernel: each last-of-key position
//     writes its key (as float) and chi at its rank.  Tile t of the keys,
//     [i0, i1), owns the key values in [key[i0], key[i1]) (from minus
//     infinity for the first tile, to plus infinity for the last): those
//     whose last position lies in the tile.  Its records are the ones in
//     [lower_bound(key[i0]), lower_bound(key[i1])) (one binary search per
//     tile, all tiles at once); the tile's distinct keys then look only at
//     that slice, from LDS when it is short.  The last tile writes K (known
//     on the device only).

constexpr int kFThreads = 256;
constexpr int kFItems = 16;
constexpr int kFTile = kFThreads * kFItems;

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

__device__ __forceinline__ bool last_of_key(const uint32_t *key, int64_t i, int64_t n) {
    return i == n - 1 || key[i] != key[i + 1];
}

// Last-of-key positions per tile: four 16-byte loads per thread (groups of
// four keys, coalesced across the wave), the key after each group from the
// next group (a cache hit).
__global__ void __launch_bounds__(kFThreads) ukey_count_kernel(const uint32_t *__restrict__ key, int64_t n,
                                                              uint32_t *__restrict__ tile_last) {
    __shared__ uint32_t sh[4];
    const int64_t t0 = (int64_t)blockIdx.x * kFTile;
    uint32_t l = 0;
    const bool vec = (reinterpret_cast<uintptr_t>(key) & 15u) == 0;
#pragma unroll
    for (int j = 0; j < kFItems / 4; ++j) {
        const int64_t g = t0 + ((int64_t)j * kFThreads + threadIdx.x) * 4;
        if (vec && g + 4 < n) {
            const uint4 w = *reinterpret_cast<const uint4 *>(key + g);
            const uint32_t nx = key[g + 4];
            l += (w.x != w.y) + (w.y != w.z) + (w.z != w.w) + (w.w != nx);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (g + q < n) l += last_of_key(key, g + q, n);
        }
    }
    l = block_sum(l, sh);
    if (threadIdx.x == 0) tile_last[blockIdx.x] = l;
}

__device__ __forceinline__ int32_t rec_change(uint64_t r) { return (int32_t)(uint32_t)r; }
__device__ __forceinline__ uint32_t rec_key(uint64_t r) { return (uint32_t)(r >> 32); }

// Change sums of record tiles [t * kFTile, (t+1) * kFTile).
__global__ void __launch_bounds__(kFThreads) rec_tile_sums_kernel(const uint64_t *__restrict__ rec, int64_t nnz,
                                                                 int64_t *__restrict__ tsum) {
    __shared__ int64_t sh[4];
    const int64_t t0 = (int64_t)blockIdx.x * kFTile;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        const int64_t i = t0 + (int64_t)j * kFThreads + threadIdx.x;
        if (i < nnz) s += rec_change(rec[i]);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

// Exclusive scans of both tile arrays in one workgroup of 1024 threads, in
// chunks of 16384 tiles: thread t holds tiles c0 + k * 1024 + t (k < 16:
// sixteen rows, every load and store coalesced).  Each row is scanned
// across the wave with shuffles; the wave totals per row go to LDS, where
// 32 threads turn them into per-wave prefixes and row totals.  The running
// carries are the same in all threads.  total_b receives the sum of b.  b may
// be null (then only a is scanned).
__global__ void __launch_bounds__(1024) fscan_tiles_kernel(int64_t *a, int64_t *b, int64_t nt, int64_t *total_b) {
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
            xb[k] = b && i < nt ? b[i] : 0;
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
                if (b) b[i] = cb + wsb[k][wave] + (lane > 0 ? pb : 0);
            }
            ca += tota[k];
            cb += totb[k];
        }
        __syncthreads();  // the LDS rows are rewritten by the next chunk
    }
    if (tid == 0 && b && total_b) *total_b = cb;
}

// LDS slot of tile position i: one pad word per 16 entries, so that a
// thread's run of 16 (thread t reads 17 t + j) spreads over the banks.
__device__ __forceinline__ int fpad(int i) { return i + (i >> 4); }

// Inclusive prefix of the records' changes: the tile's changes staged in LDS
// (coalesced loads), a thread's run of kFItems scanned, the runs scanned over
// the workgroup with the tile's offset added, the prefixes staged back for
// coalesced stores.
__global__ void __launch_bounds__(kFThreads) rec_prefix_kernel(const uint64_t *__restrict__ rec, int64_t nnz,
                                                              const int64_t *__restrict__ tbase,
                                                              int64_t *__restrict__ prefix) {
    __shared__ int64_t st[kFTile + kFTile / 16];
    __shared__ int64_t ws[kFThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kFTile;
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        const int i = j * kFThreads + tid;
        st[fpad(i)] = t0 + i < nnz ? rec_change(rec[t0 + i]) : 0;
    }
    __syncthreads();
    const int r0 = tid * kFItems;
    int64_t v[kFItems], s = 0;
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        v[j] = st[fpad(r0 + j)];
        s += v[j];
    }
    int64_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t u = __shfl_up(x, off, 64);
        if (lane >= off) x += u;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    int64_t p = tbase[blockIdx.x] + x - s;
    for (int w = 0; w < wave; ++w) p += ws[w];
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        p += v[j];
        st[fpad(r0 + j)] = p;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        const int i = j * kFThreads + tid;
        if (t0 + i < nnz) prefix[t0 + i] = st[fpad(i)];
    }
}

// First record index in [lo, hi) whose key is >= k (strict: > k), or hi.
template <bool STRICT>
__device__ __forceinline__ int64_t rec_bound(const uint64_t *rec, int64_t lo, int64_t hi, uint32_t k) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const uint32_t x = rec_key(rec[mid]);
        if (STRICT ? x <= k : x < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// bound[t] = the first record whose key is >= the first key of key tile t
// (0 for t = 0; the record count for t = nt): one thread per tile, all
// searches in flight together.
__global__ void __launch_bounds__(256) slice_bounds_kernel(const uint32_t *__restrict__ key, int64_t n, int64_t nt,
                                                           const uint64_t *__restrict__ rec, int64_t nnz,
                                                           int64_t *__restrict__ bound) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > nt) return;
    bound[t] = t == 0 ? 0 : t == nt ? nnz : rec_bound<false>(rec, 0, nnz, key[t * kFTile]);
}

// Records of a tile's slice kept in LDS (keys and prefixes): short slices
// (most tiles) in a small copy that leaves room for many workgroups per CU;
// the long ones (the tiles of the lowest and highest values, where the
// critical points gather) in a second launch with a large copy.
constexpr int kShortSlice = 512;
constexpr int kLongSlice = 4096;

// Thread t takes the run of kFItems sorted keys at t * kFItems of the tile
// (16-byte loads; the key after the run from the next lane, or from memory
// for the wave's last lane) and puts its distinct keys, in rank order, into
// LDS; the workgroup then takes them one per thread at a time (a binary
// search of the slice each, coalesced stores).  LONG = false takes the tiles
// whose slice has at most kShortSlice records, LONG = true the others: up to
// kLongSlice from LDS, beyond that (images with very few distinct values) one
// binary search in memory per distinct key.
template <bool LONG>
__global__ void __launch_bounds__(kFThreads) curve_write_kernel(const uint32_t *__restrict__ key, int64_t n,
                                                               int64_t nt, const uint32_t *__restrict__ tile_base,
                                                               const int64_t *__restrict__ bound,
                                                               const uint64_t *__restrict__ rec,
                                                               const int64_t *__restrict__ prefix,
                                                               float *__restrict__ out_keys,
                                                               int64_t *__restrict__ out_chi, int64_t *kcount) {
    constexpr int CAP = LONG ? kLongSlice : kShortSlice;
    __shared__ uint32_t sl[CAP];
    __shared__ int64_t sp[CAP + 1];  // sp[i] = P at record j0 + i - 1 (0 before the first)
    __shared__ uint32_t ck[kFTile];   // the tile's distinct keys
    __shared__ uint32_t ws[kFThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kFTile;
    const int64_t j0 = bound[blockIdx.x], j1 = bound[blockIdx.x + 1];
    const int64_t len = j1 - j0;
    if ((len > kShortSlice) != LONG) return;  // (uniform) the other launch's tile
    const bool in_lds = len <= CAP;
    const int64_t base = tile_base[blockIdx.x];
    const int64_t i0 = t0 + (int64_t)tid * kFItems;
    uint32_t k[kFItems + 1];
    static_assert(kFItems % 4 == 0, "runs of whole 16-byte groups");
    if ((reinterpret_cast<uintptr_t>(key) & 15u) == 0 && i0 + kFItems <= n) {
        const uint4 *k4 = reinterpret_cast<const uint4 *>(key + i0);
#pragma unroll
        for (int q = 0; q < kFItems / 4; ++q) {
            const uint4 w = k4[q];
            k[4 * q] = w.x;
            k[4 * q + 1] = w.y;
            k[4 * q + 2] = w.z;
            k[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kFItems; ++j) k[j] = i0 + j < n ? key[i0 + j] : 0u;
    }
    {
        const uint32_t nx = __shfl_down(k[0], 1, 64);  // the next lane's first key
        const int64_t after = i0 + kFItems;
        k[kFItems] = lane < 63 ? nx : (after < n ? key[after] : 0u);
    }
    if (in_lds) {
        for (int i = tid; i < (int)len; i += kFThreads) {
            sl[i] = rec_key(rec[j0 + i]);
            sp[i + 1] = prefix[j0 + i];
        }
        if (tid == 0) sp[0] = j0 > 0 ? prefix[j0 - 1] : 0;
    }
    uint32_t s = 0;
    bool last[kFItems];
#pragma unroll
    for (int j = 0; j < kFItems; ++j) {
        const int64_t i = i0 + j;
        last[j] = i < n && (i == n - 1 || k[j] != k[j + 1]);
        s += last[j];
    }
    uint32_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(x, off, 64);
        if (lane >= off) x += u;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();  // (also: the slice is staged)
    int64_t r = base + x - s;
    uint32_t cnt = 0;
    for (int w = 0; w < kFThreads / 64; ++w) {
        if (w < wave) r += ws[w];
        cnt += ws[w];
    }
    if (tid == 0 && (int64_t)blockIdx.x == nt - 1) *kcount = base + cnt;
    // the tile's distinct keys in rank order, then one per thread at a time:
    // a binary search of the slice each, coalesced stores
    const uint32_t rl = (uint32_t)(r - base);
    {
        uint32_t q = rl;
#pragma unroll
        for (int j = 0; j < kFItems; ++j)
            if (last[j]) ck[q++] = k[j];
    }
    __syncthreads();
    for (uint32_t q = tid; q < cnt; q += kFThreads) {
        const uint32_t v = ck[q];
        int64_t chi;
        if (in_lds) {
            int lo = 0, hi = (int)len;  // first record above v
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sl[mid] <= v) lo = mid + 1;
                else hi = mid;
            }
            chi = sp[lo];
        } else {
            const int64_t u = rec_bound<true>(rec, j0, j1, v);
            chi = u > 0 ? prefix[u - 1] : 0;
        }
        out_keys[base + q] = key_to_f32(v);
        out_chi[base + q] = chi;
    }
}

int launch_float_curve(const uint32_t *key, int64_t n, const uint64_t *rec, int64_t nnz, int64_t *prefix,
                       uint32_t *tile_cnt, uint32_t *sums, int64_t *tile_sum, int64_t *bound, int64_t *kcount,
                       float *out_keys, int64_t *out_chi, hipStream_t stream) {
    const int64_t nt = (n + kFTile - 1) / kFTile;
    if (nt > INT32_MAX || nnz > n) {
        set_error("float curve: too many keys");
        return ECC_E_UNSUPPORTED;
    }
    // the distinct keys' first rank per key tile
    hipLaunchKernelGGL(ukey_count_kernel, dim3((unsigned)nt), dim3(kFThreads), 0, stream, key, n, tile_cnt);
    ECC_HIP(hipGetLastError());
    int rc = exclusive_scan_u32(tile_cnt, nt, sums, stream);
    if (rc) return rc;
    // the records' prefix
    const int64_t rt = (nnz + kFTile - 1) / kFTile;
    if (rt > 0) {
        hipLaunchKernelGGL(rec_tile_sums_kernel, dim3((unsigned)rt), dim3(kFThreads), 0, stream, rec, nnz, tile_sum);
        ECC_HIP(hipGetLastError());
        hipLaunchKernelGGL(fscan_tiles_kernel, dim3(1), dim3(1024), 0, stream, tile_sum, (int64_t *)nullptr, rt,
                           (int64_t *)nullptr);
        ECC_HIP(hipGetLastError());
        hipLaunchKernelGGL(rec_prefix_kernel, dim3((unsigned)rt), dim3(kFThreads), 0, stream, rec, nnz,
                           (const int64_t *)tile_sum, prefix);
        ECC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(slice_bounds_kernel, dim3((unsigned)((nt + 256) / 256)), dim3(256), 0, stream, key, n, nt, rec,
                       nnz, bound);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(curve_write_kernel<false>, dim3((unsigned)nt), dim3(kFThreads), 0, stream, key, n, nt,
                       (const uint32_t *)tile_cnt, (const int64_t *)bound, rec, (const int64_t *)prefix, out_keys,
                       out_chi, kcount);
    ECC_HIP(hipGetLastError());
    hipLaunchKernelGGL(curve_write_kernel<true>, dim3((unsigned)nt), dim3(kFThreads), 0, stream, key, n, nt,
                       (const uint32_t *)tile_cnt, (const int64_t *)bound, rec, (const int64_t *)prefix, out_keys,
                       out_chi, kcount);
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

// invert: writes limit - 1 - v (the image whose smallest-value curve gives
// the largest-value curve, see launch_reflect_curve); values >= limit set
// the status bit either way.
template <typename T>
__global__ void __launch_bounds__(256) int_to_f32_kernel(const T *__restrict__ img, int64_t n, uint32_t limit,
                                                         int invert, float *__restrict__ out, uint32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = img[i];
        bad |= v >= limit;
        out[i] = invert ? (float)((int32_t)limit - 1 - (int32_t)v) : (float)v;
    }
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, kStatusRange);
}

int launch_int_to_f32(const void *img, int elem, int64_t n, uint32_t limit, int invert, float *out,
                      uint32_t *status, hipStream_t stream) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (elem == 1)
        hipLaunchKernelGGL(int_to_f32_kernel<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const uint8_t *)img, n, limit, invert, out, status);
    else
        hipLaunchKernelGGL(int_to_f32_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const uint16_t *)img, n, limit, invert, out, status);
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

// Largest-value convention from the smallest-value curve g of the inverted
// image (values m - 1 - v): a cell's largest value is <= t exactly when its
// smallest inverted value is >= m - 1 - t, so the cells counted at t are all
// cells (the whole box, chi = 1) less those counted in g at m - 2 - t:
//   curve:   out[t] = 1 - g[m - 2 - t]
//   changes: out[t] = g[m - 1 - t] - g[m - 2 - t]
// (g[-1] = 0).
__global__ void __launch_bounds__(256) reflect_curve_kernel(const int64_t *__restrict__ g, int m, int changes,
                                                            int64_t *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t below = t <= m - 2 ? g[m - 2 - t] : 0;
    out[t] = changes ? g[m - 1 - t] - below : 1 - below;
}

int launch_reflect_curve(const int64_t *g, int m, int changes, int64_t *out, hipStream_t stream) {
    hipLaunchKernelGGL(reflect_curve_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, g, m, changes, out);
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
