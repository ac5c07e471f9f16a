// Integer-valued images: the vector of changes (VCEC) of Sec. 3 computed on
// gfx950, one LDS histogram per workgroup.
//
// Cells are grouped by which in-plane axes are singleton factors (Sec. 2,
// "Cubical Cell").  For a set S of in-plane axes, the values of the cells
// that are singletons exactly on S (and on any choice along axis 0) are the
// 2-window minima of the image along the axes of S (Sec. 2, "Sublevel Set
// Filtration": minimum over the containing voxels).  Along axis 0 each line
// of such a field is a 1-D complex: its edges carry the field values and each
// vertex takes the smaller of its two edges.  Charging every vertex to the
// edge it takes its value from (the earlier edge on ties) gives edge i the
// change c_{i-1} - c_i with c_i = [g_{i+1} < g_i] and c_{-1} = 1, c_{n-1} = 0,
// so only positions where the comparison flips touch the histogram.  The sign
// of a field is (-1)^(number of in-plane interval axes).  On the far edge of
// an in-plane axis i not in S, the line of the field for S equals the line of
// the field for S+{i} one position further out, with the opposite sign, so
// both are skipped: every field then lives on the voxel grid itself.
//
// This is the per-voxel bookkeeping of Algorithm 1 reorganised for a
// 64-wide wavefront: instead of inspecting all 3^d - 1 neighbours of one voxel
// (the paper's O(3^d) term), a wave keeps 2^(d-1) running minima per lane and
// one comparison per field against the next plane.  Chunks merge by plain
// addition (Sec. 3, "Parallel Computations"); each tile needs one plane of
// collar below and above and one row/column of collar on the low side of each
// in-plane axis.
//
// Layout: lanes are consecutive x (the contiguous axis), so every load of a
// wave is one coalesced 64-element segment; a wave owns R rows (nin == 2) or
// R x-segments (nin == 1) and walks the planes of its tile.  Field values are
// kept pre-multiplied by 4 so they are LDS byte offsets of their bins.

#include <cstring>

#include "ecc_internal.h"

namespace ecc {

struct KParams {
    PlaneSrc src;
    int32_t n1, n2;
    int32_t e0, e1;
    int32_t lo_inf, hi_inf;
    int32_t zc;
    int32_t tiles_x, tiles_y, tiles_z;
    int32_t win_shift;    // kXfWindow: bin = clamp(v - win_shift, 0, 16383)
    int32_t per_wg;       // tiles per workgroup (at most)
    int32_t tile_stride;  // 0: consecutive runs of per_wg tiles; 1: strided by the grid
    int32_t wx, wy;
    int32_t *partial;
    uint32_t *status;
    int64_t *zero_vcec;  // cleared by workgroup 0 when not null
    int32_t pair;        // 16-bit values, two in-plane axes: row-pair layout (see tile_body)
    uint32_t *high_flag; // 32768-bin passes: set to 1 when a value >= 32768 is loaded (may be null)
};

// Fourth word of a raw buffer resource on gfx9-family parts (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;

// transforms of the loaded values (template parameter XF)
constexpr int kXfNone = 0;
constexpr int kXfInvert = 1;
constexpr int kXfWindow = 2;
// 16-bit values in 32768-bin passes: the fields are the raw values (32-bit,
// kInfRaw above all of them) and each update's LDS address is
// 4 * (value - win_shift); kXfRange: every value of the image lies in the
// pass's range; kXfRangeMasked: the adds of values outside it are masked off.
constexpr int kXfRange = 3;
constexpr int kXfRangeMasked = 4;
constexpr bool raw_fields(int xf) { return xf == kXfRange || xf == kXfRangeMasked; }
constexpr uint32_t kInfRaw = 0x10000u;

// Field values are LDS byte offsets of their bins (value * 4), computed with
// packed 16-bit ops.  The 16-bit VOP2 forms (v_lshlrev_b16, v_min_u16) write
// only the low half of their destination on gfx950 and keep whatever the upper
// half held, so they are not used here: the VOP3P forms write the whole
// register, and with zero-extended inputs (ushort/ubyte loads) the upper half
// of the result is 0.  For 14-bit data stored in 16 bits the offset wraps
// modulo 65536, so a bad input can never address outside the histogram; such
// inputs are reported through the status word instead.  kInf compares above
// every offset (offsets are <= 0xFFFC).
constexpr uint32_t kInf = 0xFFFFu;

// Shifts by an inline constant use op_sel_hi:[0,1]: the high lane then reads
// the constant's low half too.  With the default op_sel_hi the high lane
// reads bits 31:16 of the 32-bit constant 2, i.e. 0, and is not shifted.
#define ECC_PK_SHL2 "v_pk_lshlrev_b16 %0, 2, %1 op_sel_hi:[0,1]"

// v: zero-extended 16-bit value
__device__ __forceinline__ uint32_t bin_off(uint32_t v) {
    uint32_t r;
    asm(ECC_PK_SHL2 : "=v"(r) : "v"(v));
    return r;
}
// a, b: zero-extended 16-bit values
__device__ __forceinline__ uint32_t bin_off_min(uint32_t a, uint32_t b) {
    uint32_t m, r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(a), "v"(b));
    asm(ECC_PK_SHL2 : "=v"(r) : "v"(m));
    return r;
}
// Both inputs are zero-extended offsets, so a 32-bit minimum is exact.
__device__ __forceinline__ uint32_t min_off(uint32_t a, uint32_t b) { return a < b ? a : b; }
// The same for raw 16-bit values, as one 32-bit VALU op the compiler cannot
// narrow: with zero-extended inputs it would pick v_min_u16, whose upper
// half of the result is not written (see above).
__device__ __forceinline__ uint32_t min_raw(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_min_u32_e32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Row pairs (interior waves of 16-bit images with even rows, see tile_body):
// each lane loads the aligned dword that holds the value at its column x,
// i.e. the values at x & ~1 and (x & ~1) + 1.  The waves start at odd
// columns, so the left neighbour x-1 is either the low half of the lane's own
// dword (x odd) or the value of the lane before it (x even).  Both values of
// the dword are scaled to byte offsets with one packed shift; the lane's own
// offset is one bit-field extract (shift 16 for odd x, 0 for even x); one
// wave shift moves every lane's own offset to the next lane, and lane 0,
// which has no lane before it (and an odd column), keeps its own scaled
// dword instead, whose low half is the offset of x-1.  The window field is
// then one packed minimum of that and the own offset, whose high half is
// min(.., 0) = 0.  No lane needs another wave's values, and every image load
// stays 4-byte aligned.
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i-1 (lane 0 has no source)

// d: the loaded dword (already transformed); sh: 16 for odd x, 0 for even x.
// f0 = 4 * value at x, fx = 4 * min(value at x-1, value at x).
__device__ __forceinline__ void pair_offsets(uint32_t d, uint32_t sh, uint32_t &f0, uint32_t &fx) {
    uint32_t d4, m;
    asm(ECC_PK_SHL2 : "=v"(d4) : "v"(d));
    f0 = __builtin_amdgcn_ubfe(d4, sh, 16);
    // lanes 1..63: the previous lane's f0; lane 0 (bound_ctrl off): d4 itself
    const uint32_t pv = (uint32_t)__builtin_amdgcn_update_dpp((int)d4, (int)f0, kDppWaveShr1, 0xF, 0xF, false);
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(pv), "v"(f0));
    fx = m;
}
// The same without the scaling: f0 = value at x, fx = min(value at x-1,
// value at x), both raw (high half 0).
__device__ __forceinline__ void pair_values(uint32_t d, uint32_t sh, uint32_t &f0, uint32_t &fx) {
    uint32_t m;
    f0 = __builtin_amdgcn_ubfe(d, sh, 16);
    const uint32_t pv = (uint32_t)__builtin_amdgcn_update_dpp((int)d, (int)f0, kDppWaveShr1, 0xF, 0xF, false);
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(pv), "v"(f0));
    fx = m;
}
// clamp(v - s, 0, 16383) on both halves; s2 = s | s << 16 (0 <= s < 65536)
__device__ __forceinline__ uint32_t pair_window(uint32_t q, uint32_t s2) {
    uint32_t m, d, r;
    asm("v_pk_max_u16 %0, %1, %2" : "=v"(m) : "v"(q), "s"(s2));
    asm("v_pk_sub_u16 %0, %1, %2" : "=v"(d) : "v"(m), "s"(s2));
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(d), "s"(0x3FFF3FFFu));
    return r;
}

__device__ __forceinline__ uint32_t load_elem(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, int esz) {
    if (esz == 1) return __builtin_amdgcn_raw_buffer_load_b8(rs, voff, soff, 0);
    return __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0);
}

__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// ----------------------------------------------------------------------------
// Histogram updates of four (row, field) items at once.  Item i adds at byte
// offset g_i on the lanes whose ownership flag flips between planes
// (p_i != c_i): +s_i where it falls (p_i set, c_i clear) and -s_i where it
// rises.  Two forms per item, chosen at compile time (bit i of DM):
//  - select (bit clear): one add of e_i = (p_i ? s_i : -s_i) on the lanes of
//    p_i ^ c_i; e_i is built beforehand with full EXEC (it depends only on the
//    previous plane's mask, so it is off the critical path);
//  - split (bit set): an add of the constant +-1 on p_i & ~c_i and one of the
//    opposite constant on c_i & ~p_i: no vector select, but two LDS
//    instructions.
// The block sets EXEC directly from the lane masks and restores it before
// returning, so the compiler never sees a modified EXEC.  The histogram is the
// kernel's only LDS object, at LDS address 0, so the bin offsets are LDS
// addresses.  The scalar ops of the block write SCC, which is therefore
// declared clobbered: the compiler must not keep a comparison result in SCC
// across the block.  SG: bit i set = item i has sign -1.
#define ECC_SEL(i) "s_xor_b64 exec, %[c" #i "], %[p" #i "]\n\tds_add_u32 %[g" #i "], %[e" #i "]\n\t"
#define ECC_SPL(i, FALL, RISE)                                                   \
    "s_andn2_b64 exec, %[p" #i "], %[c" #i "]\n\tds_add_u32 %[g" #i "], %[" FALL \
    "]\n\ts_andn2_b64 exec, %[c" #i "], %[p" #i "]\n\tds_add_u32 %[g" #i "], %[" RISE "]\n\t"
#define ECC_SPP(i) ECC_SPL(i, "one", "mone")
#define ECC_SPM(i) ECC_SPL(i, "mone", "one")
#define ECC_UPD(A, B, C, D)                                                                                       \
    asm volatile("s_mov_b64 %[sv], exec\n\t" A(0) B(1) C(2) D(3) "s_mov_b64 exec, %[sv]"                        \
                 : [sv] "=&s"(sv)                                                                                 \
                 : [g0] "v"(g0), [g1] "v"(g1), [g2] "v"(g2), [g3] "v"(g3), [e0] "v"(e0), [e1] "v"(e1),          \
                   [e2] "v"(e2), [e3] "v"(e3), [c0] "s"(c0), [c1] "s"(c1), [c2] "s"(c2), [c3] "s"(c3),          \
                   [p0] "s"(p0), [p1] "s"(p1), [p2] "s"(p2), [p3] "s"(p3), [one] "v"(one), [mone] "v"(mone) \
                 : "memory", "scc")

// The select form with a further lane mask per item (r_i: the lanes whose
// value lies in the pass's range).
#define ECC_SELR(i) \
    "s_xor_b64 exec, %[c" #i "], %[p" #i "]\n\ts_and_b64 exec, exec, %[r" #i "]\n\tds_add_u32 %[g" #i "], %[e" #i "]\n\t"
__device__ __forceinline__ void update4_masked(uint32_t g0, uint32_t g1, uint32_t g2, uint32_t g3, uint64_t c0,
                                               uint64_t c1, uint64_t c2, uint64_t c3, uint64_t p0, uint64_t p1,
                                               uint64_t p2, uint64_t p3, uint64_t r0, uint64_t r1, uint64_t r2,
                                               uint64_t r3, uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3) {
    uint64_t sv;
    asm volatile("s_mov_b64 %[sv], exec\n\t" ECC_SELR(0) ECC_SELR(1) ECC_SELR(2) ECC_SELR(3) "s_mov_b64 exec, %[sv]"
                 : [sv] "=&s"(sv)
                 : [g0] "v"(g0), [g1] "v"(g1), [g2] "v"(g2), [g3] "v"(g3), [e0] "v"(e0), [e1] "v"(e1),
                   [e2] "v"(e2), [e3] "v"(e3), [c0] "s"(c0), [c1] "s"(c1), [c2] "s"(c2), [c3] "s"(c3),
                   [p0] "s"(p0), [p1] "s"(p1), [p2] "s"(p2), [p3] "s"(p3), [r0] "s"(r0), [r1] "s"(r1),
                   [r2] "s"(r2), [r3] "s"(r3)
                 : "memory", "scc");
}
#undef ECC_SELR

template <int SG, int DM>
__device__ __forceinline__ void update4(uint32_t g0, uint32_t g1, uint32_t g2, uint32_t g3, uint64_t c0, uint64_t c1,
                                        uint64_t c2, uint64_t c3, uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3,
                                        uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3, uint32_t one,
                                        uint32_t mone) {
    uint64_t sv;
    if constexpr (DM == 0) ECC_UPD(ECC_SEL, ECC_SEL, ECC_SEL, ECC_SEL);
    else if constexpr (SG == 0b0110 && DM == 0b0110) ECC_UPD(ECC_SEL, ECC_SPM, ECC_SPM, ECC_SEL);
    else if constexpr (SG == 0b0110 && DM == 0b1001) ECC_UPD(ECC_SPP, ECC_SEL, ECC_SEL, ECC_SPP);
    else if constexpr (SG == 0b0110 && DM == 0b1111) ECC_UPD(ECC_SPP, ECC_SPM, ECC_SPM, ECC_SPP);
    else if constexpr (SG == 0b0101 && DM == 0b0101) ECC_UPD(ECC_SPM, ECC_SEL, ECC_SPM, ECC_SEL);
    else if constexpr (SG == 0b0101 && DM == 0b1010) ECC_UPD(ECC_SEL, ECC_SPP, ECC_SEL, ECC_SPP);
    else if constexpr (SG == 0b0101 && DM == 0b1111) ECC_UPD(ECC_SPM, ECC_SPP, ECC_SPM, ECC_SPP);
    else static_assert(DM < 0, "update4: form not instantiated");
}
#undef ECC_UPD
#undef ECC_SPM
#undef ECC_SPP
#undef ECC_SPL
#undef ECC_SEL

// +-1 of an item from the previous plane's ownership mask p (lane bit set:
// the vertex below was owned by this edge, so a flip removes it: +s).
__device__ __forceinline__ uint32_t flip_value(uint64_t p, int s) {
    return __builtin_amdgcn_inverse_ballot_w64(p) ? (uint32_t)s : (uint32_t)(-s);
}

// Update forms per group of four items (DM of update4).  Mode 0: all select;
// 1: split on the items of sign -1 (nin == 2) or of the vertex field
// (nin == 1); 2: split on the others; 3: all split.
template <int NIN, int MODE>
constexpr int group_dm() {
    constexpr int half = (NIN == 2) ? 0b0110 : 0b0101;
    return MODE == 0 ? 0 : MODE == 1 ? half : MODE == 2 ? (0b1111 ^ half) : 0b1111;
}

template <int NIN, int R>
struct Walker {
    static constexpr int K = 1 << NIN;                 // fields per row
    static constexpr int NR = (NIN == 2) ? R + 1 : R;  // loaded rows per plane
    static constexpr int NI = R * K;                   // (row, field) items per plane
    static_assert(NI % 4 == 0, "items come in groups of four");

    // Fields of one plane, flattened as item i = r*K + k.  a[rr], b[rr]: raw
    // values at x and at x-1 (clamped) of loaded row rr (NIN == 2: rr = 0 is
    // the collar row y0-1); xf(v): the value transform, applied as each value
    // is consumed.
    template <typename X>
    static __device__ __forceinline__ void fields(const uint32_t (&a)[NR], const uint32_t (&b)[NR],
                                                  uint32_t (&g)[NI], X xf) {
        if constexpr (NIN == 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t va = xf(a[r]);
                g[2 * r + 0] = bin_off(va);
                g[2 * r + 1] = bin_off_min(va, xf(b[r]));
            }
        } else {
            uint32_t f0[NR], fx[NR];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const uint32_t va = xf(a[rr]);
                f0[rr] = bin_off(va);
                fx[rr] = bin_off_min(va, xf(b[rr]));
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                g[4 * r + 0] = f0[r + 1];
                g[4 * r + 1] = fx[r + 1];
                g[4 * r + 2] = min_off(f0[r], f0[r + 1]);
                g[4 * r + 3] = min_off(fx[r], fx[r + 1]);
            }
        }
    }

    // The same fields (NIN == 2) from the loaded dwords d[rr] of the row-pair
    // layout; sh: the lane's half (16 for odd x, 0 for even x); xfp: the
    // value transform applied to both halves of a dword.
    template <typename X>
    static __device__ __forceinline__ void fields_pair(const uint32_t (&d)[NR], uint32_t sh, uint32_t (&g)[NI],
                                                       X xfp) {
        static_assert(NIN == 2, "row pairs: two in-plane axes");
        uint32_t f0[NR], fx[NR];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) pair_offsets(xfp(d[rr]), sh, f0[rr], fx[rr]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            g[4 * r + 0] = f0[r + 1];
            g[4 * r + 1] = fx[r + 1];
            g[4 * r + 2] = min_off(f0[r], f0[r + 1]);
            g[4 * r + 3] = min_off(fx[r], fx[r + 1]);
        }
    }

    // Raw-value fields (32768-bin passes): the element form and the row-pair
    // form without the scaling to offsets.
    static __device__ __forceinline__ void fields_raw(const uint32_t (&a)[NR], const uint32_t (&b)[NR],
                                                      uint32_t (&g)[NI]) {
        if constexpr (NIN == 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                g[2 * r + 0] = a[r];
                g[2 * r + 1] = min_raw(a[r], b[r]);
            }
        } else {
            uint32_t fx[NR];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) fx[rr] = min_raw(a[rr], b[rr]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                g[4 * r + 0] = a[r + 1];
                g[4 * r + 1] = fx[r + 1];
                g[4 * r + 2] = min_raw(a[r], a[r + 1]);
                g[4 * r + 3] = min_raw(fx[r], fx[r + 1]);
            }
        }
    }
    static __device__ __forceinline__ void fields_pair_raw(const uint32_t (&d)[NR], uint32_t sh, uint32_t (&g)[NI]) {
        static_assert(NIN == 2, "row pairs: two in-plane axes");
        uint32_t f0[NR], fx[NR];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) pair_values(d[rr], sh, f0[rr], fx[rr]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            g[4 * r + 0] = f0[r + 1];
            g[4 * r + 1] = fx[r + 1];
            g[4 * r + 2] = min_raw(f0[r], f0[r + 1]);
            g[4 * r + 3] = min_raw(fx[r], fx[r + 1]);
        }
    }

    static __device__ __forceinline__ void set_inf(uint32_t (&g)[NI], uint32_t inf) {
#pragma unroll
        for (int i = 0; i < NI; ++i) g[i] = inf;
    }

    // sign (-1)^(in-plane interval axes) of item i = r*K + k, k's bits = singleton axes
    static constexpr int sign(int i) { return (((NIN - __builtin_popcount(i % K)) & 1) ? -1 : 1); }
    // sign bits of a group of four items (bit j set: item j has sign -1)
    static constexpr int kGroupSigns = (NIN == 2) ? 0b0110 : 0b0101;
};

// Validity on the far edges of the in-plane axes (see the boundary rule at the
// top): field k of row r is valid at lanes with x <= n2-2 (fields without x)
// or x < n2 (fields with x), on rows with y <= n1-2 (fields without y) or
// y < n1 (fields with y).  For NIN == 1 "rows" are x-segments: a segment
// group is either wholly inside (FULL) or walked one segment at a time, so one
// pair of lane masks describes it.
struct EdgeMasks {
    uint64_t lx_int;   // lanes with x <= n2-2 (NIN == 1: of the first segment)
    uint64_t lx_any;   // lanes with x <  n2
    uint64_t lx_int2;  // NIN == 1: the same for the second segment of a pair
    uint64_t lx_any2;
    uint32_t ry_int;   // NIN == 2, bit r: row r has y <= n1-2
    uint32_t ry_any;   // NIN == 2, bit r: row r has y <  n1
};

template <int NIN>
__device__ __forceinline__ uint64_t edge_mask(const EdgeMasks &em, int i) {
    constexpr int K = 1 << NIN;
    const int k = i % K, r = i / K;
    if constexpr (NIN == 1) {
        // edge groups are walked as pairs of segments (items 0,1 | 2,3)
        return r == 0 ? ((k & 1) ? em.lx_any : em.lx_int) : ((k & 1) ? em.lx_any2 : em.lx_int2);
    } else {
        const uint64_t lm = (k & 1) ? em.lx_any : em.lx_int;
        const uint32_t rb = (k & 2) ? em.ry_any : em.ry_int;
        return ((rb >> r) & 1u) ? lm : 0ull;
    }
}

constexpr int lcm(int a, int b) {
    int x = a, y = b;
    while (y) {
        const int t = x % y;
        x = y;
        y = t;
    }
    return a / x * b;
}

// One wave walks the planes [zs, ze) of its rows.  FULL: no position of this
// wave lies on a far edge, so the comparison masks need no validity mask.
// PAIR (FULL waves of the row-pair layout): one aligned dword load per row at
// byte offset vx[rr], and psel, the lane's half of it (16 for odd x, 0 for
// even x); vxl is unused.
// PD: planes of raw loads kept in flight ahead of the plane being compared.
// The plane loop is unrolled by lcm(2, PD+1) so that every register buffer is
// addressed with a compile-time index (plane p of the tile uses raw buffer
// (p - zs) mod (PD+1) and field buffer (p - zs) mod 2).
template <typename T, int NIN, int R, int MODE, bool FULL, int PD, int XF, bool PAIR = false>
__device__ __forceinline__ void walk(const KParams &P, int zs, int ze, const uint32_t (&vx)[R + 1],
                                     const uint32_t (&vxl)[R + 1], const uint32_t (&soff)[R + 1], const EdgeMasks &em,
                                     uint32_t &orv, uint32_t psel = 0) {
    static_assert(!PAIR || (FULL && NIN == 2 && sizeof(T) == 2), "row pairs: interior 16-bit waves, 2 axes");
    using W = Walker<NIN, R>;
    constexpr int NR = W::NR;
    constexpr int NI = W::NI;
    constexpr int ESZ = sizeof(T);
    constexpr uint32_t kInvMask = ESZ == 1 ? 255u : 16383u;
    constexpr int NB = PD + 1;
    constexpr int U = lcm(2, NB);
    constexpr bool RAW = raw_fields(XF);
    constexpr uint32_t kSent = RAW ? kInfRaw : kInf;  // planes outside the image
    const int64_t pb = P.src.plane_bytes;
    const int32_t pbytes = (int32_t)pb;
    // planes zs-1 and ze are +inf outside the image
    const bool lo_real = !(zs == P.e0 && P.lo_inf);
    const bool hi_real = !(ze == P.e1 && P.hi_inf);
    auto real = [&](int p) { return p < ze || (p == ze && hi_real); };  // for p >= zs

    auto load_at = [&](const uint8_t *pp, uint32_t (&a)[NR], uint32_t (&b)[NR]) {
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)pp, (short)0, pbytes, kBufferWord3);
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            if constexpr (PAIR) {
                a[rr] = __builtin_amdgcn_raw_buffer_load_b32(rs, vx[rr], soff[rr], 0);
            } else {
                a[rr] = load_elem(rs, vx[rr], soff[rr], ESZ);
                b[rr] = load_elem(rs, vxl[rr], soff[rr], ESZ);
            }
        }
    };
    auto plane_ptr = [&](int p) { return (p < 0 ? P.src.lo_base : P.src.base) + p * pb; };
    auto load_plane = [&](int p, uint32_t (&a)[NR], uint32_t (&b)[NR]) { load_at(plane_ptr(p), a, b); };
    auto range_acc = [&](const uint32_t (&a)[NR]) {
        // rows owned by this wave (the collar row is checked by its owner);
        // every 16-bit value is valid for the window passes
        // (32768-bin passes: whether any value >= 32768 occurs)
        if constexpr (XF == kXfNone || XF == kXfInvert || raw_fields(XF)) {
#pragma unroll
            for (int rr = NR - R; rr < NR; ++rr) orv |= a[rr];
        }
    };
    // Fields of a loaded plane.  The value transform is applied here, where
    // the values are consumed, not at the load: there it would make each load
    // wait at once and lose the planes of look-ahead.
    const int32_t wshift = P.win_shift;
    auto fields = [&](const uint32_t (&a)[NR], const uint32_t (&b)[NR], uint32_t (&g)[NI]) {
        if constexpr (RAW) {
            if constexpr (PAIR) W::fields_pair_raw(a, psel, g);
            else W::fields_raw(a, b, g);
            return;
        }
        if constexpr (PAIR) {
            W::fields_pair(a, psel, g, [&](uint32_t q) -> uint32_t {
                if constexpr (XF == kXfInvert) return q ^ (kInvMask * 0x10001u);
                else if constexpr (XF == kXfWindow) return pair_window(q, (uint32_t)wshift * 0x10001u);
                else return q;
            });
            return;
        }
        W::fields(a, b, g, [&](uint32_t v) -> uint32_t {
            if constexpr (XF == kXfInvert) return v ^ kInvMask;  // M-1-v (M a power of two)
            else if constexpr (XF == kXfWindow)  // 16-bit window: v - shift clamped to 0..16383
                return (uint32_t)max(0, min(16383, (int32_t)v - wshift));
            else return v;
        });
    };
    auto cmp = [&](uint32_t lo, uint32_t hi, int i) -> uint64_t {
        const uint64_t c = ballot(lo < hi);
        if constexpr (FULL) return c;
        else return c & edge_mask<NIN>(em, i);
    };
    // Compare plane z+1 (gn) with plane z (gc) and add the changes of plane z.
    constexpr int DM = group_dm<NIN, MODE>();
    const uint32_t one = 1u, mone = 0xFFFFFFFFu;
    static_assert(!RAW || (MODE == 0 && sizeof(T) == 2), "32768-bin passes: 16-bit values, select updates");
    const uint32_t abase = RAW ? (uint32_t)(-4 * (int64_t)P.win_shift) : 0u;
    constexpr uint32_t kAddrEnd = RAW ? 4u * 32768u : 0u;
    auto step = [&](const uint32_t (&gc)[NI], const uint32_t (&gn)[NI], uint64_t (&cp)[NI]) {
#pragma unroll
        for (int i = 0; i < NI; i += 4) {
            uint32_t e[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) e[j] = ((DM >> j) & 1) ? one : flip_value(cp[i + j], W::sign(i + j));
            const uint64_t c0 = cmp(gn[i], gc[i], i), c1 = cmp(gn[i + 1], gc[i + 1], i + 1);
            const uint64_t c2 = cmp(gn[i + 2], gc[i + 2], i + 2), c3 = cmp(gn[i + 3], gc[i + 3], i + 3);
            if constexpr (RAW) {
                // LDS addresses 4 * (value - win_shift); outside the pass's
                // range they wrap above 4 * M
                uint32_t a[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = (gc[i + j] << 2) + abase;
                if constexpr (XF == kXfRangeMasked) {
                    uint64_t r[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) r[j] = ballot(a[j] < kAddrEnd);
                    update4_masked(a[0], a[1], a[2], a[3], c0, c1, c2, c3, cp[i], cp[i + 1], cp[i + 2], cp[i + 3],
                                   r[0], r[1], r[2], r[3], e[0], e[1], e[2], e[3]);
                } else {
                    update4<W::kGroupSigns, DM>(a[0], a[1], a[2], a[3], c0, c1, c2, c3, cp[i], cp[i + 1], cp[i + 2],
                                                cp[i + 3], e[0], e[1], e[2], e[3], one, mone);
                }
            } else {
                update4<W::kGroupSigns, DM>(gc[i], gc[i + 1], gc[i + 2], gc[i + 3], c0, c1, c2, c3, cp[i], cp[i + 1],
                                            cp[i + 2], cp[i + 3], e[0], e[1], e[2], e[3], one, mone);
            }
            cp[i] = c0;
            cp[i + 1] = c1;
            cp[i + 2] = c2;
            cp[i + 3] = c3;
        }
    };

    uint32_t ra[NB][NR], rb[NB][NR];
    uint32_t g[2][NI];
    uint64_t cp[NI];

    // g[1] <- plane zs-1 (or +inf), g[0] <- plane zs, cp <- [g0 < g1]
    if (lo_real) {
        load_plane(zs - 1, ra[NB - 1], rb[NB - 1]);
        fields(ra[NB - 1], rb[NB - 1], g[1]);
    } else {
        W::set_inf(g[1], kSent);
    }
    load_plane(zs, ra[0], rb[0]);
    fields(ra[0], rb[0], g[0]);
    range_acc(ra[0]);
#pragma unroll
    for (int i = 0; i < NI; ++i) cp[i] = cmp(g[0][i], g[1][i], i);
#pragma unroll
    for (int j = 1; j <= PD; ++j)
        if (real(zs + j)) load_plane(zs + j, ra[j], rb[j]);

    // Phase u of a block handles plane z+u: start the load of plane z+u+1+PD
    // into the buffer that held plane z+u, turn plane z+u+1 into fields and
    // compare.  `nxt` points at the next plane to load.  Steady state: every
    // plane touched lies inside the tile.
    const uint8_t *nxt = plane_ptr(zs + 1 + PD);  // zs >= -1, so this plane is in `base`
    int z = zs;
    for (; z + U + PD < ze; z += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            load_at(nxt, ra[u % NB], rb[u % NB]);
            nxt += pb;
            fields(ra[(u + 1) % NB], rb[(u + 1) % NB], g[(u + 1) & 1]);
            range_acc(ra[(u + 1) % NB]);
            step(g[u & 1], g[(u + 1) & 1], cp);
        }
    }
    // Last planes, with boundary tests.
    while (z < ze) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int zz = z + u;
            if (zz < ze) {
                if (real(zz + 1 + PD)) load_at(nxt, ra[u % NB], rb[u % NB]);
                nxt += pb;
                if (real(zz + 1)) {
                    fields(ra[(u + 1) % NB], rb[(u + 1) % NB], g[(u + 1) & 1]);
                    if (zz + 1 < ze) range_acc(ra[(u + 1) % NB]);
                } else {
                    W::set_inf(g[(u + 1) & 1], kSent);
                }
                step(g[u & 1], g[(u + 1) & 1], cp);
            }
        }
        z += U;
    }
}

// One tile per workgroup.  Workgroups are dispatched round-robin over the 8
// XCDs; the tile index is permuted so that the workgroups of one XCD take
// neighbouring tiles, which share collar rows and planes through its L2.
// Occupancy the register budget is fitted to (waves per SIMD).  The LDS
// histogram allows two 16-wave workgroups per CU: R == 2 is fitted to both
// (8 waves per SIMD, 64 registers), R == 4 to one (4 waves per SIMD), which
// leaves room for deep load pipelines instead.
template <int NIN, int R, int PD>
constexpr int kWavesPerEU() {
    return (R <= 2) ? 8 : 4;
}

// The tiles of one workgroup of one image: b = the workgroup's index among
// the image's G workgroups (G <= tiles).  Writes the counts of its tiles to
// row b of P.partial.
template <typename T, int M, int NIN, int R, int MODE, int PD, int XF = kXfNone>
__device__ __forceinline__ void tile_body(const KParams &P, int32_t *hist, const int b, const int G) {
    using W = Walker<NIN, R>;
    constexpr int NR = W::NR;
    constexpr int ESZ = sizeof(T);

    const int tid = threadIdx.x;
    // The update blocks address bins by their LDS byte offset: the histogram
    // must sit at LDS address 0 (it is this kernel's only LDS object).
    if ((uint32_t)(size_t)(__attribute__((address_space(3))) int32_t *)hist != 0u) {
        if (tid == 0) atomicOr(P.status, 0x80000000u);
        return;
    }
    // (loops with a uniform trip count: a thread-dependent one makes the
    // compiler treat later lane masks as divergent)
    for (int i0 = 0; i0 < M; i0 += (int)blockDim.x)
        if (i0 + tid < M) hist[i0 + tid] = 0;
    if (P.zero_vcec && b == 0)
        for (int i0 = 0; i0 < M; i0 += (int)blockDim.x)
            if (i0 + tid < M) P.zero_vcec[i0 + tid] = 0;
    __syncthreads();

    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wxi = wave % P.wx;
    const int wyi = wave / P.wx;
    // (batched launches use a fixed workgroup size: waves past wx * wy idle)
    const bool wave_in = wave < P.wx * P.wy;
    const int32_t n1 = P.n1, n2 = P.n2;
    const bool pair = NIN == 2 && ESZ == 2 && P.pair;

    // workgroup b (permuted: the workgroups of one XCD take neighbouring
    // indices) walks its tiles into one histogram: a run of per_wg
    // consecutive tiles, or (tile_stride) tiles bp, bp + G, bp + 2G, ...
    const int bp = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    const int ntiles = P.tiles_x * P.tiles_y * P.tiles_z;
    const int tstep = P.tile_stride ? G : 1;
    const int t0 = P.tile_stride ? bp : bp * P.per_wg;
    const int t1 = P.tile_stride ? ntiles : min(t0 + P.per_wg, ntiles);
    uint32_t orv = 0;
    for (int t = t0; t < t1; t += tstep) {
    const int tx = t % P.tiles_x;
    const int ty = (t / P.tiles_x) % P.tiles_y;
    const int tz = t / (P.tiles_x * P.tiles_y);
    const int zs = P.e0 + tz * P.zc;
    const int ze = min(zs + P.zc, P.e1);

    // Per loaded row: byte offsets of x and of x-1 (clamped into the row) and
    // the row's byte offset within a plane.  NIN == 1: row r is the 64-wide
    // x-segment seg0 + r of the single in-plane axis.
    uint32_t vx[R + 1] = {}, vxl[R + 1] = {}, soff[R + 1] = {};
    EdgeMasks em{};
    bool full = false, any = false;
    uint32_t psel = 0;
    if constexpr (NIN == 1) {
        const int32_t seg0 = (tx * P.wx + wxi) * R;
        any = wave_in && seg0 * kWave < n2;
        full = (seg0 + R) * kWave - 1 <= n2 - 2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t xcl = min((seg0 + r) * kWave + lane, n2 - 1);
            vx[r] = (uint32_t)xcl * ESZ;
            vxl[r] = (uint32_t)(xcl > 0 ? xcl - 1 : 0) * ESZ;
        }
    } else {
        // Row-pair layout: waves start at odd columns (x0 = 64 k + 1) and
        // column 0 is taken by the lane of column n2 (n2 is even there, so
        // that lane exists, in the last wave of the row, an edge wave).
        const int32_t x0 = (tx * P.wx + wxi) * kWave + (pair ? 1 : 0);
        int32_t x = x0 + lane;
        if (pair && x == n2) x = 0;
        const int32_t y0 = (ty * P.wy + wyi) * R;
        any = wave_in && x0 < n2 && y0 < n1;
        full = (x0 + kWave - 1 <= n2 - 2) && (y0 + R - 1 <= n1 - 2);
        psel = (x & 1) ? 16u : 0u;
        const int32_t xcl = min(x, n2 - 1);
        const uint32_t ox = (uint32_t)xcl * ESZ, oxl = (uint32_t)(xcl > 0 ? xcl - 1 : 0) * ESZ;
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            // row pairs: the aligned dword holding column x
            vx[rr] = (pair && full) ? (uint32_t)(x & ~1) * 2u : ox;
            vxl[rr] = oxl;
            const int32_t y = min(max(y0 + rr - 1, 0), n1 - 1);
            soff[rr] = (uint32_t)y * (uint32_t)n2 * ESZ;
        }
        if (!full) {
            em.lx_int = ballot(x <= n2 - 2);
            em.lx_any = ballot(x < n2);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                em.ry_int |= (uint32_t)(y0 + r <= n1 - 2) << r;
                em.ry_any |= (uint32_t)(y0 + r < n1) << r;
            }
        }
    }
    if (any && zs < ze) {
        if (full) {
            if constexpr (NIN == 2 && ESZ == 2) {
                if (pair)
                    walk<T, NIN, R, MODE, true, PD, XF, true>(P, zs, ze, vx, vxl, soff, em, orv, psel);
                else
                    walk<T, NIN, R, MODE, true, PD, XF>(P, zs, ze, vx, vxl, soff, em, orv);
            } else {
                walk<T, NIN, R, MODE, true, PD, XF>(P, zs, ze, vx, vxl, soff, em, orv);
            }
        } else if constexpr (NIN == 1) {
            // An edge group of segments is walked as pairs of segments, each
            // pair with its own lane masks.
            const int32_t seg0 = (tx * P.wx + wxi) * R;
#pragma unroll
            for (int r = 0; r < R; r += 2) {
                const int32_t xs = (seg0 + r) * kWave;
                if (xs >= n2) break;
                const int32_t xa = xs + lane, xb = xs + kWave + lane;
                EdgeMasks e2{};
                e2.lx_int = ballot(xa <= n2 - 2);
                e2.lx_any = ballot(xa < n2);
                e2.lx_int2 = ballot(xb <= n2 - 2);
                e2.lx_any2 = ballot(xb < n2);
                const uint32_t v2[3] = {vx[r], vx[r + 1], 0u}, vl2[3] = {vxl[r], vxl[r + 1], 0u};
                const uint32_t s2[3] = {0u, 0u, 0u};
                walk<T, 1, 2, MODE, false, 1, XF>(P, zs, ze, v2, vl2, s2, e2, orv);
            }
        } else {
            walk<T, NIN, R, MODE, false, PD, XF>(P, zs, ze, vx, vxl, soff, em, orv);
        }
    }
    }  // tiles

    if constexpr (raw_fields(XF)) {
        // every 16-bit value is valid; the caller may want to know of the
        // values >= 32768 (row pairs hold a second value in the high half)
        if (P.high_flag && ((orv | (orv >> 16)) & 0x8000u)) *P.high_flag = 1u;
    } else if constexpr (M != 256) {
        // (row pairs hold a second value in the high half)
        if (((orv | (orv >> 16)) & 0xFFFFu) >= (uint32_t)M) atomicOr(P.status, kStatusRange);
    }
    // the update blocks' LDS adds are not tracked by the compiler's counters
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
    int32_t *dst = P.partial + (size_t)b * M;
    for (int i0 = 0; i0 < M; i0 += (int)blockDim.x)
        if (i0 + tid < M) dst[i0 + tid] = hist[i0 + tid];
}

// XF, a transform of every loaded value v:
//  kXfInvert: M-1-v, so the histogram counts each cell at M-1 minus the
//    maximum over its voxels (the largest-value convention, read back
//    reversed by the merge);
//  kXfWindow (16-bit images, M = 16384 bins per pass): v - win_shift
//    clamped to 0..16383; the host keeps the bins of the window's values and
//    drops guard bins 0 / 16383 where values lie below / above it.  The
//    monotone clamp keeps every comparison that decides a kept bin, since
//    each involves the counted value itself.
// (32768 bins: a 128 KiB histogram, one workgroup per CU, four waves per SIMD)
template <typename T, int M, int NIN, int R, int MODE, int PD, int XF = kXfNone>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(M > 16384 ? 4 : kWavesPerEU<NIN, R, PD>())))
int_vcec_kernel(KParams P) {
    static_assert(raw_fields(XF) == (M == 32768), "32768 bins: raw-value passes, and only those");
    __shared__ int32_t hist[M];
    tile_body<T, M, NIN, R, MODE, PD, XF>(P, hist, blockIdx.x, gridDim.x);
}

// Batched form: the tiles of every image of a batch in one persistent
// launch.  Image j owns tiles [tile_begin[j], tile_begin[j+1]) and its
// parameters are jobs[j]; its kind selects the value type and rank.  Each
// workgroup takes the next tile from the table's work counter (a global
// atomic; the value is passed through hist[0] before tile_body clears the
// histogram) until the tiles run out.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<2, 2, 1>())))
int_vcec_persistent_kernel(uint8_t *__restrict__ table) {
    __shared__ int32_t hist[16384];
    BatchHeader *H = (BatchHeader *)table;
    const int ntiles = H->ntiles, njobs = H->njobs;
    const KParams *jobs = (const KParams *)(table + H->off_kparams);
    const int32_t *tile_begin = (const int32_t *)(table + H->off_tile_begin);
    const int32_t *kind = (const int32_t *)(table + H->off_kind);
    for (;;) {
        if (threadIdx.x == 0) hist[0] = (int32_t)atomicAdd(&H->next_tile, 1u);
        __syncthreads();
        const int v = __builtin_amdgcn_readfirstlane(hist[0]);
        __syncthreads();
        if (v >= ntiles) break;
        int lo = 0, hi = njobs - 1;  // last j with tile_begin[j] <= v
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_begin[mid] <= v) lo = mid;
            else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const KParams P = jobs[lo];
        const int b = v - tile_begin[lo], G = tile_begin[lo + 1] - tile_begin[lo];
        switch (__builtin_amdgcn_readfirstlane(kind[lo])) {
        case 0: tile_body<uint8_t, 256, 1, 2, 0, 1>(P, hist, b, G); break;
        case 1: tile_body<uint8_t, 256, 2, 2, 0, 1>(P, hist, b, G); break;
        case 2: tile_body<uint16_t, 16384, 1, 2, 0, 1>(P, hist, b, G); break;
        default: tile_body<uint16_t, 16384, 2, 2, 0, 1>(P, hist, b, G); break;
        }
        __syncthreads();  // the histogram's write-out is done before hist[0] is reused
    }
}

template <typename T, int M, int NIN, int R, int MODE, int PD, int XF = kXfNone>
static int launch_one(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    const int threads = kWave * tl.wx * tl.wy;
    void *tok = nullptr;
    int rc = profile_begin(stream, &tok);
    if (rc) return rc;
    hipLaunchKernelGGL((int_vcec_kernel<T, M, NIN, R, MODE, PD, XF>), dim3(tl.grid), dim3(threads), 0, stream, p);
    ECC_HIP(hipGetLastError());
    return profile_end(stream, tok);
}

template <typename T, int M, int NIN, int R, int MODE>
static int launch_pd(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    if (tl.pd == 1) return launch_one<T, M, NIN, R, MODE, 1>(p, tl, stream);
    if (tl.pd == 2) return launch_one<T, M, NIN, R, MODE, 2>(p, tl, stream);
    set_error("integer kernel: prefetch depth %d not built", tl.pd);
    return ECC_E_UNSUPPORTED;
}

template <typename T, int M, int NIN, int R>
static int launch_mode(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    switch (tl.mode) {
    case 0: return launch_pd<T, M, NIN, R, 0>(p, tl, stream);
    case 1: return launch_pd<T, M, NIN, R, 1>(p, tl, stream);
    case 3: return launch_pd<T, M, NIN, R, 3>(p, tl, stream);
    default: break;
    }
    set_error("integer kernel: update mode %d not built", tl.mode);
    return ECC_E_UNSUPPORTED;
}

template <typename T, int M, int NIN>
static int launch_rows(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    switch (tl.rows) {
    case 2: return launch_mode<T, M, NIN, 2>(p, tl, stream);
    case 4: return launch_mode<T, M, NIN, 4>(p, tl, stream);
    default: break;
    }
    set_error("integer kernel: %d rows per wave not built", tl.rows);
    return ECC_E_UNSUPPORTED;
}

// Transformed values (largest-value convention, 16-bit windows): walking
// mode 0, the tiling's planes of look-ahead.
template <typename T, int M, int NIN, int XF>
static int launch_transformed(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    const bool pd2 = tl.pd == 2;
    switch (tl.rows) {
    case 2: return pd2 ? launch_one<T, M, NIN, 2, 0, 2, XF>(p, tl, stream) : launch_one<T, M, NIN, 2, 0, 1, XF>(p, tl, stream);
    case 4: return pd2 ? launch_one<T, M, NIN, 4, 0, 2, XF>(p, tl, stream) : launch_one<T, M, NIN, 4, 0, 1, XF>(p, tl, stream);
    default: break;
    }
    set_error("integer kernel: %d rows per wave not built", tl.rows);
    return ECC_E_UNSUPPORTED;
}

// 16-bit values in a 32768-bin pass: two rows per wave, two planes of
// look-ahead (four rows would spill the lane masks of the range checks).
template <int NIN, int XF>
static int launch_range(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    if (tl.rows != 2 || tl.pd != 2) {
        set_error("integer kernel: 32768-bin passes take 2 rows and 2 planes of look-ahead (got %d, %d)", tl.rows,
                  tl.pd);
        return ECC_E_UNSUPPORTED;
    }
    return launch_one<uint16_t, 32768, NIN, 2, 0, 2, XF>(p, tl, stream);
}

static KParams make_params(const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status,
                           int64_t *zero_vcec) {
    KParams p{};
    p.src = job.src;
    p.n1 = job.view.n1;
    p.n2 = job.view.n2;
    p.e0 = job.e0;
    p.e1 = job.e1;
    p.lo_inf = job.lo_inf;
    p.hi_inf = job.hi_inf;
    p.zc = tl.zc;
    p.wx = tl.wx;
    p.wy = tl.wy;
    const int nin = job.view.nin;
    const int64_t xw = (int64_t)kWave * tl.wx * (nin == 1 ? tl.rows : 1);
    p.tiles_x = (int32_t)((job.view.n2 + xw - 1) / xw);
    p.tiles_y = nin == 1 ? 1 : (int32_t)((job.view.n1 + (int64_t)tl.rows * tl.wy - 1) / ((int64_t)tl.rows * tl.wy));
    p.tiles_z = (job.e1 - job.e0 + tl.zc - 1) / tl.zc;
    p.per_wg = tl.per_wg > 0 ? tl.per_wg : 1;
    p.tile_stride = tl.tile_stride;
    p.win_shift = job.win_shift;
    // row pairs need every row to start 4-byte aligned
    p.pair = nin == 2 && elem_bytes(job.dtype) == 2 && job.view.n2 % 2 == 0 &&
             ((uintptr_t)job.src.base & 3) == 0 && ((uintptr_t)job.src.lo_base & 3) == 0 && tl.pair != 0;
    p.partial = partial;
    p.status = status;
    p.zero_vcec = zero_vcec;
    p.high_flag = job.high_flag;
    return p;
}

int launch_int_partial(const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status,
                       int64_t *zero_vcec, hipStream_t stream) {
    const KParams p = make_params(job, tl, partial, status, zero_vcec);
    const int nin = job.view.nin;
    if (job.dtype == ECC_U16 && job.range_pass == 1)  // 32768 values from win_shift on: all of the image's
        return nin == 1 ? launch_range<1, kXfRange>(p, tl, stream) : launch_range<2, kXfRange>(p, tl, stream);
    if (job.dtype == ECC_U16 && job.range_pass == 2)  // the same, values outside masked off
        return nin == 1 ? launch_range<1, kXfRangeMasked>(p, tl, stream)
                        : launch_range<2, kXfRangeMasked>(p, tl, stream);
    if (job.dtype == ECC_U16)  // one window of 16382 values per launch
        return nin == 1 ? launch_transformed<uint16_t, 16384, 1, kXfWindow>(p, tl, stream)
                        : launch_transformed<uint16_t, 16384, 2, kXfWindow>(p, tl, stream);
    if (job.invert) {
        if (job.dtype == ECC_U8)
            return nin == 1 ? launch_transformed<uint8_t, 256, 1, kXfInvert>(p, tl, stream)
                            : launch_transformed<uint8_t, 256, 2, kXfInvert>(p, tl, stream);
        if (job.dtype == ECC_U14)
            return nin == 1 ? launch_transformed<uint16_t, 16384, 1, kXfInvert>(p, tl, stream)
                            : launch_transformed<uint16_t, 16384, 2, kXfInvert>(p, tl, stream);
    }
    if (job.dtype == ECC_U8)
        return nin == 1 ? launch_rows<uint8_t, 256, 1>(p, tl, stream) : launch_rows<uint8_t, 256, 2>(p, tl, stream);
    if (job.dtype == ECC_U14)
        return nin == 1 ? launch_rows<uint16_t, 16384, 1>(p, tl, stream)
                        : launch_rows<uint16_t, 16384, 2>(p, tl, stream);
    set_error("integer kernel: unsupported dtype %d", job.dtype);
    return ECC_E_UNSUPPORTED;
}

size_t kparams_bytes() { return sizeof(KParams); }

void fill_kparams(void *dst, const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status) {
    const KParams p = make_params(job, tl, partial, status, nullptr);
    memcpy(dst, &p, sizeof p);
}

int launch_int_persistent(const void *table_dev, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(int_vcec_persistent_kernel, dim3(grid), dim3(1024), 0, stream, (uint8_t *)table_dev);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

}  // namespace ecc
