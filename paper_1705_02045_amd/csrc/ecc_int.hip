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

#include "ecc_internal.h"

namespace ecc {

struct KParams {
    PlaneSrc src;
    int32_t n1, n2;
    int32_t e0, e1;
    int32_t lo_inf, hi_inf;
    int32_t zc;
    int32_t tiles_x, tiles_y, tiles_z;
    int32_t wx, wy;
    int32_t *partial;
    uint32_t *status;
};

__device__ __forceinline__ const uint8_t *plane_ptr(const PlaneSrc &s, int32_t p) {
    return p < (int32_t)s.seg0_planes ? s.seg0 + (int64_t)p * s.plane_bytes
                                      : s.seg1 + (int64_t)(p - (int32_t)s.seg0_planes) * s.plane_bytes;
}

// Fourth word of a raw buffer resource on gfx9-family parts (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;

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

// v: zero-extended 16-bit value
__device__ __forceinline__ uint32_t bin_off(uint32_t v) {
    uint32_t r;
    asm("v_pk_lshlrev_b16 %0, 2, %1" : "=v"(r) : "v"(v));
    return r;
}
// a, b: zero-extended 16-bit values
__device__ __forceinline__ uint32_t bin_off_min(uint32_t a, uint32_t b) {
    uint32_t m, r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(a), "v"(b));
    asm("v_pk_lshlrev_b16 %0, 2, %1" : "=v"(r) : "v"(m));
    return r;
}
// Both inputs are zero-extended offsets, so a 32-bit minimum is exact.
__device__ __forceinline__ uint32_t min_off(uint32_t a, uint32_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint32_t load_elem(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, int esz) {
    if (esz == 1) return __builtin_amdgcn_raw_buffer_load_b8(rs, voff, soff, 0);
    return __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0);
}

__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// ----------------------------------------------------------------------------
// Histogram updates of four (row, field) items at once.  For item i the lanes
// whose ownership flag flips between planes (p_i != c_i) add
// e = (p_i ? s_i : -s_i) at byte offset g_i.  The block sets EXEC directly
// from the two lane masks and restores it before returning, so the compiler
// never sees a modified EXEC.  Per item either
//   CND: one v_cndmask builds +-1 and one ds_add covers both directions, or
//   DBL: two masked ds_adds with the constant registers +1 / -1 (no VALU).
// The histogram is the kernel's only LDS object, at LDS address 0, so the bin
// offsets are LDS addresses.  The scalar ops of the block write SCC, which is
// therefore declared clobbered: the compiler must not keep a comparison
// result in SCC across the block.
#define ECC_CND(i, NEG, POS)                                                                   \
    "s_xor_b64 exec, %[c" #i "], %[p" #i "]\n\t"                                               \
    "v_cndmask_b32_e64 %[t" #i "], " NEG ", " POS ", %[p" #i "]\n\t"                           \
    "ds_add_u32 %[g" #i "], %[t" #i "]\n\t"
#define ECC_DBL(i, PFLIP, CFLIP)                                                              \
    "s_andn2_b64 exec, %[p" #i "], %[c" #i "]\n\t"                                             \
    "ds_add_u32 %[g" #i "], %[" PFLIP "]\n\t"                                                  \
    "s_andn2_b64 exec, %[c" #i "], %[p" #i "]\n\t"                                             \
    "ds_add_u32 %[g" #i "], %[" CFLIP "]\n\t"
// sign +1: p=1,c=0 -> +1 ; sign -1: p=1,c=0 -> -1
#define ECC_CNDP(i) ECC_CND(i, "-1", "1")
#define ECC_CNDM(i) ECC_CND(i, "1", "-1")
#define ECC_DBLP(i) ECC_DBL(i, "one", "mone")
#define ECC_DBLM(i) ECC_DBL(i, "mone", "one")

#define ECC_UPD_ASM(BODY)                                                                      \
    asm volatile("s_mov_b64 %[sv], exec\n\t" BODY "s_mov_b64 exec, %[sv]"                      \
                 : [sv] "=&s"(sv), [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3) \
                 : [g0] "v"(g0), [g1] "v"(g1), [g2] "v"(g2), [g3] "v"(g3), [c0] "s"(c0), [c1] "s"(c1), \
                   [c2] "s"(c2), [c3] "s"(c3), [p0] "s"(p0), [p1] "s"(p1), [p2] "s"(p2), [p3] "s"(p3),  \
                   [one] "v"(one), [mone] "v"(mone)                                             \
                 : "memory", "scc")

// SIGNS: bit i set = item i has sign -1.  DBL: bit i set = item i uses DBL.
template <int SIGNS, int DBL>
__device__ __forceinline__ void update4(uint32_t g0, uint32_t g1, uint32_t g2, uint32_t g3, uint64_t c0, uint64_t c1,
                                        uint64_t c2, uint64_t c3, uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3,
                                        uint32_t one, uint32_t mone) {
    uint64_t sv;
    uint32_t t0, t1, t2, t3;
    // NIN == 2 signs (+,-,-,+) = 0b0110; NIN == 1 signs (-,+,-,+) = 0b0101.
    if constexpr (SIGNS == 0b0110 && DBL == 0b0000) {
        ECC_UPD_ASM(ECC_CNDP(0) ECC_CNDM(1) ECC_CNDM(2) ECC_CNDP(3));
    } else if constexpr (SIGNS == 0b0110 && DBL == 0b0110) {
        ECC_UPD_ASM(ECC_CNDP(0) ECC_DBLM(1) ECC_DBLM(2) ECC_CNDP(3));
    } else if constexpr (SIGNS == 0b0110 && DBL == 0b1001) {
        ECC_UPD_ASM(ECC_DBLP(0) ECC_CNDM(1) ECC_CNDM(2) ECC_DBLP(3));
    } else if constexpr (SIGNS == 0b0110 && DBL == 0b1111) {
        ECC_UPD_ASM(ECC_DBLP(0) ECC_DBLM(1) ECC_DBLM(2) ECC_DBLP(3));
    } else if constexpr (SIGNS == 0b0101 && DBL == 0b0000) {
        ECC_UPD_ASM(ECC_CNDM(0) ECC_CNDP(1) ECC_CNDM(2) ECC_CNDP(3));
    } else if constexpr (SIGNS == 0b0101 && DBL == 0b1111) {
        ECC_UPD_ASM(ECC_DBLM(0) ECC_DBLP(1) ECC_DBLM(2) ECC_DBLP(3));
    } else if constexpr (SIGNS == 0b0101 && DBL == 0b0101) {
        ECC_UPD_ASM(ECC_DBLM(0) ECC_CNDP(1) ECC_DBLM(2) ECC_CNDP(3));
    } else {
        static_assert(SIGNS < 0, "update4: combination not instantiated");
    }
}

template <int NIN, int R>
struct Walker {
    static constexpr int K = 1 << NIN;                 // fields per row
    static constexpr int NR = (NIN == 2) ? R + 1 : R;  // loaded rows per plane
    static constexpr int NI = R * K;                   // (row, field) items per plane
    static_assert(NI % 4 == 0, "items come in groups of four");

    // Fields of one plane, flattened as item i = r*K + k.  a[rr], b[rr]: raw
    // values at x and at x-1 (clamped) of loaded row rr (NIN == 2: rr = 0 is
    // the collar row y0-1).
    static __device__ __forceinline__ void fields(const uint32_t (&a)[NR], const uint32_t (&b)[NR],
                                                  uint32_t (&g)[NI]) {
        if constexpr (NIN == 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                g[2 * r + 0] = bin_off(a[r]);
                g[2 * r + 1] = bin_off_min(a[r], b[r]);
            }
        } else {
            uint32_t f0[NR], fx[NR];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                f0[rr] = bin_off(a[rr]);
                fx[rr] = bin_off_min(a[rr], b[rr]);
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

    static __device__ __forceinline__ void set_inf(uint32_t (&g)[NI]) {
#pragma unroll
        for (int i = 0; i < NI; ++i) g[i] = kInf;
    }

    static constexpr int kSigns = (NIN == 2) ? 0b0110 : 0b0101;
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

// One wave walks the planes [zs, ze) of its rows.  FULL: no position of this
// wave lies on a far edge, so the comparison masks need no validity mask.
template <typename T, int NIN, int R, int DBL, bool FULL>
__device__ __forceinline__ void walk(const KParams &P, int zs, int ze, const uint32_t (&voff)[2][R + 1],
                                     const uint32_t (&soff)[R + 1], const EdgeMasks &em, uint32_t &orv) {
    using W = Walker<NIN, R>;
    constexpr int NR = W::NR;
    constexpr int NI = W::NI;
    constexpr int ESZ = sizeof(T);
    const int32_t pbytes = (int32_t)P.src.plane_bytes;
    const uint32_t one = 1u, mone = 0xFFFFFFFFu;
    // planes zs-1 and ze are +inf outside the image
    const bool lo_real = !(zs == P.e0 && P.lo_inf);
    const bool hi_real = !(ze == P.e1 && P.hi_inf);

    auto load_plane = [&](int p, uint32_t (&a)[NR], uint32_t (&b)[NR]) {
        const uint8_t *pp = plane_ptr(P.src, p);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)pp, (short)0, pbytes, kBufferWord3);
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            a[rr] = load_elem(rs, voff[0][rr], soff[rr], ESZ);
            b[rr] = load_elem(rs, voff[1][rr], soff[rr], ESZ);
        }
    };
    auto range_acc = [&](const uint32_t (&a)[NR]) {
        // rows owned by this wave (the collar row is checked by its owner)
#pragma unroll
        for (int rr = NR - R; rr < NR; ++rr) orv |= a[rr];
    };
    auto cmp = [&](uint32_t lo, uint32_t hi, int i) -> uint64_t {
        const uint64_t c = ballot(lo < hi);
        if constexpr (FULL) return c;
        else return c & edge_mask<NIN>(em, i);
    };
    // Compare plane z+1 (gn) with plane z (gc) and add the changes of plane z.
    auto step = [&](const uint32_t (&gc)[NI], const uint32_t (&gn)[NI], uint64_t (&cp)[NI]) {
#pragma unroll
        for (int i = 0; i < NI; i += 4) {
            const uint64_t c0 = cmp(gn[i], gc[i], i), c1 = cmp(gn[i + 1], gc[i + 1], i + 1);
            const uint64_t c2 = cmp(gn[i + 2], gc[i + 2], i + 2), c3 = cmp(gn[i + 3], gc[i + 3], i + 3);
            update4<W::kSigns, DBL>(gc[i], gc[i + 1], gc[i + 2], gc[i + 3], c0, c1, c2, c3, cp[i], cp[i + 1],
                                    cp[i + 2], cp[i + 3], one, mone);
            cp[i] = c0;
            cp[i + 1] = c1;
            cp[i + 2] = c2;
            cp[i + 3] = c3;
        }
    };
    // fields of plane p from raw (a, b), or +inf for the plane past the end
    auto next_fields = [&](int p, const uint32_t (&a)[NR], const uint32_t (&b)[NR], uint32_t (&g)[NI]) {
        if (p < ze || hi_real) {
            W::fields(a, b, g);
            if (p < ze) range_acc(a);
        } else {
            W::set_inf(g);
        }
    };

    uint32_t g0[NI], g1[NI];
    uint64_t cp[NI];
    uint32_t a0[NR], b0[NR], a1[NR], b1[NR];

    // g1 <- plane zs-1 (or +inf), g0 <- plane zs, cp <- [g0 < g1]
    if (lo_real) {
        load_plane(zs - 1, a0, b0);
        W::fields(a0, b0, g1);
    } else {
        W::set_inf(g1);
    }
    load_plane(zs, a1, b1);
    W::fields(a1, b1, g0);
    range_acc(a1);
#pragma unroll
    for (int i = 0; i < NI; ++i) cp[i] = cmp(g0[i], g1[i], i);

    // Invariant at the top of each iteration: g0 holds plane z, a0/b0 hold
    // the raw values of plane z+1.  Two planes per iteration so that the roles
    // of (g0, a0/b0) and (g1, a1/b1) alternate without register copies.  The
    // steady-state loop runs while planes z+1..z+3 are inside the tile, so it
    // has no boundary tests; the last planes are done after it.
    if (zs + 1 < ze || hi_real) load_plane(zs + 1, a0, b0);
    int z = zs;
    for (; z + 3 < ze; z += 2) {
        load_plane(z + 2, a1, b1);
        W::fields(a0, b0, g1);
        range_acc(a0);
        step(g0, g1, cp);
        load_plane(z + 3, a0, b0);
        W::fields(a1, b1, g0);
        range_acc(a1);
        step(g1, g0, cp);
    }
    // at most three planes left: z, z+1, z+2 (< ze)
    if (z < ze) {
        if (z + 2 < ze || (z + 2 == ze && hi_real)) load_plane(z + 2, a1, b1);
        next_fields(z + 1, a0, b0, g1);
        step(g0, g1, cp);
        ++z;
        if (z < ze) {
            if (z + 2 < ze || (z + 2 == ze && hi_real)) load_plane(z + 2, a0, b0);
            next_fields(z + 1, a1, b1, g0);
            step(g1, g0, cp);
            ++z;
            if (z < ze) {
                next_fields(z + 1, a0, b0, g1);
                step(g0, g1, cp);
            }
        }
    }
}

template <typename T, int M, int NIN, int R, int DBL>
__global__ void __launch_bounds__(1024) int_vcec_kernel(KParams P) {
    using W = Walker<NIN, R>;
    constexpr int NR = W::NR;
    constexpr int NI = W::NI;
    constexpr int ESZ = sizeof(T);
    __shared__ int32_t hist[M];

    const int tid = threadIdx.x;
    // The update blocks address bins by their LDS byte offset: the histogram
    // must sit at LDS address 0 (it is this kernel's only LDS object).
    if ((uint32_t)(size_t)(__attribute__((address_space(3))) int32_t *)hist != 0u) {
        if (tid == 0) atomicOr(P.status, 0x80000000u);
        return;
    }
    for (int i = tid; i < M; i += blockDim.x) hist[i] = 0;
    __syncthreads();

    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wxi = wave % P.wx;
    const int wyi = wave / P.wx;
    const int32_t n1 = P.n1, n2 = P.n2;

    // Tiles handed out so that the workgroups resident on one XCD (blockIdx
    // mod 8 under round-robin dispatch) work on neighbouring tiles, which share
    // collar rows and planes through that XCD's L2.
    const int ntiles = P.tiles_x * P.tiles_y * P.tiles_z;
    int t0, tstep, tend;
    if ((gridDim.x & 7) == 0 && ntiles >= (int)gridDim.x) {
        const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3, per = gridDim.x >> 3;
        t0 = (int)((int64_t)ntiles * xcd / 8) + j;
        tend = (int)((int64_t)ntiles * (xcd + 1) / 8);
        tstep = per;
    } else {
        t0 = blockIdx.x;
        tend = ntiles;
        tstep = gridDim.x;
    }

    uint32_t orv = 0;
    for (int t = t0; t < tend; t += tstep) {
        const int tx = t % P.tiles_x;
        const int ty = (t / P.tiles_x) % P.tiles_y;
        const int tz = t / (P.tiles_x * P.tiles_y);
        const int zs = P.e0 + tz * P.zc;
        const int ze = min(zs + P.zc, P.e1);
        if (zs >= ze) continue;

        // Byte offsets of x and of x-1 (clamped into the row) per loaded row,
        // the row's byte offset within a plane, and the edge masks.
        uint32_t voff[2][R + 1] = {};
        uint32_t soff[R + 1] = {};
        EdgeMasks em{};
        bool full, any;
        if constexpr (NIN == 1) {
            const int32_t seg0 = (tx * P.wx + wxi) * R;
            any = seg0 * kWave < n2;
            full = (seg0 + R) * kWave - 1 <= n2 - 2;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int32_t x = (seg0 + r) * kWave + lane;
                const int32_t xcl = min(x, n2 - 1);
                voff[0][r] = (uint32_t)xcl * ESZ;
                voff[1][r] = (uint32_t)(xcl > 0 ? xcl - 1 : 0) * ESZ;
                soff[r] = 0;
            }
        } else {
            const int32_t x0 = (tx * P.wx + wxi) * kWave;
            const int32_t x = x0 + lane;
            const int32_t y0 = (ty * P.wy + wyi) * R;
            any = x0 < n2 && y0 < n1;
            full = (x0 + kWave - 1 <= n2 - 2) && (y0 + R - 1 <= n1 - 2);
            const int32_t xcl = min(x, n2 - 1);
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                voff[0][rr] = (uint32_t)xcl * ESZ;
                voff[1][rr] = (uint32_t)(xcl > 0 ? xcl - 1 : 0) * ESZ;
                const int32_t y = min(max(y0 + rr - 1, 0), n1 - 1);
                soff[rr] = (uint32_t)y * (uint32_t)n2 * ESZ;
            }
            em.lx_int = ballot(x <= n2 - 2);
            em.lx_any = ballot(x < n2);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                em.ry_int |= (uint32_t)(y0 + r <= n1 - 2) << r;
                em.ry_any |= (uint32_t)(y0 + r < n1) << r;
            }
        }
        if (!any) continue;
        if (full) {
            walk<T, NIN, R, DBL, true>(P, zs, ze, voff, soff, em, orv);
        } else if constexpr (NIN == 1) {
            // An edge group of segments is walked as pairs of segments, each
            // with its own lane masks.
#pragma unroll
            for (int r = 0; r < R; r += 2) {
                const int32_t xs = ((tx * P.wx + wxi) * R + r) * kWave;
                if (xs >= n2) break;
                const int32_t xa = xs + lane, xb = xs + kWave + lane;
                EdgeMasks e2{};
                e2.lx_int = ballot(xa <= n2 - 2);
                e2.lx_any = ballot(xa < n2);
                e2.lx_int2 = ballot(xb <= n2 - 2);
                e2.lx_any2 = ballot(xb < n2);
                const uint32_t vo[2][3] = {{voff[0][r], voff[0][r + 1], 0u}, {voff[1][r], voff[1][r + 1], 0u}};
                const uint32_t so[3] = {0u, 0u, 0u};
                walk<T, 1, 2, DBL, false>(P, zs, ze, vo, so, e2, orv);
            }
        } else {
            walk<T, NIN, R, DBL, false>(P, zs, ze, voff, soff, em, orv);
        }
    }

    if constexpr (M != 256) {
        if (orv >= (uint32_t)M) atomicOr(P.status, kStatusRange);
    }
    // the update blocks' LDS adds are not tracked by the compiler's counters
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
    int32_t *dst = P.partial + (size_t)blockIdx.x * M;
    for (int i = tid; i < M; i += blockDim.x) dst[i] = hist[i];
}

template <typename T, int M, int NIN, int R, int DBL>
static int launch_one(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    const int threads = kWave * tl.wx * tl.wy;
    void *tok = nullptr;
    int rc = profile_begin(stream, &tok);
    if (rc) return rc;
    hipLaunchKernelGGL((int_vcec_kernel<T, M, NIN, R, DBL>), dim3(tl.grid), dim3(threads), 0, stream, p);
    ECC_HIP(hipGetLastError());
    return profile_end(stream, tok);
}

template <typename T, int M, int NIN, int R>
static int launch_dbl(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    if constexpr (NIN == 2) {
        switch (tl.dbl) {
        case 0b0000: return launch_one<T, M, NIN, R, 0b0000>(p, tl, stream);
        case 0b0110: return launch_one<T, M, NIN, R, 0b0110>(p, tl, stream);
        case 0b1001: return launch_one<T, M, NIN, R, 0b1001>(p, tl, stream);
        case 0b1111: return launch_one<T, M, NIN, R, 0b1111>(p, tl, stream);
        default: break;
        }
    } else {
        switch (tl.dbl) {
        case 0b0000: return launch_one<T, M, NIN, R, 0b0000>(p, tl, stream);
        case 0b0101: return launch_one<T, M, NIN, R, 0b0101>(p, tl, stream);
        case 0b1111: return launch_one<T, M, NIN, R, 0b1111>(p, tl, stream);
        default: break;
        }
    }
    set_error("integer kernel: update mode %d not built", tl.dbl);
    return ECC_E_UNSUPPORTED;
}

template <typename T, int M, int NIN>
static int launch_rows(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    switch (tl.rows) {
    case 2: return launch_dbl<T, M, NIN, 2>(p, tl, stream);
    case 4: return launch_dbl<T, M, NIN, 4>(p, tl, stream);
    default: break;
    }
    set_error("integer kernel: %d rows per wave not built", tl.rows);
    return ECC_E_UNSUPPORTED;
}

int launch_int_partial(const IntJob &job, const IntTiling &tl, int32_t *partial, uint32_t *status,
                       hipStream_t stream) {
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
    p.partial = partial;
    p.status = status;
    if (job.dtype == ECC_U8)
        return nin == 1 ? launch_rows<uint8_t, 256, 1>(p, tl, stream) : launch_rows<uint8_t, 256, 2>(p, tl, stream);
    if (job.dtype == ECC_U14)
        return nin == 1 ? launch_rows<uint16_t, 16384, 1>(p, tl, stream)
                        : launch_rows<uint16_t, 16384, 2>(p, tl, stream);
    set_error("integer kernel: unsupported dtype %d", job.dtype);
    return ECC_E_UNSUPPORTED;
}

}  // namespace ecc
