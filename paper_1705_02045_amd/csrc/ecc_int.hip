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

__device__ __forceinline__ const uint8_t *plane_ptr(const PlaneSrc &s, int64_t p) {
    return p < s.seg0_planes ? s.seg0 + p * s.plane_bytes : s.seg1 + (p - s.seg0_planes) * s.plane_bytes;
}

// Fourth word of a raw buffer resource on gfx9-family parts (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;

// Value -> LDS byte offset of its bin, in 16-bit arithmetic (a 16-bit op
// leaves the upper half of the register zero on gfx950).  For 14-bit data
// stored in 16 bits the offset wraps modulo 65536, so a bad input can never
// address outside the histogram; such inputs are reported through the status
// word instead.  kInf compares above every offset (offsets are <= 0xFFFC).
using u16 = uint16_t;
constexpr u16 kInf = 0xFFFF;

__device__ __forceinline__ u16 bin_off(u16 v) { return (u16)(v << 2); }
__device__ __forceinline__ u16 min16(u16 a, u16 b) { return a < b ? a : b; }

__device__ __forceinline__ u16 load_elem(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, int esz) {
    if (esz == 1) return (u16)__builtin_amdgcn_raw_buffer_load_b8(rs, voff, soff, 0);
    return (u16)__builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0);
}

__device__ __forceinline__ bool lanes(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

template <int NIN, int R>
struct Walker {
    static constexpr int K = 1 << NIN;                 // fields per row
    static constexpr int NR = (NIN == 2) ? R + 1 : R;  // loaded rows per plane

    // Fields of one plane.  a[rr], b[rr]: raw values at x and at x-1 (clamped)
    // of loaded row rr (NIN == 2: rr = 0 is the collar row y0-1).
    static __device__ __forceinline__ void fields(const u16 (&a)[NR], const u16 (&b)[NR], u16 (&g)[R][K]) {
        if constexpr (NIN == 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                g[r][0] = bin_off(a[r]);
                g[r][1] = bin_off(min16(a[r], b[r]));
            }
        } else {
            u16 f0[NR], fx[NR];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                f0[rr] = bin_off(a[rr]);
                fx[rr] = bin_off(min16(a[rr], b[rr]));
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                g[r][0] = f0[r + 1];
                g[r][1] = fx[r + 1];
                g[r][2] = min16(f0[r], f0[r + 1]);
                g[r][3] = min16(fx[r], fx[r + 1]);
            }
        }
    }

    static __device__ __forceinline__ void set_inf(u16 (&g)[R][K]) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k) g[r][k] = kInf;
    }

    static constexpr int sign(int k) {
        // (-1)^(NIN - |S|), S encoded by the bits of k (bit 0: x, bit 1: y)
        return (((NIN - __builtin_popcount(k)) & 1) ? -1 : 1);
    }
};

// Validity of field k of row r in a wave that touches the far edge of an
// in-plane axis: positions x <= n2-2 (fields without x) or x < n2 (with x),
// rows y <= n1-2 (fields without y) or y < n1 (with y).  The lane masks are
// per wave; the row conditions are wave-uniform.
struct EdgeMasks {
    uint64_t lx_int;  // lanes with x <= n2-2
    uint64_t lx_any;  // lanes with x <  n2
    uint32_t ry_int;  // bit r: row r has y <= n1-2
    uint32_t ry_any;  // bit r: row r has y <  n1
};

template <int NIN>
__device__ __forceinline__ uint64_t edge_mask(const EdgeMasks &em, int r, int k) {
    const uint64_t lm = (k & 1) ? em.lx_any : em.lx_int;
    if constexpr (NIN == 1) return lm;
    const uint32_t rb = (k & 2) ? em.ry_any : em.ry_int;
    return ((rb >> r) & 1u) ? lm : 0ull;
}

// One wave walks the planes [zs, ze) of its rows.  FULL: no position of this
// wave lies on a far edge, so the comparison masks need no validity mask.
template <typename T, int NIN, int R, bool FULL>
__device__ __forceinline__ void walk(const KParams &P, char *hbytes, int zs, int ze, const uint32_t (&voff)[2][R + 1],
                                     const uint32_t (&soff)[R + 1], const EdgeMasks &em, uint32_t &orv) {
    using W = Walker<NIN, R>;
    constexpr int K = W::K;
    constexpr int NR = W::NR;
    constexpr int ESZ = sizeof(T);
    const int32_t pbytes = (int32_t)P.src.plane_bytes;

    auto is_real = [&](int p) { return !((p == P.e0 - 1 && P.lo_inf) || (p == P.e1 && P.hi_inf)); };
    auto load_plane = [&](int p, u16 (&a)[NR], u16 (&b)[NR]) {
        const uint8_t *pp = plane_ptr(P.src, p);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)pp, (short)0, pbytes, kBufferWord3);
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            a[rr] = load_elem(rs, voff[0][rr], soff[rr], ESZ);
            b[rr] = load_elem(rs, voff[1][rr], soff[rr], ESZ);
        }
    };
    auto range_acc = [&](const u16 (&a)[NR]) {
        // rows owned by this wave (the collar row is checked by its owner)
#pragma unroll
        for (int rr = NR - R; rr < NR; ++rr) orv |= a[rr];
    };
    auto cmp = [&](u16 lo, u16 hi, int r, int k) -> uint64_t {
        const uint64_t c = __builtin_amdgcn_ballot_w64(lo < hi);
        if constexpr (FULL) return c;
        else return c & edge_mask<NIN>(em, r, k);
    };
    // Compare plane z+1 (gn) with plane z (gc), add the changes of plane z.
    auto step = [&](const u16 (&gc)[R][K], const u16 (&gn)[R][K], uint64_t (&cp)[R][K]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t c = cmp(gn[r][k], gc[r][k], r, k);
                if (lanes(c ^ cp[r][k])) {
                    const int s = W::sign(k);
                    const int e = lanes(cp[r][k]) ? s : -s;
                    __hip_atomic_fetch_add((int32_t *)__builtin_assume_aligned(hbytes + (uint32_t)gc[r][k], 4), e,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                cp[r][k] = c;
            }
        }
    };

    u16 g0[R][K], g1[R][K];
    uint64_t cp[R][K];
    u16 a0[NR], b0[NR], a1[NR], b1[NR];

    // g1 <- plane zs-1 (or +inf), g0 <- plane zs, cp <- [g0 < g1]
    if (is_real(zs - 1)) {
        load_plane(zs - 1, a0, b0);
        W::fields(a0, b0, g1);
    } else {
        W::set_inf(g1);
    }
    load_plane(zs, a1, b1);
    W::fields(a1, b1, g0);
    range_acc(a1);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < K; ++k) cp[r][k] = cmp(g0[r][k], g1[r][k], r, k);

    // Two planes per iteration so that the roles of (g0, a0/b0) and (g1,
    // a1/b1) alternate without register copies.  Invariant at the top: g0
    // holds plane z, a0/b0 hold the raw values of plane z+1 (when real).
    if (is_real(zs + 1)) load_plane(zs + 1, a0, b0);
    int z = zs;
    for (; z + 1 < ze; z += 2) {
        if (is_real(z + 2)) load_plane(z + 2, a1, b1);
        if (is_real(z + 1)) {
            W::fields(a0, b0, g1);
            range_acc(a0);
        } else {
            W::set_inf(g1);
        }
        step(g0, g1, cp);
        if (z + 3 <= ze && is_real(z + 3)) load_plane(z + 3, a0, b0);
        if (is_real(z + 2)) {
            W::fields(a1, b1, g0);
            range_acc(a1);
        } else {
            W::set_inf(g0);
        }
        step(g1, g0, cp);
    }
    if (z < ze) {
        if (is_real(z + 1)) {
            W::fields(a0, b0, g1);
            range_acc(a0);
        } else {
            W::set_inf(g1);
        }
        step(g0, g1, cp);
    }
}

template <typename T, int M, int NIN, int R>
__global__ void __launch_bounds__(1024) int_vcec_kernel(KParams P) {
    using W = Walker<NIN, R>;
    constexpr int NR = W::NR;
    constexpr int ESZ = sizeof(T);
    __shared__ int32_t hist[M];

    const int tid = threadIdx.x;
    for (int i = tid; i < M; i += blockDim.x) hist[i] = 0;
    __syncthreads();

    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wxi = wave % P.wx;
    const int wyi = wave / P.wx;
    const int32_t n1 = P.n1, n2 = P.n2;
    char *hbytes = reinterpret_cast<char *>(hist);

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
        // and the row's byte offset within a plane.
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
            // NIN == 1 keeps one lane mask per segment in lx_*: segments past
            // the first edge segment are entirely beyond the row.
            em.lx_int = 0; em.lx_any = 0;
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
            em.lx_int = __builtin_amdgcn_ballot_w64(x <= n2 - 2);
            em.lx_any = __builtin_amdgcn_ballot_w64(x < n2);
            em.ry_int = 0; em.ry_any = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                em.ry_int |= (uint32_t)(y0 + r <= n1 - 2) << r;
                em.ry_any |= (uint32_t)(y0 + r < n1) << r;
            }
        }
        if (!any) continue;
        if (full) {
            walk<T, NIN, R, true>(P, hbytes, zs, ze, voff, soff, em, orv);
        } else if constexpr (NIN == 1) {
            // Segment-by-segment masks: walk each 64-wide segment of the edge
            // group on its own so that one lane mask pair describes it.
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int32_t x = ((tx * P.wx + wxi) * R + r) * kWave + lane;
                if (((tx * P.wx + wxi) * R + r) * kWave >= n2) break;
                EdgeMasks e1{};
                e1.lx_int = __builtin_amdgcn_ballot_w64(x <= n2 - 2);
                e1.lx_any = __builtin_amdgcn_ballot_w64(x < n2);
                uint32_t vo1[2][2] = {{voff[0][r], voff[0][r]}, {voff[1][r], voff[1][r]}};
                uint32_t so1[2] = {0, 0};
                walk<T, NIN, 1, false>(P, hbytes, zs, ze, vo1, so1, e1, orv);
            }
        } else {
            walk<T, NIN, R, false>(P, hbytes, zs, ze, voff, soff, em, orv);
        }
    }

    if constexpr (M != 256) {
        if (orv >= (uint32_t)M) atomicOr(P.status, kStatusRange);
    }
    __syncthreads();
    int32_t *dst = P.partial + (size_t)blockIdx.x * M;
    for (int i = tid; i < M; i += blockDim.x) dst[i] = hist[i];
}

template <typename T, int M, int NIN, int R>
static int launch_one(const KParams &p, const IntTiling &tl, hipStream_t stream) {
    const int threads = kWave * tl.wx * tl.wy;
    void *tok = nullptr;
    int rc = profile_begin(stream, &tok);
    if (rc) return rc;
    hipLaunchKernelGGL((int_vcec_kernel<T, M, NIN, R>), dim3(tl.grid), dim3(threads), 0, stream, p);
    ECC_HIP(hipGetLastError());
    return profile_end(stream, tok);
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
    if (tl.rows != 4) {
        set_error("integer kernel: unsupported rows per wave %d", tl.rows);
        return ECC_E_UNSUPPORTED;
    }
    if (job.dtype == ECC_U8) {
        return nin == 1 ? launch_one<uint8_t, 256, 1, 4>(p, tl, stream)
                        : launch_one<uint8_t, 256, 2, 4>(p, tl, stream);
    }
    if (job.dtype == ECC_U14) {
        return nin == 1 ? launch_one<uint16_t, 16384, 1, 4>(p, tl, stream)
                        : launch_one<uint16_t, 16384, 2, 4>(p, tl, stream);
    }
    set_error("integer kernel: unsupported dtype %d", job.dtype);
    return ECC_E_UNSUPPORTED;
}

}  // namespace ecc
