/*
 * Seeded synthetic image generators, device side: the integer value-noise
 * family of eccgen_host.c restated for the GPU, producing the same bytes, for
 * images generated one range of axis-0 planes at a time in device memory
 * (volumes larger than host or device memory, made slab by slab where they
 * are consumed).
 *
 * This module only produces input bytes and holds none of the Euler
 * characteristic arithmetic.  Definitions (as in eccgen_host.c):
 *   mix64, key(seed, stream), h(seed, stream, i) = mix64(key + (i + 1) * GAMMA)
 *   U(node) = h(seed, 1, node_linear) >> (64 - bits), node grid
 *             N_k = ((n_k - 1) >> lshift) + 2 per axis, C order;
 *   base    = (sum over the 2^d lattice corners of U * prod_k w_k + L^d / 2)
 *             >> (d * lshift), w_k = L - r_k or r_k, r_k = p_k mod L;
 *   J       = (((h(seed, 2, i) >> 32) * (2A + 1)) >> 32) - A, i = the voxel's
 *             C-order index in the whole image;
 *   v       = clamp(base + J, 0, 2^bits - 1).
 * Neither the node index nor i depends on n_0, so planes [z0, z1) of an image
 * are the same bytes whatever its number of planes.
 *
 * Layout: 3-D only, bits + 2 * lshift <= 24.  Two kernels per call:
 *   lattice: the U values of the node planes that [z0, z1) touches, as a
 *            uint16 table [nzn][N1][N2] (caller's device buffer);
 *   voxels:  each thread makes two x-neighbours of one row (same lattice
 *            cell, since L >= 2 and x is even): the (z, y)-bilinear sums at
 *            the cell's two x nodes, then one x interpolation per voxel.
 *            Integer sums are exact, so the grouping does not change a value.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

namespace {

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t key_of(uint64_t seed, uint64_t stream) { return mix64(seed * GAMMA + stream); }

__global__ void __launch_bounds__(256) lattice_kernel(uint64_t key1, int shift, uint64_t node0, int64_t count,
                                                      uint16_t *__restrict__ table) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        table[i] = (uint16_t)(mix64(key1 + (node0 + (uint64_t)i + 1) * GAMMA) >> shift);
}

// High 32 bits of mix64(z): only they feed the jitter.  The last product is
// formed for its high word only: (z ^ (z >> 31)) >> 32 = h ^ (h >> 31) with
// h = (z >> 32).
__device__ inline uint32_t mix64_hi(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = z ^ (z >> 27);
    const uint32_t lo = (uint32_t)z, hi = (uint32_t)(z >> 32);
    const uint32_t h = __umulhi(lo, 0x133111EBu) + lo * 0x94D049BBu + hi * 0x133111EBu;
    return h ^ (h >> 31);
}

struct VoxArgs {
    const uint16_t *table;
    uint64_t key2;
    uint64_t row_step;  // GAMMA * n2 * gridDim.y: jitter counter advance per row iteration
    int32_t dq, dr;     // gridDim.y = dq * n1 + dr
    int64_t z0;      // first generated plane
    int64_t zn0;     // first node plane held by the table
    int64_t rows;    // (z1 - z0) * n1
    int32_t n1, n2;  // in-plane sizes
    int32_t N1, N2;  // in-plane node counts
    int32_t lshift;
    int32_t amp;
    int32_t maxv;
};

// ctr = key2 + (i + 1) * GAMMA for the voxel's C-order index i
template <typename T>
__device__ inline T finish_voxel(uint32_t acc, const VoxArgs &a, uint64_t ctr) {
    const int dl = 3 * a.lshift;
    const int32_t bv = (int32_t)((acc + (1u << (dl - 1))) >> dl);
    const int32_t jit = (int32_t)__umulhi(mix64_hi(ctr), (uint32_t)(2 * a.amp + 1)) - a.amp;
    int32_t v = bv + jit;
    v = v < 0 ? 0 : (v > a.maxv ? a.maxv : v);
    return (T)v;
}

// grid: x over pairs of one row, y strides over the rows of the slab
template <typename T, bool PAIRED_STORE>
__global__ void __launch_bounds__(256) voxel_kernel(VoxArgs a, T *__restrict__ out) {
    const int32_t x = 2 * (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x >= a.n2) return;
    const int32_t L = 1 << a.lshift;
    const int32_t xn = x >> a.lshift, rx = x & (L - 1);
    const bool two = x + 1 < a.n2;
    const int64_t plane_nodes = (int64_t)a.N1 * a.N2;
    // jitter counter of voxel (row, x): key2 + ((z0 * n1 + row) * n2 + x + 1) * GAMMA (mod 2^64)
    uint64_t ctr = a.key2 + (((uint64_t)a.z0 * (uint64_t)a.n1 + blockIdx.y) * (uint64_t)a.n2 + (uint64_t)x + 1) * GAMMA;
    // row = zr * n1 + y, advanced by gridDim.y = dq * n1 + dr per iteration
    int64_t zr = blockIdx.y / a.n1;
    int32_t y = (int32_t)(blockIdx.y % a.n1);
    for (int64_t row = blockIdx.y; row < a.rows; row += gridDim.y, ctr += a.row_step) {
        if (row != blockIdx.y) {
            zr += a.dq;
            y += a.dr;
            if (y >= a.n1) {
                y -= a.n1;
                ++zr;
            }
        }
        const int64_t z = a.z0 + zr;
        const int64_t zn = z >> a.lshift;
        const uint32_t rz = (uint32_t)(z & (L - 1));
        const int32_t yn = y >> a.lshift;
        const uint32_t ry = (uint32_t)(y & (L - 1));
        const uint16_t *t00 = a.table + ((zn - a.zn0) * a.N1 + yn) * (int64_t)a.N2 + xn;
        const uint16_t *t01 = t00 + a.N2;
        const uint16_t *t10 = t00 + plane_nodes;
        const uint16_t *t11 = t10 + a.N2;
        // every factor below is < 2^24 (values < 2^bits, weights <= 2^lshift,
        // bits + 2 * lshift <= 24), so the 24-bit multiplier gives the exact
        // 32-bit products
        const uint32_t wz0 = (uint32_t)L - rz, wz1 = rz, wy0 = (uint32_t)L - ry, wy1 = ry;
        const uint32_t s0 = __umul24(__umul24(t00[0], wy0) + __umul24(t01[0], wy1), wz0) +
                            __umul24(__umul24(t10[0], wy0) + __umul24(t11[0], wy1), wz1);
        const uint32_t s1 = __umul24(__umul24(t00[1], wy0) + __umul24(t01[1], wy1), wz0) +
                            __umul24(__umul24(t10[1], wy0) + __umul24(t11[1], wy1), wz1);
        const T v0 = finish_voxel<T>(__umul24(s0, L - rx) + __umul24(s1, rx), a, ctr);
        T *o = out + row * a.n2 + x;
        if (two) {
            const T v1 = finish_voxel<T>(__umul24(s0, L - rx - 1) + __umul24(s1, rx + 1), a, ctr + GAMMA);
            if constexpr (PAIRED_STORE) {
                if constexpr (sizeof(T) == 2) {
                    *(uint32_t *)o = (uint32_t)v0 | ((uint32_t)v1 << 16);
                } else {
                    *(uint16_t *)o = (uint16_t)((uint32_t)v0 | ((uint32_t)v1 << 8));
                }
            } else {
                o[0] = v0;
                o[1] = v1;
            }
        } else {
            o[0] = v0;
        }
    }
}

bool table_shape(int d, const int64_t *dims, int lshift, int64_t z0, int64_t z1, int64_t *zn0, int64_t *nzn,
                 int64_t *N1, int64_t *N2) {
    if (d != 3 || !dims || lshift < 1 || lshift > 8) return false;
    for (int k = 0; k < 3; ++k)
        if (dims[k] < 1) return false;
    if (dims[1] > INT32_MAX || dims[2] > INT32_MAX - 1) return false;
    if (z0 < 0 || z1 <= z0 || z1 > dims[0]) return false;
    *N1 = ((dims[1] - 1) >> lshift) + 2;
    *N2 = ((dims[2] - 1) >> lshift) + 2;
    *zn0 = z0 >> lshift;
    *nzn = ((z1 - 1) >> lshift) - *zn0 + 2;
    return true;
}

}  // namespace

extern "C" {

/* Number of uint16 entries of the lattice table that eccgen_dev_value_noise
 * needs for planes [z0, z1) of a 3-D image of dims.  Returns 0, or -1 on bad
 * arguments. */
int eccgen_dev_table_entries(int d, const int64_t *dims, int lshift, int64_t z0, int64_t z1, int64_t *entries) {
    int64_t zn0, nzn, N1, N2;
    if (!entries || !table_shape(d, dims, lshift, z0, z1, &zn0, &nzn, &N1, &N2)) return -1;
    *entries = nzn * N1 * N2;
    return 0;
}

/* Integer value noise for planes [z0, z1) of the 3-D image dims, written to
 * out (device memory, (z1 - z0) * dims[1] * dims[2] elements of elem = 1 or 2
 * bytes, C order) on stream (hipStream_t, may be NULL).  table: device buffer
 * of table_entries uint16 (eccgen_dev_table_entries), overwritten.  Returns 0
 * once the work is enqueued, -1 on bad arguments, -2 on a HIP error. */
int eccgen_dev_value_noise(uint64_t seed, int d, const int64_t *dims, int lshift, int bits, int amp, int64_t z0,
                           int64_t z1, void *out, int elem, uint16_t *table, int64_t table_entries, void *stream) {
    int64_t zn0, nzn, N1, N2;
    if (!out || !table || !table_shape(d, dims, lshift, z0, z1, &zn0, &nzn, &N1, &N2)) return -1;
    if ((elem != 1 && elem != 2) || bits < 1 || bits > 8 * elem || amp < 0 || amp > (1 << 16)) return -1;
    if (2 * lshift + bits > 24) return -1;  // interpolation factors fit the 24-bit multiplier
    const int64_t count = nzn * N1 * N2;
    if (table_entries < count) return -1;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t node0 = (uint64_t)zn0 * (uint64_t)N1 * (uint64_t)N2;
    int64_t lb = (count + 255) / 256;
    if (lb > 65536) lb = 65536;
    hipLaunchKernelGGL(lattice_kernel, dim3((unsigned)lb), dim3(256), 0, s, key_of(seed, 1), 64 - bits, node0, count,
                       table);
    if (hipGetLastError() != hipSuccess) return -2;

    VoxArgs a;
    a.table = table;
    a.key2 = key_of(seed, 2);
    a.z0 = z0;
    a.zn0 = zn0;
    a.rows = (z1 - z0) * dims[1];
    a.n1 = (int32_t)dims[1];
    a.n2 = (int32_t)dims[2];
    a.N1 = (int32_t)N1;
    a.N2 = (int32_t)N2;
    a.lshift = lshift;
    a.amp = amp;
    a.maxv = (int32_t)((1u << bits) - 1);
    const int64_t pairs = (dims[2] + 1) / 2;
    const dim3 grid((unsigned)((pairs + 255) / 256), (unsigned)(a.rows < 65535 ? a.rows : 65535));
    a.row_step = (uint64_t)grid.y * (uint64_t)dims[2] * GAMMA;
    a.dq = (int32_t)(grid.y / dims[1]);
    a.dr = (int32_t)(grid.y % dims[1]);
    const bool paired = dims[2] % 2 == 0 && (uintptr_t)out % (2 * elem) == 0;
    if (elem == 2) {
        if (paired)
            hipLaunchKernelGGL((voxel_kernel<uint16_t, true>), grid, dim3(256), 0, s, a, (uint16_t *)out);
        else
            hipLaunchKernelGGL((voxel_kernel<uint16_t, false>), grid, dim3(256), 0, s, a, (uint16_t *)out);
    } else {
        if (paired)
            hipLaunchKernelGGL((voxel_kernel<uint8_t, true>), grid, dim3(256), 0, s, a, (uint8_t *)out);
        else
            hipLaunchKernelGGL((voxel_kernel<uint8_t, false>), grid, dim3(256), 0, s, a, (uint8_t *)out);
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
