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

// Inclusive prefix sum of m int64 values by one workgroup: chunks of
// blockDim*16 values, each thread scanning 16 consecutive values of a chunk,
// the thread totals scanned across the block, a running carry between chunks.
__device__ void block_scan_write(const int64_t *__restrict__ in, int m, int64_t *out) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int c0 = 0; c0 < m; c0 += (int)blockDim.x * 16) {
        const int base = c0 + tid * 16;
        int64_t loc[16];
        int64_t run = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            run += (base + j < m) ? in[base + j] : 0;
            loc[j] = run;
        }
        int64_t v = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t u = __shfl_up(v, off, 64);
            if (lane >= off) v += u;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        if (wave == 0) {
            int64_t w = lane < nwaves ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const int64_t u = __shfl_up(w, off, 64);
                if (lane >= off) w += u;
            }
            if (lane < nwaves) wsum[lane] = w;
        }
        __syncthreads();
        const int64_t offset = carry_s + (v - run) + (wave > 0 ? wsum[wave - 1] : 0);
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (base + j < m) out[base + j] = offset + loc[j];
        __syncthreads();
        if (tid == 0) carry_s += wsum[nwaves - 1];
        __syncthreads();
    }
}

// Merge of the per-workgroup rows [rows][m] (int32) into the int64 change
// vector, in kernels that follow each other on the stream (the kernel
// boundary orders their memory; no fences or counters):
//  1. colsum_kernel, block (bx, by): rows by, by+BY, ... of columns
//     bx*1024 .. +1023 (256 threads x 4 columns, 16-byte loads), written to
//     stage[by][column], or, with BY == 1, straight into vcec;
//  2. fold_kernel (BY > 1): the BY stage rows of each column into vcec;
//  3. scan_kernel (one block): the curve is the prefix sum of vcec, written
//     if the status word is clear; the status is copied and cleared.
// vcec is overwritten, or added to with `accumulate`.
__global__ void __launch_bounds__(256) colsum_kernel(const int32_t *__restrict__ partial, int rows, int m,
                                                     int64_t *__restrict__ dst, int accumulate) {
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
    int64_t *d = dst + (size_t)blockIdx.y * m + c0;
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

__global__ void __launch_bounds__(256) fold_kernel(const int64_t *__restrict__ stage, int by, int m,
                                                   int64_t *__restrict__ vcec, int accumulate) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= m) return;
    int64_t t = accumulate ? vcec[c] : 0;
    for (int y = 0; y < by; ++y) t += stage[(size_t)y * m + c];
    vcec[c] = t;
}

__global__ void __launch_bounds__(1024) scan_kernel(const int64_t *__restrict__ vcec, int m, int64_t *chi,
                                                    uint32_t *status, uint32_t *status_out) {
    const uint32_t stv = *status;
    if (stv == 0) block_scan_write(vcec, m, chi);
    if (threadIdx.x == 0) {
        if (status_out) *status_out = stv;
        *status = 0u;
    }
}

int merge_stage_rows(int rows) {
    int by = 1;
    while (by < 32 && by * 8 <= rows) by *= 2;
    return by;
}

int launch_merge(const int32_t *partial, int rows, int m, int64_t *stage, int64_t *vcec, bool accumulate,
                 bool do_scan, int64_t *chi, uint32_t *status, uint32_t *status_out, hipStream_t stream) {
    if (m % 4 != 0 || m > 65536) {
        set_error("launch_merge: m = %d not supported", m);
        return ECC_E_ARG;
    }
    if (rows > 0) {
        const int bx = (m + 1023) / 1024;
        const int by = merge_stage_rows(rows);
        hipLaunchKernelGGL(colsum_kernel, dim3(bx, by), dim3(256), 0, stream, partial, rows, m,
                           by == 1 ? vcec : stage, (by == 1 && accumulate) ? 1 : 0);
        ECC_HIP(hipGetLastError());
        if (by > 1) {
            hipLaunchKernelGGL(fold_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, (const int64_t *)stage, by,
                               m, vcec, accumulate ? 1 : 0);
            ECC_HIP(hipGetLastError());
        }
    }
    if (do_scan) {
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, (const int64_t *)vcec, m, chi, status,
                           status_out);
        ECC_HIP(hipGetLastError());
    }
    return ECC_OK;
}

}  // namespace ecc
