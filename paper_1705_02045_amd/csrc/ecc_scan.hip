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

// Column sums of the [rows][m] int32 table into int64 vcec.  Block (bx, by)
// sums rows by, by + gridDim.y, ... of columns bx*256 .. bx*256+255, then adds
// its partial sum with one 64-bit atomic per column.
__global__ void reduce_rows_kernel(const int32_t *__restrict__ partial, int rows, int m,
                                   unsigned long long *vcec) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= m) return;
    int64_t s = 0;
    for (int r = blockIdx.y; r < rows; r += gridDim.y) s += partial[(size_t)r * m + col];
    if (s != 0) atomicAdd(&vcec[col], (unsigned long long)s);
}

int launch_reduce_rows(const int32_t *partial, int rows, int m, int64_t *vcec, bool accumulate,
                       hipStream_t stream) {
    if (!accumulate) {
        int rc = launch_zero(vcec, (size_t)m * sizeof(int64_t), stream);
        if (rc) return rc;
    }
    const int threads = 256;
    const int bx = (m + threads - 1) / threads;
    int by = 1;
    while (by < 32 && bx * by < 512 && by * 8 <= rows) by *= 2;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(bx, by), dim3(threads), 0, stream, partial, rows, m,
                       (unsigned long long *)vcec);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

// Inclusive prefix sum of m int64 values by one workgroup of 1024 threads.
// The curve is written only if the status word reports a valid input; the
// status is copied to status_out when that is given.
__global__ void __launch_bounds__(1024) scan_kernel(const int64_t *__restrict__ vcec, int m, int64_t *chi,
                                                   const uint32_t *status, uint32_t *status_out) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const uint32_t st = status ? *status : 0u;
    if (status_out && tid == 0) *status_out = st;
    if (st != 0) return;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < m; base += 1024) {
        const int i = base + tid;
        int64_t v = i < m ? vcec[i] : 0;
        // wave-level inclusive scan
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t u = __shfl_up(v, off, 64);
            if (lane >= off) v += u;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        if (wave == 0) {
            int64_t w = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const int64_t u = __shfl_up(w, off, 64);
                if (lane >= off) w += u;
            }
            if (lane < 16) wsum[lane] = w;  // inclusive totals of waves 0..lane
        }
        __syncthreads();
        const int64_t carry = carry_s;
        const int64_t before = wave > 0 ? wsum[wave - 1] : 0;
        if (i < m) chi[i] = carry + before + v;
        __syncthreads();
        if (tid == 0) carry_s = carry + wsum[15];
        __syncthreads();
    }
}

int launch_scan(const int64_t *vcec, int m, int64_t *chi, const uint32_t *status, uint32_t *status_out,
                hipStream_t stream) {
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, vcec, m, chi, status, status_out);
    ECC_HIP(hipGetLastError());
    return ECC_OK;
}

}  // namespace ecc
