// Matrix ingest kernels: CSR validation, the Jacobi diagonal, conversion to
// the SELL-64 layout, and the sparse outer product of the adjoint.
#include "prcg_device.h"

namespace prcg {

namespace {

constexpr int kSetupBlock = 256;

inline dim3 rows_grid(int64_t rows) { return dim3((unsigned)((rows + kSetupBlock - 1) / kSetupBlock)); }

// flags: 1 row_ptr[0] != 0, 2 decreasing row_ptr or out of [0, nnz],
// 4 row_ptr[n] != nnz, 8 column index out of range.  Column indices are only
// read where the row's range is a valid sub-range of [0, nnz).
__global__ void k_validate(int64_t n, int64_t nnz, const int32_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col, int32_t* __restrict__ flags, int32_t* __restrict__ maxlen)
{
    const int64_t i = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t a = row_ptr[i], b = row_ptr[i + 1];
    int f = 0;
    if (i == 0 && a != 0) f |= 1;
    if (i == n - 1 && b != nnz) f |= 4;
    if (a < 0 || b < a || b > nnz) {
        f |= 2;
    } else {
        for (int64_t e = a; e < b; ++e) {
            const int32_t c = col[e];
            if (c < 0 || c >= n) {
                f |= 8;
                break;
            }
        }
        atomicMax(maxlen, (int32_t)(b - a));
    }
    if (f) atomicOr(flags, f);
}

// d_i = 1 / a_ii (duplicates summed); flag 16 if a_ii is missing or not > 0.
__global__ void k_jacobi(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         const double* __restrict__ val, double* __restrict__ d, int32_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    int found = 0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        if (col[e] == i) {
            a += val[e];
            found = 1;
        }
    }
    if (!found || !(a > 0.0) || !__builtin_isfinite(a)) {
        atomicOr(flags, 16);
        d[i] = 0.0;
    } else {
        d[i] = 1.0 / a;
    }
}

// sizes[s] = 64 * (longest row of slice s).
__global__ void k_slice_sizes(int64_t n, int64_t nslices, const int32_t* __restrict__ row_ptr,
                              int64_t* __restrict__ sizes)
{
    const int64_t i = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    const int64_t s = i / kSlice;
    int len = 0;
    if (i < n) len = row_ptr[i + 1] - row_ptr[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
    if ((threadIdx.x & 63) == 0 && s < nslices) sizes[s] = (int64_t)kSlice * len;
}

// out[j] = sum_{i<j} in[i] for j = 0..m (out has m+1 entries); one workgroup.
__global__ __launch_bounds__(1024) void k_exclusive_scan(const int64_t* __restrict__ in, int64_t* __restrict__ out,
                                                         int64_t m)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (m + 1023) / 1024;
    const int64_t lo = t * chunk, hi = lo + chunk < m ? lo + chunk : m;
    int64_t s = 0;
    for (int64_t j = lo; j < hi; ++j) s += in[j];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int q = 0; q < 1024; ++q) {
            const int64_t v = part[q];
            part[q] = run;
            run += v;
        }
        out[m] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t j = lo; j < hi; ++j) {
        out[j] = run;
        run += in[j];
    }
}

// Scatter CSR rows into SELL-64 slices; padding has value 0 and the row's
// own index (or n-1 past the last row) as column.
__global__ void k_fill_sell(int64_t n, int64_t nslices, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col, const double* __restrict__ val,
                            const int64_t* __restrict__ slice_ptr, int32_t* __restrict__ scol,
                            double* __restrict__ sval, int write_cols)
{
    const int64_t i = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    const int64_t s = i / kSlice;
    if (s >= nslices) return;
    const int lane = (int)(i % kSlice);
    const int64_t base = slice_ptr[s];
    const int width = (int)((slice_ptr[s + 1] - base) / kSlice);
    const int32_t a = i < n ? row_ptr[i] : 0;
    const int len = i < n ? row_ptr[i + 1] - a : 0;
    const int32_t pad_col = (int32_t)(i < n ? i : n - 1);
    for (int j = 0; j < width; ++j) {
        const int64_t pos = base + (int64_t)j * kSlice + lane;
        if (j < len) {
            if (write_cols) scol[pos] = col[a + j];
            sval[pos] = val[a + j];
        } else {
            if (write_cols) scol[pos] = pad_col;
            sval[pos] = 0.0;
        }
    }
}

// flags |= 32 if a row of system s has a column outside [off[s], off[s+1]).
__global__ void k_block_check(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                              const int32_t* __restrict__ row_sys, const int64_t* __restrict__ sys_off,
                              int32_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    if (i >= n) return;
    const int s = row_sys[i];
    const int64_t lo = sys_off[s], hi = sys_off[s + 1];
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int64_t c = col[e];
        if (c < lo || c >= hi) {
            atomicOr(flags, 32);
            return;
        }
    }
}

// g_e = -lambda_{row(e)} * x_{col(e)} for every stored entry (the gradient
// of w^T A^{-1} b with respect to entry e, given lambda = A^{-1} w).
__global__ void k_outer_csr(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ lam, const double* __restrict__ x, double* __restrict__ g)
{
    const int64_t i = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    if (i >= n) return;
    const double li = -lam[i];
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) g[e] = li * x[col[e]];
}

}  // namespace

hipError_t launch_validate(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, int32_t* flags,
                           int32_t* maxlen, hipStream_t st)
{
    hipLaunchKernelGGL(k_validate, rows_grid(n), dim3(kSetupBlock), 0, st, n, nnz, row_ptr, col, flags, maxlen);
    return hipGetLastError();
}

hipError_t launch_jacobi(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val, double* d,
                         int32_t* flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_jacobi, rows_grid(n), dim3(kSetupBlock), 0, st, n, row_ptr, col, val, d, flags);
    return hipGetLastError();
}

hipError_t launch_slice_sizes(int64_t n, const int32_t* row_ptr, int64_t* sizes, hipStream_t st)
{
    const int64_t nslices = (n + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_slice_sizes, rows_grid(nslices * kSlice), dim3(kSetupBlock), 0, st, n, nslices, row_ptr,
                       sizes);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int64_t* in, int64_t* out, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(1024), 0, st, in, out, m);
    return hipGetLastError();
}

hipError_t launch_fill_sell(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                            const int64_t* slice_ptr, int32_t* scol, double* sval, int write_cols, hipStream_t st)
{
    const int64_t nslices = (n + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_fill_sell, rows_grid(nslices * kSlice), dim3(kSetupBlock), 0, st, n, nslices, row_ptr, col,
                       val, slice_ptr, scol, sval, write_cols);
    return hipGetLastError();
}

hipError_t launch_block_check(int64_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* row_sys,
                              const int64_t* sys_off, int32_t* flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_block_check, rows_grid(n), dim3(kSetupBlock), 0, st, n, row_ptr, col, row_sys, sys_off,
                       flags);
    return hipGetLastError();
}

hipError_t launch_outer_csr(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* lam, const double* x,
                            double* g, hipStream_t st)
{
    hipLaunchKernelGGL(k_outer_csr, rows_grid(n), dim3(kSetupBlock), 0, st, n, row_ptr, col, lam, x, g);
    return hipGetLastError();
}

}  // namespace prcg
