// Matrix ingest kernels: CSR validation, the Jacobi diagonal, conversion to
// the SELL-64 layout, and the sparse outer product of the adjoint.
#include <climits>

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

// Slice planning, one wavefront per 64-row slice.  Each lane holds one row;
// the union of the column offsets (col - row) of the slice is found by
// repeatedly taking the wavefront minimum of the lanes' next offsets (rows
// must be sorted by column).  A slice is stored offset-aligned when that
// union has at most 1.5x the longest row and at most 64 members: slot j then
// holds, for every row, its entry at offset union[j] or a zero.  Otherwise
// the slice is packed: slot j holds each row's j-th entry and its column.
// width[s] = slots of the slice; aligned[s] = 1 for offset-aligned.
__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int offset_limit(int maxlen) { return min(kSlice, maxlen + maxlen / 2); }

// Row of lane `lane` of slice s: 64 s + lane, or row0[s] + lane when the
// slices follow a geometry of their own (batched systems); rows past the
// slice's end are marked -1.
__device__ __forceinline__ int64_t slice_lane_row(int64_t s, int lane, int64_t n, const int64_t* row0,
                                                  const int32_t* nrows)
{
    if (row0) return lane < nrows[s] ? row0[s] + lane : -1;
    const int64_t i = s * kSlice + lane;
    return i < n ? i : -1;
}

__global__ void k_slice_plan(int64_t n, int64_t nslices, const int32_t* __restrict__ row_ptr,
                             const int32_t* __restrict__ col, const int64_t* __restrict__ row0,
                             const int32_t* __restrict__ nrows, int32_t* __restrict__ width,
                             int32_t* __restrict__ aligned)
{
    const int64_t t = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    const int64_t s = t / kSlice;
    if (s >= nslices) return;  // whole wavefronts leave together (nslices * 64 threads are useful)
    const int64_t i = slice_lane_row(s, (int)(t % kSlice), n, row0, nrows);
    const int32_t a = i >= 0 ? row_ptr[i] : 0;
    const int32_t e = i >= 0 ? row_ptr[i + 1] : 0;
    const int len = e - a;
    int sorted = 1;
    for (int32_t q = a + 1; q < e; ++q)
        if (col[q] <= col[q - 1]) sorted = 0;
    const int maxlen = wave_max_i32(len);
    const int all_sorted = wave_min_i32(sorted);
    int slots = -1;
    if (all_sorted && maxlen > 0) {
        const int limit = offset_limit(maxlen);
        int32_t q = a;
        int count = 0;
        for (;;) {
            const int head = q < e ? (int)(col[q] - i) : INT_MAX;
            const int m = wave_min_i32(head);
            if (m == INT_MAX) break;
            if (++count > limit) break;
            if (head == m) ++q;
        }
        if (count <= limit) slots = count;
    }
    if ((threadIdx.x & 63) == 0) {
        width[s] = slots >= 0 ? slots : maxlen;
        aligned[s] = slots >= 0 ? 1 : 0;
    }
}

// Fill the SELL-64 storage planned above.  slice_ptr: value offsets;
// slice_meta[s] = start of the slice's offsets in soff (aligned) or -1;
// slice_shape[s]: width and slot stride.
// Packed padding has value 0 and the row's own index (n-1 past the last
// row) as column.
__global__ void k_fill_sell(int64_t n, int64_t nslices, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col, const double* __restrict__ val,
                            const int64_t* __restrict__ row0, const int32_t* __restrict__ nrows,
                            const int64_t* __restrict__ slice_ptr, const int32_t* __restrict__ slice_meta,
                            const int32_t* __restrict__ slice_shape, int32_t* __restrict__ soff,
                            int32_t* __restrict__ scol, double* __restrict__ sval, int write_cols)
{
    const int64_t t = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    const int64_t s = t / kSlice;
    if (s >= nslices) return;
    const int lane = (int)(t % kSlice);
    const int64_t i = slice_lane_row(s, lane, n, row0, nrows);
    const int64_t base = slice_ptr[s];
    const int width = shape_width(slice_shape[s]);
    const int64_t stride = shape_stride(slice_shape[s]);
    const int32_t a = i >= 0 ? row_ptr[i] : 0;
    const int32_t e = i >= 0 ? row_ptr[i + 1] : 0;
    const int meta = slice_meta[s];
    if (meta >= 0) {
        int32_t q = a;
        for (int j = 0; j < width; ++j) {
            const int head = q < e ? (int)(col[q] - i) : INT_MAX;
            const int m = wave_min_i32(head);
            const int64_t pos = base + (int64_t)j * stride + lane;
            if (head == m) {
                sval[pos] = val[q];
                ++q;
            } else {
                sval[pos] = 0.0;
            }
            if (write_cols && lane == 0) soff[meta + j] = m;
        }
    } else {
        const int len = e - a;
        const int32_t pad_col = (int32_t)(i >= 0 ? i : n - 1);
        for (int j = 0; j < width; ++j) {
            const int64_t pos = base + (int64_t)j * stride + lane;
            if (j < len) {
                if (write_cols) scol[pos] = col[a + j];
                sval[pos] = val[a + j];
            } else {
                if (write_cols) scol[pos] = pad_col;
                sval[pos] = 0.0;
            }
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
// of w^T A^{-1} b with respect to entry e, given lambda = A^{-1} w): L lanes per row,
// lane t of a row taking its entries t, t + L, ..., so that the lanes of a
// wavefront read col and write g in consecutive runs (rows are consecutive
// in CSR) instead of one strided run per thread.
template <int L>
__global__ void k_outer_csr(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ lam, const double* __restrict__ x, double* __restrict__ g)
{
    const int64_t t = (int64_t)blockIdx.x * kSetupBlock + threadIdx.x;
    const int64_t i = t / L;
    if (i >= n) return;
    const int lane = (int)(t % L);
    const double li = -lam[i];
    const int32_t e1 = row_ptr[i + 1];
    for (int32_t e = row_ptr[i] + lane; e < e1; e += L) g[e] = li * x[col[e]];
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

hipError_t launch_slice_plan(int64_t n, int64_t nslices, const int32_t* row_ptr, const int32_t* col,
                             const int64_t* row0, const int32_t* nrows, int32_t* width, int32_t* aligned,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_slice_plan, rows_grid(nslices * kSlice), dim3(kSetupBlock), 0, st, n, nslices, row_ptr, col,
                       row0, nrows, width, aligned);
    return hipGetLastError();
}

hipError_t launch_fill_sell(int64_t n, int64_t nslices, const int32_t* row_ptr, const int32_t* col, const double* val,
                            const int64_t* row0, const int32_t* nrows, const int64_t* slice_ptr,
                            const int32_t* slice_meta, const int32_t* slice_shape, int32_t* soff, int32_t* scol,
                            double* sval, int write_cols, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_sell, rows_grid(nslices * kSlice), dim3(kSetupBlock), 0, st, n, nslices, row_ptr, col,
                       val, row0, nrows, slice_ptr, slice_meta, slice_shape, soff, scol, sval, write_cols);
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
                            double* g, double mean_row, hipStream_t st)
{
    // lanes per row: the power of two at or above the mean row length, 4..32
    auto go = [&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        hipLaunchKernelGGL((k_outer_csr<L>), rows_grid(n * L), dim3(kSetupBlock), 0, st, n, row_ptr, col, lam, x, g);
    };
    if (mean_row <= 4.0)
        go(std::integral_constant<int, 4>{});
    else if (mean_row <= 8.0)
        go(std::integral_constant<int, 8>{});
    else if (mean_row <= 16.0)
        go(std::integral_constant<int, 16>{});
    else
        go(std::integral_constant<int, 32>{});
    return hipGetLastError();
}

}  // namespace prcg
