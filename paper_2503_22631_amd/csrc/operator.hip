// Operator set-up on the device.
//
// Validation: every product kernel indexes x with colind and walks rows with rowptr, so
// fab_csr_create refuses a malformed CSR before anything else touches it.
//
// Transpose, for the adjoint solve on A^T.  The derivative of <c, f(t A) b> with respect to b is
// f(t A^T) c (the adjoint identity <c, f(A) b> = <f(A^T) c, b>); the adjoint runs the same
// restarted sketched Krylov method on A^T, so A^T is stored as a CSR matrix of its own.
// Steps: count the entries of every column; exclusive scan of the counts gives the row pointers of
// A^T; scatter every entry (i, c, v) to row c of A^T through a per-row cursor; sort every row of
// A^T by column index, so the result is canonical (independent of the order of the scatter's
// atomics).
#include "fab_internal.h"

namespace fab {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;                          // items per thread
constexpr int kScanBlock = kScanThreads * kScanPer;  // items per block

// ---------------------------------------------------------------------------------- validation
// flag bit 0: rowptr not monotone or rowptr[0] != 0 or rowptr[n] != nnz; bit 1: column out of range.
__global__ void k_csr_validate(int n, int nnz, const int* __restrict__ rowptr, const int* __restrict__ colind,
                               int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n; i += stride) {
    const int a = rowptr[i], b = rowptr[i + 1];
    if (a > b || (i == 0 && a != 0) || (i == n - 1 && b != nnz)) bad |= 1;
  }
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < (int64_t)nnz; p += stride) {
    const int c = colind[p];
    if (c < 0 || c >= n) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// off[p] = colind[p] - (first row of the row's kThreads-row tile), the fused product's 16-bit column
// form; flag = 1 when some offset does not fit in 16 bits (off is then not used).
__global__ void k_col_offsets(int n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                              int16_t* __restrict__ off, int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n; i += stride) {
    const int row0 = (int)(i - i % kThreads);
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const int dlt = colind[p] - row0;
      if (dlt < -32768 || dlt > 32767)
        bad = 1;
      else
        off[p] = (int16_t)dlt;
    }
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void k_count_cols(int nnz, const int* __restrict__ colind, int* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < (int64_t)nnz; p += stride)
    atomicAdd(&cnt[colind[p]], 1);
}

// Exclusive scan of v[0..len) within blocks of kScanBlock items; block totals go to sums.
__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(int len, int* __restrict__ v, int* __restrict__ sums) {
  __shared__ int wsum[kScanThreads / 64];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int loc[kScanPer];
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    loc[q] = (base + q < len) ? v[base + q] : 0;
    s += loc[q];
  }
  // inclusive scan of the per-thread sums across the block: wavefront scan, then wave offsets
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = s;
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int woff = 0;
  for (int q = 0; q < wv; ++q) woff += wsum[q];
  int run = woff + inc - s;  // exclusive prefix of this thread's first item
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < len) v[base + q] = run;
    run += loc[q];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = woff + inc;
}

// Exclusive scan of the block totals in place, one block, in chunks of kScanThreads with a carry.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int nb, int* __restrict__ sums) {
  __shared__ int wsum[kScanThreads / 64];
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c0 = 0; c0 < nb; c0 += kScanThreads) {
    const int i = c0 + threadIdx.x;
    const int x = (i < nb) ? sums[i] : 0;
    int inc = x;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int woff = 0;
    for (int q = 0; q < wv; ++q) woff += wsum[q];
    const int carry = carry_s;
    if (i < nb) sums[i] = carry + woff + inc - x;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry_s = carry + woff + inc;
    __syncthreads();
  }
}

__global__ void k_scan_add(int len, int* __restrict__ v, const int* __restrict__ sums) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)len; i += stride)
    v[i] += sums[i / kScanBlock];
}

template <typename T>
__global__ void k_scatter_t(int n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                            const T* __restrict__ vals, int* __restrict__ cursor, int* __restrict__ colT,
                            T* __restrict__ valT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n; i += stride) {
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const int pos = atomicAdd(&cursor[colind[p]], 1);
      colT[pos] = (int)i;
      valT[pos] = vals[p];
    }
  }
}

// Insertion sort of every row of A^T by column index (rows of a PDE operator are short; a row of
// length L costs O(L^2) on its thread).
template <typename T>
__global__ void k_sort_rows(int n, const int* __restrict__ rowptrT, int* __restrict__ colT, T* __restrict__ valT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < (int64_t)n; r += stride) {
    const int a = rowptrT[r], b = rowptrT[r + 1];
    for (int p = a + 1; p < b; ++p) {
      const int c = colT[p];
      const T v = valT[p];
      int q = p - 1;
      while (q >= a && colT[q] > c) {
        colT[q + 1] = colT[q];
        valT[q + 1] = valT[q];
        --q;
      }
      colT[q + 1] = c;
      valT[q + 1] = v;
    }
  }
}

// ---------------------------------------------------------------------------------- transpose
static int grid_for(int64_t items, int threads, int cap) {
  int64_t g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_csr_validate(hipStream_t s, int n, int nnz, const int* rowptr, const int* colind, int* flag) {
  const int64_t items = (int64_t)(n > nnz ? n : nnz);
  hipLaunchKernelGGL(k_csr_validate, dim3(grid_for(items, 256, 4096)), dim3(256), 0, s, n, nnz, rowptr, colind, flag);
  return hipGetLastError();
}

hipError_t launch_col_offsets(hipStream_t s, int n, const int* rowptr, const int* colind, int16_t* off, int* flag) {
  hipLaunchKernelGGL(k_col_offsets, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, rowptr, colind, off, flag);
  return hipGetLastError();
}

size_t transpose_scan_blocks(int64_t len) { return (size_t)((len + kScanBlock - 1) / kScanBlock); }

// rowptrT must hold n+1 zeroed ints; cursor n ints; sums transpose_scan_blocks(n+1) ints.
hipError_t launch_transpose(hipStream_t s, int dtype, int n, int nnz, const int* rowptr, const int* colind,
                            const void* vals, int* rowptrT, int* colT, void* valT, int* cursor, int* sums) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, s, nnz, colind, rowptrT);
  const int len = n + 1;
  const int nb = (int)transpose_scan_blocks(len);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kScanThreads), 0, s, len, rowptrT, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, nb, sums);
  hipLaunchKernelGGL(k_scan_add, dim3(grid_for(len, 256, 8192)), dim3(256), 0, s, len, rowptrT, sums);
  hipError_t e = hipMemcpyAsync(cursor, rowptrT, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  const int g = grid_for(n, 256, 8192);
  if (dtype == 0) {
    hipLaunchKernelGGL(k_scatter_t<double>, dim3(g), dim3(256), 0, s, n, rowptr, colind, (const double*)vals, cursor,
                       colT, (double*)valT);
    hipLaunchKernelGGL(k_sort_rows<double>, dim3(g), dim3(256), 0, s, n, rowptrT, colT, (double*)valT);
  } else {
    hipLaunchKernelGGL(k_scatter_t<float>, dim3(g), dim3(256), 0, s, n, rowptr, colind, (const float*)vals, cursor,
                       colT, (float*)valT);
    hipLaunchKernelGGL(k_sort_rows<float>, dim3(g), dim3(256), 0, s, n, rowptrT, colT, (float*)valT);
  }
  return hipGetLastError();
}

}  // namespace fab
