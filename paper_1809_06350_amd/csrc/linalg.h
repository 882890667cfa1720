// Block-sparse products over the shared node-graph pattern.
//
// Layout: 16 lanes per row (node), 16 rows per 256-thread workgroup; rows have
// W fixed block slots (a multiple of 16, padding slots hold zeros), so lane l
// of row i handles blocks W*i + l, + 16, ... without reading row pointers.
// Block values are entry-major (A[e][nnzb]): the 16 lanes of a row -- and the
// 64 lanes of a wavefront, which cover 4 consecutive rows -- read one aligned
// 128-byte (FP64) segment per entry e.  In the wide FP64 products (A, full)
// the matrix values and column indices, streamed once per product, are loaded
// non-temporally, which leaves L2 to the gathered vector entries; in the
// narrow and FP32 products plain loads measured faster.  Sums are accumulated
// in FP64 for both FP64 and FP32 storage and reduced across the 16 lanes with
// xor shuffles (fixed order).
//
// Every kernel takes an optional device flag `done`: a Krylov level that has
// already converged skips the product (launches queued past convergence).
#pragma once

#include "vms_internal.h"

#define SPMV_ROWS_PER_BLOCK 16

template <typename T>
__device__ __forceinline__ double ld(const T *p, int64_t i) { return (double)p[i]; }
// matrix values and column indices, non-temporal when NT
template <bool NT, typename T>
__device__ __forceinline__ double ldm(const T *p, int64_t i) {
  if (NT) return (double)__builtin_nontemporal_load(p + i);
  return (double)p[i];
}
template <bool NT>
__device__ __forceinline__ int ldc(const int32_t *p, int64_t i) {
  if (NT) return __builtin_nontemporal_load(p + i);
  return p[i];
}

__device__ __forceinline__ double reduce16(double v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}

#define SPMV_PROLOGUE                                                        \
  if (done && *done) return;                                               \
  const int lane = threadIdx.x & 15;                                       \
  const int row = xcd_block(blockIdx.x, gridDim.x) * SPMV_ROWS_PER_BLOCK + \
                  (threadIdx.x >> 4);                                      \
  const bool act = row < n;                                                \
  const int b0 = act ? W * row : 0;                                        \
  const int b1 = act ? b0 + W : 0;

// y[n][3] = yin + s * A x,  A 3x3 blocks, x[n][3]
template <typename TM, typename TV>
__global__ void __launch_bounds__(VMS_BLOCK)
k_spmv_A(int n, int64_t nnzb, int W, const int32_t *__restrict__ col,
         const TM *__restrict__ A, const TV *__restrict__ x, TV *y, const TV *yin, double s,
         const int *done, int *worked = nullptr) {
  SPMV_PROLOGUE
  if (worked && blockIdx.x == 0 && threadIdx.x == 0) *worked = 1;   // launch timing: this launch did work
  constexpr bool NT = sizeof(TM) == 8;
  const int64_t o = 3 * (int64_t)(act ? row : 0);
  double y0 = 0, y1 = 0, y2 = 0;   // yin of the row, loaded ahead of the product
  if (yin) { y0 = ld(yin, o); y1 = ld(yin, o + 1); y2 = ld(yin, o + 2); }
  double a0 = 0, a1 = 0, a2 = 0;
  for (int b = b0 + lane; b < b1; b += 16) {
    const int c = ldc<NT>(col, b);
    const double x0 = ld(x, 3 * (int64_t)c), x1 = ld(x, 3 * (int64_t)c + 1), x2 = ld(x, 3 * (int64_t)c + 2);
    a0 += ldm<NT>(A, 0 * nnzb + b) * x0 + ldm<NT>(A, 1 * nnzb + b) * x1 + ldm<NT>(A, 2 * nnzb + b) * x2;
    a1 += ldm<NT>(A, 3 * nnzb + b) * x0 + ldm<NT>(A, 4 * nnzb + b) * x1 + ldm<NT>(A, 5 * nnzb + b) * x2;
    a2 += ldm<NT>(A, 6 * nnzb + b) * x0 + ldm<NT>(A, 7 * nnzb + b) * x1 + ldm<NT>(A, 8 * nnzb + b) * x2;
  }
  a0 = reduce16(a0);
  a1 = reduce16(a1);
  a2 = reduce16(a2);
  if (act && lane == 0) {
    y[o] = (TV)(y0 + s * a0); y[o + 1] = (TV)(y1 + s * a1); y[o + 2] = (TV)(y2 + s * a2);
  }
}

// y[n][3] = yin + s * B x, B 3x1 blocks, x[n]
template <typename TM, typename TV>
__global__ void __launch_bounds__(VMS_BLOCK)
k_spmv_B(int n, int64_t nnzb, int W, const int32_t *__restrict__ col,
         const TM *__restrict__ B, const TV *__restrict__ x, TV *y, const TV *yin, double s,
         const int *done) {
  SPMV_PROLOGUE
  const int64_t o = 3 * (int64_t)(act ? row : 0);
  double y0 = 0, y1 = 0, y2 = 0;
  if (yin) { y0 = ld(yin, o); y1 = ld(yin, o + 1); y2 = ld(yin, o + 2); }
  double a0 = 0, a1 = 0, a2 = 0;
  for (int b = b0 + lane; b < b1; b += 16) {
    const double xp = ld(x, col[b]);
    a0 += ld(B, 0 * nnzb + b) * xp;
    a1 += ld(B, 1 * nnzb + b) * xp;
    a2 += ld(B, 2 * nnzb + b) * xp;
  }
  a0 = reduce16(a0);
  a1 = reduce16(a1);
  a2 = reduce16(a2);
  if (act && lane == 0) {
    y[o] = (TV)(y0 + s * a0); y[o + 1] = (TV)(y1 + s * a1); y[o + 2] = (TV)(y2 + s * a2);
  }
}

// y[n] = yin + s * C x (C 1x3 blocks, x[n][3]) + sd * D xd (D 1x1, xd[n]; skipped if xd == NULL)
template <typename TM, typename TV>
__global__ void __launch_bounds__(VMS_BLOCK)
k_spmv_CD(int n, int64_t nnzb, int W, const int32_t *__restrict__ col,
          const TM *__restrict__ C, const TM *__restrict__ D, const TV *__restrict__ x,
          const TV *__restrict__ xd, TV *y, const TV *yin, double s, double sd, const int *done) {
  SPMV_PROLOGUE
  const double yi = (yin && act) ? ld(yin, row) : 0.0;
  double a = 0, d = 0;
  for (int b = b0 + lane; b < b1; b += 16) {
    const int c = col[b];
    if (x) {
      a += ld(C, 0 * nnzb + b) * ld(x, 3 * (int64_t)c) + ld(C, 1 * nnzb + b) * ld(x, 3 * (int64_t)c + 1) +
           ld(C, 2 * nnzb + b) * ld(x, 3 * (int64_t)c + 2);
    }
    if (xd) d += ld(D, b) * ld(xd, c);
  }
  a = reduce16(a);
  d = reduce16(d);
  if (act && lane == 0) y[row] = (TV)(yi + s * a + sd * d);
}

// y[n][4] = K x, K = [[A, B], [C, D]] with node-interleaved x[n][4]
__global__ void __launch_bounds__(VMS_BLOCK)
k_spmv_full(int n, int64_t nnzb, int W, const int32_t *__restrict__ col,
            const double *__restrict__ A, const double *__restrict__ B, const double *__restrict__ C,
            const double *__restrict__ D, const double *__restrict__ x, double *__restrict__ y,
            const int *done) {
  SPMV_PROLOGUE
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int b = b0 + lane; b < b1; b += 16) {
    const int64_t c = 4 * (int64_t)ldc<true>(col, b);
    const double x0 = x[c], x1 = x[c + 1], x2 = x[c + 2], x3 = x[c + 3];
    a0 += ldm<true>(A, 0 * nnzb + b) * x0 + ldm<true>(A, 1 * nnzb + b) * x1 + ldm<true>(A, 2 * nnzb + b) * x2 +
          ldm<true>(B, 0 * nnzb + b) * x3;
    a1 += ldm<true>(A, 3 * nnzb + b) * x0 + ldm<true>(A, 4 * nnzb + b) * x1 + ldm<true>(A, 5 * nnzb + b) * x2 +
          ldm<true>(B, 1 * nnzb + b) * x3;
    a2 += ldm<true>(A, 6 * nnzb + b) * x0 + ldm<true>(A, 7 * nnzb + b) * x1 + ldm<true>(A, 8 * nnzb + b) * x2 +
          ldm<true>(B, 2 * nnzb + b) * x3;
    a3 += ldm<true>(C, 0 * nnzb + b) * x0 + ldm<true>(C, 1 * nnzb + b) * x1 + ldm<true>(C, 2 * nnzb + b) * x2 +
          ldm<true>(D, b) * x3;
  }
  a0 = reduce16(a0);
  a1 = reduce16(a1);
  a2 = reduce16(a2);
  a3 = reduce16(a3);
  if (act && lane == 0) {
    const int64_t o = 4 * (int64_t)row;
    y[o] = a0; y[o + 1] = a1; y[o + 2] = a2; y[o + 3] = a3;
  }
}

inline int spmv_grid(int n) { return (n + SPMV_ROWS_PER_BLOCK - 1) / SPMV_ROWS_PER_BLOCK; }
