// Shared device helpers for the vembddc kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step.  Operand layout (wave64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator element r of lane l holds
// D[row(l/16, r)][l%16] with row = l/16 + 4r for FP64 and 4(l/16) + r for
// FP32 (measured on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

// Pointers read from job descriptors are generic; loads through them become
// flat loads, which also count on lgkmcnt and so serialise with LDS reads.
// Device memory is the global address space: say so.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const T *p) {
  return (const __attribute__((address_space(1))) T *)p;
}

// Dense partial LDL^T job: column-major A (n x n, leading dimension ld),
// eliminate columns [0, e), pivot sign +1 for columns < p, -1 otherwise.
template <typename T> struct LdlJob {
  T *A;
  int64_t ld;
  int n, e, p, pad;
  T *invL;     // per panel: NB*NB block (column-major) of inv(L_jj); panels stored consecutively
  int *info;   // 0 or 1 + column of the first pivot at or below pmin (after its sign)
  double pmin; // a signed pivot (d_j times the diagonal entry, before its square root)
               // must exceed this value; 0: only wrong-signed or zero pivots fail
  int zrow;    // 0, or the first row of an identity block I (rows zrow + t, columns t < e)
               // below the eliminated columns: row zrow + t of L is zero left of column t,
               // so every update from columns below c leaves rows >= zrow + c untouched
               // and is skipped there
  int zpad;
};

// Batched C = alpha * A * B^T + beta * C, all column-major.
template <typename T> struct GemmJob {
  const T *A;
  const T *B;
  T *C;
  int64_t lda, ldb, ldc;
  int m, n, k, pad;
  T alpha, beta;
};

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float warp_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum over blockDim.x threads (multiple of 64), result valid in all threads.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
  v = warp_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}
