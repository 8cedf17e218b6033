// Batched dense kernels: blocked partial signed LDL^T and MFMA GEMM.
//
// The local Dirichlet problems of the method are symmetric saddle matrices
// [A B^T; B 0] with A SPD and B of full row rank on the mean-zero pressures
// (eq. uipi).  With all velocity unknowns ordered before the pressures they
// factor without pivoting as L D L^T, D = diag(+I, -I) (block Cholesky of A,
// then Cholesky of B A^-1 B^T).  Eliminating only the interior columns of a
// matrix bordered by the interface rows leaves the Schur complement
// S_Gamma^(i) (eq. firstSchur) in the trailing block.
//
// Right-looking blocked algorithm, panel width NB:
//   diag  : factor the NB x NB diagonal block in LDS and invert L_jj;
//   panel : L_ij = A_ij inv(L_jj)^T D_j for every row block below;
//   update: A_ik -= L_ij D_j L_kj^T on the lower triangle of the trailing
//           matrix, 64x64 tiles on the 16x16x4 matrix cores.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace vb {

constexpr int TILE = 64;

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ldl_diag(const LdlJob<T> *jobs, int j0) {
  const LdlJob<T> J = jobs[blockIdx.x];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  // lower triangle: L_jj; strict upper triangle S[c][r] (r > c): inv(L_jj)[r][c]
  __shared__ T S[NB][NB + 1];
  __shared__ T Xd[NB];
  __shared__ T piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int r = idx % NB, c = idx / NB;
    T v = 0;
    if (r < b && c < b && r >= c) v = J.A[(int64_t)(j0 + r) + (int64_t)(j0 + c) * J.ld];
    S[r][c] = v;
  }
  __syncthreads();
  for (int c = 0; c < b; ++c) {
    if (tid == 0) {
      T d = (j0 + c < J.p) ? T(1) : T(-1);
      T v = d * S[c][c];
      if (!(v > T(0))) {  // wrong-signed or zero pivot: report, keep going finitely
        if (!bad) { bad = 1; atomicCAS(J.info, 0, j0 + c + 1); }
        v = T(1);
      }
      T l = sqrt(v);
      S[c][c] = l;
      piv = d * l;
    }
    __syncthreads();
    const T pv = piv;
    for (int r = c + 1 + tid; r < b; r += blockDim.x) S[r][c] /= pv;
    __syncthreads();
    // trailing update inside the block: S[r][k] -= l_rc d_c l_kc, r >= k > c
    const int m = b - c - 1;
    const T d = (j0 + c < J.p) ? T(1) : T(-1);
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      int r = c + 1 + idx % m, k = c + 1 + idx / m;
      if (r >= k) S[r][k] -= S[r][c] * d * S[k][c];
    }
    __syncthreads();
  }
  // write L_jj
  for (int idx = tid; idx < b * b; idx += blockDim.x) {
    int r = idx % b, c = idx / b;
    if (r >= c) J.A[(int64_t)(j0 + r) + (int64_t)(j0 + c) * J.ld] = S[r][c];
  }
  // inv(L_jj) by forward substitution, one column per thread; column `col`
  // of the inverse goes to the strict upper part of row `col` of S.
  if (tid < b) {
    const int col = tid;
    const T dcol = T(1) / S[col][col];
    Xd[col] = dcol;
    for (int r = col + 1; r < b; ++r) {
      T s = -S[r][col] * dcol;
      for (int t = col + 1; t < r; ++t) s -= S[r][t] * S[col][t];
      S[col][r] = s / S[r][r];
    }
  }
  __syncthreads();
  T *inv = J.invL + (int64_t)(j0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int r = idx % NB, c = idx / NB;
    T v = 0;
    if (r < b && c < b) v = (r == c) ? Xd[c] : ((r > c) ? S[c][r] : T(0));
    inv[idx] = v;
  }
}

// L_ij = A_ij inv(L_jj)^T D_j for rows [j0+b, n) in tiles of PROWS rows.
constexpr int PROWS = 32;
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ldl_panel(const LdlJob<T> *jobs, int j0) {
  const LdlJob<T> J = jobs[blockIdx.y];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  const int r0 = j0 + b + blockIdx.x * PROWS;
  if (r0 >= J.n) return;
  __shared__ T Li[NB][NB];
  __shared__ T At[NB][PROWS];
  const int tid = threadIdx.x;
  const T *inv = J.invL + (int64_t)(j0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) Li[idx % NB][idx / NB] = inv[idx];
  for (int idx = tid; idx < PROWS * NB; idx += blockDim.x) {
    int r = idx % PROWS, t = idx / PROWS;
    T v = 0;
    if (r0 + r < J.n && t < b) v = J.A[(int64_t)(r0 + r) + (int64_t)(j0 + t) * J.ld];
    At[t][r] = v;
  }
  __syncthreads();
  const int r = tid % PROWS;
  const int cg = tid / PROWS;  // 0..7
  if (r0 + r >= J.n) return;
  for (int c = cg; c < b; c += 8) {
    T s = 0;
    for (int t = 0; t <= c; ++t) s += At[t][r] * Li[c][t];
    T d = (j0 + c < J.p) ? T(1) : T(-1);
    J.A[(int64_t)(r0 + r) + (int64_t)(j0 + c) * J.ld] = d * s;
  }
}

// A_ik -= L_ij D_j L_kj^T on lower-triangle 64x64 tiles of the trailing matrix.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ldl_update(const LdlJob<T> *jobs, int j0) {
  typedef Mfma<T> M;
  const LdlJob<T> J = jobs[blockIdx.y];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  const int m0 = j0 + b;
  const int nt = (J.n - m0 + TILE - 1) / TILE;
  const int t = blockIdx.x;
  if (m0 >= J.n) return;
  // tile index -> (ti, tk), ti >= tk
  int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tk = t - ti * (ti + 1) / 2;
  if (ti >= nt) return;
  const int i0 = m0 + ti * TILE, k0 = m0 + tk * TILE;
  constexpr int KC = 32;
  __shared__ T Pi[KC][TILE];
  __shared__ T Pk[KC][TILE];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int wi = w >> 1, wk = w & 1;
  typename M::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = M::zero();
  const int lr = l & 15, lk = l >> 4;
  for (int cc = 0; cc < NB; cc += KC) {
    __syncthreads();
    for (int idx = tid; idx < TILE * KC; idx += blockDim.x) {
      int r = idx % TILE, c = idx / TILE;
      T vi = 0, vk = 0;
      if (cc + c < b) {
        const T *col = J.A + (int64_t)(j0 + cc + c) * J.ld;
        if (i0 + r < J.n) vi = col[i0 + r];
        if (k0 + r < J.n) vk = col[k0 + r] * ((j0 + cc + c < J.p) ? T(1) : T(-1));
      }
      Pi[c][r] = vi;
      Pk[c][r] = vk;
    }
    __syncthreads();
    for (int c0 = 0; c0 < KC; c0 += 4) {
      T av[2], bv[2];
      for (int q = 0; q < 2; ++q) {
        av[q] = Pk[c0 + lk][32 * wk + 16 * q + lr];
        bv[q] = Pi[c0 + lk][32 * wi + 16 * q + lr];
      }
      for (int bi = 0; bi < 2; ++bi)
        for (int bk = 0; bk < 2; ++bk) acc[bi][bk] = M::mma(av[bk], bv[bi], acc[bi][bk]);
    }
  }
  for (int bi = 0; bi < 2; ++bi)
    for (int bk = 0; bk < 2; ++bk) {
      const int row = i0 + 32 * wi + 16 * bi + lr;
      if (row >= J.n) continue;
      for (int q = 0; q < 4; ++q) {
        const int col = k0 + 32 * wk + 16 * bk + M::row(lk, q);
        if (col < J.n) J.A[(int64_t)row + (int64_t)col * J.ld] -= acc[bi][bk][q];
      }
    }
}

// C = alpha A B^T + beta C (column-major), 64x64 tiles, K in chunks of 64.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nt(const GemmJob<T> *jobs) {
  typedef Mfma<T> M;
  const GemmJob<T> J = jobs[blockIdx.z];
  const int i0 = blockIdx.x * TILE, j0 = blockIdx.y * TILE;
  if (i0 >= J.m || j0 >= J.n) return;
  constexpr int KC = 32;
  __shared__ T As[KC][TILE];
  __shared__ T Bs[KC][TILE];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int wi = w >> 1, wj = w & 1, lr = l & 15, lk = l >> 4;
  typename M::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = M::zero();
  for (int k0 = 0; k0 < J.k; k0 += KC) {
    __syncthreads();
    for (int idx = tid; idx < TILE * KC; idx += blockDim.x) {
      int r = idx % TILE, c = idx / TILE;
      T va = 0, vb = 0;
      if (k0 + c < J.k) {
        if (i0 + r < J.m) va = J.A[(int64_t)(i0 + r) + (int64_t)(k0 + c) * J.lda];
        if (j0 + r < J.n) vb = J.B[(int64_t)(j0 + r) + (int64_t)(k0 + c) * J.ldb];
      }
      As[c][r] = va;
      Bs[c][r] = vb;
    }
    __syncthreads();
    for (int c0 = 0; c0 < KC; c0 += 4) {
      T av[2], bv[2];
      for (int q = 0; q < 2; ++q) {
        av[q] = Bs[c0 + lk][32 * wj + 16 * q + lr];
        bv[q] = As[c0 + lk][32 * wi + 16 * q + lr];
      }
      for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = M::mma(av[bj], bv[bi], acc[bi][bj]);
    }
  }
  for (int bi = 0; bi < 2; ++bi)
    for (int bj = 0; bj < 2; ++bj) {
      const int row = i0 + 32 * wi + 16 * bi + lr;
      if (row >= J.m) continue;
      for (int q = 0; q < 4; ++q) {
        const int col = j0 + 32 * wj + 16 * bj + M::row(lk, q);
        if (col >= J.n) continue;
        T *c = J.C + (int64_t)row + (int64_t)col * J.ldc;
        *c = J.alpha * acc[bi][bj][q] + (J.beta == T(0) ? T(0) : J.beta * *c);
      }
    }
}

// ---------------------------------------------------------------- launchers
template <typename T>
hipError_t ldl_batched(const LdlJob<T> *d_jobs, int batch, int max_n, int max_e, int nb,
                       hipStream_t s, KTimer *timer, const std::vector<int> *hn,
                       const std::vector<int> *he) {
  if (batch == 0 || max_e == 0) return hipSuccess;
  for (int j0 = 0; j0 < max_e; j0 += nb) {
    // algorithmic flops of this trailing update: b * m (m + 1) per matrix
    // (symmetric rank-b update of the m x m lower triangle)
    double flops = 0.0;
    if (timer && hn && he)
      for (size_t q = 0; q < hn->size(); ++q) {
        if (j0 >= (*he)[q]) continue;
        const double b = std::min(nb, (*he)[q] - j0);
        const double m = (*hn)[q] - j0 - b;
        if (m > 0) flops += b * m * (m + 1.0);
      }
    const int rows = max_n - j0;  // upper bound on rows below the panel start
    const int rt = (rows + TILE - 1) / TILE;
    const int nt = rt * (rt + 1) / 2;
    const int pt = (rows + PROWS - 1) / PROWS;
    if (nb == 64) {
      hipLaunchKernelGGL((k_ldl_diag<T, 64>), dim3(batch), dim3(256), 0, s, d_jobs, j0);
      if (rt > 0) {
        hipLaunchKernelGGL((k_ldl_panel<T, 64>), dim3(pt, batch), dim3(256), 0, s, d_jobs, j0);
        if (timer) { hipError_t r = timer->begin(s, flops); if (r != hipSuccess) return r; }
        hipLaunchKernelGGL((k_ldl_update<T, 64>), dim3(nt, batch), dim3(256), 0, s, d_jobs, j0);
        if (timer) { hipError_t r = timer->end(s); if (r != hipSuccess) return r; }
      }
    } else {
      hipLaunchKernelGGL((k_ldl_diag<T, 32>), dim3(batch), dim3(256), 0, s, d_jobs, j0);
      if (rt > 0) {
        hipLaunchKernelGGL((k_ldl_panel<T, 32>), dim3(pt, batch), dim3(256), 0, s, d_jobs, j0);
        hipLaunchKernelGGL((k_ldl_update<T, 32>), dim3(nt, batch), dim3(256), 0, s, d_jobs, j0);
      }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t gemm_nt_batched(const GemmJob<T> *d_jobs, int batch, int max_m, int max_n,
                           hipStream_t s) {
  if (batch == 0 || max_m == 0 || max_n == 0) return hipSuccess;
  dim3 g((max_m + TILE - 1) / TILE, (max_n + TILE - 1) / TILE, batch);
  hipLaunchKernelGGL((k_gemm_nt<T>), g, dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

template hipError_t ldl_batched<double>(const LdlJob<double> *, int, int, int, int, hipStream_t,
                                        KTimer *, const std::vector<int> *, const std::vector<int> *);
template hipError_t ldl_batched<float>(const LdlJob<float> *, int, int, int, int, hipStream_t,
                                       KTimer *, const std::vector<int> *, const std::vector<int> *);
template hipError_t gemm_nt_batched<double>(const GemmJob<double> *, int, int, int, hipStream_t);
template hipError_t gemm_nt_batched<float>(const GemmJob<float> *, int, int, int, hipStream_t);

}  // namespace vb
