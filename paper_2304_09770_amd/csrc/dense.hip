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
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace vb {

constexpr int TILE = 64;

// Rows of J that an update from the columns below `end` can change: all of
// them, or, for an identity-bordered matrix, those above zrow + end (the
// identity rows further down are still zero in those columns).
template <typename T> __host__ __device__ __forceinline__ int row_limit(const LdlJob<T> &J, int end) {
  return J.zrow > 0 ? min(J.n, J.zrow + end) : J.n;
}

// Broadcast of lane `l` (a compile-time constant after unrolling) to the wave.
__device__ __forceinline__ float lane_bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_bcast(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, l), hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// f(integral_constant<I>) for I = B .. E - 1, unrolled at compile time (the
// register arrays below are indexed only by these constants).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(const F &f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// The NB x NB diagonal block of a panel, one wave per matrix, lane r holding
// row r in registers: column by column the pivot d_c a_cc (lane c) and the
// column entries l_kc (lane k) are broadcast, each lane scales its entry of
// the column and updates its row (a right-looking unblocked LDL^T).  Then
// inv(L_jj) in place, row by row (forward substitution of L X = I: row t of
// X is final once lane t has divided by l_tt; the lanes below subtract
// l_rt times it).  Rows and columns at or beyond b hold zeros.
template <typename T, int NB>
__global__ __launch_bounds__(64) void k_ldl_diag(const LdlJob<T> *jobs, int j0) {
  const LdlJob<T> J = jobs[blockIdx.x];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  const int r = threadIdx.x;
  const bool row = r < b;
  T a[NB];
  static_for<0, NB>([&](auto k) {
    a[k] = (row && k <= r && k < b) ? J.A[(int64_t)(j0 + r) + (int64_t)(j0 + k) * J.ld] : T(0);
  });
  bool bad = false;
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if (c < b) {  // uniform
      const T d = (j0 + c < J.p) ? T(1) : T(-1);
      T v = d * lane_bcast(a[c], c);
      if (!(v > T(J.pmin))) {  // wrong-signed, zero or too small pivot: report, keep going finitely
        if (!bad && r == 0) atomicCAS(J.info, 0, j0 + c + 1);
        bad = true;
        v = T(1);
      }
      const T l = sqrt(v);
      if (r == c) a[c] = l;
      if (r > c) a[c] /= d * l;
      const T f = (r > c) ? a[c] * d : T(0);  // l_rc d_c on the rows below
      static_for<c + 1, NB>([&](auto k) { a[k] -= f * lane_bcast(a[c], k); });
    }
  });
  if (row)
    static_for<0, NB>([&](auto k) {
      if (k <= r) J.A[(int64_t)(j0 + r) + (int64_t)(j0 + k) * J.ld] = a[k];
    });
  // X = inv(L_jj) over the same registers: after step t, lanes r <= t hold
  // row r of X, lanes r > t the partial rows of the remaining system
  static_for<0, NB>([&](auto tt) {
    constexpr int t = decltype(tt)::value;
    if (t < b) {  // uniform
      const T rd = T(1) / lane_bcast(a[t], t);
      if (r == t) {
        static_for<0, t>([&](auto k) { a[k] *= rd; });
        a[t] = rd;
      }
      const T lrt = a[t];  // l_rt on the rows below t
      static_for<0, t + 1>([&](auto k) {
        const T x = lane_bcast(a[k], t);  // X[t][k]
        if (r > t) a[k] = (k < t) ? a[k] - lrt * x : -lrt * x;
      });
    }
  });
  T *inv = J.invL + (int64_t)(j0 / NB) * NB * NB;
  if (r < NB) static_for<0, NB>([&](auto k) { inv[r + k * NB] = (row && k <= r) ? a[k] : T(0); });
}

// L_ij = A_ij inv(L_jj)^T D_j for rows [j0+b, n) in tiles of PROWS rows.
constexpr int PROWS = 32;
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ldl_panel(const LdlJob<T> *jobs, int j0) {
  const LdlJob<T> J = jobs[blockIdx.y];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  const int nl = row_limit(J, j0 + b);
  const int r0 = j0 + b + blockIdx.x * PROWS;
  if (r0 >= nl) return;
  __shared__ T Li[NB][NB];
  __shared__ T At[NB][PROWS];
  const int tid = threadIdx.x;
  const T *inv = J.invL + (int64_t)(j0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) Li[idx % NB][idx / NB] = inv[idx];
  for (int idx = tid; idx < PROWS * NB; idx += blockDim.x) {
    int r = idx % PROWS, t = idx / PROWS;
    T v = 0;
    if (r0 + r < nl && t < b) v = J.A[(int64_t)(r0 + r) + (int64_t)(j0 + t) * J.ld];
    At[t][r] = v;
  }
  __syncthreads();
  const int r = tid % PROWS;
  const int cg = tid / PROWS;  // 0..7
  if (r0 + r >= nl) return;
  for (int c = cg; c < b; c += 8) {
    T s = 0;
    for (int t = 0; t <= c; ++t) s += At[t][r] * Li[c][t];
    T d = (j0 + c < J.p) ? T(1) : T(-1);
    J.A[(int64_t)(r0 + r) + (int64_t)(j0 + c) * J.ld] = d * s;
  }
}

// The same panel on the matrix cores (NB = 64): a workgroup takes 64 rows,
// C[c][r] = sum_t inv(L_jj)[c][t] A[r][t] (t <= c; the inverse block is
// lower triangular, zero above), then L[r][c] = d_c C[c][r].  Both operands
// are staged in LDS; each wave computes a 32 x 32 block.
template <typename T>
__global__ __launch_bounds__(256) void k_ldl_panel_mfma(const LdlJob<T> *jobs, int j0) {
  typedef Mfma<T> M;
  constexpr int NB = 64, PR = 64;
  const LdlJob<T> J = jobs[blockIdx.y];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  const int nl = row_limit(J, j0 + b);
  const int r0 = j0 + b + blockIdx.x * PR;
  if (r0 >= nl) return;
  __shared__ T Pc[NB][NB + 1];  // Pc[t][c] = inv(L_jj)[c][t]
  __shared__ T Pr[NB][PR + 1];  // Pr[t][r] = A[r0 + r][j0 + t]
  const int tid = threadIdx.x;
  const T *inv = J.invL + (int64_t)(j0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) Pc[idx / NB][idx % NB] = inv[idx];
  for (int idx = tid; idx < PR * NB; idx += blockDim.x) {
    const int r = idx % PR, t = idx / PR;
    T v = 0;
    if (r0 + r < nl && t < b) v = J.A[(int64_t)(r0 + r) + (int64_t)(j0 + t) * J.ld];
    Pr[t][r] = v;
  }
  __syncthreads();
  const int w = tid >> 6, l = tid & 63;
  const int wr = w >> 1, wc = w & 1, lr = l & 15, lk = l >> 4;
  typename M::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = M::zero();
  for (int t0 = 0; t0 < NB; t0 += 4) {
    T av[2], bv[2];
    for (int q = 0; q < 2; ++q) {
      av[q] = Pc[t0 + lk][32 * wc + 16 * q + lr];
      bv[q] = Pr[t0 + lk][32 * wr + 16 * q + lr];
    }
    for (int br = 0; br < 2; ++br)
      for (int bc = 0; bc < 2; ++bc) acc[br][bc] = M::mma(av[bc], bv[br], acc[br][bc]);
  }
  for (int br = 0; br < 2; ++br)
    for (int bc = 0; bc < 2; ++bc) {
      const int row = r0 + 32 * wr + 16 * br + lr;
      if (row >= nl) continue;
      for (int q = 0; q < 4; ++q) {
        const int c = 32 * wc + 16 * bc + M::row(lk, q);
        if (c < b) {
          const T d = (j0 + c < J.p) ? T(1) : T(-1);
          J.A[(int64_t)row + (int64_t)(j0 + c) * J.ld] = d * acc[br][bc][q];
        }
      }
    }
}

// A_ik -= L_ij D_j L_kj^T on 64x64 tiles of the trailing matrix, restricted
// to columns < col_end (the rest of the current super-panel): tile (ti, tk)
// with ti >= tk from a rectangular grid of nt x ntk tiles.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ldl_update(const LdlJob<T> *jobs, int j0, int col_end,
                                                    int ntk_max) {
  typedef Mfma<T> M;
  const LdlJob<T> J = jobs[blockIdx.y];
  if (j0 >= J.e) return;
  const int b = min(NB, J.e - j0);
  const int m0 = j0 + b;
  const int ce = min(col_end, J.e);
  const int nl = row_limit(J, j0 + b);
  if (m0 >= nl || m0 >= ce) return;
  const int nt = (nl - m0 + TILE - 1) / TILE;
  const int ti = blockIdx.x / ntk_max, tk = blockIdx.x % ntk_max;
  if (ti >= nt || tk > ti) return;
  const int i0 = m0 + ti * TILE, k0 = m0 + tk * TILE;
  if (k0 >= ce) return;
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
  const int r = tid & (TILE - 1), c4 = tid >> 6;  // staging: row r, columns c4 + 4q
  const int ri = min(i0 + r, J.n - 1), rk = min(k0 + r, J.n - 1);
  const bool oki = (i0 + r < nl), okk = (k0 + r < ce);
  for (int cc = 0; cc < NB; cc += KC) {
    T vi[KC / 4], vk[KC / 4];
#pragma unroll
    for (int q = 0; q < KC / 4; ++q) {
      const int c = cc + c4 + 4 * q;
      const int cl = j0 + min(c, b - 1);
      const auto col = gptr(J.A + (int64_t)cl * J.ld);
      const T a0 = col[ri], a1 = col[rk];
      const bool okc = c < b;
      const T d = (j0 + c < J.p) ? T(1) : T(-1);
      vi[q] = (okc && oki) ? a0 : T(0);
      vk[q] = (okc && okk) ? a1 * d : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KC / 4; ++q) {
      Pi[c4 + 4 * q][r] = vi[q];
      Pk[c4 + 4 * q][r] = vk[q];
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
      if (row >= nl) continue;
      for (int q = 0; q < 4; ++q) {
        const int col = k0 + 32 * wk + 16 * bk + M::row(lk, q);
        if (col < ce) J.A[(int64_t)row + (int64_t)col * J.ld] -= acc[bi][bk][q];
      }
    }
}

// Rank-(super-panel) trailing update A_ik -= sum_{c in [kb, ke)} L_ic d_c L_kc
// on the lower triangle beyond the super-panel, 128x128 tiles (each wave a
// 64x64 block of 4x4 matrix-core tiles).  The panel columns are staged
// through LDS in chunks of KW; the next chunk is loaded into registers
// (branch-free, clamped addresses) while the current one is multiplied.
constexpr int WT = 128;
// Panel columns staged per pass: the FP32 products take half the matrix-core
// time of FP64 ones, so FP32 stages twice as many columns (same LDS bytes) to
// keep the prefetch of the next chunk hidden behind the current one.
template <typename T> struct WideKW { static constexpr int value = 16; };
template <> struct WideKW<float> { static constexpr int value = 32; };
// RECT: only the columns [ke, min(col_end, e)) of the trailing matrix (the
// rest of an enclosing super-panel); the tiles are enumerated column block
// by column block, nt_max row tiles per block.  Otherwise the whole lower
// triangle beyond ke, tiles enumerated row by row.
template <typename T, bool RECT>
__device__ __forceinline__ void ldl_update_wide_body(const LdlJob<T> *jobs, int J0, int SB,
                                                     int col_end, int nt_max) {
  typedef Mfma<T> M;
  constexpr int KW = WideKW<T>::value;
  const LdlJob<T> J = jobs[blockIdx.y];
  const int kb = J0, ke = min(J0 + SB, J.e);
  if (kb >= ke) return;
  const int m0 = ke;
  const int nl = row_limit(J, ke);
  if (m0 >= nl) return;
  const int nt = (nl - m0 + WT - 1) / WT;
  const int t = blockIdx.x;
  int ti, tk, ce;
  if (RECT) {
    ce = min(col_end, J.e);
    if (ce <= m0) return;
    const int ntk = (ce - m0 + WT - 1) / WT;
    int rem = t;
    tk = 0;
    while (tk < ntk && rem >= nt_max - tk) {
      rem -= nt_max - tk;
      ++tk;
    }
    if (tk >= ntk) return;
    ti = tk + rem;
  } else {
    ce = nl;
    ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    tk = t - ti * (ti + 1) / 2;
  }
  if (ti >= nt) return;
  const int i0 = m0 + ti * WT, k0 = m0 + tk * WT;
  extern __shared__ unsigned char smem_raw[];
  T *Pi = reinterpret_cast<T *>(smem_raw);
  T *Pk = Pi + KW * WT;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int wi = w >> 1, wk = w & 1;
  const int lr = l & 15, lk = l >> 4;
  // staging map: row r (128), columns c = c0 + 2q (q < KW/2)
  const int r = tid & (WT - 1), c0 = tid >> 7;
  const int ri = min(i0 + r, J.n - 1), rk = min(k0 + r, J.n - 1);
  const bool oki = (i0 + r < nl), okk = (k0 + r < ce);
  constexpr int NQ = KW / 2;
  T bi_[NQ], bk_[NQ];
  // raw loads only: the masks and pivot signs are applied when the values are
  // stored to LDS, after the current chunk's products, so every load of a
  // chunk stays in flight while the matrix cores work
  auto load = [&](int cc) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int cl = min(cc + c0 + 2 * q, ke - 1);
      const auto col = gptr(J.A + (int64_t)cl * J.ld);
      bi_[q] = col[ri];
      bk_[q] = col[rk];
    }
  };
  typename M::acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = M::zero();
  load(kb);
  for (int cc = kb; cc < ke; cc += KW) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = cc + c0 + 2 * q;
      const bool okc = c < ke;
      const T d = (c < J.p) ? T(1) : T(-1);
      Pi[(c0 + 2 * q) * WT + r] = (okc && oki) ? bi_[q] : T(0);
      Pk[(c0 + 2 * q) * WT + r] = (okc && okk) ? bk_[q] * d : T(0);
    }
    __syncthreads();
    if (cc + KW < ke) load(cc + KW);
#pragma unroll 2
    for (int s0 = 0; s0 < KW; s0 += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = Pk[(s0 + lk) * WT + 64 * wk + 16 * q + lr];
        bv[q] = Pi[(s0 + lk) * WT + 64 * wi + 16 * q + lr];
      }
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bk = 0; bk < 4; ++bk) acc[bi][bk] = M::mma(av[bk], bv[bi], acc[bi][bk]);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bk = 0; bk < 4; ++bk) {
      const int row = i0 + 64 * wi + 16 * bi + lr;
      if (row >= nl) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = k0 + 64 * wk + 16 * bk + M::row(lk, q);
        if (col < ce) J.A[(int64_t)row + (int64_t)col * J.ld] -= acc[bi][bk][q];
      }
    }
}

// FP64: 206 VGPRs, two waves per SIMD.  FP32: 124 VGPRs and half the LDS
// bytes per stage, four waves per SIMD.
// The triangular update for matrices whose columns start on 16-byte
// boundaries (leading dimension a multiple of 16 bytes): the panel strips go
// from HBM straight into LDS (global_load_lds_dwordx4, no registers, no LDS
// stores), double-buffered in chunks of 16 (FP32) or 8 (FP64) columns, so
// each chunk costs one barrier and the next chunk's loads overlap the
// current chunk's matrix-core work.  Every load is 16-byte aligned: the tile
// grid starts at ke rounded down to a multiple of VW = 16 / sizeof(T) rows;
// a group of VW rows that starts below ld is read as it is (ld is a multiple
// of VW, so it ends inside the column), a group starting at or beyond ld is
// read from the column's last VW rows instead; rows below ke (panel rows)
// and at or beyond n enter the products only for outputs that are never
// written; columns at or beyond ke are loaded as (finite) copies of column
// ke-1 and weighted 0.
template <typename T> struct Dma {
  static constexpr int VW = 16 / sizeof(T);   // entries per 16-byte load
  static constexpr int KW = 64 / sizeof(T);   // columns per chunk (16 KB per buffer pair)
  static constexpr int CPI = 64 * VW / WT;    // strip columns per wave-wide load
};
template <typename T>
__device__ __forceinline__ void dma16(const T *g, T *lds_wave_base) {
  __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                   (void __attribute__((address_space(3))) *)lds_wave_base, 16, 0, 0);
}
template <typename T>
__device__ __forceinline__ void ldl_update_dma_body(const LdlJob<T> *jobs, int J0, int SB) {
  typedef Mfma<T> M;
  constexpr int VW = Dma<T>::VW, DKW = Dma<T>::KW, CPI = Dma<T>::CPI;
  constexpr int NI = DKW / CPI / 4;  // wave-wide loads per strip, wave and chunk
  const LdlJob<T> J = jobs[blockIdx.y];
  const int kb = J0, ke = min(J0 + SB, J.e);
  if (kb >= ke) return;
  const int m0 = ke;
  const int nl = row_limit(J, ke);
  if (m0 >= nl) return;
  const int m0a = m0 & ~(VW - 1);
  const int nt = (nl - m0a + WT - 1) / WT;
  const int t = blockIdx.x;
  int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tk = t - ti * (ti + 1) / 2;
  if (ti >= nt) return;
  const int i0 = m0a + ti * WT, k0 = m0a + tk * WT;
  __shared__ __align__(16) T PiA[DKW * WT], PkA[DKW * WT], PiB[DKW * WT], PkB[DKW * WT];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int wi = w >> 1, wk = w & 1, lr = l & 15, lk = l >> 4;
  // load map: wave w, load j -> strip columns CPI (w + 4 j) .. + CPI - 1;
  // lane l -> column + l / (WT / VW), rows VW (l % (WT / VW)) .. + VW - 1
  const int lc = l / (WT / VW), lrow = VW * (l % (WT / VW));
  const int64_t last = J.ld - VW;  // the last group of a column
  const int64_t ri = min((int64_t)(i0 + lrow), last), rk = min((int64_t)(k0 + lrow), last);
  auto issue = [&](int cc, T *Pi, T *Pk) {
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int c0 = CPI * (w + 4 * j);
      const int cl = min(cc + c0 + lc, ke - 1);
      const T *col = J.A + (int64_t)cl * J.ld;
      dma16(col + ri, Pi + c0 * WT);
      dma16(col + rk, Pk + c0 * WT);
    }
  };
  typename M::acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = M::zero();
  auto compute = [&](int cc, const T *Pi, const T *Pk) {
#pragma unroll
    for (int s0 = 0; s0 < DKW; s0 += 4) {
      const int c = cc + s0 + lk;
      const T d = (c < ke) ? ((c < J.p) ? T(1) : T(-1)) : T(0);
      T av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = Pk[(s0 + lk) * WT + 64 * wk + 16 * q + lr] * d;
        bv[q] = Pi[(s0 + lk) * WT + 64 * wi + 16 * q + lr];
      }
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bk = 0; bk < 4; ++bk) acc[bi][bk] = M::mma(av[bk], bv[bi], acc[bi][bk]);
    }
  };
  issue(kb, PiA, PkA);
  for (int cc = kb; cc < ke; cc += 2 * DKW) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads of chunk cc
    __syncthreads();
    if (cc + DKW < ke) issue(cc + DKW, PiB, PkB);
    compute(cc, PiA, PkA);
    if (cc + DKW >= ke) break;
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (cc + 2 * DKW < ke) issue(cc + 2 * DKW, PiA, PkA);
    compute(cc + DKW, PiB, PkB);
  }
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bk = 0; bk < 4; ++bk) {
      const int row = i0 + 64 * wi + 16 * bi + lr;
      if (row < m0 || row >= nl) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = k0 + 64 * wk + 16 * bk + M::row(lk, q);
        if (col >= m0 && col < nl) J.A[(int64_t)row + (int64_t)col * J.ld] -= acc[bi][bk][q];
      }
    }
}

// The local Dirichlet factorisations (timed per launch), the other
// factorisations (Neumann, deluxe, coarse, face problems) and matrices that
// are not 16-byte aligned (staged kernel) run under separate kernel names so
// that profiles separate them.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ldl_update_wide_f32(const LdlJob<float> *jobs, int J0, int SB) {
  ldl_update_dma_body<float>(jobs, J0, SB);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_ldl_update_wide_f64(const LdlJob<double> *jobs, int J0, int SB) {
  ldl_update_dma_body<double>(jobs, J0, SB);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ldl_update_wide_aux_f32(const LdlJob<float> *jobs, int J0, int SB) {
  ldl_update_dma_body<float>(jobs, J0, SB);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_ldl_update_wide_aux_f64(const LdlJob<double> *jobs, int J0, int SB) {
  ldl_update_dma_body<double>(jobs, J0, SB);
}

// the staged kernel for matrices that are not 16-byte aligned
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_ldl_update_wide_u_f64(const LdlJob<double> *jobs, int J0, int SB) {
  ldl_update_wide_body<double, false>(jobs, J0, SB, 0, 0);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ldl_update_wide_u_f32(const LdlJob<float> *jobs, int J0, int SB) {
  ldl_update_wide_body<float, false>(jobs, J0, SB, 0, 0);
}
// the update inside an enclosing super-panel (columns up to its end)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_ldl_update_rect_f64(const LdlJob<double> *jobs, int J0, int SB, int col_end, int nt_max) {
  ldl_update_wide_body<double, true>(jobs, J0, SB, col_end, nt_max);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_ldl_update_rect_f32(const LdlJob<float> *jobs, int J0, int SB, int col_end, int nt_max) {
  ldl_update_wide_body<float, true>(jobs, J0, SB, col_end, nt_max);
}
template <typename T> struct WideKernel;
template <> struct WideKernel<double> {
  static constexpr auto fn = k_ldl_update_wide_f64;       // 16-byte aligned, Dirichlet
  static constexpr auto aux = k_ldl_update_wide_aux_f64;  // 16-byte aligned, others
  static constexpr auto u = k_ldl_update_wide_u_f64;      // not aligned
  static constexpr auto rect = k_ldl_update_rect_f64;
};
template <> struct WideKernel<float> {
  static constexpr auto fn = k_ldl_update_wide_f32;
  static constexpr auto aux = k_ldl_update_wide_aux_f32;
  static constexpr auto u = k_ldl_update_wide_u_f32;
  static constexpr auto rect = k_ldl_update_rect_f32;
};

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
template <typename T, int NB>
static hipError_t ldl_panel_step(const LdlJob<T> *d_jobs, int batch, int max_n, int j0, int col_end,
                                 hipStream_t s) {
  const int rows = max_n - j0;
  const int pt = (rows + PROWS - 1) / PROWS;
  const int rt = (rows + TILE - 1) / TILE;
  const int ntk = (col_end - j0 + TILE - 1) / TILE;
  hipLaunchKernelGGL((k_ldl_diag<T, NB>), dim3(batch), dim3(64), 0, s, d_jobs, j0);
  if (rows > 0) {
    if (NB == 64)
      hipLaunchKernelGGL((k_ldl_panel_mfma<T>), dim3((rows + 63) / 64, batch), dim3(256), 0, s,
                         d_jobs, j0);
    else
      hipLaunchKernelGGL((k_ldl_panel<T, NB>), dim3(pt, batch), dim3(256), 0, s, d_jobs, j0);
    if (ntk > 0)
      hipLaunchKernelGGL((k_ldl_update<T, NB>), dim3(rt * ntk, batch), dim3(256), 0, s, d_jobs,
                         j0, col_end, ntk);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t ldl_batched(const LdlJob<T> *d_jobs, int batch, int max_n, int max_e, int nb,
                       hipStream_t s, KTimer *timer, const std::vector<int> *hn,
                       const std::vector<int> *he, bool dirichlet, bool aligned16, int sb1,
                       const std::vector<int> *hz) {
  if (batch == 0 || max_e == 0) return hipSuccess;
  // the largest row bound over the jobs for an update from the columns below end
  auto rows_to = [&](int end) {
    if (!hz || !hn) return max_n;
    int r = 0;
    for (size_t q = 0; q < hn->size(); ++q)
      r = std::max(r, (*hz)[q] > 0 ? std::min((*hn)[q], (*hz)[q] + end) : (*hn)[q]);
    return std::min(r, max_n);
  };
  if (nb != 32 && nb != 64) return hipErrorInvalidValue;
  if (sb1 == 0) sb1 = 16 * nb;
  if (sb1 <= 0 || sb1 % (4 * nb)) return hipErrorInvalidValue;
  static bool attr = false;
  const size_t lds = 2 * (size_t)WideKW<T>::value * WT * sizeof(T);
  if (!attr) {
    hipError_t r = hipFuncSetAttribute((const void *)k_ldl_update_wide_u_f64,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void *)k_ldl_update_wide_u_f32,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void *)k_ldl_update_rect_f64,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void *)k_ldl_update_rect_f32,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (r != hipSuccess) return r;
    attr = true;
  }
  // two levels of super-panels: the columns of an outer super-panel (SB1)
  // are factored in inner super-panels (SB2) of nb-wide panels; the update
  // of the rest of the outer super-panel follows each inner one, the update
  // of the whole trailing matrix each outer one (rank SB1)
  const int SB1 = sb1, SB2 = 4 * nb;
  for (int J0 = 0; J0 < max_e; J0 += SB1) {
    const int j1end = std::min(J0 + SB1, max_e);
    for (int J1 = J0; J1 < j1end; J1 += SB2) {
      const int j2end = std::min(J1 + SB2, max_e);
      for (int j0 = J1; j0 < j2end; j0 += nb) {
        const int mr = rows_to(j0 + nb);
        hipError_t r = (nb == 64) ? ldl_panel_step<T, 64>(d_jobs, batch, mr, j0, J1 + SB2, s)
                                  : ldl_panel_step<T, 32>(d_jobs, batch, mr, j0, J1 + SB2, s);
        if (r != hipSuccess) return r;
      }
      const int ncols = J0 + SB1 - (J1 + SB2);
      const int mr = rows_to(J1 + SB2);
      if (ncols > 0 && mr > J1) {
        const int nt_max = (mr - J1 + WT - 1) / WT;
        const int ntk = std::min(nt_max, (ncols + WT - 1) / WT);
        const int ntiles = ntk * nt_max - ntk * (ntk - 1) / 2;
        hipLaunchKernelGGL(WideKernel<T>::rect, dim3(ntiles, batch), dim3(256), lds, s, d_jobs, J1,
                           SB2, J0 + SB1, nt_max);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    // algorithmic flops of the trailing update: K * m * (m + 1) per matrix
    // (symmetric rank-K update of the m x m lower triangle)
    double flops = 0.0;
    if (timer && hn && he)
      for (size_t q = 0; q < hn->size(); ++q) {
        if (J0 >= (*he)[q]) continue;
        const int ke = std::min(J0 + SB1, (*he)[q]);
        const int nl = (hz && (*hz)[q] > 0) ? std::min((*hn)[q], (*hz)[q] + ke) : (*hn)[q];
        const double K = ke - J0;
        const double m = nl - ke;
        if (m > 0) flops += K * m * (m + 1.0);
      }
    // a job whose elimination ends inside this super-panel has n - e_job
    // trailing rows: size the grid by the upper bound max_n - J0 (or the
    // identity-bordered jobs' row bound)
    const int rows = rows_to(J0 + SB1) - J0;
    if (rows > 0) {
      // the aligned kernels start their tile grid up to VW - 1 rows lower
      const int wt = (rows + (aligned16 ? Dma<T>::VW : 0) + WT - 1) / WT;
      const int ntiles = wt * (wt + 1) / 2;
      if (timer) { hipError_t r = timer->begin(s, flops); if (r != hipSuccess) return r; }
      if (!aligned16)
        hipLaunchKernelGGL(WideKernel<T>::u, dim3(ntiles, batch), dim3(256), lds, s, d_jobs, J0,
                           SB1);
      else if (dirichlet)
        hipLaunchKernelGGL(WideKernel<T>::fn, dim3(ntiles, batch), dim3(256), 0, s, d_jobs, J0, SB1);
      else
        hipLaunchKernelGGL(WideKernel<T>::aux, dim3(ntiles, batch), dim3(256), 0, s, d_jobs, J0,
                           SB1);
      if (timer) { hipError_t r = timer->end(s); if (r != hipSuccess) return r; }
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
                                        KTimer *, const std::vector<int> *, const std::vector<int> *,
                                        bool, bool, int, const std::vector<int> *);
template hipError_t ldl_batched<float>(const LdlJob<float> *, int, int, int, int, hipStream_t,
                                       KTimer *, const std::vector<int> *, const std::vector<int> *,
                                       bool, bool, int, const std::vector<int> *);
template hipError_t gemm_nt_batched<double>(const GemmJob<double> *, int, int, int, hipStream_t);
template hipError_t gemm_nt_batched<float>(const GemmJob<float> *, int, int, int, hipStream_t);

}  // namespace vb
