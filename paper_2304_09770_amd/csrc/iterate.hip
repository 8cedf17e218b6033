// Per-iteration kernels of PCG + BDDC (HBM-bound dense GEMVs, gathers,
// deterministic interface assembly and the CG recurrences).
#include <algorithm>

#include "common.h"
#include "iterate.h"

namespace vb {

// y_b[j] = alpha * sum_i A_b[i + j*lda] x_b[i] (+ y_b[j] if accumulate), one
// wave per column, CPB columns per workgroup.  Columns are contiguous in HBM:
// every wave streams its columns.  x_b (gathered through xidx if given) is
// staged through LDS in chunks of GT_CHUNK rows, so a workgroup holds 16 KB
// of LDS whatever the size of its operator and many workgroups share a CU
// (the largest operators of an uneven decomposition would otherwise run at
// two workgroups per CU).
constexpr int GT_CHUNK = 2048;
// The body of one workgroup (bx, by) of the launch: shared by the standalone
// kernel and the persistent PCG kernel (xs: GT_CHUNK doubles of LDS).
template <int CPB>
__device__ __forceinline__ void gemv_t_block(const GemvJob *jobs, int bx, int by, double *xs) {
  constexpr int NQ = CPB / 4;
  const GemvJob J = jobs[by];
  const int j0 = bx * CPB;
  if (j0 >= J.n) return;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int c0 = 0; c0 < J.m; c0 += GT_CHUNK) {
    const int cm = min(GT_CHUNK, J.m - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < cm; i += blockDim.x)
      xs[i] = J.xidx ? J.x[J.xidx[c0 + i]] : J.x[c0 + i];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = j0 + w + 4 * q;
      if (j >= J.n) break;
      // eight loads per lane in flight, then pairs, then the last row
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      auto dot = [&](auto col) {
        int i = l;
        for (; i + 448 < cm; i += 512) {
          const double a0 = col[i], a1 = col[i + 64], a2 = col[i + 128], a3 = col[i + 192];
          const double a4 = col[i + 256], a5 = col[i + 320], a6 = col[i + 384], a7 = col[i + 448];
          s0 += a0 * xs[i] + a4 * xs[i + 256];
          s1 += a1 * xs[i + 64] + a5 * xs[i + 320];
          s2 += a2 * xs[i + 128] + a6 * xs[i + 384];
          s3 += a3 * xs[i + 192] + a7 * xs[i + 448];
        }
        for (; i + 64 < cm; i += 128) {
          s0 += (double)col[i] * xs[i];
          s1 += (double)col[i + 64] * xs[i + 64];
        }
        if (i < cm) s0 += (double)col[i] * xs[i];
      };
      if (J.a_f32)
        dot(gptr((const float *)J.A + (int64_t)j * J.lda + c0));
      else
        dot(gptr((const double *)J.A + (int64_t)j * J.lda + c0));
      acc[q] += (s0 + s1) + (s2 + s3);
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int j = j0 + w + 4 * q;
    if (j >= J.n) break;
    const double s = warp_sum(acc[q]);
    if (l == 0) {
      double v = J.alpha * s;
      if (J.acc) v += J.y[j];
      J.y[j] = v;
      if (J.y2) J.y2[j] = (J.xidx ? J.x[J.xidx[j]] : J.x[j]) - v;
    }
  }
}

template <int CPB>
__global__ __launch_bounds__(256) void k_gemv_t(const GemvJob *jobs) {
  __shared__ double xs[GT_CHUNK];
  gemv_t_block<CPB>(jobs, blockIdx.x, blockIdx.y, xs);
}

// y_b[i] = base_b[i] + sum_j A_b[i + j*lda] x_b[j], one thread per row,
// x_b (length n, gathered through xidx) staged in LDS.
__device__ __forceinline__ void gemv_n_block(const GemvJob *jobs, int bx, int by, double *xs) {
  const GemvJob J = jobs[by];
  __syncthreads();  // xs may still be read by the previous block of a persistent loop
  for (int j = threadIdx.x; j < J.n; j += blockDim.x)
    xs[j] = J.xidx ? J.x[J.xidx[j]] : J.x[j];
  __syncthreads();
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= J.m) return;
  double s = J.base ? J.base[i] : 0.0;
  if (J.a_f32) {
    const auto a = gptr((const float *)J.A + i);
    for (int j = 0; j < J.n; ++j) s += (double)a[(int64_t)j * J.lda] * xs[j];
  } else {
    const auto a = gptr((const double *)J.A + i);
    for (int j = 0; j < J.n; ++j) s += a[(int64_t)j * J.lda] * xs[j];
  }
  J.y[i] = s;
}

__global__ __launch_bounds__(256) void k_gemv_n(const GemvJob *jobs) {
  extern __shared__ double xs[];
  gemv_n_block(jobs, blockIdx.x, blockIdx.y, xs);
}

// The staged vectors can exceed the default 64 KB of dynamic LDS; CDNA4 has
// 160 KB per CU.
static hipError_t allow_big_lds() {
  static int done = 0;
  if (done) return hipSuccess;
  const void *fs[] = {(const void *)k_gemv_n};
  for (const void *f : fs) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  done = 1;
  return hipSuccess;
}

// cpb: columns per workgroup (8, 16, 32 or 64), chosen by the autotuner.
hipError_t gemv_t_cpb(const GemvJob *d_jobs, int batch, int max_m, int max_n, int cpb,
                      hipStream_t s) {
  if (!batch || !max_n) return hipSuccess;
  (void)max_m;
  const size_t lds = 0;
  switch (cpb) {
    case 8:
      hipLaunchKernelGGL((k_gemv_t<8>), dim3((max_n + 7) / 8, batch), dim3(256), lds, s, d_jobs);
      break;
    case 16:
      hipLaunchKernelGGL((k_gemv_t<16>), dim3((max_n + 15) / 16, batch), dim3(256), lds, s, d_jobs);
      break;
    case 64:
      hipLaunchKernelGGL((k_gemv_t<64>), dim3((max_n + 63) / 64, batch), dim3(256), lds, s, d_jobs);
      break;
    default:
      hipLaunchKernelGGL((k_gemv_t<32>), dim3((max_n + 31) / 32, batch), dim3(256), lds, s, d_jobs);
      break;
  }
  return hipGetLastError();
}

hipError_t gemv_t(const GemvJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s) {
  return gemv_t_cpb(d_jobs, batch, max_m, max_n, 32, s);
}

hipError_t gemv_n(const GemvJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s) {
  if (!batch || !max_m) return hipSuccess;
  size_t lds = (size_t)(max_n > 0 ? max_n : 1) * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = allow_big_lds();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gemv_n, dim3((max_m + 255) / 256, batch), dim3(256), lds, s, d_jobs);
  return hipGetLastError();
}

// y[g] = (bidx ? bsrc[bidx[g]] : 0) + sum_{t in [ptr[g], ptr[g+1])} src[idx[t]]
// (deterministic assembly of subdomain contributions, fixed order).
__device__ __forceinline__ void owner_sum_at(int64_t g, int n, const int64_t *ptr, const int64_t *idx,
                                             const double *src, const int64_t *bidx,
                                             const double *bsrc, double *y) {
  if (g >= n) return;
  double s = bidx ? bsrc[bidx[g]] : 0.0;
  for (int64_t t = ptr[g]; t < ptr[g + 1]; ++t) s += src[idx[t]];
  y[g] = s;
}

__global__ void k_owner_sum(int n, const int64_t *ptr, const int64_t *idx, const double *src,
                            const int64_t *bidx, const double *bsrc, double *y) {
  owner_sum_at((int64_t)blockIdx.x * blockDim.x + threadIdx.x, n, ptr, idx, src, bidx, bsrc, y);
}

hipError_t owner_sum(int n, const int64_t *ptr, const int64_t *idx, const double *src,
                     const int64_t *bidx, const double *bsrc, double *y, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_owner_sum, dim3((n + 255) / 256), dim3(256), 0, s, n, ptr, idx, src, bidx,
                     bsrc, y);
  return hipGetLastError();
}

// y[dst[i]] = scale * src[sidx ? sidx[i] : i]
__global__ void k_scatter_copy(int n, const double *src, const int64_t *sidx, const int64_t *dst,
                               double *y, double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[dst ? dst[i] : i] = scale * src[sidx ? sidx[i] : i];
}

hipError_t scatter_copy(int n, const double *src, const int64_t *sidx, const int64_t *dst,
                        double *y, double scale, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_copy, dim3((n + 255) / 256), dim3(256), 0, s, n, src, sidx, dst, y,
                     scale);
  return hipGetLastError();
}

// Deluxe extension: z[gid[m]] = sum_q (D_q w_q)[m] over the subdomains of
// the entity (D_q = null: counting weights 1/card); for a pair of
// subdomains whose matrices sum to the identity, z = w_2 + D_1 (w_1 - w_2),
// so only D_1 is read.  A workgroup takes 128 rows: each lane two adjacent
// rows with one 16-byte (FP64) or 8-byte (FP32 storage) load per column (the
// matrices are stored with an even leading dimension, so the pair is
// aligned; the row past an odd m is in the column's storage and feeds no
// output).  The vector the matrix multiplies is staged in LDS in chunks of
// EXT_CHUNK columns, which the four waves split, four (FP64) or eight (FP32)
// columns in flight per lane; the partial sums are added through LDS in a
// fixed order.
constexpr int EXT_CHUNK = 1024;
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ v2d load2(const double *p) {
  return *(const __attribute__((address_space(1))) v2d *)p;
}
__device__ __forceinline__ v2d load2(const float *p) {
  const v2f f = *(const __attribute__((address_space(1))) v2f *)p;
  return v2d{(double)f.x, (double)f.y};
}
template <typename T> struct ExtUnroll { static constexpr int value = 4; };
template <> struct ExtUnroll<float> { static constexpr int value = 8; };

// s += D[m0:m0+2, :] (u - v) (v may be null); called by the whole workgroup
template <typename T>
__device__ __forceinline__ void ext_matvec(const T *D, int64_t ld, const double *u, const double *v,
                                           int m, int m0, bool rows, int wv, double *xs, double &s0,
                                           double &s1) {
  constexpr int U = ExtUnroll<T>::value;
  for (int cb = 0; cb < m; cb += EXT_CHUNK) {
    const int cm = min(EXT_CHUNK, m - cb);
    __syncthreads();
    for (int i = threadIdx.x; i < cm; i += blockDim.x) xs[i] = v ? u[cb + i] - v[cb + i] : u[cb + i];
    __syncthreads();
    if (!rows) continue;
    const int k0 = cm * wv / 4, k1 = cm * (wv + 1) / 4;
    const T *a = D + m0 + (int64_t)cb * ld;
    double t[U], q[U];
#pragma unroll
    for (int j = 0; j < U; ++j) t[j] = q[j] = 0.0;
    int l = k0;
    for (; l + U <= k1; l += U) {
      v2d d[U];
#pragma unroll
      for (int j = 0; j < U; ++j) d[j] = load2(a + (int64_t)(l + j) * ld);
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const double x = xs[l + j];
        t[j] += d[j].x * x;
        q[j] += d[j].y * x;
      }
    }
    for (; l < k1; ++l) {
      const v2d d0 = load2(a + (int64_t)l * ld);
      t[0] += d0.x * xs[l];
      q[0] += d0.y * xs[l];
    }
#pragma unroll
    for (int w = U / 2; w >= 1; w /= 2)
#pragma unroll
      for (int j = 0; j < w; ++j) {
        t[j] += t[j + w];
        q[j] += q[j + w];
      }
    s0 += t[0];
    s1 += q[0];
  }
}

// xs: EXT_CHUNK doubles of LDS, part: 4 x 128 doubles of LDS
__device__ __forceinline__ void extend_block(const ExtJob *jobs, const ExtPart *parts,
                                             const double *w, double *z, int bx, int by,
                                             double *xs, double (*part)[128]) {
  const ExtJob J = jobs[by];
  const int r0 = bx * 128;
  if (r0 >= J.m) return;  // uniform over the workgroup
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m0 = r0 + 2 * lane;
  const bool rows = m0 < J.m;
  double s0 = 0.0, s1 = 0.0;
  auto matvec = [&](const ExtPart &P, const double *u, const double *v) {
    if (P.f32)
      ext_matvec((const float *)P.D, P.ld, u, v, J.m, m0, rows, wv, xs, s0, s1);
    else
      ext_matvec((const double *)P.D, P.ld, u, v, J.m, m0, rows, wv, xs, s0, s1);
  };
  const double *wlast = nullptr;
  if (J.pair) {
    const ExtPart P = parts[J.part0], Q = parts[J.part0 + 1];
    wlast = w + Q.woff;
    matvec(P, w + P.woff, wlast);
  } else {
    for (int q = 0; q < J.nparts; ++q) {
      const ExtPart P = parts[J.part0 + q];
      const double *wq = w + P.woff;
      if (P.D) {
        matvec(P, wq, nullptr);
      } else if (wv == 0 && rows) {
        s0 += wq[m0] * P.scale;
        if (m0 + 1 < J.m) s1 += wq[m0 + 1] * P.scale;
      }
    }
  }
  __syncthreads();
  part[wv][2 * lane] = s0;
  part[wv][2 * lane + 1] = s1;
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 128 && r0 + t < J.m) {
    const int r = r0 + t;
    double v = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
    if (wlast) v += wlast[r];
    z[J.gids[r]] = v;
  }
}

__global__ __launch_bounds__(256) void k_extend(const ExtJob *jobs, const ExtPart *parts,
                                                const double *w, double *z) {
  __shared__ double xs[EXT_CHUNK];
  __shared__ double part[4][128];
  extend_block(jobs, parts, w, z, blockIdx.x, blockIdx.y, xs, part);
}

hipError_t extend(const ExtJob *d_jobs, int njobs, int max_m, const ExtPart *d_parts,
                  const double *w, double *z, hipStream_t s) {
  if (!njobs || !max_m) return hipSuccess;
  hipLaunchKernelGGL(k_extend, dim3((max_m + 127) / 128, njobs), dim3(256), 0, s, d_jobs, d_parts,
                     w, z);
  return hipGetLastError();
}

// ------------------------------------------------------------- CG recurrences
// Partial dot products of (a,b) and optionally (c,d): part[2*blk + {0,1}].
__global__ __launch_bounds__(256) void k_dot2(int64_t n, const double *a, const double *b,
                                              const double *c, const double *d, double *part) {
  __shared__ double red[16];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    s0 += a[i] * b[i];
    if (c) s1 += c[i] * d[i];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}

// Final reduction (fixed order) and scalar bookkeeping of PCG.
//  mode 0: sc[PQ] = s0; alpha = sc[RZ]/pq, history
//  mode 1: sc[RR] = s0
//  mode 2: rz_new = s0; beta = rz_new / sc[RZ]; sc[RZ] = rz_new, history
//  mode 3: sc[RZ] = s0 (first iteration); mode 4: sc[GG] = s0 ; mode 5: sc[TMP] = s0
__global__ void k_dot_final(int nblk, const double *part, double *sc, int mode, int it,
                            double *hist_a, double *hist_b) {
  if (threadIdx.x != 0) return;
  double s0 = 0.0;
  for (int i = 0; i < nblk; ++i) s0 += part[2 * i];
  switch (mode) {
    case 0: {
      sc[SC_PQ] = s0;
      const double a = sc[SC_RZ] / s0;
      sc[SC_ALPHA] = a;
      if (!(s0 > 0.0) || !(a == a)) sc[SC_FLAG] = 1.0;
      if (hist_a) hist_a[it] = a;
      break;
    }
    case 1: sc[SC_RR] = s0; break;
    case 2: {
      const double b = s0 / sc[SC_RZ];
      sc[SC_BETA] = b;
      sc[SC_RZ] = s0;
      if (hist_b) hist_b[it] = b;
      break;
    }
    case 3: sc[SC_RZ] = s0; break;
    case 4: sc[SC_GG] = s0; break;
    default: sc[SC_TMP] = s0; break;
  }
}

hipError_t dot(int64_t n, const double *a, const double *b, double *part, double *sc, int mode,
               int it, double *hist_a, double *hist_b, hipStream_t s) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > DOT_BLOCKS) nblk = DOT_BLOCKS;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(k_dot2, dim3(nblk), dim3(256), 0, s, n, a, b, (const double *)nullptr,
                     (const double *)nullptr, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, s, nblk, part, sc, mode, it, hist_a, hist_b);
  return hipGetLastError();
}

// x += alpha p ; r -= alpha q ; partial r.r
__global__ __launch_bounds__(256) void k_update_xr(int64_t n, const double *sc, double *x, double *r,
                                                   const double *p, const double *q, double *part) {
  __shared__ double red[16];
  const double a = sc[SC_ALPHA];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s;
    part[2 * blockIdx.x + 1] = 0.0;
  }
}

hipError_t update_xr(int64_t n, const double *sc, double *x, double *r, const double *p,
                     const double *q, double *part, double *scw, hipStream_t s) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > DOT_BLOCKS) nblk = DOT_BLOCKS;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(k_update_xr, dim3(nblk), dim3(256), 0, s, n, sc, x, r, p, q, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, s, nblk, part, scw, 1, 0,
                     (double *)nullptr, (double *)nullptr);
  return hipGetLastError();
}

// p = z + beta p (beta = 0 on the first iteration via sc[SC_BETA] reset)
__global__ void k_update_p(int64_t n, const double *sc, double *p, const double *z) {
  const double b = sc[SC_BETA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + b * p[i];
}

hipError_t update_p(int64_t n, const double *sc, double *p, const double *z, hipStream_t s) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > DOT_BLOCKS) nblk = DOT_BLOCKS;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(k_update_p, dim3(nblk), dim3(256), 0, s, n, sc, p, z);
  return hipGetLastError();
}

// y = a - b (elementwise)
__global__ void k_sub(int64_t n, const double *a, const double *b, double *y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

hipError_t vsub(int64_t n, const double *a, const double *b, double *y, hipStream_t s) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > DOT_BLOCKS) nblk = DOT_BLOCKS;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(k_sub, dim3(nblk), dim3(256), 0, s, n, a, b, y);
  return hipGetLastError();
}

// y += a x (elementwise)
__global__ void k_axpy(int64_t n, double a, const double *x, double *y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

hipError_t axpy(int64_t n, double a, const double *x, double *y, hipStream_t s) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > DOT_BLOCKS) nblk = DOT_BLOCKS;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(k_axpy, dim3(nblk), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

// Recovery output: local DoF vector in CSR order.  Velocities from the
// interior solve or the interface solution, pressures c = H [p_I; 0] + p0.
__global__ void k_recover_out(const RecJob *jobs, const double *x_orig, int64_t nG) {
  const RecJob J = jobs[blockIdx.x];
  __shared__ double red[16];
  // v^T [p_I; 0]
  double t = 0.0;
  for (int k = threadIdx.x; k < J.nel - 1; k += blockDim.x) t += J.hv[k] * J.z[J.nv + k];
  t = block_sum(t, red);
  const double tau = J.hv[J.nel];
  const double p0 = x_orig[nG + J.sub];
  for (int i = threadIdx.x; i < J.n; i += blockDim.x) {
    const int k = J.kind[i];
    const int p = J.pos[i];
    double v;
    if (k == 0) {
      v = J.z[p];
      if (J.sep_out) J.sep_out[p] = v;
    } else if (k == 1) {
      v = x_orig[J.gid[i]];
    } else {
      const int q = p - J.nv;
      const double pi = (q < J.nel - 1) ? J.z[p] : 0.0;
      v = pi - tau * J.hv[q] * t + p0;
    }
    const int o = J.oidx ? J.oidx[i] : i;
    if (o >= 0) J.out[o] = v;
  }
  if (J.c_out)
    for (int q = threadIdx.x; q < J.nel; q += blockDim.x) {
      const double pi = (q < J.nel - 1) ? J.z[J.nv + q] : 0.0;
      J.c_out[q] = pi - tau * J.hv[q] * t + p0;
    }
}

hipError_t recover_out(const RecJob *d_jobs, int nsub, const double *x_orig, int64_t nG,
                       hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_recover_out, dim3(nsub), dim3(256), 0, s, d_jobs, x_orig, nG);
  return hipGetLastError();
}


// ------------------------------------------ PCG over several problems
__device__ __forceinline__ int64_t seg_index(const Seg &S, int64_t k) {
  return (k < S.n0) ? S.a0 + k : S.a1 + (k - S.n0);
}

// part[p * G + c] = sum over problem p's entries handled by block c of a.b
__device__ __forceinline__ void sdot_block(const Seg *segs, const double *a, const double *b,
                                           double *part, int bx, int by, int G, double *red) {
  const Seg S = segs[by];
  const int64_t n = S.n0 + S.n1;
  double s = 0.0;
  for (int64_t k = (int64_t)bx * blockDim.x + threadIdx.x; k < n; k += (int64_t)G * blockDim.x) {
    const int64_t i = seg_index(S, k);
    s += a[i] * b[i];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(int64_t)by * G + bx] = s;
}

__global__ __launch_bounds__(256) void k_sdot(const Seg *segs, const double *a, const double *b,
                                              double *part) {
  __shared__ double red[16];
  sdot_block(segs, a, b, part, blockIdx.x, blockIdx.y, gridDim.x, red);
}

// Problem p: fixed-order sum of its G partials, then the scalar bookkeeping
// of the mode.
__device__ __forceinline__ void sfinal_at(int p, int P, int G, const double *part, double *sc,
                                          int mode, double *hist_a, double *hist_b, int hist_ld) {
  if (p >= P) return;
  double s0 = 0.0;
  for (int c = 0; c < G; ++c) s0 += part[(int64_t)p * G + c];
  double *q = sc + (int64_t)p * SC_STRIDE;
  const bool done = q[SC_DONE] != 0.0;
  switch (mode) {
    case 0: {
      q[SC_PQ] = s0;
      q[SC_ACTIVE] = done ? 0.0 : 1.0;
      if (done) {
        q[SC_ALPHA] = 0.0;
        break;
      }
      const double a = q[SC_RZ] / s0;
      if (!(s0 > 0.0) || !(a == a)) {  // breakdown: stop this problem
        q[SC_FLAG] = 1.0;
        q[SC_ALPHA] = 0.0;
        q[SC_ACTIVE] = 0.0;
        q[SC_DONE] = 1.0;
        q[SC_TDONE] = (double)wall_clock64();
        break;
      }
      q[SC_ALPHA] = a;
      if (hist_a) hist_a[(int64_t)p * hist_ld + (int64_t)q[SC_IT]] = a;
      break;
    }
    case 1: {
      if (q[SC_ACTIVE] == 0.0) break;
      q[SC_RR] = s0;
      q[SC_IT] += 1.0;
      if (sqrt(s0) <= q[SC_TOL] * sqrt(q[SC_GG])) {
        q[SC_DONE] = 1.0;
        q[SC_TDONE] = (double)wall_clock64();
      } else if (q[SC_IT] >= q[SC_MAXIT]) {
        q[SC_FLAG] = 2.0;
        q[SC_DONE] = 1.0;
        q[SC_TDONE] = (double)wall_clock64();
      }
      break;
    }
    case 2: {
      if (done) {
        q[SC_BETA] = 0.0;
        break;
      }
      const double b = s0 / q[SC_RZ];
      q[SC_BETA] = b;
      q[SC_RZ] = s0;
      if (hist_b) hist_b[(int64_t)p * hist_ld + (int64_t)q[SC_IT] - 1] = b;
      break;
    }
    case 3: q[SC_RZ] = s0; break;
    case 4: q[SC_GG] = s0; break;
    case 5: q[SC_TMP] = s0; break;
    default: {
      q[SC_RR] = s0;
      if (!isfinite(s0) || !isfinite(q[SC_GG])) {  // NaN/Inf data: a breakdown, not convergence
        q[SC_FLAG] = 1.0;
        q[SC_DONE] = 1.0;
        q[SC_TDONE] = (double)wall_clock64();
        break;
      }
      if (!(sqrt(s0) > q[SC_TOL] * sqrt(q[SC_GG]))) {
        q[SC_DONE] = 1.0;
        q[SC_TDONE] = (double)wall_clock64();
      }
      break;
    }
  }
}

__global__ void k_sfinal(int P, int G, const double *part, double *sc, int mode, double *hist_a,
                         double *hist_b, int hist_ld) {
  sfinal_at(blockIdx.x * blockDim.x + threadIdx.x, P, G, part, sc, mode, hist_a, hist_b, hist_ld);
}

hipError_t sdot(const Seg *segs, int P, int G, const double *a, const double *b, double *part,
                double *sc, int mode, double *hist_a, double *hist_b, int hist_ld, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sdot, dim3(G, P), dim3(256), 0, s, segs, a, b, part);
  hipLaunchKernelGGL(k_sfinal, dim3((P + 63) / 64), dim3(64), 0, s, P, G, part, sc, mode, hist_a,
                     hist_b, hist_ld);
  return hipGetLastError();
}

// x += alpha_p p ; r -= alpha_p q ; partial r.r per (problem, block)
__device__ __forceinline__ void supdate_xr_block(const Seg *segs, const double *sc, double *x,
                                                 double *r, const double *p, const double *q,
                                                 double *part, int bx, int by, int G, double *red) {
  const Seg S = segs[by];
  const double a = sc[(int64_t)by * SC_STRIDE + SC_ALPHA];
  const int64_t n = S.n0 + S.n1;
  double s = 0.0;
  for (int64_t k = (int64_t)bx * blockDim.x + threadIdx.x; k < n; k += (int64_t)G * blockDim.x) {
    const int64_t i = seg_index(S, k);
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(int64_t)by * G + bx] = s;
}

__global__ __launch_bounds__(256) void k_supdate_xr(const Seg *segs, const double *sc, double *x,
                                                    double *r, const double *p, const double *q,
                                                    double *part) {
  __shared__ double red[16];
  supdate_xr_block(segs, sc, x, r, p, q, part, blockIdx.x, blockIdx.y, gridDim.x, red);
}

hipError_t supdate_xr(const Seg *segs, int P, int G, double *sc, double *x, double *r,
                      const double *p, const double *q, double *part, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_supdate_xr, dim3(G, P), dim3(256), 0, s, segs, sc, x, r, p, q, part);
  hipLaunchKernelGGL(k_sfinal, dim3((P + 63) / 64), dim3(64), 0, s, P, G, part, sc, 1,
                     (double *)nullptr, (double *)nullptr, 0);
  return hipGetLastError();
}

__device__ __forceinline__ void supdate_p_block(const Seg *segs, const double *sc, double *p,
                                                const double *z, int bx, int by, int G) {
  const Seg S = segs[by];
  const double b = sc[(int64_t)by * SC_STRIDE + SC_BETA];
  const int64_t n = S.n0 + S.n1;
  for (int64_t k = (int64_t)bx * blockDim.x + threadIdx.x; k < n; k += (int64_t)G * blockDim.x) {
    const int64_t i = seg_index(S, k);
    p[i] = z[i] + b * p[i];
  }
}

__global__ void k_supdate_p(const Seg *segs, const double *sc, double *p, const double *z) {
  supdate_p_block(segs, sc, p, z, blockIdx.x, blockIdx.y, gridDim.x);
}

hipError_t supdate_p(const Seg *segs, int P, int G, const double *sc, double *p, const double *z,
                     hipStream_t s) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_supdate_p, dim3(G, P), dim3(256), 0, s, segs, sc, p, z);
  return hipGetLastError();
}

__global__ void k_sinit(int P, const double *tol, int maxit, double *sc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double *q = sc + (int64_t)p * SC_STRIDE;
  for (int k = 0; k < SC_STRIDE; ++k) q[k] = 0.0;
  q[SC_TOL] = tol[p];
  q[SC_MAXIT] = (double)maxit;
  q[SC_T0] = (double)wall_clock64();
}

hipError_t sinit(int P, const double *tol, int maxit, double *sc, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sinit, dim3((P + 63) / 64), dim3(64), 0, s, P, tol, maxit, sc);
  return hipGetLastError();
}
// ------------------------------------------------ symmetric matrix-vector
// Tile (ti, tj), tj <= ti, of job `by` (tile index t = ti (ti + 1) / 2 + tj):
// lane l of every wave holds rows R0 + l + 64 k (k < 4) of the tile, so each
// column read is four coalesced 64-entry loads (no alignment needed); the
// four waves split the tile's columns and take them SYMV_U at a time, so
// that 4 SYMV_U loads per lane are in flight.  Row sums use x of the columns
// (staged in LDS), column sums x of the rows (in registers): the SYMV_U
// column sums of a step are reduced across the wave together by a butterfly
// (each exchange halves the values a lane carries), after which lanes
// 8u .. 8u + 7 hold column u's sum.  On a diagonal tile the row sums take
// the entries on and below the diagonal, the column sums those strictly
// below, so that every entry of the full matrix is used once.
constexpr int SYMV_U = 8;

template <typename T>
__device__ __forceinline__ void symv_tile(const SymvJob &J, int t, double *xs, double (*red)[SYMV_T]) {
  int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int R0 = ti * SYMV_T, C0 = tj * SYMV_T;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  for (int c = threadIdx.x; c < SYMV_T; c += blockDim.x) {
    const int j = C0 + c;
    xs[c] = j < J.n ? (J.xidx ? J.x[J.xidx[j]] : J.x[j]) : 0.0;
  }
  double xr[4], racc[4];
  bool rin[4];
  int rr[4];  // the rows read: rows at or beyond n read row n - 1 and are weighted 0
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = R0 + lane + 64 * k;
    rin[k] = r < J.n;
    rr[k] = min(r, J.n - 1);
    xr[k] = rin[k] ? (J.xidx ? J.x[J.xidx[r]] : J.x[r]) : 0.0;
    racc[k] = 0.0;
  }
  __syncthreads();
  const bool diag = ti == tj;
  const T *A = (const T *)J.A;
  double *P = J.part + (int64_t)t * 2 * SYMV_T;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  const int c0 = 64 * w, c1 = min(c0 + 64, J.n - C0);
  for (int c = c0; c < c1; c += SYMV_U) {  // c + SYMV_U - 1 <= c0 + 63
    // every load in bounds and unconditional (columns past c1 read column
    // c1 - 1), so that all 4 SYMV_U of them are issued before the first use
    double v[SYMV_U][4];
#pragma unroll
    for (int u = 0; u < SYMV_U; ++u) {
      const bool cin = c + u < c1;
      const auto col = gptr(A + (int64_t)(C0 + min(c + u, c1 - 1)) * J.lda);
#pragma unroll
      for (int k = 0; k < 4; ++k)  // weighted, not selected: the load stays unconditional
        v[u][k] = (double)col[rr[k]] * ((cin && rin[k]) ? 1.0 : 0.0);
    }
    double cp[SYMV_U];
#pragma unroll
    for (int u = 0; u < SYMV_U; ++u) {
      const int j = C0 + c + u;
      const double xj = xs[c + u];
      double sc = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = R0 + lane + 64 * k;
        const double vr = (!diag || r >= j) ? v[u][k] : 0.0;
        const double vc = (!diag || r > j) ? v[u][k] : 0.0;
        racc[k] += vr * xj;
        sc += vc * xr[k];
      }
      cp[u] = sc;
    }
    // butterfly over lane bits 5, 4, 3: the lane keeps the half of its
    // values selected by its bit and adds the partner's copy of that half
    double a4[4], a2[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double keep = b5 ? cp[i + 4] : cp[i], send = b5 ? cp[i] : cp[i + 4];
      a4[i] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double keep = b4 ? a4[i + 2] : a4[i], send = b4 ? a4[i] : a4[i + 2];
      a2[i] = keep + __shfl_xor(send, 16);
    }
    double a1 = (b3 ? a2[1] : a2[0]) + __shfl_xor(b3 ? a2[0] : a2[1], 8);
    a1 += __shfl_xor(a1, 4);
    a1 += __shfl_xor(a1, 2);
    a1 += __shfl_xor(a1, 1);
    const int u = lane >> 3;  // the column this lane now holds
    if ((lane & 7) == 0 && c + u < c1) P[SYMV_T + c + u] = a1;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[w][lane + 64 * k] = racc[k];
  __syncthreads();
  for (int r = threadIdx.x; r < SYMV_T; r += blockDim.x)
    P[r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
}

// y[i] = alpha (sum of the row sums of the tiles in i's tile row + the
// column sums of the tiles on and below the diagonal in i's tile column)
// (+ y[i]).
__device__ __forceinline__ void symv_reduce_at(const SymvJob &J, int i) {
  if (i >= J.n) return;
  const int ti = i / SYMV_T, il = i % SYMV_T, T = (J.n + SYMV_T - 1) / SYMV_T;
  double s = 0.0;
  for (int tj = 0; tj <= ti; ++tj) s += J.part[(int64_t)(ti * (ti + 1) / 2 + tj) * 2 * SYMV_T + il];
  for (int t2 = ti; t2 < T; ++t2)
    s += J.part[(int64_t)(t2 * (t2 + 1) / 2 + ti) * 2 * SYMV_T + SYMV_T + il];
  double v = J.alpha * s;
  if (J.acc) v += J.y[i];
  J.y[i] = v;
}

__global__ __launch_bounds__(256) void k_symv_tiles(const SymvJob *jobs) {
  const SymvJob J = jobs[blockIdx.y];
  if ((int)blockIdx.x >= symv_tiles(J.n)) return;
  __shared__ double xs[SYMV_T];
  __shared__ double red[4][SYMV_T];
  if (J.a_f32)
    symv_tile<float>(J, blockIdx.x, xs, red);
  else
    symv_tile<double>(J, blockIdx.x, xs, red);
}

__global__ __launch_bounds__(256) void k_symv_reduce(const SymvJob *jobs) {
  const SymvJob J = jobs[blockIdx.y];
  symv_reduce_at(J, blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t symv(const SymvJob *d_jobs, int batch, int max_n, hipStream_t s) {
  if (!batch || !max_n) return hipSuccess;
  hipLaunchKernelGGL(k_symv_tiles, dim3(symv_tiles(max_n), batch), dim3(256), 0, s, d_jobs);
  hipLaunchKernelGGL(k_symv_reduce, dim3((max_n + 255) / 256, batch), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// ------------------------------------------- persistent PCG iteration loop
// Grid-wide barrier of a cooperative launch (every block co-resident): one
// arrival counter and a generation word; thread 0 of each block arrives
// (release), the last arrival resets the counter and advances the
// generation, the others wait for it (acquire).  A wait longer than about
// 20 s of the constant device clock (100 MHz) returns false, so every
// block leaves instead of hanging.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned nblocks) {
  constexpr unsigned long long limit = 2000000000ull;
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned g = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned a = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > limit) {
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return ok != 0;
}

template <int CPB>
__device__ __forceinline__ void gemv_phase_t(const GemvPhase &ph, double *xs) {
  const int nv = ph.gx * ph.batch;
  for (int v = blockIdx.x; v < nv; v += gridDim.x) gemv_t_block<CPB>(ph.jobs, v % ph.gx, v / ph.gx, xs);
}

__device__ __forceinline__ void gemv_phase(const GemvPhase &ph, double *xs) {
  switch (ph.cpb) {
    case 8: gemv_phase_t<8>(ph, xs); break;
    case 16: gemv_phase_t<16>(ph, xs); break;
    case 64: gemv_phase_t<64>(ph, xs); break;
    default: gemv_phase_t<32>(ph, xs); break;
  }
}

// The PCG iterations of every problem until all have stopped (converged,
// broken down or at maxit; the per-problem scalars decide, as in the
// launch-by-launch iteration), each phase of an iteration spread over the
// resident blocks and followed by a grid barrier.  The arithmetic and its
// order are those of the launch-by-launch iteration.
__global__ __launch_bounds__(256) void k_pcg_persistent(const PcgPlan *plan) {
  const PcgPlan L = *plan;
  __shared__ double xs[GT_CHUNK];
  __shared__ double part4[4][SYMV_T];  // extend's 4 x 128 partial sums, or symv's 4 x 256
  __shared__ double red[16];
  const unsigned nb = gridDim.x;
  const int tid = threadIdx.x, bsz = blockDim.x;
  const int nv_dot = L.G * L.P;
  auto sync = [&]() -> bool {
    if (grid_barrier(L.bar, nb)) return true;
    if (tid == 0) atomicExch(L.err, 1);
    return false;
  };
  for (int it = 0; it < L.max_iter; ++it) {
    bool all = true;
    for (int pp = 0; pp < L.P; ++pp)
      all = all && ((volatile const double *)L.sc)[(int64_t)pp * SC_STRIDE + SC_DONE] != 0.0;
    if (all) break;
    // q = S~ p
    if (L.ssym) {
      const int nv = L.ssym_tiles * L.ssym_batch;
      for (int v = blockIdx.x; v < nv; v += nb) {
        const SymvJob J = L.ssym[v / L.ssym_tiles];
        const int t = v % L.ssym_tiles;
        if (t >= symv_tiles(J.n)) continue;
        if (J.a_f32)
          symv_tile<float>(J, t, xs, (double(*)[SYMV_T])&part4[0][0]);
        else
          symv_tile<double>(J, t, xs, (double(*)[SYMV_T])&part4[0][0]);
      }
      if (!sync()) return;
      const int nr = L.ssym_rows * L.ssym_batch;
      for (int v = blockIdx.x * bsz + tid; v < nr; v += nb * bsz)
        symv_reduce_at(L.ssym[v / L.ssym_rows], v % L.ssym_rows);
    } else {
      gemv_phase(L.schur, xs);
    }
    if (!sync()) return;
    for (int64_t g = (int64_t)blockIdx.x * bsz + tid; g < L.n_own; g += (int64_t)nb * bsz)
      owner_sum_at(g, L.n_own, L.own_ptr, L.own_idx, L.yloc, nullptr, nullptr, L.q);
    if (!sync()) return;
    // alpha = rz / p.q ; x += alpha p ; r -= alpha q ; convergence
    for (int v = blockIdx.x; v < nv_dot; v += nb)
      sdot_block(L.segs, L.p, L.q, L.part, v % L.G, v / L.G, L.G, red);
    if (!sync()) return;
    for (int pp = blockIdx.x * bsz + tid; pp < L.P; pp += nb * bsz)
      sfinal_at(pp, L.P, L.G, L.part, L.sc, 0, L.hist_a, nullptr, L.hist_ld);
    if (!sync()) return;
    for (int v = blockIdx.x; v < nv_dot; v += nb)
      supdate_xr_block(L.segs, L.sc, L.x, L.r, L.p, L.q, L.part, v % L.G, v / L.G, L.G, red);
    if (!sync()) return;
    for (int pp = blockIdx.x * bsz + tid; pp < L.P; pp += nb * bsz)
      sfinal_at(pp, L.P, L.G, L.part, L.sc, 1, nullptr, nullptr, 0);
    if (!sync()) return;
    // z = M~^-1 r
    if (L.restrict_.batch) {
      gemv_phase(L.restrict_, xs);
      if (!sync()) return;
    }
    if (L.nsym) {  // [S_DD^-1 | Phi]^T g: the symmetric block's tiles and the Phi block
      const int nv = L.nsym_tiles * L.nsym_batch;
      for (int v = blockIdx.x; v < nv; v += nb) {
        const SymvJob J = L.nsym[v / L.nsym_tiles];
        const int t = v % L.nsym_tiles;
        if (t >= symv_tiles(J.n)) continue;
        if (J.a_f32)
          symv_tile<float>(J, t, xs, (double(*)[SYMV_T])&part4[0][0]);
        else
          symv_tile<double>(J, t, xs, (double(*)[SYMV_T])&part4[0][0]);
      }
      gemv_phase(L.nphi, xs);
      if (!sync()) return;
      const int nr = L.nsym_rows * L.nsym_batch;
      for (int v = blockIdx.x * bsz + tid; v < nr; v += nb * bsz)
        symv_reduce_at(L.nsym[v / L.nsym_rows], v % L.nsym_rows);
    } else {
      gemv_phase(L.neu1, xs);
    }
    if (!sync()) return;
    for (int64_t g = (int64_t)blockIdx.x * bsz + tid; g < L.n_cs; g += (int64_t)nb * bsz)
      owner_sum_at(g, L.n_cs, L.c_ptr, L.c_idx, L.tv, L.c_base, L.r, L.rc);
    if (!sync()) return;
    gemv_phase(L.coarse, xs);
    if (!sync()) return;
    if (L.neu2.batch) {
      const int nv = L.neu2.gx * L.neu2.batch;
      for (int v = blockIdx.x; v < nv; v += nb) gemv_n_block(L.neu2.jobs, v % L.neu2.gx, v / L.neu2.gx, xs);
      if (!sync()) return;
    }
    if (L.n_ext) {
      const int nv = L.ext_gx * L.n_ext;
      for (int v = blockIdx.x; v < nv; v += nb)
        extend_block(L.ext, L.extpart, L.wv, L.z, v % L.ext_gx, v / L.ext_gx, xs,
                     (double(*)[128])&part4[0][0]);
    }
    for (int64_t i = (int64_t)blockIdx.x * bsz + tid; i < L.n_cs; i += (int64_t)nb * bsz)
      L.z[L.uc_dst[i]] = L.uc[i];
    if (!sync()) return;
    // beta = r.z / rz ; p = z + beta p
    for (int v = blockIdx.x; v < nv_dot; v += nb)
      sdot_block(L.segs, L.r, L.z, L.part, v % L.G, v / L.G, L.G, red);
    if (!sync()) return;
    for (int pp = blockIdx.x * bsz + tid; pp < L.P; pp += nb * bsz)
      sfinal_at(pp, L.P, L.G, L.part, L.sc, 2, nullptr, L.hist_b, L.hist_ld);
    if (!sync()) return;
    for (int v = blockIdx.x; v < nv_dot; v += nb)
      supdate_p_block(L.segs, L.sc, L.p, L.z, v % L.G, v / L.G, L.G);
    if (!sync()) return;
  }
}

int pcg_persistent_blocks(int per_cu) {
  int dev = 0, coop = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_pcg_persistent, 256, 0) != hipSuccess)
    return 0;
  return std::max(0, std::min(occ, per_cu)) * cus;
}

hipError_t pcg_persistent(const PcgPlan *d_plan, int nblocks, hipStream_t s) {
  void *args[] = {(void *)&d_plan};
  return hipLaunchCooperativeKernel((const void *)k_pcg_persistent, dim3(nblocks), dim3(256), args, 0,
                                    s);
}

}  // namespace vb
