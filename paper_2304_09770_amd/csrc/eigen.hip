// Dense symmetric eigen-solver pieces for the adaptive face eigenproblems
// (Sec. 6): after the pencil has been reduced to a standard symmetric matrix
// C = L^-1 At L^-T, one workgroup per face
//   * reduces C to tridiagonal form T = Q^T C Q with Householder reflectors,
//   * counts the eigenvalues of T below sigma = 1/theta by Sturm sequences and
//     finds each of them by bisection,
//   * computes their eigenvectors by inverse iteration on T (tridiagonal LU
//     with partial pivoting, re-orthogonalised), and
//   * applies Q to them.
// Also: the rows L y of the new constraints, the per-entity reflectors of the
// change of basis applied to row segments of a matrix, column normalisation.
#include "common.h"
#include "kernels.h"

namespace vb {

// ------------------------------------------------------- tridiagonalisation
// Full symmetric storage (both triangles), column-major.  Step k:
// v = x - alpha e_0 for x = A[k+1:, k], alpha = -sign(x_0) |x|,
// tau = 2 / v^T v; p = tau A22 v; w = p - (tau/2)(p^T v) v;
// A22 -= v w^T + w v^T.  v is kept in A[k+1:, k] for the back-transform.
__global__ __launch_bounds__(1024) void k_tridiag(const EigJob *jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  extern __shared__ double sh[];
  double *v = sh, *p = sh + n;
  __shared__ double red[16];
  const int tid = threadIdx.x, bs = blockDim.x;
  double *A = J.A;
  const int64_t ld = J.ld;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    const int64_t c0 = (int64_t)(k + 1) * ld + (k + 1);  // A22 origin
    double s = 0.0;
    for (int i = tid; i < m; i += bs) {
      const double x = A[(int64_t)(k + 1 + i) + (int64_t)k * ld];
      v[i] = x;
      s += x * x;
    }
    s = block_sum(s, red);
    const double x0 = v[0];
    const double nrm = sqrt(s);
    const double alpha = (nrm == 0.0) ? 0.0 : ((x0 >= 0.0) ? -nrm : nrm);
    const double vtv = s - 2.0 * alpha * x0 + alpha * alpha;
    const double tau = (nrm == 0.0 || !(vtv > 0.0)) ? 0.0 : 2.0 / vtv;
    __syncthreads();
    if (tid == 0) {
      v[0] = x0 - alpha;
      J.d[k] = A[(int64_t)k + (int64_t)k * ld];
      J.e[k] = alpha;
      J.tau[k] = tau;
    }
    __syncthreads();
    for (int i = tid; i < m; i += bs) A[(int64_t)(k + 1 + i) + (int64_t)k * ld] = v[i];
    if (tau == 0.0) {
      __syncthreads();
      continue;
    }
    // p = tau A22 v (row i of A22 read along its columns: coalesced per j)
    for (int i = tid; i < m; i += bs) {
      const double *a = A + c0 + i;
      double acc0 = 0.0, acc1 = 0.0;
      int j = 0;
      for (; j + 1 < m; j += 2) {
        acc0 += a[(int64_t)j * ld] * v[j];
        acc1 += a[(int64_t)(j + 1) * ld] * v[j + 1];
      }
      if (j < m) acc0 += a[(int64_t)j * ld] * v[j];
      p[i] = tau * (acc0 + acc1);
    }
    __syncthreads();
    double t = 0.0;
    for (int i = tid; i < m; i += bs) t += p[i] * v[i];
    t = block_sum(t, red);
    const double K = 0.5 * tau * t;
    for (int i = tid; i < m; i += bs) p[i] -= K * v[i];
    __syncthreads();
    for (int i = tid; i < m; i += bs) {
      double *a = A + c0 + i;
      const double vi = v[i], wi = p[i];
      for (int j = 0; j < m; ++j) a[(int64_t)j * ld] -= vi * p[j] + wi * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      J.d[n - 2] = A[(int64_t)(n - 2) + (int64_t)(n - 2) * ld];
      J.e[n - 2] = A[(int64_t)(n - 1) + (int64_t)(n - 2) * ld];
      J.tau[n - 2] = 0.0;
    }
    J.d[n - 1] = A[(int64_t)(n - 1) + (int64_t)(n - 1) * ld];
    J.e[n - 1] = 0.0;
    J.tau[n - 1] = 0.0;
  }
}

hipError_t tridiag(const EigJob *d_jobs, int njobs, int max_n, hipStream_t s) {
  if (!njobs) return hipSuccess;
  const size_t lds = 2 * (size_t)max_n * sizeof(double);
  if (lds > 159 * 1024) return hipErrorInvalidValue;  // the static LDS comes on top
  if (lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)k_tridiag,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tridiag, dim3(njobs), dim3(1024), lds, s, d_jobs);
  return hipGetLastError();
}

// ------------------------------------------------ eigenpairs of T below sigma
// Number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence of
// the LDL^T pivots of T - x I; tiny pivots replaced by -pivmin).
__device__ int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// LDS layout per job: d, e, e2, and the LU factors of T - lambda I
// (diagonal u0, first and second superdiagonals u1, u2, multipliers l,
// row-swap flags), plus one work vector.
__global__ __launch_bounds__(256) void k_tridiag_eig(const EigJob *jobs, int mcap) {
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  extern __shared__ double sh[];
  double *d = sh, *e = d + n, *e2 = e + n, *u0 = e2 + n, *u1 = u0 + n, *u2 = u1 + n,
         *lm = u2 + n, *x = lm + n;
  unsigned char *sw = reinterpret_cast<unsigned char *>(x + n);
  __shared__ double red[16];
  __shared__ double s_lo, s_norm, s_piv;
  __shared__ int s_cnt;
  const int tid = threadIdx.x, bs = blockDim.x;
  for (int i = tid; i < n; i += bs) {
    d[i] = J.d[i];
    e[i] = (i + 1 < n) ? J.e[i] : 0.0;
    e2[i] = e[i] * e[i];
  }
  __syncthreads();
  if (tid == 0) {
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      emax = fmax(emax, e2[i]);
    }
    const double nrm = fmax(fabs(lo), fabs(hi));
    s_norm = nrm;
    s_lo = lo - 2.2e-16 * nrm * 4.0 - 1e-300;
    s_piv = fmax(1e-300, 2.3e-308 * fmax(1.0, emax));
    s_cnt = sturm_count(d, e2, n, J.sigma, s_piv);
    *J.count = s_cnt;
  }
  __syncthreads();
  const int m = min(s_cnt, mcap);
  const double tnorm = s_norm, pivmin = s_piv;
  // bisection, one thread per eigenvalue index
  for (int t = tid; t < m; t += bs) {
    double lo = s_lo, hi = J.sigma;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.2e-16 * 2.0 * fmax(fabs(lo), fabs(hi)) + 1e-300 || mid == lo || mid == hi)
        break;
      if (sturm_count(d, e2, n, mid, pivmin) > t)
        hi = mid;
      else
        lo = mid;
    }
    J.lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // inverse iteration, eigenvalue by eigenvalue (clusters re-orthogonalised)
  const double eps_piv = 2.2e-16 * fmax(tnorm, 1e-300);
  for (int t = 0; t < m; ++t) {
    const double lam = J.lam[t];
    if (tid == 0) {  // LU with partial pivoting of T - lam I
      for (int i = 0; i < n; ++i) {
        u0[i] = d[i] - lam;
        u1[i] = e[i];
        u2[i] = 0.0;
      }
      for (int i = 0; i + 1 < n; ++i) {
        const double sub = e[i];  // T[i+1][i]
        if (fabs(u0[i]) >= fabs(sub)) {
          sw[i] = 0;
          if (u0[i] == 0.0) u0[i] = eps_piv;
          const double f = sub / u0[i];
          lm[i] = f;
          u0[i + 1] -= f * u1[i];
        } else {
          sw[i] = 1;
          const double f = u0[i] / sub;
          lm[i] = f;
          u0[i] = sub;
          const double tmp = u1[i];
          u1[i] = u0[i + 1];
          u0[i + 1] = tmp - f * u0[i + 1];
          if (i + 2 < n) {
            u2[i] = u1[i + 1];
            u1[i + 1] = -f * u1[i + 1];
          }
        }
      }
      if (u0[n - 1] == 0.0) u0[n - 1] = eps_piv;
    }
    // deterministic start vector
    for (int i = tid; i < n; i += bs) {
      unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((t + 1) * 40503u);
      h ^= h >> 13;
      h *= 0x5bd1e995u;
      h ^= h >> 15;
      x[i] = 0.5 + (double)(h & 0xffff) / 65536.0;
    }
    __syncthreads();
    double *z = J.Z + (int64_t)t * J.ldz;
    for (int it = 0; it < 3; ++it) {
      if (tid == 0) {  // solve (T - lam I) y = x in place
        for (int i = 0; i + 1 < n; ++i) {
          if (sw[i] == 0) {
            x[i + 1] -= lm[i] * x[i];
          } else {
            const double tmp = x[i];
            x[i] = x[i + 1];
            x[i + 1] = tmp - lm[i] * x[i];
          }
        }
        x[n - 1] /= u0[n - 1];
        if (n > 1) x[n - 2] = (x[n - 2] - u1[n - 2] * x[n - 1]) / u0[n - 2];
        for (int i = n - 3; i >= 0; --i)
          x[i] = (x[i] - u1[i] * x[i + 1] - u2[i] * x[i + 2]) / u0[i];
      }
      __syncthreads();
      // scale, then orthogonalise twice against the previous eigenvectors
      double ss = 0.0;
      for (int i = tid; i < n; i += bs) ss += x[i] * x[i];
      ss = block_sum(ss, red);
      const double sc = (ss > 0.0) ? 1.0 / sqrt(ss) : 0.0;
      for (int i = tid; i < n; i += bs) x[i] *= sc;
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < t; ++q) {
          const double *zq = J.Z + (int64_t)q * J.ldz;
          double dt = 0.0;
          for (int i = tid; i < n; i += bs) dt += zq[i] * x[i];
          dt = block_sum(dt, red);
          for (int i = tid; i < n; i += bs) x[i] -= dt * zq[i];
          __syncthreads();
        }
      ss = 0.0;
      for (int i = tid; i < n; i += bs) ss += x[i] * x[i];
      ss = block_sum(ss, red);
      const double s2 = (ss > 0.0) ? 1.0 / sqrt(ss) : 0.0;
      for (int i = tid; i < n; i += bs) x[i] *= s2;
      __syncthreads();
    }
    for (int i = tid; i < n; i += bs) z[i] = x[i];
    __syncthreads();
  }
}

hipError_t tridiag_eig(const EigJob *d_jobs, int njobs, int max_n, int mcap, hipStream_t s) {
  if (!njobs) return hipSuccess;
  const size_t lds = 8 * (size_t)max_n * sizeof(double) + (size_t)max_n + 16;
  if (lds > 159 * 1024) return hipErrorInvalidValue;  // the static LDS comes on top
  if (lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)k_tridiag_eig,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tridiag_eig, dim3(njobs), dim3(256), lds, s, d_jobs, mcap);
  return hipGetLastError();
}

// Z <- Q Z with Q = H_0 H_1 ... H_{n-3} (reflectors kept below the
// subdiagonal of A): apply H_k for k descending to the first `ncols` columns.
__global__ __launch_bounds__(256) void k_back_transform(const EigJob *jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n, nc = J.ncols;
  if (nc <= 0) return;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int k = n - 3; k >= 0; --k) {
    const double tau = J.tau[k];
    if (tau == 0.0) continue;  // uniform across the block
    const double *v = J.A + (int64_t)(k + 1) + (int64_t)k * J.ld;
    const int m = n - k - 1;
    for (int c = w; c < nc; c += 4) {
      double *z = J.Z + (int64_t)c * J.ldz + (k + 1);
      double s = 0.0;
      for (int i = l; i < m; i += 64) s += v[i] * z[i];
      s = warp_sum(s) * tau;
      for (int i = l; i < m; i += 64) z[i] -= s * v[i];
    }
    __syncthreads();
  }
}

hipError_t back_transform(const EigJob *d_jobs, int njobs, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_back_transform, dim3(njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// R[:, c] = L Z[:, c] with L lower triangular (column-major), c < ncols.
__global__ __launch_bounds__(256) void k_lower_times(const RowJob *jobs) {
  const RowJob J = jobs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= J.ncols) return;
  extern __shared__ double zs[];
  const double *z = J.Z + (int64_t)c * J.ldz;
  for (int i = threadIdx.x; i < J.n; i += blockDim.x) zs[i] = z[i];
  __syncthreads();
  double *r = J.R + (int64_t)c * J.ldr;
  for (int i = threadIdx.x; i < J.n; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j <= i; ++j) s += J.L[(int64_t)i + (int64_t)j * J.ld] * zs[j];
    r[i] = s;
  }
}

hipError_t lower_times(const RowJob *d_jobs, int njobs, int max_n, int max_cols, hipStream_t s) {
  if (!njobs || !max_cols) return hipSuccess;
  const size_t lds = (size_t)max_n * sizeof(double);
  if (lds > 159 * 1024) return hipErrorInvalidValue;  // the static LDS comes on top
  if (lds > 60 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)k_lower_times,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_lower_times, dim3(max_cols, njobs), dim3(256), lds, s, d_jobs);
  return hipGetLastError();
}

// Rows [off, off + n_E) of every column of A <- T_E^T (dir +1) or T_E (dir -1)
// applied to them, with the entity's Householder reflectors.  One wave per
// column.
__global__ __launch_bounds__(256) void k_face_transform(const FaceTJob *jobs) {
  const FaceTJob J = jobs[blockIdx.y];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + w;
  if (j >= J.ncols) return;
  const EntDev E = *J.ent;
  const int rk = *E.rank;
  double *x = J.A + (int64_t)j * J.ld + J.off;
  for (int kk = 0; kk < rk; ++kk) {
    const int k = (J.dir > 0) ? kk : rk - 1 - kk;
    const double *v = E.V + (int64_t)k * E.n;
    double s = 0.0;
    for (int c = k + l; c < E.n; c += 64) s += v[c] * x[c];
    s = warp_sum(s) * E.tau[k];
    for (int c = k + l; c < E.n; c += 64) x[c] -= s * v[c];
  }
}

hipError_t face_transform(const FaceTJob *d_jobs, int njobs, int max_cols, hipStream_t s) {
  if (!njobs || !max_cols) return hipSuccess;
  hipLaunchKernelGGL(k_face_transform, dim3((max_cols + 3) / 4, njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// A <- (A + A^T) / 2 for square blocks (one thread per lower entry).
__global__ void k_sym_average(const SymJob *jobs) {
  const SymJob J = jobs[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)J.n * J.n;
  if (idx >= nn) return;
  const int r = (int)(idx % J.n), c = (int)(idx / J.n);
  if (r <= c) return;
  double *a = J.A + r + (int64_t)c * J.ld, *b = J.A + c + (int64_t)r * J.ld;
  const double m = 0.5 * (*a + *b);
  *a = m;
  *b = m;
}

hipError_t sym_average(const SymJob *d_jobs, int njobs, int max_n, hipStream_t s) {
  if (!njobs || !max_n) return hipSuccess;
  const int64_t nn = (int64_t)max_n * max_n;
  hipLaunchKernelGGL(k_sym_average, dim3((unsigned)((nn + 255) / 256), njobs), dim3(256), 0, s,
                     d_jobs);
  return hipGetLastError();
}

// A += rel * max|diag(A)| * I on square blocks (one block per job).
__global__ void k_shift_diag(const SymJob *jobs, double rel) {
  const SymJob J = jobs[blockIdx.x];
  __shared__ double red[16];
  double m = 0.0;
  for (int i = threadIdx.x; i < J.n; i += blockDim.x)
    m = fmax(m, fabs(J.A[(int64_t)i + (int64_t)i * J.ld]));
  // block max through the sum helper's layout: reduce by waves then lanes
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double mx = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) mx = fmax(mx, red[q]);
  const double sh = rel * mx;
  for (int i = threadIdx.x; i < J.n; i += blockDim.x) J.A[(int64_t)i + (int64_t)i * J.ld] += sh;
}

hipError_t shift_diag(const SymJob *d_jobs, int njobs, double rel, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_shift_diag, dim3(njobs), dim3(256), 0, s, d_jobs, rel);
  return hipGetLastError();
}

// Columns of R (n rows, ld) scaled to unit 2-norm (one wave per column).
__global__ void k_normalize_cols(const RowJob *jobs) {
  const RowJob J = jobs[blockIdx.y];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + w;
  if (c >= J.ncols) return;
  double *r = J.R + (int64_t)c * J.ldr;
  double s = 0.0;
  for (int i = l; i < J.n; i += 64) s += r[i] * r[i];
  s = warp_sum(s);
  const double sc = (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
  for (int i = l; i < J.n; i += 64) r[i] *= sc;
}

hipError_t normalize_cols(const RowJob *d_jobs, int njobs, int max_cols, hipStream_t s) {
  if (!njobs || !max_cols) return hipSuccess;
  hipLaunchKernelGGL(k_normalize_cols, dim3((max_cols + 3) / 4, njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

}  // namespace vb
