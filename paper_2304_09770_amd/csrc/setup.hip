// Setup kernels: local dense matrices, the Q_I / Q_0 pressure split, the
// primal change of basis, block gathers, interior recovery and the
// refinement steps of the mixed-precision path.  The dense local matrices
// are stored in T = double (FP64 path) or float (mixed path).
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace vb {

template <typename T> __device__ __forceinline__ T *Wp(const SubDev &S) { return (T *)S.W; }

// Scatter the local CSR (both triangles) and the right-hand side into the
// dense bordered matrix [[K, r], [r^T, 0]] with the DoF order
// [interior velocity | element pressures | interface | rhs].  One wave per
// CSR row, the lanes over its nonzeros (all of a row's stores in flight).
template <typename T>
__global__ __launch_bounds__(256) void k_densify(const SubDev *subs) {
  const SubDev S = subs[blockIdx.y];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (row >= S.n_csr) return;
  T *W = Wp<T>(S);
  const int pr = S.pos[row];
  for (int64_t q = S.indptr[row] + l; q < S.indptr[row + 1]; q += 64) {
    const int pc = S.pos[S.indices[q]];
    W[(int64_t)pr + (int64_t)pc * S.ld] = (T)S.vals[q];
  }
  if (l == 0) {
    const int last = S.N - 1;
    W[(int64_t)pr + (int64_t)last * S.ld] = (T)S.rhs[row];
    W[(int64_t)last + (int64_t)pr * S.ld] = (T)S.rhs[row];
  }
}

hipError_t densify(const SubDev *d_subs, int nsub, int max_rows, bool fp32, hipStream_t s) {
  if (!nsub) return hipSuccess;
  dim3 g((max_rows + 3) / 4, nsub);
  if (fp32)
    hipLaunchKernelGGL(k_densify<float>, g, dim3(256), 0, s, d_subs);
  else
    hipLaunchKernelGGL(k_densify<double>, g, dim3(256), 0, s, d_subs);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_cast_f32(const double *src, float *dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

hipError_t cast_to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// B0_Gamma^(i): the equation tested with the constant pressure on the
// subdomain (eq. discMat) is the sum of the element flux rows; by symmetry of
// the local matrix, entry l is the sum over pressure columns of interface row
// l.  b0[ng] = the p0 right-hand side (sum of the pressure right-hand sides).
// Computed from the FP64 CSR, deterministic.
__global__ void k_flux_rows(const SubDev *subs) {
  const SubDev S = subs[blockIdx.y];
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= S.n_csr) return;
  const int pr = S.pos[row];
  const int g0 = S.nv + S.nel;
  if (pr >= g0) {  // interface row
    double s = 0.0;
    for (int64_t q = S.indptr[row]; q < S.indptr[row + 1]; ++q) {
      const int pc = S.pos[S.indices[q]];
      if (pc >= S.nv && pc < g0) s += S.vals[q];
    }
    S.b0[pr - g0] = s;
  }
  if (row == 0) {
    double s = 0.0;
    for (int i = 0; i < S.n_csr; ++i) {
      const int p = S.pos[i];
      if (p >= S.nv && p < g0) s += S.rhs[i];
    }
    S.b0[S.ng] = s;
  }
}

hipError_t flux_rows(const SubDev *d_subs, int nsub, int max_rows, hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_flux_rows, dim3((max_rows + 255) / 256, nsub), dim3(256), 0, s, d_subs);
  return hipGetLastError();
}

// Householder reflector H = I - tau v v^T with H w = -sign(w_last)|w| e_last
// for the element volumes w: columns 0..nel-2 of H span Q_I (volume-weighted
// mean zero, eq. discVQ), the last coordinate is the w direction.
__global__ void k_house_vec(const SubDev *subs) {
  const SubDev S = subs[blockIdx.x];
  __shared__ double red[16];
  double ss = 0.0;
  for (int i = threadIdx.x; i < S.nel; i += blockDim.x) ss += S.pweight[i] * S.pweight[i];
  ss = block_sum(ss, red);
  const double nrm = sqrt(ss);
  const double wl = S.pweight[S.nel - 1];
  const double alpha = (wl >= 0.0) ? -nrm : nrm;
  for (int i = threadIdx.x; i < S.nel; i += blockDim.x)
    S.hv[i] = S.pweight[i] - ((i == S.nel - 1) ? alpha : 0.0);
  __syncthreads();
  double vv = 0.0;
  for (int i = threadIdx.x; i < S.nel; i += blockDim.x) vv += S.hv[i] * S.hv[i];
  vv = block_sum(vv, red);
  if (threadIdx.x == 0) S.hv[S.nel] = (vv > 0.0) ? 2.0 / vv : 0.0;
}

// rows: W[p, j] <- H W[p, j] for every column j (one wave per column)
template <typename T>
__global__ void k_house_rows(const SubDev *subs) {
  const SubDev S = subs[blockIdx.y];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + w;
  if (j >= S.N) return;
  T *col = Wp<T>(S) + (int64_t)j * S.ld + S.nv;
  const double tau = S.hv[S.nel];
  double s = 0.0;
  for (int r = l; r < S.nel; r += 64) s += S.hv[r] * (double)col[r];
  s = warp_sum(s);
  for (int r = l; r < S.nel; r += 64) col[r] = (T)((double)col[r] - tau * S.hv[r] * s);
}

// cols: W[i, p] <- W[i, p] H for every row i (one thread per row, coalesced)
template <typename T>
__global__ void k_house_cols(const SubDev *subs) {
  const SubDev S = subs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.N) return;
  const double tau = S.hv[S.nel];
  T *base = Wp<T>(S) + i + (int64_t)S.nv * S.ld;
  double s = 0.0;
  for (int c = 0; c < S.nel; ++c) s += (double)base[(int64_t)c * S.ld] * S.hv[c];
  for (int c = 0; c < S.nel; ++c)
    base[(int64_t)c * S.ld] = (T)((double)base[(int64_t)c * S.ld] - tau * s * S.hv[c]);
}

hipError_t house_pressure(const SubDev *d_subs, int nsub, int max_N, bool fp32, hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_house_vec, dim3(nsub), dim3(256), 0, s, d_subs);
  dim3 gr((max_N + 3) / 4, nsub), gc((max_N + 255) / 256, nsub);
  if (fp32) {
    hipLaunchKernelGGL(k_house_rows<float>, gr, dim3(256), 0, s, d_subs);
    hipLaunchKernelGGL(k_house_cols<float>, gc, dim3(256), 0, s, d_subs);
  } else {
    hipLaunchKernelGGL(k_house_rows<double>, gr, dim3(256), 0, s, d_subs);
    hipLaunchKernelGGL(k_house_cols<double>, gc, dim3(256), 0, s, d_subs);
  }
  return hipGetLastError();
}

// Householder QR with column pivoting of C^T (n x n_con) per entity: the
// first `rank` reflectors map the constraint span onto the leading
// coordinates; columns whose residual norm falls below tol * (largest
// initial norm) are dependent and dropped (Sec. 5.1).  One block per entity.
__global__ void k_entity_qr(const EntDev *ents, int rmax, double tol) {
  const EntDev E = ents[blockIdx.x];
  const int n = E.n, r = E.n_con;
  double *M = E.work;          // n x r column-major working copy of C^T
  __shared__ double nrm[1024]; // residual column norms^2 (r <= 1024)
  __shared__ double red[16];
  __shared__ int piv;
  for (int idx = threadIdx.x; idx < n * r; idx += blockDim.x) {
    int i = idx % n, c = idx / n;
    M[idx] = E.con[(int64_t)c * n + i];
  }
  __syncthreads();
  double maxn0 = 0.0;
  for (int c = 0; c < r; ++c) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += M[i + c * n] * M[i + c * n];
    s = block_sum(s, red);
    if (threadIdx.x == 0) nrm[c] = s;
    maxn0 = fmax(maxn0, s);
    __syncthreads();
  }
  int rank = 0;
  const int kmax = min(min(r, n), rmax);
  for (int k = 0; k < kmax; ++k) {
    if (threadIdx.x == 0) {
      int best = k;
      for (int c = k + 1; c < r; ++c)
        if (nrm[c] > nrm[best]) best = c;
      piv = best;
    }
    __syncthreads();
    const int p = piv;
    // exact residual norm of the pivot column rows k..n-1
    double s = 0.0;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) s += M[i + p * n] * M[i + p * n];
    s = block_sum(s, red);
    if (!(s > tol * tol * maxn0) || maxn0 == 0.0) break;
    if (p != k) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double t = M[i + k * n];
        M[i + k * n] = M[i + p * n];
        M[i + p * n] = t;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = nrm[k];
        nrm[k] = nrm[p];
        nrm[p] = t;
      }
    }
    __syncthreads();
    const double sig = sqrt(s);
    const double x0 = M[k + k * n];
    const double alpha = (x0 >= 0.0) ? -sig : sig;
    // v = x - alpha e_k (rows k..n-1), tau = 2 / v^T v
    double *V = E.V + (int64_t)k * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      V[i] = (i < k) ? 0.0 : M[i + k * n] - ((i == k) ? alpha : 0.0);
    __syncthreads();
    double vv = 0.0;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) vv += V[i] * V[i];
    vv = block_sum(vv, red);
    const double tau = 2.0 / vv;
    if (threadIdx.x == 0) E.tau[k] = tau;
    // apply to the remaining columns
    for (int c = k + 1; c < r; ++c) {
      double d = 0.0;
      for (int i = k + threadIdx.x; i < n; i += blockDim.x) d += V[i] * M[i + c * n];
      d = block_sum(d, red);
      for (int i = k + threadIdx.x; i < n; i += blockDim.x) M[i + c * n] -= tau * d * V[i];
      __syncthreads();
      double t = 0.0;
      for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) t += M[i + c * n] * M[i + c * n];
      t = block_sum(t, red);
      if (threadIdx.x == 0) nrm[c] = t;
      __syncthreads();
    }
    rank = k + 1;
  }
  if (threadIdx.x == 0) *E.rank = rank;
}

hipError_t entity_qr(const EntDev *d_ents, int nent, int rmax, double tol, hipStream_t s) {
  if (!nent) return hipSuccess;
  hipLaunchKernelGGL(k_entity_qr, dim3(nent), dim3(256), 0, s, d_ents, rmax, tol);
  return hipGetLastError();
}

// A_b[(r0 + i) + (c0 + i) * ld] = val for i < cnt (identity blocks).
__global__ void k_set_diag(const DiagJob *jobs) {
  const DiagJob J = jobs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= J.cnt) return;
  const int64_t o = (int64_t)(J.r0 + i) + (int64_t)(J.c0 + i) * J.ld;
  if (J.f32)
    ((float *)J.A)[o] = (float)J.val;
  else
    ((double *)J.A)[o] = J.val;
}

hipError_t set_diag(const DiagJob *d_jobs, int batch, int max_cnt, hipStream_t s) {
  if (!batch || !max_cnt) return hipSuccess;
  hipLaunchKernelGGL(k_set_diag, dim3((max_cnt + 255) / 256, batch), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// out[i] = A[i + i * ld] for i < n (the diagonal of a column-major matrix,
// made contiguous for one small copy to the host).
__global__ void k_diag_gather(const double *A, int64_t ld, int n, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = A[(int64_t)i * (ld + 1)];
}

hipError_t diag_gather(const double *A, int64_t ld, int n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_gather, dim3((n + 255) / 256), dim3(256), 0, s, A, ld, n, out);
  return hipGetLastError();
}

// Coarse matrix of the partially assembled problem (eq. BDDCprec):
// [[sum_i R_Pi^T S_Pi^(i) R_Pi, B0_Pi^T], [B0_Pi, -w w^T]] with w the
// normalised subdomain volumes (removes the constant-p0 kernel of the
// no-slip problem), bordered with the identity for the inverse.  Single
// block, subdomains in order: the sums are deterministic.
__global__ void k_coarse_assemble(const CoarseSub *cs, int nsub, double *K, int64_t ld, int nC,
                                  const double *w) {
  for (int s = 0; s < nsub; ++s) {
    const CoarseSub C = cs[s];
    const int m = C.npi;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int a = idx % m, b = idx / m;
      K[(int64_t)C.cidx[a] + (int64_t)C.cidx[b] * ld] += C.SPi[(int64_t)a + (int64_t)b * C.ld];
    }
    for (int a = threadIdx.x; a < m; a += blockDim.x) {
      const double v = C.b0[C.pl[a]];
      K[(int64_t)(nC + s) + (int64_t)C.cidx[a] * ld] = v;
      K[(int64_t)C.cidx[a] + (int64_t)(nC + s) * ld] = v;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < nsub * nsub; idx += blockDim.x) {
    const int a = idx % nsub, b = idx / nsub;
    K[(int64_t)(nC + a) + (int64_t)(nC + b) * ld] = -w[a] * w[b];
  }
}

hipError_t coarse_assemble(const CoarseSub *d_cs, int nsub, double *K, int64_t ld, int nC,
                           const double *w, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_assemble, dim3(1), dim3(1024), 0, s, d_cs, nsub, K, ld, nC, w);
  return hipGetLastError();
}

// Symmetrize square blocks: upper <- lower.
template <typename T>
__global__ void k_symmetrize(void *const *mats, const int64_t *lds, const int32_t *ns) {
  T *A = (T *)mats[blockIdx.z];
  const int64_t ld = lds[blockIdx.z];
  const int n = ns[blockIdx.z];
  __shared__ T t[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;  // tile (bi, bj) with bi > bj is the source
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    int r = bi * 32 + tx, c = bj * 32 + yy;
    t[yy][tx] = (r < n && c < n) ? A[r + c * ld] : T(0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    int r = bj * 32 + tx, c = bi * 32 + yy;  // destination (r, c) = source (c, r)
    if (r < n && c < n && c > r) A[r + c * ld] = t[tx][yy];
  }
}

hipError_t symmetrize(void *const *mats, const int64_t *lds, const int32_t *ns, int batch,
                      int max_n, bool fp32, hipStream_t s) {
  if (!batch || !max_n) return hipSuccess;
  int nt = (max_n + 31) / 32;
  if (fp32)
    hipLaunchKernelGGL(k_symmetrize<float>, dim3(nt, nt, batch), dim3(256), 0, s, mats, lds, ns);
  else
    hipLaunchKernelGGL(k_symmetrize<double>, dim3(nt, nt, batch), dim3(256), 0, s, mats, lds, ns);
  return hipGetLastError();
}

// In-place transpose of square blocks (swap tiles (bi,bj) and (bj,bi)).
template <typename T>
__global__ void k_transpose_sq(void *const *mats, const int64_t *lds, const int32_t *ns) {
  T *A = (T *)mats[blockIdx.z];
  const int64_t ld = lds[blockIdx.z];
  const int n = ns[blockIdx.z];
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  __shared__ T ta[32][33], tb[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    int r = bi * 32 + tx, c = bj * 32 + yy;
    ta[yy][tx] = (r < n && c < n) ? A[r + c * ld] : T(0);
    r = bj * 32 + tx;
    c = bi * 32 + yy;
    tb[yy][tx] = (r < n && c < n) ? A[r + c * ld] : T(0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    int r = bj * 32 + tx, c = bi * 32 + yy;
    if (r < n && c < n) A[r + c * ld] = ta[tx][yy];
    r = bi * 32 + tx;
    c = bj * 32 + yy;
    if (r < n && c < n) A[r + c * ld] = tb[tx][yy];
  }
}

hipError_t transpose_sq(void *const *mats, const int64_t *lds, const int32_t *ns, int batch,
                        int max_n, bool fp32, hipStream_t s) {
  if (!batch || !max_n) return hipSuccess;
  int nt = (max_n + 31) / 32;
  if (fp32)
    hipLaunchKernelGGL(k_transpose_sq<float>, dim3(nt, nt, batch), dim3(256), 0, s, mats, lds, ns);
  else
    hipLaunchKernelGGL(k_transpose_sq<double>, dim3(nt, nt, batch), dim3(256), 0, s, mats, lds, ns);
  return hipGetLastError();
}

// X <- X T for the condensed bordered interface block X (size ng+1): for
// every local entity, apply its reflectors H_0, H_1, ... to the entity's
// columns.  A workgroup takes R rows of one entity block into LDS, applies
// all the entity's reflectors there (256/R lanes per row; a lane always owns
// the same columns, so the rows need no barrier between reflectors: the dot
// products meet in shuffles), and writes the block back once.
template <typename T, int R>
__global__ __launch_bounds__(256) void k_apply_T_cols(const SubDev *subs, const EntDev *ents) {
  constexpr int L = 256 / R;
  const SubDev S = subs[blockIdx.z];
  if ((int)blockIdx.y >= S.n_ent) return;
  const int nx = S.ng + 1;
  const int i0 = blockIdx.x * R;
  if (i0 >= nx) return;
  const EntDev E = ents[S.ent[blockIdx.y]];
  const int rk = *E.rank, n = E.n;
  if (rk <= 0) return;
  extern __shared__ __align__(16) unsigned char smem_t[];
  T *Xs = reinterpret_cast<T *>(smem_t);  // R x n, column-major
  T *X = (T *)S.X + (int64_t)S.ent_off[blockIdx.y] * S.xld;
  const int rows = min(R, nx - i0);
  for (int idx = threadIdx.x; idx < R * n; idx += blockDim.x) {
    const int r = idx % R, c = idx / R;
    Xs[idx] = (r < rows) ? X[(int64_t)(i0 + r) + (int64_t)c * S.xld] : T(0);
  }
  __syncthreads();
  const int r = threadIdx.x / L, l = threadIdx.x % L;
  for (int k = 0; k < rk; ++k) {
    const double *v = E.V + (int64_t)k * n;
    double t = 0.0;
    for (int c = l; c < n; c += L)
      if (c >= k) t += (double)Xs[c * R + r] * v[c];
    for (int m = L / 2; m > 0; m >>= 1) t += __shfl_xor(t, m, L);
    t *= E.tau[k];
    for (int c = l; c < n; c += L)
      if (c >= k) Xs[c * R + r] = (T)((double)Xs[c * R + r] - t * v[c]);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < R * n; idx += blockDim.x) {
    const int rr = idx % R, c = idx / R;
    if (rr < rows) X[(int64_t)(i0 + rr) + (int64_t)c * S.xld] = Xs[idx];
  }
}

template <typename T, int R>
static hipError_t launch_apply_T(const SubDev *d_subs, const EntDev *d_ents, int nsub, int nx,
                                 int max_ent, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)k_apply_T_cols<T, R>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_apply_T_cols<T, R>), dim3((nx + R - 1) / R, max_ent, nsub), dim3(256), lds,
                     s, d_subs, d_ents);
  return hipGetLastError();
}

template <typename T>
static hipError_t apply_T_typed(const SubDev *d_subs, const EntDev *d_ents, int nsub, int nx,
                                int max_ent, int max_en, hipStream_t s) {
  // rows per workgroup: more rows read longer contiguous segments of each
  // column, but past 48 KB of LDS fewer workgroups share a CU (at the
  // 216-subdomain workload the setup took about 90 ms longer with 16 rows
  // in 101 KB than with 4 rows in 25 KB)
  const size_t row = (size_t)std::max(max_en, 1) * sizeof(T);
  if (16 * row <= 48 * 1024) return launch_apply_T<T, 16>(d_subs, d_ents, nsub, nx, max_ent, 16 * row, s);
  if (8 * row <= 48 * 1024) return launch_apply_T<T, 8>(d_subs, d_ents, nsub, nx, max_ent, 8 * row, s);
  if (4 * row <= 150 * 1024) return launch_apply_T<T, 4>(d_subs, d_ents, nsub, nx, max_ent, 4 * row, s);
  return hipErrorInvalidValue;  // an entity larger than 4 rows of LDS can hold
}

hipError_t apply_T_cols(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ng,
                        int max_ent, int max_en, bool fp32, hipStream_t s) {
  if (!nsub || !max_ent) return hipSuccess;
  return fp32 ? apply_T_typed<float>(d_subs, d_ents, nsub, max_ng + 1, max_ent, max_en, s)
              : apply_T_typed<double>(d_subs, d_ents, nsub, max_ng + 1, max_ent, max_en, s);
}

// T^T applied from the left to one entity's rows (ent_off .. ent_off + n) of
// every column of the bordered block X.  The entity's segment of a column is
// contiguous: a wave (n > 32: entries lane + 64 q, in the storage type) or a
// group of G lanes (G the smallest power of two >= n: one entry each) reads
// it with coalesced loads and keeps it in registers.  The (at most
// APPLY_T_RK) reflectors act at once in their compact form,
// H_{r-1} ... H_0 = I - V Tw^T V^T with Tw upper triangular (Tw_ii = tau_i,
// Tw[0:i, i] = -tau_i Tw[0:i, 0:i] V[:, 0:i]^T v_i): w = V^T x (r dot
// products, reduced in the group together), u = Tw^T w, x -= V u.  V and Tw
// are staged in LDS once per workgroup of up to 256 columns (the reflectors
// are stored with zeros above their leading entry).  (X T = (T^T X^T)^T for
// the symmetric X: applied, transposed, applied.)
constexpr int APPLY_T_EPL = 32, APPLY_T_RK = 4;

// x -= V Tw^T V^T x on one segment of n <= 64 APPLY_T_EPL entries held by a
// whole wave (entry lane + 64 q).
template <typename T>
__device__ __forceinline__ void seg_apply_wave(T *col, int n, int rk, const double *Vs, const double *Tw,
                                               int lane) {
  constexpr int EPL = APPLY_T_EPL, RK = APPLY_T_RK;
  T x[EPL];
#pragma unroll
  for (int q = 0; q < EPL; ++q) x[q] = (64 * q < n && lane + 64 * q < n) ? col[lane + 64 * q] : T(0);
  double wv[RK];
#pragma unroll
  for (int k = 0; k < RK; ++k) {
    double t = 0.0;
    if (k < rk) {
      const double *v = Vs + k * n + lane;
#pragma unroll
      for (int q = 0; q < EPL; ++q)
        if (64 * q < n && lane + 64 * q < n) t += (double)x[q] * v[64 * q];
    }
    wv[k] = t;
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1)
#pragma unroll
    for (int k = 0; k < RK; ++k) wv[k] += __shfl_xor(wv[k], m);
  double u[RK];
#pragma unroll
  for (int i = 0; i < RK; ++i) {  // u = Tw^T w
    double t = 0.0;
#pragma unroll
    for (int a = 0; a <= i; ++a) t += Tw[a + i * RK] * wv[a];
    u[i] = i < rk ? t : 0.0;
  }
#pragma unroll
  for (int q = 0; q < EPL; ++q)
    if (64 * q < n && lane + 64 * q < n) {
      double t = (double)x[q];
#pragma unroll
      for (int k = 0; k < RK; ++k)
        if (k < rk) t -= Vs[k * n + lane + 64 * q] * u[k];
      col[lane + 64 * q] = (T)t;
    }
}

// The same for a segment of n <= G entries held by a group of G lanes (one
// entry per lane).
template <typename T>
__device__ __forceinline__ void seg_apply_group(T *col, int n, int rk, const double *Vs, const double *Tw,
                                                int gl, int G) {
  constexpr int RK = APPLY_T_RK;
  const bool in = gl < n;
  const double x = in ? (double)col[gl] : 0.0;
  double wv[RK];
#pragma unroll
  for (int k = 0; k < RK; ++k) wv[k] = (in && k < rk) ? x * Vs[k * n + gl] : 0.0;
  for (int m = G / 2; m > 0; m >>= 1)
#pragma unroll
    for (int k = 0; k < RK; ++k) wv[k] += __shfl_xor(wv[k], m, G);
  double t = x;
#pragma unroll
  for (int i = 0; i < RK; ++i) {
    double ui = 0.0;
#pragma unroll
    for (int a = 0; a <= i; ++a) ui += Tw[a + i * RK] * wv[a];
    if (in && i < rk) t -= Vs[i * n + gl] * ui;
  }
  if (in) col[gl] = (T)t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_apply_T_rows(const SubDev *subs, const EntDev *ents, int cols) {
  constexpr int RK = APPLY_T_RK;
  const SubDev S = subs[blockIdx.z];
  if ((int)blockIdx.y >= S.n_ent) return;
  const int nx = S.ng + 1;
  const int c0 = blockIdx.x * cols;
  if (c0 >= nx) return;
  const EntDev E = ents[S.ent[blockIdx.y]];
  const int rk = min(*E.rank, RK), n = E.n;  // the host checked rank <= RK
  if (rk <= 0) return;  // uniform over the workgroup
  extern __shared__ __align__(16) unsigned char smem_r[];
  double *Vs = reinterpret_cast<double *>(smem_r);  // rk x n, reflector k at k * n
  __shared__ double Gm[RK * RK], Tw[RK * RK];
  for (int idx = threadIdx.x; idx < rk * n; idx += blockDim.x) Vs[idx] = E.V[idx];
  if (threadIdx.x < RK * RK) Tw[threadIdx.x] = 0.0;
  __syncthreads();
  if (threadIdx.x < rk * rk) {  // Gram matrix V^T V (the strict upper part is used)
    const int a = threadIdx.x % rk, b = threadIdx.x / rk;
    double g = 0.0;
    if (a < b)
      for (int c = 0; c < n; ++c) g += Vs[a * n + c] * Vs[b * n + c];
    Gm[a + b * RK] = g;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < rk; ++i) {
      const double ti = E.tau[i];
      for (int a = 0; a < i; ++a) {
        double s = 0.0;
        for (int b = a; b < i; ++b) s += Tw[a + b * RK] * Gm[b + i * RK];
        Tw[a + i * RK] = -ti * s;
      }
      Tw[i + i * RK] = ti;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T *Xe = (T *)S.X + S.ent_off[blockIdx.y];
  const int c1 = min(c0 + cols, nx);
  if (n > 32) {  // a wave per column
    for (int j = c0 + w; j < c1; j += 4) seg_apply_wave(Xe + (int64_t)j * S.xld, n, rk, Vs, Tw, lane);
  } else {  // groups of G <= 32 lanes, one column each
    int G = 1;
    while (G < n) G *= 2;
    const int gpw = 64 / G, g = lane / G, gl = lane % G;
    for (int j = c0 + w * gpw + g; j < c1; j += 4 * gpw)  // uniform over each group
      seg_apply_group(Xe + (int64_t)j * S.xld, n, rk, Vs, Tw, gl, G);
  }
}

// Left application to every entity block when the largest entity fits the
// registers (n <= 64 EPL), its reflectors the LDS and their count APPLY_T_RK
// (bounded on the host by min(n_con, n)); false: the caller applies the
// column kernel instead.
hipError_t apply_T_rows(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ng, int max_ent,
                        int max_en, int max_rn, int max_rank, bool fp32, bool *done, hipStream_t s) {
  *done = false;
  if (!nsub || !max_ent) {
    *done = true;
    return hipSuccess;
  }
  const size_t lds = (size_t)std::max(max_rn, 1) * sizeof(double);
  if (max_en > 64 * APPLY_T_EPL || max_rank > APPLY_T_RK || lds > 140 * 1024) return hipSuccess;
  const int cols = 256, nx = max_ng + 1;
  const dim3 grid((nx + cols - 1) / cols, max_ent, nsub);
  hipError_t e = hipSuccess;
  if (fp32) {
    if (lds > 48 * 1024)
      e = hipFuncSetAttribute((const void *)k_apply_T_rows<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e == hipSuccess)
      hipLaunchKernelGGL((k_apply_T_rows<float>), grid, dim3(256), lds, s, d_subs, d_ents, cols);
  } else {
    if (lds > 48 * 1024)
      e = hipFuncSetAttribute((const void *)k_apply_T_rows<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e == hipSuccess)
      hipLaunchKernelGGL((k_apply_T_rows<double>), grid, dim3(256), lds, s, d_subs, d_ents, cols);
  }
  if (e != hipSuccess) return e;
  e = hipGetLastError();
  if (e == hipSuccess) *done = true;
  return e;
}

// b0~ = T^T b0 (per local entity, reflectors in order H_0, H_1, ...).
__global__ void k_transform_b0(const SubDev *subs, const EntDev *ents) {
  const SubDev S = subs[blockIdx.x];
  __shared__ double red[16];
  for (int q = 0; q < S.n_ent; ++q) {
    const EntDev E = ents[S.ent[q]];
    const int o = S.ent_off[q];
    const int rk = *E.rank;
    for (int k = 0; k < rk; ++k) {
      const double *v = E.V + (int64_t)k * E.n;
      double t = 0.0;
      for (int c = k + threadIdx.x; c < E.n; c += blockDim.x) t += S.b0[o + c] * v[c];
      t = block_sum(t, red) * E.tau[k];
      for (int c = k + threadIdx.x; c < E.n; c += blockDim.x) S.b0[o + c] -= t * v[c];
      __syncthreads();
    }
  }
}

hipError_t transform_b0(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ent,
                        hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_transform_b0, dim3(nsub), dim3(256), 0, s, d_subs, d_ents);
  return hipGetLastError();
}

// Global vector in the entity blocks: dir=+1 x <- T^T x, dir=-1 x <- T x.
__global__ void k_transform_vec(const EntDev *ents, double *x, int dir) {
  const EntDev E = ents[blockIdx.x];
  __shared__ double red[16];
  const int rk = *E.rank;
  for (int kk = 0; kk < rk; ++kk) {
    const int k = (dir > 0) ? kk : rk - 1 - kk;
    const double *v = E.V + (int64_t)k * E.n;
    double t = 0.0;
    for (int c = k + threadIdx.x; c < E.n; c += blockDim.x) t += x[E.gids[c]] * v[c];
    t = block_sum(t, red) * E.tau[k];
    for (int c = k + threadIdx.x; c < E.n; c += blockDim.x) x[E.gids[c]] -= t * v[c];
    __syncthreads();
  }
}

hipError_t transform_vec(const EntDev *d_ents, int nent, double *x, int dir, hipStream_t s) {
  if (!nent) return hipSuccess;
  hipLaunchKernelGGL(k_transform_vec, dim3(nent), dim3(256), 0, s, d_ents, x, dir);
  return hipGetLastError();
}

// out[i + j*ldo] (+)= scale * in[ri[i] + ci[j]*ldi].  A workgroup takes a
// 64 x 64 block, a lane a row, each wave 16 of the columns: all 16 source
// loads are issued before the first store (clamped, unconditional addresses
// for the rows and columns past the block's edge, which are not stored).
__global__ __launch_bounds__(256) void k_gather_blocks(const GatherJob *jobs) {
  constexpr int Q = 16;
  const GatherJob J = jobs[blockIdx.z];
  if ((int)blockIdx.x * 64 >= J.m || (int)blockIdx.y * 64 >= J.n) return;  // uniform
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j0 = blockIdx.y * 64 + (threadIdx.x >> 6);
  const bool row = i < J.m;
  const int ri = J.ri[min(i, J.m - 1)];
  double v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = min(j0 + 4 * q, J.n - 1);
    const int64_t src = (int64_t)ri + (int64_t)J.ci[j] * J.ldi;
    v[q] = J.in_f32 ? (double)((const float *)J.in)[src] : ((const double *)J.in)[src];
  }
  if (!row) return;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = j0 + 4 * q;
    if (j >= J.n) break;
    const double x = v[q] * J.scale;
    const int64_t dst = (int64_t)i + (int64_t)j * J.ldo;
    if (J.out_f32) {
      float *o = (float *)J.out + dst;
      *o = J.add ? (float)((double)*o + x) : (float)x;
    } else {
      double *o = (double *)J.out + dst;
      *o = J.add ? *o + x : x;
    }
  }
}

hipError_t gather_blocks(const GatherJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s) {
  if (!batch || !max_m || !max_n) return hipSuccess;
  hipLaunchKernelGGL(k_gather_blocks, dim3((max_m + 63) / 64, (max_n + 63) / 64, batch), dim3(256),
                     0, s, d_jobs);
  return hipGetLastError();
}

// ---------------------------------------------------------------- recovery
// y = L_rI^T - L_GammaI^T u_Gamma over the eliminated columns (eq. uipi after
// the factorisation: K_II^-1 (r_I - C u_Gamma) = L_II^-T y).  One wave per column.
template <typename T>
__global__ void k_recover_rhs(const SubDev *subs, const double *x, double *y, const int64_t *yoff) {
  const SubDev S = subs[blockIdx.y];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + w;
  if (j >= S.e) return;
  const auto col = gptr(Wp<T>(S) + (int64_t)j * S.ld + (S.e + 1));
  double s = 0.0;
  for (int r = l; r < S.ng; r += 64) s += (double)col[r] * x[S.gidl[r]];
  s = warp_sum(s);
  if (l == 0) y[yoff[blockIdx.y] + j] = (double)col[S.ng] - s;
}

hipError_t recover_rhs(const SubDev *d_subs, const double *x_orig, double *y, const int64_t *yoff,
                       int nsub, int max_e, bool fp32, hipStream_t s) {
  if (!nsub) return hipSuccess;
  dim3 g((max_e + 3) / 4, nsub);
  if (fp32)
    hipLaunchKernelGGL(k_recover_rhs<float>, g, dim3(256), 0, s, d_subs, x_orig, y, yoff);
  else
    hipLaunchKernelGGL(k_recover_rhs<double>, g, dim3(256), 0, s, d_subs, x_orig, y, yoff);
  return hipGetLastError();
}

// Four consecutive entries of a column (16-byte aligned), widened to FP64.
__device__ __forceinline__ void load4(const float *p, double v[4]) {
  const float4 f = *reinterpret_cast<const float4 *>(p);
  v[0] = f.x, v[1] = f.y, v[2] = f.z, v[3] = f.w;
}
__device__ __forceinline__ void load4(const double *p, double v[4]) {
  const double2 *q = reinterpret_cast<const double2 *>(p);
  const double2 a = q[0], b = q[1];
  v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
}

// Right-looking block back substitution for L_II^T z = y, step for the block
// i = [i0, i0+b): z_i = inv(L_ii)^T y_i (every workgroup recomputes it from
// the cached inverse, staged in LDS; workgroup 0 stores it), then
// y_k -= L[i-block, k]^T z_i for the columns k < i0 of this workgroup's range
// of RS_COLS.  The block rows of a column are contiguous in the column-major
// factor: 16 lanes cover them with 16-byte loads (4 rows each, z in
// registers) and reduce with 4 shuffles; each group of 16 lanes keeps four
// columns in flight (loads issued together, clamped to a column of the
// range, the reductions interleaved), so a wave finishes 16 columns per step.
// (1,024 columns per workgroup amortised the z preamble better but left the
// late steps of the largest matrices with too few workgroups: slower.)
constexpr int RS_COLS = 256;
template <typename T>
__global__ __launch_bounds__(256) void k_recover_step(const SubDev *subs, const T *invL,
                                                      const int64_t *invoff, double *y,
                                                      double *z, const int64_t *yoff, int i0,
                                                      int nb) {
  const SubDev S = subs[blockIdx.y];
  if (i0 >= S.e) return;
  const int k0 = blockIdx.x * RS_COLS;
  if (k0 > 0 && k0 >= i0) return;
  const int b = min(nb, S.e - i0);
  double *ys = y + yoff[blockIdx.y];
  double *zs = z + yoff[blockIdx.y];
  __shared__ T inv_s[64 * 65];
  __shared__ double yi[64], zi[64];
  const T *inv = invL + invoff[blockIdx.y] + (int64_t)(i0 / nb) * nb * nb;
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) inv_s[(t / nb) * 65 + t % nb] = inv[t];
  if (threadIdx.x < b) yi[threadIdx.x] = ys[i0 + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < b) {
    const int c = threadIdx.x;
    double s = 0.0;  // (inv^T y)_c = sum_{r >= c} inv[r][c] y_r
    for (int r = c; r < b; ++r) s += (double)inv_s[c * 65 + r] * yi[r];
    zi[c] = s;
    if (blockIdx.x == 0) zs[i0 + c] = s;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, q = l & 15;
  double zq[4];
  for (int t = 0; t < 4; ++t) zq[t] = (4 * q + t < b) ? zi[4 * q + t] : 0.0;
  const bool full = 4 * q + 3 < b;
  const T *W = Wp<T>(S) + i0 + 4 * q;
  const int kend = min(k0 + RS_COLS, i0);  // columns [k0, kend) of this workgroup
  // group (w, g) takes columns k0 + 16 it + 4 w + g, four values of it at a time
  for (int it = 0; k0 + 16 * it < kend; it += 4) {
    double s[4];
    int kk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      kk[u] = k0 + 16 * (it + u) + 4 * w + g;
      const T *col = W + (int64_t)min(kk[u], kend - 1) * S.ld;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (full) {
        load4(col, v);
      } else {
        for (int t = 0; t < 4; ++t)
          if (4 * q + t < b) v[t] = (double)col[t];
      }
      s[u] = v[0] * zq[0] + v[1] * zq[1] + v[2] * zq[2] + v[3] * zq[3];
    }
#pragma unroll
    for (int m = 1; m < 16; m *= 2)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += __shfl_xor(s[u], m, 16);
    if (q == 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (kk[u] < kend) ys[kk[u]] -= s[u];
    }
  }
}

hipError_t recover_backsolve(const SubDev *d_subs, const void *invL, const int64_t *invoff,
                             double *y, double *z, const int64_t *yoff, int nsub, int i0, int nb,
                             bool fp32, hipStream_t s) {
  if (!nsub) return hipSuccess;
  if (nb != 32 && nb != 64) return hipErrorInvalidValue;
  const int gx = i0 > 0 ? (i0 + RS_COLS - 1) / RS_COLS : 1;
  if (fp32)
    hipLaunchKernelGGL(k_recover_step<float>, dim3(gx, nsub), dim3(256), 0, s, d_subs,
                       (const float *)invL, invoff, y, z, yoff, i0, nb);
  else
    hipLaunchKernelGGL(k_recover_step<double>, dim3(gx, nsub), dim3(256), 0, s, d_subs,
                       (const double *)invL, invoff, y, z, yoff, i0, nb);
  return hipGetLastError();
}

// ------------------------------------------------- mixed-precision refinement
// R = f - K u on every subdomain's local system (CSR order, FP64): one wave
// per row, lanes over the row's nonzeros (coalesced), wave reduction.
__global__ __launch_bounds__(256) void k_local_residual(const SubDev *subs, const double *u,
                                                        const int64_t *uoff, double *R) {
  const SubDev S = subs[blockIdx.y];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (row >= S.n_csr) return;
  const double *us = u + uoff[blockIdx.y];
  double s = 0.0;
  for (int64_t q = S.indptr[row] + l; q < S.indptr[row + 1]; q += 64)
    s += S.vals[q] * us[S.indices[q]];
  s = warp_sum(s);
  if (l == 0) R[uoff[blockIdx.y] + row] = S.rhs[row] - s;
}

hipError_t local_residual(const SubDev *d_subs, const double *u, const int64_t *uoff, double *R,
                          int nsub, int max_rows, hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_local_residual, dim3((max_rows + 3) / 4, nsub), dim3(256), 0, s, d_subs,
                     u, uoff, R);
  return hipGetLastError();
}

// y[pos[i]] = R[i] (dense order; R[oidx[i]] through the row map when given,
// 0 where it is -1), pressures rotated by the reflector H; r0 = sum of the
// (unrotated) pressure residuals.  One block per subdomain.
__global__ void k_residual_to_dense(const SubDev *subs, const double *R, const int64_t *roff,
                                    double *y, const int64_t *yoff, double *r0) {
  const SubDev S = subs[blockIdx.x];
  const double *Rs = R + roff[blockIdx.x];
  double *ys = y + yoff[blockIdx.x];
  __shared__ double red[16];
  double vr = 0.0, sr = 0.0;
  for (int i = threadIdx.x; i < S.n_csr; i += blockDim.x) {
    const int p = S.pos[i];
    const int o = S.oidx ? S.oidx[i] : i;
    const double v = o >= 0 ? Rs[o] : 0.0;
    ys[p] = v;
    if (p >= S.nv && p < S.nv + S.nel) {
      vr += S.hv[p - S.nv] * v;
      sr += v;
    }
  }
  vr = block_sum(vr, red);
  sr = block_sum(sr, red);
  __syncthreads();
  const double tau = S.hv[S.nel];
  for (int q = threadIdx.x; q < S.nel; q += blockDim.x) ys[S.nv + q] -= tau * S.hv[q] * vr;
  if (threadIdx.x == 0) r0[blockIdx.x] = sr;
}

hipError_t residual_to_dense(const SubDev *d_subs, const double *R, const int64_t *roff,
                             double *y, const int64_t *yoff, double *r0, int nsub, int max_rows,
                             hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_residual_to_dense, dim3(nsub), dim3(256), 0, s, d_subs, R, roff, y, yoff, r0);
  return hipGetLastError();
}

// Forward substitution step for block [i0, i0+b) of L (all rows below the
// block, interface rows included): z_i = inv(L_ii) y_i (inverse staged in
// LDS, recomputed by every workgroup, stored by workgroup 0);
// y_r -= sum_c L[r, i0+c] z_c for r in [i0+b, N-1).  Each thread owns 4
// consecutive rows (16-byte loads along the contiguous columns), a
// workgroup 1024 rows.
template <typename T>
__global__ __launch_bounds__(256) void k_forward_step(const SubDev *subs, const T *invL,
                                                      const int64_t *invoff, double *y, double *z,
                                                      const int64_t *yoff, int i0, int nb) {
  const SubDev S = subs[blockIdx.y];
  if (i0 >= S.e) return;
  const int b = min(nb, S.e - i0);
  const int rbeg = i0 + b, rend = S.N - 1;  // rows updated: [rbeg, rend)
  const int r0 = (rbeg & ~3) + blockIdx.x * 1024;
  if (r0 >= rend) return;  // never workgroup 0: rend > e >= rbeg
  double *ys = y + yoff[blockIdx.y];
  double *zs = z + yoff[blockIdx.y];
  __shared__ T inv_s[64 * 64];
  __shared__ double yi[64], zi[64];
  const T *inv = invL + invoff[blockIdx.y] + (int64_t)(i0 / nb) * nb * nb;
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) inv_s[t] = inv[t];
  if (threadIdx.x < b) yi[threadIdx.x] = ys[i0 + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < b) {
    const int r = threadIdx.x;
    double s = 0.0;  // (inv y)_r = sum_{c <= r} inv[r][c] y_c
    for (int c = 0; c <= r; ++c) s += (double)inv_s[r + c * nb] * yi[c];
    zi[r] = s;
    if (blockIdx.x == 0) zs[i0 + r] = s;
  }
  __syncthreads();
  const int r = r0 + 4 * threadIdx.x;
  if (r >= rend) return;
  const T *base = Wp<T>(S) + (int64_t)i0 * S.ld + r;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (r >= rbeg && r + 4 <= rend) {
#pragma unroll 8
    for (int c = 0; c < b; ++c) {
      double v[4];
      load4(base + (int64_t)c * S.ld, v);
      const double zc = zi[c];
      acc[0] += v[0] * zc, acc[1] += v[1] * zc, acc[2] += v[2] * zc, acc[3] += v[3] * zc;
    }
    for (int t = 0; t < 4; ++t) ys[r + t] -= acc[t];
  } else {
    for (int t = 0; t < 4; ++t) {
      if (r + t < rbeg || r + t >= rend) continue;
      double a = 0.0;
      for (int c = 0; c < b; ++c) a += (double)base[(int64_t)c * S.ld + t] * zi[c];
      ys[r + t] -= a;
    }
  }
}

hipError_t forward_step(const SubDev *d_subs, const void *invL, const int64_t *invoff, double *y,
                        double *z, const int64_t *yoff, int nsub, int i0, int nb, int max_N,
                        bool fp32, hipStream_t s) {
  if (!nsub) return hipSuccess;
  if (nb != 32 && nb != 64) return hipErrorInvalidValue;
  const int rows = max_N - i0 + 4;
  const int gx = rows > 0 ? (rows + 1023) / 1024 : 1;
  if (fp32)
    hipLaunchKernelGGL(k_forward_step<float>, dim3(gx, nsub), dim3(256), 0, s, d_subs,
                       (const float *)invL, invoff, y, z, yoff, i0, nb);
  else
    hipLaunchKernelGGL(k_forward_step<double>, dim3(gx, nsub), dim3(256), 0, s, d_subs,
                       (const double *)invL, invoff, y, z, yoff, i0, nb);
  return hipGetLastError();
}

// y2_j = d_j z_j over the eliminated columns (the interior correction's
// right-hand side before the interface term -L_GammaI^T dx, which a GEMV over
// the factor's interface rows adds).
__global__ void k_back_init(const SubDev *subs, const double *z, double *y2, const int64_t *yoff) {
  const SubDev S = subs[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.e) return;
  const int64_t o = yoff[blockIdx.y] + j;
  y2[o] = (j < S.nv) ? z[o] : -z[o];
}

hipError_t back_init(const SubDev *d_subs, const double *z, double *y2, const int64_t *yoff, int nsub,
                     int max_e, hipStream_t s) {
  if (!nsub || max_e <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_back_init, dim3((max_e + 255) / 256, nsub), dim3(256), 0, s, d_subs, z, y2, yoff);
  return hipGetLastError();
}

}  // namespace vb
