// Two-level nested dissection of the local Dirichlet problems (eq. uipi).
//
// Each subdomain is split into sub-boxes whose interiors (velocities and
// element pressures) do not couple; the separator DoFs between them join the
// interface DoFs at the second level.  A front is one sub-box: its dense
// matrix [[K_bb, K_bB], [K_Bb, 0]] is factored by the batched signed LDL^T
// up to its kept pressure coordinate (the volume-weighted direction of the
// sub-box's element pressures, as for a subdomain), and its trailing block
// [kept | B | rhs] is added into the second-level matrix of its subdomain,
// with the kept coordinate rescaled to the sub-box's constant pressure.  The
// second level is then a subdomain whose "elements" are the sub-boxes.
#include "common.h"
#include "kernels.h"

namespace vb {

// W2 += D T D over the front's trailing block T (rows and columns [e, e + m)
// of the front matrix, lower triangle read), D = diag(gamma, 1, ..., 1), at
// the second-level positions map[0..m), into W2's lower triangle only (the
// entry of a pair of positions goes to (max, min); the second level reads no
// other: its LDL^T works on the lower triangle, and the pressure rotation that
// precedes it reads the upper triangle only inside the sub-box constant
// block, where a front adds its one diagonal entry).  One thread per entry
// of the lower triangle's bounding square; a launch holds fronts of distinct
// subdomains only, so no two threads add into the same entry.
template <typename T>
__global__ __launch_bounds__(256) void k_front_scatter(const FrontJob *jobs) {
  const FrontJob J = jobs[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mm = (int64_t)J.m * J.m;
  if (t >= mm) return;
  const int a = (int)(t % J.m), b = (int)(t / J.m);
  if (a < b) return;
  const T *Wf = (const T *)J.Wf;
  T *W2 = (T *)J.W2;
  const double v = (double)Wf[(int64_t)(J.e + a) + (int64_t)(J.e + b) * J.ldf] *
                   (a == 0 ? J.gamma : 1.0) * (b == 0 ? J.gamma : 1.0);
  const int64_t pa = J.map[a], pb = J.map[b];
  const int64_t o = (pa >= pb) ? pa + pb * J.ld2 : pb + pa * J.ld2;
  W2[o] = (T)((double)W2[o] + v);
}

hipError_t front_scatter(const FrontJob *d_jobs, int njobs, int max_m, bool fp32, hipStream_t s) {
  if (!njobs || !max_m) return hipSuccess;
  const int64_t mm = (int64_t)max_m * max_m;
  dim3 g((unsigned)((mm + 255) / 256), njobs);
  if (fp32)
    hipLaunchKernelGGL(k_front_scatter<float>, g, dim3(256), 0, s, d_jobs);
  else
    hipLaunchKernelGGL(k_front_scatter<double>, g, dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// The trailing rows of a front's forward-substituted residual, added into
// its subdomain's second-level residual: y2[map[0]] += gamma yf[e] (the kept
// coordinate as the sub-box constant), y2[map[k]] += yf[e + k] for the
// separator and interface rows k = 1 .. m - 2 (the rhs slot is left out).
__global__ __launch_bounds__(256) void k_front_rhs(const FrontJob *jobs) {
  const FrontJob J = jobs[blockIdx.x];
  for (int k = threadIdx.x; k < J.m - 1; k += blockDim.x) {
    const double v = J.yf[J.e + k] * (k == 0 ? J.gamma : 1.0);
    J.y2[J.map[k]] += v;
  }
}

hipError_t front_rhs(const FrontJob *d_jobs, int njobs, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_front_rhs, dim3(njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// Second-level residual in dense order: the separator and interface rows of
// the local residual R (full CSR order, through oidx) are added to what the
// fronts put there, then the sub-box constant block (nel entries, filled by
// the fronts) is rotated by the second-level reflector.  One workgroup per
// subdomain.
__global__ __launch_bounds__(256) void k_l2_residual(const SubDev *subs, const double *R,
                                                     const int64_t *roff, double *y,
                                                     const int64_t *yoff) {
  const SubDev S = subs[blockIdx.x];
  const double *Rs = R + roff[blockIdx.x];
  double *ys = y + yoff[blockIdx.x];
  __shared__ double red[16];
  for (int i = threadIdx.x; i < S.n_csr; i += blockDim.x) ys[S.pos[i]] += Rs[S.oidx[i]];
  __syncthreads();
  double vr = 0.0;
  for (int q = threadIdx.x; q < S.nel; q += blockDim.x) vr += S.hv[q] * ys[S.nv + q];
  vr = block_sum(vr, red);
  const double tau = S.hv[S.nel];
  for (int q = threadIdx.x; q < S.nel; q += blockDim.x) ys[S.nv + q] -= tau * S.hv[q] * vr;
}

hipError_t l2_residual(const SubDev *d_subs, const double *R, const int64_t *roff, double *y,
                       const int64_t *yoff, int nsub, hipStream_t s) {
  if (!nsub) return hipSuccess;
  hipLaunchKernelGGL(k_l2_residual, dim3(nsub), dim3(256), 0, s, d_subs, R, roff, y, yoff);
  return hipGetLastError();
}

// out[s] = sum over items [first[s], first[s+1]) of in (fixed order).
__global__ void k_segment_sum(int n, const int32_t *first, const double *in, double *out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double v = 0.0;
  for (int f = first[s]; f < first[s + 1]; ++f) v += in[f];
  out[s] = v;
}

hipError_t segment_sum(int n, const int32_t *first, const double *in, double *out, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_segment_sum, dim3((n + 255) / 256), dim3(256), 0, s, n, first, in, out);
  return hipGetLastError();
}

}  // namespace vb
