// Learned predictor of the adaptive face constraints: per dual coordinate of
// a face, features of the reduced pencil matrix C = L^-1 At L^-T and a small
// fully connected network (tanh, tanh, sigmoid) predicting the coordinate's
// participation in the eigenvectors below 1/theta; FP32 forward, backward
// (deterministic block-partial reduction) and Adam.  Also the pieces of the
// warm-started Chebyshev-filtered subspace iteration that uses it.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace vb {

// parameter offsets in the flat layout [W1 H*F | b1 H | W2 H*H | b2 H | w3 H | b3]
constexpr int P_W1 = 0;
constexpr int P_B1 = P_W1 + MLP_H * MLP_F;
constexpr int P_W2 = P_B1 + MLP_H;
constexpr int P_B2 = P_W2 + MLP_H * MLP_H;
constexpr int P_W3 = P_B2 + MLP_H;
constexpr int P_B3 = P_W3 + MLP_H;
static_assert(P_B3 + 1 == MLP_NPARAMS, "parameter layout");

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

// ---------------------------------------------------------------- features
// One block per face.  C is n x n full symmetric (column-major, ld).  For
// coordinate c (x is written row-major, MLP_F per coordinate):
//  0 C_cc   1 log10 C_cc   2 sum_j |C_cj|   3 C_cc - sum_{j!=c} |C_cj|   4 c/n
//  5 mean_c C_cc   6 min_c C_cc   7 fraction of C_cc < sigma   8 log10 n
//  9 log10(tr At_par / tr B)   10 |log10(tr A_i / tr A_j)|   11 sigma
// rho[face] = max_c sum_j |C_cj| (Gershgorin bound of the spectrum).
__global__ __launch_bounds__(256) void k_face_features(const FeatJob *jobs) {
  const FeatJob J = jobs[blockIdx.x];
  const int n = J.n;
  __shared__ double red[16];
  __shared__ double s_mean, s_min, s_frac, s_rho;
  double sm = 0.0, mn = 1e300, fr = 0.0, rho = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double d = J.C[(int64_t)c + (int64_t)c * J.ld];
    sm += d;
    mn = fmin(mn, d);
    fr += (d < J.sigma) ? 1.0 : 0.0;
  }
  // row sums: thread per row, coalesced over j for consecutive rows
  sm = block_sum(sm, red);
  fr = block_sum(fr, red);
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmin(m, red[q]);
    s_min = m;
    s_mean = sm / n;
    s_frac = fr / n;
  }
  __syncthreads();
  // trp = [tr At_par, tr B], tra = [tr(A_i + A_j), tr A_j]
  const double lr = log10(fmax(J.trp[0], 1e-300) / fmax(J.trp[1], 1e-300));
  const double lc = fabs(log10(fmax(J.tra[0] - J.tra[1], 1e-300) / fmax(J.tra[1], 1e-300)));
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j) rs += fabs(J.C[(int64_t)c + (int64_t)j * J.ld]);
    const double d = J.C[(int64_t)c + (int64_t)c * J.ld];
    rho = fmax(rho, rs);
    float *x = J.X + (int64_t)c * MLP_F;
    x[0] = (float)d;
    x[1] = (float)log10(fmax(d, 1e-12));
    x[2] = (float)rs;
    x[3] = (float)(2.0 * d - rs);
    x[4] = (float)((double)c / n);
    x[5] = (float)s_mean;
    x[6] = (float)s_min;
    x[7] = (float)s_frac;
    x[8] = (float)log10((double)n);
    x[9] = (float)lr;
    x[10] = (float)lc;
    x[11] = (float)J.sigma;
  }
  for (int o = 32; o > 0; o >>= 1) rho = fmax(rho, __shfl_xor(rho, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rho;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
    J.rho[0] = m;
  }
}

hipError_t face_features(const FeatJob *d_jobs, int njobs, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_face_features, dim3(njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// Traces of square blocks (one block per job): out[q] = sum_i A_q[i + i ld].
__global__ void k_traces(const SymJob *jobs, double *out) {
  const SymJob J = jobs[blockIdx.x];
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < J.n; i += blockDim.x) s += J.A[(int64_t)i + (int64_t)i * J.ld];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

hipError_t traces(const SymJob *d_jobs, int njobs, double *out, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_traces, dim3(njobs), dim3(256), 0, s, d_jobs, out);
  return hipGetLastError();
}

// Labels: participation of coordinate c in the selected eigenvectors,
// y_c = sum_{t < m} Z[c, t]^2 (1 for every coordinate of a face whose
// eigenvalues are all selected).  One block per face.
__global__ void k_face_labels(const LabelJob *jobs) {
  const LabelJob J = jobs[blockIdx.x];
  for (int c = threadIdx.x; c < J.n; c += blockDim.x) {
    double s = 0.0;
    if (J.full) {
      s = 1.0;
    } else {
      for (int t = 0; t < J.m; ++t) {
        const double z = J.Z[(int64_t)c + (int64_t)t * J.ldz];
        s += z * z;
      }
    }
    J.y[c] = (float)s;
  }
}

hipError_t face_labels(const LabelJob *d_jobs, int njobs, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_face_labels, dim3(njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// ------------------------------------------------------------------ network
// Standardisation x' = (x - mu) / sd is applied on load (mu, sd: MLP_F each).
__device__ __forceinline__ void load_x(const float *X, int64_t i, const float *mu, const float *sd,
                                       float *x) {
#pragma unroll
  for (int f = 0; f < MLP_F; ++f) x[f] = (X[i * MLP_F + f] - mu[f]) / sd[f];
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *p, const float *mu,
                                                     const float *sd, const float *X, int64_t N,
                                                     float *s) {
  __shared__ float P[MLP_NPARAMS];
  for (int q = threadIdx.x; q < MLP_NPARAMS; q += blockDim.x) P[q] = p[q];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float x[MLP_F], h1[MLP_H];
  load_x(X, i, mu, sd, x);
  for (int a = 0; a < MLP_H; ++a) {
    float z = P[P_B1 + a];
    for (int f = 0; f < MLP_F; ++f) z += P[P_W1 + a * MLP_F + f] * x[f];
    h1[a] = tanhf(z);
  }
  float z3 = P[P_B3];
  for (int a = 0; a < MLP_H; ++a) {
    float z = P[P_B2 + a];
    for (int b = 0; b < MLP_H; ++b) z += P[P_W2 + a * MLP_H + b] * h1[b];
    z3 += P[P_W3 + a] * tanhf(z);
  }
  s[i] = sigm(z3);
}

hipError_t mlp_forward(const float *p, const float *mu, const float *sd, const float *X, int64_t N,
                       float *s, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, p, mu, sd,
                     X, N, s);
  return hipGetLastError();
}

// Gradient of L = (1/N) sum (s - y)^2: 64 samples per block; per-sample
// forward/backward by one thread each into LDS, then every parameter's sum
// over the block's samples (fixed order) into partial[block][param], and the
// block's loss into lpart[block].
constexpr int GB = 64;
__global__ __launch_bounds__(256) void k_mlp_grad(const float *p, const float *mu, const float *sd,
                                                  const float *X, const float *y, int64_t N,
                                                  float *partial, double *lpart) {
  __shared__ float P[MLP_NPARAMS];
  __shared__ float xs[GB][MLP_F], h1s[GB][MLP_H], h2s[GB][MLP_H], d1s[GB][MLP_H], d2s[GB][MLP_H];
  __shared__ float d3s[GB];
  __shared__ double ls[GB];
  for (int q = threadIdx.x; q < MLP_NPARAMS; q += blockDim.x) P[q] = p[q];
  __syncthreads();
  const int j = threadIdx.x;
  if (j < GB) {
    const int64_t i = (int64_t)blockIdx.x * GB + j;
    if (i < N) {
      float x[MLP_F];
      load_x(X, i, mu, sd, x);
      for (int f = 0; f < MLP_F; ++f) xs[j][f] = x[f];
      for (int a = 0; a < MLP_H; ++a) {
        float z = P[P_B1 + a];
        for (int f = 0; f < MLP_F; ++f) z += P[P_W1 + a * MLP_F + f] * x[f];
        h1s[j][a] = tanhf(z);
      }
      float z3 = P[P_B3];
      for (int a = 0; a < MLP_H; ++a) {
        float z = P[P_B2 + a];
        for (int b = 0; b < MLP_H; ++b) z += P[P_W2 + a * MLP_H + b] * h1s[j][b];
        const float h = tanhf(z);
        h2s[j][a] = h;
        z3 += P[P_W3 + a] * h;
      }
      const float s = sigm(z3);
      const float r = s - y[i];
      ls[j] = (double)r * (double)r;
      const float d3 = (2.0f / (float)N) * r * s * (1.0f - s);
      d3s[j] = d3;
      for (int a = 0; a < MLP_H; ++a) {
        const float h = h2s[j][a];
        d2s[j][a] = d3 * P[P_W3 + a] * (1.0f - h * h);
      }
      for (int b = 0; b < MLP_H; ++b) {
        float t = 0.0f;
        for (int a = 0; a < MLP_H; ++a) t += d2s[j][a] * P[P_W2 + a * MLP_H + b];
        const float h = h1s[j][b];
        d1s[j][b] = t * (1.0f - h * h);
      }
    } else {
      for (int f = 0; f < MLP_F; ++f) xs[j][f] = 0.0f;
      for (int a = 0; a < MLP_H; ++a) h1s[j][a] = h2s[j][a] = d1s[j][a] = d2s[j][a] = 0.0f;
      d3s[j] = 0.0f;
      ls[j] = 0.0;
    }
  }
  __syncthreads();
  float *out = partial + (int64_t)blockIdx.x * MLP_NPARAMS;
  for (int q = threadIdx.x; q < MLP_NPARAMS; q += blockDim.x) {
    float g = 0.0f;
    if (q < P_B1) {
      const int a = (q - P_W1) / MLP_F, f = (q - P_W1) % MLP_F;
      for (int jj = 0; jj < GB; ++jj) g += d1s[jj][a] * xs[jj][f];
    } else if (q < P_W2) {
      const int a = q - P_B1;
      for (int jj = 0; jj < GB; ++jj) g += d1s[jj][a];
    } else if (q < P_B2) {
      const int a = (q - P_W2) / MLP_H, b = (q - P_W2) % MLP_H;
      for (int jj = 0; jj < GB; ++jj) g += d2s[jj][a] * h1s[jj][b];
    } else if (q < P_W3) {
      const int a = q - P_B2;
      for (int jj = 0; jj < GB; ++jj) g += d2s[jj][a];
    } else if (q < P_B3) {
      const int a = q - P_W3;
      for (int jj = 0; jj < GB; ++jj) g += d3s[jj] * h2s[jj][a];
    } else {
      for (int jj = 0; jj < GB; ++jj) g += d3s[jj];
    }
    out[q] = g;
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int jj = 0; jj < GB; ++jj) t += ls[jj];
    lpart[blockIdx.x] = t;
  }
}

// grad[q] = sum over blocks (fixed order); loss = sum lpart / N into *loss.
__global__ void k_mlp_reduce(const float *partial, const double *lpart, int nblk, int64_t N,
                             float *grad, double *loss) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < MLP_NPARAMS) {
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += partial[(int64_t)b * MLP_NPARAMS + q];
    grad[q] = g;
  }
  if (q == 0) {
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += lpart[b];
    *loss = t / (double)N;
  }
}

hipError_t mlp_grad(const float *p, const float *mu, const float *sd, const float *X,
                    const float *y, int64_t N, float *partial, double *lpart, float *grad,
                    double *loss, hipStream_t st) {
  if (N <= 0) return hipErrorInvalidValue;
  const int nblk = (int)((N + GB - 1) / GB);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, st, p, mu, sd, X, y, N, partial, lpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, st, partial,
                     lpart, nblk, N, grad, loss);
  return hipGetLastError();
}

// Adam with the step counter kept on the device (so a captured epoch can be
// replayed): t <- t + 1, then the bias-corrected update; hist[t-1] = loss.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int *t, float lr,
                       const double *loss, double *hist) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int step = *t + 1;
  if (q < MLP_NPARAMS) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float mq = b1 * m[q] + (1.0f - b1) * g[q];
    const float vq = b2 * v[q] + (1.0f - b2) * g[q] * g[q];
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.0f - powf(b1, (float)step));
    const float vh = vq / (1.0f - powf(b2, (float)step));
    p[q] -= lr * mh / (sqrtf(vh) + 1e-8f);
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (hist) hist[step - 1] = *loss;
  }
}

// t is advanced by a separate single-thread kernel so that every block of
// k_adam reads the same step.
__global__ void k_adam_tick(int *t) { *t += 1; }

hipError_t mlp_adam(float *p, const float *g, float *m, float *v, int *t, float lr,
                    const double *loss, double *hist, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, st, p, g, m, v, t, lr,
                     loss, hist);
  hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(1), 0, st, t);
  return hipGetLastError();
}

// Column means and standard deviations of X (N x MLP_F, row-major): one
// block per feature, two passes in FP64.
__global__ void k_standardize(const float *X, int64_t N, float *mu, float *sd) {
  const int f = blockIdx.x;
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) s += X[i * MLP_F + f];
  s = block_sum(s, red);
  const double m = s / (double)N;
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double d = X[i * MLP_F + f] - m;
    q += d * d;
  }
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    const double sdv = sqrt(q / (double)N);
    mu[f] = (float)m;
    sd[f] = (float)((sdv > 1e-12) ? sdv : 1.0);
  }
}

hipError_t mlp_standardize(const float *X, int64_t N, float *mu, float *sd, hipStream_t st) {
  if (N <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_standardize, dim3(MLP_F), dim3(256), 0, st, X, N, mu, sd);
  return hipGetLastError();
}

// ------------------------------------------- warm-started subspace iteration
// Chebyshev three-term step on blocks kept transposed (b x n, ld b):
// out <- beta * cur + gamma * prev (then a GEMM adds alpha * cur . C).
__global__ void k_cheb_combine(const ChebJob *jobs) {
  const ChebJob J = jobs[blockIdx.y];
  const int64_t len = (int64_t)J.b * J.n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    J.out[i] = J.beta * J.cur[i] + (J.prev ? J.gamma * J.prev[i] : 0.0);
}

hipError_t cheb_combine(const ChebJob *d_jobs, int njobs, int64_t max_len, hipStream_t s) {
  if (!njobs || max_len <= 0) return hipSuccess;
  const int gx = (int)std::min<int64_t>((max_len + 255) / 256, 256);
  hipLaunchKernelGGL(k_cheb_combine, dim3(gx, njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// Orthonormalise the b rows of Vt (b x n, ld b) in place by classical
// Gram-Schmidt applied twice; a row that vanishes is replaced by a unit
// vector of a coordinate and re-orthogonalised.  One block per face.
__global__ __launch_bounds__(256) void k_orth_rows(const OrthJob *jobs) {
  const OrthJob J = jobs[blockIdx.x];
  __shared__ double red[16];
  double *V = J.Vt;
  const int b = J.b, n = J.n;
  for (int t = 0; t < b; ++t) {
    for (int attempt = 0; attempt < 2; ++attempt) {
      for (int pass = 0; pass < 2; ++pass)
        for (int s = 0; s < t; ++s) {
          double d = 0.0;
          for (int c = threadIdx.x; c < n; c += blockDim.x)
            d += V[s + (int64_t)c * b] * V[t + (int64_t)c * b];
          d = block_sum(d, red);
          for (int c = threadIdx.x; c < n; c += blockDim.x)
            V[t + (int64_t)c * b] -= d * V[s + (int64_t)c * b];
          __syncthreads();
        }
      double q = 0.0;
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const double v = V[t + (int64_t)c * b];
        q += v * v;
      }
      q = block_sum(q, red);
      if (q > 1e-28) {
        const double sc = 1.0 / sqrt(q);
        for (int c = threadIdx.x; c < n; c += blockDim.x) V[t + (int64_t)c * b] *= sc;
        __syncthreads();
        break;
      }
      // degenerate: restart the row as a coordinate vector
      const int pick = (t * 7919 + attempt * 104729) % n;
      for (int c = threadIdx.x; c < n; c += blockDim.x) V[t + (int64_t)c * b] = (c == pick) ? 1.0 : 0.0;
      __syncthreads();
    }
  }
}

hipError_t orth_rows(const OrthJob *d_jobs, int njobs, hipStream_t s) {
  if (!njobs) return hipSuccess;
  hipLaunchKernelGGL(k_orth_rows, dim3(njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

// Ritz vectors and residuals: with U = Vt C (b x n) and the eigenpairs
// (theta_t, Z_H[:, t]) of H = Vt U^T,
//   y_t = V Z_H[:, t]  (written to Y, n x b column-major, and transposed to Vt2),
//   r_t = U^T Z_H[:, t] - theta_t y_t, res[t] = |r_t|.
__global__ __launch_bounds__(256) void k_ritz(const RitzJob *jobs) {
  const RitzJob J = jobs[blockIdx.y];
  const int t = blockIdx.x;
  if (t >= J.b) return;
  __shared__ double red[16];
  __shared__ double zh[64];
  const int b = J.b, n = J.n;
  for (int s = threadIdx.x; s < b; s += blockDim.x) zh[s] = J.ZH[s + (int64_t)t * J.ldzh];
  __syncthreads();
  const double th = J.theta[t];
  double rr = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double y = 0.0, u = 0.0;
    for (int s = 0; s < b; ++s) {
      y += J.Vt[s + (int64_t)c * b] * zh[s];
      u += J.U[s + (int64_t)c * b] * zh[s];
    }
    J.Y[(int64_t)c + (int64_t)t * J.ldy] = y;
    J.Vt2[t + (int64_t)c * b] = y;
    const double r = u - th * y;
    rr += r * r;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) J.res[t] = sqrt(rr);
}

hipError_t ritz(const RitzJob *d_jobs, int njobs, int max_b, hipStream_t s) {
  if (!njobs || !max_b) return hipSuccess;
  hipLaunchKernelGGL(k_ritz, dim3(max_b, njobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

}  // namespace vb
