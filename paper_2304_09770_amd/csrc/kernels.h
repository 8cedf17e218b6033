// Host-callable launchers of the vembddc device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>
#include "common.h"

namespace vb {

// Device timing of individual kernel launches with HIP events on the
// launching stream; `work` is the algorithmic flops or bytes of the launch.
struct KTimer {
  std::vector<hipEvent_t> ev;
  std::vector<double> work;
  int used = 0;
  hipError_t begin(hipStream_t s, double w) {
    if ((int)ev.size() < 2 * (used + 1)) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
      }
    }
    if ((int)work.size() <= used) work.push_back(0.0);
    work[used] = w;
    return hipEventRecord(ev[2 * used], s);
  }
  hipError_t end(hipStream_t s) { return hipEventRecord(ev[2 * used++ + 1], s); }
  hipError_t collect(int *n, double *ms, double *w) {
    *n = used;
    *ms = 0.0;
    *w = 0.0;
    for (int i = 0; i < used; ++i) {
      float t = 0.f;
      hipError_t r = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
      if (r != hipSuccess) return r;
      *ms += t;
      *w += work[i];
    }
    return hipSuccess;
  }
  void reset() { used = 0; }
  void destroy() {
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.clear();
    used = 0;
  }
};

// ---------------------------------------------------------------- dense
// nb: panel width (32 or 64); sb1: columns of an outer super-panel, whose
// trailing update is one rank-sb1 product (a multiple of 4 nb; 0 = 16 nb);
// hz: the jobs' zrow (with hn, it sizes the grids of identity-bordered jobs
// to the rows each step can change; without it, grids span max_n)
template <typename T>
hipError_t ldl_batched(const LdlJob<T> *d_jobs, int batch, int max_n, int max_e, int nb,
                       hipStream_t s, KTimer *timer = nullptr,
                       const std::vector<int> *hn = nullptr, const std::vector<int> *he = nullptr,
                       bool dirichlet = false, bool aligned16 = false, int sb1 = 0,
                       const std::vector<int> *hz = nullptr);
template <typename T>
hipError_t gemm_nt_batched(const GemmJob<T> *d_jobs, int batch, int max_m, int max_n,
                           hipStream_t s);

// ---------------------------------------------------------------- setup
// Per-subdomain description shared by the setup and recovery kernels.
struct SubDev {
  void *W;          // dense local matrix (double or float), column-major, ld
  int64_t ld;
  void *X;          // condensed bordered interface block (ng+1)^2: inside W, or a
  int64_t xld;      // compact copy when the local matrices are processed in waves
  int nv, nel, ng;  // interior velocity, element pressures, interface DoFs
  int N;            // nv + nel + ng + 1 (last row/col: right-hand side)
  int e;            // eliminated columns = nv + nel - 1
  int n_csr;        // local CSR size
  const int64_t *indptr;
  const int32_t *indices;
  const double *vals;
  const double *rhs;
  const int32_t *pos;     // dense position of every CSR DoF
  const double *pweight;  // element volumes (length nel, dense pressure order)
  double *hv;             // Householder vector (nel) ; hv[nel] = tau
  double *b0;             // ng + 1: flux row over the interface (+ p0 right-hand side)
  const int64_t *gidl;    // ng: global interface id of each local interface DoF
  int n_ent;              // entities touching the subdomain
  const int32_t *ent;     // [n_ent] entity ids
  const int32_t *ent_off; // [n_ent] local offset of each entity block
  const int32_t *oidx;    // null, or per CSR row its row in the subdomain's full CSR
                          // (-1: none); the local residual is read through it
};

// One front of the two-level factorisation: its trailing block [kept | B |
// rhs] (m rows from row e of the front matrix) and where those rows sit in
// its subdomain's second-level matrix and vectors.
struct FrontJob {
  const void *Wf;       // front matrix (double, or float in mixed precision)
  int64_t ldf;
  int e, m;
  void *W2;             // second-level matrix of the subdomain
  int64_t ld2;
  const int32_t *map;   // m second-level dense positions
  double gamma;         // kept coordinate -> sub-box constant pressure
  const double *yf;     // front residual (dense order), for front_rhs
  double *y2;           // second-level residual (dense order)
};
hipError_t front_scatter(const FrontJob *d_jobs, int njobs, int max_m, bool fp32, hipStream_t s);
hipError_t front_rhs(const FrontJob *d_jobs, int njobs, hipStream_t s);
hipError_t l2_residual(const SubDev *d_subs, const double *R, const int64_t *roff, double *y,
                       const int64_t *yoff, int nsub, hipStream_t s);
hipError_t segment_sum(int n, const int32_t *first, const double *in, double *out, hipStream_t s);

struct EntDev {
  int n;          // DoFs
  int n_con;      // constraint rows
  const double *con;  // row-major n_con x n
  const int64_t *gids;
  double *V;      // n x rmax Householder vectors (column-major, ld n)
  double *tau;    // rmax
  int *rank;      // selected primal count
  double *work;   // n x n_con scratch
};

struct DiagJob {
  void *A;  // double, or float if f32
  int64_t ld;
  int r0, c0, cnt;
  double val;
  int f32;
};
hipError_t set_diag(const DiagJob *d_jobs, int batch, int max_cnt, hipStream_t s);
hipError_t diag_gather(const double *A, int64_t ld, int n, double *out, hipStream_t s);

struct CoarseSub {
  const double *SPi;   // npi x npi (full), leading dimension ld
  int64_t ld;
  int npi;
  const int32_t *cidx; // coarse index of each local primal coordinate
  const int32_t *pl;   // local interface index of each local primal coordinate
  const double *b0;    // transformed flux row (local interface order)
};
hipError_t coarse_assemble(const CoarseSub *d_cs, int nsub, double *K, int64_t ld, int nC,
                           const double *w, hipStream_t s);

// fp32: the dense local matrices W are float (mixed precision), else double
hipError_t densify(const SubDev *d_subs, int nsub, int max_rows, bool fp32, hipStream_t s);
// dst[i] = src[i] rounded to FP32, i < n
hipError_t cast_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
hipError_t flux_rows(const SubDev *d_subs, int nsub, int max_rows, hipStream_t s);
hipError_t house_pressure(const SubDev *d_subs, int nsub, int max_N, bool fp32, hipStream_t s);
hipError_t entity_qr(const EntDev *d_ents, int nent, int rmax, double tol, hipStream_t s);
hipError_t symmetrize(void *const *mats, const int64_t *lds, const int32_t *ns, int batch,
                      int max_n, bool fp32, hipStream_t s);
hipError_t transpose_sq(void *const *mats, const int64_t *lds, const int32_t *ns, int batch,
                        int max_n, bool fp32, hipStream_t s);
// T^T X per entity block from the left (contiguous column segments); *done
// false when an entity is too large for it (the caller then uses apply_T_cols
// on the transposed block).  max_rn: the largest min(n_con, n) * n over the
// entities, max_rank the largest min(n_con, n).
hipError_t apply_T_rows(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ng, int max_ent,
                        int max_en, int max_rn, int max_rank, bool fp32, bool *done, hipStream_t s);
hipError_t apply_T_cols(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ng,
                        int max_ent, int max_en, bool fp32, hipStream_t s);
hipError_t transform_b0(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ent,
                        hipStream_t s);
// global vector <-> transformed coordinates (dir = +1: x~ = T^T x, -1: x = T x~)
hipError_t transform_vec(const EntDev *d_ents, int nent, double *x, int dir, hipStream_t s);

// gather / scatter of dense sub-blocks by index lists:
// out_b[i + j*ldo] = in_b[ri[i] + ci[j]*ldi] (ri/ci < 0 -> value (ri==ci? diag : 0))
struct GatherJob {
  const void *in;  // double, or float if in_f32
  int64_t ldi;
  void *out;       // double, or float if out_f32
  int64_t ldo;
  const int32_t *ri;
  const int32_t *ci;
  int m, n;
  double scale;
  int add;  // accumulate into out
  int in_f32, out_f32;
};
hipError_t gather_blocks(const GatherJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s);

// ---------------------------------------------------------------- recovery
hipError_t recover_rhs(const SubDev *d_subs, const double *x_orig, double *y, const int64_t *yoff,
                       int nsub, int max_e, bool fp32, hipStream_t s);
// invL: double or float (fp32) inverse diagonal blocks of the factorisation
hipError_t recover_backsolve(const SubDev *d_subs, const void *invL, const int64_t *invoff,
                             double *y, double *z, const int64_t *yoff, int nsub, int i0, int nb,
                             bool fp32, hipStream_t s);

// ---- mixed-precision refinement (FP64 residuals, FP32 factors)
// R = f - K u for every subdomain's local system (CSR order, FP64)
hipError_t local_residual(const SubDev *d_subs, const double *u, const int64_t *uoff, double *R,
                          int nsub, int max_rows, hipStream_t s);
// y (dense order, length N-1) from R: permutation + pressure reflector;
// r0[s] = sum of the pressure residuals (the p0 equation)
hipError_t residual_to_dense(const SubDev *d_subs, const double *R, const int64_t *roff,
                             double *y, const int64_t *yoff, double *r0, int nsub, int max_rows,
                             hipStream_t s);
// forward substitution step for the block [i0, i0+nb): z_i = inv(L_ii) y_i,
// y_r -= L[r, i-block] z_i for r in [i0+b, N-1)
hipError_t forward_step(const SubDev *d_subs, const void *invL, const int64_t *invoff, double *y,
                        double *z, const int64_t *yoff, int nsub, int i0, int nb, int max_N,
                        bool fp32, hipStream_t s);
// back-substitution right-hand side: y2_j = d_j z_j - sum_l L[e+1+l, j] dx[gid_l]
hipError_t back_init(const SubDev *d_subs, const double *z, double *y2, const int64_t *yoff, int nsub,
                     int max_e, hipStream_t s);
// ---- adaptive face eigenproblems (dense symmetric eigen-solver pieces)
struct EigJob {
  double *A;      // n x n full symmetric (column-major); reflectors stored below the subdiagonal
  int64_t ld;
  int n;
  int ncols;      // eigenvectors to back-transform
  double *d, *e, *tau;  // tridiagonal diagonal, off-diagonal, reflector factors (length n)
  double *Z;      // n x mcap eigenvectors
  int64_t ldz;
  double *lam;    // mcap eigenvalues below sigma, ascending
  int *count;     // number of eigenvalues below sigma
  double sigma;
};
struct RowJob {
  const double *L;  // n x n lower triangular
  int64_t ld;
  int n, ncols;
  const double *Z;
  int64_t ldz;
  double *R;
  int64_t ldr;
};
struct FaceTJob {
  double *A;      // rows [off, off + n_E) of columns [0, ncols)
  int64_t ld;
  int ncols, off;
  const EntDev *ent;
  int dir;        // +1: T_E^T, -1: T_E
};
struct SymJob {
  double *A;
  int64_t ld;
  int n;
};
hipError_t tridiag(const EigJob *d_jobs, int njobs, int max_n, hipStream_t s);
hipError_t tridiag_eig(const EigJob *d_jobs, int njobs, int max_n, int mcap, hipStream_t s);
hipError_t back_transform(const EigJob *d_jobs, int njobs, hipStream_t s);
hipError_t lower_times(const RowJob *d_jobs, int njobs, int max_n, int max_cols, hipStream_t s);
hipError_t face_transform(const FaceTJob *d_jobs, int njobs, int max_cols, hipStream_t s);
hipError_t sym_average(const SymJob *d_jobs, int njobs, int max_n, hipStream_t s);
hipError_t shift_diag(const SymJob *d_jobs, int njobs, double rel, hipStream_t s);
hipError_t normalize_cols(const RowJob *d_jobs, int njobs, int max_cols, hipStream_t s);

// ---- learned predictor of the adaptive constraints (network F -> H -> H -> 1)
constexpr int MLP_F = 12;
constexpr int MLP_H = 32;
constexpr int MLP_NPARAMS = MLP_H * MLP_F + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;
struct FeatJob {
  const double *C;    // n x n reduced pencil matrix (full symmetric)
  int64_t ld;
  int n;
  double sigma;
  const double *trp;  // [tr At_par, tr B]
  const double *tra;  // [tr(A_i + A_j), tr A_j]
  float *X;           // n x MLP_F features (row-major)
  double *rho;        // Gershgorin bound of C
};
struct LabelJob {
  const double *Z;    // n x m eigenvectors of C
  int64_t ldz;
  int n, m, full;
  float *y;
};
struct ChebJob {
  const double *cur, *prev;
  double *out;
  int b, n;
  double beta, gamma;
};
struct OrthJob {
  double *Vt;  // b x n (ld b)
  int b, n;
};
struct RitzJob {
  const double *Vt, *U;  // b x n (ld b)
  const double *ZH;      // b x b eigenvectors of H
  int64_t ldzh;
  const double *theta;
  int b, n;
  double *Y;             // n x b
  int64_t ldy;
  double *Vt2;           // b x n: the Ritz vectors, transposed
  double *res;
};
hipError_t face_features(const FeatJob *d_jobs, int njobs, hipStream_t s);
hipError_t traces(const SymJob *d_jobs, int njobs, double *out, hipStream_t s);
hipError_t face_labels(const LabelJob *d_jobs, int njobs, hipStream_t s);
hipError_t mlp_forward(const float *p, const float *mu, const float *sd, const float *X, int64_t N,
                       float *s, hipStream_t st);
hipError_t mlp_grad(const float *p, const float *mu, const float *sd, const float *X,
                    const float *y, int64_t N, float *partial, double *lpart, float *grad,
                    double *loss, hipStream_t st);
hipError_t mlp_adam(float *p, const float *g, float *m, float *v, int *t, float lr,
                    const double *loss, double *hist, hipStream_t st);
hipError_t mlp_standardize(const float *X, int64_t N, float *mu, float *sd, hipStream_t st);
hipError_t cheb_combine(const ChebJob *d_jobs, int njobs, int64_t max_len, hipStream_t s);
hipError_t orth_rows(const OrthJob *d_jobs, int njobs, hipStream_t s);
hipError_t ritz(const RitzJob *d_jobs, int njobs, int max_b, hipStream_t s);

}  // namespace vb
