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
template <typename T>
hipError_t ldl_batched(const LdlJob<T> *d_jobs, int batch, int max_n, int max_e, int nb,
                       hipStream_t s, KTimer *timer = nullptr,
                       const std::vector<int> *hn = nullptr, const std::vector<int> *he = nullptr);
template <typename T>
hipError_t gemm_nt_batched(const GemmJob<T> *d_jobs, int batch, int max_m, int max_n,
                           hipStream_t s);

// ---------------------------------------------------------------- setup
// Per-subdomain description shared by the setup and recovery kernels.
struct SubDev {
  double *W;        // dense local matrix, column-major, ld
  int64_t ld;
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
};

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
  double *A;
  int64_t ld;
  int r0, c0, cnt;
  double val;
};
hipError_t set_diag(const DiagJob *d_jobs, int batch, int max_cnt, hipStream_t s);

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

hipError_t densify(const SubDev *d_subs, int nsub, int max_rows, hipStream_t s);
hipError_t flux_rows(const SubDev *d_subs, int nsub, int max_ng, hipStream_t s);
hipError_t house_pressure(const SubDev *d_subs, int nsub, int max_N, hipStream_t s);
hipError_t entity_qr(const EntDev *d_ents, int nent, int rmax, double tol, hipStream_t s);
hipError_t symmetrize(double *const *mats, const int64_t *lds, const int32_t *ns, int batch,
                      int max_n, hipStream_t s);
hipError_t transpose_sq(double *const *mats, const int64_t *lds, const int32_t *ns, int batch,
                        int max_n, hipStream_t s);
hipError_t apply_T_cols(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ng,
                        int max_ent, hipStream_t s);
hipError_t transform_b0(const SubDev *d_subs, const EntDev *d_ents, int nsub, int max_ent,
                        hipStream_t s);
// global vector <-> transformed coordinates (dir = +1: x~ = T^T x, -1: x = T x~)
hipError_t transform_vec(const EntDev *d_ents, int nent, double *x, int dir, hipStream_t s);

// gather / scatter of dense sub-blocks by index lists:
// out_b[i + j*ldo] = in_b[ri[i] + ci[j]*ldi] (ri/ci < 0 -> value (ri==ci? diag : 0))
struct GatherJob {
  const double *in;
  int64_t ldi;
  double *out;
  int64_t ldo;
  const int32_t *ri;
  const int32_t *ci;
  int m, n;
  double scale;
  int add;  // accumulate into out
};
hipError_t gather_blocks(const GatherJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s);

// ---------------------------------------------------------------- recovery
hipError_t recover_rhs(const SubDev *d_subs, const double *x_orig, double *y, const int64_t *yoff,
                       int nsub, int max_e, hipStream_t s);
hipError_t recover_backsolve(const SubDev *d_subs, const double *invL, const int64_t *invoff,
                             double *y, double *z, const int64_t *yoff, int nsub, int i0, int nb,
                             hipStream_t s);

}  // namespace vb
