// Per-iteration kernel launchers and job descriptors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vb {

// Per-problem PCG scalars: SC_STRIDE doubles per problem.
enum {
  SC_RZ = 0, SC_PQ, SC_ALPHA, SC_BETA, SC_RR, SC_GG, SC_FLAG, SC_TMP,
  SC_DONE,    // 1 once converged, stopped at maxit or broken down
  SC_ACTIVE,  // 1 if the problem took part in the current iteration
  SC_IT,      // iterations taken
  SC_TOL,     // relative tolerance on ||r|| / ||b||
  SC_MAXIT,
  SC_T0,      // device clock at the start of the solve
  SC_TDONE,   // device clock when SC_DONE was set
  SC_COUNT
};
constexpr int SC_STRIDE = 16;
static_assert(SC_COUNT <= SC_STRIDE, "scalar slots");
constexpr int DOT_BLOCKS = 512;

// A problem's entries of the global interface vector: [a0, a0+n0) then [a1, a1+n1).
struct Seg {
  int64_t a0, n0, a1, n1;
};

struct GemvJob {
  const void *A;       // double, or float if a_f32 (FP32 storage, FP64 accumulation)
  int64_t lda;
  int m, n;            // A is m x n
  const double *x;     // gathered through xidx when given
  const int64_t *xidx;
  const double *base;  // gemv_n: y = base + A x
  double *y;
  double alpha;        // gemv_t: y = alpha A^T x (+ y if acc)
  int acc;
  int a_f32;
  double *y2;          // gemv_t, square A, no acc: y2[j] = x_j - y[j] (x_j gathered like
                       // the rows), the complement (I - A)^T x of the same product
};

// y = alpha A x (+ y if acc) for a symmetric A (n x n, column-major) read
// through its lower triangle only, in SYMV_T x SYMV_T tiles: each tile adds
// its rows' and (off the diagonal) its columns' contributions to `part`
// (SYMV_T row sums, then SYMV_T column sums, per tile), which a second pass
// reduces in a fixed order.
constexpr int SYMV_T = 256;
struct SymvJob {
  const void *A;       // double, or float if a_f32
  int64_t lda;
  int n, a_f32;
  const double *x;
  const int64_t *xidx;
  double *y;
  double alpha;
  int acc;
  double *part;        // symv_tiles(n) * 2 * SYMV_T doubles
};
__host__ __device__ inline int symv_tiles(int n) {
  const int T = (n + SYMV_T - 1) / SYMV_T;
  return T * (T + 1) / 2;
}
hipError_t symv(const SymvJob *d_jobs, int batch, int max_n, hipStream_t s);

struct ExtPart {
  const void *D;    // m x m column-major, double or float if f32 (null: counting weight `scale`)
  int64_t ld;
  int64_t woff;     // offset of this subdomain's entity block in w
  double scale;
  int f32;
};
struct ExtJob {
  int m;
  int nparts;
  int part0;
  const int64_t *gids;  // m global positions
  int pair;             // two parts whose matrices sum to I: only the first one's D is
                        // read, z = w_2 + D_1 (w_1 - w_2)
};

struct RecJob {
  int sub, n, nv, nel;
  const int32_t *kind;
  const int32_t *pos;
  const int64_t *gid;
  const double *hv;
  const double *z;   // interior solution in dense order
  double *out;
  const int32_t *oidx;  // null, or per CSR DoF its index in out (-1: not written)
  double *sep_out;      // null, or receives z at the dense positions of the kind-0 DoFs
  double *c_out;        // null, or receives the nel pressure values (rows need not be CSR DoFs)
};

hipError_t gemv_t(const GemvJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s);
hipError_t gemv_t_cpb(const GemvJob *d_jobs, int batch, int max_m, int max_n, int cpb,
                      hipStream_t s);
hipError_t gemv_n(const GemvJob *d_jobs, int batch, int max_m, int max_n, hipStream_t s);
hipError_t owner_sum(int n, const int64_t *ptr, const int64_t *idx, const double *src,
                     const int64_t *bidx, const double *bsrc, double *y, hipStream_t s);
hipError_t scatter_copy(int n, const double *src, const int64_t *sidx, const int64_t *dst,
                        double *y, double scale, hipStream_t s);
hipError_t extend(const ExtJob *d_jobs, int njobs, int max_m, const ExtPart *d_parts,
                  const double *w, double *z, hipStream_t s);
hipError_t dot(int64_t n, const double *a, const double *b, double *part, double *sc, int mode,
               int it, double *hist_a, double *hist_b, hipStream_t s);
hipError_t update_xr(int64_t n, const double *sc, double *x, double *r, const double *p,
                     const double *q, double *part, double *scw, hipStream_t s);
hipError_t update_p(int64_t n, const double *sc, double *p, const double *z, hipStream_t s);
hipError_t vsub(int64_t n, const double *a, const double *b, double *y, hipStream_t s);
hipError_t axpy(int64_t n, double a, const double *x, double *y, hipStream_t s);

// ---- PCG over several independent problems (segments), scalars per problem.
// mode 0: PQ, alpha (0 when done), history;  1: RR after the update, iteration
// count, convergence / maxit;  2: beta, RZ, history;  3: RZ;  4: GG;  5: TMP;
// 6: RR at the start with the initial convergence test.
hipError_t sdot(const Seg *segs, int P, int G, const double *a, const double *b, double *part,
                double *sc, int mode, double *hist_a, double *hist_b, int hist_ld, hipStream_t s);
hipError_t supdate_xr(const Seg *segs, int P, int G, double *sc, double *x, double *r,
                      const double *p, const double *q, double *part, hipStream_t s);
hipError_t supdate_p(const Seg *segs, int P, int G, const double *sc, double *p, const double *z,
                     hipStream_t s);
// per-problem scalar initialisation: zero, TOL = tol[p], MAXIT, T0 = device clock
hipError_t sinit(int P, const double *tol, int maxit, double *sc, hipStream_t s);
hipError_t recover_out(const RecJob *d_jobs, int nsub, const double *x_orig, int64_t nG,
                       hipStream_t s);

// ---- the whole PCG iteration loop in one persistent cooperative launch
// One GEMV launch of the iteration: its jobs, batch, grid width and columns
// per workgroup (the autotuned tile).
struct GemvPhase {
  const GemvJob *jobs;
  int batch, gx, cpb;
};
// Everything one iteration (S~ p, M~^-1 r, recurrences, as launched one by
// one in the graph-replayed iteration) reads and writes.
struct PcgPlan {
  GemvPhase schur, restrict_, neu1, coarse, neu2;  // neu2: gemv_n (batch 0: none)
  const SymvJob *ssym;  // non-null: S~ p by the symmetric kernel (schur unused)
  int ssym_batch, ssym_tiles, ssym_rows;
  const SymvJob *nsym;  // non-null: the S_DD^-1 block of neu1 by the symmetric kernel and
  int nsym_batch, nsym_tiles, nsym_rows;  // its Phi block by nphi (neu1 unused)
  GemvPhase nphi;
  const ExtJob *ext;
  const ExtPart *extpart;
  int n_ext, ext_gx;
  const double *wv;
  int n_own;
  const int64_t *own_ptr, *own_idx;
  const double *yloc;
  int n_cs;
  const int64_t *c_ptr, *c_idx, *c_base;
  const double *tv;
  double *rc;
  const double *uc;
  const int64_t *uc_dst;
  const Seg *segs;
  int P, G;
  double *part, *sc, *hist_a, *hist_b;
  int hist_ld;
  double *x, *r, *p, *q, *z;
  unsigned *bar;     // 2 words: arrivals, generation (zero before the launch)
  int *err;          // set to 1 if a grid barrier timed out
  int max_iter;      // iterations at most (every problem stops at its maxit before)
};
// Blocks of the persistent launch (co-resident: occupancy x CUs, at most
// `per_cu` per CU); 0 if cooperative launches are not available.
int pcg_persistent_blocks(int per_cu);
hipError_t pcg_persistent(const PcgPlan *d_plan, int nblocks, hipStream_t s);

}  // namespace vb
