// vembddc runtime: the C-ABI of include/vembddc.h.
//
// Host code only orchestrates: index bookkeeping of the caller's data
// (interface numbering, entity membership, offsets) and kernel launches.
// Every arithmetic step of setup, preconditioner, PCG and recovery runs in
// the HIP kernels of dense.hip, setup.hip and iterate.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/vembddc.h"
#include "common.h"
#include "iterate.h"
#include "kernels.h"

using namespace vb;

namespace {

constexpr int NB = 64;  // panel width of the dense factorisations

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct SubH {
  int n = 0;
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  std::vector<double> vals, rhs;
  std::vector<int32_t> kind;
  std::vector<int64_t> gid;
  int nv = 0, nel = 0, ng = 0, N = 0, e = 0;
  int64_t ld = 0;
  std::vector<int32_t> pos;
  std::vector<double> pw;       // element volumes in dense pressure order
  std::vector<int64_t> gidl;    // local interface index -> global id
  std::vector<int32_t> ents, ent_off;
  double vol = 0.0;
  // filled in setup
  std::vector<int32_t> pl, dl, cidx;
  std::vector<int64_t> doff;    // per local entity: offset of its dual block in the local dual vector
  int npi = 0, ndl = 0;
  // device
  int64_t W_off = 0, inv_off = 0, b0_off = 0, hv_off = 0, y_off = 0;
  void *X = nullptr;            // condensed block (ng+1)^2 of W, or its compact copy
  int64_t xld = 0, X_off = 0;
  int64_t *d_indptr = nullptr;
  int32_t *d_indices = nullptr, *d_pos = nullptr, *d_kind = nullptr;
  double *d_vals = nullptr, *d_rhs = nullptr, *d_pw = nullptr;
  int64_t *d_gidl = nullptr, *d_gid = nullptr;
  int32_t *d_ents = nullptr, *d_entoff = nullptr;
  void *Nmat = nullptr;         // augmented Neumann matrix (FP32 in mixed precision)
  int64_t Nld = 0;
  int Nn = 0;
  void *G1 = nullptr;           // [S_DD^-1 | Phi] (FP32 in mixed precision)
  double *Spi = nullptr;        // local coarse block S_Pi (npi x npi), setup scope
  // two-level nested dissection (sub-box labels given): the fields above
  // describe the second level (CSR over the separator and interface DoFs,
  // "pressures" = the sub-box constants); n stays the full local size
  std::vector<int32_t> part;    // sub-box labels as given (empty: none)
  int n2 = 0;                   // CSR rows of the fields above (= n without the split)
  int nsep = 0, nbox = 0;
  int first_front = 0;          // fronts [first_front, first_front + nbox)
  std::vector<int32_t> oidx;    // second-level CSR row -> full CSR row
  int32_t *d_oidx = nullptr;
  // the full local CSR (flux rows and local residuals) and its single-level
  // dense positions
  int f_nv = 0, f_nel = 0;
  std::vector<int64_t> f_indptr;
  std::vector<int32_t> f_indices, f_pos;
  std::vector<double> f_vals, f_rhs;
  int64_t *d_f_indptr = nullptr;
  int32_t *d_f_indices = nullptr, *d_f_pos = nullptr;
  double *d_f_vals = nullptr, *d_f_rhs = nullptr;
  int64_t sep_off = 0;          // its separator values in the second-level vector
};

// A front of the two-level factorisation: one sub-box of a subdomain, with
// the SubH fields describing its dense matrix [interior velocity | element
// pressures | B (separator and interface DoFs it couples to) | rhs].
struct FrontH {
  SubH S;
  int sub = 0, box = 0;
  std::vector<int32_t> oidx;    // front CSR row -> full CSR row of its subdomain (-1: B rows)
  std::vector<int32_t> map;     // second-level dense positions of [kept | B | rhs]
  std::vector<int32_t> bsep;    // per B DoF: separator index, or -1 (interface DoF)
  std::vector<int64_t> bgid;    // per B DoF: global interface id (interface DoFs)
  double gamma = 1.0;           // kept coordinate -> sub-box constant pressure
  int32_t *d_oidx = nullptr, *d_map = nullptr;
};

struct EntH {
  int kind = 0, n = 0, ncon = 0;
  std::vector<int64_t> gids;
  std::vector<double> con;
  std::vector<int> subs;  // subdomains sharing the entity (ascending)
  int rank = 0;
  int64_t *d_gids = nullptr;
  double *d_con = nullptr, *d_V = nullptr, *d_tau = nullptr, *d_work = nullptr;
  int *d_rank = nullptr;
  // the given constraints (a setup may append adaptive rows to a copy)
  int ncon0 = 0;
  std::vector<double> con0;
  double *d_con0 = nullptr, *d_V0 = nullptr, *d_tau0 = nullptr, *d_work0 = nullptr;
  // deluxe
  double *Daug = nullptr;
  int64_t Dld = 0;
  std::vector<double *> D;  // per sharing subdomain (null: I - D[0] for a pair)
  std::vector<const void *> Dit;  // the copies the iteration reads (FP32 in mixed precision)
  int64_t Dmld = 0;         // leading dimension of the D matrices (even)
  std::vector<double *> Sbar;
  int64_t *d_dual_gids = nullptr;
};

}  // namespace

struct vb_ctx {
  vb_options opt{};
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;  // 0 created, 1 assembled, 2 set up
  std::vector<void *> allocs;        // assemble scope (until destroy)
  std::vector<void *> setup_allocs;  // setup scratch (back to the pool when setup ends)
  std::vector<void *> setup_keep;    // setup results (freed by the next setup)
  int cur_scope = 0;                 // 0: allocs, 2: setup_keep
  KTimer t_ldl, t_gemv;              // per-launch device timing of the dominant kernels

  int64_t nG = 0;
  int nS = 0;
  std::vector<SubH> subs;
  std::vector<EntH> ents;
  int max_n_csr = 0, max_N = 0, max_e = 0, max_ng = 0, max_ent = 0;
  int max_n_full = 0;  // largest full local CSR
  // two-level nested dissection of every subdomain (sub-box labels given)
  bool nd = false, nd_any = false, nd_none = true;
  std::vector<FrontH> fronts;
  int max_nf_csr = 0, max_Nf = 0, max_ef = 0, max_nbox = 0, max_fm = 0;
  void *FW = nullptr, *invLf = nullptr;  // front matrices and inverse diagonal blocks
  SubDev *d_frdev = nullptr, *d_fulldev = nullptr;
  std::vector<SubDev> frdev, fulldev;
  int *info_f = nullptr;
  double *hvf = nullptr;
  double *G2 = nullptr, *G2d = nullptr;  // [interface vector | separator values | sub-box constants]
  int64_t n_sep_tot = 0, g2_c0 = 0, n_g2 = 0;
  int32_t *d_fr_first = nullptr;         // per subdomain: first front (nS + 1)
  std::vector<std::vector<FrontJob>> fj_scatter;  // per box index: that box's front of every subdomain
  std::vector<FrontJob *> d_fj_scatter;
  int64_t *d_yofff = nullptr, *d_invofff = nullptr, *d_yoff2f = nullptr, *d_roff_f = nullptr;
  RecJob *j_recf = nullptr, *j_rec_irf = nullptr;
  double *r0f = nullptr;
  int64_t n_ir2 = 0;                     // second-level part of y_ir / z_ir / zst
  int64_t *sep_src = nullptr, *sep_dst = nullptr;  // separator corrections -> G2d
  // the interior correction's interface term -L_GammaI^T dx as GEMVs over the
  // FP32 factors' interface rows (second level from dx, fronts from G2d)
  GemvJob *j_brhs = nullptr, *j_brhsf = nullptr;
  int brhs_m = 0, brhs_mf = 0;
  std::vector<std::vector<FrontJob>> fj_rhs;
  std::vector<FrontJob *> d_fj_rhs;

  // device buffers
  bool fp32 = false;      // mixed precision: FP32 local Dirichlet factors
  size_t wsz = 8;         // bytes per entry of W and invL
  void *W = nullptr;
  void *invL = nullptr;
  // dense local matrices: one wave holding every subdomain, or (FP64 beyond
  // the memory limit) waves of consecutive subdomains sharing W, with the
  // condensed blocks copied to Xc and the factors recomputed for recovery
  bool stream_w = false;
  std::vector<std::pair<int, int>> waves;
  int w_wave = -1;  // the wave whose factors W holds (several waves), or -1
  void *Xc = nullptr;
  double *b0 = nullptr, *hv = nullptr;
  int *info = nullptr;
  SubDev *d_subdev = nullptr;
  EntDev *d_entdev = nullptr;
  std::vector<SubDev> subdev;
  std::vector<EntDev> entdev, entdev0;
  // independent problems assembled into this context (appended by vb_assemble)
  struct Prob {
    int64_t g0 = 0, ng = 0;  // interface ids [g0, g0 + ng)
    int s0 = 0, ns = 0;      // subdomains [s0, s0 + ns); p0 entries at nG + s
    int e0 = 0, ne = 0;      // entities [e0, e0 + ne)
    int cbase = 0, nprim = 0;  // coarse block [cbase, cbase + nprim + ns)
  };
  std::vector<Prob> probs;
  bool finalized = false;
  Seg *d_segs = nullptr;
  int seg_G = 1;
  double *d_tol = nullptr;
  int max_ncs = 0;
  std::vector<int32_t> ent_cbase, sub_cp0;
  std::vector<int64_t> gc_off;  // per problem: offset of its coarse inverse in Gc
  hipGraph_t it_graph = nullptr;
  hipGraphExec_t it_exec = nullptr;
  // the persistent launch of the PCG iterations: its plan (rebuilt after each
  // setup), barrier words and error flag, and the resident block count
  PcgPlan plan_h{};
  PcgPlan *d_plan = nullptr;
  unsigned *d_pbar = nullptr;  // [arrivals, generation, error flag, spare]
  bool plan_valid = false;
  int pnb = -1;                // blocks of the persistent launch (0: unavailable)
  int last_launch = 0;         // VB_PCG_GRAPH or VB_PCG_PERSISTENT, last pcg_core
  std::vector<vb_solve_info> pinfo;  // per problem, last solve
  // autotuned columns per workgroup of the per-iteration GEMVs:
  // 0 S_hat p, 1 Neumann, 2 deluxe restriction, 3 coarse (0 = not tuned yet)
  int cpb[4] = {0, 0, 0, 0};
  // factorisation classes (0: local Dirichlet or its fronts, 1: second
  // level, 2: local Neumann): panel width and outer super-panel, 0 = not yet
  // chosen
  int fac_nb[3] = {0, 0, 0}, fac_sb[3] = {0, 0, 0};
  double clock_khz = 0.0;
  // adaptive coarse space of the last setup
  std::vector<vb_face_info> face_info;
  std::vector<double> face_eigs;
  float *d_feat = nullptr, *d_lab = nullptr;  // per face coordinate (faces solved exactly)
  int64_t n_coord = 0;

  // iteration structures
  int nC = 0, nCS = 0;
  double *Kaug = nullptr, *Gc = nullptr;
  int64_t Kld = 0;
  double *g = nullptr;  // transformed right-hand side (global layout)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *tmp = nullptr;
  double *yloc = nullptr, *gD = nullptr, *wv = nullptr, *tv = nullptr, *rc = nullptr, *uc = nullptr;
  double *sc = nullptr, *part = nullptr, *hist_a = nullptr, *hist_b = nullptr;
  GemvJob *j_schur = nullptr, *j_restrict = nullptr, *j_neu1 = nullptr, *j_coarse = nullptr,
          *j_neu2 = nullptr;
  int n_restrict = 0, max_rm = 0;
  ExtJob *j_ext = nullptr;
  ExtPart *j_extpart = nullptr;
  int n_ext = 0, max_ext_m = 0;
  int64_t *own_ptr = nullptr, *own_idx = nullptr;        // S_hat assembly
  int64_t *g_ptr = nullptr, *g_idx = nullptr;            // g~ assembly (offsets into W)
  int64_t *c_ptr = nullptr, *c_idx = nullptr, *c_base = nullptr;  // coarse rhs
  int64_t *uc_dst = nullptr;                             // primal/p0 positions of uc
  int64_t *p0_src = nullptr, *p0_dst = nullptr;
  int max_gt_m = 0, max_gt_n = 0, max_ndl = 0, max_npi = 0, max_nt = 0;
  int64_t n_yloc = 0, n_gD = 0, n_tv = 0;
  double schur_bytes = 0.0;  // algorithmic bytes of one S~ GEMV launch
  // S~ p through the lower triangle only (chosen by the autotuner when faster)
  SymvJob *j_ssym = nullptr;
  bool ssym_on = false;
  SymvJob *j_nsym = nullptr;  // the S_DD^-1 blocks of the Neumann operators, lower triangle
  GemvJob *j_nphi = nullptr;  // their Phi blocks
  bool nsym_on = false;
  std::vector<int> fp64_retried;  // subdomains whose Dirichlet factorisation was redone in FP64
  double schur_bytes_full = 0.0, schur_bytes_sym = 0.0;
  // recovery
  double *yrec = nullptr, *zrec = nullptr, *rec_out = nullptr;
  int64_t *d_yoff = nullptr, *d_invoff = nullptr;
  RecJob *j_rec = nullptr;
  std::vector<int64_t> rec_off;
  // mixed-precision refinement buffers
  double *u_loc = nullptr, *R_loc = nullptr, *y_ir = nullptr, *z_ir = nullptr, *r0 = nullptr;
  double *dgv = nullptr, *dx = nullptr, *zst = nullptr;
  int64_t *d_uoff = nullptr, *d_yoff2 = nullptr;
  int64_t *ir_ptr = nullptr, *ir_idx = nullptr;  // condensed residual assembly (offsets in y_ir)
  RecJob *j_rec_ir = nullptr;                    // local vector from (zst, x)
  int64_t n_ir = 0;                              // length of y_ir / z_ir / zst
  std::vector<int64_t> uoff;
  int last_outer = 0, last_inner = 0;
  // per problem: the relative condensed residual before each refinement step
  // (and after the last) and the inner iterations of each step
  std::vector<std::vector<double>> ref_rel;
  std::vector<std::vector<int>> ref_inner;
  int recover_steps = 4;  // interior refinement passes of vb_recover_all (mixed)
  // the interface solution of the last mixed solve, whose interior state zst
  // was refined with it: recovery at that x starts from zst
  double *x_last = nullptr;
  bool zst_valid = false;
  // y_ir, z_ir and r0 still hold the condensed residual at (x_last, zst): the
  // check that ended the last mixed solve, which recovery can take as it is
  bool cond_fresh = false;

  double setup_ms = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // setup phases: events at the start of phases 2..9 (phase 1 starts at
  // ev0, the last ends at ev1) and the last setup's phase times
  static constexpr int kPhases = 9;
  hipEvent_t ph_ev[kPhases] = {};
  double phase_ms[kPhases] = {};

  int fail(int code, const std::string &m) {
    err = m;
    return code;
  }
  // Setup scratch: small allocations come from 64 MB device chunks, each
  // with a pinned host mirror at the same offsets.  An upload only writes
  // the mirror and widens the chunk's dirty range; flush() copies every
  // dirty range with one asynchronous copy on the context's stream and runs
  // before each device operation of the setup (the CHK macro), so the
  // thousands of small index and job arrays of a setup cost a few copies.
  // Everything is released when the setup ends, after a synchronisation.
  static constexpr size_t kChunk = 64ull << 20, kSmall = 4ull << 20;
  struct Chunk {
    char *dev = nullptr, *host = nullptr;
    size_t used = 0, lo = 0, hi = 0;  // [lo, hi): bytes waiting for the copy
  };
  std::vector<Chunk> chunks;
  bool dirty = false;

  size_t cur_chunk = 0;  // chunks are kept for the context's lifetime and rewound per setup
  hipError_t arena_alloc(void **p, size_t bytes, char **host = nullptr) {
    bytes = (bytes + 255) & ~size_t(255);
    while (cur_chunk < chunks.size() && chunks[cur_chunk].used + bytes > kChunk) ++cur_chunk;
    if (cur_chunk == chunks.size()) {
      Chunk c;
      hipError_t e = hipMalloc((void **)&c.dev, kChunk);
      if (e != hipSuccess) return e;
      e = hipHostMalloc((void **)&c.host, kChunk, hipHostMallocDefault);
      if (e != hipSuccess) {
        (void)hipFree(c.dev);
        return e;
      }
      chunks.push_back(c);
    }
    Chunk &c = chunks[cur_chunk];
    *p = c.dev + c.used;
    if (host) {
      *host = c.host + c.used;
      if (c.lo == c.hi) c.lo = c.used;
      c.hi = c.used + bytes;
      dirty = true;
    }
    c.used += bytes;
    return hipSuccess;
  }
  hipError_t flush() {
    if (!dirty) return hipSuccess;
    dirty = false;
    for (Chunk &c : chunks)
      if (c.hi > c.lo) {
        hipError_t e = hipMemcpyAsync(c.dev + c.lo, c.host + c.lo, c.hi - c.lo,
                                      hipMemcpyHostToDevice, stream);
        c.lo = c.hi = 0;
        if (e != hipSuccess) return e;
      }
    return hipSuccess;
  }
  // end of a setup: every copy has completed once the stream is idle
  hipError_t release_setup_scratch() {
    hipError_t e = flush();
    hipError_t e2 = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = e2;
    for (Chunk &c : chunks) c.used = c.lo = c.hi = 0;
    cur_chunk = 0;
    dirty = false;
    for (void *q : setup_allocs) pool_put(q);
    setup_allocs.clear();
    return e;
  }
  // Device blocks of the setup (scratch and results) are kept between
  // setups and handed out again by best fit: a new setup of the same
  // problem finds every large buffer it needs without hipMalloc/hipFree
  // (which synchronise and, for buffers of tens of GB, can stall for
  // seconds).  Unused blocks are released when an allocation fails and when
  // the context is destroyed.
  struct PBlock {
    void *p;
    size_t bytes;
    bool used;
  };
  std::vector<PBlock> pool;
  hipError_t pool_get(void **out, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    int best = -1;
    for (size_t i = 0; i < pool.size(); ++i) {
      const PBlock &b = pool[i];
      if (b.used || b.bytes < bytes || b.bytes > bytes + bytes / 2 + (size_t(64) << 20)) continue;
      if (best < 0 || b.bytes < pool[best].bytes) best = (int)i;
    }
    if (best >= 0) {
      pool[best].used = true;
      *out = pool[best].p;
      return hipSuccess;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      pool_trim();
      e = hipMalloc(out, bytes);
    }
    if (e == hipSuccess) pool.push_back({*out, bytes, true});
    return e;
  }
  void pool_put(void *p) {
    for (PBlock &b : pool)
      if (b.p == p) {
        b.used = false;
        return;
      }
    (void)hipFree(p);  // not a pool block
  }
  void pool_trim() {
    (void)hipStreamSynchronize(stream);
    std::vector<PBlock> keep;
    for (PBlock &b : pool) {
      if (b.used)
        keep.push_back(b);
      else
        (void)hipFree(b.p);
    }
    pool.swap(keep);
  }
  // whether pool_get would hand out an existing block for this request
  bool pool_has(size_t bytes) const {
    bytes = (bytes + 255) & ~size_t(255);
    for (const PBlock &b : pool)
      if (!b.used && b.bytes >= bytes && b.bytes <= bytes + bytes / 2 + (size_t(64) << 20)) return true;
    return false;
  }
  // the largest unused pool block of at least lo and at most hi bytes (0: none)
  size_t pool_fit(size_t lo, size_t hi) const {
    size_t best = 0;
    for (const PBlock &b : pool)
      if (!b.used && b.bytes >= lo && b.bytes <= hi && b.bytes > best) best = b.bytes;
    return best;
  }
  size_t pool_unused_bytes() const {
    size_t t = 0;
    for (const PBlock &b : pool)
      if (!b.used) t += b.bytes;
    return t;
  }
  void free_chunks() {
    for (Chunk &c : chunks) {
      (void)hipFree(c.dev);
      (void)hipHostFree(c.host);
    }
    chunks.clear();
    cur_chunk = 0;
  }
  template <class T>
  hipError_t dalloc(T **p, size_t count, bool setup_scope = false) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (setup_scope && count * sizeof(T) <= kSmall) return arena_alloc((void **)p, count * sizeof(T));
    hipError_t e;
    if (setup_scope || cur_scope == 2) {
      e = pool_get((void **)p, count * sizeof(T));
    } else {
      e = hipMalloc((void **)p, count * sizeof(T));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        pool_trim();
        e = hipMalloc((void **)p, count * sizeof(T));
      }
    }
    if (e == hipSuccess)
      (setup_scope ? setup_allocs : (cur_scope == 2 ? setup_keep : allocs)).push_back(*p);
    return e;
  }
  // a setup-scope allocation no longer needed before the setup ends
  void free_setup_early(void *p) {
    auto it = std::find(setup_allocs.begin(), setup_allocs.end(), p);
    if (it == setup_allocs.end()) return;  // arena memory: reclaimed with the arena
    (void)hipStreamSynchronize(stream);
    pool_put(p);
    setup_allocs.erase(it);
  }
  template <class T>
  hipError_t upload(T **p, const std::vector<T> &v, bool setup_scope = false) {
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (setup_scope && bytes <= kSmall) {
      char *h = nullptr;
      hipError_t e = arena_alloc((void **)p, bytes, &h);
      if (e == hipSuccess && !v.empty()) std::memcpy(h, v.data(), v.size() * sizeof(T));
      return e;
    }
    hipError_t e = dalloc(p, v.size(), setup_scope);
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    e = flush();  // keep the order of the copies
    if (e != hipSuccess) return e;
    return hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  }
};

struct vb_mlp {
  hipStream_t stream = nullptr;     // the caller's stream (NULL: the default stream)
  hipStream_t cap_stream = nullptr; // training's own stream when `stream` is NULL
  bool own_stream = false;          // cap_stream was created here
  std::string err;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *mu = nullptr, *sd = nullptr;
  int *t = nullptr;
  double *loss = nullptr;
  float *X = nullptr, *y = nullptr;  // training set
  int64_t n = 0, cap = 0;
  bool trained = false;
  int warm = 1;
  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
};

#define CHK(x)                                                                       \
  do {                                                                               \
    hipError_t f_ = ctx->flush();                                                    \
    hipError_t e_ = (f_ != hipSuccess) ? f_ : (x);                                   \
    if (e_ != hipSuccess)                                                            \
      return ctx->fail(e_ == hipErrorOutOfMemory ? VB_ERR_OOM : VB_ERR_DEVICE,        \
                       std::string(#x) + ": " + hipGetErrorString(e_));               \
  } while (0)
// allocations and uploads: no flush, so consecutive uploads share one copy
#define UCHK(x)                                                                      \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      return ctx->fail(e_ == hipErrorOutOfMemory ? VB_ERR_OOM : VB_ERR_DEVICE,        \
                       std::string(#x) + ": " + hipGetErrorString(e_));               \
  } while (0)

extern "C" {

int vb_create(vb_ctx **out, const vb_options *opt) {
  if (!out) return VB_ERR_ARG;
  vb_ctx *ctx = new vb_ctx();
  vb_options d{};
  d.precision = VB_PREC_FP64;
  d.scaling = VB_SCALING_DELUXE;
  d.tol = 1e-8;
  d.maxit = 1000;
  d.svd_tol = 1e-10;
  d.panel = NB;
  d.stream = nullptr;
  d.profile = 0;
  if (opt) {
    d = *opt;
    if (d.tol <= 0) d.tol = 1e-8;
    if (d.maxit <= 0) d.maxit = 1000;
    if (d.svd_tol <= 0) d.svd_tol = 1e-10;
    if (d.panel <= 0) d.panel = NB;
  }
  if (d.panel != 64 && d.panel != 32) {
    delete ctx;
    return VB_ERR_ARG;
  }
  // NaN fails every comparison: the limits and tolerances are checked as
  // "x >= 0" so that NaN is rejected rather than taken as a value
  if ((d.precision != VB_PREC_FP64 && d.precision != VB_PREC_MIXED) ||
      (d.scaling != VB_SCALING_DELUXE && d.scaling != VB_SCALING_COUNTING) ||
      !(d.setup_mem_limit >= 0.0) || !(d.local_mem_limit >= 0.0) || !std::isfinite(d.tol) ||
      !std::isfinite(d.svd_tol) || !(d.adaptive_theta >= 0.0) || !std::isfinite(d.adaptive_theta) ||
      d.pcg_launch < VB_PCG_AUTO || d.pcg_launch > VB_PCG_PERSISTENT || d.schur_kernel < 0 ||
      d.schur_kernel > 2 || !(d.fp32_pivot_min >= 0.0) || !std::isfinite(d.fp32_pivot_min) ||
      d.tune_factor < 0 || d.tune_factor > 2 || !(d.inner_tol >= 0.0 && d.inner_tol < 1.0)) {
    delete ctx;
    return VB_ERR_ARG;
  }
  ctx->opt = d;
  ctx->fp32 = (d.precision == VB_PREC_MIXED);
  ctx->wsz = ctx->fp32 ? sizeof(float) : sizeof(double);
  ctx->stream = (hipStream_t)d.stream;
  if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
    delete ctx;
    return VB_ERR_DEVICE;
  }
  *out = ctx;
  return VB_OK;
}

static void free_list(std::vector<void *> &v) {
  for (void *p : v) (void)hipFree(p);
  v.clear();
}

void vb_destroy(vb_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->it_exec) (void)hipGraphExecDestroy(ctx->it_exec);
  if (ctx->it_graph) (void)hipGraphDestroy(ctx->it_graph);
  (void)ctx->release_setup_scratch();
  ctx->free_chunks();
  for (void *q : ctx->setup_keep) ctx->pool_put(q);
  ctx->setup_keep.clear();
  ctx->pool_trim();
  ctx->t_ldl.destroy();
  ctx->t_gemv.destroy();
  free_list(ctx->allocs);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  for (hipEvent_t e : ctx->ph_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  delete ctx;
}

const char *vb_last_error(const vb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t vb_interface_size(const vb_ctx *ctx) { return ctx ? ctx->nG + ctx->nS : 0; }

static int assemble_impl(vb_ctx *ctx, int64_t n_iface, int n_sub, const vb_subdomain *subs,
                         int n_ent, const vb_entity *ents);

// A failed call leaves the context as it was (the problems added before).
int vb_assemble(vb_ctx *ctx, int64_t n_iface, int n_sub, const vb_subdomain *subs, int n_ent,
                const vb_entity *ents) {
  if (!ctx) return VB_ERR_ARG;
  const size_t e0 = ctx->ents.size(), s0 = ctx->subs.size();
  const int mx[5] = {ctx->max_n_csr, ctx->max_N, ctx->max_e, ctx->max_ng, ctx->max_ent};
  const int rc = assemble_impl(ctx, n_iface, n_sub, subs, n_ent, ents);
  if (rc != VB_OK && ctx->state <= 1 && !ctx->finalized) {
    ctx->ents.resize(e0);
    ctx->subs.resize(s0);
    ctx->max_n_csr = mx[0], ctx->max_N = mx[1], ctx->max_e = mx[2], ctx->max_ng = mx[3],
    ctx->max_ent = mx[4];
  }
  return rc;
}

static int assemble_impl(vb_ctx *ctx, int64_t n_iface, int n_sub, const vb_subdomain *subs,
                         int n_ent, const vb_entity *ents) {
  if (ctx->state > 1 || ctx->finalized)
    return ctx->fail(VB_ERR_STATE, "vb_assemble: problems can only be added before vb_setup");
  if (n_iface < 0 || n_sub <= 0 || !subs || n_ent < 0 || (n_ent > 0 && !ents))
    return ctx->fail(VB_ERR_ARG, "vb_assemble: bad sizes");
  vb_ctx::Prob P;
  P.g0 = ctx->nG;
  P.ng = n_iface;
  P.s0 = ctx->nS;
  P.ns = n_sub;
  P.e0 = (int)ctx->ents.size();
  P.ne = n_ent;
  const int64_t g0 = P.g0;
  const int s0 = P.s0, e0 = P.e0;
  // entities
  std::vector<int32_t> ent_of(n_iface, -1), pos_in(n_iface, -1);
  ctx->ents.resize(e0 + n_ent);
  for (int e = 0; e < n_ent; ++e) {
    const vb_entity &E = ents[e];
    if (E.n <= 0 || !E.gids || E.n_con < 0 || (E.n_con > 0 && !E.con) || E.n_con > 1024)
      return ctx->fail(VB_ERR_ARG, "vb_assemble: bad entity " + std::to_string(e));
    EntH &H = ctx->ents[e0 + e];
    H.kind = E.kind;
    H.n = E.n;
    H.ncon = E.n_con;
    H.gids.resize(E.n);
    H.con.assign(E.con, E.con + (size_t)E.n_con * E.n);
    for (int j = 0; j < E.n; ++j) {
      int64_t g = E.gids[j];
      if (g < 0 || g >= n_iface || ent_of[g] >= 0)
        return ctx->fail(VB_ERR_ARG, "vb_assemble: entity ids must cover each interface id once");
      ent_of[g] = e;
      pos_in[g] = j;
      H.gids[j] = g0 + g;
    }
  }
  for (int64_t g = 0; g < n_iface; ++g)
    if (ent_of[g] < 0) return ctx->fail(VB_ERR_ARG, "vb_assemble: interface id not in any entity");
  // subdomains
  ctx->subs.resize(s0 + n_sub);
  for (int sl = 0; sl < n_sub; ++sl) {
    const int s = s0 + sl;
    const vb_subdomain &D = subs[sl];
    SubH &S = ctx->subs[s];
    if (D.n <= 0 || D.nnz < 0 || !D.indptr || !D.indices || !D.data || !D.kind || !D.gid ||
        !D.pweight || !D.rhs)
      return ctx->fail(VB_ERR_ARG, "vb_assemble: bad subdomain " + std::to_string(sl));
    S.n = S.n2 = D.n;
    S.indptr.assign(D.indptr, D.indptr + D.n + 1);
    bool mono = S.indptr[0] == 0 && S.indptr[D.n] == D.nnz;
    for (int i = 0; i < D.n && mono; ++i) mono = S.indptr[i] <= S.indptr[i + 1];
    if (!mono)
      return ctx->fail(VB_ERR_ARG, "vb_assemble: bad indptr in subdomain " + std::to_string(sl));
    S.indices.resize(D.nnz);
    for (int64_t q = 0; q < D.nnz; ++q) {
      if (D.indices[q] < 0 || D.indices[q] >= D.n)
        return ctx->fail(VB_ERR_ARG, "vb_assemble: column index out of range");
      S.indices[q] = (int32_t)D.indices[q];
    }
    S.vals.assign(D.data, D.data + D.nnz);
    S.rhs.assign(D.rhs, D.rhs + D.n);
    S.kind.assign(D.kind, D.kind + D.n);
    S.gid.assign(D.gid, D.gid + D.n);
    std::vector<std::pair<int64_t, int>> iface;
    S.nv = S.nel = 0;
    for (int i = 0; i < D.n; ++i) {
      if (S.kind[i] == VB_KIND_INTERIOR) S.nv++;
      else if (S.kind[i] == VB_KIND_PRESSURE) S.nel++;
      else if (S.kind[i] == VB_KIND_INTERFACE) {
        int64_t g = S.gid[i];
        if (g < 0 || g >= n_iface) return ctx->fail(VB_ERR_ARG, "vb_assemble: bad gid");
        iface.push_back({((int64_t)ent_of[g] << 32) | pos_in[g], i});
        S.gid[i] = g0 + g;
      } else
        return ctx->fail(VB_ERR_ARG, "vb_assemble: bad kind");
    }
    if (S.nel < 2) return ctx->fail(VB_ERR_ARG, "vb_assemble: a subdomain needs >= 2 pressures");
    std::sort(iface.begin(), iface.end());
    S.ng = (int)iface.size();
    S.N = S.nv + S.nel + S.ng + 1;
    S.e = S.nv + S.nel - 1;
    S.ld = round_up(S.N, 32);
    S.pos.assign(D.n, -1);
    int cv = 0, cp = 0;
    S.pw.clear();
    S.vol = 0.0;
    for (int i = 0; i < D.n; ++i) {
      if (S.kind[i] == VB_KIND_INTERIOR) S.pos[i] = cv++;
      else if (S.kind[i] == VB_KIND_PRESSURE) {
        if (!(D.pweight[i] > 0.0) || !std::isfinite(D.pweight[i]))
          return ctx->fail(VB_ERR_ARG, "vb_assemble: pressure weights (element volumes) must be "
                                       "positive, subdomain " + std::to_string(sl));
        S.pos[i] = S.nv + cp++;
        S.pw.push_back(D.pweight[i]);
        S.vol += D.pweight[i];
      }
    }
    S.gidl.resize(S.ng);
    S.ents.clear();
    S.ent_off.clear();
    for (int l = 0; l < S.ng; ++l) {
      int i = iface[l].second;
      S.pos[i] = S.nv + S.nel + l;
      S.gidl[l] = S.gid[i];
      int e = e0 + ent_of[S.gid[i] - g0];
      if (S.ents.empty() || S.ents.back() != e) {
        S.ents.push_back(e);
        S.ent_off.push_back(l);
      }
    }
    for (size_t q = 0; q < S.ents.size(); ++q) {
      int e = S.ents[q];
      int cnt = (q + 1 < S.ents.size() ? S.ent_off[q + 1] : S.ng) - S.ent_off[q];
      if (cnt != ctx->ents[e].n)
        return ctx->fail(VB_ERR_ARG, "vb_assemble: subdomain " + std::to_string(sl) +
                                         " holds only part of entity " + std::to_string(e - e0));
      ctx->ents[e].subs.push_back(s);
    }
    // sub-box labels of a one-level nested dissection: checked here, used
    // when every subdomain of the context has them
    S.part.clear();
    if (D.part) {
      S.part.assign(D.part, D.part + D.n);
      int nbox = 0;
      for (int i = 0; i < D.n; ++i) {
        if (S.kind[i] == VB_KIND_INTERFACE) {
          S.part[i] = -1;
          continue;
        }
        if (S.part[i] < -1 || (S.kind[i] == VB_KIND_PRESSURE && S.part[i] < 0))
          return ctx->fail(VB_ERR_ARG, "vb_assemble: subdomain " + std::to_string(sl) +
                                           ": sub-box labels must be >= -1, and >= 0 for pressures");
        nbox = std::max(nbox, S.part[i] + 1);
      }
      std::vector<int> npress(nbox, 0);
      for (int i = 0; i < D.n; ++i)
        if (S.kind[i] == VB_KIND_PRESSURE) npress[S.part[i]]++;
      for (int b = 0; b < nbox; ++b)
        if (!npress[b])
          return ctx->fail(VB_ERR_ARG, "vb_assemble: subdomain " + std::to_string(sl) +
                                           ": sub-box " + std::to_string(b) + " holds no pressure");
      for (int i = 0; i < D.n; ++i) {
        const int a = S.part[i];
        if (a < 0) continue;
        for (int64_t q = S.indptr[i]; q < S.indptr[i + 1]; ++q) {
          const int b = S.part[S.indices[q]];
          if (b >= 0 && b != a)
            return ctx->fail(VB_ERR_ARG, "vb_assemble: subdomain " + std::to_string(sl) +
                                             ": DoFs of sub-boxes " + std::to_string(a) + " and " +
                                             std::to_string(b) + " are coupled");
        }
      }
    }
    ctx->max_n_csr = std::max(ctx->max_n_csr, S.n);
    ctx->max_n_full = std::max(ctx->max_n_full, S.n);
    ctx->max_N = std::max(ctx->max_N, S.N);
    ctx->max_e = std::max(ctx->max_e, S.e);
    ctx->max_ng = std::max(ctx->max_ng, S.ng);
    ctx->max_ent = std::max(ctx->max_ent, (int)S.ents.size());
  }
  ctx->nG += n_iface;
  ctx->nS += n_sub;
  ctx->probs.push_back(P);
  ctx->state = 1;
  return VB_OK;
}

}  // extern "C"

// Two-level nested dissection, when every subdomain carries sub-box labels:
// one front per sub-box (its interior velocities and element pressures,
// bordered by the separator and interface DoFs B it couples to), and each
// subdomain's SubH rewritten as the second level (separator velocities,
// one "pressure" per sub-box = its constant pressure, the interface DoFs).
static int build_nd(vb_ctx *ctx) {
  ctx->fronts.clear();
  ctx->max_n_csr = ctx->max_N = ctx->max_e = 0;
  ctx->max_n_full = ctx->max_nf_csr = ctx->max_Nf = ctx->max_ef = ctx->max_nbox = ctx->max_fm = 0;
  int64_t sep_off = 0;
  for (int s = 0; s < ctx->nS; ++s) {
    SubH &S = ctx->subs[s];
    const int n = S.n;
    S.f_indptr = S.indptr;
    S.f_indices = S.indices;
    S.f_vals = S.vals;
    S.f_rhs = S.rhs;
    S.f_pos = S.pos;
    S.f_nv = S.nv;
    S.f_nel = S.nel;
    int nbox = 0;
    for (int i = 0; i < n; ++i) nbox = std::max(nbox, S.part[i] + 1);
    // second-level dense positions of the separator and interface DoFs
    std::vector<int32_t> l2(n, -1);
    int nsep = 0;
    for (int i = 0; i < n; ++i)
      if (S.kind[i] == VB_KIND_INTERIOR && S.part[i] < 0) l2[i] = nsep++;
    for (int i = 0; i < n; ++i)
      if (S.kind[i] == VB_KIND_INTERFACE) l2[i] = nsep + nbox + (S.pos[i] - S.nv - S.nel);
    const int N2 = nsep + nbox + S.ng + 1;
    std::vector<double> boxvol(nbox, 0.0);
    S.first_front = (int)ctx->fronts.size();
    std::vector<int32_t> floc(n, -1);
    for (int b = 0; b < nbox; ++b) {
      ctx->fronts.emplace_back();
      FrontH &F = ctx->fronts.back();
      F.sub = s;
      F.box = b;
      SubH &T = F.S;
      std::vector<int> rows;
      for (int i = 0; i < n; ++i)
        if (S.kind[i] == VB_KIND_INTERIOR && S.part[i] == b) rows.push_back(i);
      T.nv = (int)rows.size();
      for (int i = 0; i < n; ++i)
        if (S.kind[i] == VB_KIND_PRESSURE && S.part[i] == b) rows.push_back(i);
      T.nel = (int)rows.size() - T.nv;
      std::vector<int> B;
      for (int i : rows)
        for (int64_t q = S.indptr[i]; q < S.indptr[i + 1]; ++q) {
          const int j = S.indices[q];
          if (l2[j] >= 0 && floc[j] != -2) {
            floc[j] = -2;
            B.push_back(j);
          }
        }
      std::sort(B.begin(), B.end(), [&](int a, int c) { return l2[a] < l2[c]; });
      T.ng = (int)B.size();
      const int nr = (int)rows.size();
      for (int k = 0; k < nr; ++k) floc[rows[k]] = k;
      for (int k = 0; k < T.ng; ++k) floc[B[k]] = nr + k;
      T.n = T.n2 = nr + T.ng;
      T.indptr.assign(1, 0);
      T.indices.clear();
      T.vals.clear();
      T.rhs.clear();
      for (int i : rows) {
        for (int64_t q = S.indptr[i]; q < S.indptr[i + 1]; ++q) {
          T.indices.push_back(floc[S.indices[q]]);
          T.vals.push_back(S.vals[q]);
        }
        T.indptr.push_back((int64_t)T.indices.size());
        T.rhs.push_back(S.rhs[i]);
      }
      for (int j : B) {
        for (int64_t q = S.indptr[j]; q < S.indptr[j + 1]; ++q) {
          const int c = floc[S.indices[q]];
          if (c >= 0 && c < nr && S.part[S.indices[q]] == b) {
            T.indices.push_back(c);
            T.vals.push_back(S.vals[q]);
          }
        }
        T.indptr.push_back((int64_t)T.indices.size());
        T.rhs.push_back(0.0);
      }
      T.kind.assign(T.n, VB_KIND_INTERIOR);
      for (int k = T.nv; k < nr; ++k) T.kind[k] = VB_KIND_PRESSURE;
      for (int k = nr; k < T.n; ++k) T.kind[k] = VB_KIND_INTERFACE;
      T.pos.resize(T.n);
      std::iota(T.pos.begin(), T.pos.end(), 0);
      T.pw.clear();
      double ss = 0.0;
      for (int k = T.nv; k < nr; ++k) {
        const double w = S.pw[S.pos[rows[k]] - S.nv];
        T.pw.push_back(w);
        boxvol[b] += w;
        ss += w * w;
      }
      T.vol = boxvol[b];
      // the kept coordinate (last after the reflector that maps the volumes
      // w onto it, alpha = -sign(w_last) |w|) is gamma times the constant
      // pressure of the sub-box, gamma = sum(w) / alpha
      const double alpha = (T.pw.back() >= 0.0) ? -std::sqrt(ss) : std::sqrt(ss);
      F.gamma = boxvol[b] / alpha;
      T.N = T.nv + T.nel + T.ng + 1;
      T.e = T.nv + T.nel - 1;
      T.ld = round_up(T.N, 32);
      F.oidx.assign(T.n, -1);
      for (int k = 0; k < nr; ++k) F.oidx[k] = rows[k];
      F.map.clear();
      F.map.push_back(nsep + b);
      F.bsep.clear();
      F.bgid.clear();
      for (int j : B) {
        F.map.push_back(l2[j]);
        F.bsep.push_back(S.kind[j] == VB_KIND_INTERIOR ? l2[j] : -1);
        F.bgid.push_back(S.kind[j] == VB_KIND_INTERFACE ? S.gid[j] : -1);
      }
      F.map.push_back(N2 - 1);
      for (int i : rows) floc[i] = -1;
      for (int j : B) floc[j] = -1;
      ctx->max_nf_csr = std::max(ctx->max_nf_csr, T.n);
      ctx->max_Nf = std::max(ctx->max_Nf, T.N);
      ctx->max_ef = std::max(ctx->max_ef, T.e);
      ctx->max_fm = std::max(ctx->max_fm, T.ng + 2);
    }
    // the second level: CSR over the separator and interface DoFs
    std::vector<int32_t> rows2;
    for (int i = 0; i < n; ++i)
      if (l2[i] >= 0) rows2.push_back(i);
    std::vector<int64_t> ip(1, 0);
    std::vector<int32_t> ix, kd, ps;
    std::vector<int64_t> gd;
    std::vector<double> vl, rh;
    std::vector<int32_t> loc2(n, -1);
    for (size_t k = 0; k < rows2.size(); ++k) loc2[rows2[k]] = (int32_t)k;
    for (int i : rows2) {
      for (int64_t q = S.indptr[i]; q < S.indptr[i + 1]; ++q) {
        const int c = loc2[S.indices[q]];
        if (c < 0) continue;
        ix.push_back(c);
        vl.push_back(S.vals[q]);
      }
      ip.push_back((int64_t)ix.size());
      rh.push_back(S.rhs[i]);
      kd.push_back(S.kind[i]);
      gd.push_back(S.gid[i]);
      ps.push_back(l2[i]);
    }
    S.indptr.swap(ip);
    S.indices.swap(ix);
    S.vals.swap(vl);
    S.rhs.swap(rh);
    S.kind.swap(kd);
    S.gid.swap(gd);
    S.pos.swap(ps);
    S.oidx = rows2;
    S.n2 = (int)rows2.size();
    S.nv = nsep;
    S.nel = nbox;
    S.pw = boxvol;
    S.nsep = nsep;
    S.nbox = nbox;
    S.N = N2;
    S.e = nsep + nbox - 1;
    S.ld = round_up(S.N, 32);
    S.sep_off = sep_off;
    sep_off += nsep;
    ctx->max_n_csr = std::max(ctx->max_n_csr, S.n2);
    ctx->max_N = std::max(ctx->max_N, S.N);
    ctx->max_e = std::max(ctx->max_e, S.e);
    ctx->max_n_full = std::max(ctx->max_n_full, S.n);
    ctx->max_nbox = std::max(ctx->max_nbox, nbox);
  }
  ctx->n_sep_tot = sep_off;
  ctx->nd = true;
  return VB_OK;
}

// Device data of the two-level factorisation: front matrices and their
// descriptors, the full local CSR views, the second-level vector layout
// G2 = [global interface vector | separator values | sub-box constants] and
// the scatter jobs (one list per sub-box index: no two jobs of a list add
// into the same second-level matrix).
static int finalize_nd(vb_ctx *ctx) {
  const int nS = ctx->nS, nF = (int)ctx->fronts.size();
  int64_t ftot = 0, fitot = 0, fhtot = 0;
  for (auto &F : ctx->fronts) {
    SubH &T = F.S;
    T.W_off = ftot;
    ftot += T.ld * T.N;
    T.inv_off = fitot;
    fitot += (int64_t)((T.e + NB - 1) / NB) * NB * NB;
    T.hv_off = fhtot;
    fhtot += T.nel + 1;
  }
  char *fw = nullptr, *fi = nullptr;
  UCHK(ctx->dalloc(&fw, (size_t)std::max<int64_t>(ftot, 1) * ctx->wsz));
  UCHK(ctx->dalloc(&fi, (size_t)std::max<int64_t>(fitot, 1) * ctx->wsz));
  ctx->FW = fw;
  ctx->invLf = fi;
  UCHK(ctx->dalloc(&ctx->hvf, std::max<int64_t>(fhtot, 1)));
  UCHK(ctx->dalloc(&ctx->info_f, std::max(nF, 1)));
  ctx->g2_c0 = ctx->nG + nS + ctx->n_sep_tot;
  ctx->n_g2 = ctx->g2_c0 + nF;
  UCHK(ctx->dalloc(&ctx->G2, ctx->n_g2));
  UCHK(ctx->dalloc(&ctx->G2d, ctx->n_g2));
  ctx->frdev.assign(nF, SubDev{});
  for (int f = 0; f < nF; ++f) {
    FrontH &F = ctx->fronts[f];
    SubH &T = F.S;
    const SubH &P = ctx->subs[F.sub];
    // B DoFs: separator values or interface ids in G2
    T.gidl.resize(T.ng);
    T.gid.assign(T.n, -1);
    const int nr = T.nv + T.nel;
    for (int k = 0; k < T.ng; ++k) {
      T.gidl[k] = F.bsep[k] >= 0 ? ctx->nG + nS + P.sep_off + F.bsep[k] : F.bgid[k];
      T.gid[nr + k] = T.gidl[k];
    }
    UCHK(ctx->upload(&T.d_indptr, T.indptr));
    UCHK(ctx->upload(&T.d_indices, T.indices));
    UCHK(ctx->upload(&T.d_vals, T.vals));
    UCHK(ctx->upload(&T.d_rhs, T.rhs));
    UCHK(ctx->upload(&T.d_pos, T.pos));
    UCHK(ctx->upload(&T.d_kind, T.kind));
    UCHK(ctx->upload(&T.d_gid, T.gid));
    UCHK(ctx->upload(&T.d_pw, T.pw));
    UCHK(ctx->upload(&T.d_gidl, T.gidl));
    UCHK(ctx->upload(&F.d_oidx, F.oidx));
    UCHK(ctx->upload(&F.d_map, F.map));
    SubDev &D = ctx->frdev[f];
    D.W = (char *)ctx->FW + T.W_off * ctx->wsz;
    D.ld = T.ld;
    D.nv = T.nv;
    D.nel = T.nel;
    D.ng = T.ng;
    D.N = T.N;
    D.e = T.e;
    D.n_csr = T.n;
    D.indptr = T.d_indptr;
    D.indices = T.d_indices;
    D.vals = T.d_vals;
    D.rhs = T.d_rhs;
    D.pos = T.d_pos;
    D.pweight = T.d_pw;
    D.hv = ctx->hvf + T.hv_off;
    D.gidl = T.d_gidl;
    D.oidx = F.d_oidx;
  }
  UCHK(ctx->upload(&ctx->d_frdev, ctx->frdev));
  ctx->fulldev.assign(nS, SubDev{});
  std::vector<int32_t> first(nS + 1, 0);
  for (int s = 0; s < nS; ++s) {
    SubH &S = ctx->subs[s];
    UCHK(ctx->upload(&S.d_f_indptr, S.f_indptr));
    UCHK(ctx->upload(&S.d_f_indices, S.f_indices));
    UCHK(ctx->upload(&S.d_f_vals, S.f_vals));
    UCHK(ctx->upload(&S.d_f_rhs, S.f_rhs));
    UCHK(ctx->upload(&S.d_f_pos, S.f_pos));
    SubDev &D = ctx->fulldev[s];
    D.nv = S.f_nv;
    D.nel = S.f_nel;
    D.ng = S.ng;
    D.n_csr = S.n;
    D.indptr = S.d_f_indptr;
    D.indices = S.d_f_indices;
    D.vals = S.d_f_vals;
    D.rhs = S.d_f_rhs;
    D.pos = S.d_f_pos;
    D.b0 = ctx->b0 + S.b0_off;
    first[s + 1] = S.first_front + S.nbox;
  }
  UCHK(ctx->upload(&ctx->d_fulldev, ctx->fulldev));
  UCHK(ctx->upload(&ctx->d_fr_first, first));
  ctx->fj_scatter.assign(ctx->max_nbox, {});
  for (int s = 0; s < nS; ++s) {
    const SubH &S = ctx->subs[s];
    for (int b = 0; b < S.nbox; ++b) {
      const FrontH &F = ctx->fronts[S.first_front + b];
      FrontJob J{};
      J.Wf = (char *)ctx->FW + F.S.W_off * ctx->wsz;
      J.ldf = F.S.ld;
      J.e = F.S.e;
      J.m = F.S.ng + 2;
      J.W2 = (char *)ctx->W + S.W_off * ctx->wsz;
      J.ld2 = S.ld;
      J.map = F.d_map;
      J.gamma = F.gamma;
      ctx->fj_scatter[b].push_back(J);
    }
  }
  ctx->d_fj_scatter.assign(ctx->max_nbox, nullptr);
  for (int b = 0; b < ctx->max_nbox; ++b) UCHK(ctx->upload(&ctx->d_fj_scatter[b], ctx->fj_scatter[b]));
  return VB_OK;
}

// Device copies of every assembled problem and the dense workspace (run by
// the first vb_setup, once all problems are known).
static int finalize_device(vb_ctx *ctx) {
  const int n_sub = ctx->nS;
  const int n_ent = (int)ctx->ents.size();
  const int64_t n_iface = ctx->nG;
  {
    bool all = n_sub > 0;
    for (const auto &S : ctx->subs) all = all && !S.part.empty();
    if (all) {
      int rc = build_nd(ctx);
      if (rc) return rc;
    }
  }
  // ---- device copies of the caller's data and the dense workspace
  int64_t wtot = 0, itot = 0, btot = 0, htot = 0, wmax1 = 1;
  for (auto &S : ctx->subs) {
    wtot += S.ld * S.N;
    wmax1 = std::max(wmax1, S.ld * S.N);
    S.inv_off = itot;
    itot += (int64_t)((S.e + NB - 1) / NB) * NB * NB;
    S.b0_off = btot;
    btot += S.ng + 1;
    S.hv_off = htot;
    htot += S.nel + 1;
  }
  {
    size_t fre = 0, tot = 0;
    UCHK(hipMemGetInfo(&fre, &tot));
    const double lim = ctx->opt.local_mem_limit > 0.0 ? ctx->opt.local_mem_limit : 0.45 * (double)fre;
    ctx->stream_w = !ctx->fp32 && !ctx->nd && (double)wtot * (double)ctx->wsz > lim;
    ctx->waves.clear();
    int64_t wcap = 0;
    const int64_t cap = ctx->stream_w ? std::max<int64_t>(wmax1, (int64_t)(lim / ctx->wsz)) : wtot;
    for (int s0 = 0; s0 < n_sub;) {
      int s1 = s0;
      int64_t off = 0;
      while (s1 < n_sub && (s1 == s0 || off + ctx->subs[s1].ld * ctx->subs[s1].N <= cap)) {
        ctx->subs[s1].W_off = off;
        off += ctx->subs[s1].ld * ctx->subs[s1].N;
        ++s1;
      }
      ctx->waves.push_back({s0, s1});
      wcap = std::max(wcap, off);
      s0 = s1;
    }
    char *w = nullptr, *iv = nullptr;
    UCHK(ctx->dalloc(&w, (size_t)std::max<int64_t>(wcap, 1) * ctx->wsz));
    UCHK(ctx->dalloc(&iv, (size_t)itot * ctx->wsz));
    ctx->W = w;
    ctx->invL = iv;
    int64_t xtot = 0;
    for (auto &S : ctx->subs) {
      if (ctx->stream_w) {
        S.xld = round_up(S.ng + 1, 32);
        S.X_off = xtot;
        xtot += S.xld * (S.ng + 1);
      } else {
        S.xld = S.ld;
        S.X_off = S.W_off + (S.e + 1) + (int64_t)(S.e + 1) * S.ld;
      }
    }
    if (ctx->stream_w) UCHK(ctx->dalloc(&w, (size_t)xtot * ctx->wsz));
    ctx->Xc = ctx->stream_w ? w : ctx->W;
    for (auto &S : ctx->subs) S.X = (char *)ctx->Xc + S.X_off * ctx->wsz;
  }
  UCHK(ctx->dalloc(&ctx->b0, btot));
  UCHK(ctx->dalloc(&ctx->hv, htot));
  UCHK(ctx->dalloc(&ctx->info, 4 * (size_t)n_sub + 64 + 4 * (size_t)n_ent));
  ctx->subdev.resize(n_sub);
  for (int s = 0; s < n_sub; ++s) {
    SubH &S = ctx->subs[s];
    UCHK(ctx->upload(&S.d_indptr, S.indptr));
    UCHK(ctx->upload(&S.d_indices, S.indices));
    UCHK(ctx->upload(&S.d_vals, S.vals));
    UCHK(ctx->upload(&S.d_rhs, S.rhs));
    UCHK(ctx->upload(&S.d_pos, S.pos));
    UCHK(ctx->upload(&S.d_kind, S.kind));
    UCHK(ctx->upload(&S.d_gid, S.gid));
    UCHK(ctx->upload(&S.d_pw, S.pw));
    std::vector<int64_t> gext(S.gidl);
    gext.push_back(n_iface + s);
    UCHK(ctx->upload(&S.d_gidl, gext));
    UCHK(ctx->upload(&S.d_ents, S.ents));
    UCHK(ctx->upload(&S.d_entoff, S.ent_off));
    SubDev &D = ctx->subdev[s];
    D.W = (char *)ctx->W + S.W_off * ctx->wsz;
    D.ld = S.ld;
    D.X = S.X;
    D.xld = S.xld;
    D.nv = S.nv;
    D.nel = S.nel;
    D.ng = S.ng;
    D.N = S.N;
    D.e = S.e;
    D.n_csr = S.n2;
    D.indptr = S.d_indptr;
    D.indices = S.d_indices;
    D.vals = S.d_vals;
    D.rhs = S.d_rhs;
    D.pos = S.d_pos;
    D.pweight = S.d_pw;
    D.hv = ctx->hv + S.hv_off;
    D.b0 = ctx->b0 + S.b0_off;
    D.gidl = S.d_gidl;
    D.n_ent = (int)S.ents.size();
    D.ent = S.d_ents;
    D.ent_off = S.d_entoff;
    if (ctx->nd) {
      UCHK(ctx->upload(&S.d_oidx, S.oidx));
      D.oidx = S.d_oidx;
    }
  }
  UCHK(ctx->upload(&ctx->d_subdev, ctx->subdev));
  if (ctx->nd) {
    int rc = finalize_nd(ctx);
    if (rc) return rc;
  }
  ctx->entdev.resize(n_ent);
  for (int e = 0; e < n_ent; ++e) {
    EntH &H = ctx->ents[e];
    UCHK(ctx->upload(&H.d_gids, H.gids));
    UCHK(ctx->upload(&H.d_con, H.con));
    int rmax = std::max(1, std::min(H.ncon, H.n));
    UCHK(ctx->dalloc(&H.d_V, (size_t)H.n * rmax));
    UCHK(ctx->dalloc(&H.d_tau, (size_t)rmax));
    UCHK(ctx->dalloc(&H.d_work, (size_t)H.n * std::max(1, H.ncon)));
    H.d_rank = ctx->info + 4 * n_sub + 64 + e;
    EntDev &D = ctx->entdev[e];
    D.n = H.n;
    D.n_con = H.ncon;
    D.con = H.d_con;
    D.gids = H.d_gids;
    D.V = H.d_V;
    D.tau = H.d_tau;
    D.rank = H.d_rank;
    D.work = H.d_work;
  }
  UCHK(ctx->upload(&ctx->d_entdev, ctx->entdev));
  ctx->entdev0 = ctx->entdev;
  for (auto &H : ctx->ents) {
    H.ncon0 = H.ncon;
    H.con0 = H.con;
    H.d_con0 = H.d_con;
    H.d_V0 = H.d_V;
    H.d_tau0 = H.d_tau;
    H.d_work0 = H.d_work;
  }
  // problem segments of the global interface vector
  std::vector<Seg> segs;
  int64_t maxn = 1;
  for (auto &P : ctx->probs) {
    segs.push_back({P.g0, P.ng, ctx->nG + P.s0, P.ns});
    maxn = std::max<int64_t>(maxn, P.ng + P.ns);
  }
  UCHK(ctx->upload(&ctx->d_segs, segs));
  ctx->seg_G = (int)std::min<int64_t>(DOT_BLOCKS, std::max<int64_t>(1, (maxn + 255) / 256));
  UCHK(ctx->dalloc(&ctx->d_tol, ctx->probs.size()));
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0) == hipSuccess)
    ctx->clock_khz = khz;
  ctx->finalized = true;
  return VB_OK;
}

extern "C" {

}  // extern "C"

// ------------------------------------------------------------------ setup
// Lists of values per key as CSR (ptr, idx): visit(emit) calls emit(key,
// value) for every entry in a fixed order and is run twice (count, then
// fill), so each key's values keep that order (the owner sums add them in
// it).
template <class Visit>
static void build_csr(int64_t nkeys, const Visit &visit, std::vector<int64_t> &ptr,
                      std::vector<int64_t> &idx) {
  ptr.assign(nkeys + 1, 0);
  visit([&](int64_t k, int64_t) { ++ptr[k + 1]; });
  for (int64_t k = 0; k < nkeys; ++k) ptr[k + 1] += ptr[k];
  idx.resize(ptr[nkeys]);
  std::vector<int64_t> cur(ptr.begin(), ptr.end() - 1);
  visit([&](int64_t k, int64_t v) { idx[cur[k]++] = v; });
}

template <typename T>
static int run_ldl(vb_ctx *ctx, std::vector<LdlJob<T>> &jobs, int max_n, int max_e,
                   bool timed = false, int nb = 0, int sb1 = 0) {
  if (jobs.empty()) return VB_OK;
  LdlJob<T> *dj = nullptr;
  UCHK(ctx->upload(&dj, jobs, true));
  std::vector<int> hn(jobs.size()), he(jobs.size()), hz(jobs.size());
  bool aligned16 = true;  // 16-byte aligned columns (leading dimension a multiple of 16 bytes)
  for (size_t b = 0; b < jobs.size(); ++b) {
    hn[b] = jobs[b].n;
    he[b] = jobs[b].e;
    hz[b] = jobs[b].zrow;
    aligned16 = aligned16 && (jobs[b].ld * sizeof(T)) % 16 == 0 &&
                reinterpret_cast<uintptr_t>(jobs[b].A) % 16 == 0;
  }
  CHK(ldl_batched<T>(dj, (int)jobs.size(), max_n, max_e, nb ? nb : ctx->opt.panel, ctx->stream,
                     (timed && ctx->opt.profile) ? &ctx->t_ldl : nullptr, &hn, &he, timed,
                     aligned16, sb1, &hz));
  return VB_OK;
}

// Panel width of the local Dirichlet factors of a level (0: single level or
// fronts, 1: second level): the step of the triangular sweeps over them.
static int dir_nb(const vb_ctx *ctx, int level) {
  return ctx->fac_nb[level] ? ctx->fac_nb[level] : ctx->opt.panel;
}

// The factorisation of class `cls` (see vb_ctx::fac_nb) with its chosen
// panel width and super-panel.  The first time a class runs, if the
// options ask for it, every candidate is timed on these very matrices
// (prepare() forms them again before each further run) and the fastest is
// kept for the context; the last candidate's factors stand when it is the
// fastest, otherwise the matrices are formed and factored once more.
template <typename T>
static int tuned_ldl(vb_ctx *ctx, int cls, std::vector<LdlJob<T>> &jobs, int max_n, int max_e,
                     bool timed, const std::function<int()> &prepare) {
  if (ctx->fac_nb[cls] == 0) {
    double work = 0.0;
    for (const auto &J : jobs) work += (double)J.e * J.n * J.n;
    const bool tune = !jobs.empty() && (ctx->opt.tune_factor == 1 ||
                                        (ctx->opt.tune_factor == 0 && work > 2e11));
    if (!tune) {
      ctx->fac_nb[cls] = ctx->opt.panel;
      ctx->fac_sb[cls] = 16 * ctx->opt.panel;
    } else {
      // (32-wide panels with 1024- or 256-column super-panels never won at
      // the 64- and 216-subdomain workloads and are not tried)
      static const int cand[][2] = {{64, 1024}, {64, 512}, {64, 2048}, {32, 512}};
      const int nc = (int)(sizeof(cand) / sizeof(cand[0]));
      hipEvent_t e0, e1;
      CHK(hipEventCreate(&e0));
      CHK(hipEventCreate(&e1));
      float best = 1e30f;
      int pick = 0;
      int rc = VB_OK;
      for (int c = 0; c < nc && !rc; ++c) {
        if (c > 0) rc = prepare();
        if (rc) break;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = VB_ERR_DEVICE;
        if (!rc) rc = run_ldl(ctx, jobs, max_n, max_e, false, cand[c][0], cand[c][1]);
        if (!rc && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess))
          rc = VB_ERR_DEVICE;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = VB_ERR_DEVICE;
        if (!rc && ms < best) {
          best = ms;
          pick = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (rc) return rc == VB_ERR_DEVICE ? ctx->fail(rc, "factorisation autotuner: HIP event error") : rc;
      ctx->fac_nb[cls] = cand[pick][0];
      ctx->fac_sb[cls] = cand[pick][1];
      if (pick == nc - 1 && !(timed && ctx->opt.profile)) return VB_OK;
      int rp = prepare();
      if (rp) return rp;
    }
  }
  return run_ldl(ctx, jobs, max_n, max_e, timed, ctx->fac_nb[cls], ctx->fac_sb[cls]);
}

static int run_gather(vb_ctx *ctx, const std::vector<GatherJob> &jobs, int max_m, int max_n) {
  if (jobs.empty()) return VB_OK;
  GatherJob *dj = nullptr;
  UCHK(ctx->upload(&dj, jobs, true));
  CHK(gather_blocks(dj, (int)jobs.size(), max_m, max_n, ctx->stream));
  return VB_OK;
}

static int run_diag(vb_ctx *ctx, const std::vector<DiagJob> &jobs, int max_cnt) {
  if (jobs.empty()) return VB_OK;
  DiagJob *dj = nullptr;
  UCHK(ctx->upload(&dj, jobs, true));
  CHK(set_diag(dj, (int)jobs.size(), max_cnt, ctx->stream));
  return VB_OK;
}

static int run_symm(vb_ctx *ctx, const std::vector<void *> &m, const std::vector<int64_t> &ld,
                    const std::vector<int32_t> &n, bool transpose = false, bool fp32 = false) {
  if (m.empty()) return VB_OK;
  void **dm = nullptr;
  int64_t *dld = nullptr;
  int32_t *dn = nullptr;
  UCHK(ctx->upload(&dm, m, true));
  UCHK(ctx->upload(&dld, ld, true));
  UCHK(ctx->upload(&dn, n, true));
  int mx = *std::max_element(n.begin(), n.end());
  if (transpose)
    CHK(transpose_sq(dm, dld, dn, (int)m.size(), mx, fp32, ctx->stream));
  else
    CHK(symmetrize(dm, dld, dn, (int)m.size(), mx, fp32, ctx->stream));
  return VB_OK;
}

static int check_info(vb_ctx *ctx, int count, int code, const char *what) {
  std::vector<int> h(count);
  CHK(hipMemcpyAsync(h.data(), ctx->info, count * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  CHK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < count; ++i)
    if (h[i] != 0)
      return ctx->fail(code, std::string(what) + ": pivot breakdown in block " + std::to_string(i) +
                                 " at column " + std::to_string(h[i] - 1));
  return VB_OK;
}


static void *x_block(vb_ctx *ctx, const SubH &S) {
  (void)ctx;
  return S.X;
}

// Householder QR with column pivoting of every entity's constraint rows.
static int primal_qr(vb_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const int nE = (int)ctx->ents.size();
  int rmax = 1;
  for (auto &H : ctx->ents) rmax = std::max(rmax, std::min(H.ncon, H.n));
  CHK(entity_qr(ctx->d_entdev, nE, rmax, ctx->opt.svd_tol, st));
  std::vector<int> rk(nE);
  if (nE) {
    CHK(hipMemcpyAsync(rk.data(), ctx->info + 4 * ctx->nS + 64, nE * sizeof(int),
                       hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
  }
  for (int e = 0; e < nE; ++e) ctx->ents[e].rank = rk[e];
  return VB_OK;
}

template <typename J>
static int upload_jobs(vb_ctx *ctx, J **d, const std::vector<J> &h) {
  UCHK(ctx->upload(d, h, true));
  return VB_OK;
}


// ---------------------------------------------------- predicted eigenpairs
// Buffers of one face for the predicted path: C (n x n), and where the exact
// path would put its eigenvectors (Z, n x mcap) and eigenvalues (lam).
struct PredFace {
  const double *C;
  int n;
  double *Z, *lam;
  int mcap;
};

// Warm-started Chebyshev-filtered subspace iteration on every face whose
// predicted count allows it.  The network's scores summed over a face give
// k; the block has b = max(k + 4, 1.3 k + 2) vectors (at most 64 and n/2),
// starting from the unit vectors of the b best-scored coordinates.  A pass
// applies a degree-20 Chebyshev filter damping [a, rho] (rho: the
// Gershgorin bound of C; a = 2 sigma in the first pass, then the largest
// Ritz value of the block, so that everything beyond the block is damped),
// orthonormalises, and takes Rayleigh-Ritz pairs (eigensolve of the b x b
// projection with the dense kernels).  Accepted
// when fewer than b - 2 Ritz values lie below sigma, every selected pair
// has residual <= 1e-6 rho, theta_t + r_t < sigma for the selected pairs
// and theta - r > sigma for the next one.  The residual bounds prove that
// an eigenvalue lies below sigma near each selected Ritz value (a symmetric
// matrix has an eigenvalue within the residual norm of every Ritz value);
// they do not prove that no other eigenvalue lies below sigma, since an
// eigenvector nearly orthogonal to the block is damped but not seen.  The
// count is therefore a heuristic: complete when the filter has reached
// every such eigenvector, which the two spare Ritz values above sigma and
// the filter's damping of everything beyond the block make likely, not
// certain.  Otherwise up to 6 passes, then the face falls back to the
// exact solve.
template <class GetFace>
static int predicted_eigs(vb_ctx *ctx, vb_mlp *pred, size_t nf_, GetFace get,
                          const std::vector<int64_t> &coff, const double *d_rho, double sigma,
                          std::vector<int> &path, std::vector<int> &kpred, std::vector<int> &passes,
                          std::vector<int> &hc) {
  hipStream_t st = ctx->stream;
  const int nf = (int)nf_;
  const int64_t ncoord = coff[nf];
  float *score = nullptr;
  UCHK(ctx->dalloc(&score, std::max<int64_t>(ncoord, 1), true));
  CHK(mlp_forward(pred->p, pred->mu, pred->sd, ctx->d_feat, ncoord, score, st));
  std::vector<float> hs(ncoord);
  std::vector<double> rho(nf);
  CHK(hipMemcpyAsync(hs.data(), score, ncoord * sizeof(float), hipMemcpyDeviceToHost, st));
  CHK(hipMemcpyAsync(rho.data(), d_rho, nf * sizeof(double), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  const double a = 2.0 * sigma;
  struct PF {
    int q, n, b;
    double e, c0, rho;
    int64_t o_y[3], o_u, o_v2, o_h, o_zh, o_d, o_e, o_tau, o_lam, o_res;
  };
  std::vector<PF> act;
  int64_t tot = 0;
  auto take = [&](int64_t c) {
    int64_t o = tot;
    tot += round_up(std::max<int64_t>(c, 1), 32);
    return o;
  };
  int max_b = 1, max_n = 1;
  for (int q = 0; q < nf; ++q) {
    const PredFace F = get(q);
    double ssum = 0.0;
    for (int64_t c = coff[q]; c < coff[q + 1]; ++c) ssum += hs[c];
    const int k = (int)std::lround(ssum);
    kpred[q] = k;
    const int b = std::max(k + 4, (int)std::ceil(1.3 * k) + 2);
    if (b > 64 || 2 * b > F.n || b > F.mcap || rho[q] <= a) continue;  // exact solve
    PF P{};
    P.q = q;
    P.n = F.n;
    P.b = b;
    P.rho = rho[q];
    P.e = 0.5 * (rho[q] - a);
    P.c0 = 0.5 * (rho[q] + a);
    for (int r = 0; r < 3; ++r) P.o_y[r] = take((int64_t)b * F.n);
    P.o_u = take((int64_t)b * F.n);
    P.o_v2 = take((int64_t)b * F.n);
    P.o_h = take((int64_t)b * b);
    P.o_zh = take((int64_t)b * b);
    P.o_d = take(b);
    P.o_e = take(b);
    P.o_tau = take(b);
    P.o_lam = take(b);
    P.o_res = take(b);
    act.push_back(P);
    max_b = std::max(max_b, b);
    max_n = std::max(max_n, F.n);
  }
  if (act.empty()) return VB_OK;
  const int na = (int)act.size();
  double *w = nullptr, *lr = nullptr;  // lr: per face 64 Ritz values then 64 residuals
  int *cntH = nullptr;
  UCHK(ctx->dalloc(&w, tot, true));
  UCHK(ctx->dalloc(&lr, (int64_t)na * 128, true));
  UCHK(ctx->dalloc(&cntH, na, true));
  CHK(hipMemsetAsync(w, 0, tot * sizeof(double), st));
  {  // starting blocks (b x n, ld b): unit vectors of the chosen coordinates
    std::vector<std::vector<double>> v0(na);
    for (int i = 0; i < na; ++i) {
      const PF &P = act[i];
      std::vector<int> idx(P.n);
      std::iota(idx.begin(), idx.end(), 0);
      if (pred->warm) {
        const float *sc = hs.data() + coff[P.q];
        std::partial_sort(idx.begin(), idx.begin() + P.b, idx.end(),
                          [&](int x, int y) { return sc[x] > sc[y] || (sc[x] == sc[y] && x < y); });
      } else {  // pseudo-random distinct coordinates (a fixed linear congruential shuffle)
        uint64_t st64 = 0x9e3779b97f4a7c15ull ^ (uint64_t)P.q;
        for (int t = P.n - 1; t > 0; --t) {
          st64 = st64 * 6364136223846793005ull + 1442695040888963407ull;
          std::swap(idx[t], idx[(int)((st64 >> 33) % (uint64_t)(t + 1))]);
        }
      }
      v0[i].assign((size_t)P.b * P.n, 0.0);
      for (int t = 0; t < P.b; ++t) v0[i][t + (size_t)idx[t] * P.b] = 1.0;
      CHK(hipMemcpyAsync(w + P.o_y[0], v0[i].data(), v0[i].size() * sizeof(double),
                         hipMemcpyHostToDevice, st));
    }
    CHK(hipStreamSynchronize(st));
  }
  const int deg = 20, max_pass = 6;
  std::vector<char> done(na, 0);
  for (int pass = 0; pass < max_pass; ++pass) {
    std::vector<int> live;
    for (int i = 0; i < na; ++i)
      if (!done[i]) live.push_back(i);
    if (live.empty()) break;
    // Chebyshev filter, three rotating blocks per face
    int cur = 0;
    for (int k = 0; k < deg; ++k) {
      std::vector<ChebJob> cj;
      std::vector<GemmJob<double>> gj;
      const int prev = (cur + 2) % 3, out = (cur + 1) % 3;
      for (int i : live) {
        const PF &P = act[i];
        const PredFace F = get(P.q);
        double *yc = w + P.o_y[cur], *yp = w + P.o_y[prev], *yo = w + P.o_y[out];
        if (k == 0) {
          cj.push_back({yc, nullptr, yo, P.b, P.n, -P.c0 / P.e, 0.0});
          gj.push_back({yc, F.C, yo, P.b, P.n, P.b, P.b, P.n, P.n, 0, 1.0 / P.e, 1.0});
        } else {
          cj.push_back({yc, yp, yo, P.b, P.n, -2.0 * P.c0 / P.e, -1.0});
          gj.push_back({yc, F.C, yo, P.b, P.n, P.b, P.b, P.n, P.n, 0, 2.0 / P.e, 1.0});
        }
      }
      ChebJob *dcj = nullptr;
      GemmJob<double> *dgj = nullptr;
      int rc = upload_jobs(ctx, &dcj, cj);
      if (!rc) rc = upload_jobs(ctx, &dgj, gj);
      if (rc) return rc;
      CHK(cheb_combine(dcj, (int)cj.size(), (int64_t)max_b * max_n, st));
      CHK(gemm_nt_batched<double>(dgj, (int)gj.size(), max_b, max_n, st));
      cur = out;
    }
    // orthonormalise, project, Rayleigh-Ritz
    std::vector<OrthJob> oj;
    std::vector<GemmJob<double>> gu, gh;
    std::vector<SymJob> sj;
    std::vector<EigJob> ej;
    std::vector<RitzJob> rj;
    for (size_t k = 0; k < live.size(); ++k) {
      const PF &P = act[live[k]];
      const PredFace F = get(P.q);
      double *V = w + P.o_y[cur];
      oj.push_back({V, P.b, P.n});
      gu.push_back({V, F.C, w + P.o_u, P.b, P.n, P.b, P.b, P.n, P.n, 0, 1.0, 0.0});
      gh.push_back({V, w + P.o_u, w + P.o_h, P.b, P.b, P.b, P.b, P.b, P.n, 0, 1.0, 0.0});
      sj.push_back({w + P.o_h, P.b, P.b});
      double *lam = lr + (int64_t)live[k] * 128, *res = lam + 64;
      ej.push_back({w + P.o_h, P.b, P.b, P.b, w + P.o_d, w + P.o_e, w + P.o_tau, w + P.o_zh, P.b,
                    lam, cntH + live[k], 2.0 * P.rho + 1.0});
      rj.push_back({V, w + P.o_u, w + P.o_zh, P.b, lam, P.b, P.n, F.Z, P.n, w + P.o_v2, res});
    }
    OrthJob *doj = nullptr;
    GemmJob<double> *dgu = nullptr, *dgh = nullptr;
    SymJob *dsj = nullptr;
    EigJob *dej = nullptr;
    RitzJob *drj = nullptr;
    int rc = upload_jobs(ctx, &doj, oj);
    if (!rc) rc = upload_jobs(ctx, &dgu, gu);
    if (!rc) rc = upload_jobs(ctx, &dgh, gh);
    if (!rc) rc = upload_jobs(ctx, &dsj, sj);
    if (!rc) rc = upload_jobs(ctx, &dej, ej);
    if (!rc) rc = upload_jobs(ctx, &drj, rj);
    if (rc) return rc;
    const int nl = (int)live.size();
    CHK(orth_rows(doj, nl, st));
    CHK(gemm_nt_batched<double>(dgu, nl, max_b, max_n, st));
    CHK(gemm_nt_batched<double>(dgh, nl, max_b, max_b, st));
    CHK(sym_average(dsj, nl, max_b, st));
    CHK(tridiag(dej, nl, max_b, st));
    CHK(tridiag_eig(dej, nl, max_b, max_b, st));
    CHK(back_transform(dej, nl, st));
    CHK(ritz(drj, nl, max_b, st));
    std::vector<double> hlr((size_t)na * 128);
    CHK(hipMemcpyAsync(hlr.data(), lr, hlr.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (size_t k = 0; k < live.size(); ++k) {
      PF &P = act[live[k]];
      const int q = P.q;
      const double *th = hlr.data() + (size_t)live[k] * 128, *res = th + 64;
      int kr = 0;
      while (kr < P.b && th[kr] < sigma) ++kr;
      passes[q] = pass + 1;
      if (kr >= P.b - 2) {  // no margin: the block may miss eigenvalues below sigma
        done[live[k]] = 1;
        path[q] = 2;
        continue;
      }
      double rmax = 0.0;
      bool separated = true;  // the selected Ritz values and the next one bracket sigma
      for (int t = 0; t < kr; ++t) {
        rmax = std::max(rmax, res[t]);
        separated = separated && th[t] + res[t] < sigma;
      }
      separated = separated && th[kr] - res[kr] > sigma;
      if (rmax <= 1e-6 * P.rho && separated) {
        done[live[k]] = 1;
        path[q] = 1;
        hc[q] = kr;
        if (kr > 0) {
          const PredFace F = get(q);
          CHK(hipMemcpyAsync(F.lam, lr + (int64_t)live[k] * 128, kr * sizeof(double),
                             hipMemcpyDeviceToDevice, st));
        }
      } else {  // next pass from the Ritz vectors, damping beyond the block
        const double an = th[P.b - 1];
        if (an > 1.02 * sigma && an < P.rho) {
          P.e = 0.5 * (P.rho - an);
          P.c0 = 0.5 * (P.rho + an);
        }
        CHK(hipMemcpyAsync(w + P.o_y[0], w + P.o_v2, (size_t)P.b * P.n * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
      }
    }
  }
  for (int i = 0; i < na; ++i)
    if (!done[i]) path[act[i].q] = 2;
  return VB_OK;
}

// Adaptive face constraints (Sec. 6), one pass over the faces in the bases
// of the given constraints.  Per face F (subdomains i, j), with n = the dual
// coordinates of F:
//  1. P_k = the transformed S_Gamma^(k) with F last (gathered from X, the
//     face's reflectors applied to its rows and columns): A_k = its dual
//     block; the partial LDL^T of P_k over every other coordinate leaves
//     At_k (the Schur complement onto F_Delta).
//  2. Parallel sums as Schur complements: the trailing block of
//     [[X+Y, Y], [Y, Y]] after n eliminations is X:Y (A: exact; At: the sum
//     shifted by 1e-13 max|diag| so that a common kernel of floating
//     neighbours stays factorable; the product X(..)^-1 Y annihilates it).
//  3. B = A_i:A_j = L L^T and W = L^-T from the LDL^T of [[B, .], [I, 0]];
//     C = W^T At_par W (two MFMA GEMMs), symmetrised.
//  4. C = Q T Q^T, eigenvalues of T below 1/theta by bisection, their
//     eigenvectors by inverse iteration, y = Q z.
//  5. New rows (A_i:A_j) psi = L y on F_Delta, embedded in the face block and
//     taken back to the face's own coordinates with T_F, unit norm, and
//     appended to the face's constraint rows.
static int adaptive_stage(vb_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const bool f32 = ctx->fp32;
  const double sigma = 1.0 / ctx->opt.adaptive_theta;
  struct Face {
    int e, nF, rank, nd;
    int s[2], off[2];
    int64_t ld2, o_qb, o_qa, o_qa2, o_q0, o_m, o_wt, o_t2, o_c, o_d, o_e, o_tau, o_z, o_lam, o_r;
    int mcap;
    double shift;
  };
  std::vector<Face> faces;
  for (int e = 0; e < (int)ctx->ents.size(); ++e) {
    EntH &H = ctx->ents[e];
    if (H.kind != VB_ENT_FACE || H.subs.size() != 2 || H.n - H.rank <= 0) continue;
    Face f{};
    f.e = e;
    f.nF = H.n;
    f.rank = H.rank;
    f.nd = H.n - H.rank;
    for (int k = 0; k < 2; ++k) {
      SubH &S = ctx->subs[H.subs[k]];
      f.s[k] = H.subs[k];
      int qq = (int)(std::find(S.ents.begin(), S.ents.end(), e) - S.ents.begin());
      f.off[k] = S.ent_off[qq];
    }
    faces.push_back(f);
  }
  if (faces.empty()) return VB_OK;
  const int nf = (int)faces.size();
  {  // the factorisation left S_Gamma^(k) in the lower triangle of X only
    std::vector<void *> m;
    std::vector<int64_t> ld;
    std::vector<int32_t> n;
    for (auto &S : ctx->subs) {
      m.push_back(x_block(ctx, S));
      ld.push_back(S.xld);
      n.push_back(S.ng + 1);
    }
    int rc = run_symm(ctx, m, ld, n, false, f32);
    if (rc) return rc;
  }
  // ---- per-face FP64 arena
  int64_t tot = 0;
  int max_nd = 0, max_2nd = 0;
  for (auto &f : faces) {
    const int n = f.nd;
    f.mcap = std::min(n, 256);
    f.ld2 = round_up(2 * n, 32);
    auto take = [&](int64_t cnt) {
      int64_t o = tot;
      tot += round_up(cnt, 32);
      return o;
    };
    f.o_qb = take(f.ld2 * 2 * n);
    f.o_qa = take(f.ld2 * 2 * n);
    f.o_qa2 = take(f.ld2 * 2 * n);
    f.o_q0 = take(f.ld2 * 2 * n);
    f.o_m = take(f.ld2 * 2 * n);
    f.o_wt = take((int64_t)n * n);
    f.o_t2 = take((int64_t)n * n);
    f.o_c = take((int64_t)n * n);
    f.o_d = take(n);
    f.o_e = take(n);
    f.o_tau = take(n);
    f.o_z = take((int64_t)n * f.mcap);
    f.o_lam = take(f.mcap);
    f.o_r = take((int64_t)f.nF * n);
    max_nd = std::max(max_nd, n);
    max_2nd = std::max(max_2nd, 2 * n);
  }
  double *ar = nullptr;
  UCHK(ctx->dalloc(&ar, tot, true));
  CHK(hipMemsetAsync(ar, 0, tot * sizeof(double), st));
  int *iinfo = nullptr;  // LDL pivot reports (2 per face for P, 4 for the pencil) + counts
  UCHK(ctx->dalloc(&iinfo, 7 * (int64_t)nf + 1, true));
  CHK(hipMemsetAsync(iinfo, 0, (7 * (int64_t)nf + 1) * sizeof(int), st));
  int *cnt = iinfo + 6 * nf;
  // ---- 1. P_k per face and side, in chunks bounded in memory
  {
    size_t fr = 0, totm = 0;
    CHK(hipMemGetInfo(&fr, &totm));
    fr += ctx->pool_unused_bytes();
    const double budget = std::min(32.0e9, 0.5 * (double)fr);
    size_t ci = 0;
    int32_t *d_dualidx = nullptr;  // [0, max_nd) shifted per job through the out pointer
    std::vector<int32_t> iota(std::max(max_nd, 1));
    std::iota(iota.begin(), iota.end(), 0);
    UCHK(ctx->upload(&d_dualidx, iota, true));
    double *pbuf = nullptr;
    size_t pcap = 0;
    while (ci < faces.size()) {
      size_t cj = ci;
      double bytes = 0.0;
      while (cj < faces.size()) {
        double b = 0.0;
        for (int k = 0; k < 2; ++k) {
          const SubH &S = ctx->subs[faces[cj].s[k]];
          b += 8.0 * (double)round_up(S.ng, 32) * S.ng;
        }
        if (cj > ci && bytes + b > budget) break;
        bytes += b;
        ++cj;
      }
      if ((size_t)bytes > pcap) {
        if (pbuf) CHK(hipStreamSynchronize(st));
        UCHK(ctx->dalloc(&pbuf, (size_t)(bytes / 8.0) + 64, true));
        pcap = (size_t)bytes;
      }
      std::vector<GatherJob> gp, ga0, ga1, gt0, gt1;
      std::vector<FaceTJob> ft;
      std::vector<LdlJob<double>> lj;
      std::vector<void *> tm;
      std::vector<int64_t> tld;
      std::vector<int32_t> tn;
      int64_t po = 0, invtot = 0;
      int maxg = 0, maxe = 0;
      for (size_t q = ci; q < cj; ++q) {
        const Face &f = faces[q];
        for (int k = 0; k < 2; ++k) {
          const SubH &S = ctx->subs[f.s[k]];
          const int ng = S.ng;
          const int64_t ldp = round_up(ng, 32);
          double *P = pbuf + po;
          po += ldp * ng;
          std::vector<int32_t> perm;
          perm.reserve(ng);
          for (int l = 0; l < ng; ++l)
            if (l < f.off[k] || l >= f.off[k] + f.nF) perm.push_back(l);
          for (int l = 0; l < f.nF; ++l) perm.push_back(f.off[k] + l);
          int32_t *d_perm = nullptr;
          UCHK(ctx->upload(&d_perm, perm, true));
          gp.push_back({x_block(ctx, S), S.xld, P, ldp, d_perm, d_perm, ng, ng, 1.0, 0, f32 ? 1 : 0, 0});
          ft.push_back({P, ldp, ng, ng - f.nF, ctx->d_entdev + f.e, +1});
          tm.push_back(P);
          tld.push_back(ldp);
          tn.push_back(ng);
          // dual block of P: rows/cols [ng - nd, ng)
          const double *Pd = P + (ng - f.nd) + (int64_t)(ng - f.nd) * ldp;
          double *QB = ar + f.o_qb, *QA = ar + f.o_qa;
          const int n = f.nd;
          if (k == 0) {
            ga0.push_back({Pd, ldp, QB, f.ld2, d_dualidx, d_dualidx, n, n, 1.0, 0, 0, 0});
            gt0.push_back({Pd, ldp, QA, f.ld2, d_dualidx, d_dualidx, n, n, 1.0, 0, 0, 0});
          } else {
            ga1.push_back({Pd, ldp, QB, f.ld2, d_dualidx, d_dualidx, n, n, 1.0, 1, 0, 0});
            ga1.push_back({Pd, ldp, QB + n, f.ld2, d_dualidx, d_dualidx, n, n, 1.0, 0, 0, 0});
            ga1.push_back({Pd, ldp, QB + n + (int64_t)n * f.ld2, f.ld2, d_dualidx, d_dualidx, n, n,
                           1.0, 0, 0, 0});
            gt1.push_back({Pd, ldp, QA, f.ld2, d_dualidx, d_dualidx, n, n, 1.0, 1, 0, 0});
            gt1.push_back({Pd, ldp, QA + n, f.ld2, d_dualidx, d_dualidx, n, n, 1.0, 0, 0, 0});
            gt1.push_back({Pd, ldp, QA + n + (int64_t)n * f.ld2, f.ld2, d_dualidx, d_dualidx, n,
                           n, 1.0, 0, 0, 0});
          }
          const int ee = ng - n;
          lj.push_back({P, ldp, ng, ee, ee, 0, nullptr, iinfo + 2 * q + k});
          invtot += (int64_t)((ee + NB - 1) / NB) * NB * NB;
          maxg = std::max(maxg, ng);
          maxe = std::max(maxe, ee);
        }
      }
      double *invs = nullptr;
      UCHK(ctx->dalloc(&invs, std::max<int64_t>(invtot, 1), true));
      int64_t io = 0;
      for (auto &J : lj) {
        J.invL = invs + io;
        io += (int64_t)((J.e + NB - 1) / NB) * NB * NB;
      }
      int rc = run_gather(ctx, gp, maxg, maxg);
      if (rc) return rc;
      FaceTJob *dft = nullptr;
      rc = upload_jobs(ctx, &dft, ft);
      if (rc) return rc;
      CHK(face_transform(dft, (int)ft.size(), maxg, st));
      rc = run_symm(ctx, tm, tld, tn, true, false);
      if (rc) return rc;
      CHK(face_transform(dft, (int)ft.size(), maxg, st));
      rc = run_gather(ctx, ga0, max_nd, max_nd);
      if (!rc) rc = run_gather(ctx, ga1, max_nd, max_nd);
      if (rc) return rc;
      rc = run_ldl(ctx, lj, maxg, maxe);
      if (rc) return rc;
      {  // At_k: lower triangle of the trailing block -> full
        std::vector<void *> m;
        std::vector<int64_t> ld;
        std::vector<int32_t> n;
        for (size_t t = 0; t < tm.size(); ++t) {
          const int nd = faces[ci + t / 2].nd;
          const int ng = tn[t];
          m.push_back((double *)tm[t] + (ng - nd) + (int64_t)(ng - nd) * tld[t]);
          ld.push_back(tld[t]);
          n.push_back(nd);
        }
        rc = run_symm(ctx, m, ld, n, false, false);
        if (rc) return rc;
      }
      rc = run_gather(ctx, gt0, max_nd, max_nd);
      if (!rc) rc = run_gather(ctx, gt1, max_nd, max_nd);
      if (rc) return rc;
      ci = cj;
    }
  }
  // traces of A_i + A_j and A_j (features of the learned predictor)
  double *tr_pre = nullptr, *tr_post = nullptr;
  UCHK(ctx->dalloc(&tr_pre, 2 * (int64_t)nf, true));
  UCHK(ctx->dalloc(&tr_post, 2 * (int64_t)nf, true));
  {
    std::vector<SymJob> tj;
    for (auto &f : faces) {
      tj.push_back({ar + f.o_qb, f.ld2, f.nd});
      tj.push_back({ar + f.o_qb + f.nd + (int64_t)f.nd * f.ld2, f.ld2, f.nd});
    }
    SymJob *dtj = nullptr;
    int rc = upload_jobs(ctx, &dtj, tj);
    if (rc) return rc;
    CHK(traces(dtj, (int)tj.size(), tr_pre, st));
  }
  // ---- 2. parallel sums.  At_i + At_j is singular when the two neighbours
  // float and share rigid-mode traces on F; in FP64 that common kernel comes
  // out as pivots of either sign at the level of the cancellation in At.
  // Faces whose unshifted sum breaks down are factorised again from a
  // pristine copy with the sum shifted by 1e-13, 1e-11, ... up to 1e-1 times
  // max|diag| (the first that factorises is kept and reported); the kernel
  // is annihilated by the outer factors of X (X+Y)^-1 Y either way.
  {
    std::vector<LdlJob<double>> lj;
    std::vector<GatherJob> cp;
    int32_t *d_ii = nullptr;
    {
      std::vector<int32_t> iota(std::max(max_2nd, 1));
      std::iota(iota.begin(), iota.end(), 0);
      UCHK(ctx->upload(&d_ii, iota, true));
    }
    int64_t invtot = 0;
    for (auto &f : faces) {
      f.shift = 0.0;
      invtot += 3 * (int64_t)((f.nd + NB - 1) / NB) * NB * NB;
      cp.push_back({ar + f.o_qa, f.ld2, ar + f.o_q0, f.ld2, d_ii, d_ii, 2 * f.nd, 2 * f.nd, 1.0,
                    0, 0, 0});
    }
    int rc = run_gather(ctx, cp, max_2nd, max_2nd);
    if (rc) return rc;
    double *invs = nullptr;
    UCHK(ctx->dalloc(&invs, std::max<int64_t>(invtot, 1), true));
    double *invr = nullptr;  // scratch of the retries (one panel set per face)
    UCHK(ctx->dalloc(&invr, std::max<int64_t>(invtot / 3, 1), true));
    int64_t io = 0;
    std::vector<int64_t> roff(nf);
    {
      int64_t ro = 0;
      for (int q = 0; q < nf; ++q) {
        const Face &f = faces[q];
        const int64_t per = (int64_t)((f.nd + NB - 1) / NB) * NB * NB;
        lj.push_back({ar + f.o_qb, f.ld2, 2 * f.nd, f.nd, f.nd, 0, invs + io, iinfo + 2 * nf + q});
        io += per;
        lj.push_back({ar + f.o_qa, f.ld2, 2 * f.nd, f.nd, f.nd, 0, invs + io, iinfo + 3 * nf + q});
        io += per;
        roff[q] = ro;
        ro += per;
      }
    }
    rc = run_ldl(ctx, lj, max_2nd, max_nd);
    if (rc) return rc;
    std::vector<int> hq(nf);
    CHK(hipMemcpyAsync(hq.data(), iinfo + 3 * nf, nf * sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    CHK(hipMemsetAsync(iinfo + 3 * nf, 0, nf * sizeof(int), st));
    // FP64 factors have needed at most 1e-11.  The FP32 factors of the mixed
    // path carry FP32 error amplified by the local conditioning into At (at
    // a viscosity contrast inside a subdomain, up to percent level), so the
    // ladder continues to 1e-1: a shifted face only gets a rougher set of
    // rows, and any primal enrichment keeps lambda_min >= 1.
    static const double ladder[] = {1e-13, 1e-11, 1e-9, 1e-7, 1e-5, 1e-3, 1e-1};
    std::string diag = "unshifted failures:";
    {
      int nfail = 0;
      for (int q = 0; q < nf; ++q) nfail += hq[q] != 0;
      diag += " " + std::to_string(nfail);
    }
    std::vector<int> firstcol(hq);
    for (double sh : ladder) {
      std::vector<int> todo;
      for (int q = 0; q < nf; ++q)
        if (hq[q]) todo.push_back(q);
      if (todo.empty()) break;
      std::vector<GatherJob> cp2;
      std::vector<SymJob> sj;
      std::vector<LdlJob<double>> lj2;
      for (int q : todo) {
        Face &f = faces[q];
        cp2.push_back({ar + f.o_q0, f.ld2, ar + f.o_qa2, f.ld2, d_ii, d_ii, 2 * f.nd, 2 * f.nd, 1.0,
                       0, 0, 0});
        sj.push_back({ar + f.o_qa2, f.ld2, f.nd});
        lj2.push_back({ar + f.o_qa2, f.ld2, 2 * f.nd, f.nd, f.nd, 0, invr + roff[q],
                       iinfo + 5 * nf + q});
        f.o_qa = f.o_qa2;
        f.shift = sh;
      }
      CHK(hipMemsetAsync(iinfo + 5 * nf, 0, nf * sizeof(int), st));
      rc = run_gather(ctx, cp2, max_2nd, max_2nd);
      if (rc) return rc;
      SymJob *dsj = nullptr;
      rc = upload_jobs(ctx, &dsj, sj);
      if (rc) return rc;
      CHK(shift_diag(dsj, (int)sj.size(), sh, st));
      rc = run_ldl(ctx, lj2, max_2nd, max_nd);
      if (rc) return rc;
      CHK(hipMemcpyAsync(hq.data(), iinfo + 5 * nf, nf * sizeof(int), hipMemcpyDeviceToHost, st));
      CHK(hipStreamSynchronize(st));
      int nfail = 0;
      for (int q = 0; q < nf; ++q) nfail += hq[q] != 0;
      char buf[64];
      snprintf(buf, sizeof buf, ", after shift %.0e: %d", sh, nfail);
      diag += buf;
    }
    CHK(hipMemsetAsync(iinfo + 5 * nf, 0, nf * sizeof(int), st));
    for (int q = 0; q < nf; ++q)
      if (hq[q])
        return ctx->fail(VB_ERR_NOT_SPD,
                         "adaptive: parallel sum of the face Schur complements not factorisable "
                         "with a shift up to 1e-1 max|diag| (face entity " +
                         std::to_string(faces[q].e) + ", subdomains " +
                         std::to_string(faces[q].s[0]) + "/" + std::to_string(faces[q].s[1]) +
                         ", unshifted breakdown at column " + std::to_string(firstcol[q] - 1) +
                         " of " + std::to_string(faces[q].nd) + ", last at column " +
                         std::to_string(hq[q] - 1) + "; " + diag + ")");
    // ---- 3. B = L L^T, W = L^-T; C = W^T At_par W
    std::vector<GatherJob> gm;
    std::vector<DiagJob> dm;
    std::vector<LdlJob<double>> lm;
    std::vector<void *> sm;
    std::vector<int64_t> sld;
    std::vector<int32_t> sn;
    std::vector<GatherJob> gw;
    std::vector<GemmJob<double>> g1, g2;
    int32_t *d_dualidx = nullptr;
    std::vector<int32_t> iota(std::max(max_nd, 1));
    std::iota(iota.begin(), iota.end(), 0);
    UCHK(ctx->upload(&d_dualidx, iota, true));
    for (int q = 0; q < nf; ++q) {
      const Face &f = faces[q];
      const int n = f.nd;
      double *QB = ar + f.o_qb, *QA = ar + f.o_qa, *M = ar + f.o_m;
      gm.push_back({QB + n + (int64_t)n * f.ld2, f.ld2, M, f.ld2, d_dualidx, d_dualidx, n, n, 1.0,
                    0, 0, 0});
      dm.push_back({M, f.ld2, n, 0, n, 1.0, 0});
      lm.push_back({M, f.ld2, 2 * n, n, n, 0, invs + io, iinfo + 4 * nf + q, 0.0, n});
      io += (int64_t)((n + NB - 1) / NB) * NB * NB;
      sm.push_back(QA + n + (int64_t)n * f.ld2);
      sld.push_back(f.ld2);
      sn.push_back(n);
      // W^T[i][j] = M[n + j][i]: rows i -> i * ld2, columns j -> n + j (ldi 1)
      std::vector<int32_t> ri(n), cj(n);
      for (int a = 0; a < n; ++a) {
        ri[a] = (int32_t)(a * f.ld2);
        cj[a] = n + a;
      }
      int32_t *d_ri = nullptr, *d_cj = nullptr;
      UCHK(ctx->upload(&d_ri, ri, true));
      UCHK(ctx->upload(&d_cj, cj, true));
      gw.push_back({M, 1, ar + f.o_wt, n, d_ri, d_cj, n, n, 1.0, 0, 0, 0});
      const double *Ap = QA + n + (int64_t)n * f.ld2;
      g1.push_back({ar + f.o_wt, Ap, ar + f.o_t2, n, f.ld2, n, n, n, n, 0, 1.0, 0.0});
      g2.push_back({ar + f.o_t2, ar + f.o_wt, ar + f.o_c, n, n, n, n, n, n, 0, 1.0, 0.0});
    }
    rc = run_gather(ctx, gm, max_nd, max_nd);
    if (!rc) rc = run_diag(ctx, dm, max_nd);
    if (!rc) rc = run_ldl(ctx, lm, max_2nd, max_nd);
    if (!rc) rc = run_symm(ctx, sm, sld, sn, false, false);
    if (!rc) rc = run_gather(ctx, gw, max_nd, max_nd);
    if (rc) return rc;
    std::vector<int> h(6 * nf);
    CHK(hipMemcpyAsync(h.data(), iinfo, 6 * nf * sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    static const char *what[] = {"Schur complement onto F_Delta", "parallel sum of the dual minors",
                                 "parallel sum of the Schur complements", "Cholesky of the pencil",
                                 "shifted parallel sum of the Schur complements"};
    for (int q = 0; q < 6 * nf; ++q)
      if (h[q]) {
        const int face = q < 2 * nf ? q / 2 : q % nf;
        const int stage = q < 2 * nf ? 0 : q / nf - 1;
        return ctx->fail(VB_ERR_NOT_SPD, std::string("adaptive: breakdown in the ") + what[stage] +
                                             " of face entity " + std::to_string(faces[face].e));
      }
    GemmJob<double> *dg1 = nullptr, *dg2 = nullptr;
    rc = upload_jobs(ctx, &dg1, g1);
    if (!rc) rc = upload_jobs(ctx, &dg2, g2);
    if (rc) return rc;
    CHK(gemm_nt_batched<double>(dg1, nf, max_nd, max_nd, st));
    CHK(gemm_nt_batched<double>(dg2, nf, max_nd, max_nd, st));
    std::vector<SymJob> cj;
    for (auto &f : faces) cj.push_back({ar + f.o_c, f.nd, f.nd});
    SymJob *dcj = nullptr;
    rc = upload_jobs(ctx, &dcj, cj);
    if (rc) return rc;
    CHK(sym_average(dcj, nf, max_nd, st));
  }
  // ---- 4. eigenpairs below sigma
  // 4a. traces of the parallel sums and per-coordinate features of C
  {
    std::vector<SymJob> tj;
    for (auto &f : faces) {
      tj.push_back({ar + f.o_qa + f.nd + (int64_t)f.nd * f.ld2, f.ld2, f.nd});
      tj.push_back({ar + f.o_qb + f.nd + (int64_t)f.nd * f.ld2, f.ld2, f.nd});
    }
    SymJob *dtj = nullptr;
    int rc = upload_jobs(ctx, &dtj, tj);
    if (rc) return rc;
    CHK(traces(dtj, (int)tj.size(), tr_post, st));
  }
  std::vector<int64_t> coff(nf + 1, 0);
  for (int q = 0; q < nf; ++q) coff[q + 1] = coff[q] + faces[q].nd;
  const int64_t ncoord = coff[nf];
  UCHK(ctx->dalloc(&ctx->d_feat, ncoord * MLP_F));
  UCHK(ctx->dalloc(&ctx->d_lab, ncoord));
  CHK(hipMemsetAsync(ctx->d_lab, 0xff, ncoord * sizeof(float), st));  // NaN: no label
  ctx->n_coord = ncoord;
  double *d_rho = nullptr;
  UCHK(ctx->dalloc(&d_rho, nf, true));
  {
    std::vector<FeatJob> fj0(nf);
    for (int q = 0; q < nf; ++q) {
      const Face &f = faces[q];
      fj0[q] = {ar + f.o_c, f.nd, f.nd, sigma, tr_post + 2 * q, tr_pre + 2 * q,
                ctx->d_feat + coff[q] * MLP_F, d_rho + q};
    }
    FeatJob *dfj = nullptr;
    int rc = upload_jobs(ctx, &dfj, fj0);
    if (rc) return rc;
    CHK(face_features(dfj, nf, st));
  }
  std::vector<int> path(nf, 0), kpred(nf, -1), passes(nf, 0), hc(nf, 0);
  // 4b. predicted path: warm-started Chebyshev-filtered subspace iteration
  vb_mlp *pred = (vb_mlp *)ctx->opt.predictor;
  if (pred && pred->trained) {
    int rc = predicted_eigs(ctx, pred, faces.size(), [&](int q) -> PredFace {
      const Face &f = faces[q];
      return PredFace{ar + f.o_c, f.nd, ar + f.o_z, ar + f.o_lam, f.mcap};
    }, coff, d_rho, sigma, path, kpred, passes, hc);
    if (rc) return rc;
  }
  // 4c. exact dense eigensolve for the other faces
  std::vector<EigJob> ej;
  std::vector<int> eq;
  int max_mcap = 1, max_nde = 1;
  for (int q = 0; q < nf; ++q) {
    if (path[q] == 1) continue;
    const Face &f = faces[q];
    ej.push_back({ar + f.o_c, f.nd, f.nd, 0, ar + f.o_d, ar + f.o_e, ar + f.o_tau, ar + f.o_z, f.nd,
                  ar + f.o_lam, cnt + q, sigma});
    eq.push_back(q);
    max_mcap = std::max(max_mcap, f.mcap);
    max_nde = std::max(max_nde, f.nd);
  }
  EigJob *dej = nullptr;
  int rc = 0;
  if (!ej.empty()) {
    rc = upload_jobs(ctx, &dej, ej);
    if (rc) return rc;
    CHK(tridiag(dej, (int)ej.size(), max_nde, st));
    CHK(tridiag_eig(dej, (int)ej.size(), max_nde, max_mcap, st));
    std::vector<int> hx(nf);
    CHK(hipMemcpyAsync(hx.data(), cnt, nf * sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (size_t k = 0; k < eq.size(); ++k) {
      const int q = eq[k];
      const Face &f = faces[q];
      const int m = hx[q];
      if (m > f.mcap && m < f.nd)
        return ctx->fail(VB_ERR_ARG, "adaptive: " + std::to_string(m) +
                                         " eigenvalues below 1/theta on face entity " +
                                         std::to_string(f.e) + " (at most 256 supported)");
      hc[q] = m;
      ej[k].ncols = (m >= f.nd) ? 0 : m;
    }
    rc = upload_jobs(ctx, &dej, ej);
    if (rc) return rc;
    CHK(back_transform(dej, (int)ej.size(), st));
    // 4d. labels of the exactly solved faces
    std::vector<LabelJob> lb;
    for (int q : eq) {
      const Face &f = faces[q];
      lb.push_back({ar + f.o_z, f.nd, f.nd, std::min(hc[q], f.mcap), hc[q] >= f.nd ? 1 : 0,
                    ctx->d_lab + coff[q]});
    }
    LabelJob *dlb = nullptr;
    rc = upload_jobs(ctx, &dlb, lb);
    if (rc) return rc;
    CHK(face_labels(dlb, (int)lb.size(), st));
  }
  std::vector<RowJob> rj, rn;
  std::vector<FaceTJob> fj;
  std::vector<DiagJob> dfull;
  int max_cols = 0, max_nF = 0;
  for (int q = 0; q < nf; ++q) {
    Face &f = faces[q];
    const int m = hc[q];
    const bool full = (m >= f.nd);
    const int cols = full ? f.nd : m;
    double *R = ar + f.o_r;  // nF x cols, rows [0, rank) stay zero
    if (cols > 0) {
      if (full)
        dfull.push_back({R, f.nF, f.rank, 0, f.nd, 1.0, 0});
      else
        rj.push_back({ar + f.o_m, f.ld2, f.nd, m, ar + f.o_z, f.nd, R + f.rank, f.nF});
      fj.push_back({R, f.nF, cols, 0, ctx->d_entdev + f.e, -1});
      rn.push_back({nullptr, 0, f.nF, cols, nullptr, 0, R, f.nF});
      max_cols = std::max(max_cols, cols);
      max_nF = std::max(max_nF, f.nF);
    }
  }
  if (!rj.empty()) {
    RowJob *drj = nullptr;
    rc = upload_jobs(ctx, &drj, rj);
    if (rc) return rc;
    CHK(lower_times(drj, (int)rj.size(), max_nd, max_cols, st));
  }
  rc = run_diag(ctx, dfull, max_nd);
  if (rc) return rc;
  if (!fj.empty()) {
    FaceTJob *dfj = nullptr;
    RowJob *drn = nullptr;
    rc = upload_jobs(ctx, &dfj, fj);
    if (!rc) rc = upload_jobs(ctx, &drn, rn);
    if (rc) return rc;
    CHK(face_transform(dfj, (int)fj.size(), max_cols, st));
    CHK(normalize_cols(drn, (int)rn.size(), max_cols, st));
  }
  // ---- 5. append the rows; record the faces: each face's rows (nF x cols)
  // and eigenvalues are copied into one pinned host buffer, one sync
  std::vector<int64_t> hoff(nf + 1, 0);
  for (int q = 0; q < nf; ++q) {
    const Face &f = faces[q];
    const int m = hc[q];
    const int cols = (m >= f.nd) ? f.nd : m;
    const int neig = (m >= f.nd) ? 0 : m;
    hoff[q + 1] = hoff[q] + (int64_t)f.nF * cols + neig;
  }
  double *hbuf = nullptr;
  CHK(hipHostMalloc((void **)&hbuf, std::max<int64_t>(hoff[nf], 1) * sizeof(double),
                    hipHostMallocDefault));
  struct HostFree {
    double *p;
    ~HostFree() { (void)hipHostFree(p); }
  } hb_guard{hbuf};
  for (int q = 0; q < nf; ++q) {
    const Face &f = faces[q];
    const int m = hc[q];
    const int cols = (m >= f.nd) ? f.nd : m;
    const int neig = (m >= f.nd) ? 0 : m;
    if (cols > 0)
      CHK(hipMemcpyAsync(hbuf + hoff[q], ar + f.o_r, (size_t)f.nF * cols * sizeof(double),
                         hipMemcpyDeviceToHost, st));
    if (neig > 0)
      CHK(hipMemcpyAsync(hbuf + hoff[q] + (int64_t)f.nF * cols, ar + f.o_lam, neig * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  }
  CHK(hipStreamSynchronize(st));
  int64_t extra = 0;
  for (int q = 0; q < nf; ++q) {
    const Face &f = faces[q];
    const int m = hc[q];
    const int cols = (m >= f.nd) ? f.nd : m;
    if (cols > 0) extra += (int64_t)(ctx->ents[f.e].ncon + cols) * f.nF;
  }
  for (int q = 0; q < nf; ++q) {
    Face &f = faces[q];
    EntH &H = ctx->ents[f.e];
    const int m = hc[q];
    const bool full = (m >= f.nd);
    const int cols = full ? f.nd : m;
    vb_face_info fi{f.e, f.s[0], f.s[1], f.nd, m, kpred[q], path[q], passes[q], f.shift};
    ctx->face_info.push_back(fi);
    const double *hr = hbuf + hoff[q];
    if (!full && m > 0)
      ctx->face_eigs.insert(ctx->face_eigs.end(), hr + (int64_t)f.nF * cols, hr + (int64_t)f.nF * cols + m);
    if (cols == 0) continue;
    if (H.ncon + cols > 1024)
      return ctx->fail(VB_ERR_ARG, "adaptive: more than 1024 constraint rows on face entity " +
                                       std::to_string(f.e));
    // R is nF x cols column-major: column c is row c of the constraint block
    H.con.insert(H.con.end(), hr, hr + (int64_t)f.nF * cols);
    H.ncon += cols;
  }
  // device copies of the grown constraint blocks and their QR workspace:
  // one allocation each for all faces
  {
    int64_t ccon = 0, cv = 0, ct = 0, cw = 0;
    for (int q = 0; q < nf; ++q) {
      if (hc[q] == 0) continue;
      const EntH &H = ctx->ents[faces[q].e];
      const int rmax = std::max(1, std::min(H.ncon, H.n));
      ccon += round_up((int64_t)H.ncon * H.n, 32);
      cv += round_up((int64_t)H.n * rmax, 32);
      ct += round_up(rmax, 32);
      cw += round_up((int64_t)H.n * std::max(1, H.ncon), 32);
    }
    double *dcon = nullptr, *dv = nullptr, *dt = nullptr, *dw = nullptr;
    UCHK(ctx->dalloc(&dcon, std::max<int64_t>(ccon, 1)));
    UCHK(ctx->dalloc(&dv, std::max<int64_t>(cv, 1)));
    UCHK(ctx->dalloc(&dt, std::max<int64_t>(ct, 1)));
    UCHK(ctx->dalloc(&dw, std::max<int64_t>(cw, 1)));
    std::vector<double> hcon(std::max<int64_t>(ccon, 1));
    int64_t oc = 0, ov = 0, ot = 0, ow = 0;
    for (int q = 0; q < nf; ++q) {
      if (hc[q] == 0) continue;
      EntH &H = ctx->ents[faces[q].e];
      const int rmax = std::max(1, std::min(H.ncon, H.n));
      std::copy(H.con.begin(), H.con.end(), hcon.begin() + oc);
      H.d_con = dcon + oc;
      H.d_V = dv + ov;
      H.d_tau = dt + ot;
      H.d_work = dw + ow;
      oc += round_up((int64_t)H.ncon * H.n, 32);
      ov += round_up((int64_t)H.n * rmax, 32);
      ot += round_up(rmax, 32);
      ow += round_up((int64_t)H.n * std::max(1, H.ncon), 32);
      EntDev &D = ctx->entdev[faces[q].e];
      D.n_con = H.ncon;
      D.con = H.d_con;
      D.V = H.d_V;
      D.tau = H.d_tau;
      D.work = H.d_work;
    }
    CHK(hipMemcpy(dcon, hcon.data(), hcon.size() * sizeof(double), hipMemcpyHostToDevice));
    (void)extra;
  }
  CHK(hipMemcpyAsync(ctx->d_entdev, ctx->entdev.data(), ctx->entdev.size() * sizeof(EntDev),
                     hipMemcpyHostToDevice, st));
  CHK(hipStreamSynchronize(st));
  return VB_OK;
}

static int autotune_gemvs(vb_ctx *ctx);

static int64_t inv_size(const SubH &S) { return (int64_t)((S.e + NB - 1) / NB) * NB * NB; }

// Mixed precision: the subdomains in `bad` (ascending), whose FP32 Dirichlet
// factorisation broke down, factored again in FP64 in temporary buffers:
// densified and their pressures split as before -- in the two-level scheme
// every front of theirs first, its trailing block scattered into the second
// level -- with only wrong-signed or zero pivots failing.  The FP64 factors,
// inverse diagonal blocks and Schur complements are then rounded into the
// FP32 storage that every later step reads.
static int retry_fp64(vb_ctx *ctx, const std::vector<int> &bad) {
  hipStream_t st = ctx->stream;
  const int nb = (int)bad.size();
  std::vector<int> frs;  // fronts of the bad subdomains, subdomain by subdomain
  if (ctx->nd)
    for (int s : bad)
      for (int b = 0; b < ctx->subs[s].nbox; ++b) frs.push_back(ctx->subs[s].first_front + b);
  const int nfr = (int)frs.size();
  int *d_info = nullptr;
  UCHK(ctx->dalloc(&d_info, (size_t)(nb + nfr), true));
  CHK(hipMemsetAsync(d_info, 0, (nb + nfr) * sizeof(int), st));
  auto check = [&](int off, int cnt, const std::vector<int> &ids, const char *where) -> int {
    std::vector<int> h(cnt);
    CHK(hipMemcpyAsync(h.data(), d_info + off, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (int q = 0; q < cnt; ++q)
      if (h[q])
        return ctx->fail(VB_ERR_NOT_SPD,
                         "Dirichlet factorisation (subdomain index): pivot breakdown in block " +
                             std::to_string(ids[q]) + " at column " + std::to_string(h[q] - 1) + where +
                             " in FP32 and again in its FP64 retry");
    return VB_OK;
  };
  std::vector<void *> temps;
  // ---- first level: the fronts
  std::vector<int64_t> foff(nfr + 1, 0), fioff(nfr + 1, 0);
  double *fw = nullptr, *fi = nullptr;
  if (nfr) {
    std::vector<SubDev> dv(nfr);
    std::vector<LdlJob<double>> jobs;
    std::vector<int> ids;
    int mxN = 0, mxe = 0;
    for (int q = 0; q < nfr; ++q) {
      const SubH &F = ctx->fronts[frs[q]].S;
      foff[q + 1] = foff[q] + F.ld * F.N;
      fioff[q + 1] = fioff[q] + inv_size(F);
    }
    UCHK(ctx->dalloc(&fw, (size_t)foff[nfr], true));
    UCHK(ctx->dalloc(&fi, (size_t)fioff[nfr], true));
    temps.push_back(fw);
    temps.push_back(fi);
    for (int q = 0; q < nfr; ++q) {
      const SubH &F = ctx->fronts[frs[q]].S;
      dv[q] = ctx->frdev[frs[q]];
      dv[q].W = fw + foff[q];
      jobs.push_back({fw + foff[q], F.ld, F.N, F.e, F.nv, 0, fi + fioff[q], d_info + nb + q});
      ids.push_back(ctx->fronts[frs[q]].sub);
      mxN = std::max(mxN, F.N);
      mxe = std::max(mxe, F.e);
    }
    SubDev *d_dv = nullptr;
    UCHK(ctx->upload(&d_dv, dv, true));
    CHK(hipMemsetAsync(fw, 0, foff[nfr] * sizeof(double), st));
    CHK(densify(d_dv, nfr, ctx->max_nf_csr, false, st));
    CHK(house_pressure(d_dv, nfr, mxN, false, st));
    int rc = run_ldl(ctx, jobs, mxN, mxe, false, ctx->fac_nb[0], ctx->fac_sb[0]);
    if (!rc) rc = check(nb, nfr, ids, " of a sub-box");
    if (rc) return rc;
  }
  // ---- the local matrices (two-level: the second level)
  std::vector<int64_t> woff(nb + 1, 0), ioff(nb + 1, 0);
  for (int q = 0; q < nb; ++q) {
    const SubH &S = ctx->subs[bad[q]];
    woff[q + 1] = woff[q] + S.ld * S.N;
    ioff[q + 1] = ioff[q] + inv_size(S);
  }
  double *w = nullptr, *wi = nullptr;
  UCHK(ctx->dalloc(&w, (size_t)woff[nb], true));
  UCHK(ctx->dalloc(&wi, (size_t)ioff[nb], true));
  temps.push_back(w);
  temps.push_back(wi);
  {
    std::vector<SubDev> dv(nb);
    std::vector<LdlJob<double>> jobs;
    int mxN = 0, mxe = 0;
    for (int q = 0; q < nb; ++q) {
      const SubH &S = ctx->subs[bad[q]];
      dv[q] = ctx->subdev[bad[q]];
      dv[q].W = w + woff[q];
      jobs.push_back({w + woff[q], S.ld, S.N, S.e, S.nv, 0, wi + ioff[q], d_info + q});
      mxN = std::max(mxN, S.N);
      mxe = std::max(mxe, S.e);
    }
    SubDev *d_dv = nullptr;
    UCHK(ctx->upload(&d_dv, dv, true));
    CHK(hipMemsetAsync(w, 0, woff[nb] * sizeof(double), st));
    CHK(densify(d_dv, nb, ctx->max_n_csr, false, st));
    if (ctx->nd) {  // the fronts' trailing blocks, in sub-box order as in the FP32 pass
      std::vector<int> first(nb);
      for (int q = 0, c = 0; q < nb; ++q) {
        first[q] = c;
        c += ctx->subs[bad[q]].nbox;
      }
      for (int b = 0; b < ctx->max_nbox; ++b) {
        std::vector<FrontJob> fj;
        for (int q = 0; q < nb; ++q) {
          const SubH &S = ctx->subs[bad[q]];
          if (b >= S.nbox) continue;
          const FrontH &F = ctx->fronts[S.first_front + b];
          const int fq = first[q] + b;
          FrontJob J{};
          J.Wf = fw + foff[fq];
          J.ldf = F.S.ld;
          J.e = F.S.e;
          J.m = F.S.ng + 2;
          J.W2 = w + woff[q];
          J.ld2 = S.ld;
          J.map = F.d_map;
          J.gamma = F.gamma;
          fj.push_back(J);
        }
        if (fj.empty()) continue;
        FrontJob *d_fj = nullptr;
        UCHK(ctx->upload(&d_fj, fj, true));
        CHK(front_scatter(d_fj, (int)fj.size(), ctx->max_fm, false, st));
      }
    }
    CHK(house_pressure(d_dv, nb, mxN, false, st));
    const int lv = ctx->nd ? 1 : 0;  // the inverse blocks must match the sweeps' panel width
    int rc = run_ldl(ctx, jobs, mxN, mxe, false, ctx->fac_nb[lv], ctx->fac_sb[lv]);
    if (!rc) rc = check(0, nb, bad, ctx->nd ? " of its separator level" : "");
    if (rc) return rc;
  }
  // ---- rounded into the FP32 storage; the FP32 pass's flags cleared
  for (int q = 0; q < nfr; ++q) {
    const SubH &F = ctx->fronts[frs[q]].S;
    CHK(cast_to_f32(fw + foff[q], (float *)ctx->FW + F.W_off, F.ld * F.N, st));
    CHK(cast_to_f32(fi + fioff[q], (float *)ctx->invLf + F.inv_off, inv_size(F), st));
    CHK(hipMemsetAsync(ctx->info_f + frs[q], 0, sizeof(int), st));
  }
  for (int q = 0; q < nb; ++q) {
    const SubH &S = ctx->subs[bad[q]];
    CHK(cast_to_f32(w + woff[q], (float *)ctx->W + S.W_off, S.ld * S.N, st));
    CHK(cast_to_f32(wi + ioff[q], (float *)ctx->invL + S.inv_off, inv_size(S), st));
    CHK(hipMemsetAsync(ctx->info + bad[q], 0, sizeof(int), st));
  }
  for (void *t : temps) ctx->free_setup_early(t);
  ctx->fp64_retried.insert(ctx->fp64_retried.end(), bad.begin(), bad.end());
  return VB_OK;
}

// Dense bordered local matrices of subdomains [s0, s1) (one wave sharing W):
// densify the CSR, rotate the pressures, partial LDL^T of the interior
// columns.  Deterministic: a wave factorised again reproduces its factors.
static int factor_wave(vb_ctx *ctx, int s0, int s1, bool timed) {
  hipStream_t st = ctx->stream;
  const bool f32 = ctx->fp32;
  int64_t wend = 0;
  int mxN = 0, mxe = 0;
  for (int s = s0; s < s1; ++s) {
    const SubH &S = ctx->subs[s];
    wend = std::max(wend, S.W_off + S.ld * S.N);
    mxN = std::max(mxN, S.N);
    mxe = std::max(mxe, S.e);
  }
  const int64_t w0 = ctx->subs[s0].W_off;
  auto prepare = [&]() -> int {
    CHK(hipMemsetAsync((char *)ctx->W + w0 * ctx->wsz, 0, (wend - w0) * ctx->wsz, st));
    CHK(densify(ctx->d_subdev + s0, s1 - s0, ctx->max_n_csr, f32, st));
    CHK(house_pressure(ctx->d_subdev + s0, s1 - s0, mxN, f32, st));
    CHK(hipMemsetAsync(ctx->info + s0, 0, (s1 - s0) * sizeof(int), st));
    return VB_OK;
  };
  int rc = prepare();
  if (rc) return rc;
  if (f32) {
    std::vector<LdlJob<float>> jobs;
    for (int s = s0; s < s1; ++s) {
      SubH &S = ctx->subs[s];
      jobs.push_back({(float *)ctx->W + S.W_off, S.ld, S.N, S.e, S.nv, 0,
                      (float *)ctx->invL + S.inv_off, ctx->info + s, ctx->opt.fp32_pivot_min});
    }
    rc = tuned_ldl(ctx, 0, jobs, mxN, mxe, timed, prepare);
  } else {
    std::vector<LdlJob<double>> jobs;
    for (int s = s0; s < s1; ++s) {
      SubH &S = ctx->subs[s];
      jobs.push_back({(double *)ctx->W + S.W_off, S.ld, S.N, S.e, S.nv, 0,
                      (double *)ctx->invL + S.inv_off, ctx->info + s});
    }
    rc = tuned_ldl(ctx, 0, jobs, mxN, mxe, timed, prepare);
  }
  if (rc) return rc;
  std::vector<int> h(s1 - s0), bad;
  CHK(hipMemcpyAsync(h.data(), ctx->info + s0, h.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  for (size_t q = 0; q < h.size(); ++q) {
    if (!h[q]) continue;
    if (!f32)
      return ctx->fail(VB_ERR_NOT_SPD, "Dirichlet factorisation (subdomain index): pivot breakdown in block " +
                                           std::to_string(s0 + (int)q) + " at column " +
                                           std::to_string(h[q] - 1));
    bad.push_back(s0 + (int)q);
  }
  return bad.empty() ? VB_OK : retry_fp64(ctx, bad);
}

// The two-level factorisation: every front (sub-box) densified, its
// pressures split and factored up to its kept coordinate; then every
// subdomain's second-level matrix (separator and interface rows of the local
// CSR) receives the fronts' trailing blocks, in sub-box order, and is split
// and factored like a single-level local matrix.
template <typename T>
static int factor_nd_t(vb_ctx *ctx, bool timed) {
  hipStream_t st = ctx->stream;
  const bool f32 = ctx->fp32;
  const int nS = ctx->nS, nF = (int)ctx->fronts.size();
  const FrontH &FL = ctx->fronts.back();
  auto prepare_f = [&]() -> int {
    CHK(hipMemsetAsync(ctx->FW, 0, (FL.S.W_off + FL.S.ld * FL.S.N) * ctx->wsz, st));
    CHK(densify(ctx->d_frdev, nF, ctx->max_nf_csr, f32, st));
    CHK(house_pressure(ctx->d_frdev, nF, ctx->max_Nf, f32, st));
    CHK(hipMemsetAsync(ctx->info_f, 0, nF * sizeof(int), st));
    return VB_OK;
  };
  {
    int rc = prepare_f();
    if (rc) return rc;
  }
  {
    std::vector<LdlJob<T>> jobs;
    for (int f = 0; f < nF; ++f) {
      const SubH &F = ctx->fronts[f].S;
      jobs.push_back({(T *)ctx->FW + F.W_off, F.ld, F.N, F.e, F.nv, 0, (T *)ctx->invLf + F.inv_off,
                      ctx->info_f + f, f32 ? ctx->opt.fp32_pivot_min : 0.0});
    }
    int rc = tuned_ldl(ctx, 0, jobs, ctx->max_Nf, ctx->max_ef, timed, prepare_f);
    if (rc) return rc;
  }
  std::vector<char> broke(nS, 0);  // mixed precision: subdomains to factor again in FP64
  {
    std::vector<int> h(nF);
    CHK(hipMemcpyAsync(h.data(), ctx->info_f, nF * sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (int f = 0; f < nF; ++f) {
      if (!h[f]) continue;
      if (!f32)
        return ctx->fail(VB_ERR_NOT_SPD, "Dirichlet factorisation (subdomain index): pivot breakdown in block " +
                                             std::to_string(ctx->fronts[f].sub) + " at column " +
                                             std::to_string(h[f] - 1) + " of its sub-box " +
                                             std::to_string(ctx->fronts[f].box));
      broke[ctx->fronts[f].sub] = 1;
    }
  }
  const SubH &SL = ctx->subs.back();
  auto prepare_2 = [&]() -> int {
    CHK(hipMemsetAsync(ctx->W, 0, (SL.W_off + SL.ld * SL.N) * ctx->wsz, st));
    CHK(densify(ctx->d_subdev, nS, ctx->max_n_csr, f32, st));
    for (int b = 0; b < ctx->max_nbox; ++b)
      CHK(front_scatter(ctx->d_fj_scatter[b], (int)ctx->fj_scatter[b].size(), ctx->max_fm, f32, st));
    CHK(house_pressure(ctx->d_subdev, nS, ctx->max_N, f32, st));
    CHK(hipMemsetAsync(ctx->info, 0, nS * sizeof(int), st));
    return VB_OK;
  };
  {
    int rc = prepare_2();
    if (rc) return rc;
  }
  {
    std::vector<LdlJob<T>> jobs;
    for (int s = 0; s < nS; ++s) {
      const SubH &S = ctx->subs[s];
      jobs.push_back({(T *)ctx->W + S.W_off, S.ld, S.N, S.e, S.nv, 0, (T *)ctx->invL + S.inv_off,
                      ctx->info + s, f32 ? ctx->opt.fp32_pivot_min : 0.0});
    }
    int rc = tuned_ldl(ctx, 1, jobs, ctx->max_N, ctx->max_e, timed, prepare_2);
    if (rc) return rc;
  }
  std::vector<int> h(nS);
  CHK(hipMemcpyAsync(h.data(), ctx->info, nS * sizeof(int), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  std::vector<int> bad;
  for (int s = 0; s < nS; ++s) {
    if (h[s] && !f32)
      return ctx->fail(VB_ERR_NOT_SPD, "Dirichlet factorisation (subdomain index): pivot breakdown in block " +
                                           std::to_string(s) + " at column " + std::to_string(h[s] - 1) +
                                           " of its separator level");
    if (h[s] || broke[s]) bad.push_back(s);
  }
  return bad.empty() ? VB_OK : retry_fp64(ctx, bad);
}

static int factor_nd(vb_ctx *ctx, bool timed) {
  return ctx->fp32 ? factor_nd_t<float>(ctx, timed) : factor_nd_t<double>(ctx, timed);
}

extern "C" {

static int setup_impl(vb_ctx *ctx);

int vb_setup(vb_ctx *ctx) {
  if (!ctx) return VB_ERR_ARG;
  if (ctx->state < 1) return ctx->fail(VB_ERR_STATE, "vb_setup: call vb_assemble first");
  if (!ctx->finalized) {
    int rc = finalize_device(ctx);
    if (rc) return rc;
  }
  if (ctx->it_exec) {  // the captured iteration refers to the previous setup's buffers
    (void)hipGraphExecDestroy(ctx->it_exec);
    (void)hipGraphDestroy(ctx->it_graph);
    ctx->it_exec = nullptr;
    ctx->it_graph = nullptr;
  }
  if (ctx->state == 2) {  // a new setup replaces the previous one
    CHK(hipStreamSynchronize(ctx->stream));
    for (void *q : ctx->setup_keep) ctx->pool_put(q);
    ctx->setup_keep.clear();
    for (auto &H : ctx->ents) {
      H.D.clear();
      H.Dit.clear();
      H.d_dual_gids = nullptr;
    }
    ctx->state = 1;
  }
  ctx->zst_valid = false;
  ctx->cond_fresh = false;
  ctx->n_restrict = ctx->n_ext = 0;
  ctx->max_rm = ctx->max_ext_m = ctx->max_gt_m = ctx->max_gt_n = 0;
  ctx->max_ndl = ctx->max_npi = ctx->max_nt = 0;
  ctx->cur_scope = 2;
  int rc = setup_impl(ctx);
  ctx->cur_scope = 0;
  hipError_t e = ctx->release_setup_scratch();
  if (!rc && e != hipSuccess)
    rc = ctx->fail(VB_ERR_DEVICE, std::string("setup: ") + hipGetErrorString(e));
  return rc;
}

static int setup_impl(vb_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const int nS = ctx->nS;
  const int64_t nG = ctx->nG;
  ctx->fp64_retried.clear();
  // start from the given constraints
  for (auto &H : ctx->ents) {
    H.ncon = H.ncon0;
    H.con = H.con0;
    H.d_con = H.d_con0;
    H.d_V = H.d_V0;
    H.d_tau = H.d_tau0;
    H.d_work = H.d_work0;
  }
  ctx->entdev = ctx->entdev0;
  ctx->plan_valid = false;
  CHK(hipMemcpyAsync(ctx->d_entdev, ctx->entdev.data(), ctx->entdev.size() * sizeof(EntDev),
                     hipMemcpyHostToDevice, st));
  ctx->face_info.clear();
  ctx->face_eigs.clear();
  ctx->d_feat = ctx->d_lab = nullptr;  // freed with the previous setup
  ctx->n_coord = 0;
  CHK(hipEventRecord(ctx->ev0, st));
  auto mark = [&](int ph) -> hipError_t {  // start of setup phase ph (1-based, >= 2)
    if (!ctx->ph_ev[ph - 1]) {
      hipError_t e = hipEventCreate(&ctx->ph_ev[ph - 1]);
      if (e != hipSuccess) return e;
    }
    return hipEventRecord(ctx->ph_ev[ph - 1], st);
  };
  // ---- 1.-2. per wave of subdomains: local dense bordered matrices, pressure
  //      split, Dirichlet factorisation + Schur complement (eqs. uipi,
  //      firstSchur); with several waves the condensed blocks are copied out
  const bool f32 = ctx->fp32;
  auto Xptr = [&](const SubH &S) -> void * { return S.X; };
  CHK(hipMemsetAsync(ctx->info, 0, (4 * (size_t)nS + 64 + 4 * ctx->ents.size()) * sizeof(int), st));
  if (ctx->nd)
    CHK(flux_rows(ctx->d_fulldev, nS, ctx->max_n_full, st));
  else
    CHK(flux_rows(ctx->d_subdev, nS, ctx->max_n_csr, st));
  ctx->w_wave = -1;
  for (const auto &wv : ctx->waves) {
    int rc = ctx->nd ? factor_nd(ctx, true) : factor_wave(ctx, wv.first, wv.second, true);
    if (rc) return rc;
    if (!ctx->stream_w) continue;
    ctx->w_wave = (int)(&wv - ctx->waves.data());
    for (int s = wv.first; s < wv.second; ++s) {
      const SubH &S = ctx->subs[s];
      const char *src = (const char *)ctx->W + (S.W_off + (S.e + 1) + (int64_t)(S.e + 1) * S.ld) * ctx->wsz;
      CHK(hipMemcpy2DAsync(S.X, S.xld * ctx->wsz, src, S.ld * ctx->wsz, (S.ng + 1) * ctx->wsz, S.ng + 1,
                           hipMemcpyDeviceToDevice, st));
    }
  }
  CHK(mark(2));
  // ---- 3. primal constraints: QR with column pivoting per entity
  const int nE = (int)ctx->ents.size();
  {
    int rc = primal_qr(ctx);
    if (rc) return rc;
    // adaptive enrichment of the face constraints (Sec. 6), then the bases again
    if (ctx->opt.adaptive_theta > 0.0) {
      rc = adaptive_stage(ctx);
      if (rc) return rc;
      rc = primal_qr(ctx);
      if (rc) return rc;
    }
  }
  // coarse numbering, one contiguous block per problem:
  // [primal coordinates of its entities | p0 of its subdomains]
  std::vector<int32_t> cstart(nE + 1, 0);
  for (int e = 0; e < nE; ++e) cstart[e + 1] = cstart[e] + ctx->ents[e].rank;
  ctx->nC = cstart[nE];
  ctx->nCS = ctx->nC + nS;
  ctx->ent_cbase.assign(nE, 0);
  ctx->sub_cp0.assign(nS, 0);
  ctx->max_ncs = 0;
  {
    int cb = 0;
    for (auto &P : ctx->probs) {
      P.cbase = cb;
      P.nprim = cstart[P.e0 + P.ne] - cstart[P.e0];
      for (int e = P.e0; e < P.e0 + P.ne; ++e) ctx->ent_cbase[e] = cb + cstart[e] - cstart[P.e0];
      for (int s = P.s0; s < P.s0 + P.ns; ++s) ctx->sub_cp0[s] = cb + P.nprim + (s - P.s0);
      cb += P.nprim + P.ns;
      ctx->max_ncs = std::max(ctx->max_ncs, P.nprim + P.ns);
    }
  }
  for (int s = 0; s < nS; ++s) {
    SubH &S = ctx->subs[s];
    S.pl.clear();
    S.dl.clear();
    S.cidx.clear();
    S.doff.clear();
    for (size_t q = 0; q < S.ents.size(); ++q) {
      const EntH &H = ctx->ents[S.ents[q]];
      S.doff.push_back((int64_t)S.dl.size());
      for (int j = 0; j < H.n; ++j) {
        if (j < H.rank) {
          S.pl.push_back(S.ent_off[q] + j);
          S.cidx.push_back(ctx->ent_cbase[S.ents[q]] + j);
        } else {
          S.dl.push_back(S.ent_off[q] + j);
        }
      }
    }
    S.npi = (int)S.pl.size();
    S.ndl = (int)S.dl.size();
  }
  CHK(mark(3));
  // ---- 4. change of basis on the bordered interface block: X <- T^T X T
  {
    std::vector<void *> m(nS);
    std::vector<int64_t> ld(nS);
    std::vector<int32_t> n(nS);
    for (int s = 0; s < nS; ++s) {
      SubH &S = ctx->subs[s];
      m[s] = Xptr(S);
      ld[s] = S.xld;
      n[s] = S.ng + 1;
    }
    // largest entity, and the bounds min(n_con, n) of its reflectors' count and
    // min(n_con, n) * n of their entries
    int max_en = 1, max_rn = 1, max_rank = 0;
    for (const auto &H : ctx->ents) {
      max_en = std::max(max_en, H.n);
      max_rn = std::max(max_rn, std::min(H.ncon, H.n) * H.n);
      max_rank = std::max(max_rank, std::min(H.ncon, H.n));
    }
    int rc = run_symm(ctx, m, ld, n, false, f32);
    if (rc) return rc;
    // T^T X (contiguous entity segments of the columns), transposed to X T
    // (X symmetric), T^T X T; entities too large for that kernel take the
    // column kernel on both sides instead
    bool rows = false;
    CHK(apply_T_rows(ctx->d_subdev, ctx->d_entdev, nS, ctx->max_ng, ctx->max_ent, max_en, max_rn, max_rank, f32, &rows,
                     st));
    if (!rows)
      CHK(apply_T_cols(ctx->d_subdev, ctx->d_entdev, nS, ctx->max_ng, ctx->max_ent, max_en, f32, st));
    rc = run_symm(ctx, m, ld, n, true, f32);
    if (rc) return rc;
    if (rows) {
      CHK(apply_T_rows(ctx->d_subdev, ctx->d_entdev, nS, ctx->max_ng, ctx->max_ent, max_en, max_rn, max_rank, f32, &rows,
                       st));
      if (!rows) return ctx->fail(VB_ERR_DEVICE, "change of basis: second pass not launched");
    } else {
      CHK(apply_T_cols(ctx->d_subdev, ctx->d_entdev, nS, ctx->max_ng, ctx->max_ent, max_en, f32, st));
    }
    CHK(transform_b0(ctx->d_subdev, ctx->d_entdev, nS, ctx->max_ent, st));
  }
  CHK(mark(4));
  // ---- 5. transformed right-hand side g~ (owner sums over the rhs columns)
  const int64_t nTot = nG + nS;
  UCHK(ctx->dalloc(&ctx->g, nTot));
  {
    // condensed local right-hand sides (border column of X) -> flat FP64 buffer
    std::vector<int32_t> iota(ctx->max_ng + 1);
    std::iota(iota.begin(), iota.end(), 0);
    int32_t *d_iota = nullptr;
    UCHK(ctx->upload(&d_iota, iota, true));
    int64_t ftot = 0;
    for (auto &S : ctx->subs) ftot += S.ng;
    double *gl = nullptr;
    UCHK(ctx->dalloc(&gl, std::max<int64_t>(ftot, 1), true));
    std::vector<GatherJob> gj;
    int64_t fo = 0;
    for (int s = 0; s < nS; ++s) {
      SubH &S = ctx->subs[s];
      GatherJob J{Xptr(S), S.xld, gl + fo, S.ng, d_iota, d_iota, S.ng, 1, 1.0, 0, f32 ? 1 : 0, 0};
      J.ci = d_iota + S.ng;  // column ng of X
      gj.push_back(J);
      fo += S.ng;
    }
    int rc0 = run_gather(ctx, gj, ctx->max_ng, 1);
    if (rc0) return rc0;
    std::vector<int64_t> ptr, idx;
    build_csr(nG, [&](auto emit) {
      int64_t o = 0;
      for (int s = 0; s < nS; ++s) {
        const SubH &S = ctx->subs[s];
        for (int l = 0; l < S.ng; ++l) emit(S.gidl[l], o + l);
        o += S.ng;
      }
    }, ptr, idx);
    UCHK(ctx->upload(&ctx->g_ptr, ptr, true));
    UCHK(ctx->upload(&ctx->g_idx, idx, true));
    CHK(owner_sum((int)nG, ctx->g_ptr, ctx->g_idx, gl, nullptr, nullptr, ctx->g, st));
    std::vector<int64_t> src(nS), dst(nS);
    for (int s = 0; s < nS; ++s) {
      src[s] = ctx->subs[s].b0_off + ctx->subs[s].ng;
      dst[s] = nG + s;
    }
    UCHK(ctx->upload(&ctx->p0_src, src, true));
    UCHK(ctx->upload(&ctx->p0_dst, dst, true));
    CHK(scatter_copy(nS, ctx->b0, ctx->p0_src, ctx->p0_dst, ctx->g, 1.0, st));
  }
  // border of X becomes the transformed flux row: X_s = [[S~, b0~], [b0~^T, 0]]
  {
    std::vector<GatherJob> jobs;
    std::vector<DiagJob> dj;
    std::vector<int32_t> iota(ctx->max_ng + 1);
    std::iota(iota.begin(), iota.end(), 0);
    int32_t *d_iota = nullptr;
    UCHK(ctx->upload(&d_iota, iota, true));
    for (int s = 0; s < nS; ++s) {
      SubH &S = ctx->subs[s];
      char *X = (char *)Xptr(S);
      double *b0 = ctx->b0 + S.b0_off;
      const int o32 = f32 ? 1 : 0;
      // last column: X[l, ng] = b0[l]  (in: b0 as an ng x 1 matrix)
      jobs.push_back({b0, 1, X + (int64_t)S.ng * S.xld * ctx->wsz, S.xld, d_iota, d_iota, S.ng, 1,
                      1.0, 0, 0, o32});
      // last row: X[ng, l] = b0[l]  (in: b0 as a 1 x ng matrix, ld 1)
      jobs.push_back({b0, 1, X + (int64_t)S.ng * ctx->wsz, S.xld, d_iota, d_iota, 1, S.ng, 1.0, 0, 0,
                      o32});
      dj.push_back({X, S.xld, S.ng, S.ng, 1, 0.0, o32});
    }
    int rc = run_gather(ctx, jobs, ctx->max_ng, ctx->max_ng);
    if (rc) return rc;
    rc = run_diag(ctx, dj, 1);
    if (rc) return rc;
  }
  CHK(mark(5));
  // ---- 6. local constrained Neumann problems: eliminate the duals of
  //         [[S_DD, S_DP, I], [S_PD, S_PP, 0], [I, 0, 0]] -> [[S_Pi, .], [Phi, -S_DD^-1]]
  //         The augmented matrices are formed and factored in waves of
  //         consecutive subdomains sized to the free device memory; each wave
  //         leaves G1 = [S_DD^-1 | Phi] and S_Pi behind.  In mixed
  //         precision they are FP32 (they only enter the preconditioner);
  //         S_Pi is stored in FP64 for the FP64 coarse factorisation.
  {
    const bool nf = f32;
    const size_t nsz = nf ? sizeof(float) : sizeof(double);
    auto at = [&](void *p, int64_t off) -> void * { return (char *)p + off * (int64_t)nsz; };
    int64_t gtot = 0, stot = 0, itot = 0, ntot = 0, nmax = 1;
    for (auto &S : ctx->subs) {
      S.Nn = 2 * S.ndl + S.npi;
      S.Nld = round_up(std::max(S.Nn, 1), 32);
      gtot += (int64_t)S.ndl * (S.ndl + S.npi);
      stot += (int64_t)S.npi * S.npi;
      itot += (int64_t)((S.ndl + NB - 1) / NB) * NB * NB;
      ntot += S.Nld * std::max(S.Nn, 1);
      nmax = std::max(nmax, S.Nld * std::max(S.Nn, 1));
      ctx->max_ndl = std::max(ctx->max_ndl, S.ndl);
      ctx->max_npi = std::max(ctx->max_npi, S.npi);
    }
    char *G1all = nullptr, *invN = nullptr;
    double *Spall = nullptr;
    UCHK(ctx->dalloc(&G1all, std::max<int64_t>(gtot, 1) * nsz));
    UCHK(ctx->dalloc(&Spall, std::max<int64_t>(stot, 1), true));
    UCHK(ctx->dalloc(&invN, std::max<int64_t>(itot, 1) * nsz, true));
    {
      int64_t go = 0, so = 0;
      for (auto &S : ctx->subs) {
        S.G1 = at(G1all, go);
        S.Spi = Spall + so;
        go += (int64_t)S.ndl * (S.ndl + S.npi);
        so += (int64_t)S.npi * S.npi;
      }
    }
    size_t fre = 0, tot = 0;
    CHK(hipMemGetInfo(&fre, &tot));
    fre += ctx->pool_unused_bytes();
    const double lim = ctx->opt.setup_mem_limit > 0.0 ? ctx->opt.setup_mem_limit : 0.6 * (double)fre;
    const int64_t budget = std::max<int64_t>(nmax, (int64_t)(lim / (double)nsz));
    int64_t wmax = std::min(ntot, budget);
    // the budget follows the free memory, so an earlier setup's buffer (left in
    // the pool) can be a little smaller than this request, which would then
    // need a new allocation beside it: such a buffer (at least 3/4 of the
    // request and the largest matrix) is taken whole instead
    if (!ctx->pool_has((size_t)wmax * nsz)) {
      const size_t want = (size_t)wmax * nsz;
      const size_t fit = ctx->pool_fit(std::max((size_t)nmax * nsz, want / 4 * 3), want);
      if (fit) wmax = (int64_t)(fit / nsz);
    }
    char *Nbuf = nullptr;
    UCHK(ctx->dalloc(&Nbuf, wmax * nsz, true));
    int rc = 0;
    int64_t ioff = 0;
    for (int s0 = 0; s0 < nS && !rc;) {
      int s1 = s0;
      int64_t off = 0;
      while (s1 < nS && off + ctx->subs[s1].Nld * std::max(ctx->subs[s1].Nn, 1) <= wmax)
        off += ctx->subs[s1].Nld * std::max(ctx->subs[s1].Nn, 1), ++s1;
      CHK(hipMemsetAsync(Nbuf, 0, off * nsz, st));
      std::vector<GatherJob> gj, ej;
      std::vector<DiagJob> dj;
      std::vector<LdlJob<double>> lj;
      std::vector<LdlJob<float>> lj32;
      std::vector<void *> m;
      std::vector<int64_t> ld;
      std::vector<int32_t> n;
      int max_m = 0, max_e = 0, mxg = 0, mxr = 0, mxc = 0;
      off = 0;
      for (int s = s0; s < s1; ++s) {
        SubH &S = ctx->subs[s];
        S.Nmat = at(Nbuf, off);
        off += S.Nld * std::max(S.Nn, 1);
        std::vector<int32_t> idx(S.dl);
        idx.insert(idx.end(), S.pl.begin(), S.pl.end());
        int32_t *d_idx = nullptr;
        UCHK(ctx->upload(&d_idx, idx, true));
        const int mm = S.ndl + S.npi;
        gj.push_back({Xptr(S), S.xld, S.Nmat, S.Nld, d_idx, d_idx, mm, mm, 1.0, 0, f32 ? 1 : 0,
                      nf ? 1 : 0});
        mxg = std::max(mxg, mm);
        if (S.ndl) dj.push_back({S.Nmat, S.Nld, S.ndl + S.npi, 0, S.ndl, 1.0, nf ? 1 : 0});
        // identity block at rows ndl + npi (eliminated columns 0 .. ndl - 1)
        if (nf)
          lj32.push_back({(float *)S.Nmat, S.Nld, S.Nn, S.ndl, S.ndl, 0, (float *)at(invN, ioff),
                          ctx->info + s, 0.0, S.ndl + S.npi});
        else
          lj.push_back({(double *)S.Nmat, S.Nld, S.Nn, S.ndl, S.ndl, 0, (double *)at(invN, ioff),
                        ctx->info + s, 0.0, S.ndl + S.npi});
        ioff += (int64_t)((S.ndl + NB - 1) / NB) * NB * NB;
        max_m = std::max(max_m, S.Nn);
        max_e = std::max(max_e, S.ndl);
        // trailing block after the elimination: [[S_Pi, .], [Phi, -S_DD^-1]]
        void *T = at(S.Nmat, S.ndl + S.ndl * S.Nld);
        m.push_back(T);
        ld.push_back(S.Nld);
        n.push_back(S.npi + S.ndl);
        // its pieces: (rows, cols) index lists into T
        std::vector<int32_t> rows(S.ndl), pc(S.npi);
        for (int a = 0; a < S.ndl; ++a) rows[a] = S.npi + a;
        for (int a = 0; a < S.npi; ++a) pc[a] = a;
        int32_t *dr = nullptr, *dpc = nullptr;
        UCHK(ctx->upload(&dr, rows, true));
        UCHK(ctx->upload(&dpc, pc, true));
        const int o = nf ? 1 : 0;
        if (S.ndl) {
          ej.push_back({T, S.Nld, S.G1, S.ndl, dr, dr, S.ndl, S.ndl, -1.0, 0, o, o});
          if (S.npi)
            ej.push_back({T, S.Nld, at(S.G1, (int64_t)S.ndl * S.ndl), S.ndl, dr, dpc, S.ndl, S.npi,
                          1.0, 0, o, o});
        }
        if (S.npi) ej.push_back({T, S.Nld, S.Spi, S.npi, dpc, dpc, S.npi, S.npi, 1.0, 0, o, 0});
        mxr = std::max(mxr, std::max(S.ndl, S.npi));
        mxc = std::max(mxc, std::max(S.ndl, S.npi));
      }
      const int64_t woff = off;
      auto prepare = [&]() -> int {  // the wave's augmented matrices formed again
        CHK(hipMemsetAsync(Nbuf, 0, woff * nsz, st));
        int r = run_gather(ctx, gj, mxg, mxg);
        if (!r) r = run_diag(ctx, dj, ctx->max_ndl);
        if (!r) CHK(hipMemsetAsync(ctx->info + s0, 0, (s1 - s0) * sizeof(int), st));
        return r;
      };
      rc = run_gather(ctx, gj, mxg, mxg);
      if (!rc) rc = run_diag(ctx, dj, ctx->max_ndl);
      if (!rc) {
        CHK(hipMemsetAsync(ctx->info + s0, 0, (s1 - s0) * sizeof(int), st));
        rc = nf ? tuned_ldl(ctx, 2, lj32, max_m, max_e, false, prepare)
                : tuned_ldl(ctx, 2, lj, max_m, max_e, false, prepare);
      }
      if (!rc) {
        std::vector<int> h(s1 - s0);
        CHK(hipMemcpyAsync(h.data(), ctx->info + s0, h.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        CHK(hipStreamSynchronize(st));
        for (size_t q = 0; q < h.size() && !rc; ++q)
          if (h[q])
            rc = ctx->fail(VB_ERR_NOT_SPD, "Neumann factorisation (subdomain index): pivot breakdown in block " +
                                               std::to_string(s0 + (int)q) + " at column " +
                                               std::to_string(h[q] - 1));
      }
      if (!rc) rc = run_symm(ctx, m, ld, n, false, nf);
      if (!rc) rc = run_gather(ctx, ej, mxr, mxc);
      s0 = s1;
    }
    ctx->free_setup_early(Nbuf);
    for (auto &S : ctx->subs) S.Nmat = nullptr;
    if (rc) return rc;
  }
  CHK(mark(6));
  // ---- 7. coarse problem: per problem, the inverse of the bordered coarse
  // matrix from the partial LDL^T of [[K_c, I], [I, 0]]
  {
    const int nP = (int)ctx->probs.size();
    std::vector<int64_t> koff(nP), goff(nP), ldk(nP);
    int64_t ktot = 0, gtot = 0, itot = 0;
    for (int pp = 0; pp < nP; ++pp) {
      const int ncs = ctx->probs[pp].nprim + ctx->probs[pp].ns;
      ldk[pp] = round_up(2 * ncs, 32);
      koff[pp] = ktot;
      ktot += ldk[pp] * 2 * ncs;
      goff[pp] = gtot;
      gtot += (int64_t)ncs * ncs;
      itot += (int64_t)((ncs + NB - 1) / NB) * NB * NB;
    }
    ctx->Kld = nP == 1 ? ldk[0] : 0;
    UCHK(ctx->dalloc(&ctx->Kaug, std::max<int64_t>(ktot, 1), true));
    CHK(hipMemsetAsync(ctx->Kaug, 0, ktot * sizeof(double), st));
    UCHK(ctx->dalloc(&ctx->Gc, std::max<int64_t>(gtot, 1)));
    double *invC = nullptr;
    UCHK(ctx->dalloc(&invC, std::max<int64_t>(itot, 1), true));
    std::vector<DiagJob> dj;
    std::vector<LdlJob<double>> lj;
    std::vector<void *> m;
    std::vector<int64_t> ld;
    std::vector<int32_t> n;
    std::vector<GatherJob> gj;
    int32_t *di = nullptr;
    {
      std::vector<int32_t> iota(std::max(ctx->max_ncs, 1));
      std::iota(iota.begin(), iota.end(), 0);
      UCHK(ctx->upload(&di, iota, true));
    }
    int64_t io = 0;
    for (int pp = 0; pp < nP; ++pp) {
      const auto &P = ctx->probs[pp];
      const int ncs = P.nprim + P.ns;
      double *K = ctx->Kaug + koff[pp];
      std::vector<CoarseSub> cs(P.ns);
      for (int sl = 0; sl < P.ns; ++sl) {
        SubH &S = ctx->subs[P.s0 + sl];
        std::vector<int32_t> cl(S.cidx.size());
        for (size_t a = 0; a < cl.size(); ++a) cl[a] = S.cidx[a] - P.cbase;
        int32_t *dc = nullptr, *dp = nullptr;
        UCHK(ctx->upload(&dc, cl, true));
        UCHK(ctx->upload(&dp, S.pl, true));
        cs[sl] = {S.Spi, std::max(S.npi, 1), S.npi, dc, dp, ctx->b0 + S.b0_off};
      }
      CoarseSub *dcs = nullptr;
      UCHK(ctx->upload(&dcs, cs, true));
      double vn = 0.0;
      for (int sl = 0; sl < P.ns; ++sl) vn += ctx->subs[P.s0 + sl].vol * ctx->subs[P.s0 + sl].vol;
      vn = std::sqrt(vn);
      std::vector<double> w(P.ns);
      for (int sl = 0; sl < P.ns; ++sl) w[sl] = ctx->subs[P.s0 + sl].vol / vn;
      double *dw = nullptr;
      UCHK(ctx->upload(&dw, w, true));
      CHK(coarse_assemble(dcs, P.ns, K, ldk[pp], P.nprim, dw, st));
      dj.push_back({K, ldk[pp], ncs, 0, ncs, 1.0});
      lj.push_back({K, ldk[pp], 2 * ncs, ncs, P.nprim, 0, invC + io, ctx->info + nS + pp, 0.0, ncs});
      io += (int64_t)((ncs + NB - 1) / NB) * NB * NB;
      m.push_back(K + ncs + ncs * ldk[pp]);
      ld.push_back(ldk[pp]);
      n.push_back(ncs);
      gj.push_back({K + ncs + ncs * ldk[pp], ldk[pp], ctx->Gc + goff[pp], ncs, di, di, ncs, ncs,
                    -1.0, 0, 0, 0});
    }
    // the diagonal of every coarse matrix before and after its factorisation
    // (gathered on the device, one copy to the host): a pivot that cancels to
    // 1e-10 of its column's own diagonal entry means a singular coarse
    // problem (for instance a primal space that does not see the face fluxes,
    // Assumption 1), which rounding may leave with either sign
    std::vector<int64_t> doff(nP + 1, 0);
    for (int pp = 0; pp < nP; ++pp) doff[pp + 1] = doff[pp] + ctx->probs[pp].nprim + ctx->probs[pp].ns;
    std::vector<double> dg(2 * doff[nP]);
    double *ddg = nullptr;
    UCHK(ctx->dalloc(&ddg, std::max<int64_t>(2 * doff[nP], 1), true));
    auto diag_copy = [&](int64_t half) -> hipError_t {
      for (int pp = 0; pp < nP; ++pp) {
        hipError_t e = diag_gather(ctx->Kaug + koff[pp], ldk[pp], (int)(doff[pp + 1] - doff[pp]),
                                   ddg + half + doff[pp], st);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    CHK(diag_copy(0));
    int rc = run_diag(ctx, dj, ctx->max_ncs);
    if (rc) return rc;
    rc = run_ldl(ctx, lj, 2 * ctx->max_ncs, ctx->max_ncs);
    if (rc) return rc;
    {
      std::vector<int> h(nP);
      CHK(hipMemcpyAsync(h.data(), ctx->info + nS, nP * sizeof(int), hipMemcpyDeviceToHost, st));
      CHK(diag_copy(doff[nP]));
      if (doff[nP] > 0)
        CHK(hipMemcpyAsync(dg.data(), ddg, dg.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      CHK(hipStreamSynchronize(st));
      const double *dg0 = dg.data(), *dg1 = dg.data() + doff[nP];
      for (int pp = 0; pp < nP; ++pp) {
        int bad = h[pp] ? h[pp] - 1 : -1;
        for (int64_t j = doff[pp]; bad < 0 && j < doff[pp + 1]; ++j)
          if (!(dg1[j] * dg1[j] > 1e-10 * std::fabs(dg0[j]))) bad = (int)(j - doff[pp]);
        if (bad >= 0)
          return ctx->fail(VB_ERR_SINGULAR_COARSE, "coarse factorisation of problem " +
                                                       std::to_string(pp) + ": pivot breakdown at column " +
                                                       std::to_string(bad));
      }
    }
    rc = run_symm(ctx, m, ld, n);
    if (rc) return rc;
    rc = run_gather(ctx, gj, ctx->max_ncs, ctx->max_ncs);
    if (rc) return rc;
    ctx->gc_off = goff;
  }
  CHK(mark(7));
  // ---- 8. scaling: deluxe D_E^(s) = (sum_l Sbar^(l))^-1 Sbar^(s) on the duals
  {
    std::vector<LdlJob<double>> lj;
    std::vector<GemmJob<double>> mj;
    std::vector<DiagJob> dj;
    std::vector<std::vector<GatherJob>> rounds;
    std::vector<GatherJob> sb;
    int max_m = 0;
    int64_t itot = 0;
    for (auto &H : ctx->ents) {
      int m = H.n - H.rank;
      if (m > 0) itot += (int64_t)((m + NB - 1) / NB) * NB * NB;
    }
    double *invD = nullptr;
    UCHK(ctx->dalloc(&invD, std::max<int64_t>(itot, 1), true));
    // every D_E^(s) in one allocation, each with an even leading dimension
    // (16-byte aligned columns for the extension's loads).  An entity shared
    // by two subdomains keeps only D_E^(first): the other is I - D_E^(first)
    // (the deluxe weights sum to the identity), which the restriction and the
    // extension apply without reading a second matrix.
    auto pair_of = [&](const EntH &H) {
      return ctx->opt.scaling != VB_SCALING_COUNTING && H.subs.size() == 2;
    };
    int64_t dtot = 0;
    for (auto &H : ctx->ents) {
      const int m = H.n - H.rank;
      if (m > 0) dtot += (int64_t)(pair_of(H) ? 1 : H.subs.size()) * round_up(m, 2) * m;
    }
    // (mixed precision: the iteration reads an FP32 copy, made at the end)
    double *dall = nullptr;
    UCHK(ctx->dalloc(&dall, std::max<int64_t>(dtot, 1), f32));
    // the augmented matrices [[sum Sbar, I], [I, 0]] (zeroed) and the Sbar
    // blocks of every entity, each set in one allocation
    int64_t atot = 0, stot = 0;
    if (ctx->opt.scaling != VB_SCALING_COUNTING)
      for (auto &H : ctx->ents) {
        const int m = H.n - H.rank;
        if (m <= 0) continue;
        atot += round_up(2 * m, 32) * 2 * m;
        stot += (int64_t)H.subs.size() * m * m;
      }
    double *aall = nullptr, *sall = nullptr;
    UCHK(ctx->dalloc(&aall, std::max<int64_t>(atot, 1), true));
    UCHK(ctx->dalloc(&sall, std::max<int64_t>(stot, 1), true));
    if (atot) CHK(hipMemsetAsync(aall, 0, atot * sizeof(double), st));
    if (ctx->opt.scaling == VB_SCALING_COUNTING && dtot)
      CHK(hipMemsetAsync(dall, 0, dtot * sizeof(double), st));
    int64_t doff = 0, aoff = 0, soff = 0;
    int64_t ioff = 0;
    int cnt = 0;
    for (int e = 0; e < nE; ++e) {
      EntH &H = ctx->ents[e];
      const int m = H.n - H.rank;
      H.D.assign(H.subs.size(), nullptr);
      H.Sbar.assign(H.subs.size(), nullptr);
      std::vector<int64_t> dg(H.gids.begin() + H.rank, H.gids.end());
      UCHK(ctx->upload(&H.d_dual_gids, dg));
      if (m <= 0) continue;
      max_m = std::max(max_m, m);
      const int64_t ldm = round_up(m, 2);
      H.Dmld = ldm;
      for (size_t q = 0; q < (pair_of(H) ? 1 : H.subs.size()); ++q) {
        H.D[q] = dall + doff;
        doff += ldm * m;
      }
      if (ctx->opt.scaling == VB_SCALING_COUNTING) {
        for (size_t q = 0; q < H.subs.size(); ++q) dj.push_back({H.D[q], ldm, 0, 0, m, 1.0 / H.subs.size()});
        continue;
      }
      H.Dld = round_up(2 * m, 32);
      H.Daug = aall + aoff;
      aoff += H.Dld * 2 * m;
      for (size_t q = 0; q < H.subs.size(); ++q) {
        const int s = H.subs[q];
        SubH &S = ctx->subs[s];
        int qq = (int)(std::find(S.ents.begin(), S.ents.end(), e) - S.ents.begin());
        std::vector<int32_t> idx(m);
        for (int a = 0; a < m; ++a) idx[a] = S.ent_off[qq] + H.rank + a;
        int32_t *d_idx = nullptr;
        UCHK(ctx->upload(&d_idx, idx, true));
        const void *X = Xptr(S);
        if (rounds.size() <= q) rounds.resize(q + 1);
        rounds[q].push_back({X, S.xld, H.Daug, H.Dld, d_idx, d_idx, m, m, 1.0, 1, f32 ? 1 : 0, 0});
        H.Sbar[q] = sall + soff;
        soff += (int64_t)m * m;
        sb.push_back({X, S.xld, H.Sbar[q], m, d_idx, d_idx, m, m, 1.0, 0, f32 ? 1 : 0, 0});
        if (H.D[q])
          mj.push_back({H.Daug + m + m * H.Dld, H.Sbar[q], H.D[q], H.Dld, m, ldm, m, m, m, 0, -1.0, 0.0});
      }
      dj.push_back({H.Daug, H.Dld, m, 0, m, 1.0});
      lj.push_back({H.Daug, H.Dld, 2 * m, m, m, 0, invD + ioff, ctx->info + 2 * nS + 2 + (cnt % 16), 0.0,
                    m});
      ioff += (int64_t)((m + NB - 1) / NB) * NB * NB;
      ++cnt;
    }
    for (auto &rj : rounds) {
      int rc = run_gather(ctx, rj, max_m, max_m);
      if (rc) return rc;
    }
    int rc = run_gather(ctx, sb, max_m, max_m);
    if (rc) return rc;
    rc = run_diag(ctx, dj, max_m);
    if (rc) return rc;
    if (!lj.empty()) {
      CHK(hipMemsetAsync(ctx->info + 2 * nS + 2, 0, 16 * sizeof(int), st));
      rc = run_ldl(ctx, lj, 2 * max_m, max_m);
      if (rc) return rc;
      std::vector<int> h(16);
      CHK(hipMemcpyAsync(h.data(), ctx->info + 2 * nS + 2, 16 * sizeof(int), hipMemcpyDeviceToHost, st));
      CHK(hipStreamSynchronize(st));
      for (int v : h)
        if (v) return ctx->fail(VB_ERR_NOT_SPD, "deluxe scaling: sum of face/edge Schur blocks not SPD");
      std::vector<void *> m;
      std::vector<int64_t> ld;
      std::vector<int32_t> n;
      for (auto &H : ctx->ents)
        if (H.Daug) {
          int mm = H.n - H.rank;
          m.push_back(H.Daug + mm + mm * H.Dld);
          ld.push_back(H.Dld);
          n.push_back(mm);
        }
      rc = run_symm(ctx, m, ld, n);
      if (rc) return rc;
      GemmJob<double> *dmj = nullptr;
      UCHK(ctx->upload(&dmj, mj, true));
      CHK(gemm_nt_batched<double>(dmj, (int)mj.size(), max_m, max_m, st));
    }
    // the matrices the iteration reads: in mixed precision an FP32 copy (the
    // restriction and the extension read the same rounded D, so the
    // preconditioner stays symmetric; a pair's second matrix is still
    // I - D^(1) of that copy)
    float *dall32 = nullptr;
    if (f32 && dtot > 0) {
      UCHK(ctx->dalloc(&dall32, dtot));
      CHK(cast_to_f32(dall, dall32, dtot, st));
    }
    for (auto &H : ctx->ents) {
      H.Dit.assign(H.D.size(), nullptr);
      for (size_t q = 0; q < H.D.size(); ++q)
        if (H.D[q]) H.Dit[q] = dall32 ? (const void *)(dall32 + (H.D[q] - dall)) : (const void *)H.D[q];
    }
  }
  CHK(mark(8));
  // ---- 9. iteration structures
  {
    // vectors
    UCHK(ctx->dalloc(&ctx->x, nTot));
    UCHK(ctx->dalloc(&ctx->r, nTot));
    UCHK(ctx->dalloc(&ctx->z, nTot));
    UCHK(ctx->dalloc(&ctx->p, nTot));
    UCHK(ctx->dalloc(&ctx->q, nTot));
    UCHK(ctx->dalloc(&ctx->tmp, nTot));
    UCHK(ctx->dalloc(&ctx->sc, SC_STRIDE * ctx->probs.size()));
    UCHK(ctx->dalloc(&ctx->part, std::max<int64_t>(2 * DOT_BLOCKS, (int64_t)ctx->seg_G * ctx->probs.size())));
    const int64_t nP = (int64_t)ctx->probs.size();
    UCHK(ctx->dalloc(&ctx->hist_a, (ctx->opt.maxit + 2) * nP));
    UCHK(ctx->dalloc(&ctx->hist_b, (ctx->opt.maxit + 2) * nP));
    // S_hat: per-subdomain bordered GEMV (reads p) + owner sums (into q)
    std::vector<GemvJob> js(nS);
    int64_t yoff = 0;
    for (int s = 0; s < nS; ++s) {
      SubH &S = ctx->subs[s];
      S.y_off = yoff;
      js[s] = {Xptr(S), S.xld, S.ng + 1, S.ng + 1, ctx->p, S.d_gidl, nullptr, nullptr, 1.0, 0,
               f32 ? 1 : 0};
      yoff += S.ng + 1;
    }
    ctx->n_yloc = yoff;
    ctx->schur_bytes_full = ctx->schur_bytes_sym = 0.0;
    for (auto &S : ctx->subs) {  // the bordered matrix once (its storage type) + x gather + y write
      const double n1 = S.ng + 1;
      ctx->schur_bytes_full += (double)ctx->wsz * n1 * n1 + 16.0 * n1;
      ctx->schur_bytes_sym += (double)ctx->wsz * n1 * (n1 + 1) * 0.5 + 16.0 * n1;
    }
    ctx->schur_bytes = ctx->ssym_on ? ctx->schur_bytes_sym : ctx->schur_bytes_full;
    UCHK(ctx->dalloc(&ctx->yloc, yoff));
    for (int s = 0; s < nS; ++s) js[s].y = ctx->yloc + ctx->subs[s].y_off;
    {  // the same operator through its lower triangle (tile partial sums in `part`)
      int64_t ptot = 0;
      for (auto &S : ctx->subs) ptot += (int64_t)symv_tiles(S.ng + 1) * 2 * SYMV_T;
      double *pbuf = nullptr;
      UCHK(ctx->dalloc(&pbuf, std::max<int64_t>(ptot, 1)));
      std::vector<SymvJob> sj(nS);
      int64_t po = 0;
      for (int s = 0; s < nS; ++s) {
        const SubH &S = ctx->subs[s];
        sj[s] = {Xptr(S), S.xld, S.ng + 1, f32 ? 1 : 0, ctx->p, S.d_gidl, js[s].y, 1.0, 0, pbuf + po};
        po += (int64_t)symv_tiles(S.ng + 1) * 2 * SYMV_T;
      }
      UCHK(ctx->upload(&ctx->j_ssym, sj));
    }
    std::vector<int64_t> ptr, idx;
    build_csr(nTot, [&](auto emit) {
      for (int s = 0; s < nS; ++s) {
        const SubH &S = ctx->subs[s];
        for (int l = 0; l < S.ng; ++l) emit(S.gidl[l], S.y_off + l);
        emit(nG + s, S.y_off + S.ng);
      }
    }, ptr, idx);
    UCHK(ctx->upload(&ctx->own_ptr, ptr));
    UCHK(ctx->upload(&ctx->own_idx, idx));
    // dual vectors: gD (restricted), wv (Neumann output), tv (Neumann [t1; t2])
    int64_t goff = 0, toff = 0;
    std::vector<int64_t> sgo(nS), sto(nS);
    for (int s = 0; s < nS; ++s) {
      sgo[s] = goff;
      sto[s] = toff;
      goff += ctx->subs[s].ndl;
      toff += ctx->subs[s].ndl + ctx->subs[s].npi;
    }
    ctx->n_gD = goff;
    ctx->n_tv = toff;
    UCHK(ctx->dalloc(&ctx->gD, goff));
    UCHK(ctx->dalloc(&ctx->wv, goff));
    UCHK(ctx->dalloc(&ctx->tv, toff));
    UCHK(ctx->dalloc(&ctx->rc, ctx->nCS));
    UCHK(ctx->dalloc(&ctx->uc, ctx->nCS));
    // restriction jobs per (entity, subdomain) with duals
    std::vector<GemvJob> jr;
    std::vector<ExtJob> ej;
    std::vector<ExtPart> ep;
    for (int e = 0; e < nE; ++e) {
      EntH &H = ctx->ents[e];
      const int m = H.n - H.rank;
      if (m <= 0) continue;
      const bool pair = H.D.size() == 2 && H.D[0] && !H.D[1];  // D^(2) = I - D^(1)
      ExtJob J{m, (int)H.subs.size(), (int)ep.size(), H.d_dual_gids, pair ? 1 : 0};
      std::vector<int64_t> wos;
      for (size_t qd = 0; qd < H.subs.size(); ++qd) {
        const int s = H.subs[qd];
        SubH &S = ctx->subs[s];
        int qq = (int)(std::find(S.ents.begin(), S.ents.end(), e) - S.ents.begin());
        wos.push_back(sgo[s] + S.doff[qq]);
        ep.push_back({H.Dit[qd], H.Dmld, wos.back(), 0.0, f32 ? 1 : 0});
      }
      if (pair) {  // g^(1) = D^(1)T r, g^(2) = r - g^(1): one read of D^(1)
        GemvJob G{H.Dit[0], H.Dmld, m, m, ctx->r, H.d_dual_gids, nullptr, ctx->gD + wos[0], 1.0, 0,
                  f32 ? 1 : 0};
        G.y2 = ctx->gD + wos[1];
        jr.push_back(G);
      } else {
        for (size_t qd = 0; qd < H.subs.size(); ++qd)
          jr.push_back({H.Dit[qd], H.Dmld, m, m, ctx->r, H.d_dual_gids, nullptr, ctx->gD + wos[qd], 1.0, 0,
                        f32 ? 1 : 0});
      }
      ej.push_back(J);
      ctx->max_rm = std::max(ctx->max_rm, m);
    }
    ctx->n_restrict = (int)jr.size();
    ctx->n_ext = (int)ej.size();
    ctx->max_ext_m = ctx->max_rm;
    UCHK(ctx->upload(&ctx->j_restrict, jr));
    UCHK(ctx->upload(&ctx->j_ext, ej));
    UCHK(ctx->upload(&ctx->j_extpart, ep));
    // Neumann jobs
    std::vector<GemvJob> jn1(nS), jn2(nS);
    for (int s = 0; s < nS; ++s) {
      SubH &S = ctx->subs[s];
      std::vector<int64_t> ci(S.cidx.begin(), S.cidx.end());
      int64_t *dci = nullptr;
      UCHK(ctx->upload(&dci, ci));
      const size_t gsz = ctx->fp32 ? sizeof(float) : sizeof(double);
      jn1[s] = {S.G1, std::max(S.ndl, 1), S.ndl, S.ndl + S.npi, ctx->gD + sgo[s], nullptr, nullptr,
                ctx->tv + sto[s], 1.0, 0, ctx->fp32 ? 1 : 0};
      jn2[s] = {(const char *)S.G1 + (int64_t)S.ndl * S.ndl * gsz, std::max(S.ndl, 1), S.ndl, S.npi,
                ctx->uc, dci, ctx->tv + sto[s], ctx->wv + sgo[s], 1.0, 0, ctx->fp32 ? 1 : 0};
    }
    {  // the same [S_DD^-1 | Phi]^T g as a symmetric product and a Phi^T g GEMV
      int64_t ptot = 0;
      for (auto &S : ctx->subs) ptot += (int64_t)symv_tiles(S.ndl) * 2 * SYMV_T;
      double *pbuf = nullptr;
      UCHK(ctx->dalloc(&pbuf, std::max<int64_t>(ptot, 1)));
      std::vector<SymvJob> nj(nS);
      std::vector<GemvJob> pj(nS);
      int64_t po = 0;
      const size_t gsz = ctx->fp32 ? sizeof(float) : sizeof(double);
      for (int s = 0; s < nS; ++s) {
        const SubH &S = ctx->subs[s];
        nj[s] = {S.G1, std::max(S.ndl, 1), S.ndl, ctx->fp32 ? 1 : 0, ctx->gD + sgo[s], nullptr,
                 ctx->tv + sto[s], 1.0, 0, pbuf + po};
        po += (int64_t)symv_tiles(S.ndl) * 2 * SYMV_T;
        pj[s] = {(const char *)S.G1 + (int64_t)S.ndl * S.ndl * gsz, std::max(S.ndl, 1), S.ndl, S.npi,
                 ctx->gD + sgo[s], nullptr, nullptr, ctx->tv + sto[s] + S.ndl, 1.0, 0,
                 ctx->fp32 ? 1 : 0};
      }
      UCHK(ctx->upload(&ctx->j_nsym, nj));
      UCHK(ctx->upload(&ctx->j_nphi, pj));
    }
    UCHK(ctx->upload(&ctx->j_schur, js));
    UCHK(ctx->upload(&ctx->j_neu1, jn1));
    UCHK(ctx->upload(&ctx->j_neu2, jn2));
    std::vector<GemvJob> jc;
    for (size_t pp = 0; pp < ctx->probs.size(); ++pp) {
      const auto &P = ctx->probs[pp];
      const int ncs = P.nprim + P.ns;
      jc.push_back({ctx->Gc + ctx->gc_off[pp], ncs, ncs, ncs, ctx->rc + P.cbase, nullptr, nullptr,
                    ctx->uc + P.cbase, 1.0, 0});
    }
    UCHK(ctx->upload(&ctx->j_coarse, jc));
    // coarse rhs: base = r at the primal positions (or p0), owners = Phi^T g contributions
    std::vector<int64_t> base(ctx->nCS), dst(ctx->nCS);
    for (int e = 0; e < nE; ++e) {
      EntH &H = ctx->ents[e];
      for (int j = 0; j < H.rank; ++j) base[ctx->ent_cbase[e] + j] = H.gids[j];
    }
    for (int s = 0; s < nS; ++s) base[ctx->sub_cp0[s]] = nG + s;
    std::vector<int64_t> cptr, cidx;
    build_csr(ctx->nCS, [&](auto emit) {
      for (int s = 0; s < nS; ++s) {
        const SubH &S = ctx->subs[s];
        for (int a = 0; a < S.npi; ++a) emit(S.cidx[a], sto[s] + S.ndl + a);
      }
    }, cptr, cidx);
    UCHK(ctx->upload(&ctx->c_ptr, cptr));
    UCHK(ctx->upload(&ctx->c_idx, cidx));
    UCHK(ctx->upload(&ctx->c_base, base));
    UCHK(ctx->upload(&ctx->uc_dst, base));
    for (auto &S : ctx->subs) {
      ctx->max_gt_m = std::max(ctx->max_gt_m, S.ng + 1);
      ctx->max_nt = std::max(ctx->max_nt, S.ndl + S.npi);
    }
  }
  // tile shapes of the per-iteration GEMVs, once per context
  if (!ctx->cpb[0]) {
    int rc = autotune_gemvs(ctx);
    if (rc) return rc;
  }
  CHK(mark(9));
  // ---- 10. recovery structures (second level first, then the fronts)
  {
    const int nF = (int)ctx->fronts.size();
    std::vector<int64_t> yoff(nS), invoff(nS), yofff(nF), invofff(nF);
    int64_t tot = 0, otot = 0;
    ctx->rec_off.assign(nS + 1, 0);
    for (int s = 0; s < nS; ++s) {
      yoff[s] = tot;
      tot += ctx->subs[s].e + 1;
      invoff[s] = ctx->subs[s].inv_off;
      ctx->rec_off[s + 1] = ctx->rec_off[s] + ctx->subs[s].n;
    }
    for (int f = 0; f < nF; ++f) {
      yofff[f] = tot;
      tot += ctx->fronts[f].S.e + 1;
      invofff[f] = ctx->fronts[f].S.inv_off;
    }
    otot = ctx->rec_off[nS];
    UCHK(ctx->dalloc(&ctx->yrec, tot));
    UCHK(ctx->dalloc(&ctx->zrec, tot));
    UCHK(ctx->dalloc(&ctx->rec_out, otot));
    UCHK(ctx->upload(&ctx->d_yoff, yoff));
    UCHK(ctx->upload(&ctx->d_invoff, invoff));
    // second-level jobs: separator and interface outputs; in the two-level
    // case also the separator values and the sub-box constants into G2
    auto l2job = [&](int s, const double *z, double *out) {
      SubH &S = ctx->subs[s];
      RecJob J{s, S.n2, S.nv, S.nel, S.d_kind, S.d_pos, S.d_gid, ctx->hv + S.hv_off, z, out};
      if (ctx->nd) {
        J.oidx = S.d_oidx;
        J.sep_out = ctx->G2 + ctx->nG + nS + S.sep_off;
        J.c_out = ctx->G2 + ctx->g2_c0 + S.first_front;
      }
      return J;
    };
    // front jobs: interior velocity and pressure outputs (constant = G2 entry)
    auto frjob = [&](int f, const double *z, double *out) {
      FrontH &F = ctx->fronts[f];
      SubH &T = F.S;
      RecJob J{f, T.n, T.nv, T.nel, T.d_kind, T.d_pos, T.d_gid, ctx->hvf + T.hv_off, z, out};
      J.oidx = F.d_oidx;
      return J;
    };
    std::vector<RecJob> rj(nS), rjf(nF);
    for (int s = 0; s < nS; ++s) rj[s] = l2job(s, ctx->zrec + yoff[s], ctx->rec_out + ctx->rec_off[s]);
    for (int f = 0; f < nF; ++f)
      rjf[f] = frjob(f, ctx->zrec + yofff[f], ctx->rec_out + ctx->rec_off[ctx->fronts[f].sub]);
    UCHK(ctx->upload(&ctx->j_rec, rj));
    if (nF) {
      UCHK(ctx->upload(&ctx->d_yofff, yofff));
      UCHK(ctx->upload(&ctx->d_invofff, invofff));
      UCHK(ctx->upload(&ctx->j_recf, rjf));
    }
    if (ctx->fp32) {  // refinement buffers: dense per-subdomain / per-front vectors of length N
      std::vector<int64_t> yoff2(nS), uoff(nS), yoff2f(nF), roff(nF);
      int64_t t2 = 0;
      for (int s = 0; s < nS; ++s) {
        yoff2[s] = t2;
        t2 += ctx->subs[s].N;
        uoff[s] = ctx->rec_off[s];
      }
      ctx->n_ir2 = t2;
      for (int f = 0; f < nF; ++f) {
        yoff2f[f] = t2;
        t2 += ctx->fronts[f].S.N;
        roff[f] = ctx->rec_off[ctx->fronts[f].sub];
      }
      ctx->n_ir = t2;
      UCHK(ctx->dalloc(&ctx->y_ir, t2));
      UCHK(ctx->dalloc(&ctx->z_ir, t2));
      UCHK(ctx->dalloc(&ctx->zst, t2));
      UCHK(ctx->dalloc(&ctx->x_last, nG + nS));
      CHK(hipMemsetAsync(ctx->y_ir, 0, t2 * sizeof(double), st));
      CHK(hipMemsetAsync(ctx->z_ir, 0, t2 * sizeof(double), st));
      UCHK(ctx->dalloc(&ctx->u_loc, otot));
      UCHK(ctx->dalloc(&ctx->R_loc, otot));
      UCHK(ctx->dalloc(&ctx->r0, nS));
      UCHK(ctx->dalloc(&ctx->dgv, nG + nS));
      UCHK(ctx->dalloc(&ctx->dx, nG + nS));
      UCHK(ctx->upload(&ctx->d_yoff2, yoff2));
      UCHK(ctx->upload(&ctx->d_uoff, uoff));
      {
        std::vector<GemvJob> jb(nS), jbf(nF);
        ctx->brhs_m = ctx->brhs_mf = 0;
        auto job = [&](const SubDev &D, const double *x, double *y) {
          return GemvJob{(const char *)D.W + (int64_t)(D.e + 1) * (int64_t)ctx->wsz, D.ld, D.ng, D.e, x, D.gidl,
                         nullptr, y, -1.0, 1, 1};
        };
        for (int s = 0; s < nS; ++s) {
          jb[s] = job(ctx->subdev[s], ctx->dx, ctx->y_ir + yoff2[s]);
          ctx->brhs_m = std::max(ctx->brhs_m, ctx->subdev[s].ng);
        }
        for (int f = 0; f < nF; ++f) {
          jbf[f] = job(ctx->frdev[f], ctx->G2d, ctx->y_ir + yoff2f[f]);
          ctx->brhs_mf = std::max(ctx->brhs_mf, ctx->frdev[f].ng);
        }
        UCHK(ctx->upload(&ctx->j_brhs, jb));
        if (nF) UCHK(ctx->upload(&ctx->j_brhsf, jbf));
      }
      std::vector<RecJob> rj2(nS), rj2f(nF);
      for (int s = 0; s < nS; ++s) rj2[s] = l2job(s, ctx->zst + yoff2[s], ctx->u_loc + ctx->rec_off[s]);
      UCHK(ctx->upload(&ctx->j_rec_ir, rj2));
      std::vector<int64_t> ptr, idx;
      build_csr(nG, [&](auto emit) {
        for (int s = 0; s < nS; ++s) {
          const SubH &S = ctx->subs[s];
          for (int l = 0; l < S.ng; ++l) emit(S.gidl[l], yoff2[s] + S.e + 1 + l);
        }
      }, ptr, idx);
      UCHK(ctx->upload(&ctx->ir_ptr, ptr));
      UCHK(ctx->upload(&ctx->ir_idx, idx));
      if (nF) {
        for (int f = 0; f < nF; ++f)
          rj2f[f] = frjob(f, ctx->zst + yoff2f[f], ctx->u_loc + ctx->rec_off[ctx->fronts[f].sub]);
        UCHK(ctx->upload(&ctx->j_rec_irf, rj2f));
        UCHK(ctx->upload(&ctx->d_yoff2f, yoff2f));
        UCHK(ctx->upload(&ctx->d_roff_f, roff));
        UCHK(ctx->dalloc(&ctx->r0f, nF));
        // front residual rows -> second-level residual, one list per sub-box index
        ctx->fj_rhs.assign(ctx->max_nbox, {});
        for (int s = 0; s < nS; ++s) {
          const SubH &S = ctx->subs[s];
          for (int b = 0; b < S.nbox; ++b) {
            const int f = S.first_front + b;
            const FrontH &F = ctx->fronts[f];
            FrontJob J{};
            J.e = F.S.e;
            J.m = F.S.ng + 2;
            J.map = F.d_map;
            J.gamma = F.gamma;
            J.yf = ctx->y_ir + yoff2f[f];
            J.y2 = ctx->y_ir + yoff2[s];
            ctx->fj_rhs[b].push_back(J);
          }
        }
        ctx->d_fj_rhs.assign(ctx->max_nbox, nullptr);
        for (int b = 0; b < ctx->max_nbox; ++b) UCHK(ctx->upload(&ctx->d_fj_rhs[b], ctx->fj_rhs[b]));
        // separator corrections of the second level -> G2d
        std::vector<int64_t> src, dst;
        for (int s = 0; s < nS; ++s) {
          const SubH &S = ctx->subs[s];
          for (int k = 0; k < S.nsep; ++k) {
            src.push_back(yoff2[s] + k);
            dst.push_back(ctx->nG + nS + S.sep_off + k);
          }
        }
        UCHK(ctx->upload(&ctx->sep_src, src));
        UCHK(ctx->upload(&ctx->sep_dst, dst));
      }
    }
  }
  CHK(hipEventRecord(ctx->ev1, st));
  CHK(hipEventSynchronize(ctx->ev1));
  float ms = 0.f;
  CHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  ctx->setup_ms = ms;
  for (int ph = 1; ph <= vb_ctx::kPhases; ++ph) {
    hipEvent_t a = ph == 1 ? ctx->ev0 : ctx->ph_ev[ph - 1];
    hipEvent_t b = ph == vb_ctx::kPhases ? ctx->ev1 : ctx->ph_ev[ph];
    float t = 0.f;
    ctx->phase_ms[ph - 1] = (a && b && hipEventElapsedTime(&t, a, b) == hipSuccess) ? t : -1.0;
  }
  // setup-only workspace (Neumann/deluxe augmented matrices, job arrays) is
  // released by the caller of setup_impl
  for (auto &H : ctx->ents) {
    H.Daug = nullptr;
    H.Sbar.clear();
  }
  for (auto &S : ctx->subs) S.Nmat = nullptr;
  ctx->Kaug = nullptr;
  ctx->p0_src = ctx->p0_dst = nullptr;
  ctx->g_ptr = ctx->g_idx = nullptr;
  ctx->state = 2;
  return VB_OK;
}


}  // extern "C"

// ------------------------------------------------------------------ operators
static int apply_S_internal(vb_ctx *ctx) {  // q <- S~ p
  KTimer *t = ctx->opt.profile ? &ctx->t_gemv : nullptr;
  if (t) CHK(t->begin(ctx->stream, ctx->schur_bytes));
  if (ctx->ssym_on)
    CHK(symv(ctx->j_ssym, ctx->nS, ctx->max_gt_m, ctx->stream));
  else
    CHK(gemv_t_cpb(ctx->j_schur, ctx->nS, ctx->max_gt_m, ctx->max_gt_m,
                   ctx->cpb[0] ? ctx->cpb[0] : 32, ctx->stream));
  if (t) CHK(t->end(ctx->stream));
  CHK(owner_sum((int)(ctx->nG + ctx->nS), ctx->own_ptr, ctx->own_idx, ctx->yloc, nullptr, nullptr,
                ctx->q, ctx->stream));
  return VB_OK;
}

static int apply_M_internal(vb_ctx *ctx) {  // z <- M~^-1 r
  hipStream_t st = ctx->stream;
  auto cp = [&](int k) { return ctx->cpb[k] ? ctx->cpb[k] : 32; };
  if (ctx->n_restrict)
    CHK(gemv_t_cpb(ctx->j_restrict, ctx->n_restrict, ctx->max_rm, ctx->max_rm, cp(2), st));
  if (ctx->nsym_on) {
    CHK(symv(ctx->j_nsym, ctx->nS, ctx->max_ndl, st));
    CHK(gemv_t_cpb(ctx->j_nphi, ctx->nS, ctx->max_ndl, ctx->max_npi, cp(1), st));
  } else {
    CHK(gemv_t_cpb(ctx->j_neu1, ctx->nS, ctx->max_ndl, ctx->max_nt, cp(1), st));
  }
  CHK(owner_sum(ctx->nCS, ctx->c_ptr, ctx->c_idx, ctx->tv, ctx->c_base, ctx->r, ctx->rc, st));
  CHK(gemv_t_cpb(ctx->j_coarse, (int)ctx->probs.size(), ctx->max_ncs, ctx->max_ncs, cp(3), st));
  if (ctx->max_ndl) CHK(gemv_n(ctx->j_neu2, ctx->nS, ctx->max_ndl, ctx->max_npi, st));
  if (ctx->n_ext) CHK(extend(ctx->j_ext, ctx->n_ext, ctx->max_ext_m, ctx->j_extpart, ctx->wv, ctx->z, st));
  CHK(scatter_copy(ctx->nCS, ctx->uc, nullptr, ctx->uc_dst, ctx->z, 1.0, st));
  return VB_OK;
}

// Autotuner of the per-iteration GEMVs: each candidate tile shape (columns
// per workgroup) is timed with HIP events on the operator's own jobs (one
// warm-up and three timed launches; the outputs are scratch at this point)
// and the fastest is kept for this context.
static int autotune_gemvs(vb_ctx *ctx) {
  hipStream_t st = ctx->stream;
  struct Cand {
    const GemvJob *jobs;
    int batch, m, n;
  } ops[4] = {{ctx->j_schur, ctx->nS, ctx->max_gt_m, ctx->max_gt_m},
              {ctx->j_neu1, ctx->nS, ctx->max_ndl, ctx->max_nt},
              {ctx->j_restrict, ctx->n_restrict, ctx->max_rm, ctx->max_rm},
              {ctx->j_coarse, (int)ctx->probs.size(), ctx->max_ncs, ctx->max_ncs}};
  static const int choices[] = {8, 16, 32, 64};
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  for (int k = 0; k < 4; ++k) {
    const Cand &c = ops[k];
    if (!c.jobs || c.batch <= 0 || c.n <= 0 || c.m <= 0) {
      ctx->cpb[k] = 32;
      continue;
    }
    float best = 1e30f;
    int pick = 32;
    for (int cpb : choices) {
      CHK(gemv_t_cpb(c.jobs, c.batch, c.m, c.n, cpb, st));
      CHK(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) CHK(gemv_t_cpb(c.jobs, c.batch, c.m, c.n, cpb, st));
      CHK(hipEventRecord(e1, st));
      CHK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        pick = cpb;
      }
    }
    ctx->cpb[k] = pick;
    if (k == 0) {  // S~ p: the lower-triangle kernel against the best full-matrix tile
      CHK(symv(ctx->j_ssym, ctx->nS, ctx->max_gt_m, st));
      CHK(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) CHK(symv(ctx->j_ssym, ctx->nS, ctx->max_gt_m, st));
      CHK(hipEventRecord(e1, st));
      CHK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHK(hipEventElapsedTime(&ms, e0, e1));
      ctx->ssym_on = ctx->opt.schur_kernel == 2 || (ctx->opt.schur_kernel == 0 && ms < best);
      ctx->schur_bytes = ctx->ssym_on ? ctx->schur_bytes_sym : ctx->schur_bytes_full;
    }
    if (k == 1) {  // [S_DD^-1 | Phi]^T g: symmetric block + Phi block against the full GEMV
      auto both = [&]() -> hipError_t {
        hipError_t e = symv(ctx->j_nsym, ctx->nS, ctx->max_ndl, st);
        if (e == hipSuccess && ctx->max_npi > 0)
          e = gemv_t_cpb(ctx->j_nphi, ctx->nS, ctx->max_ndl, ctx->max_npi, pick, st);
        return e;
      };
      CHK(both());
      CHK(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) CHK(both());
      CHK(hipEventRecord(e1, st));
      CHK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHK(hipEventElapsedTime(&ms, e0, e1));
      ctx->nsym_on = ctx->opt.schur_kernel == 2 || (ctx->opt.schur_kernel == 0 && ms < best);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return VB_OK;
}

extern "C" {

int vb_rhs(vb_ctx *ctx, double *g_dev) {
  if (!ctx || !g_dev) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_rhs: call vb_setup first");
  const int64_t n = ctx->nG + ctx->nS;
  CHK(hipMemcpyAsync(g_dev, ctx->g, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  CHK(transform_vec(ctx->d_entdev, (int)ctx->ents.size(), g_dev, -1, ctx->stream));
  return VB_OK;
}

int vb_schur_apply(vb_ctx *ctx, const double *x_dev, double *y_dev) {
  if (!ctx || !x_dev || !y_dev) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_schur_apply: call vb_setup first");
  const int64_t n = ctx->nG + ctx->nS;
  CHK(hipMemcpyAsync(ctx->p, x_dev, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  CHK(transform_vec(ctx->d_entdev, (int)ctx->ents.size(), ctx->p, +1, ctx->stream));
  int rc = apply_S_internal(ctx);
  if (rc) return rc;
  CHK(hipMemcpyAsync(y_dev, ctx->q, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  CHK(transform_vec(ctx->d_entdev, (int)ctx->ents.size(), y_dev, -1, ctx->stream));
  return VB_OK;
}

int vb_apply(vb_ctx *ctx, const double *r_dev, double *z_dev) {
  if (!ctx || !r_dev || !z_dev) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_apply: call vb_setup first");
  const int64_t n = ctx->nG + ctx->nS;
  CHK(hipMemcpyAsync(ctx->r, r_dev, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  CHK(transform_vec(ctx->d_entdev, (int)ctx->ents.size(), ctx->r, +1, ctx->stream));
  int rc = apply_M_internal(ctx);
  if (rc) return rc;
  CHK(hipMemcpyAsync(z_dev, ctx->z, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  CHK(transform_vec(ctx->d_entdev, (int)ctx->ents.size(), z_dev, -1, ctx->stream));
  return VB_OK;
}

}  // extern "C"

// extreme eigenvalues of the symmetric tridiagonal CG-Lanczos matrix
// (T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_j,j+1 = sqrt(b_j)/a_j) by bisection.
static void lanczos_extremes(const std::vector<double> &a, const std::vector<double> &b,
                             double *lmin, double *lmax) {
  const int m = (int)a.size();
  *lmin = *lmax = NAN;
  if (m == 0) return;
  std::vector<double> d(m), e(m, 0.0);
  for (int j = 0; j < m; ++j) {
    d[j] = 1.0 / a[j] + (j > 0 ? b[j - 1] / a[j - 1] : 0.0);
    if (j + 1 < m) e[j] = std::sqrt(std::fabs(b[j])) / a[j];
  }
  double lo = 1e300, hi = -1e300;
  for (int j = 0; j < m; ++j) {
    double rad = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(e[j]) : 0.0);
    lo = std::min(lo, d[j] - rad);
    hi = std::max(hi, d[j] + rad);
  }
  auto count_below = [&](double x) {  // Sturm count of eigenvalues < x
    int c = 0;
    double q = d[0] - x;
    if (q < 0) c++;
    for (int j = 1; j < m; ++j) {
      if (q == 0.0) q = 1e-300;
      q = d[j] - x - e[j - 1] * e[j - 1] / q;
      if (q < 0) c++;
    }
    return c;
  };
  auto kth = [&](int k) {  // k-th smallest (0-based)
    double l = lo, h = hi;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (l + h);
      if (count_below(mid) > k) h = mid; else l = mid;
    }
    return 0.5 * (l + h);
  };
  *lmin = kth(0);
  *lmax = kth(m - 1);
}

extern "C" {

}  // extern "C"

// PCG on S~ x~ = b~ in the transformed coordinates (Sec. 7), on ctx->x, for
// every problem of the context at once: the operators are block diagonal
// over the problems, the recurrences keep one set of scalars per problem
// (segmented reductions), and a problem that has converged keeps its
// iterate (alpha = 0) while the others continue.
// x_zero: start from x~ = 0 (r = b) instead of the current ctx->x.
// tol[p]: relative tolerance of problem p.  The Lanczos coefficients of each
// problem are kept in hist_a/hist_b (leading dimension maxit + 2).
struct PcgResult {
  int it = 0, status = VB_OK;  // over all problems: largest count, worst status
  double rel = 0.0;
  std::vector<double> sc;      // per-problem scalars at exit (SC_STRIDE each)
};

static int pcg_body(vb_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const int P = (int)ctx->probs.size(), G = ctx->seg_G, ld = ctx->opt.maxit + 2;
  int rc = apply_S_internal(ctx);
  if (rc) return rc;
  CHK(sdot(ctx->d_segs, P, G, ctx->p, ctx->q, ctx->part, ctx->sc, 0, ctx->hist_a, nullptr, ld, st));
  CHK(supdate_xr(ctx->d_segs, P, G, ctx->sc, ctx->x, ctx->r, ctx->p, ctx->q, ctx->part, st));
  rc = apply_M_internal(ctx);
  if (rc) return rc;
  CHK(sdot(ctx->d_segs, P, G, ctx->r, ctx->z, ctx->part, ctx->sc, 2, nullptr, ctx->hist_b, ld, st));
  CHK(supdate_p(ctx->d_segs, P, G, ctx->sc, ctx->p, ctx->z, st));
  return VB_OK;
}

// The phases of pcg_body as one plan for the persistent launch (the same
// jobs, grids and autotuned tiles).  False when the iteration does not fit
// it (the Neumann primal vectors staged in LDS exceed its buffer).
static bool persistent_plan(vb_ctx *ctx) {
  if (ctx->max_npi > 2048) return false;
  auto cp = [&](int k) { return ctx->cpb[k] ? ctx->cpb[k] : 32; };
  auto ph = [&](const GemvJob *j, int batch, int max_n, int cpb) {
    GemvPhase g{j, (j && max_n > 0) ? batch : 0, (max_n + cpb - 1) / cpb, cpb};
    return g;
  };
  PcgPlan &L = ctx->plan_h;
  L = PcgPlan{};
  L.schur = ph(ctx->j_schur, ctx->nS, ctx->max_gt_m, cp(0));
  if (ctx->ssym_on) {
    L.ssym = ctx->j_ssym;
    L.ssym_batch = ctx->nS;
    L.ssym_tiles = symv_tiles(ctx->max_gt_m);
    L.ssym_rows = ctx->max_gt_m;
  }
  L.restrict_ = ph(ctx->j_restrict, ctx->n_restrict, ctx->max_rm, cp(2));
  L.neu1 = ph(ctx->j_neu1, ctx->nS, ctx->max_nt, cp(1));
  if (ctx->nsym_on) {
    L.nsym = ctx->j_nsym;
    L.nsym_batch = ctx->nS;
    L.nsym_tiles = symv_tiles(ctx->max_ndl);
    L.nsym_rows = ctx->max_ndl;
    L.nphi = ph(ctx->j_nphi, ctx->nS, ctx->max_npi, cp(1));
  }
  L.coarse = ph(ctx->j_coarse, (int)ctx->probs.size(), ctx->max_ncs, cp(3));
  L.neu2 = GemvPhase{ctx->j_neu2, ctx->max_ndl ? ctx->nS : 0, (ctx->max_ndl + 255) / 256, 0};
  L.ext = ctx->j_ext;
  L.extpart = ctx->j_extpart;
  L.n_ext = ctx->n_ext;
  L.ext_gx = (ctx->max_ext_m + 127) / 128;
  L.wv = ctx->wv;
  L.n_own = (int)(ctx->nG + ctx->nS);
  L.own_ptr = ctx->own_ptr;
  L.own_idx = ctx->own_idx;
  L.yloc = ctx->yloc;
  L.n_cs = ctx->nCS;
  L.c_ptr = ctx->c_ptr;
  L.c_idx = ctx->c_idx;
  L.c_base = ctx->c_base;
  L.tv = ctx->tv;
  L.rc = ctx->rc;
  L.uc = ctx->uc;
  L.uc_dst = ctx->uc_dst;
  L.segs = ctx->d_segs;
  L.P = (int)ctx->probs.size();
  L.G = ctx->seg_G;
  L.part = ctx->part;
  L.sc = ctx->sc;
  L.hist_a = ctx->hist_a;
  L.hist_b = ctx->hist_b;
  L.hist_ld = ctx->opt.maxit + 2;
  L.x = ctx->x;
  L.r = ctx->r;
  L.p = ctx->p;
  L.q = ctx->q;
  L.z = ctx->z;
  L.bar = ctx->d_pbar;
  L.err = (int *)(ctx->d_pbar + 2);
  L.max_iter = ctx->opt.maxit + 1;
  return true;
}

static int pcg_loop(vb_ctx *ctx, int maxit, std::vector<double> &hs);

// Whether pcg_core runs its iterations as one persistent launch.
static bool use_persistent(vb_ctx *ctx) {
  if (ctx->opt.profile || ctx->opt.pcg_launch == VB_PCG_GRAPH) return false;
  if (ctx->opt.pcg_launch == VB_PCG_AUTO && ctx->schur_bytes >= 1e9) return false;
  if (ctx->pnb < 0) ctx->pnb = pcg_persistent_blocks(2);
  return ctx->pnb > 0;
}

static int pcg_core(vb_ctx *ctx, const double *b, bool x_zero, const std::vector<double> &tol,
                    int maxit, PcgResult *res) {
  hipStream_t st = ctx->stream;
  const int P = (int)ctx->probs.size(), G = ctx->seg_G, ld = ctx->opt.maxit + 2;
  const int64_t n = ctx->nG + ctx->nS;
  maxit = std::max(0, std::min(maxit, ctx->opt.maxit));
  CHK(hipMemcpyAsync(ctx->d_tol, tol.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
  CHK(sinit(P, ctx->d_tol, maxit, ctx->sc, st));
  if (x_zero) {
    CHK(hipMemsetAsync(ctx->x, 0, n * sizeof(double), st));
    CHK(hipMemcpyAsync(ctx->r, b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    CHK(hipMemcpyAsync(ctx->p, ctx->x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    int rc = apply_S_internal(ctx);
    if (rc) return rc;
    CHK(vsub(n, b, ctx->q, ctx->r, st));
  }
  CHK(sdot(ctx->d_segs, P, G, b, b, ctx->part, ctx->sc, 4, nullptr, nullptr, ld, st));
  CHK(sdot(ctx->d_segs, P, G, ctx->r, ctx->r, ctx->part, ctx->sc, 6, nullptr, nullptr, ld, st));
  int rc = apply_M_internal(ctx);
  if (rc) return rc;
  CHK(sdot(ctx->d_segs, P, G, ctx->r, ctx->z, ctx->part, ctx->sc, 3, nullptr, nullptr, ld, st));
  CHK(hipMemcpyAsync(ctx->p, ctx->z, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<double> hs((size_t)P * SC_STRIDE);
  bool persisted = false;
  if (use_persistent(ctx)) {
    if (!ctx->d_plan) {
      UCHK(ctx->dalloc((char **)&ctx->d_plan, sizeof(PcgPlan)));
      UCHK(ctx->dalloc(&ctx->d_pbar, 4));
    }
    if (!ctx->plan_valid) {
      if (!persistent_plan(ctx)) {
        ctx->pnb = 0;
      } else {
        CHK(hipMemcpyAsync(ctx->d_plan, &ctx->plan_h, sizeof(PcgPlan), hipMemcpyHostToDevice, st));
        ctx->plan_valid = true;
      }
    }
    if (ctx->pnb > 0) {
      // every problem's sc[MAXIT] is this call's maxit (sinit above)
      CHK(hipMemsetAsync(ctx->d_pbar, 0, 4 * sizeof(unsigned), st));
      hipError_t e = pcg_persistent(ctx->d_plan, ctx->pnb, st);
      if (e == hipSuccess) {
        unsigned flag[4] = {0, 0, 0, 0};
        CHK(hipMemcpyAsync(flag, ctx->d_pbar, sizeof(flag), hipMemcpyDeviceToHost, st));
        CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        CHK(hipStreamSynchronize(st));
        if (flag[2])
          return ctx->fail(VB_ERR_DEVICE, "persistent PCG launch: a grid barrier timed out");
        persisted = true;
        ctx->last_launch = VB_PCG_PERSISTENT;
      } else {  // cooperative launch refused: the graph-replayed iteration from now on
        (void)hipGetLastError();
        ctx->pnb = 0;
      }
    }
  }
  if (!persisted) {
    rc = pcg_loop(ctx, maxit, hs);
    if (rc) return rc;
    ctx->last_launch = VB_PCG_GRAPH;
  }
  res->it = 0;
  res->rel = 0.0;
  res->status = VB_OK;
  for (int pp = 0; pp < P; ++pp) {
    const double *q = hs.data() + (size_t)pp * SC_STRIDE;
    res->it = std::max(res->it, (int)q[SC_IT]);
    const double rel = q[SC_GG] > 0 ? std::sqrt(q[SC_RR] / q[SC_GG]) : 0.0;
    res->rel = std::max(res->rel, rel);
    if (q[SC_FLAG] == 1.0) res->status = VB_ERR_BREAKDOWN;
    else if ((q[SC_FLAG] == 2.0 || q[SC_DONE] == 0.0) && res->status == VB_OK)
      res->status = VB_ERR_NOT_CONVERGED;
  }
  res->sc = hs;
  return VB_OK;
}

// The iterations launch by launch: the first eagerly (it also runs every
// one-time attribute call), the rest as a replayed HIP graph of one
// iteration when a stream of our own is given and launches are not being
// timed one by one; the host reads the per-problem flags every `every`
// iterations (the flags freeze converged problems in between).
static int pcg_loop(vb_ctx *ctx, int maxit, std::vector<double> &hs) {
  hipStream_t st = ctx->stream;
  const int P = (int)ctx->probs.size();
  int rc = VB_OK;
  const bool graph_ok = ctx->stream != nullptr && !ctx->opt.profile;
  const int every = (ctx->schur_bytes * (8.0 / ctx->wsz) > 4e8) ? 1 : 4;
  CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  auto all_done = [&]() {
    for (int pp = 0; pp < P; ++pp)
      if (hs[(size_t)pp * SC_STRIDE + SC_DONE] == 0.0) return false;
    return true;
  };
  int launched = 0;
  bool first = true;
  while (!all_done() && launched < maxit + every) {
    for (int k = 0; k < every; ++k) {
      if (graph_ok && !first) {
        if (!ctx->it_exec) {
          CHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          int rc2 = pcg_body(ctx);
          hipError_t e = hipStreamEndCapture(st, &ctx->it_graph);
          if (rc2) return rc2;
          CHK(e);
          CHK(hipGraphInstantiate(&ctx->it_exec, ctx->it_graph, nullptr, nullptr, 0));
        }
        CHK(hipGraphLaunch(ctx->it_exec, st));
      } else {  // the first iteration also runs every one-time attribute call
        rc = pcg_body(ctx);
        if (rc) return rc;
        first = false;
      }
      ++launched;
    }
    CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
  }
  return VB_OK;
}

static int lanczos_problem(vb_ctx *ctx, int pp, int it, double *lmin, double *lmax) {
  const int ld = ctx->opt.maxit + 2;
  std::vector<double> a(it), b(it > 0 ? it - 1 : 0);
  if (it) CHK(hipMemcpy(a.data(), ctx->hist_a + (int64_t)pp * ld, it * sizeof(double), hipMemcpyDeviceToHost));
  if (it > 1) CHK(hipMemcpy(b.data(), ctx->hist_b + (int64_t)pp * ld, (it - 1) * sizeof(double), hipMemcpyDeviceToHost));
  lanczos_extremes(a, b, lmin, lmax);
  return VB_OK;
}

// Combined info over the problems (the single problem's own when there is one).
static void combine_info(const std::vector<vb_solve_info> &pi, vb_solve_info *out) {
  *out = pi[0];
  for (size_t k = 1; k < pi.size(); ++k) {
    const vb_solve_info &q = pi[k];
    out->iterations = std::max(out->iterations, q.iterations);
    out->refinement_steps = std::max(out->refinement_steps, q.refinement_steps);
    out->rel_residual = std::max(out->rel_residual, q.rel_residual);
    out->true_rel_residual = std::max(out->true_rel_residual, q.true_rel_residual);
    out->lambda_min = std::min(out->lambda_min, q.lambda_min);
    out->lambda_max = std::max(out->lambda_max, q.lambda_max);
    out->latency_ms = std::max(out->latency_ms, q.latency_ms);
    if (q.status != VB_OK && out->status == VB_OK) out->status = q.status;
  }
}

// One pass of the FP64 residual condensation used by the refinement:
// u = local vectors from (zst, x); R = f - K u (FP64, sparse); y = R in the
// dense order with rotated pressures; forward substitution with the stored
// factor over the eliminated columns (eq. uipi); on return the rows e+1.. of
// y hold the condensed interface residual of every subdomain and r0 the
// residual of its constant-pressure equation.
// u_loc <- the local solution vectors from the interior state zst and the
// interface vector x (two-level: second level first, writing the separator
// values and sub-box constants into G2, then the fronts).
static int state_to_local(vb_ctx *ctx, const double *x_orig) {
  hipStream_t st = ctx->stream;
  CHK(recover_out(ctx->j_rec_ir, ctx->nS, x_orig, ctx->nG, st));
  if (ctx->nd)
    CHK(recover_out(ctx->j_rec_irf, (int)ctx->fronts.size(), ctx->G2, ctx->g2_c0, st));
  return VB_OK;
}

// Two-level version of condense_residual: the local residual in every front,
// forward-substituted through the front's factor; its trailing rows added
// into the second-level residual (in sub-box order) with the separator and
// interface rows of the local residual; then the second-level forward
// substitution.
static int condense_residual_nd(vb_ctx *ctx, const double *x_orig) {
  hipStream_t st = ctx->stream;
  const int nS = ctx->nS, nF = (int)ctx->fronts.size(), nb = dir_nb(ctx, 0), nb2 = dir_nb(ctx, 1);
  CHK(hipMemcpyAsync(ctx->G2, x_orig, (ctx->nG + nS) * sizeof(double), hipMemcpyDeviceToDevice, st));
  int rc = state_to_local(ctx, x_orig);
  if (rc) return rc;
  CHK(local_residual(ctx->d_fulldev, ctx->u_loc, ctx->d_uoff, ctx->R_loc, nS, ctx->max_n_full, st));
  CHK(residual_to_dense(ctx->d_frdev, ctx->R_loc, ctx->d_roff_f, ctx->y_ir, ctx->d_yoff2f, ctx->r0f, nF,
                        ctx->max_nf_csr, st));
  for (int i0 = 0; i0 < ctx->max_ef; i0 += nb)
    CHK(forward_step(ctx->d_frdev, ctx->invLf, ctx->d_invofff, ctx->y_ir, ctx->z_ir, ctx->d_yoff2f, nF,
                     i0, nb, ctx->max_Nf, ctx->fp32, st));
  CHK(hipMemsetAsync(ctx->y_ir, 0, ctx->n_ir2 * sizeof(double), st));
  for (int b = 0; b < ctx->max_nbox; ++b)
    CHK(front_rhs(ctx->d_fj_rhs[b], (int)ctx->fj_rhs[b].size(), st));
  CHK(l2_residual(ctx->d_subdev, ctx->R_loc, ctx->d_uoff, ctx->y_ir, ctx->d_yoff2, nS, st));
  CHK(segment_sum(nS, ctx->d_fr_first, ctx->r0f, ctx->r0, st));
  for (int i0 = 0; i0 < ctx->max_e; i0 += nb2)
    CHK(forward_step(ctx->d_subdev, ctx->invL, ctx->d_invoff, ctx->y_ir, ctx->z_ir, ctx->d_yoff2, nS, i0,
                     nb2, ctx->max_N, ctx->fp32, st));
  return VB_OK;
}

static int condense_residual(vb_ctx *ctx, const double *x_orig) {
  if (ctx->nd) return condense_residual_nd(ctx, x_orig);
  hipStream_t st = ctx->stream;
  CHK(recover_out(ctx->j_rec_ir, ctx->nS, x_orig, ctx->nG, st));
  CHK(local_residual(ctx->d_subdev, ctx->u_loc, ctx->d_uoff, ctx->R_loc, ctx->nS, ctx->max_n_csr,
                     st));
  CHK(residual_to_dense(ctx->d_subdev, ctx->R_loc, ctx->d_uoff, ctx->y_ir, ctx->d_yoff2, ctx->r0,
                        ctx->nS, ctx->max_n_csr, st));
  const int nb = dir_nb(ctx, 0);
  for (int i0 = 0; i0 < ctx->max_e; i0 += nb)
    CHK(forward_step(ctx->d_subdev, ctx->invL, ctx->d_invoff, ctx->y_ir, ctx->z_ir, ctx->d_yoff2,
                     ctx->nS, i0, nb, ctx->max_N, ctx->fp32, st));
  return VB_OK;
}

// Interior correction for an interface correction dx (null: none):
// K_II dz = y_I - C dx through L^T, then zst += dz.
static int interior_correction(vb_ctx *ctx, const double *dx) {
  hipStream_t st = ctx->stream;
  const int nb = dir_nb(ctx, 0), nb2 = dir_nb(ctx, ctx->nd ? 1 : 0);
  if (ctx->max_e > 0) {
    CHK(back_init(ctx->d_subdev, ctx->z_ir, ctx->y_ir, ctx->d_yoff2, ctx->nS, ctx->max_e, st));
    if (dx) {
      if (dx != ctx->dx) return ctx->fail(VB_ERR_STATE, "interior correction: unexpected vector");
      CHK(gemv_t_cpb(ctx->j_brhs, ctx->nS, ctx->brhs_m, ctx->max_e, 8, st));
    }
    for (int j0 = ((ctx->max_e - 1) / nb2) * nb2; j0 >= 0; j0 -= nb2)
      CHK(recover_backsolve(ctx->d_subdev, ctx->invL, ctx->d_invoff, ctx->y_ir, ctx->z_ir,
                            ctx->d_yoff2, ctx->nS, j0, nb2, ctx->fp32, st));
  }
  if (ctx->nd) {
    // the fronts see the interface correction and the separator corrections
    // of the second level through G2d
    const int nS = ctx->nS, nF = (int)ctx->fronts.size();
    if (dx)
      CHK(hipMemcpyAsync(ctx->G2d, dx, (ctx->nG + nS) * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      CHK(hipMemsetAsync(ctx->G2d, 0, (ctx->nG + nS) * sizeof(double), st));
    CHK(scatter_copy((int)ctx->n_sep_tot, ctx->z_ir, ctx->sep_src, ctx->sep_dst, ctx->G2d, 1.0, st));
    if (ctx->max_ef > 0) {
      CHK(back_init(ctx->d_frdev, ctx->z_ir, ctx->y_ir, ctx->d_yoff2f, nF, ctx->max_ef, st));
      CHK(gemv_t_cpb(ctx->j_brhsf, nF, ctx->brhs_mf, ctx->max_ef, 8, st));
      for (int j0 = ((ctx->max_ef - 1) / nb) * nb; j0 >= 0; j0 -= nb)
        CHK(recover_backsolve(ctx->d_frdev, ctx->invLf, ctx->d_invofff, ctx->y_ir, ctx->z_ir,
                              ctx->d_yoff2f, nF, j0, nb, ctx->fp32, st));
    }
  }
  CHK(axpy(ctx->n_ir, 1.0, ctx->z_ir, ctx->zst, st));
  return VB_OK;
}

// Mixed precision (FP32 local factors and Schur operators, FP64 residuals):
// iterative refinement of the whole saddle system around the BDDC/PCG
// solve.  Each outer step condenses the FP64 residual of the local systems,
// solves the interface correction with PCG on the FP32 operators to a loose
// relative tolerance, recovers the interior correction with the FP32
// factor and updates (x, interior state).  A problem stops when its
// condensed residual has dropped by opt.tol relative to its first one.
static int mixed_solve(vb_ctx *ctx, double *x_dev, vb_solve_info *info) {
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->nG + ctx->nS;
  const int nE = (int)ctx->ents.size();
  const int P = (int)ctx->probs.size(), G = ctx->seg_G;
  const int max_outer = 30;
  // default inner tolerance: on small operators (below 1e9 bytes, where the
  // iterations run as one persistent launch) a refinement step's fixed cost
  // (condensation, interior correction, host synchronisations) outweighs a
  // few inner iterations, so fewer and tighter steps (1e-4); on large ones
  // looser steps take fewer iterations in all (1e-3)
  const double inner_floor =
      ctx->opt.inner_tol > 0.0 ? ctx->opt.inner_tol : (ctx->schur_bytes < 1e9 ? 1e-4 : 1e-3);
  ctx->ref_rel.assign(ctx->probs.size(), {});
  ctx->ref_inner.assign(ctx->probs.size(), {});
  CHK(hipEventRecord(ctx->ev0, st));
  CHK(hipMemsetAsync(ctx->zst, 0, ctx->n_ir * sizeof(double), st));
  ctx->cond_fresh = false;
  std::vector<double> r_first(P, 0.0), rel(P, 0.0), t0(P, 0.0), tdone(P, 0.0);
  std::vector<int> steps(P, 0), inner(P, 0), done(P, 0);
  std::vector<vb_solve_info> pi(P);
  int outer = 0, status = VB_OK, inner_max = 0;
  std::vector<double> hs((size_t)P * SC_STRIDE), one(P, 1.0);
  // a clock reference for the latencies: the scalars' T0 of an empty init
  CHK(hipMemcpyAsync(ctx->d_tol, one.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
  CHK(sinit(P, ctx->d_tol, 0, ctx->sc, st));
  CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  for (int pp = 0; pp < P; ++pp) t0[pp] = hs[(size_t)pp * SC_STRIDE + SC_T0];
  while (true) {
    int rc = condense_residual(ctx, x_dev);
    if (rc) return rc;
    CHK(owner_sum((int)ctx->nG, ctx->ir_ptr, ctx->ir_idx, ctx->y_ir, nullptr, nullptr, ctx->dgv,
                  st));
    CHK(scatter_copy(ctx->nS, ctx->r0, nullptr, nullptr, ctx->dgv + ctx->nG, 1.0, st));
    CHK(sdot(ctx->d_segs, P, G, ctx->dgv, ctx->dgv, ctx->part, ctx->sc, 5, nullptr, nullptr, 0, st));
    CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    bool all = true, nonfinite = false;
    std::vector<double> tin(P);
    for (int pp = 0; pp < P; ++pp) {
      const double rn = std::sqrt(hs[(size_t)pp * SC_STRIDE + SC_TMP]);
      if (!std::isfinite(rn) || (outer == 0 && !std::isfinite(r_first[pp]))) nonfinite = true;
      if (outer == 0) r_first[pp] = rn;
      rel[pp] = r_first[pp] > 0 ? rn / r_first[pp] : 0.0;
      if (!done[pp]) ctx->ref_rel[pp].push_back(rel[pp]);
      if (!done[pp] && !(rel[pp] > ctx->opt.tol)) {
        done[pp] = 1;
        if (outer == 0) tdone[pp] = t0[pp];  // converged before any step
      }
      if (!done[pp]) all = false;
      tin[pp] = done[pp] ? 1e300 : std::max(inner_floor, 0.5 * ctx->opt.tol / std::max(rel[pp], 1e-300));
    }
    if (nonfinite) {  // NaN/Inf in the data: a breakdown, not convergence
      status = VB_ERR_BREAKDOWN;
      for (int pp = 0; pp < P; ++pp) done[pp] = 0;
      break;
    }
    if (all) {
      ctx->cond_fresh = true;
      break;
    }
    if (outer >= max_outer || inner_max >= ctx->opt.maxit) {
      status = VB_ERR_NOT_CONVERGED;
      break;
    }
    // interface corrections on the FP32 operators
    CHK(transform_vec(ctx->d_entdev, nE, ctx->dgv, +1, st));
    PcgResult pr;
    rc = pcg_core(ctx, ctx->dgv, true, tin, ctx->opt.maxit - inner_max, &pr);
    if (rc) return rc;
    int mx = 0;
    for (int pp = 0; pp < P; ++pp) {
      const double *q = pr.sc.data() + (size_t)pp * SC_STRIDE;
      const int it = (int)q[SC_IT];
      if (!done[pp]) {
        inner[pp] += it;
        steps[pp] += 1;
        ctx->ref_inner[pp].push_back(it);
      }
      mx = std::max(mx, it);
      if (outer == 0) {  // Lanczos estimates of the first inner solve
        rc = lanczos_problem(ctx, pp, it, &pi[pp].lambda_min, &pi[pp].lambda_max);
        if (rc) return rc;
      }
      if (q[SC_FLAG] == 1.0) status = VB_ERR_BREAKDOWN;
    }
    inner_max += mx;
    if (status == VB_ERR_BREAKDOWN) break;
    CHK(hipMemcpyAsync(ctx->dx, ctx->x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    CHK(transform_vec(ctx->d_entdev, nE, ctx->dx, -1, st));
    rc = interior_correction(ctx, ctx->dx);
    if (rc) return rc;
    CHK(axpy(n, 1.0, ctx->dx, x_dev, st));
    ++outer;
    // device clock after this step: the latency of problems finishing here
    CHK(sinit(P, ctx->d_tol, 0, ctx->sc, st));
    CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (int pp = 0; pp < P; ++pp)
      if (!done[pp]) tdone[pp] = hs[(size_t)pp * SC_STRIDE + SC_T0];
  }
  CHK(hipEventRecord(ctx->ev1, st));
  CHK(hipEventSynchronize(ctx->ev1));
  float ms = 0.f;
  CHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  ctx->last_outer = outer;
  ctx->last_inner = inner_max;
  for (int pp = 0; pp < P; ++pp) {
    vb_solve_info &q = pi[pp];
    q.iterations = inner[pp];
    q.refinement_steps = steps[pp];
    q.rel_residual = rel[pp];
    q.true_rel_residual = rel[pp];
    q.n_coarse = ctx->probs[pp].nprim + ctx->probs[pp].ns;
    q.setup_ms = ctx->setup_ms;
    q.solve_ms = ms;
    q.status = done[pp] ? VB_OK : status;
    q.latency_ms = (ctx->clock_khz > 0 && tdone[pp] > t0[pp]) ? (tdone[pp] - t0[pp]) / ctx->clock_khz : 0.0;
  }
  ctx->pinfo = pi;
  if (status != VB_ERR_BREAKDOWN) {  // (x, zst) is a consistent iterate
    CHK(hipMemcpyAsync(ctx->x_last, x_dev, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    ctx->zst_valid = true;
  }
  if (info) {
    combine_info(pi, info);
    info->n_coarse = ctx->nCS;
    info->status = status;
  }
  if (status == VB_ERR_BREAKDOWN) return ctx->fail(status, "PCG breakdown: p^T S p <= 0 or NaN");
  if (status == VB_ERR_NOT_CONVERGED)
    return ctx->fail(status, "refinement did not reach the tolerance");
  return VB_OK;
}

extern "C" {

int vb_pcg_solve(vb_ctx *ctx, double *x_dev, vb_solve_info *info) {
  if (!ctx || !x_dev) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_pcg_solve: call vb_setup first");
  if (ctx->fp32) return mixed_solve(ctx, x_dev, info);
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->nG + ctx->nS;
  const int nE = (int)ctx->ents.size();
  const int P = (int)ctx->probs.size(), G = ctx->seg_G;
  CHK(hipEventRecord(ctx->ev0, st));
  // x~ = T^T x0 ; PCG on S~ x~ = g~
  CHK(hipMemcpyAsync(ctx->x, x_dev, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  CHK(transform_vec(ctx->d_entdev, nE, ctx->x, +1, st));
  PcgResult pr;
  std::vector<double> tol(P, ctx->opt.tol);
  int rc = pcg_core(ctx, ctx->g, false, tol, ctx->opt.maxit, &pr);
  if (rc) return rc;
  // true residual per problem (into SC_TMP)
  CHK(hipMemcpyAsync(ctx->p, ctx->x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  rc = apply_S_internal(ctx);
  if (rc) return rc;
  CHK(vsub(n, ctx->g, ctx->q, ctx->tmp, st));
  CHK(sdot(ctx->d_segs, P, G, ctx->tmp, ctx->tmp, ctx->part, ctx->sc, 5, nullptr, nullptr, 0, st));
  CHK(hipMemcpyAsync(x_dev, ctx->x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  CHK(transform_vec(ctx->d_entdev, nE, x_dev, -1, st));
  CHK(hipEventRecord(ctx->ev1, st));
  std::vector<double> hs((size_t)P * SC_STRIDE);
  CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  float ms = 0.f;
  CHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  std::vector<vb_solve_info> pi(P);
  for (int pp = 0; pp < P; ++pp) {
    const double *q = hs.data() + (size_t)pp * SC_STRIDE;
    vb_solve_info &o = pi[pp];
    o.iterations = (int)q[SC_IT];
    o.refinement_steps = 0;
    o.rel_residual = q[SC_GG] > 0 ? std::sqrt(q[SC_RR] / q[SC_GG]) : 0.0;
    o.true_rel_residual = q[SC_GG] > 0 ? std::sqrt(q[SC_TMP] / q[SC_GG]) : 0.0;
    o.n_coarse = ctx->probs[pp].nprim + ctx->probs[pp].ns;
    o.setup_ms = ctx->setup_ms;
    o.solve_ms = ms;
    o.status = q[SC_FLAG] == 1.0 ? VB_ERR_BREAKDOWN
               : (q[SC_FLAG] == 2.0 || q[SC_DONE] == 0.0) ? VB_ERR_NOT_CONVERGED : VB_OK;
    o.latency_ms = (ctx->clock_khz > 0 && q[SC_TDONE] > q[SC_T0])
                       ? (q[SC_TDONE] - q[SC_T0]) / ctx->clock_khz : 0.0;
    rc = lanczos_problem(ctx, pp, o.iterations, &o.lambda_min, &o.lambda_max);
    if (rc) return rc;
  }
  ctx->pinfo = pi;
  if (info) {
    combine_info(pi, info);
    if (P > 1) info->n_coarse = ctx->nCS;
    info->status = pr.status;
  }
  if (pr.status == VB_ERR_BREAKDOWN) return ctx->fail(pr.status, "PCG breakdown: p^T S p <= 0 or NaN");
  if (pr.status == VB_ERR_NOT_CONVERGED) return ctx->fail(pr.status, "PCG reached maxit");
  return VB_OK;
}

int vb_recover_all(vb_ctx *ctx, const double *x_dev, double *out_dev) {
  if (!ctx || !x_dev) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_recover_all: call vb_setup first");
  hipStream_t st = ctx->stream;
  if (ctx->fp32) {
    // FP32 factor: refine the interior equations in FP64 with the interface
    // data fixed at x, from the interior state of the last solve when x is
    // that solve's result (one pass, on the condensed residual the solve's
    // final check left), else from zero (recover_steps passes)
    int passes = ctx->recover_steps;
    bool from_solve = false;
    const bool fresh = ctx->cond_fresh;
    ctx->cond_fresh = false;
    if (ctx->zst_valid) {
      const int64_t n = ctx->nG + ctx->nS;
      const int P = (int)ctx->probs.size();
      CHK(vsub(n, x_dev, ctx->x_last, ctx->tmp, st));
      CHK(sdot(ctx->d_segs, P, ctx->seg_G, ctx->tmp, ctx->tmp, ctx->part, ctx->sc, 5, nullptr,
               nullptr, 0, st));
      std::vector<double> hs((size_t)P * SC_STRIDE);
      CHK(hipMemcpyAsync(hs.data(), ctx->sc, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      CHK(hipStreamSynchronize(st));
      from_solve = true;
      for (int pp = 0; pp < P; ++pp) from_solve = from_solve && hs[(size_t)pp * SC_STRIDE + SC_TMP] == 0.0;
    }
    if (from_solve) {
      passes = std::min(passes, fresh ? 1 : 2);
    } else {
      CHK(hipMemsetAsync(ctx->zst, 0, ctx->n_ir * sizeof(double), st));
      ctx->zst_valid = false;
    }
    for (int k = 0; k < passes; ++k) {
      int rc = (k == 0 && from_solve && fresh) ? VB_OK : condense_residual(ctx, x_dev);
      if (rc) return rc;
      rc = interior_correction(ctx, nullptr);
      if (rc) return rc;
    }
    if (ctx->nd)
      CHK(hipMemcpyAsync(ctx->G2, x_dev, (ctx->nG + ctx->nS) * sizeof(double), hipMemcpyDeviceToDevice, st));
    {
      int rc = state_to_local(ctx, x_dev);
      if (rc) return rc;
    }
    CHK(hipMemcpyAsync(ctx->rec_out, ctx->u_loc, ctx->rec_off[ctx->nS] * sizeof(double),
                       hipMemcpyDeviceToDevice, st));
    if (out_dev)
      CHK(hipMemcpyAsync(out_dev, ctx->u_loc, ctx->rec_off[ctx->nS] * sizeof(double),
                         hipMemcpyDeviceToDevice, st));
    return VB_OK;
  }
  const int nb = dir_nb(ctx, 0);  // the panel widths the factorisations used
  if (ctx->nd) {
    // second level: separator velocities and sub-box constants; then every
    // front from its separator and interface values and its constant
    const int nS = ctx->nS, nF = (int)ctx->fronts.size(), nb2 = dir_nb(ctx, 1);
    if (ctx->max_e > 0) {
      CHK(recover_rhs(ctx->d_subdev, x_dev, ctx->yrec, ctx->d_yoff, nS, ctx->max_e, ctx->fp32, st));
      for (int j0 = ((ctx->max_e - 1) / nb2) * nb2; j0 >= 0; j0 -= nb2)
        CHK(recover_backsolve(ctx->d_subdev, ctx->invL, ctx->d_invoff, ctx->yrec, ctx->zrec, ctx->d_yoff,
                              nS, j0, nb2, ctx->fp32, st));
    }
    CHK(hipMemcpyAsync(ctx->G2, x_dev, (ctx->nG + nS) * sizeof(double), hipMemcpyDeviceToDevice, st));
    CHK(recover_out(ctx->j_rec, nS, x_dev, ctx->nG, st));
    if (ctx->max_ef > 0) {
      CHK(recover_rhs(ctx->d_frdev, ctx->G2, ctx->yrec, ctx->d_yofff, nF, ctx->max_ef, ctx->fp32, st));
      for (int j0 = ((ctx->max_ef - 1) / nb) * nb; j0 >= 0; j0 -= nb)
        CHK(recover_backsolve(ctx->d_frdev, ctx->invLf, ctx->d_invofff, ctx->yrec, ctx->zrec,
                              ctx->d_yofff, nF, j0, nb, ctx->fp32, st));
    }
    CHK(recover_out(ctx->j_recf, nF, ctx->G2, ctx->g2_c0, st));
    if (out_dev)
      CHK(hipMemcpyAsync(out_dev, ctx->rec_out, ctx->rec_off[nS] * sizeof(double),
                         hipMemcpyDeviceToDevice, st));
    return VB_OK;
  }
  // with several waves: first the wave whose factors W still holds, then the
  // others, each factored again
  const int nw = (int)ctx->waves.size(), first = std::max(ctx->w_wave, 0);
  for (int k = 0; k < nw; ++k) {
    const int wi = (first + k) % nw;
    const auto &wv = ctx->waves[wi];
    const int s0 = wv.first, n = wv.second - wv.first;
    if (ctx->stream_w && wi != ctx->w_wave) {
      ctx->w_wave = -1;
      int rc = factor_wave(ctx, s0, wv.second, false);
      if (rc) return rc;
      ctx->w_wave = wi;
    }
    int mxe = 0;
    for (int s = s0; s < wv.second; ++s) mxe = std::max(mxe, ctx->subs[s].e);
    CHK(recover_rhs(ctx->d_subdev + s0, x_dev, ctx->yrec, ctx->d_yoff + s0, n, mxe, ctx->fp32, st));
    for (int j0 = ((mxe - 1) / nb) * nb; j0 >= 0; j0 -= nb)
      CHK(recover_backsolve(ctx->d_subdev + s0, ctx->invL, ctx->d_invoff + s0, ctx->yrec, ctx->zrec,
                            ctx->d_yoff + s0, n, j0, nb, ctx->fp32, st));
  }
  CHK(recover_out(ctx->j_rec, ctx->nS, x_dev, ctx->nG, st));
  if (out_dev)
    CHK(hipMemcpyAsync(out_dev, ctx->rec_out, ctx->rec_off[ctx->nS] * sizeof(double),
                       hipMemcpyDeviceToDevice, st));
  return VB_OK;
}

int64_t vb_local_size(const vb_ctx *ctx, int sub) {
  if (!ctx || ctx->state < 1 || sub < -1 || sub >= ctx->nS) return VB_ERR_ARG;
  if (sub >= 0) return ctx->subs[sub].n;
  int64_t tot = 0;
  for (const auto &S : ctx->subs) tot += S.n;
  return tot;
}

int vb_get_local_solution(vb_ctx *ctx, const double *x_dev, int sub, double *u_host) {
  if (!ctx || !x_dev || !u_host || sub < 0 || sub >= ctx->nS) return VB_ERR_ARG;
  int rc = vb_recover_all(ctx, x_dev, nullptr);
  if (rc) return rc;
  CHK(hipMemcpyAsync(u_host, ctx->rec_out + ctx->rec_off[sub], ctx->subs[sub].n * sizeof(double),
                     hipMemcpyDeviceToHost, ctx->stream));
  CHK(hipStreamSynchronize(ctx->stream));
  return VB_OK;
}

int vb_batched_ldl(vb_ctx *ctx, int batch, double *const *A, const int32_t *n, const int32_t *ld,
                   const int32_t *e, const int32_t *p, int32_t *info, int max_n, int max_e) {
  if (!ctx || batch < 0 || (batch > 0 && (!A || !n || !ld || !e || !p || !info)))
    return VB_ERR_ARG;
  if (batch == 0) return VB_OK;
  std::vector<double *> hA(batch);
  std::vector<int32_t> hn(batch), hld(batch), he(batch), hp(batch);
  hipStream_t st = ctx->stream;
  CHK(hipMemcpyAsync(hA.data(), A, batch * sizeof(double *), hipMemcpyDeviceToHost, st));
  CHK(hipMemcpyAsync(hn.data(), n, batch * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CHK(hipMemcpyAsync(hld.data(), ld, batch * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CHK(hipMemcpyAsync(he.data(), e, batch * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CHK(hipMemcpyAsync(hp.data(), p, batch * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  for (int b = 0; b < batch; ++b)
    if (hn[b] < 0 || hn[b] > max_n || he[b] < 0 || he[b] > hn[b] || he[b] > max_e || hld[b] < hn[b])
      return ctx->fail(VB_ERR_ARG, "vb_batched_ldl: inconsistent sizes for matrix " + std::to_string(b));
  const int64_t per = (int64_t)((max_e + NB - 1) / NB) * NB * NB;
  double *scratch = nullptr;
  CHK(hipMalloc(&scratch, std::max<int64_t>(per * batch, 1) * sizeof(double)));
  std::vector<LdlJob<double>> jobs(batch);
  // 16-byte aligned columns everywhere: the trailing updates load their
  // panel strips straight into LDS (the kernels the library's own
  // factorisations use); otherwise the staged kernels
  bool aligned16 = true;
  for (int b = 0; b < batch; ++b) {
    jobs[b] = {hA[b], hld[b], hn[b], he[b], hp[b], 0, scratch + per * b, info + b};
    aligned16 = aligned16 && hld[b] >= 2 && (hld[b] * sizeof(double)) % 16 == 0 &&
                reinterpret_cast<uintptr_t>(hA[b]) % 16 == 0;
  }
  LdlJob<double> *dj = nullptr;
  hipError_t err = hipMalloc(&dj, batch * sizeof(LdlJob<double>));
  if (err == hipSuccess) err = hipMemcpy(dj, jobs.data(), batch * sizeof(LdlJob<double>), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemsetAsync(info, 0, batch * sizeof(int32_t), st);
  if (err == hipSuccess)
    err = ldl_batched<double>(dj, batch, max_n, max_e, ctx->opt.panel, st, nullptr, &hn, &he, false,
                              aligned16);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  (void)hipFree(dj);
  (void)hipFree(scratch);
  if (err != hipSuccess) return ctx->fail(VB_ERR_DEVICE, std::string("vb_batched_ldl: ") + hipGetErrorString(err));
  return VB_OK;
}

}  // extern "C"

extern "C" {

int vb_tuned_tile(const vb_ctx *ctx, int which) {
  if (!ctx || which < 0 || which > 11) return VB_ERR_ARG;
  if (which >= 6 && which <= 8) return ctx->fac_nb[which - 6];
  if (which >= 9) return ctx->fac_sb[which - 9];
  if (which == 4) return ctx->ssym_on ? 1 : 0;
  if (which == 5) return ctx->nsym_on ? 1 : 0;
  return ctx->cpb[which];
}

int vb_num_problems(const vb_ctx *ctx) { return ctx ? (int)ctx->probs.size() : VB_ERR_ARG; }

int vb_problem_layout(const vb_ctx *ctx, int problem, vb_problem *out) {
  if (!ctx || !out || problem < 0 || problem >= (int)ctx->probs.size()) return VB_ERR_ARG;
  const auto &P = ctx->probs[problem];
  out->iface_offset = P.g0;
  out->n_iface = P.ng;
  out->p0_offset = ctx->nG + P.s0;
  out->sub_offset = P.s0;
  out->n_sub = P.ns;
  return VB_OK;
}

int vb_problem_solve_info(const vb_ctx *ctx, int problem, vb_solve_info *out) {
  if (!ctx || !out || problem < 0 || problem >= (int)ctx->probs.size()) return VB_ERR_ARG;
  if (problem >= (int)ctx->pinfo.size()) return VB_ERR_STATE;
  *out = ctx->pinfo[problem];
  return VB_OK;
}

int vb_adaptive_info(vb_ctx *ctx, int max_faces, vb_face_info *faces, int max_eigs, double *eigs) {
  if (!ctx || max_faces < 0 || max_eigs < 0) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_adaptive_info: call vb_setup first");
  const int nf = (int)ctx->face_info.size();
  if (faces)
    for (int i = 0; i < std::min(nf, max_faces); ++i) faces[i] = ctx->face_info[i];
  if (eigs)
    for (int i = 0; i < std::min((int)ctx->face_eigs.size(), max_eigs); ++i) eigs[i] = ctx->face_eigs[i];
  return nf;
}

int vb_setup_phases(const vb_ctx *ctx, int max, double *ms) {
  if (!ctx || max < 0 || (max > 0 && !ms)) return VB_ERR_ARG;
  for (int i = 0; i < std::min(max, vb_ctx::kPhases); ++i) ms[i] = ctx->phase_ms[i];
  return vb_ctx::kPhases;
}

int vb_fp64_retries(const vb_ctx *ctx, int max, int32_t *subs) {
  if (!ctx || max < 0 || (max > 0 && !subs)) return VB_ERR_ARG;
  const int n = (int)ctx->fp64_retried.size();
  for (int i = 0; i < std::min(n, max); ++i) subs[i] = ctx->fp64_retried[i];
  return n;
}

int vb_refinement_history(const vb_ctx *ctx, int problem, int max, double *rel, int32_t *inner) {
  if (!ctx || max < 0 || (max > 0 && (!rel || !inner))) return VB_ERR_ARG;
  if (problem < 0 || problem >= (int)std::max<size_t>(ctx->probs.size(), 1)) return VB_ERR_ARG;
  if (problem >= (int)ctx->ref_inner.size()) return 0;
  const std::vector<double> &r = ctx->ref_rel[problem];
  const std::vector<int> &it = ctx->ref_inner[problem];
  for (int k = 0; k < std::min((int)r.size(), max); ++k) rel[k] = r[k];
  for (int k = 0; k < std::min((int)it.size(), max); ++k) inner[k] = it[k];
  return (int)it.size();
}

int vb_pcg_launch_used(const vb_ctx *ctx) { return ctx ? ctx->last_launch : VB_ERR_ARG; }

int vb_set_profile(vb_ctx *ctx, int on) {
  if (!ctx) return VB_ERR_ARG;
  ctx->opt.profile = on ? 1 : 0;
  return VB_OK;
}

int vb_kernel_stats(vb_ctx *ctx, int which, int reset, vb_kernel_stat *out) {
  if (!ctx || !out || which < 0 || which > 1) return VB_ERR_ARG;
  KTimer &t = which == 0 ? ctx->t_ldl : ctx->t_gemv;
  CHK(hipStreamSynchronize(ctx->stream));
  double ms = 0.0, work = 0.0;
  int n = 0;
  hipError_t e = t.collect(&n, &ms, &work);
  if (e != hipSuccess) return ctx->fail(VB_ERR_DEVICE, "vb_kernel_stats: event query failed");
  out->launches = n;
  out->total_ms = ms;
  out->work = work;
  if (reset) t.reset();
  return VB_OK;
}

}  // extern "C"

// accessors for the allocation-free entry point (noalloc.hip)
namespace vb {
hipStream_t ctx_stream(const vb_ctx *ctx) { return ctx->stream; }
int ctx_panel(const vb_ctx *ctx) { return ctx->opt.panel; }
int ctx_fail(vb_ctx *ctx, int code, const char *msg) { return ctx->fail(code, msg); }
}  // namespace vb

// ------------------------------------------------------------ predictor ABI
#define MCHK(x)                                                                   \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess)                                                         \
      return m->fail(e_ == hipErrorOutOfMemory ? VB_ERR_OOM : VB_ERR_DEVICE,      \
                     std::string(#x) + ": " + hipGetErrorString(e_));             \
  } while (0)

static_assert(VB_MLP_NPARAMS == MLP_NPARAMS, "network size");
static_assert(VB_MLP_FEATURES == MLP_F, "feature count");

extern "C" {

int vb_mlp_create(vb_mlp **out, const float *init, void *stream) {
  if (!out || !init) return VB_ERR_ARG;
  vb_mlp *m = new vb_mlp();
  *out = m;
  // NULL = the default stream, as for vb_options.stream: every launch of the
  // model is then ordered after the caller's work on that stream
  m->stream = (hipStream_t)stream;
  const size_t P = MLP_NPARAMS * sizeof(float);
  MCHK(hipMalloc(&m->p, P));
  MCHK(hipMalloc(&m->m, P));
  MCHK(hipMalloc(&m->v, P));
  MCHK(hipMalloc(&m->g, P));
  MCHK(hipMalloc(&m->mu, MLP_F * sizeof(float)));
  MCHK(hipMalloc(&m->sd, MLP_F * sizeof(float)));
  MCHK(hipMalloc(&m->t, sizeof(int)));
  MCHK(hipMalloc(&m->loss, sizeof(double)));
  MCHK(hipMemcpy(m->p, init, P, hipMemcpyHostToDevice));
  std::vector<float> z(MLP_F, 0.0f), o(MLP_F, 1.0f);
  MCHK(hipMemcpy(m->mu, z.data(), MLP_F * sizeof(float), hipMemcpyHostToDevice));
  MCHK(hipMemcpy(m->sd, o.data(), MLP_F * sizeof(float), hipMemcpyHostToDevice));
  return VB_OK;
}

void vb_mlp_destroy(vb_mlp *m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  if (m->cap_stream) (void)hipStreamSynchronize(m->cap_stream);
  for (void *q : {(void *)m->p, (void *)m->m, (void *)m->v, (void *)m->g, (void *)m->mu,
                  (void *)m->sd, (void *)m->t, (void *)m->loss, (void *)m->X, (void *)m->y})
    if (q) (void)hipFree(q);
  if (m->own_stream) (void)hipStreamDestroy(m->cap_stream);
  delete m;
}

const char *vb_mlp_last_error(const vb_mlp *m) { return m ? m->err.c_str() : "null model"; }

int64_t vb_mlp_num_samples(const vb_mlp *m) { return m ? m->n : -1; }

int64_t vb_face_samples(vb_ctx *ctx, int64_t max_n, float *X_host, float *y_host) {
  if (!ctx || max_n < 0) return VB_ERR_ARG;
  if (ctx->state != 2) return ctx->fail(VB_ERR_STATE, "vb_face_samples: call vb_setup first");
  const int64_t n = std::min(ctx->n_coord, max_n);
  CHK(hipStreamSynchronize(ctx->stream));
  if (n > 0 && X_host)
    CHK(hipMemcpy(X_host, ctx->d_feat, n * MLP_F * sizeof(float), hipMemcpyDeviceToHost));
  if (n > 0 && y_host)
    CHK(hipMemcpy(y_host, ctx->d_lab, n * sizeof(float), hipMemcpyDeviceToHost));
  return ctx->n_coord;
}

static int mlp_append(vb_mlp *m, const float *Xk, const float *yk, int64_t add) {
  if (m->n + add > m->cap) {
    const int64_t cap = std::max<int64_t>(2 * m->cap, m->n + add);
    float *X2 = nullptr, *y2 = nullptr;
    MCHK(hipMalloc(&X2, cap * MLP_F * sizeof(float)));
    MCHK(hipMalloc(&y2, cap * sizeof(float)));
    if (m->n) {
      MCHK(hipMemcpy(X2, m->X, m->n * MLP_F * sizeof(float), hipMemcpyDeviceToDevice));
      MCHK(hipMemcpy(y2, m->y, m->n * sizeof(float), hipMemcpyDeviceToDevice));
    }
    if (m->X) (void)hipFree(m->X);
    if (m->y) (void)hipFree(m->y);
    m->X = X2;
    m->y = y2;
    m->cap = cap;
  }
  if (add) {
    MCHK(hipMemcpy(m->X + m->n * MLP_F, Xk, add * MLP_F * sizeof(float), hipMemcpyHostToDevice));
    MCHK(hipMemcpy(m->y + m->n, yk, add * sizeof(float), hipMemcpyHostToDevice));
  }
  m->n += add;
  return VB_OK;
}

int vb_mlp_add_data(vb_mlp *m, const float *X_host, const float *y_host, int64_t n) {
  if (!m || n < 0 || (n > 0 && (!X_host || !y_host))) return VB_ERR_ARG;
  return mlp_append(m, X_host, y_host, n);
}

int vb_mlp_add_samples(vb_mlp *m, vb_ctx *ctx) {
  if (!m || !ctx) return VB_ERR_ARG;
  if (ctx->state != 2) return m->fail(VB_ERR_STATE, "vb_mlp_add_samples: context not set up");
  const int64_t nc = ctx->n_coord;
  if (nc == 0) return 0;
  MCHK(hipStreamSynchronize(ctx->stream));
  std::vector<float> X((size_t)nc * MLP_F), y(nc);
  MCHK(hipMemcpy(X.data(), ctx->d_feat, X.size() * sizeof(float), hipMemcpyDeviceToHost));
  MCHK(hipMemcpy(y.data(), ctx->d_lab, y.size() * sizeof(float), hipMemcpyDeviceToHost));
  // keep the coordinates with a label (faces solved by the exact eigensolve)
  std::vector<float> Xk, yk;
  for (int64_t i = 0; i < nc; ++i)
    if (y[i] == y[i]) {
      Xk.insert(Xk.end(), X.begin() + i * MLP_F, X.begin() + (i + 1) * MLP_F);
      yk.push_back(y[i]);
    }
  const int64_t add = (int64_t)yk.size();
  int rc = mlp_append(m, Xk.data(), yk.data(), add);
  if (rc) return rc;
  return (int)add;
}

int vb_mlp_train(vb_mlp *m, int epochs, float lr, double *loss_history) {
  if (!m || epochs < 0 || !(lr > 0.0f)) return VB_ERR_ARG;
  if (m->n <= 0) return m->fail(VB_ERR_STATE, "vb_mlp_train: no samples");
  // the epoch is captured as a HIP graph, which the default stream cannot
  // hold: with it, training runs on a stream of its own after the default
  // stream has drained
  hipStream_t st = m->stream;
  if (!st) {
    MCHK(hipStreamSynchronize(nullptr));
    if (!m->own_stream) {
      MCHK(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
      m->own_stream = true;
    }
    st = m->cap_stream;
  }
  const int nblk = (int)((m->n + 63) / 64);
  float *partial = nullptr;
  double *lpart = nullptr, *hist = nullptr;
  MCHK(hipMalloc(&partial, (size_t)nblk * MLP_NPARAMS * sizeof(float)));
  MCHK(hipMalloc(&lpart, (size_t)nblk * sizeof(double)));
  MCHK(hipMalloc(&hist, (size_t)std::max(epochs, 1) * sizeof(double)));
  int rc = VB_OK;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto run = [&]() -> int {
    MCHK(mlp_standardize(m->X, m->n, m->mu, m->sd, st));
    // fresh optimiser state (filled by a kernel launch, not a memset, so the
    // captured epoch holds kernels only)
    std::vector<float> z(MLP_NPARAMS, 0.0f);
    MCHK(hipMemcpyAsync(m->m, z.data(), MLP_NPARAMS * sizeof(float), hipMemcpyHostToDevice, st));
    MCHK(hipMemcpyAsync(m->v, z.data(), MLP_NPARAMS * sizeof(float), hipMemcpyHostToDevice, st));
    int zero = 0;
    MCHK(hipMemcpyAsync(m->t, &zero, sizeof(int), hipMemcpyHostToDevice, st));
    MCHK(hipStreamSynchronize(st));
    if (epochs == 0) return VB_OK;
    // one epoch = gradient (block partials + fixed-order reduction) + Adam
    MCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = mlp_grad(m->p, m->mu, m->sd, m->X, m->y, m->n, partial, lpart, m->g, m->loss, st);
    hipError_t e2 = mlp_adam(m->p, m->g, m->m, m->v, m->t, lr, m->loss, hist, st);
    hipError_t e3 = hipStreamEndCapture(st, &graph);
    MCHK(e1);
    MCHK(e2);
    MCHK(e3);
    MCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    for (int ep = 0; ep < epochs; ++ep) MCHK(hipGraphLaunch(exec, st));
    MCHK(hipStreamSynchronize(st));
    if (loss_history)
      MCHK(hipMemcpy(loss_history, hist, epochs * sizeof(double), hipMemcpyDeviceToHost));
    m->trained = true;
    return VB_OK;
  };
  rc = run();
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipFree(partial);
  (void)hipFree(lpart);
  (void)hipFree(hist);
  return rc;
}

int vb_mlp_forward(vb_mlp *m, const float *X_dev, int64_t n, float *s_dev) {
  if (!m || n < 0 || (n > 0 && (!X_dev || !s_dev))) return VB_ERR_ARG;
  MCHK(mlp_forward(m->p, m->mu, m->sd, X_dev, n, s_dev, m->stream));
  MCHK(hipStreamSynchronize(m->stream));
  return VB_OK;
}

int vb_mlp_loss_grad(vb_mlp *m, const float *X_dev, const float *y_dev, int64_t n,
                     float *grad_dev, double *loss) {
  if (!m || n <= 0 || !X_dev || !y_dev || !grad_dev) return VB_ERR_ARG;
  const int nblk = (int)((n + 63) / 64);
  float *partial = nullptr;
  double *lpart = nullptr, *dl = nullptr;
  MCHK(hipMalloc(&partial, (size_t)nblk * MLP_NPARAMS * sizeof(float)));
  MCHK(hipMalloc(&lpart, (size_t)nblk * sizeof(double)));
  MCHK(hipMalloc(&dl, sizeof(double)));
  hipError_t e = mlp_grad(m->p, m->mu, m->sd, X_dev, y_dev, n, partial, lpart, grad_dev, dl, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess && loss) e = hipMemcpy(loss, dl, sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(partial);
  (void)hipFree(lpart);
  (void)hipFree(dl);
  MCHK(e);
  return VB_OK;
}

int vb_mlp_get_params(const vb_mlp *mc, float *params, float *mu, float *sd) {
  vb_mlp *m = const_cast<vb_mlp *>(mc);
  if (!m) return VB_ERR_ARG;
  MCHK(hipStreamSynchronize(m->stream));
  if (params) MCHK(hipMemcpy(params, m->p, MLP_NPARAMS * sizeof(float), hipMemcpyDeviceToHost));
  if (mu) MCHK(hipMemcpy(mu, m->mu, MLP_F * sizeof(float), hipMemcpyDeviceToHost));
  if (sd) MCHK(hipMemcpy(sd, m->sd, MLP_F * sizeof(float), hipMemcpyDeviceToHost));
  return VB_OK;
}

int vb_mlp_set_params(vb_mlp *m, const float *params, const float *mu, const float *sd) {
  if (!m) return VB_ERR_ARG;
  MCHK(hipStreamSynchronize(m->stream));
  if (params) MCHK(hipMemcpy(m->p, params, MLP_NPARAMS * sizeof(float), hipMemcpyHostToDevice));
  if (mu) MCHK(hipMemcpy(m->mu, mu, MLP_F * sizeof(float), hipMemcpyHostToDevice));
  if (sd) MCHK(hipMemcpy(m->sd, sd, MLP_F * sizeof(float), hipMemcpyHostToDevice));
  if (params && mu && sd) m->trained = true;
  return VB_OK;
}

int vb_mlp_set_warm_start(vb_mlp *m, int on) {
  if (!m) return VB_ERR_ARG;
  m->warm = on ? 1 : 0;
  return VB_OK;
}

}  // extern "C"
