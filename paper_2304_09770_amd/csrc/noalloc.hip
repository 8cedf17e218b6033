// vb_batched_ldl_noalloc: the batched dense partial signed LDL^T of
// vb_batched_ldl for callers that may not allocate device memory.
//
// Its device working memory (the job table the factorisation kernels read,
// the per-panel inverse diagonal blocks and one flag) lives in a fixed
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel or a copy: it uses
// the device address hipGetSymbolAddress returns for the current device,
// looked up once per device on the first call there.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/vembddc.h"
#include "common.h"
#include "kernels.h"

namespace vb {
hipStream_t ctx_stream(const vb_ctx *ctx);
int ctx_panel(const vb_ctx *ctx);
int ctx_fail(vb_ctx *ctx, int code, const char *msg);
}  // namespace vb

using namespace vb;

namespace {

constexpr int kNB = 64;        // panel width bound of the inverse diagonal blocks
constexpr int kMaxDevices = 64;
constexpr size_t kScratchBytes = (size_t)VB_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};  // scratch's device address on each device

// Layout of the scratch array for one call:
//   [0, 256)                 int flag: every matrix 16-byte aligned
//   [256, 256 + jobs)        LdlJob<double>[batch]
//   [inv_off, + batch * per) inverse diagonal blocks, per doubles a matrix
struct Layout {
  size_t jobs_off, inv_off, total;
};

Layout layout(int batch, int64_t per) {
  Layout L;
  L.jobs_off = 256;
  const size_t jobs = (size_t)batch * sizeof(LdlJob<double>);
  L.inv_off = (L.jobs_off + jobs + 255) / 256 * 256;
  L.total = L.inv_off + (size_t)batch * (size_t)per * sizeof(double);
  return L;
}

// One workgroup: job b from the caller's device arrays.  A matrix whose
// sizes are inconsistent (n < 0, n > max_n, e < 0, e > n, e > max_e,
// ld < n) gets info[b] = -1 and an empty job; every other info[b] is
// cleared.  flag = 1 when every matrix has 16-byte aligned columns (the
// condition of the direct-to-LDS trailing updates).
__global__ __launch_bounds__(256) void k_noalloc_jobs(double *const *A, const int32_t *n,
                                                      const int32_t *ld, const int32_t *e,
                                                      const int32_t *p, int32_t *info, int batch,
                                                      int max_n, int max_e, int64_t per,
                                                      LdlJob<double> *jobs, double *inv,
                                                      int *flag) {
  __shared__ int unaligned;
  if (threadIdx.x == 0) unaligned = 0;
  __syncthreads();
  int mine = 0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    const int nb = n[b], lb = ld[b], eb = e[b];
    double *Ab = A[b];
    const bool ok = nb >= 0 && nb <= max_n && eb >= 0 && eb <= nb && eb <= max_e && lb >= nb;
    LdlJob<double> J;
    J.A = Ab;
    J.ld = lb;
    J.n = ok ? nb : 0;
    J.e = ok ? eb : 0;
    J.p = p[b];
    J.pad = 0;
    J.invL = inv + per * b;
    J.info = info + b;
    J.pmin = 0.0;
    J.zrow = 0;
    J.zpad = 0;
    jobs[b] = J;
    info[b] = ok ? 0 : -1;
    if (ok && !(lb >= 2 && (lb % 2) == 0 && (reinterpret_cast<uintptr_t>(Ab) % 16) == 0)) mine = 1;
  }
  if (mine) atomicOr(&unaligned, 1);
  __syncthreads();
  if (threadIdx.x == 0) *flag = unaligned ? 0 : 1;
}

}  // namespace

extern "C" int vb_batched_ldl_noalloc(vb_ctx *ctx, int batch, double *const *A, const int32_t *n,
                                      const int32_t *ld, const int32_t *e, const int32_t *p,
                                      int32_t *info, int max_n, int max_e) {
  if (!ctx || batch < 0 || max_n < 0 || max_e < 0 ||
      (batch > 0 && (!A || !n || !ld || !e || !p || !info)))
    return VB_ERR_ARG;
  if (batch == 0) return VB_OK;
  const int64_t per = (int64_t)((max_e + kNB - 1) / kNB) * kNB * kNB;
  const Layout L = layout(batch, per);
  if (L.total > kScratchBytes)
    return ctx_fail(ctx, VB_ERR_ARG,
                    "vb_batched_ldl_noalloc: batch * ceil(max_e / 64) * 64 * 64 * 8 bytes of "
                    "inverse diagonal blocks plus the job table exceed VB_NOALLOC_SCRATCH_BYTES");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return ctx_fail(ctx, VB_ERR_DEVICE, "vb_batched_ldl_noalloc: no current device");
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
      void *ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
        return ctx_fail(ctx, VB_ERR_DEVICE, "vb_batched_ldl_noalloc: scratch address lookup failed");
      g_ptr[dev] = ptr;
    }
    base = g_ptr[dev];
  }
  hipStream_t st = ctx_stream(ctx);
  char *b8 = static_cast<char *>(base);
  int *d_flag = reinterpret_cast<int *>(b8);
  LdlJob<double> *jobs = reinterpret_cast<LdlJob<double> *>(b8 + L.jobs_off);
  double *inv = reinterpret_cast<double *>(b8 + L.inv_off);
  hipLaunchKernelGGL(k_noalloc_jobs, dim3(1), dim3(256), 0, st, A, n, ld, e, p, info, batch, max_n,
                     max_e, per, jobs, inv, d_flag);
  hipError_t err = hipGetLastError();
  int aligned = 0;
  if (err == hipSuccess) err = hipMemcpyAsync(&aligned, d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err == hipSuccess)
    err = ldl_batched<double>(jobs, batch, max_n, max_e, ctx_panel(ctx), st, nullptr, nullptr, nullptr,
                              false, aligned != 0);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err != hipSuccess) return ctx_fail(ctx, VB_ERR_DEVICE, hipGetErrorString(err));
  return VB_OK;
}
