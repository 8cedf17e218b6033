// Batched virtual element matrices on the device (Sec. 3, eqs. discreteA,
// discreteF): vb_vem_element_matrices.  Elements go in chunks sized to a
// fixed workspace; per chunk three launches:
//   k_vem_shared    one thread per element (geometry, mass matrices, the
//                   face and element projection systems inverted),
//   k_vem_column    one thread per element and basis function (everything
//                   linear in the degrees of freedom),
//   k_vem_products  one workgroup per element (the N x N products: the
//                   projection's degree-of-freedom matrix, the consistency
//                   term, the stabilisation; B and F).
// The per-element and per-column blocks are interleaved (element-major
// stride), so neighbouring threads read neighbouring addresses.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/vembddc.h"
#include "vem_elem.h"
#include "vem_tables.h"

namespace vb {
hipStream_t ctx_stream(const vb_ctx *ctx);
int ctx_fail(vb_ctx *ctx, int code, const char *msg);
}  // namespace vb

using namespace vb::vem;

namespace {

template <int K>
__global__ __launch_bounds__(64) void k_vem_shared(const double *X8, const double *nu, int with_load,
                                                   Tables T, double *Sb, int64_t e0, int64_t ne) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double x[24];
  for (int q = 0; q < 24; ++q) x[q] = X8[(e0 + e) * 24 + q];
  shared<K>(x, nu ? nu[e0 + e] : 1.0, with_load != 0, T, View{Sb + e, ne});
}

template <int K>
__global__ __launch_bounds__(64) void k_vem_column(Tables T, double *Sb, double *Cb, int64_t ne) {
  typedef Dims<K> D;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne * D::N) return;
  const int64_t e = t / D::N;
  const int i = (int)(t % D::N);
  column<K>(i, T, View{Sb + e, ne}, View{Cb + t, ne * D::N});
}

template <int K>
__global__ __launch_bounds__(256) void k_vem_products(const double *X8, const double *nu, int with_load,
                                                      Tables T, double *Sb, double *Cb, double *Pb,
                                                      int64_t e0, int64_t ne, double *A, double *B,
                                                      double *F) {
  typedef Dims<K> D;
  const int64_t e = blockIdx.x;
  if (e >= ne) return;
  __shared__ double x[24];
  if (threadIdx.x < 24) x[threadIdx.x] = X8[(e0 + e) * 24 + threadIdx.x];
  __syncthreads();
  const View S{Sb + e, ne};
  const ColSet C{Cb, ne * D::N, e * D::N};
  double *P = Pb + e * Products<K>::size;
  double *Ae = A + (e0 + e) * D::N * D::N, *Be = B + (e0 + e) * D::nP * D::N;
  double *Fe = F ? F + (e0 + e) * D::N : nullptr;
  const int t0 = threadIdx.x, ts = blockDim.x;
  prod_dofm<K>(x, T, S, P, t0, ts);
  __syncthreads();
  prod_dpi<K>(S, C, P, Ae, t0, ts);
  __syncthreads();
  prod_sigma<K>(S, P, Ae, t0, ts);
  __syncthreads();
  prod_final<K>(S, C, P, nu ? nu[e0 + e] : 1.0, with_load != 0 && Fe, Ae, Be, Fe, t0, ts);
}

struct DevTables {
  double *d = nullptr;
  int *i = nullptr;
  Tables T{};
  ~DevTables() {
    if (d) (void)hipFree(d);
    if (i) (void)hipFree(i);
  }
};

hipError_t upload_tables(int K, DevTables &out) {
  const HostTables H = make_tables(K);
  std::vector<double> dv;
  std::vector<int> iv;
  size_t o_ta = dv.size();
  dv.insert(dv.end(), H.ta.begin(), H.ta.end());
  size_t o_tb = dv.size();
  dv.insert(dv.end(), H.tb.begin(), H.tb.end());
  size_t o_tet = dv.size();
  dv.insert(dv.end(), H.tet.begin(), H.tet.end());
  size_t o_eg = dv.size();
  dv.insert(dv.end(), H.eg.begin(), H.eg.end());
  size_t o_lg = dv.size();
  dv.insert(dv.end(), H.lg.begin(), H.lg.end());
  size_t o_en = dv.size();
  dv.insert(dv.end(), H.enode.begin(), H.enode.end());
  size_t o_ed = iv.size();
  iv.insert(iv.end(), H.edges.begin(), H.edges.end());
  size_t o_fa = iv.size();
  iv.insert(iv.end(), H.faces.begin(), H.faces.end());
  size_t o_d4 = iv.size();
  iv.insert(iv.end(), H.d4pos.begin(), H.d4pos.end());
  hipError_t e = hipMalloc(&out.d, dv.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&out.i, iv.size() * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(out.d, dv.data(), dv.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(out.i, iv.data(), iv.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  Tables &T = out.T;
  T.nta = (int)(H.ta.size() / 4);
  T.ta = out.d + o_ta;
  T.ntb = (int)(H.tb.size() / 4);
  T.tb = out.d + o_tb;
  T.ntet = (int)(H.tet.size() / 5);
  T.tet = out.d + o_tet;
  T.neg = (int)(H.eg.size() / 2);
  T.eg = out.d + o_eg;
  T.lg = out.d + o_lg;
  T.enode = out.d + o_en;
  T.edges = out.i + o_ed;
  T.faces = out.i + o_fa;
  T.d4pos = out.i + o_d4;
  return hipSuccess;
}

template <int K>
int run(vb_ctx *ctx, int64_t n, const double *X8, const double *nu, int with_load, double *A, double *B,
        double *F) {
  typedef Dims<K> D;
  hipStream_t st = vb::ctx_stream(ctx);
  DevTables T;
  hipError_t e = upload_tables(K, T);
  if (e != hipSuccess) return vb::ctx_fail(ctx, VB_ERR_DEVICE, hipGetErrorString(e));
  // chunk: the interleaved shared, column and product blocks within 2 GiB
  const size_t per = sizeof(double) * ((size_t)Shared<K>::size + (size_t)Column<K>::size * D::N +
                                       (size_t)Products<K>::size);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)((size_t)2 << 30) / (int64_t)per));
  double *Sb = nullptr, *Cb = nullptr, *Pb = nullptr;
  e = hipMalloc(&Sb, sizeof(double) * Shared<K>::size * chunk);
  if (e == hipSuccess) e = hipMalloc(&Cb, sizeof(double) * Column<K>::size * D::N * chunk);
  if (e == hipSuccess) e = hipMalloc(&Pb, sizeof(double) * Products<K>::size * chunk);
  for (int64_t e0 = 0; e0 < n && e == hipSuccess; e0 += chunk) {
    const int64_t ne = std::min(chunk, n - e0);
    hipLaunchKernelGGL(k_vem_shared<K>, dim3((unsigned)((ne + 63) / 64)), dim3(64), 0, st, X8, nu,
                       with_load, T.T, Sb, e0, ne);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_vem_column<K>, dim3((unsigned)((ne * D::N + 63) / 64)), dim3(64), 0, st, T.T, Sb, Cb,
                       ne);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_vem_products<K>, dim3((unsigned)ne), dim3(256), 0, st, X8, nu, with_load, T.T, Sb,
                       Cb, Pb, e0, ne, A, B, F);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (Sb) (void)hipFree(Sb);
  if (Cb) (void)hipFree(Cb);
  if (Pb) (void)hipFree(Pb);
  if (e != hipSuccess) return vb::ctx_fail(ctx, VB_ERR_DEVICE, hipGetErrorString(e));
  return VB_OK;
}

}  // namespace

extern "C" int vb_vem_dofs(int k, int *n_dof, int *n_pressure) {
  if (k < 2 || k > 4 || !n_dof || !n_pressure) return VB_ERR_ARG;
  *n_dof = k == 2 ? Dims<2>::N : (k == 3 ? Dims<3>::N : Dims<4>::N);
  *n_pressure = k == 2 ? Dims<2>::nP : (k == 3 ? Dims<3>::nP : Dims<4>::nP);
  return VB_OK;
}

extern "C" int vb_vem_element_matrices(vb_ctx *ctx, int k, int64_t n_elem, const double *X8,
                                       const double *nu, int with_load, double *A, double *B, double *F) {
  if (!ctx || k < 2 || k > 4 || n_elem < 0 || (n_elem > 0 && (!X8 || !A || !B)) ||
      (with_load && n_elem > 0 && !F))
    return VB_ERR_ARG;
  if (n_elem == 0) return VB_OK;
  if (k == 2) return run<2>(ctx, n_elem, X8, nu, with_load, A, B, F);
  if (k == 3) return run<3>(ctx, n_elem, X8, nu, with_load, A, B, F);
  return run<4>(ctx, n_elem, X8, nu, with_load, A, B, F);
}
