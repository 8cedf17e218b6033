// Virtual element matrices of degree K on a hexahedron with planar faces
// (Sec. 3): the local stiffness of eq. discreteA, the divergence rows and
// the load vector of eq. discreteF, for the divergence-free space with the
// degrees of freedom D1-D5.
//
// The computation is split in three parts so that the device can spread it:
//   shared(e)     per element: geometry, the polynomial mass matrices, the
//                 face and element H1-projection systems (inverted), the
//                 restriction of the volume monomials to each face;
//   column(e, i)  per element and basis function phi_i (every quantity
//                 below is linear in the degrees of freedom, so each column
//                 is independent): the face moments, the boundary integrals,
//                 div phi_i, the volume moments, Pi^nabla_K phi_i,
//                 Pi^0_{K-1} grad phi_i, Pi^0_K phi_i;
//   the products  dof_i(Pi^nabla phi_j), the consistency term and the
//                 stabilisation (in vem.hip, one workgroup per element).
// The code is plain C++ callable from host or device: arrays are reached
// through accessors that interleave elements (or element columns) so that
// neighbouring device threads touch neighbouring addresses.
//
// Conventions (they define the numbering of the degrees of freedom):
// local vertex v = ix + 2 iy + 4 iz; local edges by axis a, then (o2, o1)
// offsets of the other two axes b < c, from vertex s to s + e_a; local faces
// 2a + side, vertices in the order (0,0), (1,0), (1,1), (0,1) of (b, c),
// their edges in local-edge order; the face frame (t1, t2, n): n the unit
// normal pointing to +axis, t1 along its first side, t2 = n x t1.
// Scaled monomials m_a = ((x - x_K)/h_K)^a by total degree, then the x
// exponent descending, then the y exponent descending; face monomials
// ((x - x_f).t1 / h_f, (x - x_f).t2 / h_f)^b likewise.
// Degrees of freedom: D1 the vertex values, D2 the values at the K - 1
// interior Gauss-Lobatto points of each edge, D3 the face moments
// (1/|f|) int v.n_f m, v.t1 m, v.t2 m for m of degree <= K-2, D4 the
// moments (1/|K|) int v.(xh ^ (e_c m_g)) for |g| <= K-3 without the pairs
// (c = z, g = z q), D5 (h_K/|K|) int div(v) m_a for the non-constant m_a of
// degree <= K-1.
#pragma once

#ifndef VEM_HD
#define VEM_HD __host__ __device__
#endif

#include <math.h>
#include <stdint.h>

namespace vb {
namespace vem {

VEM_HD constexpr int pdim3(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) * (n + 3) / 6; }
VEM_HD constexpr int pdim2(int n) { return n < 0 ? 0 : (n + 1) * (n + 2) / 2; }

template <int K> struct Dims {
  static constexpr int nf2 = pdim2(K - 2);
  static constexpr int nD4 = 3 * pdim3(K - 3) - pdim3(K - 4);
  static constexpr int nD5 = pdim3(K - 1) - 1;
  static constexpr int nP = pdim3(K - 1);
  static constexpr int off2 = 24;
  static constexpr int off3 = 24 + 36 * (K - 1);
  static constexpr int off4 = off3 + 18 * nf2;
  static constexpr int off5 = off4 + nD4;
  static constexpr int N = off5 + nD5;
  static constexpr int n1 = pdim2(K + 1);   // face monomials up to degree K+1
  static constexpr int nk2 = pdim2(K);      // face monomials up to degree K
  static constexpr int nlo = pdim2(K - 2);  // face moments that are degrees of freedom
  static constexpr int n3 = pdim3(K + 1);   // volume monomials up to degree K+1
  static constexpr int nk = pdim3(K);
  static constexpr int nkm1 = pdim3(K - 1);
  static constexpr int nkm2 = pdim3(K - 2);
  static constexpr int NE = K + 1;         // nodes per edge (vertices included)
};

// ---------------------------------------------------------------- monomials
VEM_HD inline int idx3(int a, int b, int c) {
  const int d = a + b + c;
  return pdim3(d - 1) + (d - a) * (d - a + 1) / 2 + (d - a - b);
}
VEM_HD inline void exp3(int i, int &a, int &b, int &c) {
  int d = 0;
  while (pdim3(d) <= i) ++d;
  int r = i - pdim3(d - 1);
  for (a = d; a >= 0; --a) {
    const int cnt = d - a + 1;
    if (r < cnt) break;
    r -= cnt;
  }
  b = d - a - r;
  c = d - a - b;
}
VEM_HD inline int idx2(int a, int b) { return pdim2(a + b - 1) + b; }
VEM_HD inline void exp2(int i, int &a, int &b) {
  int d = 0;
  while (pdim2(d) <= i) ++d;
  b = i - pdim2(d - 1);
  a = d - b;
}
// all monomials of degree <= n at xh: out[idx3(..)]
VEM_HD inline void eval3(const double *xh, int n, double *out) {
  double p[3][8];
  for (int d = 0; d < 3; ++d) {
    p[d][0] = 1.0;
    for (int q = 1; q <= n; ++q) p[d][q] = p[d][q - 1] * xh[d];
  }
  int i = 0;
  for (int dg = 0; dg <= n; ++dg)
    for (int a = dg; a >= 0; --a)
      for (int b = dg - a; b >= 0; --b) out[i++] = p[0][a] * p[1][b] * p[2][dg - a - b];
}
VEM_HD inline void eval2(const double *xi, int n, double *out) {
  double p[2][8];
  for (int d = 0; d < 2; ++d) {
    p[d][0] = 1.0;
    for (int q = 1; q <= n; ++q) p[d][q] = p[d][q - 1] * xi[d];
  }
  int i = 0;
  for (int dg = 0; dg <= n; ++dg)
    for (int a = dg; a >= 0; --a) out[i++] = p[0][a] * p[1][dg - a];
}
// d/dxi_d of the face monomials of degree <= n: out[2 * idx2 + d]
VEM_HD inline void grad2(const double *xi, int n, double *out) {
  double p[2][8];
  for (int d = 0; d < 2; ++d) {
    p[d][0] = 1.0;
    for (int q = 1; q <= n; ++q) p[d][q] = p[d][q - 1] * xi[d];
  }
  int i = 0;
  for (int dg = 0; dg <= n; ++dg)
    for (int a = dg; a >= 0; --a, ++i) {
      const int b = dg - a;
      out[2 * i] = a > 0 ? a * p[0][a - 1] * p[1][b] : 0.0;
      out[2 * i + 1] = b > 0 ? b * p[0][a] * p[1][b - 1] : 0.0;
    }
}
VEM_HD inline double levi(int i, int j, int k) {
  if (i == j || j == k || i == k) return 0.0;
  return ((i == 0 && j == 1) || (i == 1 && j == 2) || (i == 2 && j == 0)) ? 1.0 : -1.0;
}

// ---------------------------------------------------------------- tables
// Quadrature rules and the local topology (host-generated, device-resident).
struct Tables {
  int nta;            // face triangle rule exact to degree 2K+3: (l0, l1, l2, w)
  const double *ta;
  int ntb;            // face triangle rule exact to degree 2K+1
  const double *tb;
  int ntet;           // tetrahedron rule exact to degree 2K+1: (l0, l1, l2, l3, w)
  const double *tet;
  int neg;            // edge Gauss-Legendre rule on [0, 1]: (s, w)
  const double *eg;
  const double *lg;   // Lagrange basis of the edge nodes at the edge rule: neg x (K+1)
  const double *enode;  // the K+1 edge nodes on [0, 1]
  const int *edges;   // 12 x 3: axis, v0, v1
  const int *faces;   // 6 x 10: axis, side, 4 vertices, 4 edges
  const int *d4pos;   // 3 x pdim3(K-3): position of the D4 pair (c, g), or -1
};

// Strided views: element (or element column) `e` of an interleaved array.
struct View {
  double *p;
  int64_t stride;
  VEM_HD double &operator[](int64_t q) const { return p[q * stride]; }
};

// Gauss-Jordan elimination with partial pivoting on the n x (n + m)
// row-major block [A | B] (row stride ld): B <- A^-1 B.
VEM_HD inline void gj_solve(View M, int n, int m, int ld) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = fabs(M[(int64_t)c * ld + c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = fabs(M[(int64_t)r * ld + c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (piv != c)
      for (int j = 0; j < n + m; ++j) {
        const double t = M[(int64_t)c * ld + j];
        M[(int64_t)c * ld + j] = M[(int64_t)piv * ld + j];
        M[(int64_t)piv * ld + j] = t;
      }
    const double inv = 1.0 / M[(int64_t)c * ld + c];
    for (int j = c; j < n + m; ++j) M[(int64_t)c * ld + j] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[(int64_t)r * ld + c];
      if (f == 0.0) continue;
      for (int j = c; j < n + m; ++j) M[(int64_t)r * ld + j] -= f * M[(int64_t)c * ld + j];
    }
  }
}

// Layout of the per-element shared block (doubles).
template <int K> struct Shared {
  typedef Dims<K> D;
  static constexpr int geo = 0;                        // xK(3) hK vK xbar(3)
  static constexpr int face = 8;                       // 6 x [n t1 t2 xf hf af sig]
  static constexpr int FW = 15;
  static constexpr int mass = face + 6 * FW;           // n3 x n3
  static constexpr int rf = mass + D::n3 * D::n3;      // 6 x n1 x n3 (face b, volume a)
  static constexpr int fmh = rf + 6 * D::n1 * D::n3;   // 6 x nk2 x n1: face mass rows < nk2
  static constexpr int kinv = fmh + 6 * D::nk2 * D::n1;  // 6 x nk2 x nk2
  static constexpr int e0 = kinv + 6 * D::nk2 * D::nk2;  // 6 x 4 x NE
  static constexpr int e1 = e0 + 6 * 4 * D::NE;          // 6 x 4 x nk2 x NE
  static constexpr int k3inv = e1 + 6 * 4 * D::nk2 * D::NE;  // nk x nk
  static constexpr int m1inv = k3inv + D::nk * D::nk;        // nkm1 x nkm1
  static constexpr int mkinv = m1inv + D::nkm1 * D::nkm1;    // nk x nk
  static constexpr int fx = mkinv + D::nk * D::nk;           // 6 x nlo x nk: (1/|f|) int_f mu_b m_a
  static constexpr int fm = fx + 6 * D::nlo * D::nk;         // 3 x nk: int_K f_c m_a
  static constexpr int pb = fm + 3 * D::nk;                  // nk: int_dK m_a
  static constexpr int work = pb + D::nk;                    // elimination workspace
  static constexpr int wsize = (D::n3 > D::n1 ? D::n3 : D::n1) * (D::n3 + D::n1) + 64;
  static constexpr int size = work + wsize;
};

// Layout of the per-column block (doubles).
template <int K> struct Column {
  typedef Dims<K> D;
  static constexpr int bcoef = 0;                 // 3 x nk: Pi^nabla_K phi_i
  static constexpr int eps = bcoef + 3 * D::nk;   // 3 x 3 x nkm1: Pi^0_{K-1} of the symmetric gradient
  static constexpr int y = eps + 9 * D::nkm1;     // 3 x 3 x nkm1: its mass-weighted moments
  static constexpr int p0 = y + 9 * D::nkm1;      // 3 x nk: Pi^0_K phi_i
  static constexpr int mu = p0 + 3 * D::nk;       // nP: int_K div(phi_i) m_a
  static constexpr int out = mu + D::nP;          // outputs end here
  static constexpr int gc = out;                  // 3 x 3 x nkm1: Pi^0_{K-1} d_d (phi_i)_c
  static constexpr int bv = gc + 9 * D::nkm1;     // 3 x 3 x n3: int_dK (phi_i)_c m_a n_d
  static constexpr int bp = bv + 9 * D::n3;       // 3 x n3: int_dK (phi_i)_c m_a
  static constexpr int gq = bp + 3 * D::n3;       // n3: int_K phi_i . grad_x m_a
  static constexpr int vm = gq + D::n3;           // 3 x nk: int_K (phi_i)_c m_g
  static constexpr int size = vm + 3 * D::nk;
};

// the manufactured load of the benchmark: f = (3 pi^2 / 2) nu curl(psi),
// psi = sin(pi x) sin(pi y) sin(pi z) (1, 1, 1)
VEM_HD inline void load_field(const double *x, double nu, double *f) {
  const double pi = 3.14159265358979323846;
  const double sx = sin(pi * x[0]), sy = sin(pi * x[1]), sz = sin(pi * x[2]);
  const double cx = cos(pi * x[0]), cy = cos(pi * x[1]), cz = cos(pi * x[2]);
  const double dx = pi * cx * sy * sz, dy = pi * sx * cy * sz, dz = pi * sx * sy * cz;
  const double s = 1.5 * pi * pi * nu;
  f[0] = s * (dy - dz);
  f[1] = s * (dz - dx);
  f[2] = s * (dx - dy);
}

// ----------------------------------------------------------- shared part
template <int K>
VEM_HD void shared(const double *X8, double nu, bool with_load, const Tables &T, View S) {
  typedef Dims<K> D;
  typedef Shared<K> L;
  // ---- element geometry: volume and centroid by cones from the vertex mean
  double xb[3] = {0, 0, 0};
  for (int v = 0; v < 8; ++v)
    for (int d = 0; d < 3; ++d) xb[d] += X8[3 * v + d] / 8.0;
  double vol = 0.0, cen[3] = {0, 0, 0};
  for (int lf = 0; lf < 6; ++lf) {
    const int *F = T.faces + 10 * lf;
    for (int t = 0; t < 2; ++t) {
      const int va = F[2], vb = F[3 + t], vc = F[4 + t];
      double a[3], b[3], c[3];
      for (int d = 0; d < 3; ++d) {
        a[d] = X8[3 * va + d] - xb[d];
        b[d] = X8[3 * vb + d] - xb[d];
        c[d] = X8[3 * vc + d] - xb[d];
      }
      const double v = fabs(a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                            a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
      vol += v;
      for (int d = 0; d < 3; ++d)
        cen[d] += v * (xb[d] + X8[3 * va + d] + X8[3 * vb + d] + X8[3 * vc + d]) / 4.0;
    }
  }
  for (int d = 0; d < 3; ++d) cen[d] /= vol;
  double hK = 0.0;
  for (int i = 0; i < 8; ++i)
    for (int j = i + 1; j < 8; ++j) {
      double s = 0.0;
      for (int d = 0; d < 3; ++d) s += (X8[3 * i + d] - X8[3 * j + d]) * (X8[3 * i + d] - X8[3 * j + d]);
      hK = fmax(hK, sqrt(s));
    }
  for (int d = 0; d < 3; ++d) {
    S[L::geo + d] = cen[d];
    S[L::geo + 5 + d] = xb[d];
  }
  S[L::geo + 3] = hK;
  S[L::geo + 4] = vol;
  // ---- faces: area, centroid (two triangles), unit normal to +axis, t1
  //      along the first side, t2 = n x t1, diameter, outward sign
  for (int lf = 0; lf < 6; ++lf) {
    const int *F = T.faces + 10 * lf;
    const double *P0 = X8 + 3 * F[2], *P1 = X8 + 3 * F[3], *P2 = X8 + 3 * F[4], *P3 = X8 + 3 * F[5];
    double u1[3], u2[3], u3[3], c1[3], c2[3];
    for (int d = 0; d < 3; ++d) {
      u1[d] = P1[d] - P0[d];
      u2[d] = P2[d] - P0[d];
      u3[d] = P3[d] - P0[d];
    }
    c1[0] = u1[1] * u2[2] - u1[2] * u2[1];
    c1[1] = u1[2] * u2[0] - u1[0] * u2[2];
    c1[2] = u1[0] * u2[1] - u1[1] * u2[0];
    c2[0] = u2[1] * u3[2] - u2[2] * u3[1];
    c2[1] = u2[2] * u3[0] - u2[0] * u3[2];
    c2[2] = u2[0] * u3[1] - u2[1] * u3[0];
    const double a1 = 0.5 * sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
    const double a2 = 0.5 * sqrt(c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
    const double af = a1 + a2;
    double n[3], t1[3], t2[3], xf[3];
    for (int d = 0; d < 3; ++d) {
      xf[d] = ((P0[d] + P1[d] + P2[d]) / 3.0 * a1 + (P0[d] + P2[d] + P3[d]) / 3.0 * a2) / af;
      n[d] = c1[d] + c2[d];
    }
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const int ax = F[0];
    const double sg = n[ax] > 0 ? 1.0 : (n[ax] < 0 ? -1.0 : 0.0);
    for (int d = 0; d < 3; ++d) n[d] = n[d] / nn * sg;
    const double l1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    for (int d = 0; d < 3; ++d) t1[d] = u1[d] / l1;
    t2[0] = n[1] * t1[2] - n[2] * t1[1];
    t2[1] = n[2] * t1[0] - n[0] * t1[2];
    t2[2] = n[0] * t1[1] - n[1] * t1[0];
    double hf = 0.0;
    const double *Q[4] = {P0, P1, P2, P3};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += (Q[i][d] - Q[j][d]) * (Q[i][d] - Q[j][d]);
        hf = fmax(hf, sqrt(s));
      }
    const int o = L::face + L::FW * lf;
    for (int d = 0; d < 3; ++d) {
      S[o + d] = n[d];
      S[o + 3 + d] = t1[d];
      S[o + 6 + d] = t2[d];
      S[o + 9 + d] = xf[d];
    }
    S[o + 12] = hf;
    S[o + 13] = af;
    S[o + 14] = F[1] == 0 ? -1.0 : 1.0;
  }
  // ---- volume: the monomial mass matrix (rule exact to 2K+1), grad-grad of
  //      degree <= K, and the load moments int_K f_c m_a
  // (the grad-grad matrix accumulates in the k3inv slot, the load moments
  // in fm)
  double mm[D::n3], pt[3], xh[3];
  for (int q = 0; q < D::n3 * D::n3; ++q) S[L::mass + q] = 0.0;
  for (int q = 0; q < D::nk * D::nk; ++q) S[L::k3inv + q] = 0.0;
  for (int q = 0; q < 3 * D::nk; ++q) S[L::fm + q] = 0.0;
  for (int lf = 0; lf < 6; ++lf) {
    const int *F = T.faces + 10 * lf;
    for (int t = 0; t < 2; ++t) {
      const double *A = X8 + 3 * F[2], *B = X8 + 3 * F[3 + t], *C = X8 + 3 * F[4 + t];
      double a[3], b[3], c[3];
      for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - xb[d];
        b[d] = B[d] - xb[d];
        c[d] = C[d] - xb[d];
      }
      const double tv = fabs(a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                             a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
      for (int q = 0; q < T.ntet; ++q) {
        const double *r = T.tet + 5 * q;
        const double w = tv * r[4];
        for (int d = 0; d < 3; ++d) {
          pt[d] = r[0] * xb[d] + r[1] * A[d] + r[2] * B[d] + r[3] * C[d];
          xh[d] = (pt[d] - cen[d]) / hK;
        }
        eval3(xh, K + 1, mm);
        for (int i = 0; i < D::n3; ++i) {
          const double wi = w * mm[i];
          for (int j = 0; j < D::n3; ++j) S[L::mass + i * D::n3 + j] += wi * mm[j];
        }
        // gradients of the monomials of degree <= K (in x)
        double g[3][D::nk];
        for (int i = 0; i < D::nk; ++i) {
          int e[3];
          exp3(i, e[0], e[1], e[2]);
          for (int d = 0; d < 3; ++d) {
            if (e[d] == 0) {
              g[d][i] = 0.0;
            } else {
              int f[3] = {e[0], e[1], e[2]};
              f[d] -= 1;
              g[d][i] = e[d] * mm[idx3(f[0], f[1], f[2])] / hK;
            }
          }
        }
        for (int i = 0; i < D::nk; ++i)
          for (int j = 0; j < D::nk; ++j)
            S[L::k3inv + i * D::nk + j] += w * (g[0][i] * g[0][j] + g[1][i] * g[1][j] + g[2][i] * g[2][j]);
        if (with_load) {
          double fv[3];
          load_field(pt, nu, fv);
          for (int c = 0; c < 3; ++c)
            for (int i = 0; i < D::nk; ++i) S[L::fm + c * D::nk + i] += w * fv[c] * mm[i];
        }
      }
    }
  }
  // ---- faces: mass of the face monomials (degree <= K+1), their gradients
  //      (degree <= K), restriction of the volume monomials, boundary mean
  //      row of the face projection and the edge tables
  for (int i = 0; i < D::nk; ++i) S[L::pb + i] = 0.0;
  for (int lf = 0; lf < 6; ++lf) {
    const int *F = T.faces + 10 * lf;
    const int o = L::face + L::FW * lf;
    double n[3], t1[3], t2[3], xf[3];
    for (int d = 0; d < 3; ++d) {
      n[d] = S[o + d];
      t1[d] = S[o + 3 + d];
      t2[d] = S[o + 6 + d];
      xf[d] = S[o + 9 + d];
    }
    const double hf = S[o + 12], af = S[o + 13];
    // workspace: [FMass | R] (n1 x (n1 + n3)), row-major
    View W{&S[L::work], S.stride};
    const int ldw = D::n1 + D::n3;
    for (int q = 0; q < D::n1 * ldw; ++q) W[q] = 0.0;
    // the face grad-grad matrix accumulates in this face's kinv slot, the
    // face moments of the volume monomials in its fx slot
    const int okv = L::kinv + lf * D::nk2 * D::nk2, ofx = L::fx + lf * D::nlo * D::nk;
    for (int q = 0; q < D::nk2 * D::nk2; ++q) S[okv + q] = 0.0;
    for (int q = 0; q < D::nlo * D::nk; ++q) S[ofx + q] = 0.0;
    for (int t = 0; t < 2; ++t) {
      const double *A = X8 + 3 * F[2], *B = X8 + 3 * F[3 + t], *C = X8 + 3 * F[4 + t];
      double u[3], v[3], cr[3];
      for (int d = 0; d < 3; ++d) {
        u[d] = B[d] - A[d];
        v[d] = C[d] - A[d];
      }
      cr[0] = u[1] * v[2] - u[2] * v[1];
      cr[1] = u[2] * v[0] - u[0] * v[2];
      cr[2] = u[0] * v[1] - u[1] * v[0];
      const double ta = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int q = 0; q < T.nta; ++q) {
        const double *r = T.ta + 4 * q;
        const double w = ta * r[3];
        double xi[2];
        for (int d = 0; d < 3; ++d) {
          pt[d] = r[0] * A[d] + r[1] * B[d] + r[2] * C[d];
          xh[d] = (pt[d] - cen[d]) / hK;
        }
        xi[0] = ((pt[0] - xf[0]) * t1[0] + (pt[1] - xf[1]) * t1[1] + (pt[2] - xf[2]) * t1[2]) / hf;
        xi[1] = ((pt[0] - xf[0]) * t2[0] + (pt[1] - xf[1]) * t2[1] + (pt[2] - xf[2]) * t2[2]) / hf;
        double mf[D::n1], gf[2 * D::nk2];
        eval2(xi, K + 1, mf);
        grad2(xi, K, gf);
        eval3(xh, K + 1, mm);
        for (int i = 0; i < D::n1; ++i) {
          for (int j = 0; j < D::n1; ++j) W[i * ldw + j] += w * mf[i] * mf[j];
          for (int j = 0; j < D::n3; ++j) W[i * ldw + D::n1 + j] += w * mf[i] * mm[j];
        }
        for (int i = 0; i < D::nk2; ++i)
          for (int j = 0; j < D::nk2; ++j)
            S[okv + i * D::nk2 + j] += w * (gf[2 * i] * gf[2 * j] + gf[2 * i + 1] * gf[2 * j + 1]) / (hf * hf);
      }
      // degree 2K+1 rule: the face-moment rows of the degree-of-freedom
      // matrix and the boundary integrals of the volume monomials
      for (int q = 0; q < T.ntb; ++q) {
        const double *r = T.tb + 4 * q;
        const double w = ta * r[3];
        double xi[2];
        for (int d = 0; d < 3; ++d) {
          pt[d] = r[0] * A[d] + r[1] * B[d] + r[2] * C[d];
          xh[d] = (pt[d] - cen[d]) / hK;
        }
        xi[0] = ((pt[0] - xf[0]) * t1[0] + (pt[1] - xf[1]) * t1[1] + (pt[2] - xf[2]) * t1[2]) / hf;
        xi[1] = ((pt[0] - xf[0]) * t2[0] + (pt[1] - xf[1]) * t2[1] + (pt[2] - xf[2]) * t2[2]) / hf;
        double m2[D::nlo > 0 ? D::nlo : 1];
        eval2(xi, K - 2, m2);
        eval3(xh, K, mm);
        for (int i = 0; i < D::nk; ++i) S[L::pb + i] += w * mm[i];
        for (int b = 0; b < D::nlo; ++b)
          for (int i = 0; i < D::nk; ++i) S[ofx + b * D::nk + i] += w * m2[b] * mm[i] / af;
      }
    }
    // face mass rows < nk2 (the enhancement map), then Rf = FMass^-1 R
    for (int i = 0; i < D::nk2; ++i)
      for (int j = 0; j < D::n1; ++j) S[L::fmh + (lf * D::nk2 + i) * D::n1 + j] = W[i * ldw + j];
    gj_solve(W, D::n1, D::n3, ldw);
    for (int i = 0; i < D::n1; ++i)
      for (int j = 0; j < D::n3; ++j) S[L::rf + (lf * D::n1 + i) * D::n3 + j] = W[i * ldw + D::n1 + j];
    // edges of the face: the face-projection system's boundary row and the
    // tables of the edge integrals (Lagrange node basis x the face monomial
    // or its in-plane outward normal derivative)
    double kb0[D::nk2];
    for (int i = 0; i < D::nk2; ++i) kb0[i] = 0.0;
    for (int q4 = 0; q4 < 4; ++q4) {
      const int le = F[6 + q4];
      const int v0 = T.edges[3 * le + 1], v1 = T.edges[3 * le + 2];
      const double *A0 = X8 + 3 * v0, *A1 = X8 + 3 * v1;
      double ev[3], ne[3], mid[3];
      for (int d = 0; d < 3; ++d) {
        ev[d] = A1[d] - A0[d];
        mid[d] = 0.5 * (A0[d] + A1[d]);
      }
      const double len = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
      ne[0] = ev[1] * n[2] - ev[2] * n[1];
      ne[1] = ev[2] * n[0] - ev[0] * n[2];
      ne[2] = ev[0] * n[1] - ev[1] * n[0];
      const double nl = sqrt(ne[0] * ne[0] + ne[1] * ne[1] + ne[2] * ne[2]);
      const double so = (mid[0] - xf[0]) * ne[0] + (mid[1] - xf[1]) * ne[1] + (mid[2] - xf[2]) * ne[2];
      const double sgn = so > 0 ? 1.0 : (so < 0 ? -1.0 : 0.0);
      for (int d = 0; d < 3; ++d) ne[d] = ne[d] / nl * sgn;
      const double c1n = t1[0] * ne[0] + t1[1] * ne[1] + t1[2] * ne[2];
      const double c2n = t2[0] * ne[0] + t2[1] * ne[1] + t2[2] * ne[2];
      const int oe0 = L::e0 + (lf * 4 + q4) * D::NE;
      const int oe1 = L::e1 + (lf * 4 + q4) * D::nk2 * D::NE;
      for (int j = 0; j < D::NE; ++j) S[oe0 + j] = 0.0;
      for (int q = 0; q < D::nk2 * D::NE; ++q) S[oe1 + q] = 0.0;
      for (int q = 0; q < T.neg; ++q) {
        const double s = T.eg[2 * q], wl = T.eg[2 * q + 1] * len;
        double xi[2];
        for (int d = 0; d < 3; ++d) pt[d] = A0[d] + s * ev[d];
        xi[0] = ((pt[0] - xf[0]) * t1[0] + (pt[1] - xf[1]) * t1[1] + (pt[2] - xf[2]) * t1[2]) / hf;
        xi[1] = ((pt[0] - xf[0]) * t2[0] + (pt[1] - xf[1]) * t2[1] + (pt[2] - xf[2]) * t2[2]) / hf;
        double mq[D::nk2], gq[2 * D::nk2];
        eval2(xi, K, mq);
        grad2(xi, K, gq);
        for (int i = 0; i < D::nk2; ++i) kb0[i] += wl * mq[i];
        for (int j = 0; j < D::NE; ++j) {
          const double lw = wl * T.lg[q * D::NE + j];
          S[oe0 + j] += lw;
          for (int i = 1; i < D::nk2; ++i)
            S[oe1 + i * D::NE + j] += lw * (gq[2 * i] * c1n + gq[2 * i + 1] * c2n) / hf;
        }
      }
    }
    // the face projection system: grad-grad rows, the first row replaced
    // by the boundary integrals; inverted
    const int ldk = 2 * D::nk2;
    for (int i = 0; i < D::nk2; ++i)
      for (int j = 0; j < D::nk2; ++j) {
        W[i * ldk + j] = (i == 0) ? kb0[j] : S[okv + i * D::nk2 + j];
        W[i * ldk + D::nk2 + j] = (i == j) ? 1.0 : 0.0;
      }
    gj_solve(W, D::nk2, D::nk2, ldk);
    for (int i = 0; i < D::nk2; ++i)
      for (int j = 0; j < D::nk2; ++j) S[L::kinv + (lf * D::nk2 + i) * D::nk2 + j] = W[i * ldk + D::nk2 + j];
  }
  // ---- the element projection system (first row: boundary integrals),
  //      and the inverse mass blocks of degrees <= K-1 and <= K
  View W{&S[L::work], S.stride};
  {
    const int ld = 2 * D::nk;
    for (int i = 0; i < D::nk; ++i)
      for (int j = 0; j < D::nk; ++j) {
        W[i * ld + j] = (i == 0) ? S[L::pb + j] : S[L::k3inv + i * D::nk + j];
        W[i * ld + D::nk + j] = (i == j) ? 1.0 : 0.0;
      }
    gj_solve(W, D::nk, D::nk, ld);
    for (int i = 0; i < D::nk; ++i)
      for (int j = 0; j < D::nk; ++j) S[L::k3inv + i * D::nk + j] = W[i * ld + D::nk + j];
  }
  {
    const int n = D::nkm1, ld = 2 * n;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        W[i * ld + j] = S[L::mass + i * D::n3 + j];
        W[i * ld + n + j] = (i == j) ? 1.0 : 0.0;
      }
    gj_solve(W, n, n, ld);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) S[L::m1inv + i * n + j] = W[i * ld + n + j];
  }
  {
    const int n = D::nk, ld = 2 * n;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        W[i * ld + j] = S[L::mass + i * D::n3 + j];
        W[i * ld + n + j] = (i == j) ? 1.0 : 0.0;
      }
    gj_solve(W, n, n, ld);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) S[L::mkinv + i * n + j] = W[i * ld + n + j];
  }
}

// ---------------------------------------------------------- column part
// The degree of freedom `i` as a (kind, entity, index, component) record.
struct Dof {
  int kind;  // 1..5 (D1..D5)
  int ent;   // vertex, edge, face; D4 pair position; D5 monomial - 1
  int j;     // edge node (0 .. K-2) or face moment monomial
  int c;     // component (D1, D2) or face kind (D3: 0 normal, 1 t1, 2 t2)
};
template <int K> VEM_HD inline Dof dof_of(int i) {
  typedef Dims<K> D;
  Dof r{0, 0, 0, 0};
  if (i < D::off2) {
    r.kind = 1;
    r.ent = i / 3;
    r.c = i % 3;
  } else if (i < D::off3) {
    const int q = i - D::off2;
    r.kind = 2;
    r.c = q % 3;
    r.ent = (q / 3) / (K - 1);
    r.j = (q / 3) % (K - 1);
  } else if (i < D::off4) {
    const int q = i - D::off3;
    r.kind = 3;
    r.c = q % 3;
    r.ent = (q / 3) / D::nf2;
    r.j = (q / 3) % D::nf2;
  } else if (i < D::off5) {
    r.kind = 4;
    r.ent = i - D::off4;
  } else {
    r.kind = 5;
    r.ent = i - D::off5;
  }
  return r;
}

// (1/|K|) int_K phi_i . (xh ^ (e_kk m_gg)) for |gg| <= K-3: the D4 value of
// the pair, or for a left-out pair (kk = z, gg = z q) minus the (x, x q) and
// (y, y q) values (xh ^ (xh q) = 0)
template <int K> VEM_HD inline double d4_value(const Tables &T, const Dof &dd, int kk, int gg) {
  typedef Dims<K> D;
  if (dd.kind != 4) return 0.0;
  const int p = T.d4pos[kk * pdim3(K - 3) + gg];
  if (p >= 0) return dd.ent == p ? 1.0 : 0.0;
  int e[3];
  exp3(gg, e[0], e[1], e[2]);
  const int gx = idx3(e[0] + 1, e[1], e[2] - 1), gy = idx3(e[0], e[1] + 1, e[2] - 1);
  double v = 0.0;
  if (dd.ent == T.d4pos[0 * pdim3(K - 3) + gx]) v -= 1.0;
  if (dd.ent == T.d4pos[1 * pdim3(K - 3) + gy]) v -= 1.0;
  (void)sizeof(D);
  return v;
}

template <int K>
VEM_HD void column(int i, const Tables &T, View S, View C) {
  typedef Dims<K> D;
  typedef Shared<K> L;
  typedef Column<K> Q;
  const Dof dd = dof_of<K>(i);
  const double hK = S[L::geo + 3], vK = S[L::geo + 4];
  for (int q = 0; q < 9 * D::n3; ++q) C[Q::bv + q] = 0.0;
  for (int q = 0; q < 3 * D::n3; ++q) C[Q::bp + q] = 0.0;
  // ---- faces: moments of (phi_i)_c against the face monomials of degree
  //      <= K+1 (degrees of freedom below K-1, the face H1 projection above),
  //      restricted to the volume monomials, into the boundary integrals
  for (int lf = 0; lf < 6; ++lf) {
    const int *F = T.faces + 10 * lf;
    const int o = L::face + L::FW * lf;
    const double hf = S[o + 12], af = S[o + 13], sig = S[o + 14];
    double frame[3][3];
    for (int d = 0; d < 3; ++d) {
      frame[0][d] = S[o + d];
      frame[1][d] = S[o + 3 + d];
      frame[2][d] = S[o + 6 + d];
    }
    // is phi_i a node of this face's edges, or one of its moments?
    bool touches = dd.kind == 3 && dd.ent == lf;
    int nodeq[4] = {-1, -1, -1, -1};  // node of phi_i on each edge of the face (component dd.c)
    if (dd.kind == 1 || dd.kind == 2)
      for (int q4 = 0; q4 < 4; ++q4) {
        const int le = F[6 + q4];
        const int v0 = T.edges[3 * le + 1], v1 = T.edges[3 * le + 2];
        if (dd.kind == 1 && dd.ent == v0) nodeq[q4] = 0;
        if (dd.kind == 1 && dd.ent == v1) nodeq[q4] = K;
        if (dd.kind == 2 && dd.ent == le) nodeq[q4] = 1 + dd.j;
        if (nodeq[q4] >= 0) touches = true;
      }
    if (!touches) continue;
    for (int c = 0; c < 3; ++c) {
      double dm[D::nlo > 0 ? D::nlo : 1];
      for (int b = 0; b < D::nlo; ++b) dm[b] = 0.0;
      if (dd.kind == 3 && dd.ent == lf) dm[dd.j] = af * frame[dd.c][c];
      double rhs[D::nk2];
      for (int b = 0; b < D::nk2; ++b) rhs[b] = 0.0;
      if (dd.kind != 3 && dd.c == c)
        for (int q4 = 0; q4 < 4; ++q4) {
          if (nodeq[q4] < 0) continue;
          const int oe0 = L::e0 + (lf * 4 + q4) * D::NE;
          const int oe1 = L::e1 + (lf * 4 + q4) * D::nk2 * D::NE;
          rhs[0] += S[oe0 + nodeq[q4]];
          for (int b = 1; b < D::nk2; ++b) rhs[b] += S[oe1 + b * D::NE + nodeq[q4]];
        }
      // - int_f v_c Lap(mu_b), Lap(mu_b) of degree <= K-2 (face moments)
      for (int b = 1; b < D::nk2; ++b) {
        int a2, b2;
        exp2(b, a2, b2);
        double s = 0.0;
        if (a2 >= 2) s += a2 * (a2 - 1) * dm[idx2(a2 - 2, b2)];
        if (b2 >= 2) s += b2 * (b2 - 1) * dm[idx2(a2, b2 - 2)];
        rhs[b] -= s / (hf * hf);
      }
      double av[D::nk2];
      for (int r = 0; r < D::nk2; ++r) {
        double s = 0.0;
        for (int q = 0; q < D::nk2; ++q) s += S[L::kinv + (lf * D::nk2 + r) * D::nk2 + q] * rhs[q];
        av[r] = s;
      }
      double fmv[D::n1];
      for (int b = 0; b < D::nlo; ++b) fmv[b] = dm[b];
      for (int b = D::nlo; b < D::n1; ++b) {
        double s = 0.0;
        for (int g = 0; g < D::nk2; ++g) s += S[L::fmh + (lf * D::nk2 + g) * D::n1 + b] * av[g];
        fmv[b] = s;
      }
      for (int a = 0; a < D::n3; ++a) {
        double s = 0.0;
        for (int b = 0; b < D::n1; ++b) s += S[L::rf + (lf * D::n1 + b) * D::n3 + a] * fmv[b];
        C[Q::bp + c * D::n3 + a] += s;
        for (int d = 0; d < 3; ++d) C[Q::bv + (c * 3 + d) * D::n3 + a] += sig * frame[0][d] * s;
      }
    }
  }
  // ---- div phi_i in P_{K-1}: its moments (the flux through dK for the
  //      constant, D5 for the rest), the polynomial, int div(phi_i) m_a
  double mu[D::nkm1];
  for (int a = 0; a < D::nkm1; ++a) mu[a] = 0.0;
  if (dd.kind == 3 && dd.j == 0 && dd.c == 0) {
    const int o = L::face + L::FW * dd.ent;
    mu[0] = S[o + 14] * S[o + 13];
  }
  if (dd.kind == 5) mu[dd.ent + 1] = vK / hK;
  for (int a = 0; a < D::nP; ++a) C[Q::mu + a] = mu[a];
  double dco[D::nkm1];
  for (int r = 0; r < D::nkm1; ++r) {
    double s = 0.0;
    for (int q = 0; q < D::nkm1; ++q) s += S[L::m1inv + r * D::nkm1 + q] * mu[q];
    dco[r] = s;
  }
  // int_K phi_i . grad_x m_a = -int div(phi_i) m_a + int_dK (phi_i . n) m_a
  for (int a = 0; a < D::n3; ++a) {
    double dq = 0.0;
    for (int b = 0; b < D::nkm1; ++b) dq += dco[b] * S[L::mass + b * D::n3 + a];
    const double bn = C[Q::bv + 0 * D::n3 + a] + C[Q::bv + 4 * D::n3 + a] + C[Q::bv + 8 * D::n3 + a];
    C[Q::gq + a] = bn - dq;
  }
  // ---- volume moments int_K (phi_i)_c m_g, |g| <= K-2: e_c m_g = grad q +
  //      xh ^ r with q = xh_c m_g / (j+1), r = -curl(e_c m_g) / (j+1)
  //      (j = |g|); the x-wedge part from D4
  for (int c = 0; c < 3; ++c)
    for (int g = 0; g < D::nkm2; ++g) {
      int e[3];
      exp3(g, e[0], e[1], e[2]);
      const int j = e[0] + e[1] + e[2];
      int f[3] = {e[0], e[1], e[2]};
      f[c] += 1;
      double val = hK * C[Q::gq + idx3(f[0], f[1], f[2])] / (j + 1);
      if (j >= 1)
        for (int kk = 0; kk < 3; ++kk)
          for (int l = 0; l < 3; ++l) {
            const double eps = levi(kk, l, c);
            if (eps == 0.0 || e[l] == 0) continue;
            int h[3] = {e[0], e[1], e[2]};
            h[l] -= 1;
            const double r = -eps * e[l] / (j + 1);
            val += r * vK * d4_value<K>(T, dd, kk, idx3(h[0], h[1], h[2]));
          }
      C[Q::vm + c * D::nk + g] = val;
    }
  // ---- Pi^nabla_K phi_i: grad-grad moments (boundary term minus Laplacian
  //      moments), the first row the boundary integral
  for (int c = 0; c < 3; ++c) {
    double rhs[D::nk];
    rhs[0] = C[Q::bp + c * D::n3 + 0];
    for (int a = 1; a < D::nk; ++a) {
      int e[3];
      exp3(a, e[0], e[1], e[2]);
      double s = 0.0;
      for (int d = 0; d < 3; ++d) {
        if (e[d] >= 2) {
          int h[3] = {e[0], e[1], e[2]};
          h[d] -= 2;
          s -= e[d] * (e[d] - 1) * C[Q::vm + c * D::nk + idx3(h[0], h[1], h[2])] / (hK * hK);
        }
        if (e[d] >= 1) {
          int h[3] = {e[0], e[1], e[2]};
          h[d] -= 1;
          s += e[d] * C[Q::bv + (c * 3 + d) * D::n3 + idx3(h[0], h[1], h[2])] / hK;
        }
      }
      rhs[a] = s;
    }
    for (int r = 0; r < D::nk; ++r) {
      double s = 0.0;
      for (int q = 0; q < D::nk; ++q) s += S[L::k3inv + r * D::nk + q] * rhs[q];
      C[Q::bcoef + c * D::nk + r] = s;
    }
  }
  // ---- Pi^0_{K-1} grad phi_i: int d_d (phi_i)_c m_a = int_dK (phi_i)_c m_a
  //      n_d - int (phi_i)_c d_d m_a
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) {
      double gm[D::nkm1];
      for (int a = 0; a < D::nkm1; ++a) {
        int e[3];
        exp3(a, e[0], e[1], e[2]);
        double s = C[Q::bv + (c * 3 + d) * D::n3 + a];
        if (e[d] >= 1) {
          int h[3] = {e[0], e[1], e[2]};
          h[d] -= 1;
          s -= e[d] * C[Q::vm + c * D::nk + idx3(h[0], h[1], h[2])] / hK;
        }
        gm[a] = s;
      }
      for (int r = 0; r < D::nkm1; ++r) {
        double s = 0.0;
        for (int q = 0; q < D::nkm1; ++q) s += S[L::m1inv + r * D::nkm1 + q] * gm[q];
        C[Q::gc + (c * 3 + d) * D::nkm1 + r] = s;
      }
    }
  // ---- the moments of degrees K-1 and K (super-enhancement: the x-wedge
  //      part from Pi^nabla_K phi_i), then Pi^0_K phi_i
  for (int c = 0; c < 3; ++c)
    for (int g = D::nkm2; g < D::nk; ++g) {
      int e[3];
      exp3(g, e[0], e[1], e[2]);
      const int j = e[0] + e[1] + e[2];
      int f[3] = {e[0], e[1], e[2]};
      f[c] += 1;
      double val = hK * C[Q::gq + idx3(f[0], f[1], f[2])] / (j + 1);
      // xh ^ r, r_kk = -eps(kk, l, c) e_l m_{g - e_l} / (j+1): component
      // c2 = sum eps(c2, l2, kk) r_kk xh_l2
      for (int kk = 0; kk < 3; ++kk)
        for (int l = 0; l < 3; ++l) {
          const double eps = levi(kk, l, c);
          if (eps == 0.0 || e[l] == 0) continue;
          const double r = -eps * e[l] / (j + 1);
          for (int c2 = 0; c2 < 3; ++c2)
            for (int l2 = 0; l2 < 3; ++l2) {
              const double e2 = levi(c2, l2, kk);
              if (e2 == 0.0) continue;
              int h[3] = {e[0], e[1], e[2]};
              h[l] -= 1;
              h[l2] += 1;
              const int p = idx3(h[0], h[1], h[2]);
              double s = 0.0;
              for (int b = 0; b < D::nk; ++b) s += C[Q::bcoef + c2 * D::nk + b] * S[L::mass + b * D::n3 + p];
              val += e2 * r * s;
            }
        }
      C[Q::vm + c * D::nk + g] = val;
    }
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < D::nk; ++r) {
      double s = 0.0;
      for (int q = 0; q < D::nk; ++q) s += S[L::mkinv + r * D::nk + q] * C[Q::vm + c * D::nk + q];
      C[Q::p0 + c * D::nk + r] = s;
    }
  // ---- the consistency term's factors: eps = sym(Pi^0_{K-1} grad phi_i)
  //      and its moments against the monomials of degree <= K-1
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d)
      for (int a = 0; a < D::nkm1; ++a)
        C[Q::eps + (c * 3 + d) * D::nkm1 + a] =
            0.5 * (C[Q::gc + (c * 3 + d) * D::nkm1 + a] + C[Q::gc + (d * 3 + c) * D::nkm1 + a]);
  for (int cd = 0; cd < 9; ++cd)
    for (int a = 0; a < D::nkm1; ++a) {
      double s = 0.0;
      for (int b = 0; b < D::nkm1; ++b) s += S[L::mass + a * D::n3 + b] * C[Q::eps + cd * D::nkm1 + b];
      C[Q::y + cd * D::nkm1 + a] = s;
    }
}

// dof_i(e_c m_b), b < nk: row i of the degree-of-freedom matrix of the
// vector monomials, out[c * nk + b]
template <int K>
VEM_HD void dof_row(int i, const double *X8, const Tables &T, View S, double *out) {
  typedef Dims<K> D;
  typedef Shared<K> L;
  const Dof dd = dof_of<K>(i);
  const double hK = S[L::geo + 3], vK = S[L::geo + 4];
  double cen[3] = {S[L::geo + 0], S[L::geo + 1], S[L::geo + 2]};
  for (int q = 0; q < 3 * D::nk; ++q) out[q] = 0.0;
  double xh[3], mm[D::nk];
  if (dd.kind == 1 || dd.kind == 2) {
    double pt[3];
    if (dd.kind == 1) {
      for (int d = 0; d < 3; ++d) pt[d] = X8[3 * dd.ent + d];
    } else {
      const int v0 = T.edges[3 * dd.ent + 1], v1 = T.edges[3 * dd.ent + 2];
      const double t = T.enode[1 + dd.j];
      for (int d = 0; d < 3; ++d) pt[d] = X8[3 * v0 + d] + t * (X8[3 * v1 + d] - X8[3 * v0 + d]);
    }
    for (int d = 0; d < 3; ++d) xh[d] = (pt[d] - cen[d]) / hK;
    eval3(xh, K, mm);
    for (int b = 0; b < D::nk; ++b) out[dd.c * D::nk + b] = mm[b];
  } else if (dd.kind == 3) {
    const int o = L::face + L::FW * dd.ent;
    for (int c = 0; c < 3; ++c) {
      const double vec = S[o + 3 * dd.c + c];
      for (int b = 0; b < D::nk; ++b)
        out[c * D::nk + b] = vec * S[L::fx + (dd.ent * D::nlo + dd.j) * D::nk + b];
    }
  } else if (dd.kind == 4) {
    // the pair (kk, gg) of position dd.ent: xh ^ (e_kk m_gg), component c
    // = sum_l eps(c, l, kk) m_{gg + e_l}
    int kk = 0, gg = 0;
    for (int k2 = 0; k2 < 3; ++k2)
      for (int g2 = 0; g2 < pdim3(K - 3); ++g2)
        if (T.d4pos[k2 * pdim3(K - 3) + g2] == dd.ent) {
          kk = k2;
          gg = g2;
        }
    int e[3];
    exp3(gg, e[0], e[1], e[2]);
    for (int c = 0; c < 3; ++c)
      for (int l = 0; l < 3; ++l) {
        const double eps = levi(c, l, kk);
        if (eps == 0.0) continue;
        int h[3] = {e[0], e[1], e[2]};
        h[l] += 1;
        const int p = idx3(h[0], h[1], h[2]);
        for (int b = 0; b < D::nk; ++b) out[c * D::nk + b] += eps * S[L::mass + b * D::n3 + p] / vK;
      }
  } else {
    // (h_K/|K|) int div(e_c m_b) m_a = (1/|K|) e_c(b) int m_{b - e_c} m_a
    const int a = dd.ent + 1;
    for (int c = 0; c < 3; ++c)
      for (int b = 0; b < D::nk; ++b) {
        int e[3];
        exp3(b, e[0], e[1], e[2]);
        if (e[c] == 0) continue;
        int h[3] = {e[0], e[1], e[2]};
        h[c] -= 1;
        out[c * D::nk + b] = e[c] * S[L::mass + idx3(h[0], h[1], h[2]) * D::n3 + a] / vK;
      }
  }
}

// ------------------------------------------------------------ products
// Per element, with the columns' outputs C_j = column j's block: the
// degree-of-freedom matrix of the vector monomials, dof_i(Pi^nabla phi_j),
// the consistency term, the stabilisation sigma_i = max(h_K, consistency_ii)
// (the D-recipe reading), A = nu (consistency + (I - DPi)^T diag(sigma)
// (I - DPi)), B = the divergence moments, F = int f . Pi^0_K phi_j.  Each
// stage loops t over [t0, total) in steps of ts so that a workgroup can
// share it; the caller separates the stages.
template <int K> struct Products {
  typedef Dims<K> D;
  static constexpr int dofm = 0;                       // N x 3nk
  static constexpr int dpi = dofm + D::N * 3 * D::nk;  // N x N
  static constexpr int sigma = dpi + D::N * D::N;      // N
  static constexpr int size = sigma + D::N;
};
// stage 1: DOFM rows
template <int K>
VEM_HD void prod_dofm(const double *X8, const Tables &T, View S, double *P, int t0, int ts) {
  typedef Dims<K> D;
  for (int i = t0; i < D::N; i += ts) dof_row<K>(i, X8, T, S, P + Products<K>::dofm + (int64_t)i * 3 * D::nk);
}
// The column blocks of one element: column j at p + base + j, stride
// `stride` between entries.
struct ColSet {
  double *p;
  int64_t stride, base;
  VEM_HD View operator[](int j) const { return View{p + base + j, stride}; }
};
// stage 2: DPi and the consistency term (into A)
template <int K>
VEM_HD void prod_dpi(View S, const ColSet &Ccol, double *P, double *A, int t0, int ts) {
  typedef Dims<K> D;
  typedef Column<K> Q;
  for (int t = t0; t < D::N * D::N; t += ts) {
    const int i = t / D::N, j = t % D::N;
    const double *dr = P + Products<K>::dofm + (int64_t)i * 3 * D::nk;
    double s = 0.0;
    for (int q = 0; q < 3 * D::nk; ++q) s += dr[q] * Ccol[j][Q::bcoef + q];
    P[Products<K>::dpi + (int64_t)i * D::N + j] = s;
    double a = 0.0;
    for (int q = 0; q < 9 * D::nkm1; ++q) a += Ccol[i][Q::eps + q] * Ccol[j][Q::y + q];
    A[(int64_t)i * D::N + j] = a;
  }
  (void)S;
}
// stage 3: sigma
template <int K>
VEM_HD void prod_sigma(View S, double *P, const double *A, int t0, int ts) {
  typedef Dims<K> D;
  const double hK = S[Shared<K>::geo + 3];
  for (int i = t0; i < D::N; i += ts) P[Products<K>::sigma + i] = fmax(hK, A[(int64_t)i * D::N + i]);
}
// stage 4: A, B, F
template <int K>
VEM_HD void prod_final(View S, const ColSet &Ccol, const double *P, double nu, bool with_load, double *A,
                       double *B, double *F, int t0, int ts) {
  typedef Dims<K> D;
  typedef Column<K> Q;
  const double *dpi = P + Products<K>::dpi, *sg = P + Products<K>::sigma;
  for (int t = t0; t < D::N * D::N; t += ts) {
    const int i = t / D::N, j = t % D::N;
    double s = 0.0;
    for (int k = 0; k < D::N; ++k) {
      const double a = (k == i ? 1.0 : 0.0) - dpi[(int64_t)k * D::N + i];
      const double b = (k == j ? 1.0 : 0.0) - dpi[(int64_t)k * D::N + j];
      s += a * sg[k] * b;
    }
    A[(int64_t)i * D::N + j] = nu * (A[(int64_t)i * D::N + j] + s);
  }
  for (int t = t0; t < D::nP * D::N; t += ts) {
    const int a = t / D::N, j = t % D::N;
    B[(int64_t)a * D::N + j] = Ccol[j][Q::mu + a];
  }
  if (with_load)
    for (int j = t0; j < D::N; j += ts) {
      double s = 0.0;
      for (int q = 0; q < 3 * D::nk; ++q) s += S[Shared<K>::fm + q] * Ccol[j][Q::p0 + q];
      F[j] = s;
    }
}

}  // namespace vem
}  // namespace vb
