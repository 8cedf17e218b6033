// Host-side tables of the virtual element computation: quadrature rules
// (Gauss-Jacobi rules by the Golub-Welsch method, collapsed to triangles and
// tetrahedra), the edge nodes and their Lagrange basis, the local topology
// of a hexahedron and the positions of the D4 pairs.
#pragma once
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "vem_elem.h"

namespace vb {
namespace vem {

struct HostTables {
  std::vector<double> ta, tb, tet, eg, lg, enode;
  std::vector<int> edges, faces, d4pos;
};

// Eigen-decomposition of a small symmetric matrix (cyclic Jacobi rotations):
// A (n x n, row-major) -> eigenvalues in A's diagonal, eigenvectors in the
// columns of V.
inline void sym_eig(std::vector<double> &A, std::vector<double> &V, int n) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
    if (off < 1e-34) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- J^T A J
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// n-point Gauss rule on [0, 1] for the weight x^beta (beta >= 0): the
// Jacobi polynomials for the weight (1 + t)^beta on [-1, 1] (alpha = 0),
// nodes = eigenvalues of their Jacobi matrix, weights = mu_0 times the
// squared first eigenvector components, then mapped (x = (t + 1)/2, w / 2^(beta+1)).
inline void jacobi01(int n, double beta, std::vector<double> &x, std::vector<double> &w) {
  const double al = 0.0, be = beta;
  std::vector<double> J((size_t)n * n, 0.0), V;
  for (int k = 0; k < n; ++k) {
    const double s = 2.0 * k + al + be;
    J[(size_t)k * n + k] = (k == 0) ? (be - al) / (al + be + 2.0) : (be * be - al * al) / (s * (s + 2.0));
    if (k + 1 < n) {
      const double k1 = k + 1.0, s1 = 2.0 * k1 + al + be;
      const double b2 = 4.0 * k1 * (k1 + al) * (k1 + be) * (k1 + al + be) / (s1 * s1 * (s1 + 1.0) * (s1 - 1.0));
      J[(size_t)k * n + k + 1] = J[(size_t)(k + 1) * n + k] = std::sqrt(b2);
    }
  }
  sym_eig(J, V, n);
  const double mu0 = std::pow(2.0, be + 1.0) / (be + 1.0);
  std::vector<std::pair<double, double>> r;
  for (int k = 0; k < n; ++k) r.push_back({J[(size_t)k * n + k], mu0 * V[k] * V[k]});
  std::sort(r.begin(), r.end());
  x.resize(n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    x[k] = 0.5 * (r[k].first + 1.0);
    w[k] = r[k].second / std::pow(2.0, be + 1.0);
  }
}

// Triangle rule exact to degree d: collapsed coordinates (u with weight u,
// v plain), barycentric (1 - u, u (1 - v), u v), weights summing to 1.
inline void triangle_rule(int d, std::vector<double> &out) {
  const int n = std::max(1, (d + 2) / 2);
  std::vector<double> u, wu, v, wv;
  jacobi01(n, 1.0, u, wu);
  jacobi01(n, 0.0, v, wv);
  out.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      out.push_back(1.0 - u[i]);
      out.push_back(u[i] * (1.0 - v[j]));
      out.push_back(u[i] * v[j]);
      out.push_back(2.0 * wu[i] * wv[j]);
    }
}

// Tetrahedron rule exact to degree d: collapsed (u weight u^2, v weight v,
// w plain), barycentric (1-u, u(1-v), uv(1-w), uvw), weights summing to 1.
inline void tet_rule(int d, std::vector<double> &out) {
  const int n = std::max(1, (d + 2) / 2);
  std::vector<double> u, wu, v, wv, s, ws;
  jacobi01(n, 2.0, u, wu);
  jacobi01(n, 1.0, v, wv);
  jacobi01(n, 0.0, s, ws);
  out.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        out.push_back(1.0 - u[i]);
        out.push_back(u[i] * (1.0 - v[j]));
        out.push_back(u[i] * v[j] * (1.0 - s[k]));
        out.push_back(u[i] * v[j] * s[k]);
        out.push_back(6.0 * wu[i] * wv[j] * ws[k]);
      }
}

inline HostTables make_tables(int K) {
  HostTables T;
  triangle_rule(2 * K + 3, T.ta);
  triangle_rule(2 * K + 1, T.tb);
  tet_rule(2 * K + 1, T.tet);
  std::vector<double> s, w;
  jacobi01(K + 1, 0.0, s, w);
  for (int q = 0; q <= K; ++q) {
    T.eg.push_back(s[q]);
    T.eg.push_back(w[q]);
  }
  // edge nodes: 0, the K - 1 interior Gauss-Lobatto points (roots of P_K'
  // on [-1, 1], mapped), 1
  T.enode.push_back(0.0);
  if (K == 2) T.enode.push_back(0.5);
  if (K == 3) {
    T.enode.push_back(0.5 * (1.0 - 1.0 / std::sqrt(5.0)));
    T.enode.push_back(0.5 * (1.0 + 1.0 / std::sqrt(5.0)));
  }
  if (K == 4) {
    T.enode.push_back(0.5 * (1.0 - std::sqrt(3.0 / 7.0)));
    T.enode.push_back(0.5);
    T.enode.push_back(0.5 * (1.0 + std::sqrt(3.0 / 7.0)));
  }
  T.enode.push_back(1.0);
  for (int q = 0; q <= K; ++q)
    for (int i = 0; i <= K; ++i) {
      double l = 1.0;
      for (int j = 0; j <= K; ++j)
        if (j != i) l *= (s[q] - T.enode[j]) / (T.enode[i] - T.enode[j]);
      T.lg.push_back(l);
    }
  // local edges: axis a, other axes b < c, offsets (o1 on b, o2 on c) with
  // o2 outer, o1 inner
  auto lv = [](const int v[3]) { return v[0] + 2 * v[1] + 4 * v[2]; };
  struct E {
    int a, v0, v1, st[3];
  };
  std::vector<E> edges;
  for (int a = 0; a < 3; ++a) {
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    for (int o2 = 0; o2 < 2; ++o2)
      for (int o1 = 0; o1 < 2; ++o1) {
        int st[3] = {0, 0, 0};
        st[b] = o1;
        st[c] = o2;
        int en[3] = {st[0], st[1], st[2]};
        en[a] = 1;
        edges.push_back({a, lv(st), lv(en), {st[0], st[1], st[2]}});
      }
  }
  for (const E &e : edges) {
    T.edges.push_back(e.a);
    T.edges.push_back(e.v0);
    T.edges.push_back(e.v1);
  }
  // local faces 2a + side: vertices (o1, o2) in (0,0), (1,0), (1,1), (0,1)
  // of (b, c); edges of other axes whose start lies on the face
  const int off[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
  for (int a = 0; a < 3; ++a) {
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    for (int sd = 0; sd < 2; ++sd) {
      T.faces.push_back(a);
      T.faces.push_back(sd);
      for (int q = 0; q < 4; ++q) {
        int v[3] = {0, 0, 0};
        v[a] = sd;
        v[b] = off[q][0];
        v[c] = off[q][1];
        T.faces.push_back(lv(v));
      }
      for (int le = 0; le < 12; ++le)
        if (edges[le].a != a && edges[le].st[a] == sd) T.faces.push_back(le);
    }
  }
  // D4 pairs (c, g), |g| <= K-3, without (c = z, g_z >= 1)
  const int ng = K >= 3 ? (K - 2) * (K - 1) * K / 6 : 0;
  T.d4pos.assign(3 * std::max(ng, 1), -1);
  int p = 0;
  for (int c = 0; c < 3; ++c)
    for (int g = 0; g < ng; ++g) {
      int ea, eb, ec;
      exp3(g, ea, eb, ec);
      if (c == 2 && ec >= 1) continue;
      T.d4pos[c * ng + g] = p++;
    }
  return T;
}

}  // namespace vem
}  // namespace vb
