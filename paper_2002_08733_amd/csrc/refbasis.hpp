// refbasis.hpp -- reference-element basis and quadrature of libmdg (host code).
//
// Reference tetrahedron T^ = {x,y,z >= 0, x+y+z <= 1} with vertices
// v0=(0,0,0), v1=(1,0,0), v2=(0,1,0), v3=(0,0,1) [KS Sec. II].
//
// Volume basis: orthonormal Dubiner functions [KS Sec. II, eq. dubiner_functions]
// in the corrected form (the printed middle factor lacks (1-x)^j and the last
// Jacobi weight must be (2i+2j+2,0) for orthogonality):
//   phi_ijk = sqrt((2i+1)(2i+2j+2)(2i+2j+2k+3))
//             Q_i^(0,0)(2z-(1-x-y), 1-x-y) Q_j^(2i+1,0)(2y-(1-x), 1-x) P_k^(2i+2j+2,0)(2x-1)
// where Q_n^(a,b)(u,w) = w^n P_n^(a,b)(u/w) is the homogeneous Jacobi polynomial,
// evaluated by the homogenised three-term recurrence (no division by w, so the
// collapsed-coordinate singularities never appear). Mode order: total degree
// d = i+j+k ascending, then i ascending, then j ascending.
//
// Face basis (library-internal choice; both elements of a face use it on the
// same parametrisation): orthonormal on the parameter triangle
// {s1,s2 >= 0, s1+s2 <= 1} with measure ds1 ds2,
//   psi_ij(s1,s2) = sqrt(2(2i+1)(i+j+1)) Q_i^(0,0)(2 s2-(1-s1), 1-s1) P_j^(2i+1,0)(2 s1-1),
// ordered by d = i+j ascending then i ascending.
//
// Quadrature: tensor Gauss-Legendre rules on [0,1]^k pushed through the
// collapse (Duffy) maps, with the Jacobians (1-a)^2 (1-b) and (1-a) carried in
// the weights.
#pragma once

#include <cmath>
#include <vector>

namespace mdg {

inline int nmodes3(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
inline int nmodes2(int p) { return (p + 1) * (p + 2) / 2; }

struct Mode3 { int i, j, k; };
struct Mode2 { int i, j; };

inline std::vector<Mode3> modes3(int p) {
  std::vector<Mode3> m;
  for (int d = 0; d <= p; ++d)
    for (int i = 0; i <= d; ++i)
      for (int j = 0; j <= d - i; ++j) m.push_back({i, j, d - i - j});
  return m;
}

inline std::vector<Mode2> modes2(int p) {
  std::vector<Mode2> m;
  for (int d = 0; d <= p; ++d)
    for (int i = 0; i <= d; ++i) m.push_back({i, d - i});
  return m;
}

// Homogeneous Jacobi Q_n^(a,0)(u,w) = w^n P_n^(a,0)(u/w) for n = 0..nmax, with
// gradients: du, dw are the (constant) gradients of u and w w.r.t. the point.
template <typename T>
void hjacobi(int nmax, T a, T u, T w, const T du[3], const T dw[3], T* Q, T (*dQ)[3]) {
  Q[0] = 1;
  if (dQ) dQ[0][0] = dQ[0][1] = dQ[0][2] = 0;
  if (nmax == 0) return;
  // P_1^(a,0)(x) = (a + (a+2) x)/2  ->  Q_1 = (a w + (a+2) u)/2
  Q[1] = (a * w + (a + 2) * u) / 2;
  if (dQ)
    for (int c = 0; c < 3; ++c) dQ[1][c] = (a * dw[c] + (a + 2) * du[c]) / 2;
  for (int n = 2; n <= nmax; ++n) {
    const T c2 = 2 * n + a;  // 2n + a + b with b = 0
    const T c0 = 2 * n * (n + a) * (c2 - 2);
    const T ca = (c2 - 1) * c2 * (c2 - 2);
    const T cb = (c2 - 1) * a * a;
    const T c3 = 2 * (n + a - 1) * (n - 1) * c2;
    const T lin = ca * u + cb * w;
    Q[n] = (lin * Q[n - 1] - c3 * w * w * Q[n - 2]) / c0;
    if (dQ)
      for (int c = 0; c < 3; ++c)
        dQ[n][c] = ((ca * du[c] + cb * dw[c]) * Q[n - 1] + lin * dQ[n - 1][c] -
                    c3 * (2 * w * dw[c] * Q[n - 2] + w * w * dQ[n - 2][c])) /
                   c0;
  }
}

// Values (and optionally reference gradients) of all N modes at (x,y,z).
template <typename T>
void dubiner3(int p, T x, T y, T z, T* val, T (*grad)[3]) {
  const int N = nmodes3(p);
  std::vector<Mode3> md = modes3(p);
  // factor 1: Q_i^(0,0)(2z - (1-x-y), 1-x-y)
  const T u1 = 2 * z - (1 - x - y), w1 = 1 - x - y;
  const T du1[3] = {1, 1, 2}, dw1[3] = {-1, -1, 0};
  std::vector<T> F1(p + 1);
  std::vector<T> dF1v(3 * (p + 1));
  T(*dF1)[3] = reinterpret_cast<T(*)[3]>(dF1v.data());
  hjacobi<T>(p, 0, u1, w1, du1, dw1, F1.data(), grad ? dF1 : nullptr);
  for (int m = 0; m < N; ++m) {
    const int i = md[m].i, j = md[m].j, k = md[m].k;
    // factor 2: Q_j^(2i+1,0)(2y - (1-x), 1-x)
    std::vector<T> F2(j + 1), dF2v(3 * (j + 1));
    T(*dF2)[3] = reinterpret_cast<T(*)[3]>(dF2v.data());
    const T u2 = 2 * y - (1 - x), w2 = 1 - x;
    const T du2[3] = {1, 2, 0}, dw2[3] = {-1, 0, 0};
    hjacobi<T>(j, T(2 * i + 1), u2, w2, du2, dw2, F2.data(), grad ? dF2 : nullptr);
    // factor 3: P_k^(2i+2j+2,0)(2x-1) = Q_k(2x-1, 1)
    std::vector<T> F3(k + 1), dF3v(3 * (k + 1));
    T(*dF3)[3] = reinterpret_cast<T(*)[3]>(dF3v.data());
    const T u3 = 2 * x - 1, w3 = 1;
    const T du3[3] = {2, 0, 0}, dw3[3] = {0, 0, 0};
    hjacobi<T>(k, T(2 * i + 2 * j + 2), u3, w3, du3, dw3, F3.data(), grad ? dF3 : nullptr);
    const T nrm = std::sqrt(T((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3)));
    val[m] = nrm * F1[i] * F2[j] * F3[k];
    if (grad)
      for (int c = 0; c < 3; ++c)
        grad[m][c] = nrm * (dF1[i][c] * F2[j] * F3[k] + F1[i] * dF2[j][c] * F3[k] +
                            F1[i] * F2[j] * dF3[k][c]);
  }
}

// Face basis values at parameter point (s1, s2).
template <typename T>
void dubiner2(int p, T s1, T s2, T* val) {
  std::vector<Mode2> md = modes2(p);
  const T z3[3] = {0, 0, 0};
  std::vector<T> F1(p + 1);
  hjacobi<T>(p, 0, 2 * s2 - (1 - s1), 1 - s1, z3, z3, F1.data(), nullptr);
  for (size_t m = 0; m < md.size(); ++m) {
    const int i = md[m].i, j = md[m].j;
    std::vector<T> F2(j + 1);
    hjacobi<T>(j, T(2 * i + 1), 2 * s1 - 1, T(1), z3, z3, F2.data(), nullptr);
    val[m] = std::sqrt(T(2 * (2 * i + 1) * (i + j + 1))) * F1[i] * F2[j];
  }
}

// Gauss-Legendre rule on [0,1] with n points (Newton on P_n).
template <typename T>
void gauss_legendre01(int n, std::vector<T>& x, std::vector<T>& w) {
  x.resize(n);
  w.resize(n);
  const T pi = T(3.141592653589793238462643383279502884L);
  for (int i = 0; i < n; ++i) {
    T z = std::cos(pi * (i + T(0.75)) / (n + T(0.5)));
    T dp = 0;
    for (int it = 0; it < 100; ++it) {
      T p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        T p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      T dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < T(1e-30L) * (1 + std::fabs(z))) break;
    }
    // recompute derivative at the converged node
    {
      T p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        T p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
    }
    x[i] = (1 - z) / 2;  // map [-1,1] -> [0,1]
    w[i] = 1 / ((1 - z * z) * dp * dp);  // (2/((1-z^2)P'^2)) / 2
  }
}

// Collapsed tensor rule on the reference tet: q^3 points, exact for total
// degree <= 2q - 3.
template <typename T>
void tet_rule(int q, std::vector<T>& pts, std::vector<T>& w) {
  std::vector<T> g, gw;
  gauss_legendre01<T>(q, g, gw);
  pts.clear();
  w.clear();
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b)
      for (int c = 0; c < q; ++c) {
        const T x = g[a], y = g[b] * (1 - x), z = g[c] * (1 - x - y);
        pts.push_back(x);
        pts.push_back(y);
        pts.push_back(z);
        w.push_back(gw[a] * gw[b] * gw[c] * (1 - g[a]) * (1 - g[a]) * (1 - g[b]));
      }
}

// Collapsed rule on the parameter triangle: q^2 points, exact for degree <= 2q-2.
template <typename T>
void tri_rule(int q, std::vector<T>& pts, std::vector<T>& w) {
  std::vector<T> g, gw;
  gauss_legendre01<T>(q, g, gw);
  pts.clear();
  w.clear();
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      const T s1 = g[a], s2 = g[b] * (1 - s1);
      pts.push_back(s1);
      pts.push_back(s2);
      w.push_back(gw[a] * gw[b] * (1 - g[a]));
    }
}

// Reference vertices and the face parametrisation F^_f(s) = va + s1 (vb - va) + s2 (vc - va)
// of local face f (opposite local vertex f, face vertices ascending a < b < c).
inline void ref_vertex(int v, double out[3]) {
  out[0] = (v == 1);
  out[1] = (v == 2);
  out[2] = (v == 3);
}
inline void face_vertices(int f, int fv[3]) {
  int n = 0;
  for (int v = 0; v < 4; ++v)
    if (v != f) fv[n++] = v;
}

}  // namespace mdg
