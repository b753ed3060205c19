// GPU finite-element assembly of the Taylor-Hood P2/P1 operators (paper Sec.
// 2.2: M_V, B, M_Q; Sec. 3.2: the vector Laplacian L_V; Sec. 4.1: L_Q and the
// lumped Lambda_V), and the build of the sliced-ELL operators used inside the
// Krylov iterations.
//
// Element integrals use reference tables computed once on the host with the
// Grundmann-Moller degree-5 rule on the simplex (Grundmann & Moller, SIAM J.
// Numer. Anal. 15, 1978), which is exact for the degree-4 integrands here.
// Geometry enters through |K| and J^{-1} (x = x_0 + J xi):
//     M_ij  = |K| Mref_ij
//     L_ij  = |K| sum_pq (J^{-1} J^{-T})_pq Sref_ipjq
//     B^c_ki = |K| sum_p (J^{-1})_pc Wref_kip
// Assembly is deterministic and atomic-free: one thread owns each matrix row,
// walks the simplices incident to its node in a fixed order and adds each
// element row into its sorted CSR slots.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <functional>
#include <numeric>
#include <thread>
#include <tuple>

#include "common.h"
#include "kernels.h"
#include "ops.h"

namespace stokes {

namespace {

// reference tables of the P2/P1 pair, [2] = 2D, [3] = 3D (index by dim)
__constant__ double c_Mref3[100], c_Sref3[900], c_Wref3[120], c_M1ref3[16], c_abs3[10];
__constant__ double c_Mref2[36], c_Sref2[144], c_Wref2[36], c_M1ref2[9], c_abs2[6];
// ... and of the P3/P2 pair (velocity P3: 20 / 10 local nodes, pressure P2:
// 10 / 6; W is pressure x velocity x dim)
__constant__ double c_Mref3c[400], c_Sref3c[3600], c_Wref3c[600], c_abs3c[20];
__constant__ double c_Mref2c[100], c_Sref2c[400], c_Wref2c[120], c_abs2c[10];

struct RefTables {
  std::vector<double> M, S, W, M1, absphi;
  double mass_lo = 0, mass_hi = 0, p1_lo = 0, p1_hi = 0;
};

// Grundmann-Moller rule of degree 2s+1 on the d-simplex (volume 1/d!), points in
// barycentric coordinates.
void gm_rule(int d, int s, std::vector<std::vector<double>>& pts, std::vector<double>& wts) {
  const int deg = 2 * s + 1;
  auto fact = [](int k) {
    double f = 1;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
  };
  for (int i = 0; i <= s; ++i) {
    const double w = ((i % 2) ? -1.0 : 1.0) * std::pow(2.0, -2 * s) * std::pow(double(deg + d - 2 * i), deg) /
                     (fact(i) * fact(deg + d - i));
    const int tot = s - i;
    std::vector<int> beta(d + 1, 0);
    // enumerate compositions of tot into d+1 parts
    std::function<void(int, int)> rec = [&](int pos, int left) {
      if (pos == d) {
        beta[d] = left;
        std::vector<double> lam(d + 1);
        for (int j = 0; j <= d; ++j) lam[j] = (2.0 * beta[j] + 1.0) / double(deg + d - 2 * i);
        pts.push_back(lam);
        wts.push_back(w);
        return;
      }
      for (int b = 0; b <= left; ++b) {
        beta[pos] = b;
        rec(pos + 1, left - b);
      }
    };
    rec(0, tot);
  }
}

// Symmetric Jacobi eigenvalue sweep (small dense matrices, host).
void sym_eig_extremes(std::vector<double> A, int n, double& lo, double& hi) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = 0.5 * (A[q * n + q] - A[p * n + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  lo = hi = A[0];
  for (int i = 1; i < n; ++i) {
    lo = std::min(lo, A[i * n + i]);
    hi = std::max(hi, A[i * n + i]);
  }
}

// Local velocity basis of a simplex at barycentric point L: values phi[i]
// and gradients g[i * d + p] with respect to the reference coordinates xi_p
// (lambda_0 = 1 - sum xi, lambda_a = xi_{a-1}).  Order 2: vertex
// lambda_a (2 lambda_a - 1), edge 4 lambda_a lambda_b.  Order 3: vertex
// lambda_a (3 lambda_a - 1)(3 lambda_a - 2) / 2; per local edge (a, b) the
// node next to a, 9/2 lambda_a lambda_b (3 lambda_a - 1), then the node next
// to b; then the face (2D: interior) nodes 27 lambda_a lambda_b lambda_c of
// the faces (0,1,2), (0,1,3), (0,2,3), (1,2,3).
void local_basis(int d, int order, const std::vector<double>& L, std::vector<double>& phi, std::vector<double>& g) {
  const int nv = d + 1;
  auto dlam = [&](int a, int p) { return a == 0 ? -1.0 : (a - 1 == p ? 1.0 : 0.0); };
  std::vector<std::pair<int, int>> edges;
  for (int a = 0; a < nv; ++a)
    for (int b = a + 1; b < nv; ++b) edges.emplace_back(a, b);
  phi.clear();
  g.clear();
  auto push = [&](double v, const double* gr) {
    phi.push_back(v);
    for (int p = 0; p < d; ++p) g.push_back(gr[p]);
  };
  double gr[3];
  if (order == 2) {
    for (int a = 0; a < nv; ++a) {
      for (int p = 0; p < d; ++p) gr[p] = (4.0 * L[a] - 1.0) * dlam(a, p);
      push(L[a] * (2.0 * L[a] - 1.0), gr);
    }
    for (auto [a, b] : edges) {
      for (int p = 0; p < d; ++p) gr[p] = 4.0 * (dlam(a, p) * L[b] + L[a] * dlam(b, p));
      push(4.0 * L[a] * L[b], gr);
    }
    return;
  }
  for (int a = 0; a < nv; ++a) {
    const double t = L[a];
    // d/dt [t (3t - 1)(3t - 2) / 2] = (27 t^2 - 18 t + 2) / 2
    for (int p = 0; p < d; ++p) gr[p] = 0.5 * (27.0 * t * t - 18.0 * t + 2.0) * dlam(a, p);
    push(0.5 * t * (3.0 * t - 1.0) * (3.0 * t - 2.0), gr);
  }
  for (auto [a0, b0] : edges)
    for (int side = 0; side < 2; ++side) {
      const int a = side == 0 ? a0 : b0, b = side == 0 ? b0 : a0;  // a: the near vertex
      // 9/2 (3 la^2 lb - la lb): d/dla = 9/2 (6 la lb - lb), d/dlb = 9/2 (3 la^2 - la)
      const double da = 4.5 * (6.0 * L[a] * L[b] - L[b]), db = 4.5 * (3.0 * L[a] * L[a] - L[a]);
      for (int p = 0; p < d; ++p) gr[p] = da * dlam(a, p) + db * dlam(b, p);
      push(4.5 * L[a] * L[b] * (3.0 * L[a] - 1.0), gr);
    }
  static const int faces3[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  const int nf = d == 3 ? 4 : 1;
  for (int f = 0; f < nf; ++f) {
    const int a = faces3[f][0], b = faces3[f][1], c = faces3[f][2];
    for (int p = 0; p < d; ++p)
      gr[p] = 27.0 * (dlam(a, p) * L[b] * L[c] + L[a] * dlam(b, p) * L[c] + L[a] * L[b] * dlam(c, p));
    push(27.0 * L[a] * L[b] * L[c], gr);
  }
}

// Exact rational arithmetic on int64 (the closed forms below have small
// denominators), reduced after every operation.
struct Rat {
  int64_t p = 0, q = 1;
  Rat() = default;
  Rat(int64_t a, int64_t b = 1) : p(a), q(b) { norm(); }
  void norm() {
    if (q < 0) {
      p = -p;
      q = -q;
    }
    int64_t a = p < 0 ? -p : p, b = q;
    while (b) {
      const int64_t t = a % b;
      a = b;
      b = t;
    }
    if (a > 1) {
      p /= a;
      q /= a;
    }
  }
  Rat operator+(const Rat& o) const { return Rat(p * o.q + o.p * q, q * o.q); }
  Rat operator-(const Rat& o) const { return Rat(p * o.q - o.p * q, q * o.q); }
  Rat operator*(const Rat& o) const { return Rat(p * o.p, q * o.q); }
  double value() const { return double(p) / double(q); }
};

// int |phi| / |K| of the P3 basis.  A barycentric coordinate t = lambda_a of
// a point uniform in the d-simplex has the density d (1 - t)^(d-1); given t,
// the other coordinates are uniform on a simplex of total 1 - t, so the mean
// of another coordinate lambda_b is (1 - t) / d.  The vertex function
// t (3t - 1)(3t - 2) / 2 changes sign at t = 1/3 and 2/3, the edge function
// 9/2 lambda_a lambda_b (3 lambda_a - 1) at lambda_a = 1/3; integrating the
// t-polynomials piecewise against the density gives the exact values (here
// in rational arithmetic, rounded once).  Face (interior) functions are
// non-negative: their integral is 27 d! / (d + 3)!.
void p3_abs_values(int d, double& vtx, double& edge, double& face) {
  // integral over [lo, hi] of poly(t) d (1 - t)^(d - 1), poly as t^k
  // coefficients, with (1 - t)^(d - 1) expanded binomially
  auto integ = [d](const std::vector<Rat>& poly, Rat lo, Rat hi) {
    std::vector<Rat> w(d);
    int64_t binom = 1;
    for (int k = 0; k < d; ++k) {
      w[k] = Rat(d * binom * ((k % 2) ? -1 : 1));
      binom = binom * (d - 1 - k) / (k + 1);
    }
    std::vector<Rat> prod(poly.size() + w.size() - 1);
    for (size_t i = 0; i < poly.size(); ++i)
      for (size_t j = 0; j < w.size(); ++j) prod[i + j] = prod[i + j] + poly[i] * w[j];
    Rat r;
    for (size_t k = 0; k < prod.size(); ++k) {
      Rat hk(1), lk(1);
      for (size_t e = 0; e <= k; ++e) {
        hk = hk * hi;
        lk = lk * lo;
      }
      r = r + prod[k] * (hk - lk) * Rat(1, int64_t(k + 1));
    }
    return r;
  };
  const Rat t0(0), t1(1, 3), t2(2, 3), t3(1);
  const std::vector<Rat> gv = {Rat(0), Rat(1), Rat(-9, 2), Rat(9, 2)};  // t (3t - 1)(3t - 2) / 2
  vtx = (integ(gv, t0, t1) - integ(gv, t1, t2) + integ(gv, t2, t3)).value();
  // 9/2 t (3t - 1) (1 - t) / d = 9/(2d) (-t + 4 t^2 - 3 t^3)
  const Rat k(9, 2 * d);
  const std::vector<Rat> ge = {Rat(0), Rat(0) - k, Rat(4) * k, Rat(-3) * k};
  edge = (integ(ge, t1, t3) - integ(ge, t0, t1)).value();
  int64_t num = 27, den = 1;
  for (int i = 1; i <= d; ++i) num *= i;
  for (int i = 1; i <= d + 3; ++i) den *= i;
  face = Rat(num, den).value();
}

// Reference integrals of the velocity basis of `order` against itself and
// against the pressure basis (order 2: the P1 lambdas; order 3: the P2
// basis): M, S (gradient products in reference coordinates), W (pressure x
// velocity gradient), M1 (pressure mass, order 2 only), int |phi|, and the
// element bounds of the Jacobi-scaled velocity and pressure masses.
RefTables make_tables(int d, int order = 2) {
  RefTables t;
  const int nv = d + 1;
  const int nl = order == 3 ? (d == 3 ? 20 : 10) : (d == 3 ? 10 : 6);
  const int nq = order == 3 ? (d == 3 ? 10 : 6) : nv;
  std::vector<std::vector<double>> pts;
  std::vector<double> wts;
  gm_rule(d, order == 3 ? 3 : 2, pts, wts);  // degree 7 / 5: exact for the products here
  double volref = 1.0;
  for (int i = 2; i <= d; ++i) volref /= i;
  t.M.assign(nl * nl, 0);
  t.S.assign(nl * d * nl * d, 0);
  t.W.assign(nq * nl * d, 0);
  t.M1.assign(nq * nq, 0);
  std::vector<double> phi, g, qphi, qg;
  for (size_t q = 0; q < pts.size(); ++q) {
    const auto& L = pts[q];
    const double w = wts[q] / volref;
    local_basis(d, order, L, phi, g);
    if (order == 3) local_basis(d, 2, L, qphi, qg);
    else qphi.assign(L.begin(), L.end());
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < nl; ++j) {
        t.M[i * nl + j] += w * phi[i] * phi[j];
        for (int p = 0; p < d; ++p)
          for (int r = 0; r < d; ++r) t.S[((i * d + p) * nl + j) * d + r] += w * g[i * d + p] * g[j * d + r];
      }
    for (int k = 0; k < nq; ++k)
      for (int i = 0; i < nl; ++i)
        for (int p = 0; p < d; ++p) t.W[(k * nl + i) * d + p] += w * qphi[k] * g[i * d + p];
    for (int a = 0; a < nq; ++a)
      for (int b = 0; b < nq; ++b) t.M1[a * nq + b] += w * qphi[a] * qphi[b];
  }
  t.absphi.assign(nl, 0);
  if (order == 2) {
    // int |phi| / |K|: the vertex function lambda(2 lambda - 1) changes sign at
    // lambda = 1/2; integrating against the density d (1 - t)^(d-1) of one
    // barycentric coordinate on each side gives 3/32 (3D) and 1/8 (2D).  Edge
    // functions are non-negative, so their value is int phi = 1/5 (3D), 1/3 (2D).
    for (int i = 0; i < nl; ++i) t.absphi[i] = i < nv ? (d == 3 ? 3.0 / 32.0 : 1.0 / 8.0) : (d == 3 ? 0.2 : 1.0 / 3.0);
  } else {
    double av, ae, af;
    p3_abs_values(d, av, ae, af);
    const int ned = d == 3 ? 6 : 3;
    for (int i = 0; i < nl; ++i) t.absphi[i] = i < nv ? av : (i < nv + 2 * ned ? ae : af);
  }
  // Element bounds of the Jacobi-scaled mass matrices (shape independent on
  // affine simplices): eigenvalues of D^{-1/2} Mref D^{-1/2}.
  auto scaled = [](const std::vector<double>& A, int n) {
    std::vector<double> B(A);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) B[i * n + j] = A[i * n + j] / std::sqrt(A[i * n + i] * A[j * n + j]);
    return B;
  };
  sym_eig_extremes(scaled(t.M, nl), nl, t.mass_lo, t.mass_hi);
  sym_eig_extremes(scaled(t.M1, nq), nq, t.p1_lo, t.p1_hi);
  return t;
}

RefTables g_tab2, g_tab3, g_tab2c, g_tab3c;  // P2/P1 and P3/P2

void upload_tables() {
  static bool done = false;
  if (done) return;
  g_tab2 = make_tables(2);
  g_tab3 = make_tables(3);
  g_tab2c = make_tables(2, 3);
  g_tab3c = make_tables(3, 3);
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Mref3c), g_tab3c.M.data(), 400 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Sref3c), g_tab3c.S.data(), 3600 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Wref3c), g_tab3c.W.data(), 600 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_abs3c), g_tab3c.absphi.data(), 20 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Mref2c), g_tab2c.M.data(), 100 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Sref2c), g_tab2c.S.data(), 400 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Wref2c), g_tab2c.W.data(), 120 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_abs2c), g_tab2c.absphi.data(), 10 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Mref3), g_tab3.M.data(), 100 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Sref3), g_tab3.S.data(), 900 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Wref3), g_tab3.W.data(), 120 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_M1ref3), g_tab3.M1.data(), 16 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_abs3), g_tab3.absphi.data(), 10 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Mref2), g_tab2.M.data(), 36 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Sref2), g_tab2.S.data(), 144 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_Wref2), g_tab2.W.data(), 36 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_M1ref2), g_tab2.M1.data(), 9 * sizeof(double)));
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_abs2), g_tab2.absphi.data(), 6 * sizeof(double)));
  done = true;
}

// Reference tables of the velocity basis of order P (2 or 3) on the
// D-simplex: NL velocity nodes, NQ pressure nodes (P1 for P = 2, P2 for 3).
template <int D, int P = 2>
struct Tab {
  static constexpr int NL = P == 3 ? (D == 3 ? 20 : 10) : (D == 3 ? 10 : 6);
  static constexpr int NV = D + 1;
  static constexpr int NQ = P == 3 ? (D == 3 ? 10 : 6) : NV;
  __device__ static double M(int i, int j) {
    if (P == 3) return D == 3 ? c_Mref3c[i * NL + j] : c_Mref2c[i * NL + j];
    return D == 3 ? c_Mref3[i * NL + j] : c_Mref2[i * NL + j];
  }
  __device__ static double S(int i, int p, int j, int r) {
    const int k = ((i * D + p) * NL + j) * D + r;
    if (P == 3) return D == 3 ? c_Sref3c[k] : c_Sref2c[k];
    return D == 3 ? c_Sref3[k] : c_Sref2[k];
  }
  __device__ static double W(int k, int i, int p) {
    const int o = (k * NL + i) * D + p;
    if (P == 3) return D == 3 ? c_Wref3c[o] : c_Wref2c[o];
    return D == 3 ? c_Wref3[o] : c_Wref2[o];
  }
  __device__ static double M1(int a, int b) { return D == 3 ? c_M1ref3[a * NV + b] : c_M1ref2[a * NV + b]; }
  __device__ static double absphi(int i) {
    if (P == 3) return D == 3 ? c_abs3c[i] : c_abs2c[i];
    return D == 3 ? c_abs3[i] : c_abs2[i];
  }
};

// |K| and J^{-1} (stored [p][c]) of every simplex
template <int D>
__global__ __launch_bounds__(kBlock) void k_geom(int64_t n_e, const double* __restrict__ vc,
                                                 const int32_t* __restrict__ el, double* __restrict__ vol,
                                                 double* __restrict__ jinv) {
  GRID_STRIDE_ROWS(e, n_e) {
    double X[D + 1][D];
    for (int a = 0; a <= D; ++a)
      for (int c = 0; c < D; ++c) X[a][c] = vc[(int64_t)el[e * (D + 1) + a] * D + c];
    double J[D][D];  // J[c][p] = X[p+1][c] - X[0][c]
    for (int c = 0; c < D; ++c)
      for (int p = 0; p < D; ++p) J[c][p] = X[p + 1][c] - X[0][c];
    double det, inv[D][D];
    if (D == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      inv[0][0] = J[1][1] / det;
      inv[0][1] = -J[0][1] / det;
      inv[1][0] = -J[1][0] / det;
      inv[1][1] = J[0][0] / det;
    } else {
      const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      // inverse = adj(J) / det, adj = cofactor^T
      inv[0][0] = c00 / det;
      inv[1][0] = c01 / det;
      inv[2][0] = c02 / det;
      inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    vol[e] = fabs(det) / (D == 3 ? 6.0 : 2.0);
    for (int p = 0; p < D; ++p)
      for (int c = 0; c < D; ++c) jinv[e * D * D + p * D + c] = inv[p][c];
  }
}

__device__ __forceinline__ int64_t find_slot(const int32_t* __restrict__ cols, int64_t lo, int64_t hi, int32_t c) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (cols[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// rows of M_s and L_s over all velocity nodes (basis of order P; with P = 2
// also the P2 pressure mass and Laplacian of the P3/P2 pair)
template <int D, int P = 2>
__global__ __launch_bounds__(kBlock) void k_gather_p2(int64_t n_p2, const int64_t* __restrict__ iptr,
                                                      const int32_t* __restrict__ ilist,
                                                      const int32_t* __restrict__ p2, const double* __restrict__ vol,
                                                      const double* __restrict__ jinv, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ cols, double* __restrict__ Mo,
                                                      double* __restrict__ Lo, double* __restrict__ Do) {
  using Tb = Tab<D, P>;
  GRID_STRIDE_ROWS(v, n_p2) {
    const int64_t lo = rp[v], hi = rp[v + 1];
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k) {
      const int64_t e = ilist[k] >> kLocBits;
      const int i = ilist[k] & kLocMask;
      const double V = vol[e];
      double K[D][D];
      for (int p = 0; p < D; ++p)
        for (int r = 0; r < D; ++r) {
          double s = 0;
          for (int c = 0; c < D; ++c) s += jinv[e * D * D + p * D + c] * jinv[e * D * D + r * D + c];
          K[p][r] = s;
        }
      for (int j = 0; j < Tb::NL; ++j) {
        double l = 0;
        for (int p = 0; p < D; ++p)
          for (int r = 0; r < D; ++r) l += K[p][r] * Tb::S(i, p, j, r);
        const int64_t slot = find_slot(cols, lo, hi, p2[e * Tb::NL + j]);
        Mo[slot] += V * Tb::M(i, j);
        Lo[slot] += V * l;
        if (Do) {
          // grad-div blocks: int d_a phi_i d_b phi_j, d_a phi = sum_p Jinv[p][a] d phi / d xi_p
          for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
              double t = 0;
              for (int p = 0; p < D; ++p)
                for (int r = 0; r < D; ++r)
                  t += jinv[e * D * D + p * D + a] * jinv[e * D * D + r * D + b] * Tb::S(i, p, j, r);
              Do[slot * D * D + a * D + b] += V * t;
            }
        }
      }
    }
  }
}

// rows of B (one per pressure node, D planes) over all velocity columns
template <int D, int P = 2>
__global__ __launch_bounds__(kBlock) void k_gather_b(int64_t n_p1, const int64_t* __restrict__ iptr,
                                                     const int32_t* __restrict__ ilist,
                                                     const int32_t* __restrict__ p2, const double* __restrict__ vol,
                                                     const double* __restrict__ jinv, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ cols, double* __restrict__ Bo) {
  using Tb = Tab<D, P>;
  GRID_STRIDE_ROWS(v, n_p1) {
    const int64_t lo = rp[v], hi = rp[v + 1];
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k) {
      const int64_t e = ilist[k] >> kLocBits;
      const int a = ilist[k] & kLocMask;
      const double V = vol[e];
      for (int j = 0; j < Tb::NL; ++j) {
        const int64_t slot = find_slot(cols, lo, hi, p2[e * Tb::NL + j]);
        for (int c = 0; c < D; ++c) {
          double s = 0;
          for (int p = 0; p < D; ++p) s += jinv[e * D * D + p * D + c] * Tb::W(a, j, p);
          Bo[slot * D + c] += V * s;
        }
      }
    }
  }
}

// Strain-form velocity blocks on the SELL entries of the interior operator:
//   V[a][b] = delta_ab (alpha M + mu L)[s] + mu D[s][a][b],  s = src[k].
// Between interior nodes D[a][b] = D[b][a] (integration by parts on H^1_0),
// so each block is symmetric and its dim (dim + 1) / 2 upper entries
// (a <= b, row-major) are stored, D[a][b] taken as the mean of the two
// assembled values.  Layout: plane e of entry k at (k - k mod 64) P + 64 e +
// k mod 64 (P planes), so the lanes of a wavefront read each plane
// contiguously.
__global__ __launch_bounds__(kBlock) void k_fill_blk(int64_t n, int dd, const int32_t* __restrict__ src, double alpha,
                                                     double mu, const double* __restrict__ M,
                                                     const double* __restrict__ L, const double* __restrict__ Dg,
                                                     double* __restrict__ out, float* __restrict__ out32) {
  const int P = dd * (dd + 1) / 2;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = src[k];
    const int64_t base = (k - (k & 63)) * P + (k & 63);
    int e = 0;
    for (int a = 0; a < dd; ++a)
      for (int b = a; b < dd; ++b, ++e) {
        double o = 0;
        if (s >= 0) {
          o = 0.5 * mu * (Dg[s * dd * dd + a * dd + b] + Dg[s * dd * dd + b * dd + a]);
          if (a == b) o += alpha * M[s] + mu * L[s];
        }
        out[base + 64 * e] = o;
        out32[base + 64 * e] = (float)o;
      }
  }
}

// column-scaled copy: out[k] = vals[k] * dinv[cols[k]] over the SELL entries
__global__ __launch_bounds__(kBlock) void k_to_half(int64_t n, const double* __restrict__ x, double s,
                                                    _Float16* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (_Float16)(x[i] * s);
}

__global__ __launch_bounds__(kBlock) void k_scale_cols(int64_t n, const int32_t* __restrict__ cols,
                                                       const double* __restrict__ vals, const double* __restrict__ dinv,
                                                       double* __restrict__ out, float* __restrict__ out32,
                                                       _Float16* __restrict__ out16) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double v = vals[k] * dinv[cols[k]];
    out[k] = v;
    out32[k] = (float)v;
    out16[k] = (_Float16)v;
  }
}

// rows of X = B_I Lambda_V^-1 B_I^T (lumped-mass pressure operator of Sec. 4.3),
// one wavefront per P1 row k: each lane owns output entries (k, l) and merges
// the sorted B rows k and l, summing over the shared interior P2 columns j
//   X_kl = sum_j sum_c B_c[k, j] B_c[l, j] / Lambda_j
// in increasing j, so the result does not depend on the launch shape.
template <int D>
__global__ __launch_bounds__(kBlock) void k_gather_xl(int64_t n_p1, const int32_t* __restrict__ brp,
                                                      const int32_t* __restrict__ bcols,
                                                      const double* __restrict__ Bv, const double* __restrict__ lam,
                                                      const int32_t* __restrict__ nat2int,
                                                      const int32_t* __restrict__ xrp,
                                                      const int32_t* __restrict__ xcols, double* __restrict__ X) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); k < n_p1; k += waves) {
    for (int64_t q = xrp[k] + lane; q < xrp[k + 1]; q += 64) {
      const int64_t l = xcols[q];
      int64_t ia = brp[k], ib = brp[l];
      const int64_t ea = brp[k + 1], eb = brp[l + 1];
      double s = 0;
      while (ia < ea && ib < eb) {
        const int32_t ja = bcols[ia], jb = bcols[ib];
        if (ja < jb) {
          ++ia;
        } else if (jb < ja) {
          ++ib;
        } else {
          if (nat2int[ja] >= 0) {
            double t = 0;
            for (int c = 0; c < D; ++c) t += Bv[ia * D + c] * Bv[ib * D + c];
            s += t / lam[ja];
          }
          ++ia;
          ++ib;
        }
      }
      X[q] = s;
    }
  }
}

// rows of M_Q and L_Q
template <int D>
__global__ __launch_bounds__(kBlock) void k_gather_q(int64_t n_p1, const int64_t* __restrict__ iptr,
                                                     const int32_t* __restrict__ ilist,
                                                     const int32_t* __restrict__ el, const double* __restrict__ vol,
                                                     const double* __restrict__ jinv, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ cols, double* __restrict__ MQ,
                                                     double* __restrict__ LQ) {
  using Tb = Tab<D>;
  GRID_STRIDE_ROWS(v, n_p1) {
    const int64_t lo = rp[v], hi = rp[v + 1];
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k) {
      const int64_t e = ilist[k] >> kLocBits;
      const int a = ilist[k] & kLocMask;
      const double V = vol[e];
      double ga[D];
      for (int c = 0; c < D; ++c) {  // physical gradient of lambda_a
        double s = 0;
        for (int p = 0; p < D; ++p) s += jinv[e * D * D + p * D + c] * (a == 0 ? -1.0 : (a - 1 == p ? 1.0 : 0.0));
        ga[c] = s;
      }
      for (int b = 0; b <= D; ++b) {
        double l = 0;
        for (int c = 0; c < D; ++c) {
          double s = 0;
          for (int p = 0; p < D; ++p) s += jinv[e * D * D + p * D + c] * (b == 0 ? -1.0 : (b - 1 == p ? 1.0 : 0.0));
          l += ga[c] * s;
        }
        const int64_t slot = find_slot(cols, lo, hi, el[e * (D + 1) + b]);
        MQ[slot] += V * Tb::M1(a, b);
        LQ[slot] += V * l;
      }
    }
  }
}

template <int D, int P = 2>
__global__ __launch_bounds__(kBlock) void k_gather_lam(int64_t n_p2, const int64_t* __restrict__ iptr,
                                                       const int32_t* __restrict__ ilist,
                                                       const double* __restrict__ vol, double* __restrict__ lam) {
  GRID_STRIDE_ROWS(v, n_p2) {
    double s = 0;
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k)
      s += vol[ilist[k] >> kLocBits] * Tab<D, P>::absphi(ilist[k] & kLocMask);
    lam[v] = s;
  }
}

// out[k*planes + c] = a * v1[src*planes + c] + b * v2[...]   (0 on padding)
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, const int32_t* __restrict__ src, int planes, double a,
                                                 const double* __restrict__ v1, double b, const double* __restrict__ v2,
                                                 double* __restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = src[k];
    for (int c = 0; c < planes; ++c) {
      double o = 0;
      if (s >= 0) {
        o = a * v1[s * planes + c];
        if (v2) o += b * v2[s * planes + c];
      }
      out[k * planes + c] = o;
    }
  }
}

// inverse diagonal of a scalar SELL matrix (diagonal entry has column == row)
__global__ __launch_bounds__(kBlock) void k_dinv(int64_t nrows, const int64_t* __restrict__ sp,
                                                 const int32_t* __restrict__ cols, const double* __restrict__ vals,
                                                 double* __restrict__ out) {
  GRID_STRIDE_ROWS(row, nrows) {
    const int64_t s = row >> 6;
    double dv = 0;
    // padding entries carry column 0 and value 0: skip them (row 0 would
    // otherwise pick up a zero "diagonal")
    for (int64_t k = sp[s] + (row & 63); k < sp[s + 1]; k += 64)
      if (cols[k] == row && vals[k] != 0.0) dv = vals[k];
    out[row] = dv != 0 ? 1.0 / dv : 0.0;
  }
}

// row abs-sum times inverse diagonal (Gershgorin bound of D^{-1} S)
__global__ __launch_bounds__(kBlock) void k_gersh(int64_t nrows, const int64_t* __restrict__ sp,
                                                  const int32_t* __restrict__ vals_cols_dummy,
                                                  const double* __restrict__ vals, const double* __restrict__ dinv,
                                                  double* __restrict__ out) {
  GRID_STRIDE_ROWS(row, nrows) {
    const int64_t s = row >> 6;
    double a = 0;
    for (int64_t k = sp[s] + (row & 63); k < sp[s + 1]; k += 64) a += fabs(vals[k]);
    out[row] = a * fabs(dinv[row]);
  }
}

__global__ __launch_bounds__(kBlock) void k_lam_int(int64_t n_int, const int32_t* __restrict__ int2nat,
                                                    const double* __restrict__ lam, double* __restrict__ out) {
  GRID_STRIDE_ROWS(k, n_int) out[k] = 1.0 / lam[int2nat[k]];
}

__global__ __launch_bounds__(kBlock) void k_rowsum_csr(int64_t nrows, const int32_t* __restrict__ rp,
                                                       const double* __restrict__ v, double* __restrict__ out) {
  GRID_STRIDE_ROWS(row, nrows) {
    double s = 0;
    for (int64_t k = rp[row]; k < rp[row + 1]; ++k) s += v[k];
    out[row] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ x,
                                                double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] * x[i];
}

__global__ __launch_bounds__(kBlock) void k_sqrt(int64_t n, const double* __restrict__ a, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = sqrt(a[i]);
}

// ------------------------------------------------------------ SELL build

// Stencil slots of a structured pattern: rows of one class (the parity type
// of a grid node) share a stencil, and entry j of every row of the class is
// the same grid offset.  Rows missing an offset (next to the boundary) get a
// zero-valued pad in that slot, so the lanes of a slice gather the same
// offset of consecutive nodes together.
struct SellSlots {
  int R = 2;                      // keys: offsets in [-R, R]^3
  int nclass = 1;
  const int32_t* rxyz = nullptr;  // lattice coordinates of the source rows [3 per row]
  const int32_t* cxyz = nullptr;  // ... of the source columns (same units)
  const uint8_t* rcls = nullptr;  // class of a source row (null: 0)
  // > 0: lattice distance between consecutive nodes of one class along x.
  // The slots of a class then start with pairs of offsets on one lattice
  // line `step` apart (adjacent nodes of the column class, hence adjacent
  // columns), the other offsets after them.
  int step = 0;
  bool pair_flags = false;  // count the leading pair sub-groups of affine slices (pk = 2 + 4 sub-groups)
  int nkeys() const { return (2 * R + 1) * (2 * R + 1) * (2 * R + 1); }
  int cls(int64_t r) const { return rcls ? rcls[r] : 0; }
  int key(int64_t r, int32_t c) const {  // -1: outside the reach
    const int w = 2 * R + 1;
    int k = 0;
    for (int ax = 2; ax >= 0; --ax) {
      const int d = cxyz[3 * int64_t(c) + ax] - rxyz[3 * r + ax];
      if (d < -R || d > R) return -1;
      k = k * w + d + R;
    }
    return k;
  }
};

// Lattice coordinates of the nodes of an m^dim grid (x fastest), times `scale`.
std::vector<int32_t> lattice_coords(int dim, int64_t m, int scale) {
  const int64_t n = dim == 3 ? m * m * m : m * m;
  std::vector<int32_t> x(3 * n, 0);
  for (int64_t v = 0; v < n; ++v) {
    x[3 * v] = static_cast<int32_t>(scale * (v % m));
    x[3 * v + 1] = static_cast<int32_t>(scale * ((v / m) % m));
    x[3 * v + 2] = dim == 3 ? static_cast<int32_t>(scale * (v / (m * m))) : 0;
  }
  return x;
}

// f(begin, end) over [0, n) split across host threads (inline when small).
template <class F>
void parallel_for(int64_t n, F&& f) {
  const int T = std::max(1, std::min(16, static_cast<int>(std::thread::hardware_concurrency())));
  if (n < 65536 || T == 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t ch = (n + T - 1) / T;
  for (int t = 0; t < T; ++t) {
    const int64_t b = t * ch, e = std::min(n, b + ch);
    if (b >= e) break;
    th.emplace_back([&f, b, e] { f(b, e); });
  }
  for (auto& x : th) x.join();
}

// rows_in_order[r] = source row of output row r; entries kept where
// col_map[col] >= 0; entry_map (optional) renames source entries.  Without
// `slots` the entries of a row are sorted by column; with it they sit in the
// stencil slots of the row's class (a pattern that is not a lattice stencil
// of that reach falls back to sorted rows).  Pads carry src -1 (value 0) and
// the column of the nearest lane of the slice that has an entry in that slot
// (0 if none), which keeps the gathered addresses of a slot together.
void build_sell(const HostCsr& in, const std::vector<int32_t>& rows_in_order, const std::vector<int32_t>& col_map,
                const std::vector<int64_t>* entry_map, int planes, Sell& out, const SellSlots* slots = nullptr) {
  const int64_t nrows = static_cast<int64_t>(rows_in_order.size());
  const int64_t nsl = (nrows + 63) / 64;
  std::vector<int64_t> sp(nsl + 1, 0);
  std::vector<int32_t> len(nrows, 0), cnt(nrows, 0);
  // slot of each key per class (slots mode)
  std::vector<int32_t> slot_of, class_width;
  if (slots) {
    const int nk = slots->nkeys(), ncl = slots->nclass;
    std::vector<char> present((size_t)ncl * nk, 0);
    std::vector<std::vector<char>> part;
    std::vector<char> bad;
    const int T = std::max(1, std::min(16, static_cast<int>(std::thread::hardware_concurrency())));
    part.assign(T, std::vector<char>((size_t)ncl * nk, 0));
    bad.assign(T, 0);
    std::vector<std::thread> th;
    const int64_t ch = (nrows + T - 1) / T;
    for (int t = 0; t < T; ++t) {
      th.emplace_back([&, t] {
        for (int64_t r = t * ch; r < std::min(nrows, (t + 1) * ch); ++r) {
          const int64_t sr = rows_in_order[r];
          const int cl = slots->cls(sr);
          if (cl < 0 || cl >= ncl) {
            bad[t] = 1;
            return;
          }
          for (int64_t k = in.rowptr[sr]; k < in.rowptr[sr + 1]; ++k) {
            if (col_map[in.cols[k]] < 0) continue;
            const int key = slots->key(sr, in.cols[k]);
            if (key < 0) {
              bad[t] = 1;
              return;
            }
            part[t][(size_t)cl * nk + key] = 1;
          }
        }
      });
    }
    for (auto& x : th) x.join();
    for (int t = 0; t < T; ++t) {
      if (bad[t]) return build_sell(in, rows_in_order, col_map, entry_map, planes, out, nullptr);
      for (size_t i = 0; i < present.size(); ++i) present[i] |= part[t][i];
    }
    slot_of.assign(present.size(), -1);
    class_width.assign(ncl, 0);
    const int wk = 2 * slots->R + 1;
    for (int cl = 0; cl < ncl; ++cl) {
      if (slots->step <= 0) {
        for (int key = 0; key < nk; ++key)
          if (present[(size_t)cl * nk + key]) slot_of[(size_t)cl * nk + key] = class_width[cl]++;
        continue;
      }
      // Runs: keys of one (dz, dy) line with one dx residue mod step, dx
      // ascending in steps of `step` (consecutive keys of a run are
      // adjacent columns).  Every run gives its keys two by two to the
      // pairs, which take the first slots; the lone keys follow.
      std::vector<int> paired, lone;
      for (int zy = 0; zy < wk * wk; ++zy)
        for (int res = 0; res < slots->step; ++res) {
          std::vector<int> run;
          int prev = -1000;
          auto flush = [&]() {
            size_t i = 0;
            for (; i + 1 < run.size(); i += 2) paired.insert(paired.end(), {run[i], run[i + 1]});
            if (i < run.size()) lone.push_back(run[i]);
            run.clear();
          };
          for (int dxi = 0; dxi < wk; ++dxi) {
            const int key = zy * wk + dxi, dx = dxi - slots->R;
            if (!present[(size_t)cl * nk + key] || ((dx % slots->step) + slots->step) % slots->step != res) continue;
            if (dx - prev != slots->step) flush();
            run.push_back(key);
            prev = dx;
          }
          flush();
        }
      for (int key : paired) slot_of[(size_t)cl * nk + key] = class_width[cl]++;
      for (int key : lone) slot_of[(size_t)cl * nk + key] = class_width[cl]++;
    }
  }
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t r = b; r < e; ++r) {
      const int64_t sr = rows_in_order[r];
      int32_t c = 0;
      for (int64_t k = in.rowptr[sr]; k < in.rowptr[sr + 1]; ++k)
        if (col_map[in.cols[k]] >= 0) ++c;
      cnt[r] = c;
      len[r] = slots ? class_width[slots->cls(sr)] : c;
    }
  });
  int64_t nnz = 0;
  for (int64_t r = 0; r < nrows; ++r) nnz += cnt[r];
  for (int64_t sl = 0; sl < nsl; ++sl) {
    int32_t w = 0;
    for (int64_t r = sl * 64; r < std::min(nrows, (sl + 1) * 64); ++r) w = std::max(w, len[r]);
    sp[sl + 1] = sp[sl] + 64 * int64_t(w);
  }
  const int64_t npad = sp[nsl];
  if (npad >= (int64_t(1) << 31)) throw Error(STOKES_ERR_UNSUPPORTED, "sparse operator exceeds 2^31 entries");
  std::vector<int32_t> cols(npad, 0), src(npad, -1);
  std::vector<char> clash(nsl, 0);
  parallel_for(nsl, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, int64_t>> buf;
    for (int64_t r = b * 64; r < std::min(nrows, e * 64); ++r) {
      const int64_t sr = rows_in_order[r];
      const int64_t base = sp[r / 64] + (r % 64);
      if (slots) {
        const int cl = slots->cls(sr);
        for (int64_t k = in.rowptr[sr]; k < in.rowptr[sr + 1]; ++k) {
          const int32_t c = col_map[in.cols[k]];
          if (c < 0) continue;
          const int32_t j = slot_of[(size_t)cl * slots->nkeys() + slots->key(sr, in.cols[k])];
          if (src[base + 64 * j] >= 0) clash[r / 64] = 1;
          cols[base + 64 * j] = c;
          src[base + 64 * j] = static_cast<int32_t>(entry_map ? (*entry_map)[k] : k);
        }
        continue;
      }
      buf.clear();
      for (int64_t k = in.rowptr[sr]; k < in.rowptr[sr + 1]; ++k) {
        const int32_t c = col_map[in.cols[k]];
        if (c >= 0) buf.emplace_back(c, entry_map ? (*entry_map)[k] : k);
      }
      std::sort(buf.begin(), buf.end());
      for (size_t j = 0; j < buf.size(); ++j) {
        cols[base + 64 * j] = buf[j].first;
        src[base + 64 * j] = static_cast<int32_t>(buf[j].second);
      }
    }
  });
  for (char x : clash)
    if (x) return build_sell(in, rows_in_order, col_map, entry_map, planes, out, nullptr);
  // pads take the column of the nearest lane with an entry in the same slot;
  // packed columns: per slot a base and 8-bit lane offsets, where every slot
  // of the slice spans at most 256 columns
  std::vector<int32_t> cbase(npad / 64, 0);
  std::vector<uint8_t> cdel(npad, 0);
  std::vector<int32_t> pk(nsl, 0);
  parallel_for(nsl, [&](int64_t b, int64_t e) {
    for (int64_t sl = b; sl < e; ++sl) {
      const int64_t w = (sp[sl + 1] - sp[sl]) / 64;
      for (int64_t j = 0; j < w; ++j) {
        const int64_t b0 = sp[sl] + 64 * j;
        int first = -1;
        for (int l = 0; l < 64 && first < 0; ++l)
          if (src[b0 + l] >= 0) first = l;
        if (first < 0) continue;
        int last = first;
        for (int l = 0; l < 64; ++l) {
          if (src[b0 + l] >= 0) last = l;
          else cols[b0 + l] = cols[b0 + (l < first ? first : last)];
        }
      }
      const int lanes = static_cast<int>(std::min<int64_t>(64, nrows - sl * 64));
      bool ok = true;
      for (int64_t j = 0; j < w && ok; ++j) {
        const int64_t b0 = sp[sl] + 64 * j;
        int32_t lo = cols[b0], hi = cols[b0];
        for (int l = 1; l < lanes; ++l) {
          lo = std::min(lo, cols[b0 + l]);
          hi = std::max(hi, cols[b0 + l]);
        }
        ok = int64_t(hi) - lo <= 255;
      }
      if (!ok) continue;
      pk[sl] = 1;
      for (int64_t j = 0; j < w; ++j) {
        const int64_t b0 = sp[sl] + 64 * j;
        int32_t lo = cols[b0];
        for (int l = 1; l < lanes; ++l) lo = std::min(lo, cols[b0 + l]);
        cbase[sp[sl] / 64 + j] = lo;
        for (int l = 0; l < lanes; ++l) cdel[b0 + l] = static_cast<uint8_t>(cols[b0 + l] - lo);
      }
    }
  });
  // Affine slots: in the typed row order the 64 rows of a slice are mostly
  // consecutive nodes of one lattice line, so slot j of lane l often holds
  // the column base_j + l, with at most one jump where the slice crosses to
  // the next lattice line.  A packed slice whose every slot has that form
  // (entries only; a pad lane's formula column must merely be a valid
  // column, its value is 0) is marked pk = 2 and gets (base, brk | jump << 8)
  // per slot: the kernels that know the form compute the columns instead of
  // loading them.  Its packed offsets stay valid for every other kernel.
  int64_t ncols = 0;
  for (int32_t v : col_map) ncols = std::max<int64_t>(ncols, int64_t(v) + 1);
  std::vector<int32_t> cmeta(2 * (npad / 64), 0);
  parallel_for(nsl, [&](int64_t b, int64_t e) {
    std::vector<int32_t> base, meta;
    for (int64_t sl = b; sl < e; ++sl) {
      if (pk[sl] != 1) continue;
      const int64_t w = (sp[sl + 1] - sp[sl]) / 64;
      const int lanes = static_cast<int>(std::min<int64_t>(64, nrows - sl * 64));
      base.assign(w, 0);
      meta.assign(w, 0);
      bool ok = true;
      for (int64_t j = 0; j < w && ok; ++j) {
        const int64_t b0 = sp[sl] + 64 * j;
        int64_t d0 = cols[b0], jump = 0;
        int brk = 64;
        bool have = false;
        for (int l = 0; l < lanes && ok; ++l) {
          if (src[b0 + l] < 0) continue;
          const int64_t d = int64_t(cols[b0 + l]) - l;
          if (!have) {
            d0 = d;
            have = true;
          } else if (brk == 64) {
            if (d != d0) {
              brk = l;
              jump = d - d0;
            }
          } else if (d != d0 + jump) {
            ok = false;
          }
        }
        if (!ok || jump < -(int64_t(1) << 22) || jump >= (int64_t(1) << 22)) {
          ok = false;
          break;
        }
        for (int l = 0; l < 64 && ok; ++l) {  // every lane's formula column is a valid column
          const int64_t c = d0 + l + (l >= brk ? jump : 0);
          ok = c >= 0 && c < ncols;
        }
        base[j] = static_cast<int32_t>(d0);
        meta[j] = static_cast<int32_t>(brk | (jump * 256));
      }
      if (!ok) continue;
      // leading four-slot sub-groups of two adjacent-node pairs (same break
      // and jump), inside the eight-slot groups of the interleaved half copy
      int pg = 0;
      if (slots && slots->pair_flags)
        while (pg < 2 * (w / 8)) {
          const int64_t j = 4 * pg;
          if (base[j + 1] != base[j] + 1 || meta[j + 1] != meta[j] || base[j + 3] != base[j + 2] + 1 ||
              meta[j + 3] != meta[j + 2])
            break;
          ++pg;
        }
      pk[sl] = 2 + 4 * pg;
      for (int64_t j = 0; j < w; ++j) {
        cmeta[2 * (sp[sl] / 64 + j)] = base[j];
        cmeta[2 * (sp[sl] / 64 + j) + 1] = meta[j];
      }
    }
  });
  int64_t npk = 0, naf = 0;
  double idx_bytes = 0, idx_bytes_af = 0;
  for (int64_t sl = 0; sl < nsl; ++sl) {
    npk += pk[sl] != 0;
    naf += (pk[sl] & 3) == 2;
    const double w = double(sp[sl + 1] - sp[sl]) / 64;
    const double packed_or_wide = 12.0 + (pk[sl] ? 64.0 * w + 4.0 * w : 4.0 * 64.0 * w);  // slice offset and form, slots
    idx_bytes += packed_or_wide;
    idx_bytes_af += (pk[sl] & 3) == 2 ? 12.0 + 8.0 * w : packed_or_wide;
  }
  out.nrows = nrows;
  out.nslices = nsl;
  out.nnz = nnz;
  out.nnz_pad = npad;
  out.packed_slices = npk;
  out.affine_slices = naf;
  out.idx_bytes = idx_bytes;
  out.idx_bytes_af = idx_bytes_af;
  out.ncols = ncols;
  out.planes = planes;
  upload(out.slice_ptr, sp);
  upload(out.cols, cols);
  upload(out.src, src);
  upload(out.cbase, cbase);
  upload(out.cdel, cdel);
  upload(out.pk, pk);
  upload(out.cmeta, cmeta);
}

template <class K, class... A>
void launch(stokes_ctx* c, int64_t n, K kern, A... args) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 65535));
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, c->stream, args...);
  HIP_CHECK(hipGetLastError());
}

// Tridiagonal Lanczos extreme eigenvalues by Sturm bisection.
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lo, double& hi) {
  const int k = static_cast<int>(a.size());
  double gl = 1e300, gh = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < k ? std::fabs(b[i]) : 0);
    gl = std::min(gl, a[i] - r);
    gh = std::max(gh, a[i] + r);
  }
  auto count_below = [&](double x) {  // number of eigenvalues < x
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
      if (q == 0) q = 1e-300;
      q = a[i] - x - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  double l = gl, h = gh;
  for (int it = 0; it < 200; ++it) {  // largest: count_below(x) == k - 1 boundary
    const double m = 0.5 * (l + h);
    if (count_below(m) >= k) h = m;
    else l = m;
  }
  hi = h;
  l = gl;
  h = gh;
  for (int it = 0; it < 200; ++it) {  // smallest
    const double m = 0.5 * (l + h);
    if (count_below(m) >= 1) h = m;
    else l = m;
  }
  lo = l;
}

}  // namespace

// Lanczos on D^{-1/2} S D^{-1/2} (FP64, scalar SELL); returns Ritz extremes.
void lanczos_bounds(stokes_ctx* c, const Sell& S, const double* vals, const double* dinv, int steps, double& rlo,
                    double& rhi, double& gersh) {
  const int64_t n = S.nrows;
  double* sq = static_cast<double*>(c->workspace("lz_sq", n * sizeof(double)));
  double* v0 = static_cast<double*>(c->workspace("lz_v0", n * sizeof(double)));
  double* v1 = static_cast<double*>(c->workspace("lz_v1", n * sizeof(double)));
  double* t = static_cast<double*>(c->workspace("lz_t", n * sizeof(double)));
  double* w = static_cast<double*>(c->workspace("lz_w", n * sizeof(double)));
  launch(c, n, k_sqrt, n, dinv, sq);
  // Gershgorin bound of D^{-1} S
  launch(c, n, k_gersh, n, S.slice_ptr.as<int64_t>(), S.cols.as<int32_t>(), vals, dinv, t);
  {
    std::vector<double> h(n);
    HIP_CHECK(hipMemcpyAsync(h.data(), t, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    gersh = *std::max_element(h.begin(), h.end());
  }
  // deterministic pseudo-random start vector (SplitMix64 finaliser of the row
  // index): it has components along every eigenvector with overwhelming
  // probability, independent of how the rows are ordered
  {
    std::vector<double> h(n);
    double nn = 0;
    for (int64_t i = 0; i < n; ++i) {
      uint64_t z = 0x9E3779B97F4A7C15ULL * uint64_t(i + 1);
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z ^= z >> 31;
      h[i] = double(z >> 11) * 0x1.0p-53 - 0.5;
      nn += h[i] * h[i];
    }
    for (double& x : h) x /= std::sqrt(nn);
    HIP_CHECK(hipMemcpyAsync(v1, h.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_CHECK(hipMemsetAsync(v0, 0, n * sizeof(double), c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
  }
  std::vector<double> al, be;
  double beta_prev = 0, beta_first = 0;
  steps = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(steps, n - 1)));
  for (int j = 0; j < steps; ++j) {
    // w = sq .* S (sq .* v1)
    launch(c, n, k_mul, n, sq, v1, t);
    ops::spmv<double>(c, S, vals, 1, t, w, 1.0, nullptr, 0.0);
    launch(c, n, k_mul, n, sq, w, w);
    const double a = ops::dot_host<double>(c, n, 1, v1, w)[0];
    // w = w - a v1 - beta_prev v0
    launch(c, n, k_axpby<double>, n, -a, (const double*)v1, 1.0, w);
    if (j > 0) launch(c, n, k_axpby<double>, n, -beta_prev, (const double*)v0, 1.0, w);
    const double bn = std::sqrt(ops::dot_host<double>(c, n, 1, w, w)[0]);
    al.push_back(a);
    if (j == 0) beta_first = bn;
    if (j + 1 == steps || bn < 1e-10 * std::max(std::fabs(a), beta_first)) break;
    be.push_back(bn);
    std::swap(v0, v1);
    launch(c, n, k_axpby<double>, n, 1.0 / bn, (const double*)w, 0.0, v1);
    beta_prev = bn;
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  tridiag_extremes(al, be, rlo, rhi);
}

void assemble_ctx(stokes_ctx* c) {
  // STOKES_LOG >= 1: one stderr line per set-up phase with the elapsed time
  const char* log_env = std::getenv("STOKES_LOG");
  const bool log = log_env && std::atoi(log_env) >= 1;
  const auto t0 = std::chrono::steady_clock::now();
  auto phase = [&](const char* what) {
    if (!log) return;
    HIP_CHECK(hipStreamSynchronize(c->stream));
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[stokes] assemble %-28s %8.2f s\n", what, s);
    std::fflush(stderr);
  };
  upload_tables();
  const HostMesh& m = c->mesh;
  const int D = m.dim;
  const int K = m.order;  // velocity order: 2 (P2/P1) or 3 (P3/P2)
  const int nq = m.nqloc;
  const int64_t n_q = m.n_q;  // pressure nodes: the vertices, or the P2 nodes

  // ---- host patterns (velocity x velocity, pressure x velocity, pressure x pressure)
  HostCsr P2full, Bfull, P1;
  element_pattern(m.p2, m.nloc, m.n_p2, m.p2, m.nloc, m.n_p2, m.n_e, P2full);
  element_pattern(m.q, nq, n_q, m.p2, m.nloc, m.n_p2, m.n_e, Bfull);
  element_pattern(m.q, nq, n_q, m.q, nq, n_q, m.n_e, P1);
  if (P2full.rowptr.back() >= (int64_t(1) << 31) || Bfull.rowptr.back() * D >= (int64_t(1) << 31))
    throw Error(STOKES_ERR_UNSUPPORTED, "mesh too large for 32-bit sparse indices");
  phase("host patterns");

  // internal numbering of the interior nodes: 8 slabs along the slowest axis
  // (one per XCD, see the XCD-aware row partition of the gathering kernels);
  // inside a slab, the nodes of one type (the K^dim classes of velocity
  // nodes of the Kuhn lattice by their coordinates mod K, each with its own
  // stencil) in natural order.  Consecutive rows of a sliced-ELL slice are
  // then translates of each other, so the k-th stencil slot of the lanes
  // gathers consecutive nodes.
  const int64_t n2 = K * int64_t(m.n) + 1, plane = D == 3 ? n2 * n2 : n2;
  const int64_t nql = (K - 1) * int64_t(m.n) + 1;
  const int ntypes = D == 3 ? K * K * K : K * K;
  // lattice coordinates of velocity and pressure nodes in one unit: h / 2
  // for P2/P1 (vertices at even points), h / 6 for P3/P2; and the type of
  // every velocity node
  const int sv = K == 3 ? 2 : 1, sq = K == 3 ? 3 : 2;
  const std::vector<int32_t> p2xyz = lattice_coords(D, n2, sv), p1xyz = lattice_coords(D, nql, sq);
  std::vector<uint8_t> p2type(m.n_p2);
  for (int64_t v = 0; v < m.n_p2; ++v) {
    int t = 0;
    for (int ax = D - 1; ax >= 0; --ax) t = t * K + (p2xyz[3 * v + ax] / sv) % K;
    p2type[v] = static_cast<uint8_t>(t);
  }
  // type of every pressure node (P2 pressure: coordinates mod 2; P1: one type)
  std::vector<uint8_t> qtype(n_q, 0);
  if (K == 3)
    for (int64_t v = 0; v < n_q; ++v) {
      int t = 0;
      for (int ax = D - 1; ax >= 0; --ax) t = t * 2 + (p1xyz[3 * v + ax] / sq) % 2;
      qtype[v] = static_cast<uint8_t>(t);
    }
  // Stable bucket order by (slab, block, type), natural order inside a
  // bucket.  A block is `zblock` consecutive lattice planes of the slab (0:
  // the whole slab; by default 2 planes once a plane holds more than 2^15
  // nodes, else the whole slab): a kernel walks the rows of one type block
  // by block, so the gathered neighbours (all types, the block's planes and
  // one halo plane on each side) stay in the caches while the other types of
  // the same block are walked.  On the large meshes with many right-hand
  // sides a slab's worth of them does not (cube128 x 8: 931 -> 868 ms per
  // batched solve with 2-plane blocks, 888 with 4, 926 with 8; one
  // right-hand side: no change); on smaller ones the blocks only cost
  // (cube64: 11.64 -> 11.94 ms with 4-plane blocks).
  std::vector<int32_t> interior;
  std::vector<int32_t> h_rperm;  // slice schedule of the gathering kernels (empty: slice order)
  {
    const int64_t nK = n2 - 2;  // interior planes (3D) or lines (2D)
    std::vector<int64_t> slab_lo(9);
    for (int sl = 0; sl <= 8; ++sl) slab_lo[sl] = (sl * nK + 7) / 8;  // first K - 1 with slab >= sl
    const int64_t zbk = c->zblock >= 0 ? c->zblock : (plane > (int64_t(1) << 15) ? 2 : 0);
    const int64_t zb = zbk > 0 ? zbk : nK;
    const int64_t nblk = (nK + zb - 1) / zb + 8;  // blocks per slab, bounded
    std::vector<int64_t> start(8 * nblk * ntypes + 1, 0);
    std::vector<int32_t> bucket(m.n_p2, 0);
    for (int64_t v = 0; v < m.n_p2; ++v) {
      if (m.p2_bnd[v]) continue;
      const int64_t K = v / plane;  // 1 .. 2n-1 on interior nodes
      const int64_t sl = std::min<int64_t>(7, (K - 1) * 8 / nK);
      const int64_t blk = std::min<int64_t>(nblk - 1, (K - 1 - slab_lo[sl]) / zb);
      bucket[v] = static_cast<int32_t>((sl * nblk + blk) * ntypes + p2type[v]);
      ++start[bucket[v] + 1];
    }
    for (size_t k = 0; k + 1 < start.size(); ++k) start[k + 1] += start[k];
    const std::vector<int64_t> bbeg = start;  // bucket b holds rows [bbeg[b], bbeg[b + 1])
    interior.resize(start.back());
    for (int64_t v = 0; v < m.n_p2; ++v)
      if (!m.p2_bnd[v]) interior[start[bucket[v]]++] = static_cast<int32_t>(v);
    // Slice schedule.  A kernel walking the rows in order finishes one type
    // of a block before the next, and every type gathers the neighbours of
    // all types: the gathered vectors of the whole block (plus halo) must
    // stay in the XCD's L2 until the last type.  Launching the slices of an
    // eighth sorted by (block, relative position inside the slice's type
    // bucket, type) walks the types side by side, so a node's value is
    // gathered by all its neighbour rows within a few lattice lines.  Only
    // the launch order changes: each row is still computed once, by the
    // same arithmetic.  Types alternate in runs of `chunk` slices (64 by
    // default, on meshes whose plane exceeds 2^15 nodes, where a block's
    // gathered vectors outgrow the L2); only products with at least
    // kSchedMinW values per row use it (Sell::idx).  By default the runs
    // are whole y chunks (8 per plane) and a slab's blocks are walked
    // chunk by chunk, so the z neighbours of a node (two planes up or
    // down) are gathered one block apart instead of a whole block of
    // planes apart.
    const int64_t chunk = c->slice_sched >= 0 ? c->slice_sched : (plane > (int64_t(1) << 15) ? 64 : 0);
    const bool sched = chunk > 0;
    const int64_t nint = static_cast<int64_t>(interior.size()), nsl = (nint + 63) / 64;
    if (sched && nsl > 0) {
      h_rperm.resize(nsl);
      const int64_t xn = ((nint + 7) / 8 + 63) / 64 * 64;  // rows per eighth (XCD_ROWS_G)
      // key: (slab, y chunk, block, type, position, slice) with y chunks
      // (slice_yq > 0: the blocks of a slab walked per y chunk, so a node's
      // z neighbours come one block apart), else (block, position, type)
      std::vector<std::tuple<int64_t, int64_t, int64_t, int, double, int32_t>> keys;
      const int64_t nyq = c->slice_yq >= 0 ? c->slice_yq : 8;
      for (int64_t e = 0; e < 8; ++e) {
        const int64_t s0 = std::min(nsl, e * xn / 64);
        int64_t s1 = std::min(nsl, (e + 1) * xn / 64);
        if (s1 == nsl && nint % 64 != 0) {  // the partial last slice keeps its place
          h_rperm[nsl - 1] = static_cast<int32_t>(nsl - 1);
          --s1;
        }
        keys.clear();
        for (int64_t s = s0; s < s1; ++s) {
          const int64_t b = bucket[interior[64 * s]];
          // runs of `chunk` slices of one type: the position of the run's first slice
          const int64_t sb = std::max<int64_t>(s0, bbeg[b] / 64);
          const int64_t r0 = 64 * (sb + (s - sb) / chunk * chunk);
          const double frac = double(r0 + 32 - bbeg[b]) / double(std::max<int64_t>(1, bbeg[b + 1] - bbeg[b]));
          const int64_t grp = b / ntypes;
          const int ty = static_cast<int>(b % ntypes);
          if (nyq > 0) {
            const double fs = double(64 * s + 32 - bbeg[b]) / double(std::max<int64_t>(1, bbeg[b + 1] - bbeg[b]));
            const int64_t yq = std::min<int64_t>(nyq - 1, std::max<int64_t>(0, static_cast<int64_t>(fs * nyq)));
            keys.emplace_back(grp / nblk, yq, grp % nblk, ty, fs, static_cast<int32_t>(s));
          } else {
            keys.emplace_back(grp, 0, 0, ty, frac, static_cast<int32_t>(s));  // sorted by (block, position, type)
          }
        }
        if (nyq > 0) {
          std::stable_sort(keys.begin(), keys.end());
        } else {
          std::stable_sort(keys.begin(), keys.end(), [](const auto& a, const auto& b) {
            if (std::get<0>(a) != std::get<0>(b)) return std::get<0>(a) < std::get<0>(b);
            if (std::get<4>(a) != std::get<4>(b)) return std::get<4>(a) < std::get<4>(b);
            if (std::get<3>(a) != std::get<3>(b)) return std::get<3>(a) < std::get<3>(b);
            return std::get<5>(a) < std::get<5>(b);
          });
        }
        for (int64_t t = s0; t < s1; ++t) h_rperm[t] = std::get<5>(keys[t - s0]);
      }
      // a permutation inside every eighth (checked: the kernels trust it)
      std::vector<char> seen(nsl, 0);
      for (int64_t t = 0; t < nsl; ++t) {
        const int64_t s = h_rperm[t];
        if (s < 0 || s >= nsl || seen[s] || s * 64 / xn != t * 64 / xn)
          throw Error(STOKES_ERR_STATE, "slice schedule is not a permutation inside the eighths");
        seen[s] = 1;
      }
    }
  }
  // stencil slots: offsets reach 2 (P2/P1, units h / 2) or 6 (P3/P2, h / 6)
  SellSlots slots_p2p2, slots_p2p1, slots_p1p2;
  slots_p2p2.nclass = slots_p2p1.nclass = ntypes;
  slots_p2p2.rcls = slots_p2p1.rcls = p2type.data();
  slots_p2p2.rxyz = slots_p2p2.cxyz = slots_p2p1.rxyz = p2xyz.data();
  slots_p2p1.cxyz = p1xyz.data();
  slots_p1p2.rxyz = p1xyz.data();
  slots_p1p2.cxyz = p2xyz.data();
  // velocity slots in line order, adjacent-node pairs flagged for the
  // bfloat16 Chebyshev step (one 16-byte gather per pair)
  slots_p2p2.step = c->vel_pair ? K * sv : 0;
  slots_p2p2.pair_flags = c->vel_pair == 1;
  if (K == 3) {
    slots_p2p2.R = slots_p2p1.R = slots_p1p2.R = 6;
    slots_p1p2.nclass = D == 3 ? 8 : 4;
    slots_p1p2.rcls = qtype.data();
  }
  c->n_int = static_cast<int64_t>(interior.size());
  c->h_int2nat = interior;
  c->h_nat2int.assign(m.n_p2, -1);
  for (int64_t k = 0; k < c->n_int; ++k) c->h_nat2int[interior[k]] = static_cast<int32_t>(k);
  upload(c->int2nat, c->h_int2nat);
  upload(c->nat2int, c->h_nat2int);

  // ---- upload mesh + incidences, geometry
  DevBuf d_vc, d_el, d_p2, d_vol, d_jinv, d_i2p, d_i2l, d_i1p, d_i1l, d_q;
  upload(d_vc, m.vcoords);
  upload(d_el, m.elems);
  upload(d_p2, m.p2);
  upload(d_q, m.q);
  d_vol.alloc(m.n_e * sizeof(double));
  d_jinv.alloc(m.n_e * D * D * sizeof(double));
  if (D == 3) launch(c, m.n_e, k_geom<3>, m.n_e, d_vc.as<double>(), d_el.as<int32_t>(), d_vol.as<double>(), d_jinv.as<double>());
  else launch(c, m.n_e, k_geom<2>, m.n_e, d_vc.as<double>(), d_el.as<int32_t>(), d_vol.as<double>(), d_jinv.as<double>());
  {
    std::vector<int64_t> ptr;
    std::vector<int32_t> lst;
    incidence(m.p2, m.nloc, m.n_e, m.n_p2, ptr, lst);
    upload(d_i2p, ptr);
    upload(d_i2l, lst);
    incidence(m.q, nq, m.n_e, n_q, ptr, lst);
    upload(d_i1p, ptr);
    upload(d_i1l, lst);
  }
  auto up_csr = [&](const HostCsr& h, DevCsr& dcsr) {
    std::vector<int32_t> rp(h.rowptr.begin(), h.rowptr.end());
    dcsr.nrows = h.nrows;
    dcsr.nnz = h.rowptr.back();
    upload(dcsr.rowptr, rp);
    upload(dcsr.cols, h.cols);
  };
  up_csr(P2full, c->p2full);
  up_csr(Bfull, c->bfull);
  up_csr(P1, c->p1);
  {
    // boundary coupling of interior rows (load vector and Dirichlet lifting)
    std::vector<int32_t> rows, ptr(1, 0), cols, src;
    for (int64_t k = 0; k < c->n_int; ++k) {
      const int32_t v = c->h_int2nat[k];
      const size_t before = cols.size();
      for (int64_t e = P2full.rowptr[v]; e < P2full.rowptr[v + 1]; ++e) {
        if (!m.p2_bnd[P2full.cols[e]]) continue;
        cols.push_back(P2full.cols[e]);
        src.push_back(static_cast<int32_t>(e));
      }
      if (cols.size() > before) {
        rows.push_back(static_cast<int32_t>(k));
        ptr.push_back(static_cast<int32_t>(cols.size()));
      }
    }
    c->n_bc = static_cast<int64_t>(rows.size());
    if (c->n_bc > 0) {
      upload(c->bc_rows, rows);
      upload(c->bc_ptr, ptr);
      upload(c->bc_cols, cols);
      upload(c->bc_src, src);
    }
  }

  // ---- element gathers (FP64, full numbering)
  const int64_t nnz2 = c->p2full.nnz, nnzb = c->bfull.nnz, nnz1 = c->p1.nnz;
  c->M_full.alloc(nnz2 * sizeof(double));
  c->L_full.alloc(nnz2 * sizeof(double));
  c->B_full.alloc(nnzb * D * sizeof(double));
  c->MQ_csr.alloc(nnz1 * sizeof(double));
  c->LQ_csr.alloc(nnz1 * sizeof(double));
  c->lam_full.alloc(m.n_p2 * sizeof(double));
  HIP_CHECK(hipMemsetAsync(c->M_full.p, 0, nnz2 * sizeof(double), c->stream));
  HIP_CHECK(hipMemsetAsync(c->L_full.p, 0, nnz2 * sizeof(double), c->stream));
  if (c->strain) {
    c->D_full.alloc(nnz2 * D * D * sizeof(double));
    HIP_CHECK(hipMemsetAsync(c->D_full.p, 0, nnz2 * D * D * sizeof(double), c->stream));
  }
  HIP_CHECK(hipMemsetAsync(c->B_full.p, 0, nnzb * D * sizeof(double), c->stream));
  HIP_CHECK(hipMemsetAsync(c->MQ_csr.p, 0, nnz1 * sizeof(double), c->stream));
  HIP_CHECK(hipMemsetAsync(c->LQ_csr.p, 0, nnz1 * sizeof(double), c->stream));
  // the element gathers for one (dim, order)
  auto gathers = [&](auto Dc, auto Pc) {
    constexpr int DD = decltype(Dc)::value, PP = decltype(Pc)::value;
    launch(c, m.n_p2, k_gather_p2<DD, PP>, m.n_p2, d_i2p.as<int64_t>(), d_i2l.as<int32_t>(), d_p2.as<int32_t>(),
           d_vol.as<double>(), d_jinv.as<double>(), c->p2full.rowptr.as<int32_t>(), c->p2full.cols.as<int32_t>(),
           c->M_full.as<double>(), c->L_full.as<double>(), c->strain ? c->D_full.as<double>() : nullptr);
    launch(c, n_q, k_gather_b<DD, PP>, n_q, d_i1p.as<int64_t>(), d_i1l.as<int32_t>(), d_p2.as<int32_t>(),
           d_vol.as<double>(), d_jinv.as<double>(), c->bfull.rowptr.as<int32_t>(), c->bfull.cols.as<int32_t>(),
           c->B_full.as<double>());
    if (PP == 3)  // P2 pressure: the P2 mass and Laplacian rows
      launch(c, n_q, k_gather_p2<DD, 2>, n_q, d_i1p.as<int64_t>(), d_i1l.as<int32_t>(), d_q.as<int32_t>(),
             d_vol.as<double>(), d_jinv.as<double>(), c->p1.rowptr.as<int32_t>(), c->p1.cols.as<int32_t>(),
             c->MQ_csr.as<double>(), c->LQ_csr.as<double>(), (double*)nullptr);
    else
      launch(c, n_q, k_gather_q<DD>, n_q, d_i1p.as<int64_t>(), d_i1l.as<int32_t>(), d_el.as<int32_t>(),
             d_vol.as<double>(), d_jinv.as<double>(), c->p1.rowptr.as<int32_t>(), c->p1.cols.as<int32_t>(),
             c->MQ_csr.as<double>(), c->LQ_csr.as<double>());
    launch(c, m.n_p2, k_gather_lam<DD, PP>, m.n_p2, d_i2p.as<int64_t>(), d_i2l.as<int32_t>(), d_vol.as<double>(),
           c->lam_full.as<double>());
  };
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  if (D == 3 && K == 3) gathers(I3{}, I3{});
  else if (D == 3) gathers(I3{}, I2{});
  else if (K == 3) gathers(I2{}, I3{});
  else gathers(I2{}, I2{});

  phase("element gathers");
  // ---- SELL operators
  std::vector<int32_t> p1_rows(n_q), p1_ident(n_q);
  std::iota(p1_rows.begin(), p1_rows.end(), 0);
  std::iota(p1_ident.begin(), p1_ident.end(), 0);
  build_sell(P2full, c->h_int2nat, c->h_nat2int, nullptr, 1, c->sA, &slots_p2p2);
  c->rperm.release();
  if (!h_rperm.empty()) {
    if (c->sA.nslices != static_cast<int64_t>(h_rperm.size()))
      throw Error(STOKES_ERR_STATE, "slice schedule does not match the velocity pattern");
    upload(c->rperm, h_rperm);
  }
  c->sA.rperm = c->rperm.as<const int32_t>();
  build_sell(Bfull, p1_rows, c->h_nat2int, nullptr, D, c->sB, &slots_p1p2);
  {
    HostCsr BT, XLpat;
    std::vector<int64_t> tsrc;
    transpose_pattern(Bfull, BT, tsrc);
    build_sell(BT, c->h_int2nat, p1_ident, &tsrc, D, c->sBt, &slots_p2p1);
    if (c->rperm.p && c->sBt.nslices != c->sA.nslices)
      throw Error(STOKES_ERR_STATE, "slice schedule does not match the B^T pattern");
    c->sBt.rperm = c->rperm.as<const int32_t>();
    // B_I Lambda_V^-1 B_I^T: shared interior P2 columns only
    product_pattern(Bfull, BT, c->h_nat2int, XLpat);
    up_csr(XLpat, c->xl);
    c->XL_csr.alloc(c->xl.nnz * sizeof(double));
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n_q + 3) / 4, 65535));
    if (D == 3)
      hipLaunchKernelGGL(k_gather_xl<3>, dim3(nb), dim3(kBlock), 0, c->stream, n_q, c->bfull.rowptr.as<int32_t>(),
                         c->bfull.cols.as<int32_t>(), c->B_full.as<double>(), c->lam_full.as<double>(),
                         c->nat2int.as<int32_t>(), c->xl.rowptr.as<int32_t>(), c->xl.cols.as<int32_t>(),
                         c->XL_csr.as<double>());
    else
      hipLaunchKernelGGL(k_gather_xl<2>, dim3(nb), dim3(kBlock), 0, c->stream, n_q, c->bfull.rowptr.as<int32_t>(),
                         c->bfull.cols.as<int32_t>(), c->B_full.as<double>(), c->lam_full.as<double>(),
                         c->nat2int.as<int32_t>(), c->xl.rowptr.as<int32_t>(), c->xl.cols.as<int32_t>(),
                         c->XL_csr.as<double>());
    HIP_CHECK(hipGetLastError());
    // pressure lattice in its own units: reach 2 (P1, two element rings) or
    // 4 (P2, units h / 2)
    const std::vector<int32_t> q1 = lattice_coords(D, nql, 1);
    SellSlots slx;
    slx.R = K == 3 ? 4 : 2;
    slx.rxyz = slx.cxyz = q1.data();
    if (K == 3) {
      slx.nclass = D == 3 ? 8 : 4;
      slx.rcls = qtype.data();
    }
    build_sell(XLpat, p1_rows, p1_ident, nullptr, 1, c->sX, &slx);
  }
  {
    const std::vector<int32_t> q1 = lattice_coords(D, nql, 1);
    SellSlots slq;
    slq.R = K == 3 ? 2 : 1;
    slq.rxyz = slq.cxyz = q1.data();
    if (K == 3) {
      slq.nclass = D == 3 ? 8 : 4;
      slq.rcls = qtype.data();
    }
    build_sell(P1, p1_rows, p1_ident, nullptr, 1, c->sQ, &slq);
  }
  phase("sliced-ELL layouts");
  if (log) {
    const std::pair<const char*, const Sell*> ss[] = {{"A_II", &c->sA}, {"B", &c->sB}, {"B^T", &c->sBt},
                                                      {"X", &c->sX}, {"M_Q", &c->sQ}};
    for (const auto& e : ss)
      std::fprintf(stderr,
                   "[stokes] SELL %-5s %lld rows, %lld entries (%lld padded), %lld / %lld slices packed, %lld affine\n",
                   e.first, (long long)e.second->nrows, (long long)e.second->nnz, (long long)e.second->nnz_pad,
                   (long long)e.second->packed_slices, (long long)e.second->nslices,
                   (long long)e.second->affine_slices);
  }

  auto fill = [&](const Sell& S, DevBuf& out, double a, const DevBuf& v1, double b, const DevBuf* v2) {
    out.alloc(S.nnz_pad * S.planes * sizeof(double));
    launch(c, S.nnz_pad, k_fill, S.nnz_pad, S.src.as<int32_t>(), S.planes, a, v1.as<double>(), b,
           v2 ? v2->as<double>() : nullptr, out.as<double>());
  };
  const double alpha = c->prob.alpha, mu = c->prob.mu;
  fill(c->sA, c->A64, alpha, c->M_full, mu, &c->L_full);
  fill(c->sA, c->MV64, 1.0, c->M_full, 0.0, nullptr);
  fill(c->sB, c->B64, 1.0, c->B_full, 0.0, nullptr);
  fill(c->sBt, c->Bt64, 1.0, c->B_full, 0.0, nullptr);
  fill(c->sQ, c->MQ64, 1.0, c->MQ_csr, 0.0, nullptr);
  fill(c->sQ, c->LQ64, 1.0, c->LQ_csr, 0.0, nullptr);
  fill(c->sQ, c->XQ64, 1.0, c->MQ_csr, 1.0, &c->LQ_csr);
  fill(c->sX, c->XL64, 1.0, c->XL_csr, 0.0, nullptr);

  auto dinv = [&](const Sell& S, const DevBuf& v, DevBuf& out) {
    out.alloc(S.nrows * sizeof(double));
    launch(c, S.nrows, k_dinv, S.nrows, S.slice_ptr.as<int64_t>(), S.cols.as<int32_t>(), v.as<double>(),
           out.as<double>());
  };
  dinv(c->sA, c->A64, c->dA64);
  c->AD64.alloc(c->sA.nnz_pad * sizeof(double));
  c->AD32.alloc(c->sA.nnz_pad * sizeof(float));
  c->AD16.alloc(c->sA.nnz_pad * sizeof(_Float16));
  launch(c, c->sA.nnz_pad, k_scale_cols, c->sA.nnz_pad, c->sA.cols.as<int32_t>(), c->A64.as<double>(),
         c->dA64.as<double>(), c->AD64.as<double>(), c->AD32.as<float>(), c->AD16.as<_Float16>());
  if (c->strain) {
    c->AB64.alloc(c->sA.nnz_pad * (D * (D + 1) / 2) * sizeof(double));
    c->AB32.alloc(c->sA.nnz_pad * (D * (D + 1) / 2) * sizeof(float));
    launch(c, c->sA.nnz_pad, k_fill_blk, c->sA.nnz_pad, D, c->sA.src.as<int32_t>(), alpha, mu,
           c->M_full.as<double>(), c->L_full.as<double>(), c->D_full.as<double>(), c->AB64.as<double>(),
           c->AB32.as<float>());
  }
  dinv(c->sA, c->MV64, c->dMV64);
  dinv(c->sQ, c->MQ64, c->dMQ64);
  dinv(c->sQ, c->XQ64, c->dXQ64);
  dinv(c->sQ, c->LQ64, c->dLQ64);
  c->lamInv64.alloc(c->n_int * sizeof(double));
  launch(c, c->n_int, k_lam_int, c->n_int, c->int2nat.as<int32_t>(), c->lam_full.as<double>(), c->lamInv64.as<double>());
  c->mQ.alloc(n_q * sizeof(double));
  launch(c, n_q, k_rowsum_csr, n_q, c->p1.rowptr.as<int32_t>(), c->MQ_csr.as<double>(), c->mQ.as<double>());
  {
    std::vector<double> h(n_q);
    HIP_CHECK(hipMemcpyAsync(h.data(), c->mQ.p, n_q * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    c->mQ_sum = 0;
    for (double x : h) c->mQ_sum += x;
  }

  // FP32 copies
  auto to32 = [&](const DevBuf& src, DevBuf& dst, int64_t n) {
    dst.alloc(n * sizeof(float));
    launch(c, n, k_cast<double, float>, n, src.as<double>(), dst.as<float>());
  };
  to32(c->A64, c->A32, c->sA.nnz_pad);
  build_interleaved(c);  // AD16 and A32 are final here
  to32(c->MV64, c->MV32, c->sA.nnz_pad);
  to32(c->B64, c->B32, c->sB.nnz_pad * D);
  to32(c->Bt64, c->Bt32, c->sBt.nnz_pad * D);
  to32(c->MQ64, c->MQ32, c->sQ.nnz_pad);
  to32(c->LQ64, c->LQ32, c->sQ.nnz_pad);
  to32(c->XQ64, c->XQ32, c->sQ.nnz_pad);
  to32(c->XL64, c->XL32, c->sX.nnz_pad);
  to32(c->dA64, c->dA32, c->n_int);
  to32(c->dMV64, c->dMV32, c->n_int);
  to32(c->dMQ64, c->dMQ32, n_q);
  to32(c->dXQ64, c->dXQ32, n_q);
  to32(c->dLQ64, c->dLQ32, n_q);
  to32(c->lamInv64, c->lamInv32, c->n_int);

  // ---- Chebyshev intervals: element bounds of the Jacobi-scaled velocity
  // and pressure masses (the pressure table of a P3/P2 context is the P2 one)
  const RefTables& tb = K == 3 ? (D == 3 ? g_tab3c : g_tab2c) : (D == 3 ? g_tab3 : g_tab2);
  c->bMV = {tb.mass_lo, tb.mass_hi};
  c->bMQ = {tb.p1_lo, tb.p1_hi};
  phase("values and FP32 copies");
  estimate_bounds(c);
  phase("Chebyshev intervals");
  // the pressure multigrids (the P2 pressure of a P3/P2 context coarsens to
  // the P1 space of its mesh first); the velocity multigrid is built on
  // first use, for P2/P1 only
  build_mg(c);
  phase("multigrid hierarchies");
  HIP_CHECK(hipStreamSynchronize(c->stream));
}

// Interleaved copies of the velocity values and of the velocity pattern's
// column indices: eight-slot groups for the half-precision values read by the
// bfloat16 Chebyshev steps, four-slot groups for the FP32 values of the
// velocity product of K_gamma (16 bytes of values per lane and group).
void build_interleaved(stokes_ctx* c) {
  const Sell& S = c->sA;
  if (!c->vel_il || !c->AD16.p || S.nslices == 0) return;
  const int64_t* sp = S.slice_ptr.as<int64_t>();
  auto perm = [&](auto kern, const auto* src, auto* dst) {
    hipLaunchKernelGGL(kern, dim3(S.nslices), dim3(64), 0, c->stream, S.nslices, sp, src, dst);
    HIP_CHECK(hipGetLastError());
  };
  if (!c->AD16i.p) {
    c->AD16i.alloc(S.nnz_pad * sizeof(_Float16));
    if (S.cdel.p) {  // packed slices exist
      c->cdel_i8.alloc(S.nnz_pad * sizeof(uint8_t));
      c->cdel_i.alloc(S.nnz_pad * sizeof(uint8_t));
      perm(k_interleave<uint8_t, 8>, S.cdel.as<const uint8_t>(), c->cdel_i8.as<uint8_t>());
      perm(k_interleave<uint8_t, 4>, S.cdel.as<const uint8_t>(), c->cdel_i.as<uint8_t>());
    }
    c->cols_i8.alloc(S.nnz_pad * sizeof(int32_t));
    c->cols_i.alloc(S.nnz_pad * sizeof(int32_t));
    perm(k_interleave<int32_t, 8>, S.cols.as<const int32_t>(), c->cols_i8.as<int32_t>());
    perm(k_interleave<int32_t, 4>, S.cols.as<const int32_t>(), c->cols_i.as<int32_t>());
  }
  perm(k_interleave<uint16_t, il_width<_Float16>()>, c->AD16.as<const uint16_t>(), c->AD16i.as<uint16_t>());
  if (c->A32.p) {
    if (!c->A32i.p) c->A32i.alloc(S.nnz_pad * sizeof(float));
    perm(k_interleave<uint32_t, il_width<float>()>, c->A32.as<const uint32_t>(), c->A32i.as<uint32_t>());
  }
}

// M_Q + L_Q on a P1 mesh (a coarse level of the pressure multigrid).
void assemble_p1(stokes_ctx* c, const HostMesh& m, MgLevel& L) {
  const int D = m.dim, nv = D + 1;
  HostCsr P1;
  element_pattern(m.elems, nv, m.n_p1, m.elems, nv, m.n_p1, m.n_e, P1);
  DevBuf d_vc, d_el, d_vol, d_jinv, d_ip, d_il, rp, cols, MQ, LQ;
  upload(d_vc, m.vcoords);
  upload(d_el, m.elems);
  d_vol.alloc(m.n_e * sizeof(double));
  d_jinv.alloc(m.n_e * D * D * sizeof(double));
  if (D == 3) launch(c, m.n_e, k_geom<3>, m.n_e, d_vc.as<double>(), d_el.as<int32_t>(), d_vol.as<double>(), d_jinv.as<double>());
  else launch(c, m.n_e, k_geom<2>, m.n_e, d_vc.as<double>(), d_el.as<int32_t>(), d_vol.as<double>(), d_jinv.as<double>());
  {
    std::vector<int64_t> ptr;
    std::vector<int32_t> lst;
    incidence(m.elems, nv, m.n_e, m.n_p1, ptr, lst);
    upload(d_ip, ptr);
    upload(d_il, lst);
  }
  std::vector<int32_t> rp32(P1.rowptr.begin(), P1.rowptr.end());
  upload(rp, rp32);
  upload(cols, P1.cols);
  const int64_t nnz = P1.rowptr.back();
  MQ.alloc(nnz * sizeof(double));
  LQ.alloc(nnz * sizeof(double));
  HIP_CHECK(hipMemsetAsync(MQ.p, 0, nnz * sizeof(double), c->stream));
  HIP_CHECK(hipMemsetAsync(LQ.p, 0, nnz * sizeof(double), c->stream));
  if (D == 3)
    launch(c, m.n_p1, k_gather_q<3>, m.n_p1, d_ip.as<int64_t>(), d_il.as<int32_t>(), d_el.as<int32_t>(),
           d_vol.as<double>(), d_jinv.as<double>(), rp.as<int32_t>(), cols.as<int32_t>(), MQ.as<double>(),
           LQ.as<double>());
  else
    launch(c, m.n_p1, k_gather_q<2>, m.n_p1, d_ip.as<int64_t>(), d_il.as<int32_t>(), d_el.as<int32_t>(),
           d_vol.as<double>(), d_jinv.as<double>(), rp.as<int32_t>(), cols.as<int32_t>(), MQ.as<double>(),
           LQ.as<double>());
  std::vector<int32_t> rows(m.n_p1);
  std::iota(rows.begin(), rows.end(), 0);
  const std::vector<int32_t> q1 = lattice_coords(D, int64_t(m.n) + 1, 1);
  SellSlots sl;
  sl.R = 1;
  sl.rxyz = sl.cxyz = q1.data();
  build_sell(P1, rows, rows, nullptr, 1, L.S, &sl);
  L.nrows = m.n_p1;
  L.v64.alloc(L.S.nnz_pad * sizeof(double));
  launch(c, L.S.nnz_pad, k_fill, L.S.nnz_pad, L.S.src.as<int32_t>(), 1, 1.0, MQ.as<double>(), 1.0, LQ.as<double>(),
         L.v64.as<double>());
  L.d64.alloc(m.n_p1 * sizeof(double));
  launch(c, m.n_p1, k_dinv, m.n_p1, L.S.slice_ptr.as<int64_t>(), L.S.cols.as<int32_t>(), L.v64.as<double>(),
         L.d64.as<double>());
  L.v32.alloc(L.S.nnz_pad * sizeof(float));
  L.d32.alloc(m.n_p1 * sizeof(float));
  launch(c, L.S.nnz_pad, k_cast<double, float>, L.S.nnz_pad, L.v64.as<double>(), L.v32.as<float>());
  launch(c, m.n_p1, k_cast<double, float>, m.n_p1, L.d64.as<double>(), L.d32.as<float>());
  double lo, hi, g;
  lanczos_bounds(c, L.S, L.v64.as<double>(), L.d64.as<double>(), std::min<int>(40, (int)m.n_p1), lo, hi, g);
  L.bf.hi = std::min(g, 1.1 * hi);
  L.bf.lo = 0.9 * lo;
  L.bs.hi = L.bf.hi;
  L.bs.lo = L.bf.hi / c->mg_smooth_ratio;
  HIP_CHECK(hipStreamSynchronize(c->stream));
}

namespace {

// Device copy of one hierarchy level from a host CSR operator.
void upload_level(stokes_ctx* c, const HostCsr& A, const std::vector<double>& av, MgLevel& L) {
  const int64_t nr = A.nrows;
  std::vector<int32_t> rows(nr);
  std::iota(rows.begin(), rows.end(), 0);
  const std::vector<int32_t> q1 = lattice_coords(c->dim, int64_t(L.n) + 1, 1);
  SellSlots sl;
  sl.R = 3;
  sl.rxyz = sl.cxyz = q1.data();
  build_sell(A, rows, rows, nullptr, 1, L.S, &sl);
  L.nrows = nr;
  DevBuf dv;
  upload(dv, av);
  L.v64.alloc(L.S.nnz_pad * sizeof(double));
  launch(c, L.S.nnz_pad, k_fill, L.S.nnz_pad, L.S.src.as<int32_t>(), 1, 1.0, dv.as<double>(), 0.0, nullptr,
         L.v64.as<double>());
  L.d64.alloc(nr * sizeof(double));
  launch(c, nr, k_dinv, nr, L.S.slice_ptr.as<int64_t>(), L.S.cols.as<int32_t>(), L.v64.as<double>(),
         L.d64.as<double>());
  L.v32.alloc(L.S.nnz_pad * sizeof(float));
  L.d32.alloc(nr * sizeof(float));
  launch(c, L.S.nnz_pad, k_cast<double, float>, L.S.nnz_pad, L.v64.as<double>(), L.v32.as<float>());
  launch(c, nr, k_cast<double, float>, nr, L.d64.as<double>(), L.d32.as<float>());
  // half-precision copy for the FP32 V-cycle: values over the largest
  // magnitude of the level (a diagonal), so every row is O(1)
  double amax = 0;
  for (double v : av) amax = std::max(amax, std::fabs(v));
  if (amax > 0) {
    L.s16 = static_cast<float>(amax);
    L.v16.alloc(L.S.nnz_pad * sizeof(_Float16));
    launch(c, L.S.nnz_pad, k_to_half, L.S.nnz_pad, L.v64.as<double>(), 1.0 / double(L.s16), L.v16.as<_Float16>());
  }
  double lo, hi, g;
  lanczos_bounds(c, L.S, L.v64.as<double>(), L.d64.as<double>(), std::min<int>(40, (int)nr), lo, hi, g);
  L.bf.hi = std::min(g, 1.1 * hi);
  L.bf.lo = 0.9 * lo;
  L.bs.hi = L.bf.hi;
  L.bs.lo = L.bf.hi / c->mg_smooth_ratio;
  HIP_CHECK(hipStreamSynchronize(c->stream));  // dv is freed on return
}

void download_csr(stokes_ctx* c, const DevCsr& P, const DevBuf& v, HostCsr& h, std::vector<double>& hv) {
  std::vector<int32_t> rp(P.nrows + 1);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HIP_CHECK(hipMemcpy(rp.data(), P.rowptr.p, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  h.nrows = h.ncols = P.nrows;
  h.rowptr.assign(rp.begin(), rp.end());
  h.cols.resize(P.nnz);
  hv.resize(P.nnz);
  HIP_CHECK(hipMemcpy(h.cols.data(), P.cols.p, P.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(hv.data(), v.p, P.nnz * sizeof(double), hipMemcpyDeviceToHost));
}

}  // namespace

void assemble_galerkin(stokes_ctx* c, MgHier& H) {
  H.lv.clear();
  H.own.clear();
  H.dense_n = 0;
  const int D = c->dim;
  // level 0: B_I Lambda_V^-1 B_I^T + M_Q on the union of the two patterns
  HostCsr X, Q, A;
  std::vector<double> xv, qv, av;
  download_csr(c, c->xl, c->XL_csr, X, xv);
  download_csr(c, c->p1, c->MQ_csr, Q, qv);
  A.nrows = A.ncols = X.nrows;
  A.rowptr.assign(X.nrows + 1, 0);
  for (int64_t r = 0; r < X.nrows; ++r) {
    int64_t i = X.rowptr[r], j = Q.rowptr[r];
    const int64_t ie = X.rowptr[r + 1], je = Q.rowptr[r + 1];
    while (i < ie || j < je) {
      if (j >= je || (i < ie && X.cols[i] < Q.cols[j])) {
        A.cols.push_back(X.cols[i]);
        av.push_back(xv[i++]);
      } else if (i >= ie || Q.cols[j] < X.cols[i]) {
        A.cols.push_back(Q.cols[j]);
        av.push_back(qv[j++]);
      } else {
        A.cols.push_back(X.cols[i]);
        av.push_back(xv[i++] + qv[j++]);
      }
    }
    A.rowptr[r + 1] = static_cast<int64_t>(A.cols.size());
  }
  int n = c->mesh.order == 3 ? 2 * c->mesh.n : c->mesh.n;  // lattice intervals of the pressure nodes
  for (;;) {
    auto L = std::make_unique<MgLevel>();
    L->n = n;
    upload_level(c, A, av, *L);
    const bool p2 = c->mesh.order == 3 && H.lv.empty();  // the P2 pressure level of a P3/P2 pair
    if (p2) L->bs.lo = L->bs.hi / c->mgx_p2_ratio;
    H.lv.push_back({&L->S, &L->v64, &L->v32, &L->d64, &L->d32, &L->bs, &L->bf, n, &L->v16, L->s16,
                    p2 ? c->mgx_p2_degree : 0});
    H.own.push_back(std::move(L));
    if (!(n % 2 == 0 && n > 2 && ipow(n + 1, D) > c->mg_dense_max)) break;
    HostCsr Ac;
    std::vector<double> acv;
    galerkin_p1(D, n, n / 2, A, av, Ac, acv);
    A = std::move(Ac);
    av = std::move(acv);
    n /= 2;
  }
}

// alpha M + mu L on the interior P2 nodes of a coarse Kuhn mesh (natural
// interior order), for the velocity multigrid.
void assemble_p2_level(stokes_ctx* c, const HostMesh& m, VmgLevel& L) {
  const int D = m.dim;
  HostCsr P2;
  element_pattern(m.p2, m.nloc, m.n_p2, m.p2, m.nloc, m.n_p2, m.n_e, P2);
  std::vector<int32_t> rows, nat2int(m.n_p2, -1);
  for (int64_t v = 0; v < m.n_p2; ++v)
    if (!m.p2_bnd[v]) {
      nat2int[v] = static_cast<int32_t>(rows.size());
      rows.push_back(static_cast<int32_t>(v));
    }
  DevBuf d_vc, d_el, d_p2, d_vol, d_jinv, d_ip, d_il, rp, cols, Mf, Lf;
  upload(d_vc, m.vcoords);
  upload(d_el, m.elems);
  upload(d_p2, m.p2);
  d_vol.alloc(m.n_e * sizeof(double));
  d_jinv.alloc(m.n_e * D * D * sizeof(double));
  if (D == 3) launch(c, m.n_e, k_geom<3>, m.n_e, d_vc.as<double>(), d_el.as<int32_t>(), d_vol.as<double>(), d_jinv.as<double>());
  else launch(c, m.n_e, k_geom<2>, m.n_e, d_vc.as<double>(), d_el.as<int32_t>(), d_vol.as<double>(), d_jinv.as<double>());
  {
    std::vector<int64_t> ptr;
    std::vector<int32_t> lst;
    incidence(m.p2, m.nloc, m.n_e, m.n_p2, ptr, lst);
    upload(d_ip, ptr);
    upload(d_il, lst);
  }
  std::vector<int32_t> rp32(P2.rowptr.begin(), P2.rowptr.end());
  upload(rp, rp32);
  upload(cols, P2.cols);
  const int64_t nnz = P2.rowptr.back();
  Mf.alloc(nnz * sizeof(double));
  Lf.alloc(nnz * sizeof(double));
  HIP_CHECK(hipMemsetAsync(Mf.p, 0, nnz * sizeof(double), c->stream));
  HIP_CHECK(hipMemsetAsync(Lf.p, 0, nnz * sizeof(double), c->stream));
  if (D == 3)
    launch(c, m.n_p2, k_gather_p2<3>, m.n_p2, d_ip.as<int64_t>(), d_il.as<int32_t>(), d_p2.as<int32_t>(),
           d_vol.as<double>(), d_jinv.as<double>(), rp.as<int32_t>(), cols.as<int32_t>(), Mf.as<double>(),
           Lf.as<double>(), (double*)nullptr);
  else
    launch(c, m.n_p2, k_gather_p2<2>, m.n_p2, d_ip.as<int64_t>(), d_il.as<int32_t>(), d_p2.as<int32_t>(),
           d_vol.as<double>(), d_jinv.as<double>(), rp.as<int32_t>(), cols.as<int32_t>(), Mf.as<double>(),
           Lf.as<double>(), (double*)nullptr);
  build_sell(P2, rows, nat2int, nullptr, 1, L.S);
  const int64_t nr = L.S.nrows;
  L.nrows = nr;
  L.v64.alloc(L.S.nnz_pad * sizeof(double));
  launch(c, L.S.nnz_pad, k_fill, L.S.nnz_pad, L.S.src.as<int32_t>(), 1, c->prob.alpha, Mf.as<double>(), c->prob.mu,
         Lf.as<double>(), L.v64.as<double>());
  L.d64.alloc(nr * sizeof(double));
  launch(c, nr, k_dinv, nr, L.S.slice_ptr.as<int64_t>(), L.S.cols.as<int32_t>(), L.v64.as<double>(),
         L.d64.as<double>());
  L.v32.alloc(L.S.nnz_pad * sizeof(float));
  L.d32.alloc(nr * sizeof(float));
  launch(c, L.S.nnz_pad, k_cast<double, float>, L.S.nnz_pad, L.v64.as<double>(), L.v32.as<float>());
  launch(c, nr, k_cast<double, float>, nr, L.d64.as<double>(), L.d32.as<float>());
  double lo, hi, g;
  lanczos_bounds(c, L.S, L.v64.as<double>(), L.d64.as<double>(), std::min<int>(40, (int)nr), lo, hi, g);
  L.bf.hi = std::min(g, 1.1 * hi);
  L.bf.lo = std::max(0.9 * lo, L.bf.hi / 1000.0);
  L.bs.hi = L.bf.hi;
  L.bs.lo = L.bf.hi / c->mg_smooth_ratio;
  HIP_CHECK(hipStreamSynchronize(c->stream));  // the local buffers are freed on return
}

void estimate_bounds(stokes_ctx* c) {
  const int steps = 40;
  double lo, hi, g;
  lanczos_bounds(c, c->sA, c->A64.as<double>(), c->dA64.as<double>(), steps, lo, hi, g);
  c->bA.hi = std::min(g, 1.1 * hi);
  c->bA.lo = std::max(0.9 * lo, c->bA.hi / 1000.0);
  lanczos_bounds(c, c->sQ, c->XQ64.as<double>(), c->dXQ64.as<double>(), steps, lo, hi, g);
  c->bXQ.hi = std::min(g, 1.1 * hi);
  c->bXQ.lo = 0.9 * lo;
  c->bXQ_smooth = {c->bXQ.hi / c->mg_smooth_ratio, c->bXQ.hi};
  lanczos_bounds(c, c->sQ, c->LQ64.as<double>(), c->dLQ64.as<double>(), steps, lo, hi, g);
  c->bLQ.hi = std::min(g, 1.1 * hi);
  c->bLQ.lo = c->bLQ.hi / 100.0;  // L_Q is singular: the constant mode is projected out
}

// Re-form A = alpha M + mu L (SELL values and FP32 copy, diagonal, bounds).
void reform_A(stokes_ctx* c) {
  c->clear_graphs();  // captured Chebyshev coefficients depend on the bounds
  const int64_t n = c->sA.nnz_pad;
  launch(c, n, k_fill, n, c->sA.src.as<int32_t>(), 1, c->prob.alpha, c->M_full.as<double>(), c->prob.mu,
         c->L_full.as<double>(), c->A64.as<double>());
  launch(c, n, k_cast<double, float>, n, c->A64.as<double>(), c->A32.as<float>());
  launch(c, c->sA.nrows, k_dinv, c->sA.nrows, c->sA.slice_ptr.as<int64_t>(), c->sA.cols.as<int32_t>(),
         c->A64.as<double>(), c->dA64.as<double>());
  launch(c, c->n_int, k_cast<double, float>, c->n_int, c->dA64.as<double>(), c->dA32.as<float>());
  launch(c, n, k_scale_cols, n, c->sA.cols.as<int32_t>(), c->A64.as<double>(), c->dA64.as<double>(),
         c->AD64.as<double>(), c->AD32.as<float>(), c->AD16.as<_Float16>());
  build_interleaved(c);
  if (c->strain)
    launch(c, n, k_fill_blk, n, c->dim, c->sA.src.as<int32_t>(), c->prob.alpha, c->prob.mu, c->M_full.as<double>(),
           c->L_full.as<double>(), c->D_full.as<double>(), c->AB64.as<double>(), c->AB32.as<float>());
  double lo, hi, g;
  lanczos_bounds(c, c->sA, c->A64.as<double>(), c->dA64.as<double>(), 40, lo, hi, g);
  c->bA.hi = std::min(g, 1.1 * hi);
  c->bA.lo = std::max(0.9 * lo, c->bA.hi / 1000.0);
  HIP_CHECK(hipStreamSynchronize(c->stream));
}

}  // namespace stokes
