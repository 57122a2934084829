// Host-side setup: 1D rules, reference tables, PKD basis, geometry, connectivity.
//
// Formulas follow the paper: normalized Jacobi polynomials and Gauss rules
// (Sec. 2.4), collapsed-coordinate nodes, weights, facets and the sparse line
// structure of the SBP operators (Sec. 3.1-3.2, eqs. d_2d, d_3d, r_2d, r_3d),
// the PKD principal functions (eq. principal_functions), the isoparametric map
// (eq. poly_mapping), exact 2D metrics and conservative curl-form 3D metrics
// (eqs. metric_interpolants, conservative_curl), Nanson normals (eq. nanson),
// and the interpolated Jacobian (eq. jacobian_approx).
#include "host_setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>
#include <unordered_map>

namespace esd {

// ============================================================ 1D
static double gamma0(double a, double b) {
  return std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) / std::tgamma(a + b + 2.0);
}

void jacobi(int n, double a, double b, double x, double* P) {
  // three-term recurrence of the orthonormal Jacobi polynomials
  const double g0 = gamma0(a, b);
  P[0] = 1.0 / std::sqrt(g0);
  if (n == 0) return;
  const double g1 = (a + 1.0) * (b + 1.0) / (a + b + 3.0) * g0;
  P[1] = ((a + b + 2.0) * x / 2.0 + (a - b) / 2.0) / std::sqrt(g1);
  if (n == 1) return;
  double aold = 2.0 / (2.0 + a + b) * std::sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0));
  for (int i = 1; i < n; ++i) {
    const double h1 = 2.0 * i + a + b;
    const double anew = 2.0 / (h1 + 2.0) *
        std::sqrt((i + 1.0) * (i + 1.0 + a + b) * (i + 1.0 + a) * (i + 1.0 + b) / ((h1 + 1.0) * (h1 + 3.0)));
    const double bnew = -(a * a - b * b) / (h1 * (h1 + 2.0));
    P[i + 1] = (-aold * P[i - 1] + (x - bnew) * P[i]) / anew;
    aold = anew;
  }
}

void jacobi_deriv(int n, double a, double b, double x, double* dP) {
  dP[0] = 0.0;
  if (n == 0) return;
  std::vector<double> Q(n);
  jacobi(n - 1, a + 1.0, b + 1.0, x, Q.data());
  for (int k = 1; k <= n; ++k) dP[k] = std::sqrt(k * (k + a + b + 1.0)) * Q[k - 1];
}

void gauss_jacobi(int q, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  // zeros of P_{q+1}^{(a,b)} by Newton's method with deflation of the roots
  // already found, started from Chebyshev points (Karniadakis & Sherwin, App. B)
  const int n = q + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  std::vector<double> P(n + 1), dP(n + 1);
  for (int k = 0; k < n; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    if (k > 0) r = 0.5 * (r + x[k - 1]);
    for (int it = 0; it < 200; ++it) {
      jacobi(n, a, b, r, P.data());
      jacobi_deriv(n, a, b, r, dP.data());
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += 1.0 / (r - x[i]);
      const double delta = -P[n] / (dP[n] - s * P[n]);
      r += delta;
      if (std::fabs(delta) < 1e-16) break;
    }
    x[k] = r;
  }
  // polish without deflation
  for (int k = 0; k < n; ++k) {
    double r = x[k];
    for (int it = 0; it < 3; ++it) {
      jacobi(n, a, b, r, P.data());
      jacobi_deriv(n, a, b, r, dP.data());
      r -= P[n] / dP[n];
    }
    x[k] = r;
  }
  std::sort(x.begin(), x.end());
  // Christoffel numbers for an orthonormal family: w_i = 1 / sum_k P_k(x_i)^2
  for (int i = 0; i < n; ++i) {
    jacobi(n - 1, a, b, x[i], P.data());
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += P[k] * P[k];
    w[i] = 1.0 / s;
  }
}

Lagrange1D::Lagrange1D(const std::vector<double>& nodes) : x(nodes), lam(nodes.size()) {
  const int n = (int)x.size();
  for (int j = 0; j < n; ++j) {
    double pr = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) pr *= (x[j] - x[k]);
    lam[j] = 1.0 / pr;
  }
}

void Lagrange1D::eval(double t, double* out) const {
  const int n = (int)x.size();
  for (int j = 0; j < n; ++j)
    if (t == x[j]) {
      for (int k = 0; k < n; ++k) out[k] = (k == j) ? 1.0 : 0.0;
      return;
    }
  double den = 0.0;
  for (int j = 0; j < n; ++j) {
    out[j] = lam[j] / (t - x[j]);
    den += out[j];
  }
  for (int j = 0; j < n; ++j) out[j] /= den;
}

std::vector<double> Lagrange1D::diff_matrix() const {
  const int n = (int)x.size();
  std::vector<double> D(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
      diag -= D[i * n + j];
    }
    D[i * n + i] = diag;
  }
  return D;
}

// ============================================================ PKD basis
int n_modes(int dim, int p) {
  return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

static void modes(int dim, int p, std::vector<std::array<int, 3>>& out) {
  out.clear();
  for (int a1 = 0; a1 <= p; ++a1)
    for (int a2 = 0; a2 <= p - a1; ++a2) {
      if (dim == 2) {
        out.push_back({a1, a2, 0});
      } else {
        for (int a3 = 0; a3 <= p - a1 - a2; ++a3) out.push_back({a1, a2, a3});
      }
    }
}

// inverse collapsed map; the free coordinate at a collapsed point is -1
static void collapse(int dim, const double* xi, double* eta) {
  if (dim == 2) {
    const double den = 1.0 - xi[1];
    eta[0] = std::fabs(den) > 1e-14 ? 2.0 * (1.0 + xi[0]) / den - 1.0 : -1.0;
    eta[1] = xi[1];
    return;
  }
  const double d3 = 1.0 - xi[2];
  eta[1] = std::fabs(d3) > 1e-14 ? 2.0 * (1.0 + xi[1]) / d3 - 1.0 : -1.0;
  const double d12 = -xi[1] - xi[2];
  eta[0] = std::fabs(d12) > 1e-14 ? 2.0 * (1.0 + xi[0]) / d12 - 1.0 : -1.0;
  eta[2] = xi[2];
}

static inline double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

void pkd_eval(int dim, int p, const double* xi, int npts, double* V) {
  std::vector<std::array<int, 3>> md;
  modes(dim, p, md);
  const int NP = (int)md.size();
  std::vector<double> P1(p + 1), P2(p + 1), P3(p + 1);
  for (int k = 0; k < npts; ++k) {
    double eta[3];
    collapse(dim, xi + k * dim, eta);
    jacobi(p, 0.0, 0.0, eta[0], P1.data());
    for (int m = 0; m < NP; ++m) {
      const int i = md[m][0], j = md[m][1], l = md[m][2];
      jacobi(p, 2.0 * i + 1.0, 0.0, eta[1], P2.data());
      double v = std::sqrt(2.0) * P1[i] * ipow(1.0 - eta[1], i) * P2[j];
      if (dim == 3) {
        jacobi(p, 2.0 * (i + j) + 2.0, 0.0, eta[2], P3.data());
        v *= 2.0 * ipow(1.0 - eta[2], i + j) * P3[l];
      }
      V[(int64_t)k * NP + m] = v;
    }
  }
}

void pkd_grad(int dim, int p, const double* xi, int npts, double* dV) {
  // chain rule through the collapsed coordinates; the singular factors
  // 1/(1-eta2), 1/(1-eta3) are absorbed into the polynomial prefactors
  std::vector<std::array<int, 3>> md;
  modes(dim, p, md);
  const int NP = (int)md.size();
  std::vector<double> P1(p + 1), dP1(p + 1), P2(p + 1), dP2(p + 1), P3(p + 1), dP3(p + 1);
  const double r2 = std::sqrt(2.0);
  for (int k = 0; k < npts; ++k) {
    double eta[3];
    collapse(dim, xi + k * dim, eta);
    const double a = eta[0], b = eta[1], c = dim == 3 ? eta[2] : 0.0;
    jacobi(p, 0.0, 0.0, a, P1.data());
    jacobi_deriv(p, 0.0, 0.0, a, dP1.data());
    for (int m = 0; m < NP; ++m) {
      const int i = md[m][0], j = md[m][1], l = md[m][2];
      jacobi(p, 2.0 * i + 1.0, 0.0, b, P2.data());
      jacobi_deriv(p, 2.0 * i + 1.0, 0.0, b, dP2.data());
      const double f1 = r2 * P1[i], df1 = r2 * dP1[i];
      // psi2 = (1-b)^i P2;  bq = psi2/(1-b);  dpsi2 = d psi2 / db
      const double psi2 = ipow(1.0 - b, i) * P2[j];
      const double bq = i >= 1 ? ipow(1.0 - b, i - 1) * P2[j] : 0.0;
      const double dpsi2 = i >= 1 ? ipow(1.0 - b, i - 1) * (-i * P2[j] + (1.0 - b) * dP2[j]) : dP2[j];
      if (dim == 2) {
        dV[(int64_t)(0 * npts + k) * NP + m] = 2.0 * df1 * bq;
        dV[(int64_t)(1 * npts + k) * NP + m] = (1.0 + a) * df1 * bq + f1 * dpsi2;
        continue;
      }
      const int s = i + j;
      jacobi(p, 2.0 * s + 2.0, 0.0, c, P3.data());
      jacobi_deriv(p, 2.0 * s + 2.0, 0.0, c, dP3.data());
      const double psi3 = 2.0 * ipow(1.0 - c, s) * P3[l];
      const double cq = s >= 1 ? 2.0 * ipow(1.0 - c, s - 1) * P3[l] : 0.0;
      const double dpsi3 = s >= 1 ? 2.0 * ipow(1.0 - c, s - 1) * (-s * P3[l] + (1.0 - c) * dP3[l]) : 2.0 * dP3[l];
      (void)psi3;
      const double A = df1 * bq * cq;       // phi_a / ((1-b)(1-c))
      const double B = f1 * dpsi2 * cq;     // phi_b / (1-c)
      dV[(int64_t)(0 * npts + k) * NP + m] = 4.0 * A;
      dV[(int64_t)(1 * npts + k) * NP + m] = 2.0 * (1.0 + a) * A + 2.0 * B;
      dV[(int64_t)(2 * npts + k) * NP + m] = 2.0 * (1.0 + a) * A + (1.0 + b) * B + f1 * psi2 * dpsi3;
    }
  }
}

// ============================================================ reference tables
static void chi(int dim, const double* eta, double* xi) {
  if (dim == 2) {
    xi[0] = 0.5 * (1.0 + eta[0]) * (1.0 - eta[1]) - 1.0;
    xi[1] = eta[1];
  } else {
    xi[0] = 0.25 * (1.0 + eta[0]) * (1.0 - eta[1]) * (1.0 - eta[2]) - 1.0;
    xi[1] = 0.5 * (1.0 + eta[1]) * (1.0 - eta[2]) - 1.0;
    xi[2] = eta[2];
  }
}

RefTables build_ref_tables(int dim, int p) {
  RefTables R;
  R.dim = dim;
  R.p = p;
  const int Q = p + 1;
  R.Q = Q;
  R.NQ = dim == 2 ? Q * Q : Q * Q * Q;
  R.NP = n_modes(dim, p);
  R.NF = dim + 1;
  R.NQF = dim == 2 ? Q : Q * Q;
  R.NFQ = R.NF * R.NQF;
  gauss_jacobi(p, 0.0, 0.0, R.xl, R.wl);
  gauss_jacobi(p, 1.0, 0.0, R.xj, R.wj);
  const int P1 = p + 1;
  std::vector<double> tmp(p + 1);
  R.psi1.assign(P1 * Q, 0.0);
  R.psi2.assign(P1 * P1 * Q, 0.0);
  R.psi3.assign(P1 * P1 * Q, 0.0);
  for (int i = 0; i < Q; ++i) {
    jacobi(p, 0.0, 0.0, R.xl[i], tmp.data());
    for (int a1 = 0; a1 <= p; ++a1) R.psi1[a1 * Q + i] = std::sqrt(2.0) * tmp[a1];
    for (int a1 = 0; a1 <= p; ++a1) {
      jacobi(p, 2.0 * a1 + 1.0, 0.0, R.xl[i], tmp.data());
      for (int a2 = 0; a2 <= p; ++a2) R.psi2[(a1 * P1 + a2) * Q + i] = ipow(1.0 - R.xl[i], a1) * tmp[a2];
    }
    for (int s = 0; s <= p; ++s) {
      jacobi(p, 2.0 * s + 2.0, 0.0, R.xj[i], tmp.data());
      for (int a3 = 0; a3 <= p; ++a3) R.psi3[(s * P1 + a3) * Q + i] = 2.0 * ipow(1.0 - R.xj[i], s) * tmp[a3];
    }
  }
  // V V^T along the direction V^T contracts last and V first (eta2 of
  // triangles, eta3 of tetrahedra): per line index a (a1, or a1 + a2), the sum
  // over that line's modes b <= p - a of psi[a][b][i] psi[a][b][k]
  R.psiM.assign(P1 * Q * Q, 0.0);
  {
    const std::vector<double>& ps = dim == 2 ? R.psi2 : R.psi3;
    for (int a = 0; a <= p; ++a)
      for (int i = 0; i < Q; ++i)
        for (int k = 0; k < Q; ++k) {
          double acc = 0.0;
          for (int b = 0; b <= p - a; ++b) acc += ps[(a * P1 + b) * Q + i] * ps[(a * P1 + b) * Q + k];
          R.psiM[(a * Q + i) * Q + k] = acc;
        }
  }
  Lagrange1D LG(R.xl), GJ(R.xj);
  R.lgm1.resize(Q);
  R.lgp1.resize(Q);
  R.gjm1.resize(Q);
  LG.eval(-1.0, R.lgm1.data());
  LG.eval(1.0, R.lgp1.data());
  GJ.eval(-1.0, R.gjm1.data());
  R.I42.resize(Q * Q);
  for (int j = 0; j < Q; ++j) LG.eval(R.xj[j], &R.I42[j * Q]);
  // skew line matrices: skew parts of diag(f) W_1D D_1D along each line family
  const std::vector<double> DL = LG.diff_matrix(), DJ = GJ.diff_matrix();
  R.A.assign(5 * Q * Q, 0.0);
  auto skew = [&](int slot, auto f, const std::vector<double>& wts, const std::vector<double>& D) {
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Q; ++b) {
        const double xab = f(a) * wts[a] * D[a * Q + b];
        const double xba = f(b) * wts[b] * D[b * Q + a];
        R.A[(slot * Q + a) * Q + b] = 0.5 * (xab - xba);
      }
  };
  skew(0, [&](int) { return 1.0; }, R.wl, DL);
  skew(1, [&](int a) { return 1.0 + R.xl[a]; }, R.wl, DL);
  skew(2, [&](int a) { return 1.0 - R.xl[a]; }, R.wl, DL);
  skew(3, [&](int a) { return (1.0 - R.xl[a]) * (1.0 + R.xl[a]); }, R.wl, DL);
  skew(4, [&](int a) { return 1.0 - R.xj[a]; }, R.wj, DJ);
  // nodes and weights
  R.xi.resize(R.NQ * dim);
  R.w.resize(R.NQ);
  R.xif.resize(R.NFQ * dim);
  R.wf.resize(R.NFQ);
  if (dim == 2) {
    for (int a2 = 0; a2 < Q; ++a2)
      for (int a1 = 0; a1 < Q; ++a1) {
        const int k = a1 + Q * a2;
        const double eta[2] = {R.xl[a1], R.xl[a2]};
        chi(2, eta, &R.xi[k * 2]);
        R.w[k] = 0.5 * (1.0 - R.xl[a2]) * R.wl[a1] * R.wl[a2];
      }
    for (int i = 0; i < Q; ++i) {
      const double e0[2] = {R.xl[i], -1.0}, e1[2] = {1.0, R.xl[i]}, e2[2] = {-1.0, R.xl[i]};
      chi(2, e0, &R.xif[(0 * Q + i) * 2]);
      chi(2, e1, &R.xif[(1 * Q + i) * 2]);
      chi(2, e2, &R.xif[(2 * Q + i) * 2]);
      R.wf[0 * Q + i] = R.wl[i];
      R.wf[1 * Q + i] = std::sqrt(2.0) * R.wl[i];
      R.wf[2 * Q + i] = R.wl[i];
    }
    const double s2 = 1.0 / std::sqrt(2.0);
    R.nhat = {0.0, -1.0, s2, s2, -1.0, 0.0};
  } else {
    for (int a3 = 0; a3 < Q; ++a3)
      for (int a2 = 0; a2 < Q; ++a2)
        for (int a1 = 0; a1 < Q; ++a1) {
          const int k = a1 + Q * (a2 + Q * a3);
          const double eta[3] = {R.xl[a1], R.xl[a2], R.xj[a3]};
          chi(3, eta, &R.xi[k * 3]);
          R.w[k] = (1.0 - R.xl[a2]) * (1.0 - R.xj[a3]) / 8.0 * R.wl[a1] * R.wl[a2] * R.wj[a3];
        }
    const double fw[4] = {0.5, std::sqrt(3.0) / 2.0, 0.5, 0.5};
    for (int b = 0; b < Q; ++b)
      for (int a = 0; a < Q; ++a) {
        const int j = a + Q * b;
        const double e[4][3] = {{R.xl[a], -1.0, R.xj[b]}, {1.0, R.xl[a], R.xj[b]},
                                {-1.0, R.xl[a], R.xj[b]}, {R.xl[a], R.xj[b], -1.0}};
        for (int f = 0; f < 4; ++f) {
          chi(3, e[f], &R.xif[(f * R.NQF + j) * 3]);
          R.wf[f * R.NQF + j] = fw[f] * R.wl[a] * R.wj[b];
        }
      }
    const double s3 = 1.0 / std::sqrt(3.0);
    R.nhat = {0.0, -1.0, 0.0, s3, s3, s3, -1.0, 0.0, 0.0, 0.0, 0.0, -1.0};
  }
  std::vector<std::array<int, 3>> md;
  modes(dim, p, md);
  R.mode_a.resize(md.size() * 3);
  for (size_t m = 0; m < md.size(); ++m)
    for (int k = 0; k < 3; ++k) R.mode_a[m * 3 + k] = md[m][k];
  return R;
}

// ============================================================ interpolation on equispaced simplex nodes
static std::vector<double> equispaced(int dim, int N) {
  std::vector<double> pts;
  if (dim == 2) {
    for (int j = 0; j <= N; ++j)
      for (int i = 0; i <= N - j; ++i) {
        pts.push_back(-1.0 + 2.0 * i / N);
        pts.push_back(-1.0 + 2.0 * j / N);
      }
  } else {
    for (int k = 0; k <= N; ++k)
      for (int j = 0; j <= N - k; ++j)
        for (int i = 0; i <= N - j - k; ++i) {
          pts.push_back(-1.0 + 2.0 * i / N);
          pts.push_back(-1.0 + 2.0 * j / N);
          pts.push_back(-1.0 + 2.0 * k / N);
        }
  }
  return pts;
}

// Lagrange interpolation (degree N, equispaced nodes) to the points X:
// L [npts][Nn] and gradients dL[dim][npts][Nn].  The nodes form the principal
// lattice alpha/N in barycentric coordinates, whose Lagrange basis is the
// product  l_alpha(lambda) = prod_k prod_{j<alpha_k} (N lambda_k - j)/(alpha_k - j).
struct Interp {
  int npts = 0, Nn = 0;
  std::vector<double> L, dL;
};

static Interp lagrange_to(int dim, int N, const std::vector<double>& X) {
  Interp I;
  const std::vector<double> nodes = equispaced(dim, N);
  const int Nn = n_modes(dim, N);
  const int npts = (int)X.size() / dim;
  const int nb = dim + 1;
  // barycentric multi-index of each node
  std::vector<int> alpha((size_t)Nn * nb);
  for (int i = 0; i < Nn; ++i) {
    int s = 0;
    for (int m = 0; m < dim; ++m) {
      const int a = (int)std::lround(0.5 * (1.0 + nodes[i * dim + m]) * N);
      alpha[i * nb + 1 + m] = a;
      s += a;
    }
    alpha[i * nb] = N - s;
  }
  I.npts = npts;
  I.Nn = Nn;
  I.L.assign((size_t)npts * Nn, 0.0);
  I.dL.assign((size_t)dim * npts * Nn, 0.0);
  for (int k = 0; k < npts; ++k) {
    double lam[4];
    double s = 0.0;
    for (int m = 0; m < dim; ++m) {
      lam[1 + m] = 0.5 * (1.0 + X[k * dim + m]);
      s += lam[1 + m];
    }
    lam[0] = 1.0 - s;
    for (int i = 0; i < Nn; ++i) {
      double f[4], df[4];   // factor for each barycentric coordinate and its lambda-derivative
      for (int c = 0; c < nb; ++c) {
        const int a = alpha[i * nb + c];
        double v = 1.0, dv = 0.0;
        for (int j = 0; j < a; ++j) {
          const double t = (N * lam[c] - j) / (a - j);
          dv = dv * t + v * (double)N / (a - j);
          v *= t;
        }
        f[c] = v;
        df[c] = dv;
      }
      double prod = 1.0;
      for (int c = 0; c < nb; ++c) prod *= f[c];
      I.L[(size_t)k * Nn + i] = prod;
      double dl[4];
      for (int c = 0; c < nb; ++c) {
        double o = df[c];
        for (int cc = 0; cc < nb; ++cc)
          if (cc != c) o *= f[cc];
        dl[c] = o;
      }
      // lambda_0 = 1 - sum_m lambda_m, lambda_m = (1 + xi_m)/2
      for (int m = 0; m < dim; ++m) I.dL[((size_t)m * npts + k) * Nn + i] = 0.5 * (dl[1 + m] - dl[0]);
    }
  }
  return I;
}

void facet_point(int dim, int face, double s, double t, double* xi) {
  if (dim == 2) {
    const double e[3][2] = {{s, -1.0}, {1.0, s}, {-1.0, s}};
    chi(2, e[face], xi);
  } else {
    const double e[4][3] = {{s, -1.0, t}, {1.0, s, t}, {-1.0, s, t}, {s, t, -1.0}};
    chi(3, e[face], xi);
  }
}

// ============================================================ geometry
static const int FACET_VERTS[2][4][3] = {
    {{0, 1, -1}, {1, 2, -1}, {0, 2, -1}, {-1, -1, -1}},
    {{0, 1, 3}, {1, 2, 3}, {0, 2, 3}, {0, 1, 2}},
};
// local vertex at which the facet's LG coordinate starts (eta = -1)
static const int FACET_START[2][4] = {{0, 1, 0, -1}, {0, 1, 0, 0}};

static double det(int dim, const double* A /* [c][m] */) {
  if (dim == 2) return A[0] * A[3] - A[1] * A[2];
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

int build_geometry(const RefTables& ref, int64_t ne, const int64_t* ids, const double* coords,
                   warp_fn warp, void* ctx, HostGeometry& out, std::string& msg, bool connect) {
  const int dim = ref.dim, p = ref.p, NQ = ref.NQ, NF = ref.NF, NQF = ref.NQF, NFQ = ref.NFQ;
  const int nv = dim + 1;
  out = HostGeometry();
  out.dim = dim;
  out.p = p;
  out.ne = ne;
  out.vids.resize(ne * nv);
  out.vx.resize(ne * nv * dim);
  // ---- orientation: sort by global id, largest last; swap the first two if
  //      the affine Jacobian is negative
  for (int64_t e = 0; e < ne; ++e) {
    int ord[4] = {0, 1, 2, 3};
    std::sort(ord, ord + nv, [&](int a, int b) { return ids[e * nv + a] < ids[e * nv + b]; });
    double A[9];
    for (int c = 0; c < dim; ++c)
      for (int m = 0; m < dim; ++m)
        A[c * dim + m] = coords[(e * nv + ord[m + 1]) * dim + c] - coords[(e * nv + ord[0]) * dim + c];
    if (det(dim, A) < 0) std::swap(ord[0], ord[1]);
    for (int k = 0; k < nv; ++k) {
      out.vids[e * nv + k] = ids[e * nv + ord[k]];
      for (int c = 0; c < dim; ++c) out.vx[(e * nv + k) * dim + c] = coords[(e * nv + ord[k]) * dim + c];
    }
  }
  // ---- mapping nodes: affine images and the warp displacement there.  The
  //      map is x_h = X + I_p[delta] with X the affine map in element-local
  //      coordinates (relative to the first vertex): interpolation reproduces
  //      X exactly, so only the displacement is interpolated.
  const std::vector<double> Xg = equispaced(dim, p);
  const int Ng = n_modes(dim, p);
  std::vector<double> xm((size_t)ne * Ng * dim), xw((size_t)ne * Ng * dim);
  for (int64_t e = 0; e < ne; ++e)
    for (int g = 0; g < Ng; ++g) {
      double lam[4];
      double s = 0.0;
      for (int k = 1; k < nv; ++k) {
        lam[k] = 0.5 * (1.0 + Xg[g * dim + k - 1]);
        s += lam[k];
      }
      lam[0] = 1.0 - s;
      for (int c = 0; c < dim; ++c) {
        double x = 0.0;
        for (int k = 0; k < nv; ++k) x += lam[k] * out.vx[(e * nv + k) * dim + c];
        xm[((size_t)e * Ng + g) * dim + c] = x;
      }
    }
  if (warp)
    warp(ne * Ng, xm.data(), xw.data(), ctx);
  else
    xw = xm;
  // ---- interpolation operators (closed-form lattice Lagrange basis)
  std::vector<double> Xf(ref.xif);
  const Interp Ig = lagrange_to(dim, p, Xg);         // gradients at mapping nodes
  const Interp Iv = lagrange_to(dim, p, ref.xi);     // to volume nodes
  const Interp If = lagrange_to(dim, p, Xf);         // to facet nodes
  Interp Ic, Icv, Icf;                               // 3D curl form
  int Nc = 0;
  std::vector<double> Xc;
  if (dim == 3) {
    Xc = equispaced(3, p + 1);
    Nc = n_modes(3, p + 1);
    Ic = lagrange_to(3, p, Xc);
    Icv = lagrange_to(3, p + 1, ref.xi);
    Icf = lagrange_to(3, p + 1, Xf);
  }
  out.x_vol.assign((size_t)ne * NQ * dim, 0.0);
  out.J.assign((size_t)ne * NQ, 0.0);
  out.G.assign((size_t)ne * NQ * dim * dim, 0.0);
  out.nJ.assign((size_t)ne * NFQ * dim, 0.0);
  out.Jf.assign((size_t)ne * NFQ, 0.0);
  out.x_fac.assign((size_t)ne * NFQ * dim, 0.0);
  std::vector<int> bad(ne, 0);

  auto work = [&](int64_t e0, int64_t e1) {
    std::vector<double> dl((size_t)Ng * dim), Jm(Ng), Xa, dc, gdc, r1, r2, r3;
    if (dim == 3) {
      Xa.resize((size_t)Nc * 3);
      dc.resize((size_t)Nc * 3);
      gdc.resize((size_t)Nc * 9);
      r1.resize((size_t)Nc * 3);
      r2.resize((size_t)Nc * 3);
      r3.resize((size_t)Nc * 3);
    }
    for (int64_t e = e0; e < e1; ++e) {
      const double* vxe = &out.vx[(size_t)e * nv * dim];
      // A[c][m] = d X_c / d xi_m (constant), X(xi) = A (1 + xi)
      double A[9];
      for (int c = 0; c < dim; ++c)
        for (int m = 0; m < dim; ++m) A[c * dim + m] = 0.5 * (vxe[(m + 1) * dim + c] - vxe[c]);
      auto Xloc = [&](const double* xi, int c) {
        double s = 0.0;
        for (int m = 0; m < dim; ++m) s += A[c * dim + m] * (1.0 + xi[m]);
        return s;
      };
      for (int g = 0; g < Ng; ++g)
        for (int c = 0; c < dim; ++c)
          dl[g * dim + c] = xw[((size_t)e * Ng + g) * dim + c] - xm[((size_t)e * Ng + g) * dim + c];
      // gradient of x_h = A + grad I[delta] at the mapping nodes; J interpolated (eq. jacobian_approx)
      for (int g = 0; g < Ng; ++g) {
        double D[9];
        for (int i = 0; i < dim * dim; ++i) D[i] = A[i];
        for (int m = 0; m < dim; ++m)
          for (int k = 0; k < Ng; ++k) {
            const double d = Ig.dL[((size_t)m * Ng + g) * Ng + k];
            for (int c = 0; c < dim; ++c) D[c * dim + m] += d * dl[k * dim + c];
          }
        Jm[g] = det(dim, D);
        if (!(Jm[g] > 0)) bad[e] = 1;
      }
      for (int i = 0; i < NQ; ++i) {
        double J = 0.0;
        for (int k = 0; k < Ng; ++k) J += Iv.L[(size_t)i * Ng + k] * Jm[k];
        out.J[(size_t)e * NQ + i] = J;
        if (!(J > 0)) bad[e] = 1;
        for (int c = 0; c < dim; ++c) {
          double x = 0.0;
          for (int k = 0; k < Ng; ++k) x += Iv.L[(size_t)i * Ng + k] * dl[k * dim + c];
          out.x_vol[((size_t)e * NQ + i) * dim + c] = vxe[c] + Xloc(&ref.xi[i * dim], c) + x;
        }
      }
      for (int j = 0; j < NFQ; ++j)
        for (int c = 0; c < dim; ++c) {
          double x = 0.0;
          for (int k = 0; k < Ng; ++k) x += If.L[(size_t)j * Ng + k] * dl[k * dim + c];
          out.x_fac[((size_t)e * NFQ + j) * dim + c] = vxe[c] + Xloc(&Xf[j * dim], c) + x;
        }
      auto cross = [](const double* a, const double* b, double* o) {
        o[0] = a[1] * b[2] - a[2] * b[1];
        o[1] = a[2] * b[0] - a[0] * b[2];
        o[2] = a[0] * b[1] - a[1] * b[0];
      };
      // metric terms at point t of a target set (volume or facet nodes)
      auto metrics = [&](const Interp& I2, const Interp& I3, int npts, int t, double* G) {
        if (dim == 2) {
          double D[4] = {A[0], A[1], A[2], A[3]};
          for (int m = 0; m < 2; ++m)
            for (int k = 0; k < Ng; ++k) {
              const double d = I2.dL[((size_t)m * npts + t) * Ng + k];
              for (int c = 0; c < 2; ++c) D[c * 2 + m] += d * dl[k * 2 + c];
            }
          // adjugate: G_lm = J dxi_l/dx_m
          G[0] = D[3];
          G[1] = -D[1];
          G[2] = -D[2];
          G[3] = D[0];
          return;
        }
        // curl form: r1 = x3 grad x2, r2 = x3 grad x1, r3 = x1 grad x2 with
        // x = X + delta; the affine-affine products are linear and have curl
        // grad X_a x grad X_b, the rest is interpolated with degree q+1
        double d1[3][3] = {{0}}, d2[3][3] = {{0}}, d3[3][3] = {{0}};  // [m][comp]
        for (int m = 0; m < 3; ++m)
          for (int k = 0; k < Nc; ++k) {
            const double d = I3.dL[((size_t)m * npts + t) * Nc + k];
            for (int c = 0; c < 3; ++c) {
              d1[m][c] += d * r1[k * 3 + c];
              d2[m][c] += d * r2[k * 3 + c];
              d3[m][c] += d * r3[k * 3 + c];
            }
          }
        auto curl = [](double d[3][3], double* o) {
          o[0] = d[1][2] - d[2][1];
          o[1] = d[2][0] - d[0][2];
          o[2] = d[0][1] - d[1][0];
        };
        double c1[3], c2[3], c3[3], a32[3], a31[3], a12[3];
        curl(d1, c1);
        curl(d2, c2);
        curl(d3, c3);
        const double* g1 = &A[0];
        const double* g2 = &A[3];
        const double* g3 = &A[6];
        cross(g3, g2, a32);
        cross(g3, g1, a31);
        cross(g1, g2, a12);
        for (int l = 0; l < 3; ++l) {
          G[l * 3 + 0] = -(a32[l] + c1[l]);
          G[l * 3 + 1] = a31[l] + c2[l];
          G[l * 3 + 2] = a12[l] + c3[l];
        }
      };
      if (dim == 3) {
        for (int k = 0; k < Nc; ++k) {
          for (int c = 0; c < 3; ++c) {
            Xa[k * 3 + c] = Xloc(&Xc[k * 3], c);
            double x = 0.0;
            for (int g = 0; g < Ng; ++g) x += Ic.L[(size_t)k * Ng + g] * dl[g * 3 + c];
            dc[k * 3 + c] = x;
          }
          for (int c = 0; c < 3; ++c)
            for (int m = 0; m < 3; ++m) {
              double s = 0.0;
              for (int g = 0; g < Ng; ++g) s += Ic.dL[((size_t)m * Nc + k) * Ng + g] * dl[g * 3 + c];
              gdc[k * 9 + c * 3 + m] = s;
            }
          // x_a grad x_b without the X_a grad X_b part
          auto rv = [&](int a, int b, double* r) {
            for (int m = 0; m < 3; ++m)
              r[k * 3 + m] = Xa[k * 3 + a] * gdc[k * 9 + b * 3 + m] + dc[k * 3 + a] * A[b * 3 + m] +
                             dc[k * 3 + a] * gdc[k * 9 + b * 3 + m];
          };
          rv(2, 1, r1.data());
          rv(2, 0, r2.data());
          rv(0, 1, r3.data());
        }
      }
      for (int i = 0; i < NQ; ++i) metrics(Iv, Icv, NQ, i, &out.G[((size_t)e * NQ + i) * dim * dim]);
      for (int j = 0; j < NFQ; ++j) {
        double G[9];
        metrics(If, Icf, NFQ, j, G);
        const int f = j / NQF;
        double nrm = 0.0;
        for (int m = 0; m < dim; ++m) {
          double s = 0.0;
          for (int l = 0; l < dim; ++l) s += ref.nhat[f * dim + l] * G[l * dim + m];
          out.nJ[((size_t)e * NFQ + j) * dim + m] = s;
          nrm += s * s;
        }
        out.Jf[(size_t)e * NFQ + j] = std::sqrt(nrm);
      }
    }
  };
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (ne < 64) nth = 1;
  std::vector<std::thread> pool;
  const int64_t chunk = (ne + nth - 1) / nth;
  for (unsigned t = 0; t < nth; ++t) {
    const int64_t e0 = t * chunk, e1 = std::min<int64_t>(ne, e0 + chunk);
    if (e0 < e1) pool.emplace_back(work, e0, e1);
  }
  for (auto& th : pool) th.join();
  for (int64_t e = 0; e < ne; ++e)
    if (bad[e]) {
      msg = "mapping Jacobian not positive in element " + std::to_string(e);
      return -2;  // ESD_EJACOBIAN
    }
  if (!connect) return 0;
  // ---- connectivity: match facets by their sorted global vertex ids
  const int di = dim - 2;
  std::map<std::array<int64_t, 3>, std::vector<std::pair<int64_t, int>>> table;
  for (int64_t e = 0; e < ne; ++e)
    for (int f = 0; f < NF; ++f) {
      std::array<int64_t, 3> key = {-1, -1, -1};
      for (int k = 0; k < dim; ++k) key[k] = out.vids[e * nv + FACET_VERTS[di][f][k]];
      std::sort(key.begin(), key.begin() + dim);
      table[key].push_back({e, f});
    }
  out.nbr.assign((size_t)ne * NFQ, -1);
  const int Q = ref.Q;
  for (auto& kv : table) {
    if (kv.second.size() != 2) {
      msg = "facet shared by " + std::to_string(kv.second.size()) + " elements";
      return -5;  // ESD_ENONCONFORMING
    }
    for (int s = 0; s < 2; ++s) {
      const int64_t ea = kv.second[s].first, eb = kv.second[1 - s].first;
      const int fa = kv.second[s].second, fb = kv.second[1 - s].second;
      const bool flip = out.vids[ea * nv + FACET_START[di][fa]] != out.vids[eb * nv + FACET_START[di][fb]];
      if (dim == 3 && out.vids[ea * nv + FACET_VERTS[di][fa][2]] != out.vids[eb * nv + FACET_VERTS[di][fb][2]]) {
        msg = "facet collapse vertices differ";
        return -5;
      }
      double shift[3] = {0, 0, 0};
      for (int j = 0; j < NQF; ++j) {
        const int a1 = j % Q, a2 = j / Q;
        const int b1 = flip ? (Q - 1 - a1) : a1;
        const int jb = dim == 2 ? b1 : b1 + Q * a2;
        out.nbr[(size_t)ea * NFQ + fa * NQF + j] = ((int64_t)eb * NF + fb) * NQF + jb;
        // the matched physical nodes must coincide up to one periodic shift
        for (int c = 0; c < dim; ++c) {
          const double d = out.x_fac[((size_t)ea * NFQ + fa * NQF + j) * dim + c] -
                           out.x_fac[((size_t)eb * NFQ + fb * NQF + jb) * dim + c];
          if (j == 0) shift[c] = d;
          if (std::fabs(d - shift[c]) > 1e-9 * (1.0 + std::fabs(shift[c]))) {
            msg = "facet nodes of neighbours do not coincide";
            return -5;
          }
        }
      }
    }
  }
  return 0;
}

}  // namespace esd
