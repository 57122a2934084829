// Host-side setup of the entropy-stable tensor-product DSEM: 1D rules,
// collapsed-coordinate operator tables, PKD transforms, isoparametric geometry
// and facet connectivity.  Everything here runs once per plan on the CPU; the
// results are uploaded to HBM by the plan.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace esd {

constexpr int MAX_DEGREE = 10;

// ---------------------------------------------------------------- 1D (Sec. 2.4)
// Orthonormal Jacobi polynomials P_0..P_n at x for weight (1-x)^a (1+x)^b.
void jacobi(int n, double a, double b, double x, double* P);
// Their derivatives.
void jacobi_deriv(int n, double a, double b, double x, double* dP);
// q+1 Gauss nodes (zeros of P_{q+1}^{(a,b)}) and weights.
void gauss_jacobi(int q, double a, double b, std::vector<double>& x, std::vector<double>& w);

// Lagrange basis on a node set, barycentric form.
struct Lagrange1D {
  std::vector<double> x, lam;
  explicit Lagrange1D(const std::vector<double>& nodes);
  void eval(double t, double* out) const;            // l_j(t), j = 0..n-1
  std::vector<double> diff_matrix() const;           // D[i*n+j] = l_j'(x_i)
};

// ---------------------------------------------------------------- reference element
struct RefTables {
  int dim = 0, p = 0, Q = 0, NQ = 0, NP = 0, NF = 0, NQF = 0, NFQ = 0;
  std::vector<double> xl, wl, xj, wj;        // LG and GJ(1,0) nodes / weights
  std::vector<double> psi1, psi2, psi3;      // PKD principal functions at the line nodes
  std::vector<double> psiM;                  // [P+1][Q][Q] psi2 (tri) / psi3 (tet) line compositions, sum_b psi[a][b] psi[a][b]^T
  std::vector<double> lgm1, lgp1, gjm1;      // l(-1), l(+1) on LG; l(-1) on GJ
  std::vector<double> I42;                   // [j][k] = l^LG_k(eta^GJ_j)
  std::vector<double> A;                     // [5][Q][Q] skew line matrices
  std::vector<double> wf;                    // [NF][NQF] facet weights
  std::vector<double> xi;                    // [NQ][dim] volume nodes (reference)
  std::vector<double> xif;                   // [NF][NQF][dim] facet nodes (reference)
  std::vector<double> w;                     // [NQ] volume weights
  std::vector<double> nhat;                  // [NF][dim]
  std::vector<int32_t> mode_a;               // [NP][3] multi-indices
};
RefTables build_ref_tables(int dim, int p);
// Reference point of facet `face` at facet coordinates (s, t): s along the
// facet's Legendre direction, t (tetrahedra) the Gauss-Jacobi direction
// towards the facet's collapse vertex; the facet nodes are (xl[a], xj[b]).
void facet_point(int dim, int face, double s, double t, double* xi);

// PKD basis and gradient at reference points (Sec. 4.3).
int n_modes(int dim, int p);
void pkd_eval(int dim, int p, const double* xi, int npts, double* V /*[npts][NP]*/);
void pkd_grad(int dim, int p, const double* xi, int npts, double* dV /*[dim][npts][NP]*/);

// ---------------------------------------------------------------- mesh + geometry
struct HostGeometry {
  int dim = 0, p = 0;
  int64_t ne = 0;
  std::vector<int64_t> vids;                 // oriented [ne][dim+1]
  std::vector<double> vx;                    // oriented [ne][dim+1][dim]
  std::vector<double> x_vol, J, G;           // [ne][NQ][dim], [ne][NQ], [ne][NQ][dim][dim]
  std::vector<double> nJ, Jf, x_fac;         // [ne][NF][NQF][dim], [ne][NF][NQF], [ne][NF][NQF][dim]
  std::vector<int64_t> nbr;                  // [ne][NF][NQF] neighbour (e*NF + f)*NQF + node
};

typedef void (*warp_fn)(int64_t n, const double* xin, double* xout, void* ctx);

// Returns 0 or a negative esd_status; msg receives a description.  With
// connect = false the facet connectivity (nbr) is not built (elements of one
// degree out of a mixed-degree mesh).
int build_geometry(const RefTables& ref, int64_t ne, const int64_t* ids, const double* coords,
                   warp_fn warp, void* ctx, HostGeometry& out, std::string& msg, bool connect = true);

}  // namespace esd
