// Host build of the library's physics header (the same source the kernels
// include), exported with C linkage so that tests can compare its fluxes and
// hand-written vector-Jacobian products with the oracle's autograd.
// Built by tests/test_physics_host.py with g++; not part of the library.
#include "physics.hpp"

using namespace esd;

namespace {
template <int DIM>
bool node_from_w(const double* w, double gamma, Node<DIM>& n) {
  return from_entropy<DIM>(w, gamma, 1.0 / (gamma - 1.0), n);
}

template <int DIM, int FLUX>
void flux_batch(int64_t m, const double* wa, const double* wb, const double* nrm, const double* Jf, double gamma,
                int diss, int iface, double* F) {
  constexpr int NC = DIM + 2;
  const double g = 1.0 / (gamma - 1.0);
  for (int64_t k = 0; k < m; ++k) {
    Node<DIM> A, B;
    node_from_w<DIM>(wa + k * NC, gamma, A);
    node_from_w<DIM>(wb + k * NC, gamma, B);
    if (iface)
      interface_flux<DIM, FLUX>(A, B, nrm + k * DIM, Jf[k], gamma, g, diss, F + k * NC, wa + k * NC, wb + k * NC);
    else
      ec_flux<DIM, FLUX>(A, B, nrm + k * DIM, g, F + k * NC);
  }
}

template <int DIM, int FLUX>
void flux_vjp_batch(int64_t m, const double* wa, const double* wb, const double* nrm, const double* Jf,
                    double gamma, int diss, int iface, const double* Fb, double* wab, double* wbb) {
  constexpr int NC = DIM + 2;
  const double g = 1.0 / (gamma - 1.0);
  for (int64_t k = 0; k < m; ++k) {
    Node<DIM> A, B;
    node_from_w<DIM>(wa + k * NC, gamma, A);
    node_from_w<DIM>(wb + k * NC, gamma, B);
    NodeBar<DIM> Ab, Bb;
    zero(Ab);
    zero(Bb);
    if (iface)
      interface_flux_vjp<DIM, FLUX>(A, B, nrm + k * DIM, Jf[k], gamma, g, diss, Fb + k * NC, Ab, Bb);
    else
      ec_flux_vjp<DIM, FLUX>(A, B, nrm + k * DIM, g, Fb + k * NC, Ab, Bb);
    double xa[NC], xb[NC];
    reduce_bar<DIM>(A, Ab, xa);
    reduce_bar<DIM>(B, Bb, xb);
    xbar_to_wbar<DIM>(A, xa, g, wab + k * NC);
    xbar_to_wbar<DIM>(B, xb, g, wbb + k * NC);
  }
}
}  // namespace

extern "C" {

// F[k] = f#(U(wa_k), U(wb_k), n_k) (iface = 0) or the interface flux with
// nJ = n_k, J_f = Jf_k (iface = 1); returns the number of inadmissible states
int ph_flux(int dim, int flux, int64_t m, const double* wa, const double* wb, const double* nrm, const double* Jf,
            double gamma, int diss, int iface, double* F) {
  if (dim == 2 && flux == 0) flux_batch<2, 0>(m, wa, wb, nrm, Jf, gamma, diss, iface, F);
  else if (dim == 2) flux_batch<2, 1>(m, wa, wb, nrm, Jf, gamma, diss, iface, F);
  else if (flux == 0) flux_batch<3, 0>(m, wa, wb, nrm, Jf, gamma, diss, iface, F);
  else flux_batch<3, 1>(m, wa, wb, nrm, Jf, gamma, diss, iface, F);
  return 0;
}

// cotangents of wa and wb for the output cotangent Fb
void ph_flux_vjp(int dim, int flux, int64_t m, const double* wa, const double* wb, const double* nrm,
                 const double* Jf, double gamma, int diss, int iface, const double* Fb, double* wab, double* wbb) {
  if (dim == 2 && flux == 0) flux_vjp_batch<2, 0>(m, wa, wb, nrm, Jf, gamma, diss, iface, Fb, wab, wbb);
  else if (dim == 2) flux_vjp_batch<2, 1>(m, wa, wb, nrm, Jf, gamma, diss, iface, Fb, wab, wbb);
  else if (flux == 0) flux_vjp_batch<3, 0>(m, wa, wb, nrm, Jf, gamma, diss, iface, Fb, wab, wbb);
  else flux_vjp_batch<3, 1>(m, wa, wb, nrm, Jf, gamma, diss, iface, Fb, wab, wbb);
}

// W(u) and (dW/du)^T wb per point
void ph_entropy_vars(int dim, int64_t m, const double* u, double gamma, double* w) {
  const double g = 1.0 / (gamma - 1.0);
  for (int64_t k = 0; k < m; ++k) {
    if (dim == 2) entropy_vars<2>(u + k * 4, gamma, g, w + k * 4);
    else entropy_vars<3>(u + k * 5, gamma, g, w + k * 5);
  }
}
void ph_entropy_vars_vjp(int dim, int64_t m, const double* u, const double* wb, double gamma, double* ub) {
  const double g = 1.0 / (gamma - 1.0);
  const int nc = dim + 2;
  for (int64_t k = 0; k < m; ++k) {
    for (int c = 0; c < nc; ++c) ub[k * nc + c] = 0.0;
    if (dim == 2) entropy_vars_vjp<2>(u + k * 4, wb + k * 4, gamma, g, ub + k * 4);
    else entropy_vars_vjp<3>(u + k * 5, wb + k * 5, gamma, g, ub + k * 5);
  }
}

// log mean, reciprocal log mean and their gradients w.r.t. (a, b) through the
// logs (la = ln a, lb = ln b), for the branch tests
void ph_log_means(int64_t m, const double* a, const double* b, double* L, double* I, double* dL, double* dI) {
  for (int64_t k = 0; k < m; ++k) {
    const double la = log(a[k]), lb = log(b[k]), is = 1.0 / (a[k] + b[k]);
    L[k] = log_mean(a[k], b[k], la, lb, is);
    I[k] = inv_log_mean(a[k], b[k], la, lb, is);
    double g[4];
    log_mean_grad(a[k], b[k], la, lb, g);
    dL[2 * k] = g[0] + g[2] / a[k];
    dL[2 * k + 1] = g[1] + g[3] / b[k];
    inv_log_mean_grad(a[k], b[k], la, lb, g);
    dI[2 * k] = g[0] + g[2] / a[k];
    dI[2 * k + 1] = g[1] + g[3] / b[k];
  }
}
}
