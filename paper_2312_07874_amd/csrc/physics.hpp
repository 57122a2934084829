// Euler physics of the entropy-stable scheme, forward and vector-Jacobian
// products, as pure functions usable from device and host code.
//
//  - entropy variables W = dS/dU of S = -rho s/(gamma-1), s = ln p - gamma ln rho
//    (eq. euler_entropy) and their inverse U(W);
//  - logarithmic mean (a+ - a-)/(ln a+ - ln a-) and its reciprocal, with a
//    series for nearly equal arguments;
//  - Ranocha's entropy-conservative flux (eq. ranocha_flux; the 1/2 of the
//    energy component multiplies v-.v+ only) and Chandrashekar's;
//  - the interface flux f# - lambda/2 [u] with Davis' wave speed (eqs.
//    num_flux, wave_speed), scaled by the facet Jacobian.
// Node states are cached as (rho, ln rho, b = rho/p, ln b, p, v).
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define ESD_HD __host__ __device__ __forceinline__
#else
#define ESD_HD inline
#endif

namespace esd {

constexpr int FLUX_RANOCHA = 0;
constexpr int FLUX_CHANDRASHEKAR = 1;
constexpr double LOG_SERIES_THRESHOLD = 1.0e-4;

template <int DIM>
struct Node {
  double rho, lnrho, b, lnb, p, v[DIM];
};

// cotangent of a node state, same fields
template <int DIM>
struct NodeBar {
  double rho, lnrho, b, lnb, p, v[DIM];
};

template <int DIM>
ESD_HD void zero(NodeBar<DIM>& x) {
  x.rho = x.lnrho = x.b = x.lnb = x.p = 0.0;
  for (int i = 0; i < DIM; ++i) x.v[i] = 0.0;
}

// 1/x: hardware reciprocal estimate refined by two Newton-Raphson steps
// (each squares the relative error), correct to within an ulp
ESD_HD double frcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
#else
  return 1.0 / x;
#endif
}

// U(w): entropy-projected state from entropy variables w = (w1, w_v, w_last).
// b = -w_last = rho/p, v = w_v/b, s = gamma - (gamma-1)(w1 + b|v|^2/2),
// ln rho = -(s + ln b)/(gamma-1), p = rho/b.  Returns false if inadmissible.
template <int DIM>
ESD_HD bool from_entropy(const double* w, double gamma, double gm1_inv, Node<DIM>& n) {
  const double b = -w[DIM + 1];
  const double ib = frcp(b);
  double v2 = 0.0;
  for (int i = 0; i < DIM; ++i) {
    n.v[i] = w[1 + i] * ib;
    v2 += n.v[i] * n.v[i];
  }
  const double s = gamma - (gamma - 1.0) * (w[0] + 0.5 * b * v2);
  n.b = b;
  n.lnb = log(b);
  n.lnrho = -(s + n.lnb) * gm1_inv;
  n.rho = exp(n.lnrho);
  n.p = n.rho * ib;
  return (b > 0.0) && __builtin_isfinite(n.rho) && __builtin_isfinite(n.p) && (n.rho > 0.0);
}

// Node cotangents in the independent parameterisation x = (ln rho, ln b, v)
// (rho = e^{ln rho}, b = e^{ln b}, p = e^{ln rho - ln b}): NC numbers per node
template <int DIM>
ESD_HD void reduce_bar(const Node<DIM>& n, const NodeBar<DIM>& nb, double* xb) {
  xb[0] = nb.lnrho + n.rho * nb.rho + n.p * nb.p;
  xb[1] = nb.lnb + n.b * nb.b - n.p * nb.p;
  for (int i = 0; i < DIM; ++i) xb[2 + i] = nb.v[i];
}

// w_bar = (dx/dw)^T x_bar for the node n = U(w):
//   ln b = ln(-w_last), v = w_v / b, ln rho = w1 - gamma/(gamma-1) + |w_v|^2/(2b) - ln b/(gamma-1)
template <int DIM>
ESD_HD void xbar_to_wbar(const Node<DIM>& n, const double* xb, double gm1_inv, double* wb) {
  const double ib = frcp(n.b);
  const double L = xb[0];
  double v2 = 0.0, vx = 0.0;
  for (int i = 0; i < DIM; ++i) {
    v2 += n.v[i] * n.v[i];
    vx += n.v[i] * xb[2 + i];
    wb[1 + i] = L * n.v[i] + xb[2 + i] * ib;
  }
  wb[0] = L;
  // cotangent of b as the independent variable, b = -w_last
  wb[DIM + 1] = -((xb[1] - vx) * ib - L * (0.5 * v2 + gm1_inv * ib));
}

// entropy variables from conservative u = (rho, m, E)
template <int DIM>
ESD_HD void entropy_vars(const double* u, double gamma, double gm1_inv, double* w) {
  const double rho = u[0];
  double m2 = 0.0;
  for (int i = 0; i < DIM; ++i) m2 += u[1 + i] * u[1 + i];
  const double p = (gamma - 1.0) * (u[DIM + 1] - 0.5 * m2 / rho);
  const double s = log(p) - gamma * log(rho);
  w[0] = (gamma - s) * gm1_inv - 0.5 * m2 / (rho * p);
  for (int i = 0; i < DIM; ++i) w[1 + i] = u[1 + i] / p;
  w[DIM + 1] = -rho / p;
}

// u_bar += (dW/du)^T w_bar
template <int DIM>
ESD_HD void entropy_vars_vjp(const double* u, const double* wb, double gamma, double gm1_inv, double* ub) {
  const double rho = u[0];
  double m2 = 0.0;
  for (int i = 0; i < DIM; ++i) m2 += u[1 + i] * u[1 + i];
  const double p = (gamma - 1.0) * (u[DIM + 1] - 0.5 * m2 * frcp(rho));
  const double ip = frcp(p), ir = frcp(rho);
  // w1 = g(gamma - ln p + gamma ln rho) - m2/(2 rho p); w_v = m/p; w_last = -rho/p
  double pb = wb[0] * (-gm1_inv * ip + 0.5 * m2 * ir * ip * ip) + wb[DIM + 1] * rho * ip * ip;
  for (int i = 0; i < DIM; ++i) pb -= wb[1 + i] * u[1 + i] * ip * ip;
  double rb = wb[0] * (gm1_inv * gamma * ir + 0.5 * m2 * ir * ir * ip) - wb[DIM + 1] * ip;
  // p = (gamma-1)(E - m2/(2 rho))
  rb += pb * (gamma - 1.0) * 0.5 * m2 * ir * ir;
  ub[0] += rb;
  for (int i = 0; i < DIM; ++i)
    ub[1 + i] += -wb[0] * u[1 + i] * ir * ip + wb[1 + i] * ip - pb * (gamma - 1.0) * u[1 + i] * ir;
  ub[DIM + 1] += pb * (gamma - 1.0);
}

// ---------------------------------------------------------------- logarithmic means
// {a}_ln = (a- + a+)/2 * f/atanh f  (series: 1 - u/3 - 4u^2/45 - 44u^3/945, u = f^2),
// 1/{a}_ln = 2 (1 + u/3 + u^2/5 + u^3/7)/(a- + a+); truncation below 3e-18.
// inv_s = 1/(a- + a+).
ESD_HD double log_mean(double a, double b, double la, double lb, double inv_s) {
  const double d = b - a;
  const double f = d * inv_s, u = f * f;
  if (u < LOG_SERIES_THRESHOLD) return 0.5 * (a + b) * (1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0))));
  return d / (lb - la);
}
ESD_HD double inv_log_mean(double a, double b, double la, double lb, double inv_s) {
  const double d = b - a;
  const double f = d * inv_s, u = f * f;
  if (u < LOG_SERIES_THRESHOLD) return 2.0 * (1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)))) * inv_s;
  return (lb - la) / d;
}

// partial derivatives of the two means w.r.t. (a, b, la, lb) on the branch the
// forward evaluation takes
ESD_HD void log_mean_grad(double a, double b, double la, double lb, double* g) {
  const double s = a + b, d = b - a, is = frcp(s);
  const double f = d * is, u = f * f;
  if (u < LOG_SERIES_THRESHOLD) {
    const double t = 1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0)));
    const double dt = -(1.0 / 3.0 + u * (8.0 / 45.0 + u * (132.0 / 945.0)));
    // du/da = 2 f df/da, df/da = -2b/s^2, df/db = 2a/s^2
    const double dua = 2.0 * f * (-2.0 * b * is * is), dub = 2.0 * f * (2.0 * a * is * is);
    g[0] = 0.5 * t + 0.5 * s * dt * dua;
    g[1] = 0.5 * t + 0.5 * s * dt * dub;
    g[2] = g[3] = 0.0;
    return;
  }
  const double il = frcp(lb - la), L = d * il;
  g[0] = -il;
  g[1] = il;
  g[2] = L * il;
  g[3] = -L * il;
}
ESD_HD void inv_log_mean_grad(double a, double b, double la, double lb, double* g) {
  const double s = a + b, d = b - a, is = frcp(s);
  const double f = d * is, u = f * f;
  if (u < LOG_SERIES_THRESHOLD) {
    const double S = 1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)));
    const double dS = 1.0 / 3.0 + u * (2.0 / 5.0 + u * (3.0 / 7.0));
    const double dua = 2.0 * f * (-2.0 * b * is * is), dub = 2.0 * f * (2.0 * a * is * is);
    g[0] = 2.0 * dS * dua * is - 2.0 * S * is * is;
    g[1] = 2.0 * dS * dub * is - 2.0 * S * is * is;
    g[2] = g[3] = 0.0;
    return;
  }
  const double id = frcp(d), I = (lb - la) * id;
  g[0] = I * id;
  g[1] = -I * id;
  g[2] = -id;
  g[3] = id;
}

// Both logarithmic means of a flux pair, {rho}_ln and 1/{b}_ln, branch-free
// with one reciprocal.  The series branch is chosen where d^2 < 1e-4 s^2
// (f^2 < 1e-4); otherwise d / (ln a+ - ln a-) and its reciprocal.  With
// L = ln-difference (or 1 on the series branch), D = difference of b (or 1),
// x = L D and y = s_rho s_b, r = 1/(x y) yields 1/x = r y and 1/y = r x, hence
// 1/L, 1/D, 1/s_rho, 1/s_b by one more product each.
ESD_HD void log_means(double ra, double rb, double lra, double lrb, double ba, double bb, double lba, double lbb,
                      double& rho_ln, double& ib_ln, double& inv_sb) {
  const double dr = rb - ra, sr = ra + rb, db = bb - ba, sb = ba + bb;
  const bool ser_r = dr * dr < LOG_SERIES_THRESHOLD * (sr * sr);
  const bool ser_b = db * db < LOG_SERIES_THRESHOLD * (sb * sb);
  const double Lr = ser_r ? 1.0 : (lrb - lra);
  const double Db = ser_b ? 1.0 : db;
  const double x = Lr * Db, y = sr * sb;
  const double r = frcp(x * y);
  const double ix = r * y, iy = r * x;
  const double inv_sr = iy * sb;
  inv_sb = iy * sr;
  const double fr = dr * inv_sr, ur = fr * fr;
  const double fb = db * inv_sb, ub = fb * fb;
  const double ser_rho = 0.5 * sr * (1.0 - ur * (1.0 / 3.0 + ur * (4.0 / 45.0 + ur * (44.0 / 945.0))));
  const double ser_ib = 2.0 * (1.0 + ub * (1.0 / 3.0 + ub * (1.0 / 5.0 + ub * (1.0 / 7.0)))) * inv_sb;
  rho_ln = ser_r ? ser_rho : dr * (ix * Db);
  ib_ln = ser_b ? ser_ib : (lbb - lba) * (ix * Lr);
}

// ---------------------------------------------------------------- EC two-point flux
// directional flux f#(A, B, n) = sum_m n_m f#_m(A, B)
template <int DIM, int FLUX>
ESD_HD void ec_flux(const Node<DIM>& A, const Node<DIM>& B, const double* n, double gm1_inv, double* F) {
  double rho_ln, ib_ln, inv_sb;   // {rho}_ln, 1/{rho/p}_ln, 1/(b- + b+)
  log_means(A.rho, B.rho, A.lnrho, B.lnrho, A.b, B.b, A.lnb, B.lnb, rho_ln, ib_ln, inv_sb);
  double vavg[DIM];
  double vn = 0.0, vab = 0.0, van = 0.0, vbn = 0.0;
  for (int i = 0; i < DIM; ++i) {
    vavg[i] = 0.5 * (A.v[i] + B.v[i]);
    vn += vavg[i] * n[i];
    vab += A.v[i] * B.v[i];
    van += A.v[i] * n[i];
    vbn += B.v[i] * n[i];
  }
  const double frho = rho_ln * vn;
  F[0] = frho;
  if (FLUX == FLUX_RANOCHA) {
    const double pavg = 0.5 * (A.p + B.p);
    for (int i = 0; i < DIM; ++i) F[1 + i] = frho * vavg[i] + pavg * n[i];
    F[DIM + 1] = frho * (0.5 * vab + ib_ln * gm1_inv) + 0.5 * (A.p * vbn + B.p * van);
  } else {
    const double phat = (A.rho + B.rho) * inv_sb;   // {rho} / (2 {beta}) = sr/sb, beta = b/2
    for (int i = 0; i < DIM; ++i) F[1 + i] = frho * vavg[i] + phat * n[i];
    F[DIM + 1] = frho * (0.5 * vab + ib_ln * gm1_inv) + phat * vn;
  }
}

// (dF/dA)^T Fb and (dF/dB)^T Fb, accumulated into Ab, Bb (n held fixed)
template <int DIM, int FLUX>
ESD_HD void ec_flux_vjp(const Node<DIM>& A, const Node<DIM>& B, const double* n, double gm1_inv, const double* Fb,
                        NodeBar<DIM>& Ab, NodeBar<DIM>& Bb) {
  const double sr = A.rho + B.rho, sb = A.b + B.b;
  const double rr = frcp(sr * sb);
  const double rho_ln = log_mean(A.rho, B.rho, A.lnrho, B.lnrho, sb * rr);
  const double ib_ln = inv_log_mean(A.b, B.b, A.lnb, B.lnb, sr * rr);
  double vavg[DIM];
  double vn = 0.0, vab = 0.0, van = 0.0, vbn = 0.0;
  for (int i = 0; i < DIM; ++i) {
    vavg[i] = 0.5 * (A.v[i] + B.v[i]);
    vn += vavg[i] * n[i];
    vab += A.v[i] * B.v[i];
    van += A.v[i] * n[i];
    vbn += B.v[i] * n[i];
  }
  const double frho = rho_ln * vn;
  // reverse sweep
  double frho_b = Fb[0];
  double vavg_b[DIM];
  for (int i = 0; i < DIM; ++i) {
    frho_b += Fb[1 + i] * vavg[i];
    vavg_b[i] = Fb[1 + i] * frho;
  }
  frho_b += Fb[DIM + 1] * (0.5 * vab + ib_ln * gm1_inv);
  const double vab_b = Fb[DIM + 1] * frho * 0.5;
  const double ib_b = Fb[DIM + 1] * frho * gm1_inv;
  double vn_b = 0.0, van_b = 0.0, vbn_b = 0.0;
  if (FLUX == FLUX_RANOCHA) {
    double pavg_b = 0.0;
    for (int i = 0; i < DIM; ++i) pavg_b += Fb[1 + i] * n[i];
    Ab.p += 0.5 * pavg_b + 0.5 * Fb[DIM + 1] * vbn;
    Bb.p += 0.5 * pavg_b + 0.5 * Fb[DIM + 1] * van;
    vbn_b = 0.5 * Fb[DIM + 1] * A.p;
    van_b = 0.5 * Fb[DIM + 1] * B.p;
  } else {
    const double isb = sr * rr, phat = sr * isb;
    double phat_b = Fb[DIM + 1] * vn;
    for (int i = 0; i < DIM; ++i) phat_b += Fb[1 + i] * n[i];
    vn_b += Fb[DIM + 1] * phat;
    // phat = sr / sb
    Ab.rho += phat_b * isb;
    Bb.rho += phat_b * isb;
    Ab.b -= phat_b * phat * isb;
    Bb.b -= phat_b * phat * isb;
  }
  const double rho_ln_b = frho_b * vn;
  vn_b += frho_b * rho_ln;
  for (int i = 0; i < DIM; ++i) {
    vavg_b[i] += vn_b * n[i];
    Ab.v[i] += 0.5 * vavg_b[i] + vab_b * B.v[i] + van_b * n[i];
    Bb.v[i] += 0.5 * vavg_b[i] + vab_b * A.v[i] + vbn_b * n[i];
  }
  double g[4];
  log_mean_grad(A.rho, B.rho, A.lnrho, B.lnrho, g);
  Ab.rho += rho_ln_b * g[0];
  Bb.rho += rho_ln_b * g[1];
  Ab.lnrho += rho_ln_b * g[2];
  Bb.lnrho += rho_ln_b * g[3];
  inv_log_mean_grad(A.b, B.b, A.lnb, B.lnb, g);
  Ab.b += ib_b * g[0];
  Bb.b += ib_b * g[1];
  Ab.lnb += ib_b * g[2];
  Bb.lnb += ib_b * g[3];
}

// ---------------------------------------------------------------- interface flux
constexpr double TIE_REL = 1.0e-10;

// weights of the one-sided derivatives of max(a, b), a, b >= 0: the branch the
// value takes (a on exact ties), or 1/2 each where |a - b| <= TIE_REL max(a, b)
ESD_HD void tie_weights(double a, double b, double& wa, double& wb) {
  const double mx = a >= b ? a : b;
  if (fabs(a - b) <= TIE_REL * mx) {
    wa = wb = 0.5;
  } else {
    wa = a > b ? 1.0 : 0.0;
    wb = 1.0 - wa;
  }
}

// dU = A0 dw, A0 = dU/dW at the primitive state (rho, v, p) (symmetric positive definite):
//   [[rho, rho v^T, E], [rho v, rho v v^T + p I, rho H v], [E, rho H v^T, rho H^2 - a^2 p/(gamma-1)]]
template <int DIM>
ESD_HD void entropy_jacobian_apply(double rho, const double* v, double p, double gamma, double gm1_inv,
                                   const double* dw, double* dU) {
  double v2 = 0.0, vdw = 0.0;
  for (int i = 0; i < DIM; ++i) {
    v2 += v[i] * v[i];
    vdw += v[i] * dw[1 + i];
  }
  const double a2 = gamma * p * frcp(rho);
  const double H = a2 * gm1_inv + 0.5 * v2, E = p * gm1_inv + 0.5 * rho * v2;
  const double w0 = dw[0], wl = dw[DIM + 1];
  dU[0] = rho * w0 + rho * vdw + E * wl;
  for (int i = 0; i < DIM; ++i) dU[1 + i] = rho * v[i] * (w0 + vdw) + p * dw[1 + i] + rho * H * v[i] * wl;
  dU[DIM + 1] = E * w0 + rho * H * vdw + (rho * H * H - a2 * p * gm1_inv) * wl;
}

// |A_n| dU for the Euler flux Jacobian in the unit direction n at (rho, v, p):
// acoustic waves of speeds v.n -+ a with strengths (dp -+ rho a dv_n)/(2 a^2)
// along (1, v -+ a n, H -+ a v.n); the rest of dU at speed |v.n|
template <int DIM>
ESD_HD void abs_jacobian_apply(double rho, const double* v, double p, const double* n, double gamma,
                               double gm1_inv, const double* dU, double* out) {
  double v2 = 0.0, vn = 0.0, vdm = 0.0, dvn = 0.0;
  const double ir = frcp(rho);
  for (int i = 0; i < DIM; ++i) {
    v2 += v[i] * v[i];
    vn += v[i] * n[i];
    vdm += v[i] * dU[1 + i];
  }
  const double a = sqrt(gamma * p * ir);
  const double H = a * a * gm1_inv + 0.5 * v2;
  const double dp = (gamma - 1.0) * (dU[DIM + 1] - vdm + 0.5 * v2 * dU[0]);
  for (int i = 0; i < DIM; ++i) dvn += (dU[1 + i] - v[i] * dU[0]) * ir * n[i];
  const double i2a2 = 0.5 * frcp(a * a);
  const double am = (dp - rho * a * dvn) * i2a2, ap = (dp + rho * a * dvn) * i2a2;
  const double l0 = fabs(vn), lm = fabs(vn - a), lp = fabs(vn + a);
  // rest = dU - am r- - ap r+ goes at |v.n|
  out[0] = l0 * (dU[0] - am - ap) + lm * am + lp * ap;
  for (int i = 0; i < DIM; ++i) {
    const double rm = v[i] - a * n[i], rp = v[i] + a * n[i];
    out[1 + i] = l0 * (dU[1 + i] - am * rm - ap * rp) + lm * am * rm + lp * ap * rp;
  }
  const double hm = H - a * vn, hp = H + a * vn;
  out[DIM + 1] = l0 * (dU[DIM + 1] - am * hm - ap * hp) + lm * am * hm + lp * ap * hp;
}

// J_f f*(U-, U+, n) with nJ = J_f n:  f#(U-, U+, nJ) minus the dissipation:
//   1  (J_f lambda)/2 (U+ - U-), J_f lambda = max(|v-.nJ|, |v+.nJ|) + J_f max(c-, c+);
//   2  (J_f lambda)/2 A0(mean) (w+ - w-)  (scalar dissipation on the entropy-variable jump);
//   3  J_f/2 |A_n(mean)| A0(mean) (w+ - w-)  (matrix dissipation);
// mean: arithmetic means of rho, v, p; wm, wp: the entropy variables of U-, U+
// (needed by 2 and 3)
template <int DIM, int FLUX>
ESD_HD void interface_flux(const Node<DIM>& Um, const Node<DIM>& Up, const double* nJ, double Jf, double gamma,
                           double gm1_inv, int dissipation, double* F, const double* wm = nullptr,
                           const double* wp = nullptr) {
  ec_flux<DIM, FLUX>(Um, Up, nJ, gm1_inv, F);
  if (!dissipation) return;
  if (dissipation >= 2) {
    double dw[DIM + 2], dU[DIM + 2], vbar[DIM];
    for (int c = 0; c < DIM + 2; ++c) dw[c] = wp[c] - wm[c];
    for (int i = 0; i < DIM; ++i) vbar[i] = 0.5 * (Um.v[i] + Up.v[i]);
    const double rbar = 0.5 * (Um.rho + Up.rho), pbar = 0.5 * (Um.p + Up.p);
    entropy_jacobian_apply<DIM>(rbar, vbar, pbar, gamma, gm1_inv, dw, dU);
    if (dissipation == 2) {
      double vmn = 0.0, vpn = 0.0;
      for (int i = 0; i < DIM; ++i) {
        vmn += Um.v[i] * nJ[i];
        vpn += Up.v[i] * nJ[i];
      }
      const double am = fabs(vmn), ap = fabs(vpn);
      const double cm = sqrt(gamma * Um.p / Um.rho), cp = sqrt(gamma * Up.p / Up.rho);
      const double h = 0.5 * ((am >= ap ? am : ap) + Jf * (cm >= cp ? cm : cp));
      for (int c = 0; c < DIM + 2; ++c) F[c] -= h * dU[c];
    } else {
      double n[DIM], D[DIM + 2];
      const double iJ = frcp(Jf);
      for (int i = 0; i < DIM; ++i) n[i] = nJ[i] * iJ;
      abs_jacobian_apply<DIM>(rbar, vbar, pbar, n, gamma, gm1_inv, dU, D);
      for (int c = 0; c < DIM + 2; ++c) F[c] -= 0.5 * Jf * D[c];
    }
    return;
  }
  double vmn = 0.0, vpn = 0.0, vm2 = 0.0, vp2 = 0.0;
  for (int i = 0; i < DIM; ++i) {
    vmn += Um.v[i] * nJ[i];
    vpn += Up.v[i] * nJ[i];
    vm2 += Um.v[i] * Um.v[i];
    vp2 += Up.v[i] * Up.v[i];
  }
  const double am = fabs(vmn), ap = fabs(vpn);
  const double cm = sqrt(gamma * Um.p / Um.rho), cp = sqrt(gamma * Up.p / Up.rho);
  const double lam = (am >= ap ? am : ap) + Jf * (cm >= cp ? cm : cp);
  const double h = 0.5 * lam;
  F[0] -= h * (Up.rho - Um.rho);
  for (int i = 0; i < DIM; ++i) F[1 + i] -= h * (Up.rho * Up.v[i] - Um.rho * Um.v[i]);
  const double Em = Um.p * gm1_inv + 0.5 * Um.rho * vm2;
  const double Ep = Up.p * gm1_inv + 0.5 * Up.rho * vp2;
  F[DIM + 1] -= h * (Ep - Em);
}

template <int DIM>
ESD_HD void cons_vjp(const Node<DIM>& N, const double* Ub, double gm1_inv, NodeBar<DIM>& Nb) {
  // U = (rho, rho v, p/(gamma-1) + rho |v|^2/2)
  double v2 = 0.0;
  for (int i = 0; i < DIM; ++i) v2 += N.v[i] * N.v[i];
  Nb.rho += Ub[0] + 0.5 * v2 * Ub[DIM + 1];
  for (int i = 0; i < DIM; ++i) {
    Nb.rho += Ub[1 + i] * N.v[i];
    Nb.v[i] += Ub[1 + i] * N.rho + Ub[DIM + 1] * N.rho * N.v[i];
  }
  Nb.p += gm1_inv * Ub[DIM + 1];
}

template <int DIM, int FLUX>
ESD_HD void interface_flux_vjp(const Node<DIM>& Um, const Node<DIM>& Up, const double* nJ, double Jf, double gamma,
                               double gm1_inv, int dissipation, const double* Fb, NodeBar<DIM>& Umb,
                               NodeBar<DIM>& Upb) {
  ec_flux_vjp<DIM, FLUX>(Um, Up, nJ, gm1_inv, Fb, Umb, Upb);
  if (!dissipation) return;
  double vmn = 0.0, vpn = 0.0, vm2 = 0.0, vp2 = 0.0;
  for (int i = 0; i < DIM; ++i) {
    vmn += Um.v[i] * nJ[i];
    vpn += Up.v[i] * nJ[i];
    vm2 += Um.v[i] * Um.v[i];
    vp2 += Up.v[i] * Up.v[i];
  }
  const double am = fabs(vmn), ap = fabs(vpn);
  const double cm = sqrt(gamma * Um.p / Um.rho), cp = sqrt(gamma * Up.p / Up.rho);
  const double lam = (am >= ap ? am : ap) + Jf * (cm >= cp ? cm : cp);
  const double h = 0.5 * lam;
  const double Em = Um.p * gm1_inv + 0.5 * Um.rho * vm2;
  const double Ep = Up.p * gm1_inv + 0.5 * Up.rho * vp2;
  double dU[DIM + 2];
  dU[0] = Up.rho - Um.rho;
  for (int i = 0; i < DIM; ++i) dU[1 + i] = Up.rho * Up.v[i] - Um.rho * Um.v[i];
  dU[DIM + 1] = Ep - Em;
  // F -= h dU
  double h_b = 0.0;
  double Ub[DIM + 2], Umb_c[DIM + 2];
  for (int c = 0; c < DIM + 2; ++c) {
    h_b -= Fb[c] * dU[c];
    Ub[c] = -h * Fb[c];      // cotangent of U+ (and minus it for U-)
    Umb_c[c] = h * Fb[c];
  }
  cons_vjp<DIM>(Up, Ub, gm1_inv, Upb);
  cons_vjp<DIM>(Um, Umb_c, gm1_inv, Umb);
  const double lam_b = 0.5 * h_b;
  // lam = max(am, ap) + Jf max(cm, cp); d|x| = sign(x) (0 at 0).  max is not
  // differentiable at a tie; where its arguments agree to TIE_REL relative
  // (a tie up to rounding) the derivative is the mean of the two one-sided ones.
  double wm, wp;
  tie_weights(am, ap, wm, wp);
  const double sgm = vmn > 0.0 ? 1.0 : (vmn < 0.0 ? -1.0 : 0.0);
  const double sgp = vpn > 0.0 ? 1.0 : (vpn < 0.0 ? -1.0 : 0.0);
  for (int i = 0; i < DIM; ++i) {
    Umb.v[i] += lam_b * wm * sgm * nJ[i];
    Upb.v[i] += lam_b * wp * sgp * nJ[i];
  }
  // c = sqrt(gamma p/rho): dc/dp = c/(2p), dc/drho = -c/(2 rho)
  tie_weights(cm, cp, wm, wp);
  const double bm = 0.5 * lam_b * Jf * cm * wm, bp = 0.5 * lam_b * Jf * cp * wp;
  Umb.p += bm * frcp(Um.p);
  Umb.rho -= bm * frcp(Um.rho);
  Upb.p += bp * frcp(Up.p);
  Upb.rho -= bp * frcp(Up.rho);
}

}  // namespace esd
