// Host-side check of the hand-written reverse-mode functions of the HIP path
// (paper_2411_11229_amd/csrc/hweno_adjoint.h) against central finite
// differences of the forward functions (hweno_device.h), through the identity
// <g, J d> = <J^T g, d> for random directions d and cotangents g. Also checks
// the structured characteristic projections against the explicit L and R
// rows (L R = I, project = L U, unproject = R x). Prints one line per check
// and "ALL OK" at the end; exits non-zero on failure.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <functional>
#include <random>
#include <vector>

#include "hweno_adjoint.h"

using namespace hweno;
using Vec = std::vector<double>;

static std::mt19937_64 rng(20241111);
static double unif(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }
static int failures = 0;

// Agreement of two reverse-mode forms of one function (same derivative,
// different arithmetic), on random cotangents from a generator of their own.
static std::mt19937_64 rng2(777);
static void compare(const char* name, int m, const std::function<Vec(const Vec&)>& b1,
                    const std::function<Vec(const Vec&)>& b2, double tol = 1e-10) {
  double worst = 0.0;
  for (int trial = 0; trial < 6; ++trial) {
    Vec g(m);
    for (auto& v : g) v = std::uniform_real_distribution<double>(-1, 1)(rng2);
    const Vec r1 = b1(g), r2 = b2(g);
    double mag = 1e-300;
    for (double v : r1) mag = std::max(mag, std::fabs(v));
    for (size_t i = 0; i < r1.size(); ++i) worst = std::max(worst, std::fabs(r1[i] - r2[i]) / mag);
  }
  const bool ok = worst <= tol;
  if (!ok) ++failures;
  std::printf("%-44s max rel diff %.2e %s\n", name, worst, ok ? "ok" : "FAIL");
}

static Scheme scheme(double h, double g0) {
  Scheme s{};
  s.dx = s.dy = h;
  s.idx = s.idy = 1.0 / h;
  s.gamma0 = g0;
  s.g1 = 0.5 * (1.0 - g0);
  s.d0 = 0.9;
  s.d1 = 0.05;
  s.eps = 1e-10;
  s.gas = 1.4;
  s.adv_a = 0.7;
  s.adv_b = -1.3;
  return s;
}

// f: R^n -> R^m, vjp: (x, g) -> J^T g. <g, J d> by Richardson-extrapolated
// central differences, (4 D(e) - D(2e)) / 3 with D(e) the central quotient at
// the step e = rel * max|x| (the e^2 term of the truncation error cancels, so
// one fixed step per check suffices: a wrong reverse is off at any step),
// against <J^T g, d>, for 6 random pairs (d, g).
static void check(const char* name, const Vec& x, int m, const std::function<Vec(const Vec&)>& f,
                  const std::function<Vec(const Vec&, const Vec&)>& vjp, double tol = 2e-6,
                  double rel = 1e-6) {
  const int n = (int)x.size();
  double worst = 0.0;
  for (int trial = 0; trial < 6; ++trial) {
    Vec d(n), g(m);
    for (auto& v : d) v = unif(-1, 1);
    for (auto& v : g) v = unif(-1, 1);
    double scale = 0.0;
    for (double v : x) scale = std::max(scale, std::fabs(v));
    Vec gx = vjp(x, g);
    const double eps = rel * std::max(scale, 1e-3);
    double mag = 0.0;
    auto D = [&](double e) {
      Vec xp(x), xm(x);
      for (int i = 0; i < n; ++i) { xp[i] += e * d[i]; xm[i] -= e * d[i]; }
      Vec yp = f(xp), ym = f(xm);
      double s = 0.0;
      for (int j = 0; j < m; ++j) {
        const double dj = (yp[j] - ym[j]) / (2 * e);
        s += g[j] * dj;
        mag += std::fabs(g[j] * dj);
      }
      return s;
    };
    const double lhs = (4.0 * D(eps) - D(2.0 * eps)) / 3.0;
    double rhs = 0.0;
    for (int i = 0; i < n; ++i) { rhs += gx[i] * d[i]; mag += std::fabs(gx[i] * d[i]); }
    worst = std::max(worst, std::fabs(lhs - rhs) / std::max(mag, 1e-30));
  }
  const bool ok = worst <= tol;
  if (!ok) ++failures;
  std::printf("%-44s rel mismatch %.2e %s\n", name, worst, ok ? "ok" : "FAIL");
}

// ------------------------------------------------------------ hweno_point
static void check_hweno_point(const char* name, const Vec& x, double h, double g0) {
  const Scheme s = scheme(h, g0);
  auto f = [&](const Vec& v) {
    double uR, uL, vt;
    hweno_point<double>(v[0], v[1], v[2], v[3], v[4], s, h, 1.0 / h, uR, uL, vt);
    return Vec{uR, uL, vt};
  };
  auto b = [&](const Vec& v, const Vec& g) {
    double r[5] = {0, 0, 0, 0, 0};
    hweno_point_vjp<double>(v[0], v[1], v[2], v[3], v[4], s, h, 1.0 / h, g[0], g[1], g[2], r[0],
                            r[1], r[2], r[3], r[4]);
    return Vec(r, r + 5);
  };
  check(name, x, 3, f, b);
  // the fused form: the same cotangents, and hweno_point's forward values
  double worst_fwd = 0.0;
  const Vec y = f(x);
  auto bf = [&](const Vec& g) {
    double r[5] = {0, 0, 0, 0, 0}, fR, fL, fT;
    hweno_point_vjp_fused<double>(x[0], x[1], x[2], x[3], x[4], s, h, 1.0 / h, g[0], g[1], g[2],
                                  r[0], r[1], r[2], r[3], r[4], fR, fL, fT);
    worst_fwd = std::max({worst_fwd, std::fabs(fR - y[0]), std::fabs(fL - y[1]), std::fabs(fT - y[2])});
    return Vec(r, r + 5);
  };
  char buf[96];
  std::snprintf(buf, sizeof buf, "%s, fused form", name);
  compare(buf, 3, [&](const Vec& g) { return b(x, g); }, bf);
  double ymag = 0.0;
  for (double v : y) ymag = std::max(ymag, std::fabs(v));
  if (worst_fwd > 1e-14 * ymag) {
    std::printf("%-44s forward values differ by %.2e FAIL\n", buf, worst_fwd);
    ++failures;
  }
}

// ------------------------------------------------------------ Euler pieces
template <int DIM>
static Vec euler_state() {
  const double rho = unif(0.3, 3.0), u = unif(-2, 2), v = unif(-2, 2), p = unif(0.3, 5.0);
  if (DIM == 1) return {rho, rho * u, p / 0.4 + 0.5 * rho * u * u};
  return {rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)};
}

template <int DIM, int D>
static void check_euler(const char* tag) {
  constexpr int NC = DIM + 2;
  Euler<DIM> sy{1.4};
  using Prim = typename Euler<DIM>::template Prim<double>;
  auto arr = [](const Vec& v, int off, double (&a)[NC]) { for (int c = 0; c < NC; ++c) a[c] = v[off + c]; };
  char buf[96];
  // flux
  {
    Vec x = euler_state<DIM>();
    auto f = [&](const Vec& v) { double U[NC], F[NC]; arr(v, 0, U); auto q = sy.prim(U); sy.template flux<D>(U, q, F); return Vec(F, F + NC); };
    auto b = [&](const Vec& v, const Vec& g) {
      double U[NC], gF[NC], gU[NC] = {}; arr(v, 0, U); arr(g, 0, gF);
      Prim q = sy.prim(U); PrimBar<double> pb;
      flux_vjp<D>(sy, U, q, gF, pb, gU); prim_vjp(sy, U, q, pb, gU);
      return Vec(gU, gU + NC);
    };
    std::snprintf(buf, sizeof buf, "euler%s flux", tag);
    check(buf, x, NC, f, b);
  }
  // A(U) V
  {
    Vec x = euler_state<DIM>();
    for (int c = 0; c < NC; ++c) x.push_back(unif(-3, 3));
    auto f = [&](const Vec& v) { double U[NC], V[NC], O[NC]; arr(v, 0, U); arr(v, NC, V); auto q = sy.prim(U); sy.template jac<D>(U, q, V, O); return Vec(O, O + NC); };
    auto b = [&](const Vec& v, const Vec& g) {
      double U[NC], V[NC], gO[NC], gU[NC] = {}, gV[NC] = {}; arr(v, 0, U); arr(v, NC, V); arr(g, 0, gO);
      Prim q = sy.prim(U); PrimBar<double> pb;
      jac_vjp<D>(sy, U, q, V, gO, pb, gU, gV); prim_vjp(sy, U, q, pb, gU);
      Vec r(gU, gU + NC); r.insert(r.end(), gV, gV + NC); return r;
    };
    std::snprintf(buf, sizeof buf, "euler%s jacobian-vector", tag);
    check(buf, x, NC, f, b);
  }
  // projection w = L(U0) X and back-projection U = R(U0) x
  for (int which = 0; which < 2; ++which) {
    Vec x = euler_state<DIM>();
    for (int c = 0; c < NC; ++c) x.push_back(unif(-3, 3));
    auto f = [&](const Vec& v) {
      double U[NC], X[NC], Y[NC]; arr(v, 0, U); arr(v, NC, X);
      auto q = sy.prim(U); auto e = sy.eig(q);
      if (which == 0) sy.template project<D>(e, X, Y); else sy.template unproject<D>(e, X, Y);
      return Vec(Y, Y + NC);
    };
    auto b = [&](const Vec& v, const Vec& g) {
      double U[NC], X[NC], gY[NC], gU[NC] = {}, gX[NC] = {}; arr(v, 0, U); arr(v, NC, X); arr(g, 0, gY);
      auto q = sy.prim(U); auto e = sy.eig(q); EigBar<double> eb; PrimBar<double> pb;
      if (which == 0) project_vjp<D>(sy, e, X, gY, eb, gX); else unproject_vjp<D>(sy, e, X, gY, eb, gX);
      eig_vjp(sy, q, e, eb, pb); prim_vjp(sy, U, q, pb, gU);
      Vec r(gU, gU + NC); r.insert(r.end(), gX, gX + NC); return r;
    };
    std::snprintf(buf, sizeof buf, "euler%s %s", tag, which == 0 ? "project (L U)" : "unproject (R x)");
    check(buf, x, NC, f, b);
    if (which == 1) {   // the split form of unproject_vjp, one component at a time
      auto split = [&](const Vec& gy) {
        double U[NC], X[NC], gY[NC], gU[NC] = {}, gX[NC] = {}; arr(x, 0, U); arr(x, NC, X); arr(gy, 0, gY);
        auto q = sy.prim(U); auto e = sy.eig(q); EigBar<double> eb; PrimBar<double> pb;
        unproject_t<D>(sy, e, gY, gX);
        for (int j = 0; j < NC; ++j) unproject_eb<D>(sy, e, j, X[j], gY, eb);
        eig_vjp(sy, q, e, eb, pb); prim_vjp(sy, U, q, pb, gU);
        Vec r(gU, gU + NC); r.insert(r.end(), gX, gX + NC); return r;
      };
      std::snprintf(buf, sizeof buf, "euler%s unproject, split form", tag);
      compare(buf, NC, [&](const Vec& g) { return b(x, g); }, split);
    }
  }
  // Roe's basis of (UL, UR): every basis parameter, through a random linear
  // read-out of the projection of a fixed vector (touches mu, nu, k, c, ic,
  // H, b1, b2 at once)
  {
    const auto saved = rng;   // leaves the draws of the checks below unchanged
    Vec x = euler_state<DIM>(), xr = euler_state<DIM>();
    x.insert(x.end(), xr.begin(), xr.end());
    double X[NC];
    for (int c = 0; c < NC; ++c) X[c] = unif(-2, 2);
    auto f = [&](const Vec& v) {
      double UL[NC], UR[NC], Y[NC], Z[NC]; arr(v, 0, UL); arr(v, NC, UR);
      auto e = sy.roe_eig(UL, UR);
      sy.template project<D>(e, X, Y); sy.template unproject<D>(e, X, Z);
      Vec r(Y, Y + NC); r.insert(r.end(), Z, Z + NC); return r;
    };
    auto b = [&](const Vec& v, const Vec& g) {
      double UL[NC], UR[NC], gY[NC], gZ[NC], gX[NC] = {}, gL[NC] = {}, gR[NC] = {};
      arr(v, 0, UL); arr(v, NC, UR); arr(g, 0, gY); arr(g, NC, gZ);
      auto e = sy.roe_eig(UL, UR); EigBar<double> eb;
      project_vjp<D>(sy, e, X, gY, eb, gX); unproject_vjp<D>(sy, e, X, gZ, eb, gX);
      roe_eig_vjp(sy, UL, UR, e, eb, gL, gR);
      Vec r(gL, gL + NC); r.insert(r.end(), gR, gR + NC); return r;
    };
    std::snprintf(buf, sizeof buf, "euler%s Roe basis", tag);
    check(buf, x, 2 * NC, f, b);
    rng = saved;
  }
  // structured projections equal the explicit rows / columns; L R = I
  {
    Vec x = euler_state<DIM>();
    double U[NC]; arr(x, 0, U);
    auto q = sy.prim(U); auto e = sy.eig(q);
    double worst = 0.0;
    double X[NC], Y[NC], Z[NC];
    for (int c = 0; c < NC; ++c) X[c] = unif(-2, 2);
    sy.template project<D>(e, X, Y);
    sy.template unproject<D>(e, X, Z);
    for (int j = 0; j < NC; ++j) {
      double l[NC], r[NC];
      sy.template left<D>(e, j, l);
      double dot = 0.0;
      for (int c = 0; c < NC; ++c) dot += l[c] * X[c];
      worst = std::max(worst, std::fabs(dot - Y[j]));
      for (int k = 0; k < NC; ++k) {
        sy.template right<D>(e, k, r);
        double lr = 0.0;
        for (int c = 0; c < NC; ++c) lr += l[c] * r[c];
        worst = std::max(worst, std::fabs(lr - (j == k ? 1.0 : 0.0)));
      }
    }
    for (int c = 0; c < NC; ++c) {
      double acc = 0.0;
      for (int k = 0; k < NC; ++k) { double r[NC]; sy.template right<D>(e, k, r); acc += r[c] * X[k]; }
      worst = std::max(worst, std::fabs(acc - Z[c]));
    }
    const bool ok = worst < 1e-12;
    if (!ok) ++failures;
    std::printf("euler%-39s max err %.2e %s\n", (std::string(tag) + " L/R structure").c_str(), worst, ok ? "ok" : "FAIL");
  }
  // one cell's HWENO in characteristic variables
  for (int regime = 0; regime < 3; ++regime) {
    const double h = 0.05;
    Vec x;
    Vec a = euler_state<DIM>(), bb = euler_state<DIM>(), cc = euler_state<DIM>();
    if (regime == 0) {        // smooth: small variations around one state
      for (int k = 0; k < 3; ++k) for (int c = 0; c < NC; ++c) x.push_back(a[c] * (1 + 0.02 * (k - 1) + 0.001 * unif(-1, 1)));
      for (int k = 0; k < 2; ++k) for (int c = 0; c < NC; ++c) x.push_back(unif(-0.5, 0.5));
    } else if (regime == 1) { // a jump between i and i+1
      for (int c = 0; c < NC; ++c) x.push_back(a[c]);
      for (int c = 0; c < NC; ++c) x.push_back(a[c] * 1.01);
      for (int c = 0; c < NC; ++c) x.push_back(bb[c]);
      for (int k = 0; k < 2; ++k) for (int c = 0; c < NC; ++c) x.push_back(unif(-2, 2));
    } else {                  // three unrelated states
      for (auto* st : {&a, &bb, &cc}) for (int c = 0; c < NC; ++c) x.push_back((*st)[c]);
      for (int k = 0; k < 2; ++k) for (int c = 0; c < NC; ++c) x.push_back(unif(-2, 2));
    }
    const Scheme s = scheme(h, DIM == 1 ? 0.95 : 0.99);
    auto f = [&](const Vec& v) {
      double Um[NC], U0[NC], Up[NC], Am[NC], Ap[NC], uR[NC], uL[NC], at[NC];
      arr(v, 0, Um); arr(v, NC, U0); arr(v, 2 * NC, Up); arr(v, 3 * NC, Am); arr(v, 4 * NC, Ap);
      hweno_cell<D>(sy, s, h, 1.0 / h, Um, U0, Up, Am, Ap, uR, uL, at);
      Vec r(uR, uR + NC); r.insert(r.end(), uL, uL + NC); r.insert(r.end(), at, at + NC); return r;
    };
    auto b = [&](const Vec& v, const Vec& g) {
      double Um[NC], U0[NC], Up[NC], Am[NC], Ap[NC], gR[NC], gL[NC], gT[NC];
      arr(v, 0, Um); arr(v, NC, U0); arr(v, 2 * NC, Up); arr(v, 3 * NC, Am); arr(v, 4 * NC, Ap);
      arr(g, 0, gR); arr(g, NC, gL); arr(g, 2 * NC, gT);
      double o[5][NC] = {};
      hweno_cell_vjp<D>(sy, s, h, 1.0 / h, Um, U0, Up, Am, Ap, gR, gL, gT, o[0], o[1], o[2], o[3], o[4]);
      Vec r;
      for (int k = 0; k < 5; ++k) r.insert(r.end(), o[k], o[k] + NC);
      return r;
    };
    std::snprintf(buf, sizeof buf, "euler%s hweno_cell (%s)", tag, regime == 0 ? "smooth" : regime == 1 ? "jump" : "rough");
    check(buf, x, 3 * NC, f, b, 1e-6);
    auto bf = [&](const Vec& g) {
      double Um[NC], U0[NC], Up[NC], Am[NC], Ap[NC], gR[NC], gL[NC], gT[NC];
      arr(x, 0, Um); arr(x, NC, U0); arr(x, 2 * NC, Up); arr(x, 3 * NC, Am); arr(x, 4 * NC, Ap);
      arr(g, 0, gR); arr(g, NC, gL); arr(g, 2 * NC, gT);
      double o[5][NC] = {};
      hweno_cell_vjp<D, true>(sy, s, h, 1.0 / h, Um, U0, Up, Am, Ap, gR, gL, gT, o[0], o[1], o[2], o[3], o[4]);
      Vec r;
      for (int k = 0; k < 5; ++k) r.insert(r.end(), o[k], o[k] + NC);
      return r;
    };
    std::snprintf(buf, sizeof buf, "euler%s hweno_cell fused (%s)", tag, regime == 0 ? "smooth" : regime == 1 ? "jump" : "rough");
    compare(buf, 3 * NC, [&](const Vec& g) { return b(x, g); }, bf);
    // the interface-basis switch
    const auto saved = rng;
    auto fi = [&](const Vec& v) {
      double Um[NC], U0[NC], Up[NC], Am[NC], Ap[NC], uR[NC], uL[NC], at[NC];
      arr(v, 0, Um); arr(v, NC, U0); arr(v, 2 * NC, Up); arr(v, 3 * NC, Am); arr(v, 4 * NC, Ap);
      hweno_cell_iface<D>(sy, s, h, 1.0 / h, sy.prim(U0), Um, U0, Up, Am, Ap, uR, uL, at);
      Vec r(uR, uR + NC); r.insert(r.end(), uL, uL + NC); r.insert(r.end(), at, at + NC); return r;
    };
    auto bi = [&](const Vec& v, const Vec& g) {
      double Um[NC], U0[NC], Up[NC], Am[NC], Ap[NC], gR[NC], gL[NC], gT[NC];
      arr(v, 0, Um); arr(v, NC, U0); arr(v, 2 * NC, Up); arr(v, 3 * NC, Am); arr(v, 4 * NC, Ap);
      arr(g, 0, gR); arr(g, NC, gL); arr(g, 2 * NC, gT);
      double o[5][NC] = {};
      hweno_cell_iface_vjp<D>(sy, s, h, 1.0 / h, Um, U0, Up, Am, Ap, gR, gL, gT, o[0], o[1], o[2], o[3], o[4]);
      Vec r;
      for (int k = 0; k < 5; ++k) r.insert(r.end(), o[k], o[k] + NC);
      return r;
    };
    std::snprintf(buf, sizeof buf, "euler%s hweno_cell interface (%s)", tag, regime == 0 ? "smooth" : regime == 1 ? "jump" : "rough");
    check(buf, x, 3 * NC, fi, bi, 1e-6);
    rng = saved;
  }
}

// The kernel's rearranged combination equals the direct form of (interp),
// its mirror image and (limiter) written with the candidates p0, p1, p2.
static void check_point_direct_form() {
  double worst = 0.0;
  for (int trial = 0; trial < 200; ++trial) {
    const double h = unif(0.01, 1.0), g0 = unif(0.3, 0.99);
    const Scheme s = scheme(h, g0);
    const double um = unif(-2, 2), u0 = unif(-2, 2), up = unif(-2, 2);
    const double vm = unif(-5, 5), vp = unif(-5, 5);
    double uR, uL, vt;
    hweno_point<double>(um, u0, up, vm, vp, s, h, 1.0 / h, uR, uL, vt);
    const double e1 = u0 - um, e2 = up - u0;
    double b0;
    {
      const double a1 = -h / 4 * (vm + vp) + 0.75 * (up - um);
      const double a2 = h / 4 * (vm - vp) + (um - 2 * u0 + up);
      const double a3 = h / 4 * (vm + vp) + 0.25 * (um - up);
      const double a4 = h / 4 * (vp - vm) - 0.5 * (um - 2 * u0 + up);
      b0 = (a1 + a3 / 4) * (a1 + a3 / 4) + 13.0 / 3 * (a2 + 63.0 / 130 * a4) * (a2 + 63.0 / 130 * a4) +
           781.0 / 20 * a3 * a3 + 1421461.0 / 2275 * a4 * a4;
    }
    const double b[3] = {b0, e1 * e1, e2 * e2};
    const double tau = 0.25 * std::pow(std::fabs(b[0] - b[1]) + std::fabs(b[0] - b[2]), 2);
    auto weights = [&](const double lin[3], double w[3]) {
      double sum = 0;
      for (int l = 0; l < 3; ++l) { w[l] = lin[l] * (1 + tau / (b[l] + s.eps)); sum += w[l]; }
      for (int l = 0; l < 3; ++l) w[l] /= sum;
    };
    const double lg[3] = {s.gamma0, s.g1, s.g1}, ld[3] = {s.d0, s.d1, s.d1};
    double wg[3], wd[3];
    weights(lg, wg);
    weights(ld, wd);
    auto comb = [](const double w[3], const double lin[3], double a, double bb, double c) {
      return w[0] * (a / lin[0] - lin[1] / lin[0] * bb - lin[2] / lin[0] * c) + w[1] * bb + w[2] * c;
    };
    const double p0 = -um / 8 + 9.0 / 16 * u0 + 9.0 / 16 * up - h * (3.0 / 64 * vm + 9.0 / 64 * vp);
    const double q0 = -up / 8 + 9.0 / 16 * u0 + 9.0 / 16 * um + h * (3.0 / 64 * vp + 9.0 / 64 * vm);
    const double rR = comb(wg, lg, p0, -um / 2 + 1.5 * u0, (u0 + up) / 2);
    const double rL = comb(wg, lg, q0, (um + u0) / 2, 1.5 * u0 - up / 2);
    const double rT = comb(wd, ld, 3 / (4 * h) * (up - um) - (vm + vp) / 4, (u0 - um) / h, (up - u0) / h);
    const double sc = 1 + std::fabs(u0) + std::fabs(up) + std::fabs(um) + h * (std::fabs(vm) + std::fabs(vp));
    worst = std::max({worst, std::fabs(uR - rR) / sc, std::fabs(uL - rL) / sc,
                      std::fabs(vt - rT) * h / sc});
  }
  const bool ok = worst < 1e-13;
  if (!ok) ++failures;
  std::printf("%-44s max err %.2e %s\n", "hweno_point = direct (interp)/(limiter)", worst, ok ? "ok" : "FAIL");
}

int main() {
  check_point_direct_form();
  // HWENO point: smooth, near-critical, a jump, rough
  check_hweno_point("hweno_point smooth", {1.0, 1.1, 1.21, 2.0, 2.4}, 0.1, 0.95);
  check_hweno_point("hweno_point near extremum", {1.0, 1.0005, 0.9995, 0.02, -0.03}, 0.01, 0.95);
  check_hweno_point("hweno_point jump", {0.0, 0.01, 1.0, 0.1, 0.0}, 0.05, 0.99);
  check_hweno_point("hweno_point rough", {0.3, -1.2, 2.5, 4.0, -7.0}, 0.2, 0.99);
  // linear pieces
  {
    const double ih = 7.0;
    auto f = [&](const Vec& v) { double R, L; face_derivs<double>(v[0], v[1], v[2], v[3], v[4], ih, R, L); return Vec{R, L}; };
    auto b = [&](const Vec&, const Vec& g) { double r[5] = {}; face_derivs_vjp<double>(g[0], g[1], ih, r[0], r[1], r[2], r[3], r[4]); return Vec(r, r + 5); };
    check("face_derivs", {0.1, 0.7, -0.4, 1.3, 0.2}, 2, f, b);
  }
  {
    const double h = 0.13, ih = 1.0 / h;
    auto f = [&](const Vec& v) { double a, c; central_corr<double>(v[0], v[1], v[2], v[3], v[4], v[5], h, ih, a, c); return Vec{a, c}; };
    auto b = [&](const Vec&, const Vec& g) { double r[6] = {}; central_corr_vjp<double>(g[0], g[1], h, ih, r[0], r[1], r[2], r[3], r[4], r[5]); return Vec(r, r + 6); };
    check("central_corr", {0.3, -0.2, 0.9, 1.4, -2.0, 0.5}, 2, f, b);
  }
  // scalar systems through hweno_cell
  {
    Burgers bu;
    const Scheme s = scheme(0.1, 0.95);
    auto f = [&](const Vec& v) {
      double Um[1] = {v[0]}, U0[1] = {v[1]}, Up[1] = {v[2]}, Am[1] = {v[3]}, Ap[1] = {v[4]}, a[1], c[1], t[1];
      hweno_cell<0>(bu, s, 0.1, 10.0, Um, U0, Up, Am, Ap, a, c, t); return Vec{a[0], c[0], t[0]};
    };
    auto b = [&](const Vec& v, const Vec& g) {
      double Um[1] = {v[0]}, U0[1] = {v[1]}, Up[1] = {v[2]}, Am[1] = {v[3]}, Ap[1] = {v[4]};
      double gR[1] = {g[0]}, gL[1] = {g[1]}, gT[1] = {g[2]}, o[5][1] = {};
      hweno_cell_vjp<0>(bu, s, 0.1, 10.0, Um, U0, Up, Am, Ap, gR, gL, gT, o[0], o[1], o[2], o[3], o[4]);
      return Vec{o[0][0], o[1][0], o[2][0], o[3][0], o[4][0]};
    };
    check("burgers hweno_cell", {0.2, 0.5, 1.1, 0.4, -0.3}, 3, f, b);
    auto fj = [&](const Vec& v) { double U[1] = {v[0]}, V[1] = {v[1]}, O[1]; bu.jac<0>(U, Burgers::Prim<double>{}, V, O); return Vec{O[0]}; };
    auto bj = [&](const Vec& v, const Vec& g) { double U[1] = {v[0]}, V[1] = {v[1]}, gO[1] = {g[0]}, gU[1] = {0}, gV[1] = {0}; NoBar<double> nb; jac_vjp<0>(bu, U, Burgers::Prim<double>{}, V, gO, nb, gU, gV); return Vec{gU[0], gV[0]}; };
    check("burgers jacobian-vector", {0.7, -1.9}, 1, fj, bj);
  }
  check_euler<1, 0>("1d");
  check_euler<2, 0>("2d-x");
  check_euler<2, 1>("2d-y");
  if (failures) {
    std::printf("%d FAILED\n", failures);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
