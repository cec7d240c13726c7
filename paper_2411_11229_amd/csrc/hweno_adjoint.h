// Reverse-mode (vector-Jacobian) counterparts of the per-point functions in
// hweno_device.h, written by hand. Each *_vjp recomputes what it needs of the
// forward pass and ADDS its cotangent contributions to the output arrays.
//
// Conventions: alpha and dt are constants (not differentiated); the
// derivative of |x| at x = 0 is taken as 0 (the kinks of |beta0 - beta_k|).
#pragma once

#include "hweno_device.h"

namespace hweno {

HWENO_HD double sgn0(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// ---------------------------------------------------------------- HWENO point
// Reverse of hweno_point: given cotangents gR, gL, gT of (uR, uL, vt), adds
// the cotangents of (um, u0, up, vm, vp). Its forward part is written
// through the candidate values (unscaled weights), so it shares nothing with
// a forward hweno_point on the same data: the cheaper choice where that
// forward's intermediates could not stay in registers until the reverse.
template <typename T>
HWENO_HD void hweno_point_vjp(T um, T u0, T up, T vm, T vp, const Scheme& s, double h, double ih,
                              double gR, double gL, double gT, T& gum, T& gu0, T& gup, T& gvm,
                              T& gvp) {
  // ---- forward, exactly as hweno_point
  const double dm = (double)um, dc = (double)u0, dp = (double)up;
  const double vmd = (double)vm, vpd = (double)vp;
  const double sv = 0.25 * h * (vmd + vpd);
  const double dv = 0.25 * h * (vmd - vpd);
  const double cdf = dp - dm;
  const double sdf = dm - 2.0 * dc + dp;
  const double a1 = 0.75 * cdf - sv;
  const double a2 = sdf + dv;
  const double a3 = sv - 0.25 * cdf;
  const double a4 = -0.5 * sdf - dv;
  const double t1 = a1 + 0.25 * a3;
  const double t2 = a2 + (63.0 / 130.0) * a4;
  const double b0 = t1 * t1 + (13.0 / 3.0) * t2 * t2 + (781.0 / 20.0) * a3 * a3 +
                    (1421461.0 / 2275.0) * a4 * a4;
  const double e1 = dc - dm, e2 = dp - dc;
  const double b1 = e1 * e1, b2 = e2 * e2;
  const double ts = fabs(b0 - b1) + fabs(b0 - b2);
  const double tau = 0.25 * ts * ts;
  const double q0 = b0 + s.eps, q1 = b1 + s.eps, q2 = b2 + s.eps;
  const double q12 = q1 * q2;
  const double i3 = rcp_nr(q0 * q12);
  const double iq0 = i3 * q12, iq1 = i3 * (q0 * q2), iq2 = i3 * (q0 * q1);
  const double ti = tau * i3;
  const double o0 = 1.0 + ti * q12;
  const double o1 = 1.0 + ti * (q0 * q2);
  const double o2 = 1.0 + ti * (q0 * q1);
  const double Sg = s.gamma0 * o0 + s.g1 * (o1 + o2);
  const double Sd = s.d0 * o0 + s.d1 * (o1 + o2);
  const double inv = rcp_nr(Sg * Sd);
  const double iSg = Sd * inv, iSd = Sg * inv;
  const double P0 = -0.125 * dm + 0.5625 * (dc + dp) - h * (0.046875 * vmd + 0.140625 * vpd);
  const double P1 = -0.5 * dm + 1.5 * dc;
  const double P2 = 0.5 * (dc + dp);
  const double Q0 = -0.125 * dp + 0.5625 * (dc + dm) + h * (0.046875 * vpd + 0.140625 * vmd);
  const double Q1 = -0.5 * dp + 1.5 * dc;
  const double Q2 = 0.5 * (dc + dm);
  const double D0 = 0.75 * ih * cdf - 0.25 * (vmd + vpd);
  const double D1 = ih * e1;
  const double D2 = ih * e2;
  const double NR = o0 * (P0 - s.g1 * (P1 + P2)) + s.g1 * (o1 * P1 + o2 * P2);
  const double NL = o0 * (Q0 - s.g1 * (Q1 + Q2)) + s.g1 * (o2 * Q1 + o1 * Q2);
  const double NT = o0 * (D0 - s.d1 * (D1 + D2)) + s.d1 * (o1 * D1 + o2 * D2);
  const double uR = NR * iSg, uL = NL * iSg, vt = NT * iSd;
  // ---- reverse
  const double gNR = gR * iSg, gNL = gL * iSg, gNT = gT * iSd;
  const double gSg = -(gR * uR + gL * uL) * iSg;
  const double gSd = -gT * vt * iSd;
  const double gsum = s.g1 * gSg + s.d1 * gSd;   // shared by o1 and o2 through Sg, Sd
  const double go0 = gNR * (P0 - s.g1 * (P1 + P2)) + gNL * (Q0 - s.g1 * (Q1 + Q2)) +
                     gNT * (D0 - s.d1 * (D1 + D2)) + s.gamma0 * gSg + s.d0 * gSd;
  const double go1 = s.g1 * (gNR * P1 + gNL * Q2) + s.d1 * gNT * D1 + gsum;
  const double go2 = s.g1 * (gNR * P2 + gNL * Q1) + s.d1 * gNT * D2 + gsum;
  const double gP0 = gNR * o0, gP1 = gNR * s.g1 * (o1 - o0), gP2 = gNR * s.g1 * (o2 - o0);
  const double gQ0 = gNL * o0, gQ1 = gNL * s.g1 * (o2 - o0), gQ2 = gNL * s.g1 * (o1 - o0);
  const double gD0 = gNT * o0, gD1 = gNT * s.d1 * (o1 - o0), gD2 = gNT * s.d1 * (o2 - o0);
  // o_l = 1 + tau / q_l
  const double gtau = go0 * iq0 + go1 * iq1 + go2 * iq2;
  const double gq0 = -go0 * (o0 - 1.0) * iq0;
  const double gq1 = -go1 * (o1 - 1.0) * iq1;
  const double gq2 = -go2 * (o2 - 1.0) * iq2;
  // tau = ts^2 / 4, ts = |b0 - b1| + |b0 - b2|
  const double gts = 0.5 * ts * gtau;
  const double s1 = sgn0(b0 - b1), s2 = sgn0(b0 - b2);
  const double gb0 = gq0 + gts * (s1 + s2);
  const double gb1 = gq1 - gts * s1;
  const double gb2 = gq2 - gts * s2;
  // b1 = e1^2, b2 = e2^2 (and D1, D2)
  const double ge1 = 2.0 * e1 * gb1 + ih * gD1;
  const double ge2 = 2.0 * e2 * gb2 + ih * gD2;
  // b0 from t1, t2, a3, a4
  const double gt1 = 2.0 * t1 * gb0;
  const double gt2 = (26.0 / 3.0) * t2 * gb0;
  const double ga1 = gt1;
  const double ga2 = gt2;
  const double ga3 = (781.0 / 10.0) * a3 * gb0 + 0.25 * gt1;
  const double ga4 = (2.0 * 1421461.0 / 2275.0) * a4 * gb0 + (63.0 / 130.0) * gt2;
  const double gcdf = 0.75 * ga1 - 0.25 * ga3 + 0.75 * ih * gD0;
  const double gsdf = ga2 - 0.5 * ga4;
  const double gsv = ga3 - ga1;
  const double gdv = ga2 - ga4;
  double rum = -0.125 * gP0 - 0.5 * gP1 + 0.5625 * gQ0 + 0.5 * gQ2;
  double ru0 = 0.5625 * gP0 + 1.5 * gP1 + 0.5 * gP2 + 0.5625 * gQ0 + 1.5 * gQ1 + 0.5 * gQ2;
  double rup = 0.5625 * gP0 + 0.5 * gP2 - 0.125 * gQ0 - 0.5 * gQ1;
  double rvm = h * (0.140625 * gQ0 - 0.046875 * gP0) - 0.25 * gD0;
  double rvp = h * (0.046875 * gQ0 - 0.140625 * gP0) - 0.25 * gD0;
  rum += -gcdf + gsdf - ge1;
  ru0 += -2.0 * gsdf + ge1 - ge2;
  rup += gcdf + gsdf + ge2;
  rvm += 0.25 * h * (gsv + gdv);
  rvp += 0.25 * h * (gsv - gdv);
  gum += (T)rum;
  gu0 += (T)ru0;
  gup += (T)rup;
  gvm += (T)rvm;
  gvp += (T)rvp;
}

// The same reverse for the current hweno_point arithmetic (scaled weights
// o_l, one division), which also returns the forward values (uR, uL, vt) in
// fR, fL, fT: when it follows a forward hweno_point on the same data the
// compiler shares the forward part between the two.
template <typename T>
HWENO_HD void hweno_point_vjp_fused(T um, T u0, T up, T vm, T vp, const Scheme& s, double h,
                                    double ih, double gR, double gL, double gT, T& gum, T& gu0,
                                    T& gup, T& gvm, T& gvp, T& fR, T& fL, T& fT) {
  // ---- forward, as hweno_point
  const double dc = (double)u0;
  const double e1 = dc - (double)um, e2 = (double)up - dc;
  const double vmd = (double)vm, vpd = (double)vp;
  const double cdf = e1 + e2, sdf = e2 - e1;
  const double qh = 0.25 * h;
  const double sv = qh * (vmd + vpd), dv = qh * (vmd - vpd);
  constexpr double r13 = 2.0816659994661326;    // sqrt(13/3)
  constexpr double r781 = 6.248999919987197;    // sqrt(781/20)
  constexpr double r1421 = 24.99636017459386;   // sqrt(1421461/2275)
  constexpr double A1 = r13 * 197.0 / 260.0, A2 = r13 * 67.0 / 130.0;
  const double t1 = 0.6875 * cdf - 0.75 * sv;
  const double t2 = A1 * sdf + A2 * dv;
  const double a3 = r781 * sv - (0.25 * r781) * cdf;
  const double a4 = (-0.5 * r1421) * sdf - r1421 * dv;
  const double b0 = t1 * t1 + t2 * t2 + a3 * a3 + a4 * a4;
  const double b1 = e1 * e1, b2 = e2 * e2;
  const double d1 = b0 - b1, d2 = b0 - b2;
  const double ts = fabs(d1) + fabs(d2);
  const double tau = 0.25 * ts * ts;
  const double q0 = b0 + s.eps, q1 = b1 + s.eps, q2 = b2 + s.eps;
  const double p0 = q0 + tau, p1 = q1 + tau, p2 = q2 + tau;
  const double q12 = q1 * q2, q02 = q0 * q2, q01 = q0 * q1;
  const double o0 = q12 * p0, o1 = q02 * p1, o2 = q01 * p2;
  const double o12 = o1 + o2;
  const double Sg = s.gamma0 * o0 + s.g1 * o12;
  const double Sd = s.d0 * o0 + s.d1 * o12;
  const double inv = rcp_nr(Sg * Sd);
  const double iSg = Sd * inv, iSd = Sg * inv;
  const double X = o1 * e1 + o2 * e2;
  const double gX0 = 0.5 * s.g1 * X;
  const double K = 0.34375 - 0.5 * s.g1;
  const double base = K * cdf - 0.375 * sv;
  const double m = 0.21875 * sdf + 0.1875 * dv;
  const double P1 = o0 * base + gX0, P2 = o0 * m;
  const double NR = P1 + P2, NL = P1 - P2;
  const double c3 = (0.75 - s.d1) * ih;
  const double AT = (0.75 - s.d1) * ih * cdf - ih * sv;
  const double NT = o0 * AT + s.d1 * ih * X;
  fR = (T)(dc + NR * iSg);
  fL = (T)(dc - NL * iSg);
  fT = (T)(NT * iSd);
  // ---- reverse
  const double gNR = gR * iSg, gNL = -gL * iSg, gNT = gT * iSd;
  const double gSg = -(gNR * NR + gNL * NL) * iSg;
  const double gSd = -gNT * NT * iSd;
  const double gsum = gNR + gNL;
  const double gX = 0.5 * s.g1 * gsum + s.d1 * ih * gNT;
  const double go0 = gNR * (base + m) + gNL * (base - m) + gNT * AT + s.gamma0 * gSg + s.d0 * gSd;
  const double go12 = s.g1 * gSg + s.d1 * gSd;
  const double go1 = go12 + gX * e1, go2 = go12 + gX * e2;
  const double gbase = o0 * gsum, gm = o0 * (gNR - gNL), gAT = o0 * gNT;
  // o_l = (product of the other q's) (q_l + tau)
  const double gp0 = go0 * q12, gp1 = go1 * q02, gp2 = go2 * q01;
  const double gq0 = gp0 + go1 * q2 * p1 + go2 * q1 * p2;
  const double gq1 = gp1 + go0 * q2 * p0 + go2 * q0 * p2;
  const double gq2 = gp2 + go0 * q1 * p0 + go1 * q0 * p1;
  const double gts = 0.5 * ts * (gp0 + gp1 + gp2);
  const double gd1 = gts * sgn0(d1), gd2 = gts * sgn0(d2);
  const double gb0 = gq0 + gd1 + gd2;
  const double gb1 = gq1 - gd1, gb2 = gq2 - gd2;
  const double gt1 = 2.0 * t1 * gb0, gt2 = 2.0 * t2 * gb0;
  const double ga3 = 2.0 * a3 * gb0, ga4 = 2.0 * a4 * gb0;
  const double gcdf = 0.6875 * gt1 - (0.25 * r781) * ga3 + K * gbase + c3 * gAT;
  const double gsdf = A1 * gt2 - (0.5 * r1421) * ga4 + 0.21875 * gm;
  const double gsv = -0.75 * gt1 + r781 * ga3 - 0.375 * gbase - ih * gAT;
  const double gdv = A2 * gt2 - r1421 * ga4 + 0.1875 * gm;
  const double ge1 = gX * o1 + 2.0 * e1 * gb1 + gcdf - gsdf;
  const double ge2 = gX * o2 + 2.0 * e2 * gb2 + gcdf + gsdf;
  gum += (T)(-ge1);
  gu0 += (T)(gR + gL + ge1 - ge2);
  gup += (T)ge2;
  gvm += (T)(qh * (gsv + gdv));
  gvp += (T)(qh * (gsv - gdv));
}

// Reverse of face_derivs: cotangents gR, gL of (vR, vL) -> (um, u0, up, vm, vp).
template <typename T>
HWENO_HD void face_derivs_vjp(T gR, T gL, T ih, T& gum, T& gu0, T& gup, T& gvm, T& gvp) {
  gum += (T(0.1875) * gR - T(1.3125) * gL) * ih;
  gu0 += (T(1.5) * (gL - gR)) * ih;
  gup += (T(1.3125) * gR - T(0.1875) * gL) * ih;
  gvm += T(0.0625) * gR - T(0.1875) * gL;
  gvp += T(0.0625) * gL - T(0.1875) * gR;
}

// ------------------------------------------------------- scalar systems
// Cotangent accumulators of the per-point quantities; empty for scalars.
template <typename T> struct NoBar {};

template <int D, typename T>
HWENO_HD void flux_vjp(const Advection& sy, const T (&)[1], const Advection::Prim<T>&,
                       const T (&gF)[1], NoBar<T>&, T (&gU)[1]) {
  gU[0] += T(D == 0 ? sy.a : sy.b) * gF[0];
}
template <int D, typename T>
HWENO_HD void jac_vjp(const Advection& sy, const T (&)[1], const Advection::Prim<T>&,
                      const T (&)[1], const T (&gO)[1], NoBar<T>&, T (&)[1], T (&gV)[1]) {
  gV[0] += T(D == 0 ? sy.a : sy.b) * gO[0];
}
template <typename T>
HWENO_HD void prim_vjp(const Advection&, const T (&)[1], const Advection::Prim<T>&, NoBar<T>&,
                       T (&)[1]) {}

template <int D, typename T>
HWENO_HD void flux_vjp(const Burgers&, const T (&U)[1], const Burgers::Prim<T>&,
                       const T (&gF)[1], NoBar<T>&, T (&gU)[1]) {
  gU[0] += U[0] * gF[0];
}
template <int D, typename T>
HWENO_HD void jac_vjp(const Burgers&, const T (&U)[1], const Burgers::Prim<T>&, const T (&V)[1],
                      const T (&gO)[1], NoBar<T>&, T (&gU)[1], T (&gV)[1]) {
  gU[0] += V[0] * gO[0];
  gV[0] += U[0] * gO[0];
}
template <typename T>
HWENO_HD void prim_vjp(const Burgers&, const T (&)[1], const Burgers::Prim<T>&, NoBar<T>&,
                       T (&)[1]) {}

template <class Sys, typename T> struct BarOf { using type = NoBar<T>; };

// ------------------------------------------------------------- Euler
template <typename T>
struct PrimBar {
  T ir = T(0), mu = T(0), nu = T(0), k = T(0), p = T(0), Ep = T(0);
};
template <typename T>
struct EigBar {
  T mu = T(0), nu = T(0), k = T(0), c = T(0), ic = T(0), H = T(0), b1 = T(0), b2 = T(0);
};
template <int DIM, typename T> struct BarOf<Euler<DIM>, T> { using type = PrimBar<T>; };

// ir = 1/rho, u = m ir, v = n ir, k = (u^2+v^2)/2, P = (g-1)(E - rho k), Ep = E + P
template <int DIM, typename T>
HWENO_HD void prim_vjp(const Euler<DIM>& sy, const T (&U)[DIM + 2],
                       const typename Euler<DIM>::template Prim<T>& q, PrimBar<T>& b,
                       T (&gU)[DIM + 2]) {
  constexpr int E = DIM + 1;
  const T gm1 = T(sy.gas - 1.0);
  gU[E] += b.Ep;
  b.p += b.Ep;
  gU[E] += gm1 * b.p;
  gU[0] -= gm1 * q.k * b.p;
  b.k -= gm1 * U[0] * b.p;
  b.mu += q.mu * b.k;
  gU[1] += q.ir * b.mu;
  b.ir += U[1] * b.mu;
  if constexpr (DIM == 2) {
    b.nu += q.nu * b.k;
    gU[2] += q.ir * b.nu;
    b.ir += U[2] * b.nu;
  }
  gU[0] -= q.ir * q.ir * b.ir;
}

template <int D, int DIM, typename T>
HWENO_HD void flux_vjp(const Euler<DIM>&, const T (&U)[DIM + 2],
                       const typename Euler<DIM>::template Prim<T>& q, const T (&gF)[DIM + 2],
                       PrimBar<T>& b, T (&gU)[DIM + 2]) {
  if constexpr (DIM == 1) {
    // F = (m, m u + P, u Ep)
    gU[1] += gF[0] + q.mu * gF[1];
    b.mu += U[1] * gF[1] + q.Ep * gF[2];
    b.p += gF[1];
    b.Ep += q.mu * gF[2];
  } else if constexpr (D == 0) {
    // F = (m, m u + P, m v, u Ep)
    gU[1] += gF[0] + q.mu * gF[1] + q.nu * gF[2];
    b.mu += U[1] * gF[1] + q.Ep * gF[3];
    b.nu += U[1] * gF[2];
    b.p += gF[1];
    b.Ep += q.mu * gF[3];
  } else {
    // G = (n, n u, n v + P, v Ep)
    gU[2] += gF[0] + q.mu * gF[1] + q.nu * gF[2];
    b.mu += U[2] * gF[1];
    b.nu += U[2] * gF[2] + q.Ep * gF[3];
    b.p += gF[2];
    b.Ep += q.nu * gF[3];
  }
}

// Reverse of Euler::jac (A(U) V through du, dv, dP), cotangent gO.
template <int D, int DIM, typename T>
HWENO_HD void jac_vjp(const Euler<DIM>& sy, const T (&U)[DIM + 2],
                      const typename Euler<DIM>::template Prim<T>& q, const T (&V)[DIM + 2],
                      const T (&gO)[DIM + 2], PrimBar<T>& b, T (&gU)[DIM + 2],
                      T (&gV)[DIM + 2]) {
  const T gm1 = T(sy.gas - 1.0);
  if constexpr (DIM == 1) {
    const T du = (V[1] - q.mu * V[0]) * q.ir;
    const T dP = gm1 * (V[2] - q.mu * V[1] + q.k * V[0]);
    // O = (V1, u V1 + m du + dP, du Ep + u (V2 + dP))
    gV[1] += gO[0] + q.mu * gO[1];
    b.mu += V[1] * gO[1] + (V[2] + dP) * gO[2];
    gU[1] += du * gO[1];
    const T gdu = U[1] * gO[1] + q.Ep * gO[2];
    const T gdP = gO[1] + q.mu * gO[2];
    b.Ep += du * gO[2];
    gV[2] += q.mu * gO[2];
    // dP
    gV[2] += gm1 * gdP;
    b.mu -= gm1 * V[1] * gdP;
    gV[1] -= gm1 * q.mu * gdP;
    b.k += gm1 * V[0] * gdP;
    gV[0] += gm1 * q.k * gdP;
    // du
    gV[1] += q.ir * gdu;
    b.mu -= V[0] * q.ir * gdu;
    gV[0] -= q.mu * q.ir * gdu;
    b.ir += (V[1] - q.mu * V[0]) * gdu;
  } else {
    const T du = (V[1] - q.mu * V[0]) * q.ir;
    const T dv = (V[2] - q.nu * V[0]) * q.ir;
    const T dP = gm1 * (V[3] - q.mu * V[1] - q.nu * V[2] + q.k * V[0]);
    T gdu, gdv, gdP;
    if constexpr (D == 0) {
      // O = (V1, u V1 + m du + dP, v V1 + m dv, du Ep + u (V3 + dP))
      gV[1] += gO[0] + q.mu * gO[1] + q.nu * gO[2];
      b.mu += V[1] * gO[1] + (V[3] + dP) * gO[3];
      b.nu += V[1] * gO[2];
      gU[1] += du * gO[1] + dv * gO[2];
      gdu = U[1] * gO[1] + q.Ep * gO[3];
      gdv = U[1] * gO[2];
      gdP = gO[1] + q.mu * gO[3];
      b.Ep += du * gO[3];
      gV[3] += q.mu * gO[3];
    } else {
      // O = (V2, u V2 + n du, v V2 + n dv + dP, dv Ep + v (V3 + dP))
      gV[2] += gO[0] + q.mu * gO[1] + q.nu * gO[2];
      b.mu += V[2] * gO[1];
      b.nu += V[2] * gO[2] + (V[3] + dP) * gO[3];
      gU[2] += du * gO[1] + dv * gO[2];
      gdu = U[2] * gO[1];
      gdv = U[2] * gO[2] + q.Ep * gO[3];
      gdP = gO[2] + q.nu * gO[3];
      b.Ep += dv * gO[3];
      gV[3] += q.nu * gO[3];
    }
    // dP = (g-1)(V3 - u V1 - v V2 + k V0)
    gV[3] += gm1 * gdP;
    b.mu -= gm1 * V[1] * gdP;
    gV[1] -= gm1 * q.mu * gdP;
    b.nu -= gm1 * V[2] * gdP;
    gV[2] -= gm1 * q.nu * gdP;
    b.k += gm1 * V[0] * gdP;
    gV[0] += gm1 * q.k * gdP;
    // du = (V1 - u V0) ir, dv = (V2 - v V0) ir
    gV[1] += q.ir * gdu;
    b.mu -= V[0] * q.ir * gdu;
    gV[0] -= q.mu * q.ir * gdu;
    b.ir += (V[1] - q.mu * V[0]) * gdu;
    gV[2] += q.ir * gdv;
    b.nu -= V[0] * q.ir * gdv;
    gV[0] -= q.nu * q.ir * gdv;
    b.ir += (V[2] - q.nu * V[0]) * gdv;
  }
}

// Reverse of Euler::eig: c2 = g P ir, ic = c2^(-1/2), c = c2 ic, H = Ep ir,
// b1 = (g-1) ic^2, b2 = b1 k.
template <int DIM, typename T>
HWENO_HD void eig_vjp(const Euler<DIM>& sy, const typename Euler<DIM>::template Prim<T>& q,
                      const typename Euler<DIM>::template Eig<T>& e, EigBar<T> eb,
                      PrimBar<T>& pb) {
  eb.b1 += q.k * eb.b2;
  eb.k += e.b1 * eb.b2;
  eb.ic += T(2.0 * (sy.gas - 1.0)) * e.ic * eb.b1;
  const T c2 = T(sy.gas) * q.p * q.ir;
  T gc2 = e.ic * eb.c;
  eb.ic += c2 * eb.c;
  gc2 += T(-0.5) * e.ic * e.ic * e.ic * eb.ic;
  pb.p += T(sy.gas) * q.ir * gc2;
  pb.ir += T(sy.gas) * q.p * gc2 + q.Ep * eb.H;
  pb.Ep += q.ir * eb.H;
  pb.mu += eb.mu;
  pb.nu += eb.nu;
  pb.k += eb.k;
}

// Reverse of Euler::project<D> (w = L U): cotangent gw -> gU, eigen-parameters.
template <int D, int DIM, typename T>
HWENO_HD void project_vjp(const Euler<DIM>&, const typename Euler<DIM>::template Eig<T>& e,
                          const T (&U)[DIM + 2], const T (&gw)[DIM + 2], EigBar<T>& eb,
                          T (&gU)[DIM + 2]) {
  if constexpr (DIM == 1) {
    const T gs = T(0.5) * (gw[0] + gw[2]) - gw[1];
    const T gt = T(0.5) * (gw[0] - gw[2]);
    gU[0] += gw[1] + e.b2 * gs + e.ic * e.mu * gt;
    gU[1] += -e.b1 * e.mu * gs - e.ic * gt;
    gU[2] += e.b1 * gs;
    eb.b2 += U[0] * gs;
    eb.b1 -= (e.mu * U[1] - U[2]) * gs;
    eb.mu += -e.b1 * U[1] * gs + e.ic * U[0] * gt;
    eb.ic += (e.mu * U[0] - U[1]) * gt;
  } else {
    const T gs = T(0.5) * (gw[0] + gw[3]) - gw[1];
    const T gt = T(0.5) * (gw[0] - gw[3]);
    gU[0] += gw[1] + e.b2 * gs;
    gU[1] -= e.b1 * e.mu * gs;
    gU[2] -= e.b1 * e.nu * gs;
    gU[3] += e.b1 * gs;
    eb.b2 += U[0] * gs;
    eb.b1 -= (e.mu * U[1] + e.nu * U[2] - U[3]) * gs;
    eb.mu -= e.b1 * U[1] * gs;
    eb.nu -= e.b1 * U[2] * gs;
    if constexpr (D == 0) {
      // t = ic (u U0 - U1); w2 = U2 - v U0
      gU[0] += e.ic * e.mu * gt - e.nu * gw[2];
      gU[1] -= e.ic * gt;
      gU[2] += gw[2];
      eb.mu += e.ic * U[0] * gt;
      eb.ic += (e.mu * U[0] - U[1]) * gt;
      eb.nu -= U[0] * gw[2];
    } else {
      // t = ic (v U0 - U2); w2 = U1 - u U0
      gU[0] += e.ic * e.nu * gt - e.mu * gw[2];
      gU[2] -= e.ic * gt;
      gU[1] += gw[2];
      eb.nu += e.ic * U[0] * gt;
      eb.ic += (e.nu * U[0] - U[2]) * gt;
      eb.mu -= U[0] * gw[2];
    }
  }
}

// Reverse of Euler::unproject<D> (U = R x): cotangent gU -> gx, eigen-parameters.
template <int D, int DIM, typename T>
HWENO_HD void unproject_vjp(const Euler<DIM>&, const typename Euler<DIM>::template Eig<T>& e,
                            const T (&x)[DIM + 2], const T (&gU)[DIM + 2], EigBar<T>& eb,
                            T (&gx)[DIM + 2]) {
  if constexpr (DIM == 1) {
    const T a = x[0] + x[2], dd = x[2] - x[0];
    const T s0 = a + x[1];
    const T gS0 = gU[0] + e.mu * gU[1];
    const T gdd = e.c * gU[1] + e.mu * e.c * gU[2];
    const T ga = gS0 + e.H * gU[2];
    gx[1] += gS0 + e.k * gU[2];
    gx[0] += ga - gdd;
    gx[2] += ga + gdd;
    eb.mu += s0 * gU[1] + e.c * dd * gU[2];
    eb.c += dd * gU[1] + e.mu * dd * gU[2];
    eb.H += a * gU[2];
    eb.k += x[1] * gU[2];
  } else {
    const T a = x[0] + x[3], dd = x[3] - x[0];
    const T s0 = a + x[1];
    const T vn = D == 0 ? e.mu : e.nu, vt = D == 0 ? e.nu : e.mu;
    const T gS0 = gU[0] + e.mu * gU[1] + e.nu * gU[2];
    const T gUn = D == 0 ? gU[1] : gU[2];   // normal momentum row: vn s0 + c dd
    const T gUt = D == 0 ? gU[2] : gU[1];   // transverse momentum row: vt s0 + x2
    const T gdd = e.c * gUn + vn * e.c * gU[3];
    const T ga = gS0 + e.H * gU[3];
    gx[1] += gS0 + e.k * gU[3];
    gx[2] += gUt + vt * gU[3];
    gx[0] += ga - gdd;
    gx[3] += ga + gdd;
    const T gvn = s0 * gUn + e.c * dd * gU[3];
    const T gvt = s0 * gUt + x[2] * gU[3];
    if (D == 0) { eb.mu += gvn; eb.nu += gvt; } else { eb.nu += gvn; eb.mu += gvt; }
    eb.c += dd * gUn + vn * dd * gU[3];
    eb.H += a * gU[3];
    eb.k += x[1] * gU[3];
  }
}

// The two parts of unproject_vjp, for use one component at a time.
// unproject_t: gx += R^T gU (the cotangent of c). unproject_eb: the basis
// cotangent from component c_j alone (R c is linear in c, so the parts of all
// components add up to unproject_vjp's). With a = c_0 + c_E, dd = c_E - c_0,
// s0 = a + c_1: U = (s0, vel s0 + c dd n [+ c_2 t], H a + vn c dd + k c_1
// [+ vt c_2]).
template <int D, int DIM, typename T>
HWENO_HD void unproject_t(const Euler<DIM>&, const typename Euler<DIM>::template Eig<T>& e,
                          const T (&gU)[DIM + 2], T (&gx)[DIM + 2]) {
  if constexpr (DIM == 1) {
    const T gS0 = gU[0] + e.mu * gU[1];
    const T gdd = e.c * gU[1] + e.mu * e.c * gU[2];
    const T ga = gS0 + e.H * gU[2];
    gx[1] += gS0 + e.k * gU[2];
    gx[0] += ga - gdd;
    gx[2] += ga + gdd;
  } else {
    const T vn = D == 0 ? e.mu : e.nu, vt = D == 0 ? e.nu : e.mu;
    const T gS0 = gU[0] + e.mu * gU[1] + e.nu * gU[2];
    const T gUn = D == 0 ? gU[1] : gU[2];
    const T gUt = D == 0 ? gU[2] : gU[1];
    const T gdd = e.c * gUn + vn * e.c * gU[3];
    const T ga = gS0 + e.H * gU[3];
    gx[1] += gS0 + e.k * gU[3];
    gx[2] += gUt + vt * gU[3];
    gx[0] += ga - gdd;
    gx[3] += ga + gdd;
  }
}
template <int D, int DIM, typename T>
HWENO_HD void unproject_eb(const Euler<DIM>&, const typename Euler<DIM>::template Eig<T>& e, int j,
                           T xj, const T (&gU)[DIM + 2], EigBar<T>& eb) {
  constexpr int E = DIM + 1;
  const T gUn = (DIM == 1 || D == 0) ? gU[1] : gU[2];
  const T gUt = DIM == 1 ? T(0) : (D == 0 ? gU[2] : gU[1]);
  const T vn = D == 0 ? e.mu : e.nu;
  T gvn = T(0), gvt = T(0);
  if (j == 0 || j == E) {
    const T sg = j == 0 ? T(-1) : T(1);   // d dd / d c_j
    gvn = xj * (gUn + sg * e.c * gU[E]);
    gvt = xj * gUt;
    eb.c += sg * xj * (gUn + vn * gU[E]);
    eb.H += xj * gU[E];
  } else if (j == 1) {
    gvn = xj * gUn;
    gvt = xj * gUt;
    eb.k += xj * gU[E];
  } else {   // j == 2 in 2D: the transverse-velocity column
    gvt = xj * gU[E];
  }
  if (D == 0) { eb.mu += gvn; eb.nu += gvt; } else { eb.nu += gvn; eb.mu += gvt; }
}

// ---------------------------------------------------- one cell's HWENO
// Reverse of hweno_cell<D>: cotangents (guR, guL, gat) of (uR, uL, v~) ->
// contributions to the five stencil inputs. kFused: through
// hweno_point_vjp_fused (for callers that ran hweno_cell<D> on the same data
// just before and can keep its intermediates), else hweno_point_vjp.
template <int D, bool kFused = false, class Sys, typename T>
HWENO_HD void hweno_cell_vjp(const Sys& sy, const Scheme& s, double h, double ih,
                             const T (&Um)[Sys::NC], const T (&U0)[Sys::NC],
                             const T (&Up)[Sys::NC], const T (&Am)[Sys::NC],
                             const T (&Ap)[Sys::NC], const T (&guR)[Sys::NC],
                             const T (&guL)[Sys::NC], const T (&gat)[Sys::NC],
                             T (&gUm)[Sys::NC], T (&gU0)[Sys::NC], T (&gUp)[Sys::NC],
                             T (&gAm)[Sys::NC], T (&gAp)[Sys::NC]) {
  constexpr int NC = Sys::NC;
  if constexpr (!Sys::kChar) {
    if constexpr (kFused) {
      T fR, fL, fT;
      hweno_point_vjp_fused<T>(Um[0], U0[0], Up[0], Am[0], Ap[0], s, h, ih, (double)guR[0],
                               (double)guL[0], (double)gat[0], gUm[0], gU0[0], gUp[0], gAm[0],
                               gAp[0], fR, fL, fT);
    } else {
      hweno_point_vjp<T>(Um[0], U0[0], Up[0], Am[0], Ap[0], s, h, ih, (double)guR[0],
                         (double)guL[0], (double)gat[0], gUm[0], gU0[0], gUp[0], gAm[0], gAp[0]);
    }
  } else {
    const auto q = sy.prim(U0);
    const auto e = sy.eig(q);
    T wm[NC], w0[NC], wp[NC], am[NC], ap[NC];
    sy.template project<D>(e, Um, wm);
    sy.template project<D>(e, U0, w0);
    sy.template project<D>(e, Up, wp);
    sy.template project<D>(e, Am, am);
    sy.template project<D>(e, Ap, ap);
    EigBar<T> eb;
    T gwm[NC], gw0[NC], gwp[NC], gam[NC], gap[NC];
    if constexpr (kFused) {
      // cotangents of the characteristic values first (R^T g needs no
      // forward values), then each component's reverse, which also returns
      // its forward values for the basis cotangent
      T gcr[NC], gcl[NC], gct[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) { gcr[j] = T(0); gcl[j] = T(0); gct[j] = T(0); }
      unproject_t<D>(sy, e, guR, gcr);
      unproject_t<D>(sy, e, guL, gcl);
      unproject_t<D>(sy, e, gat, gct);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        gwm[j] = T(0); gw0[j] = T(0); gwp[j] = T(0); gam[j] = T(0); gap[j] = T(0);
        T cr, cl, ct;
        hweno_point_vjp_fused<T>(wm[j], w0[j], wp[j], am[j], ap[j], s, h, ih, (double)gcr[j],
                                 (double)gcl[j], (double)gct[j], gwm[j], gw0[j], gwp[j], gam[j],
                                 gap[j], cr, cl, ct);
        unproject_eb<D>(sy, e, j, cr, guR, eb);
        unproject_eb<D>(sy, e, j, cl, guL, eb);
        unproject_eb<D>(sy, e, j, ct, gat, eb);
      }
    } else {
      T cr[NC], cl[NC], ct[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j)
        hweno_point<T>(wm[j], w0[j], wp[j], am[j], ap[j], s, h, ih, cr[j], cl[j], ct[j]);
      T gcr[NC], gcl[NC], gct[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) { gcr[j] = T(0); gcl[j] = T(0); gct[j] = T(0); }
      unproject_vjp<D>(sy, e, cr, guR, eb, gcr);
      unproject_vjp<D>(sy, e, cl, guL, eb, gcl);
      unproject_vjp<D>(sy, e, ct, gat, eb, gct);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        gwm[j] = T(0); gw0[j] = T(0); gwp[j] = T(0); gam[j] = T(0); gap[j] = T(0);
        hweno_point_vjp<T>(wm[j], w0[j], wp[j], am[j], ap[j], s, h, ih, (double)gcr[j],
                           (double)gcl[j], (double)gct[j], gwm[j], gw0[j], gwp[j], gam[j], gap[j]);
      }
    }
    project_vjp<D>(sy, e, Um, gwm, eb, gUm);
    project_vjp<D>(sy, e, U0, gw0, eb, gU0);
    project_vjp<D>(sy, e, Up, gwp, eb, gUp);
    project_vjp<D>(sy, e, Am, gam, eb, gAm);
    project_vjp<D>(sy, e, Ap, gap, eb, gAp);
    PrimBar<T> pb;
    eig_vjp(sy, q, e, eb, pb);
    prim_vjp(sy, U0, q, pb, gU0);
  }
}

// Reverse of Euler::roe_eig (the basis of Roe's matrix of UL, UR): the
// basis cotangent eb -> contributions to both states. Forward: r = rho^-1/2,
// a = 1/(rho_L r_L + rho_R r_R), m = U_1 r, n = U_2 r, p = (g-1)(U_E - (m^2 +
// n^2)/2), X = U_E + p; mu = (m_L + m_R) a, nu = (n_L + n_R) a, H = (X_L r_L
// + X_R r_R) a, k = (mu^2 + nu^2)/2, c2 = (g-1)(H - k), ic = c2^-1/2,
// c = c2 ic, b1 = (g-1) ic^2, b2 = b1 k.
template <int DIM, typename T>
HWENO_HD void roe_eig_vjp(const Euler<DIM>& sy, const T (&UL)[DIM + 2], const T (&UR)[DIM + 2],
                          const typename Euler<DIM>::template Eig<T>& e, EigBar<T> eb,
                          T (&gUL)[DIM + 2], T (&gUR)[DIM + 2]) {
  constexpr int E = DIM + 1;
  const T gm1 = T(sy.gas - 1.0);
  const T rl = rsqrt_nr(UL[0]), rr = rsqrt_nr(UR[0]);
  const T a = rcp_nr(UL[0] * rl + UR[0] * rr);
  const T ml = UL[1] * rl, mr = UR[1] * rr;
  const T nl = DIM == 2 ? UL[2] * rl : T(0), nr = DIM == 2 ? UR[2] * rr : T(0);
  const T XL = UL[E] + gm1 * (UL[E] - T(0.5) * (ml * ml + nl * nl));
  const T XR = UR[E] + gm1 * (UR[E] - T(0.5) * (mr * mr + nr * nr));
  const T c2 = gm1 * (e.H - e.k);
  eb.b1 += e.k * eb.b2;
  eb.k += e.b1 * eb.b2;
  eb.ic += T(2) * gm1 * e.ic * eb.b1;
  T gc2 = e.ic * eb.c;
  eb.ic += c2 * eb.c;
  gc2 += T(-0.5) * e.ic * e.ic * e.ic * eb.ic;
  eb.H += gm1 * gc2;
  eb.k -= gm1 * gc2;
  eb.mu += e.mu * eb.k;
  eb.nu += e.nu * eb.k;
  const T ga = (ml + mr) * eb.mu + (nl + nr) * eb.nu + (XL * rl + XR * rr) * eb.H;
  T gml = a * eb.mu, gmr = a * eb.mu;
  T gnl = a * eb.nu, gnr = a * eb.nu;
  const T gXL = rl * a * eb.H, gXR = rr * a * eb.H;
  T grl = XL * a * eb.H, grr = XR * a * eb.H;
  gUL[E] += (T(1) + gm1) * gXL;
  gml -= gm1 * ml * gXL;
  gnl -= gm1 * nl * gXL;
  gUR[E] += (T(1) + gm1) * gXR;
  gmr -= gm1 * mr * gXR;
  gnr -= gm1 * nr * gXR;
  gUL[1] += rl * gml;
  grl += UL[1] * gml;
  gUR[1] += rr * gmr;
  grr += UR[1] * gmr;
  if constexpr (DIM == 2) {
    gUL[2] += rl * gnl;
    grl += UL[2] * gnl;
    gUR[2] += rr * gnr;
    grr += UR[2] * gnr;
  }
  const T gS = -a * a * ga;
  gUL[0] += rl * gS;
  grl += UL[0] * gS;
  gUR[0] += rr * gS;
  grr += UR[0] * gS;
  gUL[0] += T(-0.5) * rl * rl * rl * grl;
  gUR[0] += T(-0.5) * rr * rr * rr * grr;
}

// Reverse of hweno_cell_iface<D> (the interface-basis switch): the right-face
// value in the basis of Roe's matrix of (U0, Up), the left-face value in that
// of (Um, U0), v~ in the cell basis; each application is reversed with its
// basis, whose cotangent goes to the states that define it. The three
// applications run as one rolled loop (the index is wave-uniform), so that
// only one application's intermediates are live at a time.
template <int D, class Sys, typename T>
HWENO_HD void hweno_cell_iface_vjp(const Sys& sy, const Scheme& s, double h, double ih,
                                   const T (&Um)[Sys::NC], const T (&U0)[Sys::NC],
                                   const T (&Up)[Sys::NC], const T (&Am)[Sys::NC],
                                   const T (&Ap)[Sys::NC], const T (&guR)[Sys::NC],
                                   const T (&guL)[Sys::NC], const T (&gat)[Sys::NC],
                                   T (&gUm)[Sys::NC], T (&gU0)[Sys::NC], T (&gUp)[Sys::NC],
                                   T (&gAm)[Sys::NC], T (&gAp)[Sys::NC]) {
  constexpr int NC = Sys::NC;
  if constexpr (!Sys::kChar) {
    hweno_cell_vjp<D>(sy, s, h, ih, Um, U0, Up, Am, Ap, guR, guL, gat, gUm, gU0, gUp, gAm, gAp);
  } else {
#pragma unroll 1
    for (int which = 0; which < 3; ++which) {
      // the basis: Roe's matrix of (UL, UR) for the faces, the cell's for v~
      const bool roe = which < 2;
      T UL[NC], UR[NC], gout[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        UL[c] = which == 0 ? U0[c] : Um[c];
        UR[c] = which == 0 ? Up[c] : U0[c];
        gout[c] = which == 0 ? guR[c] : (which == 1 ? guL[c] : gat[c]);
      }
      const auto q = sy.prim(U0);
      const auto e = roe ? sy.roe_eig(UL, UR) : sy.eig(q);
      T wm[NC], w0[NC], wp[NC], am[NC], ap[NC];
      sy.template project<D>(e, Um, wm);
      sy.template project<D>(e, U0, w0);
      sy.template project<D>(e, Up, wp);
      sy.template project<D>(e, Am, am);
      sy.template project<D>(e, Ap, ap);
      // cotangents of the characteristic values first (R^T g needs no
      // forward values), then each component's reverse, which also returns
      // its forward values for the basis cotangent
      EigBar<T> eb;
      T gc[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) gc[j] = T(0);
      unproject_t<D>(sy, e, gout, gc);
      T gwm[NC], gw0[NC], gwp[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        gwm[j] = T(0); gw0[j] = T(0); gwp[j] = T(0);
        T gam = T(0), gap = T(0), r_, l_, t_;
        const double g = (double)gc[j];
        hweno_point_vjp_fused<T>(wm[j], w0[j], wp[j], am[j], ap[j], s, h, ih, which == 0 ? g : 0.0,
                                 which == 1 ? g : 0.0, which == 2 ? g : 0.0, gwm[j], gw0[j],
                                 gwp[j], gam, gap, r_, l_, t_);
        unproject_eb<D>(sy, e, j, which == 0 ? r_ : (which == 1 ? l_ : t_), gout, eb);
        am[j] = gam;   // the projected derivatives are not needed again
        ap[j] = gap;
      }
      // am, ap hold their cotangents now; project_vjp reads the states only
      project_vjp<D>(sy, e, Am, am, eb, gAm);
      project_vjp<D>(sy, e, Ap, ap, eb, gAp);
      project_vjp<D>(sy, e, Um, gwm, eb, gUm);
      project_vjp<D>(sy, e, U0, gw0, eb, gU0);
      project_vjp<D>(sy, e, Up, gwp, eb, gUp);
      if (roe) {
        T gL[NC], gR[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) { gL[k] = T(0); gR[k] = T(0); }
        roe_eig_vjp(sy, UL, UR, e, eb, gL, gR);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          gUm[k] += which == 1 ? gL[k] : T(0);
          gU0[k] += which == 0 ? gL[k] : gR[k];
          gUp[k] += which == 0 ? gR[k] : T(0);
        }
      } else {
        PrimBar<T> pb;
        eig_vjp(sy, q, e, eb, pb);
        prim_vjp(sy, U0, q, pb, gU0);
      }
    }
  }
}

// Either basis, by template flag.
template <int D, bool IFACE, bool kFused = false, class Sys, typename T>
HWENO_HD void hweno_cell_vjp_b(const Sys& sy, const Scheme& s, double h, double ih,
                               const T (&Um)[Sys::NC], const T (&U0)[Sys::NC],
                               const T (&Up)[Sys::NC], const T (&Am)[Sys::NC],
                               const T (&Ap)[Sys::NC], const T (&guR)[Sys::NC],
                               const T (&guL)[Sys::NC], const T (&gat)[Sys::NC],
                               T (&gUm)[Sys::NC], T (&gU0)[Sys::NC], T (&gUp)[Sys::NC],
                               T (&gAm)[Sys::NC], T (&gAp)[Sys::NC]) {
  if constexpr (IFACE)
    hweno_cell_iface_vjp<D>(sy, s, h, ih, Um, U0, Up, Am, Ap, guR, guL, gat, gUm, gU0, gUp, gAm, gAp);
  else
    hweno_cell_vjp<D, kFused>(sy, s, h, ih, Um, U0, Up, Am, Ap, guR, guL, gat, gUm, gU0, gUp, gAm, gAp);
}

// Reverse of central_corr (linear): interface cotangents (gDf, gDh) ->
// contributions to f_{i-1..i+2}, h_{i-1}, h_{i+2}.
template <typename T>
HWENO_HD void central_corr_vjp(T gDf, T gDh, T h, T ih, T& gfm1, T& gf0, T& gfp1, T& gfp2,
                               T& ghm1, T& ghp2) {
  const T a = T(-97.0 / 1920.0) * gDf;
  const T b = T(697.0 / 5184.0) * ih * gDh;
  const T c = T(61.0 / 192.0) * ih * gDh;
  gfm1 += a + b;
  gf0 += -a - c;
  gfp1 += -a + c;
  gfp2 += a - b;
  const T d = T(19.0 / 960.0) * h * gDf;
  const T e = T(37.0 / 864.0) * gDh;
  ghm1 += -d + e;
  ghp2 += d + e;
}

}  // namespace hweno
