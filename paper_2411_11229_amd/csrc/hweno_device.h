// Device math of the HWENO-I scheme for gfx950 (Xie, Tao, Jiao, Zhang,
// arXiv 2411.11229). Everything here is per point or per lane; the kernels in
// hweno_kernels.hip arrange it into marching stencil sweeps.
//
// Type conventions: T is the storage / streaming type (double or float).
// The smoothness indicators, tau, epsilon and the nonlinear-weight ratios are
// always evaluated in double, as are the flux differences and the Runge-Kutta
// combination (done by the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-point functions compile for the host too (a CPU harness checks the
// adjoint of each against finite differences); lane shifts and kernels are
// device-only.
#define HWENO_HD __host__ __device__ __forceinline__

namespace hweno {

constexpr int kWave = 64;                 // lanes per wavefront (CDNA)
constexpr int kHalo = 2;                  // stencil radius: x_{i+1/2} reads cells i-1..i+2
constexpr int kXOut = kWave - 2 * kHalo;  // output columns per wavefront

// Scheme constants as the kernels need them.
struct Scheme {
  double dx, dy, idx, idy;  // mesh widths and their inverses
  double gamma0, g1;        // linear weights of (interp); g1 = gamma1 = gamma2
  double d0, d1;            // linear weights of (limiter); d1 = d2
  double eps;               // epsilon of (nonlinear)
  double gas;               // ratio of specific heats (Euler)
  double adv_a, adv_b;      // advection speeds
};

// ---------------------------------------------------------------- lane shifts
// Values of the neighbouring lane along x (lanes are consecutive cells).
// DPP wave_shr:1 / wave_shl:1 row moves: lane i receives lane i-1 / i+1; the
// lane without a source (0, resp. 63) receives 0, which only halo lanes see.
// One VALU move per 32-bit word, with no LDS round trip.
__device__ __forceinline__ int dpp_prev_i32(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_next_i32(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x130, 0xf, 0xf, true);
}
template <typename T> __device__ __forceinline__ T from_prev(T x);
template <typename T> __device__ __forceinline__ T from_next(T x);
template <>
__device__ __forceinline__ double from_prev<double>(double x) {
  return __hiloint2double(dpp_prev_i32(__double2hiint(x)), dpp_prev_i32(__double2loint(x)));
}
template <>
__device__ __forceinline__ double from_next<double>(double x) {
  return __hiloint2double(dpp_next_i32(__double2hiint(x)), dpp_next_i32(__double2loint(x)));
}
template <>
__device__ __forceinline__ float from_prev<float>(float x) {
  return __int_as_float(dpp_prev_i32(__float_as_int(x)));
}
template <>
__device__ __forceinline__ float from_next<float>(float x) {
  return __int_as_float(dpp_next_i32(__float_as_int(x)));
}
template <typename T>
__device__ __forceinline__ T from_next2(T x) { return from_next(from_next(x)); }

// ---------------------------------------------------------------- reciprocals
// Hardware reciprocal (square root) estimate refined by Newton steps: within
// an ulp or two of the correctly rounded value, for the positive, finite,
// normal arguments the scheme produces, at half the instructions of an IEEE
// division.
HWENO_HD double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
HWENO_HD float rcp_nr(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}
HWENO_HD double rsqrt_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
  // y <- y (3 - x y^2) / 2, twice
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
#else
  return 1.0 / sqrt(x);
#endif
}
HWENO_HD float rsqrt_nr(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  float y = __builtin_amdgcn_rsqf(x);
  return y * fmaf(-0.5f * x * y, y, 1.5f);
#else
  return 1.0f / sqrtf(x);
#endif
}

// ---------------------------------------------------------------- HWENO-I
// One HWENO-I application on one scalar line (a conserved component for the
// scalar laws, a characteristic variable for systems), section 2.1:
// from u_{i-1}, u_i, u_{i+1}, v_{i-1}, v_{i+1} it returns
//   uR = u^-_{i+1/2} and uL = u^+_{i-1/2}  -- (interp) and its mirror image,
//   vt = the modified derivative at x_i    -- (limiter),
// sharing one set of smoothness indicators (GHYZ) between the three.
//
// Arithmetic: with r_l = tau/(beta_l + eps), o_l = 1 + r_l, the normalised
// weights are w_l = lin_l o_l / S, S = gamma0 o0 + g1 (o1 + o2) (gamma1 =
// gamma2 = g1, the paper's choice). The o_l are used multiplied by the
// positive common factor (beta0+eps)(beta1+eps)(beta2+eps), which the
// normalisations cancel, so no division is needed for the ratios. Written through the one-sided
// differences e1 = u_i - u_{i-1}, e2 = u_{i+1} - u_i, the candidates are
// p1 = u_i + e1/2, p2 = u_i + e2/2 and p0 = u_i + e1/8 + 9e2/16 -
// dx(3v_{i-1} + 9v_{i+1})/64; the u_i terms of (interp) add up to u_i S, so
//   u^-_{i+1/2} = u_i + [o0 B_R + (g1/2) X] / S,
//   u^+_{i-1/2} = u_i - [o0 B_L + (g1/2) X] / S,
//   v~_i        = [o0 ((3/4 - d1)(e1 + e2)/dx - (v_{i-1} + v_{i+1})/4) + d1 X/dx] / S_d,
// with X = o1 e1 + o2 e2, B_R = k1 e1 + k2 e2 - dx(3v_{i-1} + 9v_{i+1})/64,
// B_L = k2 e1 + k1 e2 - dx(9v_{i-1} + 3v_{i+1})/64, k1 = 1/8 - g1/2,
// k2 = 9/16 - g1/2 and S_d = d0 o0 + d1 (o1 + o2). Both normalisations
// share one division. Range: the scaled o_l grow like beta^4, so the product
// of the normalisations stays finite for jumps below about 1e17 in the
// variable interpolated.
template <typename T>
HWENO_HD void hweno_point(T um, T u0, T up, T vm, T vp, const Scheme& s,
                                            double h, double ih, T& uR, T& uL, T& vt) {
  const double dc = (double)u0;
  const double e1 = dc - (double)um, e2 = (double)up - dc;
  const double vmd = (double)vm, vpd = (double)vp;
  // (GHYZ) closed form: cdf = u_{i+1} - u_{i-1}, sdf = u_{i-1} - 2u_i + u_{i+1},
  // sv = dx (v_{i-1} + v_{i+1})/4, dv = dx (v_{i-1} - v_{i+1})/4
  const double cdf = e1 + e2, sdf = e2 - e1;
  const double qh = 0.25 * h;
  const double sv = qh * (vmd + vpd), dv = qh * (vmd - vpd);
  // beta0 = t1^2 + 13/3 t2^2 + 781/20 a3^2 + 1421461/2275 a4^2 with
  // t1 = a1 + a3/4, t2 = a2 + 63/130 a4, a3 = sv - cdf/4, a4 = -sdf/2 - dv;
  // the weights' square roots are folded into the combinations
  constexpr double r13 = 2.0816659994661326;    // sqrt(13/3)
  constexpr double r781 = 6.248999919987197;    // sqrt(781/20)
  constexpr double r1421 = 24.99636017459386;   // sqrt(1421461/2275)
  const double t1 = 0.6875 * cdf - 0.75 * sv;
  const double t2 = (r13 * 197.0 / 260.0) * sdf + (r13 * 67.0 / 130.0) * dv;
  const double a3 = r781 * sv - (0.25 * r781) * cdf;
  const double a4 = (-0.5 * r1421) * sdf - r1421 * dv;
  const double b0 = t1 * t1 + t2 * t2 + a3 * a3 + a4 * a4;
  const double b1 = e1 * e1, b2 = e2 * e2;
  // (nonlinear)
  const double ts = fabs(b0 - b1) + fabs(b0 - b2);
  const double tau = 0.25 * ts * ts;
  const double q0 = b0 + s.eps, q1 = b1 + s.eps, q2 = b2 + s.eps;
  // o_l scaled by P = q0 q1 q2 > 0 (every result below is homogeneous of
  // degree 0 in the o_l): P o_l = P + tau P/q_l
  const double o0 = (q1 * q2) * (q0 + tau);
  const double o1 = (q0 * q2) * (q1 + tau);
  const double o2 = (q0 * q1) * (q2 + tau);
  const double o12 = o1 + o2;
  const double Sg = s.gamma0 * o0 + s.g1 * o12;
  const double Sd = s.d0 * o0 + s.d1 * o12;
  const double inv = rcp_nr(Sg * Sd);
  const double iSg = Sd * inv, iSd = Sg * inv;
  // (Pxi), its mirror image and (limiter-p), combined as above; with
  // K = (k1 + k2)/2 and k2 - k1 = 7/16: B_R = base + m, B_L = base - m
  const double X = o1 * e1 + o2 * e2;
  const double gX = 0.5 * s.g1 * X;
  const double K = 0.34375 - 0.5 * s.g1;
  const double base = K * cdf - 0.375 * sv;
  const double m = 0.21875 * sdf + 0.1875 * dv;
  const double P1 = o0 * base + gX, P2 = o0 * m;
  uR = (T)(dc + (P1 + P2) * iSg);
  uL = (T)(dc - (P1 - P2) * iSg);
  const double AT = (0.75 - s.d1) * ih * cdf - ih * sv;
  vt = (T)((o0 * AT + s.d1 * ih * X) * iSd);
}

// ------------------------------------------------- HWENO-I, difference form
// The forward stage kernels apply the same interpolation to the stencil's
// differences, and carry every derivative multiplied by the mesh width of
// its direction (v' = dx v, w' = dy w): then no constant of the
// interpolation depends on the mesh. From e1 = u_i - u_{i-1},
// e2 = u_{i+1} - u_i, S = v'_{i-1} + v'_{i+1}, D = v'_{i-1} - v'_{i+1} (a
// linear map of the stencil, so for systems they are projected on the
// characteristic basis in place of the five values, and u_i itself is never
// projected) it returns the face corrections dR = u^-_{i+1/2} - u_i,
// dL = u_i - u^+_{i-1/2} and h times the modified derivative, with the
// arithmetic of hweno_point (there sv = S/4, dv = D/4). The smoothness
// indicators, tau, epsilon, the weights and the combinations are evaluated
// in double; q_l = beta_l + eps is formed directly (beta_1 = e1^2, ...).
struct PointK {
  double eps, gamma0, g1, d0, d1;
  double K, hg1, A;    // 11/32 - g1/2, g1/2, 3/4 - d1
};

HWENO_HD PointK point_k(const Scheme& s) {
  PointK k;
  k.eps = s.eps;
  k.gamma0 = s.gamma0;
  k.g1 = s.g1;
  k.d0 = s.d0;
  k.d1 = s.d1;
  k.K = 0.34375 - 0.5 * s.g1;
  k.hg1 = 0.5 * s.g1;
  k.A = 0.75 - s.d1;
  return k;
}

template <typename T>
HWENO_HD void hweno_point_diff(T e1_, T e2_, T S_, T D_, const PointK& k, T& dR, T& dL, T& vt) {
  constexpr double r13 = 2.0816659994661326;    // sqrt(13/3)
  constexpr double r781 = 6.248999919987197;    // sqrt(781/20)
  constexpr double r1421 = 24.99636017459386;   // sqrt(1421461/2275)
  const double e1 = (double)e1_, e2 = (double)e2_, S = (double)S_, D = (double)D_;
  const double cdf = e1 + e2, sdf = e2 - e1;
  // (GHYZ) closed form with the weights' square roots folded in
  const double t1 = fma(0.6875, cdf, -0.1875 * S);
  const double t2 = fma(r13 * 197.0 / 260.0, sdf, (r13 * 67.0 / 520.0) * D);
  const double a3 = fma(-0.25 * r781, cdf, (0.25 * r781) * S);
  const double a4 = fma(-0.5 * r1421, sdf, (-0.25 * r1421) * D);
  const double q0 = fma(t1, t1, fma(t2, t2, fma(a3, a3, fma(a4, a4, k.eps))));
  const double q1 = fma(e1, e1, k.eps), q2 = fma(e2, e2, k.eps);
  // (nonlinear), scaled by q0 q1 q2: o_l = P + tau P / q_l
  const double ts = fabs(q0 - q1) + fabs(q0 - q2);
  const double tau = (0.25 * ts) * ts;
  const double A = q1 * q2, B = q0 * q2, C = q0 * q1;
  const double P = A * q0;
  const double o0 = fma(A, tau, P), o1 = fma(B, tau, P), o2 = fma(C, tau, P);
  const double o12 = o1 + o2;
  const double Sg = fma(k.gamma0, o0, k.g1 * o12);
  const double Sd = fma(k.d0, o0, k.d1 * o12);
  const double inv = rcp_nr(Sg * Sd);
  const double iSg = Sd * inv, iSd = Sg * inv;
  // (interp) and its mirror image, (limiter)
  const double X = fma(o1, e1, o2 * e2);
  const double base = fma(k.K, cdf, -0.09375 * S);
  const double m = fma(0.21875, sdf, 0.046875 * D);
  const double P1 = fma(o0, base, k.hg1 * X), P2 = o0 * m;
  dR = (T)((P1 + P2) * iSg);
  dL = (T)((P1 - P2) * iSg);
  const double AT = fma(k.A, cdf, -0.25 * S);
  vt = (T)(fma(o0, AT, k.d1 * X) * iSd);
}

// (P'xi) and its mirror through the same differences, times h (linear, so
// valid in conserved or characteristic variables):
//   h v^-_{i+1/2} = -3/16 e1 + 21/16 e2 - S/16 + D/8,
//   h v^+_{i-1/2} = 21/16 e1 - 3/16 e2 - S/16 - D/8.
template <typename T>
HWENO_HD void face_derivs_diff(T e1, T e2, T S, T D, T& vR, T& vL) {
  const T s = T(-0.0625) * S;
  vR = fma(T(-0.1875), e1, fma(T(1.3125), e2, fma(T(0.125), D, s)));
  vL = fma(T(1.3125), e1, fma(T(-0.1875), e2, fma(T(-0.125), D, s)));
}

// (P'xi) and its mirror: v^-_{i+1/2} = p0'(x_{i+1/2}), v^+_{i-1/2} = p0'(x_{i-1/2}).
// Linear in the data, hence the same in conserved or characteristic variables.
template <typename T>
HWENO_HD void face_derivs(T um, T u0, T up, T vm, T vp, T ih, T& vR, T& vL) {
  vR = (T(0.1875) * um - T(1.5) * u0 + T(1.3125) * up) * ih + T(0.0625) * vm - T(0.1875) * vp;
  vL = (T(-1.3125) * um + T(1.5) * u0 - T(0.1875) * up) * ih - T(0.1875) * vm + T(0.0625) * vp;
}

// (Cd-1)-(DfDh), with the coefficients of each combination collected:
//   D(f) = -97/1920 (f_{i-1} - f_i - f_{i+1} + f_{i+2}) - 19/960 dx (h_{i-1} - h_{i+2})
//   D(h) = [697/5184 (f_{i-1} - f_{i+2}) - 61/192 (f_i - f_{i+1})] / dx
//          + 37/864 (h_{i-1} + h_{i+2})
template <typename T>
HWENO_HD void central_corr(T fm1, T f0, T fp1, T fp2, T hm1, T hp2, T h, T ih,
                                             T& Df, T& Dh) {
  const T s4 = (fm1 + fp2) - (f0 + fp1);
  Df = T(-97.0 / 1920.0) * s4 - T(19.0 / 960.0) * h * (hm1 - hp2);
  Dh = (T(697.0 / 5184.0) * (fm1 - fp2) - T(61.0 / 192.0) * (f0 - fp1)) * ih +
       T(37.0 / 864.0) * (hm1 + hp2);
}

// (mixed): interface value of a mixed-derivative flux.
template <typename T>
HWENO_HD T mixed_face(T em1, T e0, T ep1, T ep2) {
  return (T(7.0) * (e0 + ep1) - (em1 + ep2)) * T(1.0 / 12.0);
}

// ---------------------------------------------------------------- systems
// Each system provides, for direction D (0 = x, 1 = y):
//   prim(U)                      per-point quantities shared by the rest
//   flux<D>(U, pr, F)            f or g
//   jac<D>(U, pr, V, out)        f'(U) V (the fluxes h, eta, xi, theta)
//   eig<D>(U, pr) / left / right characteristic basis (systems only)
//   speed<D>(U)                  spectral radius for the LF alpha
//   admissible(U)                finite, and rho > 0, p > 0 for Euler
struct Advection {
  static constexpr int NC = 1;
  static constexpr bool kChar = false;
  double a, b;
  template <typename T> struct Prim {};
  template <typename T>
  HWENO_HD Prim<T> prim(const T (&)[NC]) const { return {}; }
  template <typename T> struct CellEig { Prim<T> q; };
  template <typename T>
  HWENO_HD CellEig<T> cell_eig(const T (&)[NC]) const { return {}; }
  template <int D, typename T>
  HWENO_HD void flux(const T (&U)[NC], const Prim<T>&, T (&F)[NC]) const {
    F[0] = T(D == 0 ? a : b) * U[0];
  }
  template <int D, typename T>
  HWENO_HD void jac(const T (&)[NC], const Prim<T>&, const T (&V)[NC],
                                      T (&O)[NC]) const {
    O[0] = T(D == 0 ? a : b) * V[0];
  }
  template <int D, typename T>
  HWENO_HD double speed(const T (&)[NC]) const { return fabs(D == 0 ? a : b); }
  template <typename T>
  HWENO_HD unsigned admissible(const T (&U)[NC]) const {
    return isfinite((double)U[0]) ? 0u : 1u;
  }
  // spectral radii in x and y, and the admissibility flags, in one pass
  template <typename T>
  HWENO_HD unsigned speeds(const T (&U)[NC], double& sx, double& sy) const {
    sx = fabs(a);
    sy = fabs(b);
    return admissible(U);
  }
};

struct Burgers {
  static constexpr int NC = 1;
  static constexpr bool kChar = false;
  template <typename T> struct Prim {};
  template <typename T>
  HWENO_HD Prim<T> prim(const T (&)[NC]) const { return {}; }
  template <typename T> struct CellEig { Prim<T> q; };
  template <typename T>
  HWENO_HD CellEig<T> cell_eig(const T (&)[NC]) const { return {}; }
  template <int D, typename T>
  HWENO_HD void flux(const T (&U)[NC], const Prim<T>&, T (&F)[NC]) const {
    F[0] = T(0.5) * U[0] * U[0];
  }
  template <int D, typename T>
  HWENO_HD void jac(const T (&U)[NC], const Prim<T>&, const T (&V)[NC],
                                      T (&O)[NC]) const {
    O[0] = U[0] * V[0];
  }
  template <int D, typename T>
  HWENO_HD double speed(const T (&U)[NC]) const { return fabs((double)U[0]); }
  template <typename T>
  HWENO_HD unsigned admissible(const T (&U)[NC]) const {
    return isfinite((double)U[0]) ? 0u : 1u;
  }
  template <typename T>
  HWENO_HD unsigned speeds(const T (&U)[NC], double& sx, double& sy) const {
    sx = sy = fabs((double)U[0]);
    return admissible(U);
  }
};

// Euler equations (euler1d) / (euler2d), U = (rho, rho u[, rho v], E),
// P = (gas - 1) (E - rho |vel|^2 / 2).
template <int DIM>
struct Euler {
  static constexpr int NC = DIM + 2;
  static constexpr bool kChar = true;
  static constexpr int E_ = NC - 1;
  double gas;

  template <typename T>
  struct Prim {
    T ir, mu, nu, k, p, Ep;  // 1/rho, u, v, |vel|^2/2, P, E + P
  };
  template <typename T>
  HWENO_HD Prim<T> prim(const T (&U)[NC]) const {
    Prim<T> q;
    q.ir = rcp_nr(U[0]);
    q.mu = U[1] * q.ir;
    q.nu = DIM == 2 ? U[2] * q.ir : T(0);
    q.k = T(0.5) * (q.mu * q.mu + q.nu * q.nu);
    q.p = T(gas - 1.0) * (U[E_] - U[0] * q.k);
    q.Ep = U[E_] + q.p;
    return q;
  }
  template <int D, typename T>
  HWENO_HD void flux(const T (&U)[NC], const Prim<T>& q, T (&F)[NC]) const {
    if constexpr (DIM == 1) {
      F[0] = U[1];
      F[1] = U[1] * q.mu + q.p;
      F[2] = q.mu * q.Ep;
    } else if constexpr (D == 0) {
      F[0] = U[1];
      F[1] = U[1] * q.mu + q.p;
      F[2] = U[1] * q.nu;
      F[3] = q.mu * q.Ep;
    } else {
      F[0] = U[2];
      F[1] = U[2] * q.mu;
      F[2] = U[2] * q.nu + q.p;
      F[3] = q.nu * q.Ep;
    }
  }
  // A(U) V by the chain rule through the primitives: with d(.) the derivative
  // along V, du = (V1 - u V0)/rho, dv = (V2 - v V0)/rho and
  // dP = (gas-1)(V_E - u V1 - v V2 + k V0).
  template <int D, typename T>
  HWENO_HD void jac(const T (&U)[NC], const Prim<T>& q, const T (&V)[NC],
                                      T (&O)[NC]) const {
    const T gm1 = T(gas - 1.0);
    if constexpr (DIM == 1) {
      const T du = (V[1] - q.mu * V[0]) * q.ir;
      const T dP = gm1 * (V[2] - q.mu * V[1] + q.k * V[0]);
      O[0] = V[1];
      O[1] = q.mu * V[1] + U[1] * du + dP;
      O[2] = du * q.Ep + q.mu * (V[2] + dP);
    } else {
      const T du = (V[1] - q.mu * V[0]) * q.ir;
      const T dv = (V[2] - q.nu * V[0]) * q.ir;
      const T dP = gm1 * (V[3] - q.mu * V[1] - q.nu * V[2] + q.k * V[0]);
      if constexpr (D == 0) {
        O[0] = V[1];
        O[1] = q.mu * V[1] + U[1] * du + dP;
        O[2] = q.nu * V[1] + U[1] * dv;
        O[3] = du * q.Ep + q.mu * (V[3] + dP);
      } else {
        O[0] = V[2];
        O[1] = q.mu * V[2] + U[2] * du;
        O[2] = q.nu * V[2] + U[2] * dv + dP;
        O[3] = dv * q.Ep + q.nu * (V[3] + dP);
      }
    }
  }

  // Characteristic basis of A_D(U) at a cell centre: rows of L and columns
  // of R for the eigenvalues (vel-c, vel, [vel,] vel+c); R in the textbook
  // normalisation and L = R^{-1} in closed form (b1 = (gas-1)/c^2,
  // b2 = b1 k, H = (E+P)/rho).
  template <typename T>
  struct Eig {
    T mu, nu, k, c, ic, H, b1, b2;
  };
  template <typename T>
  HWENO_HD Eig<T> eig(const Prim<T>& q) const {
    Eig<T> e;
    e.mu = q.mu;
    e.nu = q.nu;
    e.k = q.k;
    const T c2 = T(gas) * q.p * q.ir;
    e.ic = rsqrt_nr(c2);
    e.c = c2 * e.ic;
    e.H = q.Ep * q.ir;
    e.b1 = T(gas - 1.0) * e.ic * e.ic;
    e.b2 = e.b1 * q.k;
    return e;
  }
  // The same basis for Roe's matrix of the states UL, UR (the interface basis
  // of Jiang and Shu's characteristic decomposition): velocities and total
  // enthalpy averaged with weights sqrt(rho), c^2 = (gas-1)(H - |vel|^2/2).
  // With r = 1/sqrt(rho): sqrt(rho) u = m r and sqrt(rho) H = (E + P) r.
  template <typename T>
  HWENO_HD Eig<T> roe_eig(const T (&UL)[NC], const T (&UR)[NC]) const {
    const T gm1 = T(gas - 1.0);
    const T rl = rsqrt_nr(UL[0]), rr = rsqrt_nr(UR[0]);
    const T a = rcp_nr(UL[0] * rl + UR[0] * rr);
    const T ml = UL[1] * rl, mr = UR[1] * rr;                     // sqrt(rho) u
    const T nl = DIM == 2 ? UL[2] * rl : T(0), nr = DIM == 2 ? UR[2] * rr : T(0);
    const T pl = gm1 * (UL[E_] - T(0.5) * (ml * ml + nl * nl));
    const T pr = gm1 * (UR[E_] - T(0.5) * (mr * mr + nr * nr));
    Eig<T> e;
    e.mu = (ml + mr) * a;
    e.nu = (nl + nr) * a;
    e.H = ((UL[E_] + pl) * rl + (UR[E_] + pr) * rr) * a;
    e.k = T(0.5) * (e.mu * e.mu + e.nu * e.nu);
    const T c2 = gm1 * (e.H - e.k);
    e.ic = rsqrt_nr(c2);
    e.c = c2 * e.ic;
    e.b1 = gm1 * e.ic * e.ic;
    e.b2 = e.b1 * e.k;
    return e;
  }

  template <int D, typename T>
  HWENO_HD void left(const Eig<T>& e, int j, T (&l)[NC]) const {
    const T vn = D == 0 ? e.mu : e.nu;    // normal velocity
    if constexpr (DIM == 1) {
      if (j == 0) { l[0] = T(0.5) * (e.b2 + e.mu * e.ic); l[1] = T(-0.5) * (e.b1 * e.mu + e.ic); l[2] = T(0.5) * e.b1; }
      else if (j == 1) { l[0] = T(1) - e.b2; l[1] = e.b1 * e.mu; l[2] = -e.b1; }
      else { l[0] = T(0.5) * (e.b2 - e.mu * e.ic); l[1] = T(0.5) * (e.ic - e.b1 * e.mu); l[2] = T(0.5) * e.b1; }
    } else {
      if (j == 0) {
        l[0] = T(0.5) * (e.b2 + vn * e.ic);
        l[1] = T(-0.5) * (e.b1 * e.mu + (D == 0 ? e.ic : T(0)));
        l[2] = T(-0.5) * (e.b1 * e.nu + (D == 1 ? e.ic : T(0)));
        l[3] = T(0.5) * e.b1;
      } else if (j == 1) {
        l[0] = T(1) - e.b2; l[1] = e.b1 * e.mu; l[2] = e.b1 * e.nu; l[3] = -e.b1;
      } else if (j == 2) {
        if (D == 0) { l[0] = -e.nu; l[1] = T(0); l[2] = T(1); l[3] = T(0); }
        else { l[0] = -e.mu; l[1] = T(1); l[2] = T(0); l[3] = T(0); }
      } else {
        l[0] = T(0.5) * (e.b2 - vn * e.ic);
        l[1] = T(0.5) * ((D == 0 ? e.ic : T(0)) - e.b1 * e.mu);
        l[2] = T(0.5) * ((D == 1 ? e.ic : T(0)) - e.b1 * e.nu);
        l[3] = T(0.5) * e.b1;
      }
    }
  }
  template <int D, typename T>
  HWENO_HD void right(const Eig<T>& e, int j, T (&r)[NC]) const {
    const T vn = D == 0 ? e.mu : e.nu;
    if constexpr (DIM == 1) {
      if (j == 0) { r[0] = T(1); r[1] = e.mu - e.c; r[2] = e.H - e.mu * e.c; }
      else if (j == 1) { r[0] = T(1); r[1] = e.mu; r[2] = e.k; }
      else { r[0] = T(1); r[1] = e.mu + e.c; r[2] = e.H + e.mu * e.c; }
    } else {
      if (j == 0 || j == 3) {
        const T sc = j == 0 ? -e.c : e.c;
        r[0] = T(1);
        r[1] = e.mu + (D == 0 ? sc : T(0));
        r[2] = e.nu + (D == 1 ? sc : T(0));
        r[3] = e.H + vn * sc;
      } else if (j == 1) {
        r[0] = T(1); r[1] = e.mu; r[2] = e.nu; r[3] = e.k;
      } else {
        if (D == 0) { r[0] = T(0); r[1] = T(0); r[2] = T(1); r[3] = e.nu; }
        else { r[0] = T(0); r[1] = T(1); r[2] = T(0); r[3] = e.mu; }
      }
    }
  }
  // w = L U and U = R c for the basis above, with the shared terms of the
  // rows (columns) collected: for x in 2D, with s = b2 U0 - b1 (u U1 + v U2
  // - UE) and t = (u U0 - U1)/c, L U = ((s+t)/2, U0 - s, U2 - v U0, (s-t)/2).
  template <int D, typename T>
  HWENO_HD void project(const Eig<T>& e, const T (&U)[NC], T (&w)[NC]) const {
    if constexpr (DIM == 1) {
      const T s = e.b2 * U[0] - e.b1 * (e.mu * U[1] - U[2]);
      const T t = e.ic * (e.mu * U[0] - U[1]);
      w[0] = T(0.5) * (s + t);
      w[1] = U[0] - s;
      w[2] = T(0.5) * (s - t);
    } else {
      const T s = e.b2 * U[0] - e.b1 * (e.mu * U[1] + e.nu * U[2] - U[3]);
      const T t = D == 0 ? e.ic * (e.mu * U[0] - U[1]) : e.ic * (e.nu * U[0] - U[2]);
      w[0] = T(0.5) * (s + t);
      w[1] = U[0] - s;
      w[2] = D == 0 ? U[2] - e.nu * U[0] : U[1] - e.mu * U[0];
      w[3] = T(0.5) * (s - t);
    }
  }
  template <int D, typename T>
  HWENO_HD void unproject(const Eig<T>& e, const T (&c)[NC], T (&U)[NC]) const {
    if constexpr (DIM == 1) {
      const T a = c[0] + c[2], dd = c[2] - c[0];
      const T s0 = a + c[1];
      U[0] = s0;
      U[1] = e.mu * s0 + e.c * dd;
      U[2] = e.H * a + (e.mu * e.c) * dd + e.k * c[1];
    } else {
      const T a = c[0] + c[3], dd = c[3] - c[0];
      const T s0 = a + c[1];
      const T vn = D == 0 ? e.mu : e.nu, vt = D == 0 ? e.nu : e.mu;
      U[0] = s0;
      if (D == 0) {
        U[1] = e.mu * s0 + e.c * dd;
        U[2] = e.nu * s0 + c[2];
      } else {
        U[1] = e.mu * s0 + c[2];
        U[2] = e.nu * s0 + e.c * dd;
      }
      U[3] = e.H * a + (vn * e.c) * dd + e.k * c[1] + vt * c[2];
    }
  }
  // The cell basis of both directions for the difference form of the HWENO
  // (hweno_cell_diff): the primitives, c, H, and the coefficients with the
  // halves of the closed-form L folded in (b1/2, b2/2, 1/(2c)); u c, v c for
  // the back-projection.
  template <typename T>
  struct CellEig {
    Prim<T> q;
    T c, H, b1h, b2h, ich, muc, nuc;
  };
  template <typename T>
  HWENO_HD CellEig<T> cell_eig(const T (&U)[NC]) const {
    CellEig<T> e;
    e.q = prim(U);
    const T c2 = T(gas) * e.q.p * e.q.ir;
    const T ic = rsqrt_nr(c2);
    e.c = c2 * ic;
    e.H = e.q.Ep * e.q.ir;
    e.b1h = (T(0.5 * (gas - 1.0)) * ic) * ic;
    e.b2h = e.b1h * e.q.k;
    e.ich = T(0.5) * ic;
    e.muc = e.q.mu * e.c;
    e.nuc = e.q.nu * e.c;
    return e;
  }
  // w = L x (the same L as project): with s' = s/2 and t' = t/2,
  // w = (s' + t', x0 - 2 s', x2 - v x0 | x1 - u x0, s' - t').
  template <int D, typename T>
  HWENO_HD void project_half(const CellEig<T>& e, const T (&x)[NC], T (&w)[NC]) const {
    if constexpr (DIM == 1) {
      const T sh = fma(e.b2h, x[0], -e.b1h * fma(e.q.mu, x[1], -x[2]));
      const T th = e.ich * fma(e.q.mu, x[0], -x[1]);
      w[0] = sh + th;
      w[1] = fma(T(-2), sh, x[0]);
      w[2] = sh - th;
    } else {
      const T in = fma(e.q.mu, x[1], fma(e.q.nu, x[2], -x[3]));
      const T sh = fma(e.b2h, x[0], -e.b1h * in);
      const T th = D == 0 ? e.ich * fma(e.q.mu, x[0], -x[1]) : e.ich * fma(e.q.nu, x[0], -x[2]);
      w[0] = sh + th;
      w[1] = fma(T(-2), sh, x[0]);
      w[2] = D == 0 ? fma(-e.q.nu, x[0], x[2]) : fma(-e.q.mu, x[0], x[1]);
      w[3] = sh - th;
    }
  }
  // out = base + R c (NEG: base - R c); base null: R c.
  template <int D, bool NEG, typename T>
  HWENO_HD void unproject_add(const CellEig<T>& e, const T (&c)[NC], const T* base,
                              T (&out)[NC]) const {
    const T sg = NEG ? T(-1) : T(1);
    auto b = [&](int j) { return base ? base[j] : T(0); };
    if constexpr (DIM == 1) {
      const T a = c[0] + c[2], dd = c[2] - c[0];
      const T s0 = a + c[1];
      out[0] = fma(sg, s0, b(0));
      out[1] = fma(sg * e.q.mu, s0, fma(sg * e.c, dd, b(1)));
      out[2] = fma(sg * e.H, a, fma(sg * e.muc, dd, fma(sg * e.q.k, c[1], b(2))));
    } else {
      const T a = c[0] + c[3], dd = c[3] - c[0];
      const T s0 = a + c[1];
      out[0] = fma(sg, s0, b(0));
      if (D == 0) {
        out[1] = fma(sg * e.q.mu, s0, fma(sg * e.c, dd, b(1)));
        out[2] = fma(sg * e.q.nu, s0, fma(sg, c[2], b(2)));
        out[3] = fma(sg * e.H, a, fma(sg * e.muc, dd, fma(sg * e.q.k, c[1], fma(sg * e.q.nu, c[2], b(3)))));
      } else {
        out[1] = fma(sg * e.q.mu, s0, fma(sg, c[2], b(1)));
        out[2] = fma(sg * e.q.nu, s0, fma(sg * e.c, dd, b(2)));
        out[3] = fma(sg * e.H, a, fma(sg * e.nuc, dd, fma(sg * e.q.k, c[1], fma(sg * e.q.mu, c[2], b(3)))));
      }
    }
  }
  template <int D, typename T>
  HWENO_HD double speed(const T (&U)[NC]) const {
    const double r = (double)U[0];
    const double mu = (double)U[1] / r;
    const double nu = DIM == 2 ? (double)U[2] / r : 0.0;
    const double p = (gas - 1.0) * ((double)U[E_] - 0.5 * r * (mu * mu + nu * nu));
    return fabs(D == 0 ? mu : nu) + sqrt(gas * p / r);
  }
  // |u| + c and |v| + c with the admissibility flags, in one pass (Newton-
  // refined reciprocal and inverse square root).
  template <typename T>
  HWENO_HD unsigned speeds(const T (&U)[NC], double& sx, double& sy) const {
    const double r = (double)U[0];
    const double ir = rcp_nr(r);
    const double mu = (double)U[1] * ir;
    const double nu = DIM == 2 ? (double)U[2] * ir : 0.0;
    const double p = (gas - 1.0) * ((double)U[E_] - 0.5 * r * (mu * mu + nu * nu));
    const double c2 = gas * p * ir;
    const double c = c2 * rsqrt_nr(c2);
    sx = fabs(mu) + c;
    sy = fabs(nu) + c;
    unsigned f = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) f |= isfinite((double)U[k]) ? 0u : 1u;
    if (!(r > 0.0) || !(p > 0.0)) f |= 2u;
    return f;
  }
  template <typename T>
  HWENO_HD unsigned admissible(const T (&U)[NC]) const {
    unsigned f = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) f |= isfinite((double)U[c]) ? 0u : 1u;
    const double r = (double)U[0];
    const double mu = (double)U[1] / r;
    const double nu = DIM == 2 ? (double)U[2] / r : 0.0;
    const double p = (gas - 1.0) * ((double)U[E_] - 0.5 * r * (mu * mu + nu * nu));
    if (!(r > 0.0) || !(p > 0.0)) f |= 2u;
    return f;
  }
};

// HWENO-I on one cell for a system, in direction D: project the stencil on
// the characteristic basis of the cell centre, apply hweno_point to every
// characteristic variable, project back (remarks on local characteristic
// decomposition in sections 2 and 3). Scalar laws skip the projection.
template <int D, class Sys, typename T>
HWENO_HD void hweno_cell_q(const Sys& sy, const Scheme& s, double h, double ih,
                           const typename Sys::template Prim<T>& q,
                                           const T (&Um)[Sys::NC], const T (&U0)[Sys::NC],
                                           const T (&Up)[Sys::NC], const T (&Am)[Sys::NC],
                                           const T (&Ap)[Sys::NC], T (&uR)[Sys::NC],
                                           T (&uL)[Sys::NC], T (&at)[Sys::NC]) {
  constexpr int NC = Sys::NC;
  if constexpr (!Sys::kChar) {
    hweno_point<T>(Um[0], U0[0], Up[0], Am[0], Ap[0], s, h, ih, uR[0], uL[0], at[0]);
  } else {
    const auto e = sy.eig(q);
    T wm[NC], w0[NC], wp[NC], am[NC], ap[NC];
    sy.template project<D>(e, Um, wm);
    sy.template project<D>(e, U0, w0);
    sy.template project<D>(e, Up, wp);
    sy.template project<D>(e, Am, am);
    sy.template project<D>(e, Ap, ap);
    T cr[NC], cl[NC], ct[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j)
      hweno_point<T>(wm[j], w0[j], wp[j], am[j], ap[j], s, h, ih, cr[j], cl[j], ct[j]);
    sy.template unproject<D>(e, cr, uR);
    sy.template unproject<D>(e, cl, uL);
    sy.template unproject<D>(e, ct, at);
  }
}

// The interface-basis switch (Jiang and Shu's decomposition): the right-face
// value in the basis of Roe's matrix of (U0, Up), the left-face value in that
// of (Um, U0), the modified derivative in the cell basis. Three projections
// and three HWENO applications per cell instead of one (the smoothness
// indicators differ per basis); each keeps only the output it is used for.
template <int D, class Sys, typename T>
HWENO_HD void hweno_cell_iface(const Sys& sy, const Scheme& s, double h, double ih,
                               const typename Sys::template Prim<T>& q,
                               const T (&Um)[Sys::NC], const T (&U0)[Sys::NC],
                               const T (&Up)[Sys::NC], const T (&Am)[Sys::NC],
                               const T (&Ap)[Sys::NC], T (&uR)[Sys::NC], T (&uL)[Sys::NC],
                               T (&at)[Sys::NC]) {
  constexpr int NC = Sys::NC;
  if constexpr (!Sys::kChar) {
    hweno_point<T>(Um[0], U0[0], Up[0], Am[0], Ap[0], s, h, ih, uR[0], uL[0], at[0]);
  } else {
    auto apply = [&](const auto& e, int which, T (&out)[NC]) {
      T wm[NC], w0[NC], wp[NC], am[NC], ap[NC], c[NC];
      sy.template project<D>(e, Um, wm);
      sy.template project<D>(e, U0, w0);
      sy.template project<D>(e, Up, wp);
      sy.template project<D>(e, Am, am);
      sy.template project<D>(e, Ap, ap);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        T r_, l_, t_;
        hweno_point<T>(wm[j], w0[j], wp[j], am[j], ap[j], s, h, ih, r_, l_, t_);
        c[j] = which == 0 ? r_ : (which == 1 ? l_ : t_);
      }
      sy.template unproject<D>(e, c, out);
    };
    apply(sy.roe_eig(U0, Up), 0, uR);
    apply(sy.roe_eig(Um, U0), 1, uL);
    apply(sy.eig(q), 2, at);
  }
}

// Either basis, by template flag.
template <int D, bool IFACE, class Sys, typename T>
HWENO_HD void hweno_cell_b(const Sys& sy, const Scheme& s, double h, double ih,
                           const typename Sys::template Prim<T>& q, const T (&Um)[Sys::NC],
                           const T (&U0)[Sys::NC], const T (&Up)[Sys::NC], const T (&Am)[Sys::NC],
                           const T (&Ap)[Sys::NC], T (&uR)[Sys::NC], T (&uL)[Sys::NC],
                           T (&at)[Sys::NC]) {
  if constexpr (IFACE)
    hweno_cell_iface<D>(sy, s, h, ih, q, Um, U0, Up, Am, Ap, uR, uL, at);
  else
    hweno_cell_q<D>(sy, s, h, ih, q, Um, U0, Up, Am, Ap, uR, uL, at);
}

// The same, computing the centre's primitive quantities itself.
template <int D, class Sys, typename T>
HWENO_HD void hweno_cell(const Sys& sy, const Scheme& s, double h, double ih,
                         const T (&Um)[Sys::NC], const T (&U0)[Sys::NC], const T (&Up)[Sys::NC],
                         const T (&Am)[Sys::NC], const T (&Ap)[Sys::NC], T (&uR)[Sys::NC],
                         T (&uL)[Sys::NC], T (&at)[Sys::NC]) {
  hweno_cell_q<D>(sy, s, h, ih, sy.prim(U0), Um, U0, Up, Am, Ap, uR, uL, at);
}

// HWENO-I on one cell in direction D, difference form (forward kernels): from
// the conserved-variable differences E1 = U_i - U_{i-1}, E2 = U_{i+1} - U_i
// and the sums S = A'_{i-1} + A'_{i+1}, Dd = A'_{i-1} - A'_{i+1} of the
// derivative along D times the mesh width (A' = h A), it returns u at both
// faces, h times the modified derivative and h times the face derivatives of
// (P'xi). Systems project the four differences on the cell's characteristic
// basis (remarks on the local characteristic decomposition in sections 2 and
// 3), interpolate every characteristic variable and project the corrections
// back onto U_i; the face derivatives are linear and taken component-wise.
template <int D, class Sys, typename T>
HWENO_HD void hweno_cell_diff(const Sys& sy, const PointK& k,
                              const typename Sys::template CellEig<T>& ce,
                              const T (&U0)[Sys::NC], const T (&E1)[Sys::NC],
                              const T (&E2)[Sys::NC], const T (&S)[Sys::NC],
                              const T (&Dd)[Sys::NC], T (&uR)[Sys::NC], T (&uL)[Sys::NC],
                              T (&at)[Sys::NC], T (&vR)[Sys::NC], T (&vL)[Sys::NC]) {
  constexpr int NC = Sys::NC;
#pragma unroll
  for (int c = 0; c < NC; ++c) face_derivs_diff(E1[c], E2[c], S[c], Dd[c], vR[c], vL[c]);
  if constexpr (!Sys::kChar) {
    T dR, dL;
    hweno_point_diff<T>(E1[0], E2[0], S[0], Dd[0], k, dR, dL, at[0]);
    uR[0] = U0[0] + dR;
    uL[0] = U0[0] - dL;
  } else {
    T e1[NC], e2[NC], sc[NC], dc[NC];
    sy.template project_half<D>(ce, E1, e1);
    sy.template project_half<D>(ce, E2, e2);
    sy.template project_half<D>(ce, S, sc);
    sy.template project_half<D>(ce, Dd, dc);
    T cr[NC], cl[NC], ct[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j)
      hweno_point_diff<T>(e1[j], e2[j], sc[j], dc[j], k, cr[j], cl[j], ct[j]);
    sy.template unproject_add<D, false>(ce, cr, U0, uR);
    sy.template unproject_add<D, true>(ce, cl, U0, uL);
    sy.template unproject_add<D, false>(ce, ct, (const T*)nullptr, at);
  }
}

// ------------------------------------------------------------- index maps
// Boundary codes, as in the C ABI.
constexpr int kBcPeriodic = 0, kBcTransmissive = 1, kBcReflective = 2, kBcDirichlet = 3,
              kBcSplit = 4;

// Ghost cells by index map: periodic wraps, transmissive clamps (copies the
// nearest interior cell), reflective mirrors (ghost -1-k is the image of
// cell k, ghost n+k of cell n-1-k). Any integer i is accepted and the result
// is always in [0, n): lanes further out than the mirror reaches (only the
// two ghosts next to a wall enter the scheme) are clamped to an edge cell.
// Fixed-state (Dirichlet) and split-side ghosts are clamped too; the kernels
// replace or re-map them.
HWENO_HD int map_index(int i, int n, int lo, int hi) {
  if (i >= 0 && i < n) return i;
  const int side = i < 0 ? lo : hi;
  if (side == kBcPeriodic) {
    int m = i % n;
    return m < 0 ? m + n : m;
  }
  if (side == kBcReflective) {
    const int m = i < 0 ? -1 - i : 2 * n - 1 - i;
    return m < 0 ? 0 : (m > n - 1 ? n - 1 : m);
  }
  return i < 0 ? 0 : n - 1;
}

// The side (0 low, 1 high) whose fixed state a ghost cell holds, or -1.
HWENO_HD int fixed_side(int i, int n, int lo, int hi) {
  if (i < 0 && lo == kBcDirichlet) return 0;
  if (i >= n && hi == kBcDirichlet) return 1;
  return -1;
}

// True for a ghost cell behind a reflective wall.
HWENO_HD bool mirrored(int i, int n, int lo, int hi) {
  return (i < 0 && lo == kBcReflective) || (i >= n && hi == kBcReflective);
}

// Sign rules of a reflective wall normal to direction D (remarks on boundary
// conditions in sections 2 and 3, (RBC-1d), (RBC-2d-x), (RBC-2d-y)): the
// ghost state is the mirror image with the normal momentum (component 1 + D)
// negated; a derivative along the wall normal changes the sign of every other
// component, a derivative along the wall behaves like the state. Only the
// Euler systems have reflective walls.
template <class Sys, int D, typename T>
HWENO_HD void mirror_state(bool on, T (&U)[Sys::NC]) {
  if constexpr (Sys::kChar) {
    if (on) U[1 + D] = -U[1 + D];
  }
}
template <class Sys, int D, typename T>
HWENO_HD void mirror_normal_derivative(bool on, T (&A)[Sys::NC]) {
  if constexpr (Sys::kChar) {
    if (on) {
#pragma unroll
      for (int c = 0; c < Sys::NC; ++c)
        if (c != 1 + D) A[c] = -A[c];
    }
  }
}
// Whether component c of field f is negated at a wall normal to D, for the
// field order (u, derivative along x, derivative along y).
HWENO_HD bool mirror_flips(int D, int f, int c) {
  const bool normal = f == 1 + D;
  return normal ? c != 1 + D : c == 1 + D;
}

}  // namespace hweno
