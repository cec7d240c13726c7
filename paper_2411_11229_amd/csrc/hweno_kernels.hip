// HIP kernels and C ABI of the HWENO-I hot path for gfx950.
//
// Forward stage kernel ("marcher"): one wavefront per block. The 64 lanes
// hold 64 consecutive cells of a row (60 output columns plus a 2-cell halo
// on each side); x-neighbours are read across lanes. The wavefront marches
// up a strip of rows, keeping in registers (and, for the pointwise y-fluxes
// and pending updates, in LDS) what the y-stencil still needs, in a tile
// order that keeps neighbouring tiles behind one XCD's L2, so every cell's
// HWENO interpolation is done once per direction and
// every input value is read from memory once per strip (plus halos).
// Per output cell and stage it does: the x-sweep (HWENO, pointwise fluxes,
// central correction, LF flux, mixed flux, flux difference), the y-sweep
// likewise, the residual (odeH)/(ode2H) and the SSP-RK3 combination
// (fully-hweno)/(2Dfully-hweno), and the max wave speed of the new state for
// the next stage's Lax-Friedrichs alpha (after stage 3: the next step's).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <atomic>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "../../include/hweno.h"
#include "hweno_adjoint.h"
#include "hweno_device.h"

namespace hweno {

enum Mode { kRhs = 0, kStage1 = 1, kStage2 = 2, kStage3 = 3 };

// A split y side (see hweno_split): ghost (x, y) follows kind[0] where
// x < x0 + slope y + speed t, else kind[1].
struct SplitRule {
  double x0, slope, speed;
  int kind[2];
  double state[2][4];
};

// Workspace scalars of a time step. The alpha accumulators hold the
// non-negative doubles' bit patterns (atomic max): acc[0..1] the stage-2
// alphas (written by stage 1), acc[2..3] the stage-3 alphas (by stage 2),
// acc[4..5] the next stage-1 alphas, i.e. those of the step's result (by
// stage 3, or by the seeding pass before a run's first step).
struct StepScalars {
  unsigned long long acc[6];
  double dt;
  double t0;                      // the step's start time
  double tnew;                    // its end time (t0 + dt, or t_end when clipped)
  int active;
  unsigned flags;
};

// Time-step control of a stage-1 launch that computes dt itself (flux-LF): from
// its alphas by `rule` (production cfl / (ax/hx + ay/hy) with hx, hy = dx, dy;
// accuracy the same with dx^(5/3), dy^(5/3); fixed dt_fixed), clipped so that
// t + dt does not pass t_end. sc null: dt is given (frozen steps, adjoint).
struct StepCtl {
  StepScalars* sc;
  double* t;                      // the caller's time (read by stage 1, advanced by stage 2)
  double* dt_used;                // or null
  int rule, dim;
  double cfl, dt_fixed, t_end, hx, hy;
};

template <typename T>
struct StageArgs {
  const T* U;  const T* V;  const T* W;   // stage state X (W null in 1D)
  const T* Ub; const T* Vb; const T* Wb;  // RK base B^n = (U^n, V~^n, W~^n), stages 2-3
  T* Uo; T* Vo; T* Wo;                    // new state (stages) or L^1..L^3 (rhs)
  T* Vt; T* Wt;                           // stage 1: V~^n, W~^n; rhs: modified derivatives
  const double* alpha;                    // [2] LF alphas of this stage
  const double* dt;                       // stages 2-3, frozen steps: time step
  const int* active;                      // stages 2-3: 0 = the step is skipped
  unsigned long long* alpha_next;         // [2] atomic max of the new state's speeds, or null
  unsigned* flags;                        // sticky state flags, or null
  double* alpha_rec;                      // [2] record of the alphas used, or null
  int nx, ny, rows;                       // rows: output rows per block (2D)
  int plane;                              // nx * ny
  int bc[4];
  int iface;                              // host side: interface characteristic basis
  double gs[4][4];                        // fixed (Dirichlet) ghost states per side
  double gravity;                         // g of the (euler2d-s) source
  SplitRule sp[2];                        // split y sides (low, high)
  const double* t0;                       // step start time (device), null: t = 0
  double tc;                              // this stage's time: t0 + tc dt
  StepCtl ctl;                            // stage 1 computing dt, stages 2-3 of such a step
  Scheme s;
  PointK pk;                              // HWENO point constants (difference form)
};

// Start of a stage launch: the stage's dt and time, and whether the step is
// active. A stage 1 with time-step control computes dt itself from its alphas
// (every block alike); its first lane also publishes dt, the step's times and
// the record of the alphas, and clears the stage-3 accumulators. Stage 2 of
// such a step advances the caller's time and clears the next-step
// accumulators (read by stage 1, written again by stage 3); stage 3 clears
// the stage-2 accumulators. Each clear comes after the last read of those
// accumulators and before their next writer, one kernel boundary apart.
template <int MODE, typename T>
__device__ __forceinline__ bool stage_begin(const StageArgs<T>& A, bool leader, double& dt,
                                            double& tstage) {
  dt = 0.0;
  tstage = 0.0;
  if (MODE == kRhs) return true;
  const StepCtl& c = A.ctl;
  if (MODE == kStage1 && c.sc) {
    const double ax = A.alpha[0], ay = c.dim == 2 ? A.alpha[1] : 0.0;
    double d = c.rule == HWENO_DT_FIXED ? c.dt_fixed
                                        : c.cfl / (c.dim == 2 ? ax / c.hx + ay / c.hy : ax / c.hx);
    const double t0 = *c.t;
    const bool active = t0 < c.t_end;
    double tn = t0 + d;
    if (!active) {
      d = 0.0;
      tn = t0;
    } else if (tn >= c.t_end) {
      d = c.t_end - t0;
      tn = c.t_end;
    }
    if (leader) {
      c.sc->dt = d;
      c.sc->t0 = t0;
      c.sc->tnew = tn;
      c.sc->active = active ? 1 : 0;
      c.sc->acc[2] = c.sc->acc[3] = 0ull;
      if (c.dt_used) *c.dt_used = d;
      if (A.alpha_rec) {
        A.alpha_rec[0] = ax;
        A.alpha_rec[1] = ay;
      }
    }
    dt = d;
    tstage = t0;
    return active;
  }
  if (A.active && *A.active == 0) return false;
  dt = *A.dt;
  tstage = A.t0 ? *A.t0 + A.tc * dt : 0.0;
  if (leader) {
    if (A.alpha_rec) {
      A.alpha_rec[0] = A.alpha[0];
      A.alpha_rec[1] = A.ctl.dim == 1 ? 0.0 : A.alpha[1];
    }
    if (c.sc && MODE == kStage2) {
      *c.t = c.sc->tnew;
      c.sc->acc[4] = c.sc->acc[5] = 0ull;
    }
    if (c.sc && MODE == kStage3) c.sc->acc[0] = c.sc->acc[1] = 0ull;
  }
  return true;
}

// ---------------------------------------------------------------- helpers
// Element idx of a state array through a 32-bit byte offset from the uniform
// base pointer: the loads and stores then take the scalar-base form (base in
// SGPRs, offset in one VGPR) instead of a 64-bit address per lane. The host
// guarantees ncomp * plane * sizeof(T) < 2^32.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, unsigned idx) {
  return *(const T*)((const char*)base + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, unsigned idx, T v) {
  *(T*)((char*)base + idx * (unsigned)sizeof(T)) = v;
}
// Asynchronous copy of kWave consecutive elements of one row (from column
// col0, columns outside [0, nx) clamped to the edge) straight from global memory into
// LDS (dst[0..kWave)), with no VGPR in between: each 4-byte load of a wave
// writes lane i's word at byte 4i of its 256-byte part. The caller orders
// it with LDS reads of dst: wait_copies() before reading the copy,
// wait_lds_reads() after the last read of dst's previous contents.
template <typename T>
__device__ __forceinline__ void row_to_lds(const T* base, unsigned row_off, int col0, int nx, T* dst,
                                           int lane) {
  constexpr int P = sizeof(T) / 4;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int col = max(0, min(col0 + j * (kWave / P) + lane / P, nx - 1));
    const unsigned byte = (row_off + (unsigned)col) * (unsigned)sizeof(T) + 4u * (unsigned)(lane % P);
    __builtin_amdgcn_global_load_lds(
        (const __attribute__((address_space(1))) void*)((const char*)base + byte),
        (__attribute__((address_space(3))) void*)((char*)dst + 256 * j), 4, 0, 0);
  }
}
// Waits that are also compiler barriers for memory accesses (the compiler's
// own wait insertion does not order every LDS read after a pending copy)
__device__ __forceinline__ void wait_copies() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lds_reads() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}
// Atomic max of non-negative doubles through their bit patterns (ordered
// like unsigned integers); order-independent, hence deterministic.
__device__ __forceinline__ void atomic_max_pos(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// ------------------------------------------------------ x-direction sweep
// (Cd-1)-(DfDh) at one interface, with the derivative fluxes carried times
// the mesh width h (h' = h f'(u) v): D(f) and h D(h).
template <typename T>
__device__ __forceinline__ void central_corr_k(T fm1, T f0, T fp1, T fp2, T hm1, T hp2, T& Df,
                                               T& Dh) {
  const T s4 = (fm1 + fp2) - (f0 + fp1);
  Df = fma(T(-97.0 / 1920.0), s4, T(-19.0 / 960.0) * (hm1 - hp2));
  Dh = fma(T(697.0 / 5184.0), fm1 - fp2, fma(T(-61.0 / 192.0), f0 - fp1, T(37.0 / 864.0) * (hm1 + hp2)));
}

// Steps 1-4 of section 2 along x for the row held by the wavefront (one cell
// per lane). Inputs: this lane's U, V' = dx u_x and, with NF == 3,
// W' = dy u_y (derivatives carried times their mesh width, see
// hweno_cell_diff), and the cell's characteristic basis and primitives
// `ce`. Outputs: the residual parts -(F_{i+1/2} - F_{i-1/2})/dx of the u-,
// v- and w-equations (the last from the mixed flux eta = f'(u) w),
// accumulated in double and unscaled, and dx v~. Valid on lanes 2..61.
template <int NF, bool IFACE, class Sys, typename T>
__device__ __forceinline__ void sweep_x(const Sys& sy, const Scheme& s, const PointK& pk,
                                        double alpha,
                                        const typename Sys::template CellEig<T>& ce,
                                        const T (&U)[Sys::NC], const T (&V)[Sys::NC],
                                        const T (&W)[Sys::NC], double (&RU)[Sys::NC],
                                        double (&RV)[Sys::NC], double (&RW)[Sys::NC],
                                        T (&vt)[Sys::NC]) {
  constexpr int NC = Sys::NC;
  // Step 1: HWENO once per cell -> u at both faces, v~ at the centre, and the
  // face derivatives of (P'xi)
  T uR[NC], uL[NC], vR[NC], vL[NC];
  if constexpr (IFACE) {
    T Um[NC], Up[NC], Vm[NC], Vp[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Um[c] = from_prev(U[c]);
      Up[c] = from_next(U[c]);
      Vm[c] = from_prev(V[c]);
      Vp[c] = from_next(V[c]);
    }
    // mesh width 1 for the scaled derivatives
    hweno_cell_b<0, true>(sy, s, 1.0, 1.0, ce.q, Um, U, Up, Vm, Vp, uR, uL, vt);
#pragma unroll
    for (int c = 0; c < NC; ++c) face_derivs(Um[c], U[c], Up[c], Vm[c], Vp[c], T(1), vR[c], vL[c]);
  } else {
    // the stencil as differences: E1 = U_i - U_{i-1}, E2 = U_{i+1} - U_i
    // (E1 of the next lane), S and D the sum and difference of V'_{i-1}, V'_{i+1}
    T E1[NC], E2[NC], Sv[NC], Dv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) E1[c] = U[c] - from_prev(U[c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      E2[c] = from_next(E1[c]);
      const T vm = from_prev(V[c]), vp = from_next(V[c]);
      Sv[c] = vm + vp;
      Dv[c] = vm - vp;
    }
    hweno_cell_diff<0>(sy, pk, ce, U, E1, E2, Sv, Dv, uR, uL, vt, vR, vL);
  }
  // pointwise f, h' = f'(u) v', eta' = f'(u) w' at the cell centre
  T f[NC], hf[NC], e[NC];
  sy.template flux<0>(U, ce.q, f);
  sy.template jac<0>(U, ce.q, V, hf);
  if constexpr (NF == 3) sy.template jac<0>(U, ce.q, W, e);
  // Lax-Friedrichs sums of this cell's faces (flux-LF), halved at the
  // interface: f(u^-) + a u^- at x_{i+1/2}, f(u^+) - a u^+ at x_{i-1/2}
  T mF[NC], mH[NC], pF[NC], pH[NC];
  {
    const T a = T(alpha);
    T fr[NC], hr[NC], fl[NC], hl[NC];
    const auto qr = sy.prim(uR);
    sy.template flux<0>(uR, qr, fr);
    sy.template jac<0>(uR, qr, vR, hr);
    const auto ql = sy.prim(uL);
    sy.template flux<0>(uL, ql, fl);
    sy.template jac<0>(uL, ql, vL, hl);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      mF[c] = fma(a, uR[c], fr[c]);
      mH[c] = fma(a, vR[c], hr[c]);
      pF[c] = fma(-a, uL[c], fl[c]);
      pH[c] = fma(-a, vL[c], hl[c]);
    }
  }
  // Steps 2-3 at x_{i+1/2}, then Step 4; the v-equation's fluxes carry a
  // factor dx, eta' a factor dy, removed in the flux differences
  const double cv = s.idx * s.idx, cw = s.idx * s.idy * (1.0 / 12.0);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const T fm1 = from_prev(f[c]), fp1 = from_next(f[c]), fp2 = from_next(fp1);
    const T hm1 = from_prev(hf[c]), hp1 = from_next(hf[c]), hp2 = from_next(hp1);
    T Df, Dh;
    central_corr_k(fm1, f[c], fp1, fp2, hm1, hp2, Df, Dh);
    const T Fi = fma(T(0.5), mF[c] + from_next(pF[c]), Df);
    const T Hi = fma(T(0.5), mH[c] + from_next(pH[c]), Dh);
    RU[c] = ((double)from_prev(Fi) - (double)Fi) * s.idx;
    RV[c] = ((double)from_prev(Hi) - (double)Hi) * cv;
    if constexpr (NF == 3) {
      // (mixed) times 12: 7 (e_i + e_{i+1}) - (e_{i-1} + e_{i+2})
      const T em1 = from_prev(e[c]), ep1 = from_next(e[c]), ep2 = from_next(ep1);
      const T Ei = fma(T(7), e[c] + ep1, -(em1 + ep2));
      RW[c] = ((double)from_prev(Ei) - (double)Ei) * cw;
    }
  }
}

// The Runge-Kutta combination (fully-hweno)/(2Dfully-hweno) of one value,
// written as a part known before the y-sweep's flux difference L_y and the
// weight of L_y: X_new = rk_part + rk_wl dt L_y, with
//   stage 1: X + dt L_x,  stage 2: 3/4 B + 1/4 (X + dt L_x),
//   stage 3: 1/3 B + 2/3 (X + dt L_x),  operator only (rhs): L_x.
// All in double, one rounding at the store. The stage-3 weights multiply (an
// FP64 division would cost about ten instructions per value).
template <int MODE>
__device__ __forceinline__ double rk_part(double x, double base, double dt, double Lx) {
  if constexpr (MODE == kStage1) return fma(dt, Lx, x);
  else if constexpr (MODE == kStage2) return fma(0.25 * dt, Lx, fma(0.25, x, 0.75 * base));
  else if constexpr (MODE == kStage3)
    return fma((2.0 / 3.0) * dt, Lx, fma(2.0 / 3.0, x, (1.0 / 3.0) * base));
  else return Lx;
}
template <int MODE>
__device__ __forceinline__ double rk_wl(double dt) {
  if constexpr (MODE == kStage1) return dt;
  else if constexpr (MODE == kStage2) return 0.25 * dt;
  else if constexpr (MODE == kStage3) return (2.0 / 3.0) * dt;
  else return 1.0;
}

// ------------------------------------------------------------ 1D stage kernel
template <class Sys, typename T, int MODE, bool IFACE>
__global__ __launch_bounds__(64) void stage1d_kernel(StageArgs<T> A, Sys sy) {
  constexpr int NC = Sys::NC;
  const int lane = threadIdx.x;
  double dt, tstage;
  if (!stage_begin<MODE>(A, blockIdx.x == 0 && lane == 0, dt, tstage)) return;
  const int col = blockIdx.x * kXOut - kHalo + lane;
  const int g = map_index(col, A.nx, A.bc[0], A.bc[1]);
  const bool out = lane >= kHalo && lane < kWave - kHalo && col < A.nx;
  const double ax = A.alpha[0];
  T U[NC], V[NC], W[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    U[c] = A.U[c * A.plane + g];
    V[c] = A.V[c * A.plane + g];
  }
  {
    const bool m = mirrored(col, A.nx, A.bc[0], A.bc[1]);
    mirror_state<Sys, 0>(m, U);
    mirror_normal_derivative<Sys, 0>(m, V);
    const int fs = fixed_side(col, A.nx, A.bc[0], A.bc[1]);
    if (fs >= 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        U[c] = T(A.gs[fs][c]);
        V[c] = T(0);
      }
    }
  }
  // derivatives carried times dx (see sweep_x)
#pragma unroll
  for (int c = 0; c < NC; ++c) V[c] = T(A.s.dx) * V[c];
  double RU[NC], RV[NC], RW[NC];
  T vt[NC];
  const auto ce = sy.cell_eig(U);
  sweep_x<2, IFACE>(sy, A.s, A.pk, ax, ce, U, V, W, RU, RV, RW, vt);
  double smax = 0.0;
  unsigned flag = 0;
  if (out) {
    T Un[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int o = c * A.plane + col;
      const double ub = MODE >= kStage2 ? (double)A.Ub[o] : 0.0;
      const double vb = MODE >= kStage2 ? (double)A.Vb[o] : 0.0;
      const double vtc = (double)vt[c] * A.s.idx;
      Un[c] = (T)rk_part<MODE>((double)U[c], ub, dt, RU[c]);
      A.Uo[o] = Un[c];
      A.Vo[o] = (T)rk_part<MODE>(vtc, vb, dt, RV[c]);
      if (MODE == kStage1 || MODE == kRhs) A.Vt[o] = (T)vtc;
    }
    if (A.alpha_next) {
      double sy_;
      flag = sy.speeds(Un, smax, sy_);
    }
  }
  if (A.alpha_next) {
    smax = wave_max(smax);
    flag = wave_or(flag);
    if (lane == 0) {
      atomic_max_pos(A.alpha_next, smax);
      if (flag && A.flags) atomicOr(A.flags, flag);
    }
  }
}

// ------------------------------------------------------------ 2D stage kernel
// Loads row r of column gcol (ghost rows and columns by index map). With
// WALLS (some boundary is reflective or fixed): xm, this lane is a ghost
// column behind a reflective wall; xf, the fixed side whose state this ghost
// lane holds (or -1); xwall, some lane of the wavefront is either
// (wave-uniform, so unaffected blocks skip this code). Problems with neither
// use the kernel without this code, whose register allocation it would
// disturb.
template <class Sys, bool WALLS, typename T>
__device__ __forceinline__ void load_row(const StageArgs<T>& A, double tstage, int r, int col,
                                         int gcol, T (&U)[Sys::NC], T (&V)[Sys::NC],
                                         T (&W)[Sys::NC], int& split_rule) {
  int gr = map_index(r, A.ny, A.bc[2], A.bc[3]);
  // split side: this lane's rule from its x, the ghost row's y and the
  // stage time (0: transmissive, 1: reflective, 2 + k: fixed state k)
  split_rule = -1;
  if constexpr (WALLS) {
    const int yside = r < 0 ? 0 : (r >= A.ny ? 1 : -1);
    if (yside >= 0 && A.bc[2 + yside] == kBcSplit) {
      const SplitRule& sr = A.sp[yside];
      const double xs = sr.x0 + sr.slope * ((r + 0.5) * A.s.dy) + sr.speed * tstage;
      const int k = (col + 0.5) * A.s.dx < xs ? 0 : 1;
      const int kind = sr.kind[k];
      split_rule = kind == kBcReflective ? 1 : (kind == kBcDirichlet ? 2 + k : 0);
      if (split_rule == 1) gr = map_index(r, A.ny, kBcReflective, kBcReflective);
    }
  }
  const unsigned off = (unsigned)(gr * A.nx + gcol);
#pragma unroll
  for (int c = 0; c < Sys::NC; ++c) {
    const unsigned i = (unsigned)(c * A.plane) + off;
    U[c] = ld32(A.U, i);
    V[c] = ld32(A.V, i);
    W[c] = ld32(A.W, i);
  }
}

// What load_row leaves to the row's first use (so that the loads stay in
// flight until then): the ghost rules of walls, fixed states and split sides,
// and the derivatives times their mesh width (see sweep_x).
template <class Sys, bool WALLS, typename T>
__device__ __forceinline__ void finish_row(const StageArgs<T>& A, int r, bool xwall, bool xm,
                                           int xf, int split_rule, T (&U)[Sys::NC],
                                           T (&V)[Sys::NC], T (&W)[Sys::NC]) {
  if constexpr (WALLS) {
    auto fix = [&](int side) {
#pragma unroll
      for (int c = 0; c < Sys::NC; ++c) {
        U[c] = T(A.gs[side][c]);
        V[c] = T(0);
        W[c] = T(0);
      }
    };
    if (xwall) {
      mirror_state<Sys, 0>(xm, U);
      mirror_normal_derivative<Sys, 0>(xm, V);
      mirror_state<Sys, 0>(xm, W);
      if (xf >= 0) fix(xf);
    }
    if (mirrored(r, A.ny, A.bc[2], A.bc[3]) || split_rule == 1) {
      mirror_state<Sys, 1>(true, U);
      mirror_state<Sys, 1>(true, V);
      mirror_normal_derivative<Sys, 1>(true, W);
    }
    const int yf = fixed_side(r, A.ny, A.bc[2], A.bc[3]);
    if (yf >= 0) fix(2 + yf);
    if (split_rule >= 2) {
      const SplitRule& sr = A.sp[r < 0 ? 0 : 1];
#pragma unroll
      for (int c = 0; c < Sys::NC; ++c) {
        U[c] = T(sr.state[split_rule - 2][c]);
        V[c] = T(0);
        W[c] = T(0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < Sys::NC; ++c) {
    V[c] = T(A.s.dx) * V[c];
    W[c] = T(A.s.dy) * W[c];
  }
}

// VAR: kVarWalls (some boundary is reflective or fixed), kVarIface (interface
// basis), kVarSource (the gravity source of (euler2d-s)); each combination is
// its own instantiation, so the common one carries no code of the others.
constexpr int kVarWalls = 1, kVarIface = 2, kVarSource = 4;

// Tile of a workgroup in a 2D grid of tiles (row-major, gridDim.x tiles a
// row). Workgroups go to the eight XCDs (each with its own L2) in turn by
// linear id; this gives every XCD one contiguous run of tiles, so that
// horizontally adjacent tiles, which re-read each other's halo columns and
// share the cache lines at their edges, mostly sit behind the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int nbx = gridDim.x, n = nbx * gridDim.y;
  const int h = blockIdx.x + nbx * blockIdx.y;
  const int q = n / kXcds, rem = n % kXcds;   // XCDs below rem take q + 1 tiles
  const int x = h % kXcds;
  const int L = x * q + min(x, rem) + h / kXcds;
  by = L / nbx;
  bx = L - by * nbx;
}

template <class Sys, typename T, int MODE, int VAR>
__global__ __launch_bounds__(64) void stage2d_kernel(StageArgs<T> A, Sys sy) {
  constexpr bool WALLS = (VAR & kVarWalls) != 0;
  constexpr bool IFACE = (VAR & kVarIface) != 0;
  constexpr bool SOURCE = (VAR & kVarSource) != 0 && Sys::kChar && Sys::NC == 4;
  constexpr int NC = Sys::NC;
  const Scheme& s = A.s;
  const int lane = threadIdx.x;
  double dt, tstage;
  int bx, by;
  xcd_tile(bx, by);
  if (!stage_begin<MODE>(A, bx == 0 && by == 0 && lane == 0, dt, tstage)) return;
  const int col = bx * kXOut - kHalo + lane;
  const int gcol = map_index(col, A.nx, A.bc[0], A.bc[1]);
  const bool out_col = lane >= kHalo && lane < kWave - kHalo && col < A.nx;
  const bool xm = mirrored(col, A.nx, A.bc[0], A.bc[1]);
  const int xf = fixed_side(col, A.nx, A.bc[0], A.bc[1]);
  const int col0 = bx * kXOut - kHalo;   // the wavefront's first column
  auto special = [](int b) { return b == kBcReflective || b == kBcDirichlet; };
  const bool xwall = (special(A.bc[0]) && col0 < 0) || (special(A.bc[1]) && col0 + kWave > A.nx);
  const int y0 = by * A.rows;
  const int y1 = min(y0 + A.rows, A.ny);
  const double ax = A.alpha[0], ay = A.alpha[1];
  const T a_y = T(ay);
  // weights of the y flux differences (fprev - F) in the new state: the
  // stage's weight of dt L times 1/dy (and 1/(12 dy) for the mixed flux,
  // which is carried times 12)
  const double wl = rk_wl<MODE>(dt) * s.idy;
  // the v-equation's y-fluxes carry 12 dx, the w-equation's dy
  const double wlv = wl * s.idx * (1.0 / 12.0), wlw = wl * s.idy;

  // Rows march upwards; at iteration r the rows r-2, r-1 (registers) and r
  // (just loaded) are present. Iteration r does: the pointwise y-fluxes of
  // row r; the HWENO of row r-1 in y, then in x with the same
  // characteristic basis; the y-interface (r-2)+1/2 and with it the output
  // row r-2; the x-sweep of row r-1, whose flux difference and RK
  // combination wait in LDS (pend) until the next iteration adds the
  // y-part. U, W of rows r-2, r-1 and V of row r-1 stay in registers.
  T Ua[NC], Ub[NC], Wa[NC], Wb[NC], Vb[NC];
  // pointwise g, theta, xi of rows r-3, r-2, r-1, slot (row mod 3); each
  // lane only touches its own column
  __shared__ T ring[3][3][NC][kWave];
  int slot = ((y0 - 2) % 3 + 3) % 3;     // slot of row r (and of row r-3)
  // Lax-Friedrichs sums g(u) + a u, theta + a w at the top face of row r-2
  __shared__ T topr[2][NC][kWave];
  // y-interface fluxes g, theta, 12 xi at (r-3)+1/2
  __shared__ T fprev[3][NC][kWave];
  // RK combination of row r-2 (u, v, w) without its y flux difference
  __shared__ double pend[3][NC][kWave];
  double smx = 0.0, smy = 0.0;
  unsigned flag = 0;

  T Un[NC], Vn[NC], Wn[NC];
  T Bu[NC], Bv[NC], Bw[NC];              // RK base of row r-1 (stages 2-3)
  // The y-work below runs in every iteration, also in the first ones, whose
  // results are never used (so that it forms one block of straight-line code
  // the compiler can schedule across): start from an admissible state.
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    Ua[c] = Ub[c] = T(c == 0 ? 1.0 : (c == NC - 1 ? 2.0 : 0.0));
    Wa[c] = Wb[c] = Vb[c] = T(0);
  }
  int rule_n;
  load_row<Sys, WALLS>(A, tstage, y0 - 2, col, gcol, Un, Vn, Wn, rule_n);
  for (int r = y0 - 2; r < y1 + 2; ++r) {
    T Uc[NC], Vc[NC], Wc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) { Uc[c] = Un[c]; Vc[c] = Vn[c]; Wc[c] = Wn[c]; }
    finish_row<Sys, WALLS>(A, r, xwall, xm, xf, rule_n, Uc, Vc, Wc);
    if (r + 1 < y1 + 2) load_row<Sys, WALLS>(A, tstage, r + 1, col, gcol, Un, Vn, Wn, rule_n);  // prefetch
    // RK base of row r, for the x-sweep of the next iteration (rows and
    // columns clamped into the array: the values outside are never used)
    T Bun[NC], Bvn[NC], Bwn[NC];
    if constexpr (MODE >= kStage2) {
      const int rr = min(max(r, 0), A.ny - 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const unsigned idx = (unsigned)(c * A.plane + rr * A.nx + gcol);
        Bun[c] = ld32(A.Ub, idx);
        Bvn[c] = ld32(A.Vb, idx);
        Bwn[c] = ld32(A.Wb, idx);
      }
    }
    // pointwise g, theta = g'(u) w, xi = g'(u) v of row r
    T gc[NC], tc[NC], xc[NC];
    {
      const auto q = sy.prim(Uc);
      sy.template flux<1>(Uc, q, gc);
      sy.template jac<1>(Uc, q, Wc, tc);
      sy.template jac<1>(Uc, q, Vc, xc);
    }
    // HWENO in y of row r-1: u at its top and bottom faces, w~, and the LF
    // sums there
    typename Sys::template CellEig<T> ce;
    T mG[NC], mT[NC], pG[NC], pT[NC], wt[NC];
    {
      ce = sy.cell_eig(Ub);
      T uT[NC], uB[NC], wT[NC], wB[NC];
      if constexpr (IFACE) {
        // mesh width 1 for the scaled derivatives
        hweno_cell_b<1, true>(sy, s, 1.0, 1.0, ce.q, Ua, Ub, Uc, Wa, Wc, uT, uB, wt);
#pragma unroll
        for (int c = 0; c < NC; ++c) face_derivs(Ua[c], Ub[c], Uc[c], Wa[c], Wc[c], T(1), wT[c], wB[c]);
      } else {
        T E1[NC], E2[NC], Sw[NC], Dw[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          E1[c] = Ub[c] - Ua[c];
          E2[c] = Uc[c] - Ub[c];
          Sw[c] = Wa[c] + Wc[c];
          Dw[c] = Wa[c] - Wc[c];
        }
        hweno_cell_diff<1>(sy, A.pk, ce, Ub, E1, E2, Sw, Dw, uT, uB, wt, wT, wB);
      }
      T gt[NC], tt[NC], gb[NC], tb[NC];
      const auto qt = sy.prim(uT);
      sy.template flux<1>(uT, qt, gt);
      sy.template jac<1>(uT, qt, wT, tt);
      const auto qb = sy.prim(uB);
      sy.template flux<1>(uB, qb, gb);
      sy.template jac<1>(uB, qb, wB, tb);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        mG[c] = fma(a_y, uT[c], gt[c]);
        mT[c] = fma(a_y, wT[c], tt[c]);
        pG[c] = fma(-a_y, uB[c], gb[c]);
        pT[c] = fma(-a_y, wB[c], tb[c]);
      }
    }
    // y-interface (r-2)+1/2: minus side = top face of row r-2, plus side =
    // bottom face of row r-1; central correction from rows r-3..r
    T Gn[NC], Tn[NC], Xn[NC];
    {
      const int s3 = slot, s2 = slot == 2 ? 0 : slot + 1, s1 = slot == 0 ? 2 : slot - 1;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T g3 = ring[s3][0][c][lane], g2 = ring[s2][0][c][lane], g1 = ring[s1][0][c][lane];
        const T t3 = ring[s3][1][c][lane];
        const T x3 = ring[s3][2][c][lane], x2 = ring[s2][2][c][lane], x1 = ring[s1][2][c][lane];
        T Dg, Dt;
        central_corr_k(g3, g2, g1, gc[c], t3, tc[c], Dg, Dt);
        Gn[c] = fma(T(0.5), topr[0][c][lane] + pG[c], Dg);
        Tn[c] = fma(T(0.5), topr[1][c][lane] + pT[c], Dt);
        Xn[c] = fma(T(7), x2 + x1, -(x3 + xc[c]));
      }
    }
    // row r takes the ring slot of row r-3; row r-1's top-face sums replace
    // row r-2's
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ring[slot][0][c][lane] = gc[c];
      ring[slot][1][c][lane] = tc[c];
      ring[slot][2][c][lane] = xc[c];
      topr[0][c][lane] = mG[c];
      topr[1][c][lane] = mT[c];
    }
    // output row o = r - 2: the pending combination plus its y flux
    // difference (odeH)/(ode2H), Step 4
    T Unew[NC], Vnew[NC], Wnew[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Unew[c] = (T)fma(wl, (double)fprev[0][c][lane] - (double)Gn[c], pend[0][c][lane]);
      Vnew[c] = (T)fma(wlv, (double)fprev[2][c][lane] - (double)Xn[c], pend[1][c][lane]);
      Wnew[c] = (T)fma(wlw, (double)fprev[1][c][lane] - (double)Tn[c], pend[2][c][lane]);
      fprev[0][c][lane] = Gn[c];
      fprev[1][c][lane] = Tn[c];
      fprev[2][c][lane] = Xn[c];
    }
    if (r >= y0 + 2 && out_col) {
      const unsigned row = (unsigned)((r - 2) * A.nx + col);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const unsigned idx = (unsigned)(c * A.plane) + row;
        st32(A.Uo, idx, Unew[c]);
        st32(A.Vo, idx, Vnew[c]);
        st32(A.Wo, idx, Wnew[c]);
      }
      if (A.alpha_next) {
        double sx_, sy_;
        flag |= sy.speeds(Unew, sx_, sy_);
        smx = fmax(smx, sx_);
        smy = fmax(smy, sy_);
      }
    }
    if (r >= y0 + 1 && r <= y1) {
      // x-sweep of row r-1 and its RK combination without the y part.
      // Keep the scheduler from interleaving it with the y-work above:
      // both working sets live at once would spill.
      __builtin_amdgcn_sched_barrier(0);
      double RU[NC], RV[NC], RW[NC];
      T vt[NC];
      sweep_x<3, IFACE>(sy, s, A.pk, ax, ce, Ub, Vb, Wb, RU, RV, RW, vt);
      if (out_col) {
        const unsigned row = (unsigned)((r - 1) * A.nx + col);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double lu = RU[c], lv = RV[c], lw = RW[c];
          if constexpr (SOURCE) {
            // S(X) = g (0, 0, X_0, X_2) for X = u, v, w of the stage state
            // (v, w held times dx, dy)
            if (c >= 2) {
              const int k = c == 2 ? 0 : 2;
              lu = fma(A.gravity, (double)Ub[k], lu);
              lv = fma(A.gravity * s.idx, (double)Vb[k], lv);
              lw = fma(A.gravity * s.idy, (double)Wb[k], lw);
            }
          }
          const double ub = MODE >= kStage2 ? (double)Bu[c] : 0.0;
          const double vb = MODE >= kStage2 ? (double)Bv[c] : 0.0;
          const double wb = MODE >= kStage2 ? (double)Bw[c] : 0.0;
          const double vtc = (double)vt[c] * s.idx, wtc = (double)wt[c] * s.idy;
          pend[0][c][lane] = rk_part<MODE>((double)Ub[c], ub, dt, lu);
          pend[1][c][lane] = rk_part<MODE>(vtc, vb, dt, lv);
          pend[2][c][lane] = rk_part<MODE>(wtc, wb, dt, lw);
          if (MODE == kStage1 || MODE == kRhs) {
            const unsigned idx = (unsigned)(c * A.plane) + row;
            st32(A.Vt, idx, (T)vtc);
            st32(A.Wt, idx, (T)wtc);
          }
        }
      }
    }
    // rotate the registers
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Ua[c] = Ub[c]; Ub[c] = Uc[c];
      Wa[c] = Wb[c]; Wb[c] = Wc[c];
      Vb[c] = Vc[c];
      if (MODE >= kStage2) { Bu[c] = Bun[c]; Bv[c] = Bvn[c]; Bw[c] = Bwn[c]; }
    }
    slot = slot == 2 ? 0 : slot + 1;
  }
  if (A.alpha_next) {
    smx = wave_max(smx);
    smy = wave_max(smy);
    flag = wave_or(flag);
    if (lane == 0) {
      atomic_max_pos(A.alpha_next, smx);
      atomic_max_pos(A.alpha_next + 1, smy);
      if (flag && A.flags) atomicOr(A.flags, flag);
    }
  }
}

// -------------------------------------------- wave-speed reduction (flux-LF)
// Per-block maxima of the spectral radius over interior cells, in x and y;
// also raises the state flags.
template <class Sys, typename T, int DIM>
__global__ __launch_bounds__(256) void speed_partial_kernel(const T* U, int plane, Sys sy,
                                                            double* partial, unsigned* flags) {
  constexpr int NC = Sys::NC;
  double mx = 0.0, my = 0.0;
  unsigned flag = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += gridDim.x * blockDim.x) {
    T u[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] = U[c * plane + i];
    double sx_, sy_;
    flag |= sy.speeds(u, sx_, sy_);
    mx = fmax(mx, sx_);
    if (DIM == 2) my = fmax(my, sy_);
  }
  __shared__ double sx[4], sy_[4];
  __shared__ unsigned sf[4];
  mx = wave_max(mx);
  my = wave_max(my);
  flag = wave_or(flag);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { sx[w] = mx; sy_[w] = my; sf[w] = flag; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    for (int k = 1; k < nw; ++k) { mx = fmax(mx, sx[k]); my = fmax(my, sy_[k]); flag |= sf[k]; }
    partial[2 * blockIdx.x] = mx;
    partial[2 * blockIdx.x + 1] = my;
    if (flag && flags) atomicOr(flags, flag);
  }
}

__device__ void reduce_partials(const double* partial, int n, double* ax, double* ay) {
  __shared__ double rx[256], ry[256];
  double mx = 0.0, my = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    mx = fmax(mx, partial[2 * i]);
    my = fmax(my, partial[2 * i + 1]);
  }
  rx[threadIdx.x] = mx;
  ry[threadIdx.x] = my;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      rx[threadIdx.x] = fmax(rx[threadIdx.x], rx[threadIdx.x + st]);
      ry[threadIdx.x] = fmax(ry[threadIdx.x], ry[threadIdx.x + st]);
    }
    __syncthreads();
  }
  *ax = rx[0];
  *ay = ry[0];
}

__global__ __launch_bounds__(256) void alpha_out_kernel(const double* partial, int n, double* alpha) {
  double ax, ay;
  reduce_partials(partial, n, &ax, &ay);
  if (threadIdx.x == 0) { alpha[0] = ax; alpha[1] = ay; }
}

// Seeds a run of steps (flux-LF): reduces the per-block maxima of the state's
// spectral radii into the next-step accumulators (the stage-1 alphas of the
// first step) and clears the stage-2 and stage-3 accumulators.
__global__ __launch_bounds__(256) void alpha_seed_kernel(const double* partial, int n,
                                                         StepScalars* sc) {
  double ax, ay;
  reduce_partials(partial, n, &ax, &ay);
  if (threadIdx.x != 0) return;
  sc->acc[4] = (unsigned long long)__double_as_longlong(ax);
  sc->acc[5] = (unsigned long long)__double_as_longlong(ay);
  for (int k = 0; k < 4; ++k) sc->acc[k] = 0ull;
}

__global__ void ws_init_kernel(StepScalars* sc) {
  for (int k = 0; k < 6; ++k) sc->acc[k] = 0ull;
  sc->dt = sc->t0 = sc->tnew = 0.0;
  sc->active = 0;
  sc->flags = 0u;
}

// ================================================================ adjoint
// Vector-Jacobian product of one stage for the x direction, on lines laid
// out along memory rows (1D, or each row of a 2D field). Given the
// state X = (u, a, o) -- a the derivative along the line, o the other one --
// and cotangents a_B of B(X) = (u, a~, ...) and b of L(X), it writes
//   G = (dB/dX)^T a_B + (dL_dir/dX)^T b
// restricted to this direction's terms (in 2D it adds that to G, which
// holds the y-direction terms). Lanes hold "virtual" cells v =
// 60 b - 4 + lane (ghost cells included), so every virtual cell in
// [-2, n+2) is an output lane of exactly one block; contributions to ghost
// cells go to a side buffer and are folded into their images by
// ghost_fold_kernel (the transpose of the ghost index map).
template <typename T>
struct VjpArgs {
  const T* X[3];          // u, along-derivative, other derivative (null in 1D)
  const T* b[3];          // b = cb dt lam_b: the one cotangent state L sees
  const T* a[3][2];       // a_B = sum_k ca_k lam_k (u and along fields)
  double ca[3];
  double cb;              // multiplied by *dt
  const double* dt;
  const double* alpha;    // [2]; this pass uses alpha[dir]
  int dir;
  int add_identity;       // add the u-part of a_B (B's u-component is the identity)
  int accumulate;         // 2D: add the result and the y-pass's folds to G (else overwrite G)
  T* G[3];                // outputs (u, along, other)
  // with accumulate: the y-pass's strip halos [strip][2 sides][u, w][NC][n]
  // and ghost rows [4][3][NC][n], its strip height and count, the y sides
  // ghost row k (-2, -1, ny, ny+1): the row it folds into (-1: none), whether
  // the wall's sign rules apply, the strip (-1: none) and side of the halo
  // term aimed at it
  const T* yhalo;
  const T* yghost;
  int yR, ystrips;
  int yimg[4], yflip[4], yqj[4], yqs[4];
  T* ghost;               // [rows][4][3][NC] contributions of virtual cells -2, -1, n, n+1
  int n, rows, plane;
  int bc_lo, bc_hi;
  double gs[2][4];        // fixed ghost states of the low and high side
  double h, ih;
  Scheme s;
};

// The y-pass strip whose halo term is aimed at virtual row q: strip j (rows
// [-2 + jR, -2 + (j+1)R)) sends side 0 to its row o0 - 1 and side 1 to its
// row o1. Returns j (side in `side`), or -1.
HWENO_HD int halo_source(int q, int R, int nstrips, int& side) {
  if ((q + 3) % R == 0) {
    const int j = (q + 3) / R;
    if (j >= 1 && j <= nstrips - 1) {
      side = 0;
      return j;
    }
  }
  if ((q + 2) % R == 0) {
    const int j = (q + 2) / R - 1;
    if (j >= 0 && j <= nstrips - 2) {
      side = 1;
      return j;
    }
  }
  return -1;
}

template <class Sys, typename T, int D, int NF, int NA, bool WALLS, bool IFACE = false>
__global__ __launch_bounds__(64) void vjp_row_kernel(VjpArgs<T> A, Sys sy) {
  // WALLS: some side of this direction is reflective or fixed
  constexpr int NC = Sys::NC;
  using Bar = typename BarOf<Sys, T>::type;
  const int lane = threadIdx.x;
  int bx, row;
  xcd_tile(bx, row);
  const int v = bx * kXOut - 4 + lane;
  const int g = map_index(v, A.n, A.bc_lo, A.bc_hi);
  const bool interior = v >= 0 && v < A.n;
  const bool out = lane >= kHalo && lane < kWave - kHalo && v >= -2 && v < A.n + 2;
  const int base = row * A.n;
  const double dtv = A.dt ? *A.dt : 0.0;
  const T alpha = T(A.alpha[A.dir]);
  const T h = T(A.h), ih = T(A.ih);
  const Scheme& s = A.s;

  // with A.accumulate, the values this pass adds to, and the y-pass halo
  // term aimed at this row (u, w), copied into LDS while the lane works
  __shared__ T gin[NF][NC][kWave];
  __shared__ T yh[2][NC][kWave];
  int hside = 0;
  const int hj = A.accumulate ? halo_source(row, A.yR, A.ystrips, hside) : -1;
  if (A.accumulate) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int f = 0; f < NF; ++f)
        row_to_lds(A.G[f], (unsigned)(c * A.plane + base), bx * kXOut - 4, A.n, &gin[f][c][0], lane);
    if (hj >= 0) {
#pragma unroll
      for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          row_to_lds(A.yhalo, (unsigned)(((hj * 4 + hside * 2 + hf) * NC + c) * A.n),
                     bx * kXOut - 4, A.n, &yh[hf][c][0], lane);
    }
  }
  T U[NC], Av[NC], Ov[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const unsigned i = (unsigned)(c * A.plane + base + g);
    U[c] = ld32(A.X[0], i);
    Av[c] = ld32(A.X[1], i);
    Ov[c] = NF == 3 ? ld32(A.X[2], i) : T(0);
  }
  if constexpr (WALLS) {
    const bool m = mirrored(v, A.n, A.bc_lo, A.bc_hi);
    mirror_state<Sys, D>(m, U);
    mirror_normal_derivative<Sys, D>(m, Av);
    mirror_state<Sys, D>(m, Ov);
    const int fs = fixed_side(v, A.n, A.bc_lo, A.bc_hi);
    if (fs >= 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        U[c] = T(A.gs[fs][c]);
        Av[c] = T(0);
        Ov[c] = T(0);
      }
    }
  }
  // cotangents; zero at ghost cells (L and B are defined on interior cells)
  T aU[NC], aA[NC], bU[NC], bA[NC], bO[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) { aU[c] = T(0); aA[c] = T(0); bU[c] = T(0); bA[c] = T(0); bO[c] = T(0); }
  if (interior) {
    const T cbt = T(A.cb * dtv);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const unsigned idx = (unsigned)(c * A.plane + base + v);
      bU[c] = cbt * ld32(A.b[0], idx);
      bA[c] = cbt * ld32(A.b[1], idx);
      if (NF == 3) bO[c] = cbt * ld32(A.b[2], idx);
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        aU[c] += T(A.ca[k]) * ld32(A.a[k][0], idx);
        aA[c] += T(A.ca[k]) * ld32(A.a[k][1], idx);
      }
    }
  }
  // ---- forward recompute of this cell's interface values
  T Um[NC], Up[NC], Am[NC], Ap[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    Um[c] = from_prev(U[c]);
    Up[c] = from_next(U[c]);
    Am[c] = from_prev(Av[c]);
    Ap[c] = from_next(Av[c]);
  }
  T uR[NC], uL[NC], at_[NC], vR[NC], vL[NC];
  hweno_cell_b<D, IFACE>(sy, s, A.h, A.ih, sy.prim(U), Um, U, Up, Am, Ap, uR, uL, at_);
#pragma unroll
  for (int c = 0; c < NC; ++c) face_derivs(Um[c], U[c], Up[c], Am[c], Ap[c], ih, vR[c], vL[c]);
  // ---- interface cotangents: L_i = -(F_{i+1/2} - F_{i-1/2}) / h
  T lF[NC], lH[NC], lE[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    lF[c] = (from_next(bU[c]) - bU[c]) * ih;
    lH[c] = (from_next(bA[c]) - bA[c]) * ih;
    lE[c] = NF == 3 ? (from_next(bO[c]) - bO[c]) * ih : T(0);
  }
  // ---- Lax-Friedrichs halves: minus side of x_{v+1/2} (uR, vR) and plus
  // side of x_{v-1/2} (uL, vL)
  T guR[NC], gvR[NC], guL[NC], gvL[NC];
  {
    T hF[NC], hH[NC], pF[NC], pH[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      hF[c] = T(0.5) * lF[c];
      hH[c] = T(0.5) * lH[c];
      pF[c] = T(0.5) * from_prev(lF[c]);
      pH[c] = T(0.5) * from_prev(lH[c]);
      guR[c] = alpha * hF[c];
      gvR[c] = alpha * hH[c];
      guL[c] = -alpha * pF[c];
      gvL[c] = -alpha * pH[c];
    }
    const auto qr = sy.prim(uR);
    Bar br{};
    flux_vjp<D>(sy, uR, qr, hF, br, guR);
    jac_vjp<D>(sy, uR, qr, vR, hH, br, guR, gvR);
    prim_vjp(sy, uR, qr, br, guR);
    const auto ql = sy.prim(uL);
    Bar bl{};
    flux_vjp<D>(sy, uL, ql, pF, bl, guL);
    jac_vjp<D>(sy, uL, ql, vL, pH, bl, guL, gvL);
    prim_vjp(sy, uL, ql, bl, guL);
  }
  // ---- central correction and mixed flux: gather from interfaces v-2..v+1
  T gU[NC], gA[NC], gO[NC];
  {
    T gf[NC], gh[NC], ge[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T F1 = from_next(lF[c]), F0 = lF[c], Fm1 = from_prev(lF[c]), Fm2 = from_prev(Fm1);
      const T H1 = from_next(lH[c]), H0 = lH[c], Hm1 = from_prev(lH[c]), Hm2 = from_prev(Hm1);
      gf[c] = T(97.0 / 1920.0) * ((F0 + Fm1) - (F1 + Fm2)) +
              ih * (T(697.0 / 5184.0) * (H1 - Hm2) + T(61.0 / 192.0) * (Hm1 - H0));
      gh[c] = T(19.0 / 960.0) * h * (Fm2 - F1) + T(37.0 / 864.0) * (H1 + Hm2);
      if constexpr (NF == 3) {
        const T E1 = from_next(lE[c]), E0 = lE[c], Em1 = from_prev(lE[c]), Em2 = from_prev(Em1);
        ge[c] = (T(7.0) * (E0 + Em1) - (E1 + Em2)) * T(1.0 / 12.0);
      } else {
        ge[c] = T(0);
      }
      gU[c] = T(0);
      gA[c] = T(0);
      gO[c] = T(0);
    }
    // pointwise f, f'(u) a, f'(u) o at the cell
    const auto q = sy.prim(U);
    Bar bq{};
    flux_vjp<D>(sy, U, q, gf, bq, gU);
    jac_vjp<D>(sy, U, q, Av, gh, bq, gU, gA);
    if constexpr (NF == 3) jac_vjp<D>(sy, U, q, Ov, ge, bq, gU, gO);
    prim_vjp(sy, U, q, bq, gU);
  }
  // ---- face derivatives and HWENO of this cell -> its stencil
  T tm[NC], tc[NC], tp[NC], tAm[NC], tAp[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    tm[c] = T(0); tc[c] = T(0); tp[c] = T(0); tAm[c] = T(0); tAp[c] = T(0);
    face_derivs_vjp(gvR[c], gvL[c], ih, tm[c], tc[c], tp[c], tAm[c], tAp[c]);
  }
  hweno_cell_vjp_b<D, IFACE, true>(sy, s, A.h, A.ih, Um, U, Up, Am, Ap, guR, guL, aA, tm, tc, tp,
                                   tAm, tAp);
  // ---- gather: own + right-neighbour part of the left lane + left part of the right lane
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    gU[c] += tc[c] + from_prev(tp[c]) + from_next(tm[c]);
    gA[c] += from_prev(tAp[c]) + from_next(tAm[c]);
    if (A.add_identity) gU[c] += aU[c];
  }
  unsigned gmask = 0;   // y ghost rows folding into this row
  if (A.accumulate) {
    wait_copies();
#pragma unroll
    for (int k = 0; k < 4; ++k) gmask |= A.yimg[k] == row ? 1u << k : 0u;
  }
  if (out) {
    if (interior) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const unsigned idx = (unsigned)(c * A.plane + base + v);
        if (A.accumulate) {
          gU[c] += gin[0][c][lane];
          gA[c] += gin[1][c][lane];
          if (NF == 3) gO[c] += gin[NF - 1][c][lane];
          if (hj >= 0) {
            gU[c] += yh[0][c][lane];
            if (NF == 3) gO[c] += yh[1][c][lane];
          }
          // the y ghost rows whose image is this row (edge rows only), each
          // with the halo term aimed at it, with the y walls' sign rules
          if (gmask) {
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
              if (!((gmask >> k) & 1u)) continue;
              const int qj = A.yqj[k], qs = A.yqs[k];
              T gv[3];
#pragma unroll
              for (int f = 0; f < 3; ++f) {
                gv[f] = A.yghost[((size_t)(k * 3 + f) * NC + c) * A.n + v];
                if (qj >= 0 && f != 1)
                  gv[f] += A.yhalo[((size_t)(qj * 4 + qs * 2 + (f == 0 ? 0 : 1)) * NC + c) * A.n + v];
                if (A.yflip[k] && mirror_flips(1, f, c)) gv[f] = -gv[f];
              }
              gU[c] += gv[0];
              gA[c] += gv[1];
              if (NF == 3) gO[c] += gv[2];
            }
          }
        }
        st32(A.G[0], idx, gU[c]);
        st32(A.G[1], idx, gA[c]);
        if (NF == 3) st32(A.G[2], idx, gO[c]);
      }
    } else {
      const int slot = v < 0 ? v + 2 : v - A.n + 2;
      T* gp = A.ghost + ((size_t)row * 4 + slot) * 3 * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        gp[c] = gU[c];
        gp[NC + c] = gA[c];
        gp[2 * NC + c] = gO[c];
      }
    }
  }
}

// y-direction VJP by marching up strips of rows (2D; natural layout, no
// transposes). Each lane owns one column and needs no neighbour lane. Strip k
// owns the virtual rows [o0, o1) of [-2, ny+2) and reverses the HWENO of its
// own cells only: the contributions of cell o0 to row o0-1 and of cell o1-1
// to row o1 go to a halo buffer, and the x-pass (vjp_row_kernel) adds them,
// and the ghost rows kept in a side buffer, to the rows they belong to. At iteration r (row r
// loaded): the interface cotangents of (r-1)+1/2, the reverse of cell r-1's
// HWENO and face values if the strip owns it (contributions to rows r-2..r),
// and the reverse of row r-2's pointwise fluxes; row r-2 is then complete up
// to the halo terms and is stored to G (the x-pass, which runs next, adds
// its own result). The next row's inputs are copied into LDS while a row is
// computed, so a row's loads wait on memory only once per strip.
template <typename T>
struct VjpYArgs {
  const T* X[3];          // u, v, w
  const T* b[3];          // b = cb dt lam_b (u, v, w)
  const T* aw[3];         // w fields of the a sets: a_w = sum_k ca_k lam_k,w
  double ca[3];
  double cb;              // multiplied by *dt
  int na;                 // number of a sets (1 or 3)
  const double* dt;
  const double* alpha;    // [2]; uses alpha[1]
  T* G[3];                // out (overwritten): u, v, w
  T* ghost;               // [4][3][NC][nx]: rows -2, -1, ny, ny+1
  T* halo;                // [strip][2: to row o0-1, to row o1][2: u, w][NC][nx]
  int nx, ny, rows, plane;
  int bc_lo, bc_hi;
  double gs[2][4];        // fixed ghost states of the low and high side (y)
  Scheme s;
};

template <class Sys, typename T, bool WALLS, bool IFACE = false>
__global__ __launch_bounds__(64) void vjp_y_kernel(VjpYArgs<T> A, Sys sy) {
  constexpr int NC = Sys::NC;
  using Bar = typename BarOf<Sys, T>::type;
  const int lane = threadIdx.x;
  const int x = blockIdx.x * kWave + lane;
  const bool colok = x < A.nx;
  const int o0 = -2 + blockIdx.y * A.rows;
  const int o1 = min(o0 + A.rows, A.ny + 2);
  const double dtv = A.dt ? *A.dt : 0.0;
  const T alpha = T(A.alpha[1]);
  const Scheme& s = A.s;
  const T h = T(s.dy), ih = T(s.idy);
  const T cbt = T(A.cb * dtv);
  // interface cotangents (G, theta, xi) of the 3 previous interfaces, slot k mod 3
  __shared__ T lring[3][3][NC][kWave];
  // the next row's inputs, copied in while the current row is computed:
  // u, v, w, b_u, b_v, b_w, then the a_w sets
  __shared__ T stage[9][NC][kWave];
  const int col0 = blockIdx.x * kWave;
  auto fetch = [&](int rr) {
    const int g = map_index(rr, A.ny, A.bc_lo, A.bc_hi);
    const bool in = rr >= 0 && rr < A.ny;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const unsigned off = (unsigned)(c * A.plane + g * A.nx);
#pragma unroll
      for (int f = 0; f < 3; ++f) row_to_lds(A.X[f], off, col0, A.nx, &stage[f][c][0], lane);
      if (in) {
#pragma unroll
        for (int f = 0; f < 3; ++f) row_to_lds(A.b[f], off, col0, A.nx, &stage[3 + f][c][0], lane);
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (k < A.na) row_to_lds(A.aw[k], off, col0, A.nx, &stage[6 + k][c][0], lane);
      }
    }
  };
  T Ua[NC], Ub[NC], Va[NC], Vb[NC], Wa[NC], Wb[NC];   // rows r-2, r-1
  T bU1[NC], bV1[NC], bW1[NC], aW1[NC];              // cotangents of row r-1
  T accUa[NC], accWa[NC], accUb[NC], accWb[NC];      // HWENO-reverse sums of rows r-2, r-1
#pragma unroll
  for (int c = 0; c < NC; ++c) { accUa[c] = T(0); accWa[c] = T(0); accUb[c] = T(0); accWb[c] = T(0); }
  fetch(o0 - 2);
  for (int r = o0 - 2; r < o1 + 2; ++r) {
    const bool inrow = r >= 0 && r < A.ny;
    wait_copies();
    T Uc[NC], Vc[NC], Wc[NC], bUc[NC], bVc[NC], bWc[NC], aWc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Uc[c] = stage[0][c][lane];
      Vc[c] = stage[1][c][lane];
      Wc[c] = stage[2][c][lane];
      bUc[c] = T(0); bVc[c] = T(0); bWc[c] = T(0); aWc[c] = T(0);
      if (inrow) {
        bUc[c] = cbt * stage[3][c][lane];
        bVc[c] = cbt * stage[4][c][lane];
        bWc[c] = cbt * stage[5][c][lane];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (k < A.na) aWc[c] += T(A.ca[k]) * stage[6 + k][c][lane];
      }
    }
    wait_lds_reads();
    if (r + 1 < o1 + 2) fetch(r + 1);
    if constexpr (WALLS) {
      if (mirrored(r, A.ny, A.bc_lo, A.bc_hi)) {
        mirror_state<Sys, 1>(true, Uc);
        mirror_state<Sys, 1>(true, Vc);
        mirror_normal_derivative<Sys, 1>(true, Wc);
      }
      const int fs = fixed_side(r, A.ny, A.bc_lo, A.bc_hi);
      if (fs >= 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          Uc[c] = T(A.gs[fs][c]);
          Vc[c] = T(0);
          Wc[c] = T(0);
        }
      }
    }
    // interface (r-1)+1/2: L_j = -(F_{j+1/2} - F_{j-1/2}) / dy
    T lG[NC], lT[NC], lX[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      lG[c] = (bUc[c] - bU1[c]) * ih;
      lT[c] = (bWc[c] - bW1[c]) * ih;
      lX[c] = (bVc[c] - bV1[c]) * ih;
    }
    const int s1 = ((r - 1) % 3 + 3) % 3;        // slot of interface r-1 (and r-4)
    const int s2 = s1 == 0 ? 2 : s1 - 1;          // interface r-2
    const int s3 = s2 == 0 ? 2 : s2 - 1;          // interface r-3
    T accUc[NC], accWc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) { accUc[c] = T(0); accWc[c] = T(0); }
    if (r >= o0 + 1 && r <= o1) {
      // reverse of cell r-1's faces: top face -> interface (r-1)+1/2 (minus
      // side), bottom face -> interface (r-2)+1/2 (plus side)
      T uT[NC], uB[NC], wt_[NC], wT[NC], wB[NC];
      hweno_cell_b<1, IFACE>(sy, s, s.dy, s.idy, sy.prim(Ub), Ua, Ub, Uc, Wa, Wc, uT, uB, wt_);
#pragma unroll
      for (int c = 0; c < NC; ++c) face_derivs(Ua[c], Ub[c], Uc[c], Wa[c], Wc[c], ih, wT[c], wB[c]);
      T hG[NC], hT[NC], pG[NC], pT[NC], guT[NC], gwT[NC], guB[NC], gwB[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        hG[c] = T(0.5) * lG[c];
        hT[c] = T(0.5) * lT[c];
        pG[c] = T(0.5) * lring[s2][0][c][lane];
        pT[c] = T(0.5) * lring[s2][1][c][lane];
        guT[c] = alpha * hG[c];
        gwT[c] = alpha * hT[c];
        guB[c] = -alpha * pG[c];
        gwB[c] = -alpha * pT[c];
      }
      {
        const auto qt = sy.prim(uT);
        Bar bt{};
        flux_vjp<1>(sy, uT, qt, hG, bt, guT);
        jac_vjp<1>(sy, uT, qt, wT, hT, bt, guT, gwT);
        prim_vjp(sy, uT, qt, bt, guT);
        const auto qb = sy.prim(uB);
        Bar bb{};
        flux_vjp<1>(sy, uB, qb, pG, bb, guB);
        jac_vjp<1>(sy, uB, qb, wB, pT, bb, guB, gwB);
        prim_vjp(sy, uB, qb, bb, guB);
      }
      T tm[NC], tc[NC], tWm[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        tm[c] = T(0); tc[c] = T(0); tWm[c] = T(0);
        face_derivs_vjp(gwT[c], gwB[c], ih, tm[c], tc[c], accUc[c], tWm[c], accWc[c]);
      }
      // the fused point reverse (one forward evaluation fewer) pays in FP32;
      // in FP64 its live intermediates spill (backward 76 -> 97 ms at 512^2)
      hweno_cell_vjp_b<1, IFACE, std::is_same<T, float>::value>(
          sy, s, s.dy, s.idy, Ua, Ub, Uc, Wa, Wc, guT, guB, aW1, tm, tc, accUc, tWm, accWc);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        accUa[c] += tm[c];
        accWa[c] += tWm[c];
        accUb[c] += tc[c];
      }
    }
    if (r == o0 + 1 && colok) {
      // row r-2 = o0-1 belongs to the strip below: its sums (from cell o0
      // alone) leave through the halo buffer
      T* hb = A.halo + (size_t)blockIdx.y * 4 * NC * A.nx + x;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        hb[(0 * NC + c) * A.nx] = accUa[c];
        hb[(1 * NC + c) * A.nx] = accWa[c];
      }
    }
    if (r >= o0 + 2) {
      // reverse of row r-2's pointwise g, theta, xi (interfaces r-4..r-1)
      const int o = r - 2;
      T gg[NC], gt[NC], gx[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T G1 = lG[c], G0 = lring[s2][0][c][lane], Gm1 = lring[s3][0][c][lane], Gm2 = lring[s1][0][c][lane];
        const T T1 = lT[c], T0 = lring[s2][1][c][lane], Tm1 = lring[s3][1][c][lane], Tm2 = lring[s1][1][c][lane];
        const T X1 = lX[c], X0 = lring[s2][2][c][lane], Xm1 = lring[s3][2][c][lane], Xm2 = lring[s1][2][c][lane];
        gg[c] = T(97.0 / 1920.0) * ((G0 + Gm1) - (G1 + Gm2)) +
                ih * (T(697.0 / 5184.0) * (T1 - Tm2) + T(61.0 / 192.0) * (Tm1 - T0));
        gt[c] = T(19.0 / 960.0) * h * (Gm2 - G1) + T(37.0 / 864.0) * (T1 + Tm2);
        gx[c] = (T(7.0) * (X0 + Xm1) - (X1 + Xm2)) * T(1.0 / 12.0);
      }
      T gU[NC], gV[NC], gW[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) { gU[c] = accUa[c]; gW[c] = accWa[c]; gV[c] = T(0); }
      const auto q = sy.prim(Ua);
      Bar bq{};
      flux_vjp<1>(sy, Ua, q, gg, bq, gU);
      jac_vjp<1>(sy, Ua, q, Wa, gt, bq, gU, gW);
      jac_vjp<1>(sy, Ua, q, Va, gx, bq, gU, gV);
      prim_vjp(sy, Ua, q, bq, gU);
      if (colok) {
        if (o >= 0 && o < A.ny) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const unsigned idx = (unsigned)(c * A.plane + o * A.nx + x);
            st32(A.G[0], idx, gU[c]);
            st32(A.G[1], idx, gV[c]);
            st32(A.G[2], idx, gW[c]);
          }
        } else {
          const int slot = o < 0 ? o + 2 : o - A.ny + 2;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            T* gp = A.ghost + ((size_t)slot * 3 * NC) * A.nx + x;
            gp[(0 * NC + c) * A.nx] = gU[c];
            gp[(1 * NC + c) * A.nx] = gV[c];
            gp[(2 * NC + c) * A.nx] = gW[c];
          }
        }
      }
    }
    // interface (r-1)+1/2 replaces (r-4)+1/2; rotate rows
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      lring[s1][0][c][lane] = lG[c];
      lring[s1][1][c][lane] = lT[c];
      lring[s1][2][c][lane] = lX[c];
      Ua[c] = Ub[c]; Ub[c] = Uc[c];
      Va[c] = Vb[c]; Vb[c] = Vc[c];
      Wa[c] = Wb[c]; Wb[c] = Wc[c];
      bU1[c] = bUc[c]; bV1[c] = bVc[c]; bW1[c] = bWc[c]; aW1[c] = aWc[c];
      accUa[c] = accUb[c]; accWa[c] = accWb[c];
      accUb[c] = accUc[c]; accWb[c] = accWc[c];
    }
  }
  // row o1 belongs to the strip above: its sums (from cell o1-1 alone) leave
  // through the halo buffer
  if (colok) {
    T* hb = A.halo + (size_t)blockIdx.y * 4 * NC * A.nx + x;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      hb[(2 * NC + c) * A.nx] = accUa[c];
      hb[(3 * NC + c) * A.nx] = accWa[c];
    }
  }
}

// Adds the ghost-cell contributions to the cells they were copied from (with
// the reflective sign rules where a wall mirrors them), in a fixed order (one
// thread per line, field and component).
template <typename T>
__global__ __launch_bounds__(256) void ghost_fold_kernel(T* __restrict__ G0, T* __restrict__ G1,
                                                         T* __restrict__ G2,
                                                         const T* __restrict__ ghost, int n, int rows,
                                                         int plane, int nc, int nf, int lo, int hi) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = rows * nf * nc;
  if (t >= total) return;
  const int c = t % nc;
  const int f = (t / nc) % nf;
  const int row = t / (nc * nf);
  T* G = (f == 0 ? G0 : (f == 1 ? G1 : G2)) + (size_t)c * plane + (size_t)row * n;
  const T* gp = ghost + (size_t)row * 4 * 3 * nc + f * nc + c;
  const int gs = 3 * nc;
  const T gv[4] = {gp[0], gp[gs], gp[2 * gs], gp[3 * gs]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {   // virtual cells -2, -1, n, n+1
    const int v = k < 2 ? k - 2 : n + k - 2;
    if (fixed_side(v, n, lo, hi) >= 0) continue;    // fixed states: no image
    const bool neg = mirrored(v, n, lo, hi) && mirror_flips(0, f, c);
    G[map_index(v, n, lo, hi)] += neg ? -gv[k] : gv[k];
  }
}

// Transpose of the gravity source (euler2d-s) of one stage:
// G_f += S^T (c dt b_f) for the fields f = u, v, w, where S(X) = g (0, 0,
// X_0, X_2): G_f[0] += g c dt b_f[2], G_f[2] += g c dt b_f[3].
template <typename T>
__global__ __launch_bounds__(256) void source_vjp_kernel(T* __restrict__ G0, T* __restrict__ G1,
                                                         T* __restrict__ G2, const T* __restrict__ b0,
                                                         const T* __restrict__ b1,
                                                         const T* __restrict__ b2, double cb,
                                                         const double* dt, double g, int plane) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  const T k = T(g * cb * *dt);
  T* Gs[3] = {G0, G1, G2};
  const T* bs[3] = {b0, b1, b2};
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    Gs[f][i] += k * bs[f][2 * plane + i];
    Gs[f][2 * plane + i] += k * bs[f][3 * plane + i];
  }
}

}  // namespace hweno

// The device scratch of hweno_step_noalloc: the workspace of a step (step
// scalars, per-block maxima, the stage states and the RK base derivatives)
// for callers that cannot allocate. One copy per GPU, held while the process
// lives. Host code must not pass `scratch` itself to a kernel (in host code it
// names a host-side stand-in): it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// =================================================================== host side
using namespace hweno;

namespace {

constexpr size_t kScalarBytes = 4096;
constexpr int kPartialBlocks = 1024;
constexpr size_t kPartialBytes = kPartialBlocks * 2 * sizeof(double);
constexpr int kRowsPerBlock = 32;

// Strip height of the 2D forward stage kernels set by hweno_set_strip_rows
// (0: chosen by the occupancy model).
std::atomic<int> g_strip_rows{0};

struct Geometry {
  int nc, nf;           // components; fields per state (2 in 1D: u, v; 3 in 2D)
  size_t esize;         // element size
  size_t plane;         // cells
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// A finite Euler state (rho, momenta..., E) with rho > 0 and P > 0.
bool admissible_state(const double* q, int nc, double gas) {
  for (int c = 0; c < nc; ++c)
    if (!std::isfinite(q[c])) return false;
  double m2 = 0.0;
  for (int c = 1; c < nc - 1; ++c) m2 += q[c] * q[c];
  return q[0] > 0.0 && (gas - 1.0) * (q[nc - 1] - 0.5 * m2 / q[0]) > 0.0;
}

bool has_split(const hweno_problem* p) {
  return p->bc[2] == HWENO_SPLIT || p->bc[3] == HWENO_SPLIT;
}

hweno_status validate(const hweno_problem* p) {
  if (!p) return HWENO_EINVAL;
  if (p->dim != 1 && p->dim != 2) return HWENO_EINVAL;
  if (p->nx < 5) return HWENO_EINVAL;
  if (p->dim == 2 && p->ny < 5) return HWENO_EINVAL;
  if (p->dim == 1 && p->ny != 1) return HWENO_EINVAL;
  if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return HWENO_EINVAL;
  if (p->dim == 2 && (!(p->dy > 0.0) || !std::isfinite(p->dy))) return HWENO_EINVAL;
  if (p->system < HWENO_ADVECTION || p->system > HWENO_EULER) return HWENO_EINVAL;
  if (p->system == HWENO_EULER && !(p->gas_gamma > 1.0)) return HWENO_EINVAL;
  if (p->system == HWENO_ADVECTION && (!std::isfinite(p->adv_a) || !std::isfinite(p->adv_b)))
    return HWENO_EINVAL;
  if (!(p->gamma0 > 0.0 && p->gamma0 < 1.0)) return HWENO_EINVAL;
  if (!(p->d0 > 0.0 && p->d0 < 1.0)) return HWENO_EINVAL;
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return HWENO_EINVAL;
  for (int k = 0; k < 4; ++k) {
    if (p->bc[k] != HWENO_PERIODIC && p->bc[k] != HWENO_TRANSMISSIVE &&
        p->bc[k] != HWENO_REFLECTIVE && p->bc[k] != HWENO_DIRICHLET && p->bc[k] != HWENO_SPLIT)
      return HWENO_EINVAL;
    if (p->bc[k] == HWENO_SPLIT) {
      if (k < 2 || p->dim != 2 || p->system != HWENO_EULER) return HWENO_EINVAL;
      const hweno_split& sp = p->split[k - 2];
      if (!std::isfinite(sp.x0) || !std::isfinite(sp.slope) || !std::isfinite(sp.speed))
        return HWENO_EINVAL;
      for (int j = 0; j < 2; ++j) {
        const int kind = sp.kind[j];
        if (kind != HWENO_TRANSMISSIVE && kind != HWENO_REFLECTIVE && kind != HWENO_DIRICHLET)
          return HWENO_EINVAL;
        if (kind == HWENO_DIRICHLET && !admissible_state(sp.state[j], 4, p->gas_gamma))
          return HWENO_EINVAL;
      }
    }
    // reflective walls are defined for the Euler equations only
    if (p->bc[k] == HWENO_REFLECTIVE && p->system != HWENO_EULER) return HWENO_EINVAL;
    if (p->bc[k] == HWENO_DIRICHLET && (k < 2 || p->dim == 2)) {
      const double* q = p->bc_state[k];
      const int nc = p->system == HWENO_EULER ? p->dim + 2 : 1;
      if (p->system == HWENO_EULER) {
        if (!admissible_state(q, nc, p->gas_gamma)) return HWENO_EINVAL;
      } else if (!std::isfinite(q[0])) {
        return HWENO_EINVAL;
      }
    }
  }
  if (!std::isfinite(p->gravity)) return HWENO_EINVAL;
  if (p->gravity != 0.0 && !(p->system == HWENO_EULER && p->dim == 2)) return HWENO_EINVAL;
  if ((p->bc[0] == HWENO_PERIODIC) != (p->bc[1] == HWENO_PERIODIC)) return HWENO_EINVAL;
  if (p->dim == 2 && (p->bc[2] == HWENO_PERIODIC) != (p->bc[3] == HWENO_PERIODIC))
    return HWENO_EINVAL;
  if (p->precision != HWENO_F64 && p->precision != HWENO_F32) return HWENO_EINVAL;
  if (p->char_basis != HWENO_BASIS_CELL && p->char_basis != HWENO_BASIS_INTERFACE)
    return HWENO_EINVAL;
  const int nc = p->system == HWENO_EULER ? p->dim + 2 : 1;
  // 32-bit element offsets inside a state array, and 32-bit byte offsets in
  // the stage kernels
  if ((double)nc * (double)p->nx * (double)p->ny >= 2147483647.0) return HWENO_EINVAL;
  const double esize = p->precision == HWENO_F64 ? 8.0 : 4.0;
  if ((double)nc * (double)p->nx * (double)p->ny * esize >= 4294967296.0) return HWENO_EINVAL;
  return HWENO_OK;
}

Geometry geometry(const hweno_problem* p) {
  Geometry g;
  g.nc = p->system == HWENO_EULER ? p->dim + 2 : 1;
  g.nf = p->dim == 1 ? 2 : 3;
  g.esize = p->precision == HWENO_F64 ? 8 : 4;
  g.plane = (size_t)p->nx * (size_t)p->ny;
  return g;
}

// Workspace: scalars | per-block partial maxima | states | adjoint scratch.
// States are stored densely ([field][comp][ny][nx]); each region starts on a
// 256-byte boundary. Regions: X^(1), X^(2), the RK base derivatives
// (V~^n[, W~^n]), and for the adjoint: lambda^(2), lambda^(1), the
// ghost-cell side buffers and (2D) the y-pass strip halo terms.
struct WsLayout {
  StepScalars* sc;
  double* partial;
  char* x1;
  char* x2;
  char* base;
  char* lam2;
  char* lam1;
  char* ghost;     // x-pass ghost columns [ny][4][3][NC]
  char* ghost_y;   // y-pass ghost rows [4][3][NC][nx]
  char* halo;      // y-pass strip halo terms [strips][2][2][NC][nx]
  size_t state_bytes;
};

size_t state_bytes(const Geometry& g) { return align_up((size_t)g.nf * g.nc * g.plane * g.esize, 256); }
size_t base_bytes(const Geometry& g) { return align_up((size_t)(g.nf - 1) * g.nc * g.plane * g.esize, 256); }
size_t ghost_x_bytes(const hweno_problem* p, const Geometry& g) {
  return align_up((size_t)p->ny * 4 * 3 * g.nc * g.esize, 256);
}
size_t ghost_y_bytes(const hweno_problem* p, const Geometry& g) {
  return p->dim == 2 ? align_up((size_t)p->nx * 4 * 3 * g.nc * g.esize, 256) : 0;
}
// y-VJP strips have at least kMinStripRows of the ny + 4 virtual rows
constexpr int kMinStripRows = 4;
size_t halo_bytes(const hweno_problem* p, const Geometry& g) {
  if (p->dim != 2) return 0;
  const size_t strips = (size_t)(p->ny + 4 + kMinStripRows - 1) / kMinStripRows;
  return align_up(strips * 4 * g.nc * (size_t)p->nx * g.esize, 256);
}
size_t ghost_bytes(const hweno_problem* p, const Geometry& g) {
  return ghost_x_bytes(p, g) + ghost_y_bytes(p, g) + halo_bytes(p, g);
}
size_t ws_total(const hweno_problem* p, const Geometry& g) {
  return kScalarBytes + kPartialBytes + 4 * state_bytes(g) + base_bytes(g) + ghost_bytes(p, g);
}

// The part of the workspace a forward step uses (ws_layout puts it first):
// scalars, partial maxima, X^(1), X^(2), the RK base derivatives.
size_t ws_step_bytes(const Geometry& g) {
  return kScalarBytes + kPartialBytes + 2 * state_bytes(g) + base_bytes(g);
}

// Device address of `scratch` on the current device, looked up once per
// device (hipGetSymbolAddress with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hweno_status scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HWENO_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HWENO_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HWENO_OK;
}

WsLayout ws_layout(const hweno_problem* p, void* ws, const Geometry& g) {
  WsLayout w;
  char* b = (char*)ws;
  w.sc = (StepScalars*)b;
  w.partial = (double*)(b + kScalarBytes);
  w.state_bytes = state_bytes(g);
  w.x1 = b + kScalarBytes + kPartialBytes;
  w.x2 = w.x1 + w.state_bytes;
  w.base = w.x2 + w.state_bytes;
  w.lam2 = w.base + base_bytes(g);
  w.lam1 = w.lam2 + w.state_bytes;
  w.ghost = w.lam1 + w.state_bytes;
  w.ghost_y = w.ghost + ghost_x_bytes(p, g);
  w.halo = w.ghost_y + ghost_y_bytes(p, g);
  return w;
}

Scheme make_scheme(const hweno_problem* p) {
  Scheme s;
  s.dx = p->dx;
  s.dy = p->dim == 2 ? p->dy : 1.0;
  s.idx = 1.0 / s.dx;
  s.idy = 1.0 / s.dy;
  s.gamma0 = p->gamma0;
  s.g1 = 0.5 * (1.0 - p->gamma0);
  s.d0 = p->d0;
  s.d1 = 0.5 * (1.0 - p->d0);
  s.eps = p->eps;
  s.gas = p->gas_gamma;
  s.adv_a = p->adv_a;
  s.adv_b = p->adv_b;
  return s;
}

inline hweno_status check_launch() {
  return hipGetLastError() == hipSuccess ? HWENO_OK : HWENO_EDEVICE;
}

// Calls f(Sys{}, T{}, DIM) for the problem's system, element type and dimension.
template <class F>
hweno_status dispatch(const hweno_problem* p, F&& f) {
  auto by_type = [&](auto tag) -> hweno_status {
    using T = decltype(tag);
    if (p->dim == 1) {
      switch (p->system) {
        case HWENO_ADVECTION: return f(Advection{p->adv_a, p->adv_b}, T{}, std::integral_constant<int, 1>{});
        case HWENO_BURGERS: return f(Burgers{}, T{}, std::integral_constant<int, 1>{});
        default: return f(Euler<1>{p->gas_gamma}, T{}, std::integral_constant<int, 1>{});
      }
    }
    switch (p->system) {
      case HWENO_ADVECTION: return f(Advection{p->adv_a, p->adv_b}, T{}, std::integral_constant<int, 2>{});
      case HWENO_BURGERS: return f(Burgers{}, T{}, std::integral_constant<int, 2>{});
      default: return f(Euler<2>{p->gas_gamma}, T{}, std::integral_constant<int, 2>{});
    }
  };
  return p->precision == HWENO_F64 ? by_type(double{}) : by_type(float{});
}

// Occupancy of `kernel` (block size BLOCK) on the current device: blocks per
// CU from the occupancy query (cached per kernel instance and TAG) and the CU
// count (asked each time). False if unknown.
template <int TAG, int BLOCK, class K>
bool occupancy(K kernel, int* per_cu, int* cus) {
  static std::atomic<int> per_cu_cache{0};
  int pc = per_cu_cache.load(std::memory_order_relaxed);
  if (pc <= 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kernel, BLOCK, 0) != hipSuccess || pc <= 0)
      return false;
    per_cu_cache.store(pc, std::memory_order_relaxed);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || *cus <= 0)
    return false;
  *per_cu = pc;
  return true;
}

// Strip height R of a one-wavefront-per-block marcher: col_blocks blocks side
// by side, each marching strips of R of `rows` rows. A strip costs R +
// overhead row units (its warm-up rows). With k of its blocks per SIMD a
// round of 4 CUs k blocks takes k (R + overhead) / g(k), g(1) = 1 and g(k>1)
// = 1.1 (the measured gain of a second wavefront on a SIMD in these
// VALU-bound kernels); R minimises the total over rounds. `fallback` if the
// occupancy is unknown.
int balanced_rows(long col_blocks, int rows, bool known, int per_cu, int cus, double overhead,
                  int fallback, int rmin = 1) {
  if (!known) return fallback < rmin ? rmin : fallback;
  const long simds = 4L * cus;
  const long lanes = per_cu >= 4 ? simds : (long)cus * per_cu;   // blocks at one per SIMD
  const long kmax = per_cu >= 4 ? per_cu / 4 : 1;
  int best = rows > rmin ? rows : rmin;
  double best_cost = 1e300;
  for (int r = rmin; r <= rows; ++r) {
    const long blocks = col_blocks * ((rows + r - 1) / r);
    long k = (blocks + lanes - 1) / lanes;
    if (k > kmax) k = kmax;
    const long rounds = (blocks + lanes * k - 1) / (lanes * k);
    const double cost = (double)rounds * k * (r + overhead) / (k > 1 ? 1.1 : 1.0);
    if (cost < best_cost) {
      best_cost = cost;
      best = r;
    }
  }
  return best;
}


template <class Sys, typename T, int DIM>
hweno_status launch_stage(int mode, const StageArgs<T>& A0, const Sys& sy, hipStream_t st) {
  StageArgs<T> A = A0;
  if constexpr (DIM == 1) {
    dim3 grid((A.nx + kXOut - 1) / kXOut);
    auto modes = [&](auto iface) {
      constexpr bool I = decltype(iface)::value;
      switch (mode) {
        case kRhs: stage1d_kernel<Sys, T, kRhs, I><<<grid, kWave, 0, st>>>(A, sy); break;
        case kStage1: stage1d_kernel<Sys, T, kStage1, I><<<grid, kWave, 0, st>>>(A, sy); break;
        case kStage2: stage1d_kernel<Sys, T, kStage2, I><<<grid, kWave, 0, st>>>(A, sy); break;
        default: stage1d_kernel<Sys, T, kStage3, I><<<grid, kWave, 0, st>>>(A, sy); break;
      }
    };
    if constexpr (Sys::kChar) {
      if (A.iface)
        modes(std::true_type{});
      else
        modes(std::false_type{});
    } else {
      modes(std::false_type{});
    }
  } else {
    auto go = [&](auto kernel, auto tag) {
      int per_cu = 0, cus = 0;
      const bool known = occupancy<decltype(tag)::value, kWave>(kernel, &per_cu, &cus);
      // warm-up: two rows of loads and y-pointwise fluxes, two of y-HWENO,
      // about one full row in all
      const int forced = g_strip_rows.load(std::memory_order_relaxed);
      A.rows = forced > 0 ? forced
                          : balanced_rows((A.nx + kXOut - 1) / kXOut, A.ny, known, per_cu, cus, 1.0, 32);
      dim3 grid((A.nx + kXOut - 1) / kXOut, (A.ny + A.rows - 1) / A.rows);
      kernel<<<grid, kWave, 0, st>>>(A, sy);
    };
    auto modes = [&](auto var) {
      constexpr int V = decltype(var)::value;
      constexpr int kT = 16 * V;   // separate occupancy cache entries
      switch (mode) {
        case kRhs: go(stage2d_kernel<Sys, T, kRhs, V>, std::integral_constant<int, kRhs + kT>{}); break;
        case kStage1: go(stage2d_kernel<Sys, T, kStage1, V>, std::integral_constant<int, kStage1 + kT>{}); break;
        case kStage2: go(stage2d_kernel<Sys, T, kStage2, V>, std::integral_constant<int, kStage2 + kT>{}); break;
        default: go(stage2d_kernel<Sys, T, kStage3, V>, std::integral_constant<int, kStage3 + kT>{}); break;
      }
    };
    bool walls = false;
    for (int k = 0; k < 4; ++k)
      walls = walls || A.bc[k] == kBcReflective || A.bc[k] == kBcDirichlet || A.bc[k] == kBcSplit;
    const int var = (walls ? kVarWalls : 0) | (Sys::kChar && A.iface ? kVarIface : 0) |
                    (Sys::kChar && A.gravity != 0.0 ? kVarSource : 0);
    if constexpr (Sys::kChar) {
      switch (var) {
        case 0: modes(std::integral_constant<int, 0>{}); break;
        case 1: modes(std::integral_constant<int, 1>{}); break;
        case 2: modes(std::integral_constant<int, 2>{}); break;
        case 3: modes(std::integral_constant<int, 3>{}); break;
        case 4: modes(std::integral_constant<int, 4>{}); break;
        case 5: modes(std::integral_constant<int, 5>{}); break;
        case 6: modes(std::integral_constant<int, 6>{}); break;
        default: modes(std::integral_constant<int, 7>{}); break;
      }
    } else if (walls) {
      modes(std::integral_constant<int, kVarWalls>{});
    } else {
      modes(std::integral_constant<int, 0>{});
    }
  }
  return check_launch();
}

template <typename T>
StageArgs<T> base_args(const hweno_problem* p) {
  StageArgs<T> A;
  std::memset(&A, 0, sizeof(A));
  A.nx = p->nx;
  A.ny = p->ny;
  A.rows = kRowsPerBlock;
  A.plane = p->nx * p->ny;
  for (int k = 0; k < 4; ++k) A.bc[k] = p->bc[k];
  A.iface = p->char_basis == HWENO_BASIS_INTERFACE;
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 4; ++c) A.gs[k][c] = p->bc_state[k][c];
  A.gravity = p->system == HWENO_EULER && p->dim == 2 ? p->gravity : 0.0;
  for (int k = 0; k < 2; ++k) {
    A.sp[k].x0 = p->split[k].x0;
    A.sp[k].slope = p->split[k].slope;
    A.sp[k].speed = p->split[k].speed;
    for (int j = 0; j < 2; ++j) {
      A.sp[k].kind[j] = p->split[k].kind[j];
      for (int c = 0; c < 4; ++c) A.sp[k].state[j][c] = p->split[k].state[j][c];
    }
  }
  A.t0 = nullptr;
  A.tc = 0.0;
  A.ctl.dim = p->dim;
  A.s = make_scheme(p);
  A.pk = point_k(A.s);
  return A;
}

int partial_blocks(size_t plane) {
  size_t b = (plane + 255) / 256;
  return (int)(b < (size_t)kPartialBlocks ? b : (size_t)kPartialBlocks);
}

template <class Sys, typename T, int DIM>
hweno_status launch_speed_partial(const hweno_problem* p, const T* U, const Sys& sy, double* partial,
                                  unsigned* flags, hipStream_t st, int* nb) {
  const size_t plane = (size_t)p->nx * p->ny;
  *nb = partial_blocks(plane);
  speed_partial_kernel<Sys, T, DIM><<<*nb, 256, 0, st>>>(U, (int)plane, sy, partial, flags);
  return check_launch();
}

// One VJP of a stage: the x-pass writes out[], the 2D y-pass marches up
// column strips and adds to it; each pass then folds its ghost cells.
struct Cot {
  const void* b[3];       // the flux cotangent state (u, v, w; w null in 1D), scaled by cb dt
  double cb;
  const void* a[3][3];    // the a sets (u, v, w each)
  double ca[3];
  int na;                 // 1 or 3
};

template <class Sys, typename T, int DIM>
hweno_status launch_vjp(const hweno_problem* p, const Sys& sy, const Geometry& g,
                        const WsLayout& wl, const T* X[3], const Cot& cot,
                        const double* alpha, const double* dt, T* out[3], hipStream_t st) {
  constexpr int NC = Sys::NC;
  const Scheme sc = make_scheme(p);
  const int nx = p->nx, ny = p->ny, plane = nx * ny;
  // the interface basis changes only the per-cell reverse (three bases)
  const bool iface = Sys::kChar && p->char_basis == HWENO_BASIS_INTERFACE;
  // y-pass (2D): overwrites out; its strip halos and ghost rows are folded
  // in by the x-pass
  int ystrip_rows = 0, ystrips = 0;
  if constexpr (DIM == 2) {
    VjpYArgs<T> A;
    std::memset(&A, 0, sizeof(A));
    for (int f = 0; f < 3; ++f) {
      A.X[f] = X[f];
      A.b[f] = (const T*)cot.b[f];
    }
    for (int k = 0; k < cot.na; ++k) {
      A.aw[k] = (const T*)cot.a[k][2];
      A.ca[k] = cot.ca[k];
    }
    A.na = cot.na;
    A.cb = cot.cb;
    A.dt = dt;
    A.alpha = alpha;
    for (int f = 0; f < 3; ++f) A.G[f] = out[f];
    A.ghost = (T*)wl.ghost_y;
    A.halo = (T*)wl.halo;
    A.nx = nx;
    A.ny = ny;
    A.plane = plane;
    A.bc_lo = p->bc[2];
    A.bc_hi = p->bc[3];
    for (int c = 0; c < 4; ++c) {
      A.gs[0][c] = p->bc_state[2][c];
      A.gs[1][c] = p->bc_state[3][c];
    }
    A.s = sc;
    // strips of at least kMinStripRows rows (the halo buffer is sized for
    // that); warm-up: four rows of loads
    bool walls = false;
    for (int k = 0; k < 4; ++k) walls = walls || p->bc[k] == HWENO_REFLECTIVE || p->bc[k] == HWENO_DIRICHLET;
    int nstrips = 0;
    auto go = [&](auto kernel, auto tag) {
      int per_cu = 0, cus = 0;
      const bool known = occupancy<decltype(tag)::value, kWave>(kernel, &per_cu, &cus);
      A.rows = balanced_rows((nx + kWave - 1) / kWave, ny + 4, known, per_cu, cus, 1.0, 16,
                             kMinStripRows);
      nstrips = (ny + 4 + A.rows - 1) / A.rows;
      dim3 grid((nx + kWave - 1) / kWave, nstrips);
      kernel<<<grid, kWave, 0, st>>>(A, sy);
    };
    if (iface) {
      if constexpr (Sys::kChar) {
        if (walls)
          go(vjp_y_kernel<Sys, T, true, true>, std::integral_constant<int, 20>{});
        else
          go(vjp_y_kernel<Sys, T, false, true>, std::integral_constant<int, 4>{});
      }
    } else if (walls) {
      go(vjp_y_kernel<Sys, T, true>, std::integral_constant<int, 20>{});
    } else {
      go(vjp_y_kernel<Sys, T, false>, std::integral_constant<int, 4>{});
    }
    if (check_launch() != HWENO_OK) return HWENO_EDEVICE;
    ystrip_rows = A.rows;
    ystrips = nstrips;
  }
  // x-pass (in 2D after the y-pass, adding to its result), then the fold
  // of its ghost columns
  {
    VjpArgs<T> A;
    std::memset(&A, 0, sizeof(A));
    for (int f = 0; f < 3; ++f) {
      A.X[f] = X[f];
      A.b[f] = (const T*)cot.b[f];
    }
    for (int k = 0; k < cot.na; ++k) {
      A.a[k][0] = (const T*)cot.a[k][0];
      A.a[k][1] = (const T*)cot.a[k][1];
      A.ca[k] = cot.ca[k];
    }
    A.cb = cot.cb;
    A.dt = dt;
    A.alpha = alpha;
    A.dir = 0;
    A.add_identity = 1;
    A.accumulate = DIM == 2;   // in 2D the y-pass has written out
    if (DIM == 2) {
      A.yhalo = (const T*)wl.halo;
      A.yghost = (const T*)wl.ghost_y;
      A.yR = ystrip_rows;
      A.ystrips = ystrips;
      for (int k = 0; k < 4; ++k) {
        const int q = k < 2 ? k - 2 : ny + k - 2;
        const bool fixed = fixed_side(q, ny, p->bc[2], p->bc[3]) >= 0;
        A.yimg[k] = fixed ? -1 : map_index(q, ny, p->bc[2], p->bc[3]);
        A.yflip[k] = mirrored(q, ny, p->bc[2], p->bc[3]);
        A.yqj[k] = halo_source(q, ystrip_rows, ystrips, A.yqs[k]);
      }
    }
    for (int f = 0; f < 3; ++f) A.G[f] = out[f];
    A.ghost = (T*)wl.ghost;
    A.n = nx;
    A.rows = ny;
    A.plane = plane;
    A.bc_lo = p->bc[0];
    A.bc_hi = p->bc[1];
    for (int c = 0; c < 4; ++c) {
      A.gs[0][c] = p->bc_state[0][c];
      A.gs[1][c] = p->bc_state[1][c];
    }
    A.h = sc.dx;
    A.ih = sc.idx;
    A.s = sc;
    dim3 grid((nx + 4 + kXOut - 1) / kXOut, ny);
    auto special = [](int b) { return b == HWENO_REFLECTIVE || b == HWENO_DIRICHLET; };
    const bool xwalls = special(p->bc[0]) || special(p->bc[1]);
    auto go = [&](auto walls, auto ifc) {
      constexpr bool W = decltype(walls)::value, I = decltype(ifc)::value;
      if (cot.na == 1)
        vjp_row_kernel<Sys, T, 0, DIM + 1, 1, W, I><<<grid, kWave, 0, st>>>(A, sy);
      else
        vjp_row_kernel<Sys, T, 0, DIM + 1, 3, W, I><<<grid, kWave, 0, st>>>(A, sy);
    };
    auto go_w = [&](auto ifc) {
      if (xwalls)
        go(std::true_type{}, ifc);
      else
        go(std::false_type{}, ifc);
    };
    if constexpr (Sys::kChar) {
      if (iface)
        go_w(std::true_type{});
      else
        go_w(std::false_type{});
    } else {
      go_w(std::false_type{});
    }
    if (check_launch() != HWENO_OK) return HWENO_EDEVICE;
    {
      const int tot = ny * g.nf * NC;
      ghost_fold_kernel<T><<<(tot + 255) / 256, 256, 0, st>>>(out[0], out[1], out[2], (const T*)wl.ghost,
                                                             nx, ny, plane, NC, g.nf,
                                                             p->bc[0], p->bc[1]);
      if (check_launch() != HWENO_OK) return HWENO_EDEVICE;
    }
  }
  if constexpr (DIM == 2) {
    if (Sys::kChar && NC == 4 && p->gravity != 0.0) {
      source_vjp_kernel<T><<<(plane + 255) / 256, 256, 0, st>>>(
          out[0], out[1], out[2], (const T*)cot.b[0], (const T*)cot.b[1], (const T*)cot.b[2], cot.cb,
          dt, p->gravity, plane);
      if (check_launch() != HWENO_OK) return HWENO_EDEVICE;
    }
  }
  return HWENO_OK;
}

// Time-stepping loop of hweno_step(s) ((fully-hweno), (2Dfully-hweno)): one
// seeding pass (per-block maxima of the spectral radii of the initial state,
// reduced into the stage-1 alphas), then three stage launches per step. Stage 1 computes the
// step's dt from its alphas, stage 3 reduces the next step's stage-1 alphas
// in its epilogue, so steady-state steps launch the three stage kernels only.
hweno_status run_steps(const hweno_problem* p, void* u, void* v, void* w, int32_t nsteps,
                       int32_t dt_rule, double cfl, double dt_fixed, double t_end, double* t,
                       double* dt_used, double* alpha_rec, void* stages, void* ws,
                       hipStream_t stream, hipEvent_t* events) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!u || !v || !t || !ws || nsteps < 1) return HWENO_EINVAL;
  if (p->dim == 2 && !w) return HWENO_EINVAL;
  if (p->dim == 1 && w) return HWENO_EINVAL;
  if (dt_rule < HWENO_DT_PRODUCTION || dt_rule > HWENO_DT_FIXED) return HWENO_EINVAL;
  if (dt_rule == HWENO_DT_FIXED ? !(dt_fixed > 0.0) : !(cfl > 0.0)) return HWENO_EINVAL;
  if (std::isnan(t_end)) return HWENO_EINVAL;
  if (stages && nsteps != 1) return HWENO_EINVAL;
  const Geometry g = geometry(p);
  WsLayout wl = ws_layout(p, ws, g);
  return dispatch(p, [&](auto sy, auto tag, auto dimc) -> hweno_status {
    using T = decltype(tag);
    using Sys = decltype(sy);
    constexpr int DIM = decltype(dimc)::value;
    const size_t P = g.plane;
    // stage states: the caller's `stages` buffer when given, else the workspace
    char* x1 = stages ? (char*)stages : wl.x1;
    char* x2 = stages ? (char*)stages + (size_t)g.nf * g.nc * P * sizeof(T) : wl.x2;
    T* Vt = (T*)wl.base;
    T* Wt = DIM == 2 ? Vt + (size_t)g.nc * P : nullptr;
    auto F = [&](char* b, int f) { return (T*)(b + (size_t)f * g.nc * P * sizeof(T)); };
    int nb;
    hweno_status s2 = launch_speed_partial<Sys, T, DIM>(p, (const T*)u, sy, wl.partial,
                                                        &wl.sc->flags, stream, &nb);
    if (s2 != HWENO_OK) return s2;
    alpha_seed_kernel<<<1, 256, 0, stream>>>(wl.partial, nb, wl.sc);
    if ((s2 = check_launch()) != HWENO_OK) return s2;
    StageArgs<T> A = base_args<T>(p);
    A.dt = &wl.sc->dt;
    A.active = &wl.sc->active;
    A.flags = &wl.sc->flags;
    A.t0 = &wl.sc->t0;            // stage times t0, t0 + dt, t0 + dt/2
    A.ctl.sc = wl.sc;
    A.ctl.t = t;
    A.ctl.rule = dt_rule;
    A.ctl.cfl = cfl;
    A.ctl.dt_fixed = dt_fixed;
    A.ctl.t_end = t_end;
    if (dt_rule == HWENO_DT_ACCURACY) {
      A.ctl.hx = std::pow(p->dx, 5.0 / 3.0);
      A.ctl.hy = DIM == 2 ? std::pow(p->dy, 5.0 / 3.0) : 1.0;
    } else {
      A.ctl.hx = p->dx;
      A.ctl.hy = DIM == 2 ? p->dy : 1.0;
    }
    for (int k = 0; k < nsteps; ++k) {
      hipEvent_t* ev = events ? events + 4 * k : nullptr;
      auto mark = [&](int j) -> bool { return !ev || hipEventRecord(ev[j], stream) == hipSuccess; };
      double* rec = alpha_rec ? alpha_rec + 6 * k : nullptr;
      A.ctl.dt_used = dt_used ? dt_used + k : nullptr;
      // stage 1: X^n -> X^(1), V~^n, W~^n; computes dt
      if (!mark(0)) return HWENO_EDEVICE;
      A.U = (const T*)u; A.V = (const T*)v; A.W = (const T*)w;
      A.Ub = nullptr; A.Vb = nullptr; A.Wb = nullptr;
      A.Uo = F(x1, 0); A.Vo = F(x1, 1); A.Wo = DIM == 2 ? F(x1, 2) : nullptr;
      A.Vt = Vt; A.Wt = Wt;
      A.alpha = (const double*)&wl.sc->acc[4];
      A.alpha_next = &wl.sc->acc[0];
      A.alpha_rec = rec;
      A.tc = 0.0;
      if ((s2 = launch_stage<Sys, T, DIM>(kStage1, A, sy, stream)) != HWENO_OK) return s2;
      if (!mark(1)) return HWENO_EDEVICE;
      // stage 2: X^(1) -> X^(2) with base (U^n, V~^n, W~^n)
      A.U = F(x1, 0); A.V = F(x1, 1); A.W = DIM == 2 ? F(x1, 2) : nullptr;
      A.Ub = (const T*)u; A.Vb = Vt; A.Wb = Wt;
      A.Uo = F(x2, 0); A.Vo = F(x2, 1); A.Wo = DIM == 2 ? F(x2, 2) : nullptr;
      A.Vt = nullptr; A.Wt = nullptr;
      A.alpha = (const double*)&wl.sc->acc[0];
      A.alpha_next = &wl.sc->acc[2];
      A.alpha_rec = rec ? rec + 2 : nullptr;
      A.tc = 1.0;
      if ((s2 = launch_stage<Sys, T, DIM>(kStage2, A, sy, stream)) != HWENO_OK) return s2;
      if (!mark(2)) return HWENO_EDEVICE;
      // stage 3: X^(2) -> X^{n+1}, in place on (u, v, w); the result's alphas
      // are the next step's stage-1 alphas
      A.U = F(x2, 0); A.V = F(x2, 1); A.W = DIM == 2 ? F(x2, 2) : nullptr;
      A.Uo = (T*)u; A.Vo = (T*)v; A.Wo = (T*)w;
      A.alpha = (const double*)&wl.sc->acc[2];
      A.alpha_next = &wl.sc->acc[4];
      A.alpha_rec = rec ? rec + 4 : nullptr;
      A.tc = 0.5;
      if ((s2 = launch_stage<Sys, T, DIM>(kStage3, A, sy, stream)) != HWENO_OK) return s2;
      if (!mark(3)) return HWENO_EDEVICE;
    }
    return HWENO_OK;
  });
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* hweno_status_string(hweno_status s) {
  switch (s) {
    case HWENO_OK: return "ok";
    case HWENO_EINVAL: return "invalid argument";
    case HWENO_EUNSUPPORTED: return "unsupported";
    case HWENO_EDEVICE: return "HIP runtime error";
    case HWENO_ENONFINITE: return "non-finite state";
    case HWENO_ENONPHYSICAL: return "non-physical state (density or pressure <= 0)";
    case HWENO_ESCRATCH: return "problem exceeds the static scratch of hweno_step_noalloc";
  }
  return "unknown status";
}

hweno_status hweno_workspace_bytes(const hweno_problem* p, size_t* bytes) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!bytes) return HWENO_EINVAL;
  const Geometry g = geometry(p);
  *bytes = ws_total(p, g);
  return HWENO_OK;
}

hweno_status hweno_workspace_init(const hweno_problem* p, void* ws, hipStream_t stream) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!ws) return HWENO_EINVAL;
  ws_init_kernel<<<1, 1, 0, stream>>>((StepScalars*)ws);
  return check_launch();
}

hweno_status hweno_max_wavespeed(const hweno_problem* p, const void* u, double* alpha, void* ws,
                                 hipStream_t stream) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!u || !alpha || !ws) return HWENO_EINVAL;
  const Geometry g = geometry(p);
  WsLayout w = ws_layout(p, ws, g);
  return dispatch(p, [&](auto sy, auto tag, auto dimc) -> hweno_status {
    using T = decltype(tag);
    using Sys = decltype(sy);
    constexpr int DIM = decltype(dimc)::value;
    int nb;
    hweno_status s2 = launch_speed_partial<Sys, T, DIM>(p, (const T*)u, sy, w.partial,
                                                        &w.sc->flags, stream, &nb);
    if (s2 != HWENO_OK) return s2;
    alpha_out_kernel<<<1, 256, 0, stream>>>(w.partial, nb, alpha);
    return check_launch();
  });
}

hweno_status hweno_rhs(const hweno_problem* p, const void* u, const void* v, const void* w,
                       const double* alpha, void* Lu, void* Lv, void* Lw, void* vtilde,
                       void* wtilde, void* ws, hipStream_t stream) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!u || !v || !alpha || !Lu || !Lv || !vtilde || !ws) return HWENO_EINVAL;
  if (p->dim == 2 && (!w || !Lw || !wtilde)) return HWENO_EINVAL;
  if (p->dim == 1 && (w || Lw || wtilde)) return HWENO_EINVAL;
  const void* ins[3] = {u, v, w};
  void* outs[5] = {Lu, Lv, Lw, vtilde, wtilde};
  for (auto o : outs)
    for (auto i : ins)
      if (o && i && o == i) return HWENO_EINVAL;
  return dispatch(p, [&](auto sy, auto tag, auto dimc) -> hweno_status {
    using T = decltype(tag);
    using Sys = decltype(sy);
    constexpr int DIM = decltype(dimc)::value;
    StageArgs<T> A = base_args<T>(p);
    A.U = (const T*)u; A.V = (const T*)v; A.W = (const T*)w;
    A.Uo = (T*)Lu; A.Vo = (T*)Lv; A.Wo = (T*)Lw;
    A.Vt = (T*)vtilde; A.Wt = (T*)wtilde;
    A.alpha = alpha;
    return launch_stage<Sys, T, DIM>(kRhs, A, sy, stream);
  });
}

hweno_status hweno_step(const hweno_problem* p, void* u, void* v, void* w, int32_t dt_rule,
                        double cfl, double dt_fixed, double t_end, double* t, double* dt_used,
                        double* alpha_rec, void* stages, void* ws, hipStream_t stream) {
  return run_steps(p, u, v, w, 1, dt_rule, cfl, dt_fixed, t_end, t, dt_used, alpha_rec, stages, ws,
                   stream, nullptr);
}

hweno_status hweno_step_profiled(const hweno_problem* p, void* u, void* v, void* w,
                                 int32_t dt_rule, double cfl, double dt_fixed, double t_end,
                                 double* t, double* dt_used, double* alpha_rec, void* stages,
                                 void* ws, hipStream_t stream, hipEvent_t* events) {
  return run_steps(p, u, v, w, 1, dt_rule, cfl, dt_fixed, t_end, t, dt_used, alpha_rec, stages, ws,
                   stream, events);
}

hweno_status hweno_steps(const hweno_problem* p, void* u, void* v, void* w, int32_t nsteps,
                         int32_t dt_rule, double cfl, double dt_fixed, double t_end, double* t,
                         double* dt_used, double* alpha_rec, void* ws, hipStream_t stream,
                         hipEvent_t* events) {
  return run_steps(p, u, v, w, nsteps, dt_rule, cfl, dt_fixed, t_end, t, dt_used, alpha_rec,
                   nullptr, ws, stream, events);
}

hweno_status hweno_step_noalloc(const hweno_problem* p, void* u, void* v, void* w,
                                int32_t dt_rule, double cfl, double dt_fixed, double t_end,
                                double* t, double* dt_used, double* alpha_rec,
                                hipStream_t stream) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (ws_step_bytes(geometry(p)) > kScratchBytes) return HWENO_ESCRATCH;
  if (!u || !v || !t) return HWENO_EINVAL;
  void* ws = nullptr;
  if ((st = scratch_on_current_device(&ws)) != HWENO_OK) return st;
  // the scratch keeps the previous call's contents: clear the step scalars
  // (alpha accumulators, flags) with a kernel, before the step's launches
  ws_init_kernel<<<1, 1, 0, stream>>>((StepScalars*)ws);
  if ((st = check_launch()) != HWENO_OK) return st;
  return run_steps(p, u, v, w, 1, dt_rule, cfl, dt_fixed, t_end, t, dt_used, alpha_rec, nullptr,
                   ws, stream, nullptr);
}

hweno_status hweno_set_strip_rows(int32_t rows) {
  if (rows < 0) return HWENO_EINVAL;
  g_strip_rows.store(rows, std::memory_order_relaxed);
  return HWENO_OK;
}

hweno_status hweno_step_frozen(const hweno_problem* p, void* u, void* v, void* w, void* u_out,
                               void* v_out, void* w_out, const double* dt, const double* alpha_rec,
                               void* stages, void* ws, hipStream_t stream) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!u || !v || !dt || !alpha_rec || !ws) return HWENO_EINVAL;
  if (p->dim == 2 && !w) return HWENO_EINVAL;
  if (p->dim == 1 && w) return HWENO_EINVAL;
  if (has_split(p)) return HWENO_EUNSUPPORTED;   // no step time here
  if (u_out) {
    if (!v_out || (p->dim == 2) != (w_out != nullptr)) return HWENO_EINVAL;
    const void* ins[4] = {u, v, w, stages};
    for (const void* o : {(const void*)u_out, (const void*)v_out, (const void*)w_out})
      for (const void* i : ins)
        if (o && i && o == i) return HWENO_EINVAL;
  } else if (v_out || w_out) {
    return HWENO_EINVAL;
  }
  const Geometry g = geometry(p);
  WsLayout wl = ws_layout(p, ws, g);
  return dispatch(p, [&](auto sy, auto tag, auto dimc) -> hweno_status {
    using T = decltype(tag);
    using Sys = decltype(sy);
    constexpr int DIM = decltype(dimc)::value;
    const size_t fs = (size_t)g.nc * g.plane;
    char* x1 = stages ? (char*)stages : wl.x1;
    char* x2 = stages ? (char*)stages + (size_t)g.nf * fs * sizeof(T) : wl.x2;
    auto F = [&](char* b, int f) { return (T*)(b + (size_t)f * fs * sizeof(T)); };
    T* Vt = (T*)wl.base;
    T* Wt = DIM == 2 ? Vt + fs : nullptr;
    StageArgs<T> A = base_args<T>(p);
    A.dt = dt;
    hweno_status s2;
    A.U = (const T*)u; A.V = (const T*)v; A.W = (const T*)w;
    A.Uo = F(x1, 0); A.Vo = F(x1, 1); A.Wo = DIM == 2 ? F(x1, 2) : nullptr;
    A.Vt = Vt; A.Wt = Wt;
    A.alpha = alpha_rec;
    if ((s2 = launch_stage<Sys, T, DIM>(kStage1, A, sy, stream)) != HWENO_OK) return s2;
    A.U = F(x1, 0); A.V = F(x1, 1); A.W = DIM == 2 ? F(x1, 2) : nullptr;
    A.Ub = (const T*)u; A.Vb = Vt; A.Wb = Wt;
    A.Uo = F(x2, 0); A.Vo = F(x2, 1); A.Wo = DIM == 2 ? F(x2, 2) : nullptr;
    A.Vt = nullptr; A.Wt = nullptr;
    A.alpha = alpha_rec + 2;
    if ((s2 = launch_stage<Sys, T, DIM>(kStage2, A, sy, stream)) != HWENO_OK) return s2;
    A.U = F(x2, 0); A.V = F(x2, 1); A.W = DIM == 2 ? F(x2, 2) : nullptr;
    if (u_out) {
      A.Uo = (T*)u_out; A.Vo = (T*)v_out; A.Wo = (T*)w_out;
    } else {
      A.Uo = (T*)u; A.Vo = (T*)v; A.Wo = (T*)w;
    }
    A.alpha = alpha_rec + 4;
    return launch_stage<Sys, T, DIM>(kStage3, A, sy, stream);
  });
}

hweno_status hweno_adjoint_step(const hweno_problem* p, const void* u_n, const void* v_n,
                                const void* w_n, const void* stages, const double* dt,
                                const double* alpha_rec, const void* lam_u_in,
                                const void* lam_v_in, const void* lam_w_in, void* lam_u_out,
                                void* lam_v_out, void* lam_w_out, void* ws, hipStream_t stream) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  const bool two = p->dim == 2;
  if (!u_n || !v_n || !dt || !alpha_rec || !lam_u_in || !lam_v_in || !lam_u_out || !lam_v_out || !ws)
    return HWENO_EINVAL;
  if (has_split(p)) return HWENO_EUNSUPPORTED;
  if (two && (!w_n || !lam_w_in || !lam_w_out)) return HWENO_EINVAL;
  if (!two && (w_n || lam_w_in || lam_w_out)) return HWENO_EINVAL;
  const void* ins[8] = {u_n, v_n, w_n, stages, lam_u_in, lam_v_in, lam_w_in, nullptr};
  void* outs[3] = {lam_u_out, lam_v_out, lam_w_out};
  for (auto o : outs)
    for (auto i : ins)
      if (o && i && o == i) return HWENO_EINVAL;
  const Geometry g = geometry(p);
  WsLayout wl = ws_layout(p, ws, g);
  return dispatch(p, [&](auto sy, auto tag, auto dimc) -> hweno_status {
    using T = decltype(tag);
    using Sys = decltype(sy);
    constexpr int DIM = decltype(dimc)::value;
    const size_t P = g.plane;
    const size_t fs = (size_t)g.nc * P;        // elements per field
    char* x1 = stages ? (char*)stages : wl.x1;
    char* x2 = stages ? (char*)stages + (size_t)g.nf * fs * sizeof(T) : wl.x2;
    auto F = [&](char* b, int f) { return (T*)(b + (size_t)f * fs * sizeof(T)); };
    hweno_status s2;
    if (!stages) {
      // recompute X^(1), X^(2) with the recorded alphas and dt
      T* Vt = (T*)wl.base;
      T* Wt = DIM == 2 ? Vt + fs : nullptr;
      StageArgs<T> A = base_args<T>(p);
      A.dt = dt;
      A.U = (const T*)u_n; A.V = (const T*)v_n; A.W = (const T*)w_n;
      A.Uo = F(x1, 0); A.Vo = F(x1, 1); A.Wo = DIM == 2 ? F(x1, 2) : nullptr;
      A.Vt = Vt; A.Wt = Wt;
      A.alpha = alpha_rec;
      if ((s2 = launch_stage<Sys, T, DIM>(kStage1, A, sy, stream)) != HWENO_OK) return s2;
      A.U = F(x1, 0); A.V = F(x1, 1); A.W = DIM == 2 ? F(x1, 2) : nullptr;
      A.Ub = (const T*)u_n; A.Vb = Vt; A.Wb = Wt;
      A.Uo = F(x2, 0); A.Vo = F(x2, 1); A.Wo = DIM == 2 ? F(x2, 2) : nullptr;
      A.Vt = nullptr; A.Wt = nullptr;
      A.alpha = alpha_rec + 2;
      if ((s2 = launch_stage<Sys, T, DIM>(kStage2, A, sy, stream)) != HWENO_OK) return s2;
    }
    T* l2[3] = {F(wl.lam2, 0), F(wl.lam2, 1), DIM == 2 ? F(wl.lam2, 2) : nullptr};
    T* l1[3] = {F(wl.lam1, 0), F(wl.lam1, 1), DIM == 2 ? F(wl.lam1, 2) : nullptr};
    T* lo[3] = {(T*)lam_u_out, (T*)lam_v_out, (T*)lam_w_out};
    const T* X2[3] = {F(x2, 0), F(x2, 1), DIM == 2 ? F(x2, 2) : nullptr};
    const T* X1[3] = {F(x1, 0), F(x1, 1), DIM == 2 ? F(x1, 2) : nullptr};
    const T* X0[3] = {(const T*)u_n, (const T*)v_n, (const T*)w_n};
    // lambda^(2) = vjp(X^(2); 2/3 lambda, 2/3 dt lambda)
    const void* lin[3] = {lam_u_in, lam_v_in, lam_w_in};
    Cot c3{};
    for (int f = 0; f < 3; ++f) c3.b[f] = c3.a[0][f] = lin[f];
    c3.cb = 2.0 / 3.0;
    c3.ca[0] = 2.0 / 3.0;
    c3.na = 1;
    if ((s2 = launch_vjp<Sys, T, DIM>(p, sy, g, wl, X2, c3, alpha_rec + 4, dt, l2, stream)) != HWENO_OK)
      return s2;
    // lambda^(1) = vjp(X^(1); 1/4 lambda^(2), 1/4 dt lambda^(2))
    Cot c2{};
    for (int f = 0; f < 3; ++f) c2.b[f] = c2.a[0][f] = l2[f];
    c2.cb = 0.25;
    c2.ca[0] = 0.25;
    c2.na = 1;
    if ((s2 = launch_vjp<Sys, T, DIM>(p, sy, g, wl, X1, c2, alpha_rec + 2, dt, l1, stream)) != HWENO_OK)
      return s2;
    // lambda^n = vjp(X^n; lambda^(1) + 3/4 lambda^(2) + 1/3 lambda, dt lambda^(1))
    Cot c1{};
    for (int f = 0; f < 3; ++f) {
      c1.b[f] = c1.a[0][f] = l1[f];
      c1.a[1][f] = l2[f];
      c1.a[2][f] = lin[f];
    }
    c1.cb = 1.0;
    c1.ca[0] = 1.0;
    c1.ca[1] = 0.75;
    c1.ca[2] = 1.0 / 3.0;
    c1.na = 3;
    return launch_vjp<Sys, T, DIM>(p, sy, g, wl, X0, c1, alpha_rec, dt, lo, stream);
  });
}

hweno_status hweno_health(const hweno_problem* p, void* ws, hipStream_t stream, int32_t clear) {
  hweno_status st = validate(p);
  if (st != HWENO_OK) return st;
  if (!ws) return HWENO_EINVAL;
  unsigned flags = 0;
  StepScalars* sc = (StepScalars*)ws;
  if (hipMemcpyAsync(&flags, &sc->flags, sizeof(unsigned), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return HWENO_EDEVICE;
  if (hipStreamSynchronize(stream) != hipSuccess) return HWENO_EDEVICE;
  if (clear) {
    ws_init_kernel<<<1, 1, 0, stream>>>(sc);
    if (check_launch() != HWENO_OK) return HWENO_EDEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return HWENO_EDEVICE;
  }
  if (flags & 1u) return HWENO_ENONFINITE;
  if (flags & 2u) return HWENO_ENONPHYSICAL;
  return HWENO_OK;
}

}  // extern "C"
