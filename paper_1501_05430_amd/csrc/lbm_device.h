// Device helpers shared by the step kernel file (lbm_kernels.hip) and the adjoint file (lbm_adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "lbm_internal.h"

namespace lbm {
namespace {

__device__ constexpr int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

constexpr int WAVE = 64;
constexpr int BLOCK = 256;  // block size of the auxiliary kernels

template <class S>
struct ComputeOf;
template <>
struct ComputeOf<double> { typedef double type; };
template <>
struct ComputeOf<float> { typedef float type; };

// Global-address-space views: loads and stores address an SGPR base plus a 32-bit lane offset.
template <class S>
struct Gbl;
template <>
struct Gbl<float> { typedef __attribute__((address_space(1))) float T; };
template <>
struct Gbl<double> { typedef __attribute__((address_space(1))) double T; };
typedef __attribute__((address_space(1))) const double GCD;

__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline int wrapx(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// Fused multiply-add a * b + c, rounded once. The step's arithmetic is written with these where it fuses and with
// contraction off elsewhere, so that every kernel inlining it rounds identically, whatever the surrounding code
// would let the compiler fuse (the one-step and two-step kernels must agree bit for bit).
__device__ inline float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------------------------------------------------ EOS / psi
// p(rho) of the instance's EOS and psi = sqrt(2 (p - rho/3) / G) (Eq. 10 with c = 1); the argument is clamped at
// 0 (counted) where it is negative. The EOS is Carnahan-Starling or the piecewise-linear one of Eq. 11; the choice
// is per instance, so uniform over a block.

// Eq. 11: the segment is chosen by rho <= rho_1, rho <= rho_2, else the liquid branch.
template <class T>
__device__ inline T pw_pressure(const InstDesc& d, T rho) {
  if (rho <= (T)d.pw_r1) return rho * (T)d.pw_t[0];
  if (rho <= (T)d.pw_r2) return fmac(rho - (T)d.pw_r1, (T)d.pw_t[1], (T)d.pw_p1);
  return fmac(rho - (T)d.pw_r2, (T)d.pw_t[2], (T)d.pw_p2);
}

// FP64 mode: IEEE division and square root.
__device__ inline double psi_f64(const InstDesc& d, double rho, bool& clamped) {
  double p;
  if (d.eos_kind == 1) {
    p = pw_pressure(d, rho);
  } else {
    const double eta = d.eos_b4 * rho;
    const double om = 1.0 - eta;
    p = rho * d.RT * (1.0 + eta + eta * eta - eta * eta * eta) / (om * om * om) - d.eos_a * rho * rho;
  }
  double arg = d.two_over_Gpsi * (p - rho * (1.0 / 3.0));
  clamped = arg < 0.0;
  if (clamped) arg = 0.0;
  return sqrt(arg);
}

// Hardware reciprocal / reciprocal square root refined by Newton steps (about 1 ulp of FP64): used where the
// result is rounded to FP32 afterwards.
__device__ inline double rcp64(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  return r;
}
__device__ inline double sqrt64(double x) {
  if (!(x > 0.0)) return 0.0;
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  return fma(fma(-s, s, x), h, s);
}

// For results rounded to FP32: the hardware reciprocal / reciprocal square root (relative error below about 2^-23)
// refined by one Newton / Goldschmidt step, about 2^-46: far inside FP32's half unit, two steps fewer than above.
__device__ inline double rcp64_for_f32(double b) {
  const double r = __builtin_amdgcn_rcp(b);
  return fma(fma(-b, r, 1.0), r, r);
}
__device__ inline double sqrt64_for_f32(double x) {
  if (!(x > 0.0)) return 0.0;
  const double y = __builtin_amdgcn_rsq(x);
  const double s = x * y, h = 0.5 * y;
  return fma(s, fma(-s, h, 0.5), s);
}

// psi of an FP32 density from the FP64 EOS, rounded to FP32. FULL: reciprocal and square root refined to about
// 1 ulp of FP64 (the mixed form, whose long-run accuracy spends that margin); otherwise once (the FP32 form).
template <bool FULL>
__device__ inline float psi_f32_via64(const InstDesc& d, float rho, bool& clamped) {
#pragma clang fp contract(off)
  const double r = (double)rho;
  double p;
  if (d.eos_kind == 1) {
    p = pw_pressure(d, r);
  } else {
    // Carnahan-Starling: 1 + e + e^2 - e^3 = 1 + e (1 + e (1 - e))
    const double eta = d.eos_b4 * r;
    const double om = 1.0 - eta;
    const double poly = fmac(eta, fmac(eta, 1.0 - eta, 1.0), 1.0);
    p = fmac(r * d.RT * poly, FULL ? rcp64(om * om * om) : rcp64_for_f32(om * om * om), -(d.eos_a * r) * r);
  }
  const double arg = d.two_over_Gpsi * fmac(r, -1.0 / 3.0, p);
  clamped = arg < 0.0;
  return (float)(FULL ? sqrt64(arg) : sqrt64_for_f32(arg));
}

// FP32 modes: below rho_fp64_below the EOS is evaluated in FP64 (vapour side of a large density ratio),
// elsewhere in FP32 with the hardware reciprocal and square root.
__device__ inline float psi_f32(const InstDesc& d, float rho, bool& clamped) {
#pragma clang fp contract(off)
  const bool pw = d.eos_kind == 1;
  if (rho < (float)d.rho_fp64_below) return psi_f32_via64<false>(d, rho, clamped);
  float p;
  if (pw) {
    p = pw_pressure(d, rho);
  } else {
    const float eta = (float)d.eos_b4 * rho;
    const float om = 1.0f - eta;
    const float poly = fmac(eta, fmac(eta, 1.0f - eta, 1.0f), 1.0f);
    p = fmac(rho * (float)d.RT * poly, __builtin_amdgcn_rcpf(om * om * om), -((float)d.eos_a * rho) * rho);
  }
  float arg = (float)d.two_over_Gpsi * fmac(rho, -1.0f / 3.0f, p);
  clamped = arg < 0.0f;
  if (clamped) arg = 0.0f;
  return __builtin_amdgcn_sqrtf(arg);
}

__device__ inline double psi_eval(const InstDesc& d, double rho, bool& cl) { return psi_f64(d, rho, cl); }
__device__ inline float psi_eval(const InstDesc& d, float rho, bool& cl) { return psi_f32(d, rho, cl); }

// Density and momentum as sums of opposite pairs: the rounded results are then exactly symmetric under the
// mirrors x -> -x and y -> -y, as in exact arithmetic, since IEEE addition is commutative and a - b = -(b - a). A
// left-to-right sum rounds differently at mirrored nodes and, step after step, pushes a symmetric droplet
// sideways along its neutral translation mode. (The two diagonal pairs are joined before they meet the rest.)
template <class C>
__device__ inline C sum9(const C (&f)[9]) {
  return ((f[0] + (f[1] + f[3])) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8]));
}
template <class C>
__device__ inline C mom_x(const C (&f)[9]) {
  return (f[1] - f[3]) + ((f[5] - f[7]) + (f[8] - f[6]));
}
template <class C>
__device__ inline C mom_y(const C (&f)[9]) {
  return (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
}

// Interaction force of Eq. 9 (plus the body force) from psi of the centre (pc), its row neighbours (L, R) and the
// rows below (m) and above (n), in the arithmetic type T. Evaluated without fused multiply-adds and with
// psi_R^2 - psi_L^2 = (psi_R - psi_L)(psi_R + psi_L), so the rounded force is exactly odd under x -> -x and
// y -> -y, as the exact one is (a fused a*a - b*b is not the negative of b*b - a*a).
template <class T>
__device__ inline void hybrid_force(const InstDesc& d, T pc, T pcL, T pcR, T pm, T pmL, T pmR, T pn, T pnL, T pnR,
                                    T& Fx, T& Fy) {
#pragma clang fp contract(off)
  const T k1 = (T)(1.0 / 3.0), k2 = (T)(1.0 / 12.0), A = (T)d.A, Gf = (T)d.G_f;
  const T spx = k1 * (pcR - pcL) + k2 * ((pnR - pnL) + (pmR - pmL));
  const T spy = k1 * (pn - pm) + k2 * ((pnR + pnL) - (pmR + pmL));
  const T sux = k1 * ((pcR - pcL) * (pcR + pcL)) + k2 * ((pnR - pnL) * (pnR + pnL) + (pmR - pmL) * (pmR + pmL));
  const T suy = k1 * ((pn - pm) * (pn + pm)) + k2 * ((pnR * pnR + pnL * pnL) - (pmR * pmR + pmL * pmL));
  Fx = -Gf * ((T)0.5 * A * sux + ((T)1 - A) * pc * spx) + (T)d.body_fx;
  Fy = -Gf * ((T)0.5 * A * suy + ((T)1 - A) * pc * spy) + (T)d.body_fy;
}

// psi of the FP32 storage modes: LBM_F32 / LBM_F32_SHIFTED evaluate the EOS in FP32 (in FP64 below
// rho_fp64_below); LBM_F32_SHIFTED_MIXED (MIX) always in FP64, rounded to FP32.
template <bool MIX, class C>
__device__ inline C node_psi(const InstDesc& d, C rho, bool& cl) {
  if constexpr (MIX) return psi_f32_via64<true>(d, rho, cl);
  else return psi_eval(d, rho, cl);
}

// The rounding is spelled out: no contraction, and the fused multiply-adds written where they are wanted, so that
// every kernel inlining this (one step or two steps per launch, any arithmetic) rounds identically, whatever the
// surrounding code would let the compiler fuse. Each fused form is even or odd under the mirrors as its exact value
// is. C is the type of the populations and of the sums over them (momentum, and the rest population's mass
// balance); A the type of everything between: velocity, equilibrium and forcing (A = C except in
// LBM_F32_SHIFTED_MIXED, where A is double for FP32 populations).
template <class C, class A, bool TAU1>
__device__ inline void collide(const C (&f)[9], A rho, A delta, A Fx, A Fy, A inv_tau, A pref, A irho, C (&fs)[9]) {
#pragma clang fp contract(off)
  const A w1 = (A)(1.0 / 9.0), w2 = (A)(1.0 / 36.0);
  const A jx = (A)mom_x(f), jy = (A)mom_y(f);
  const A vx = fmac((A)0.5, Fx, jx) * irho;
  const A vy = fmac((A)0.5, Fy, jy) * irho;
  const A vF = fmac(vx, Fx, vy * Fy);
  const A eq0 = fmac((A)-1.5 * rho, fmac(vx, vx, vy * vy), delta);  // zeroth + second-order isotropic part of f_eq
  const A fo0 = -(A)3 * pref * vF;                                  // isotropic part of the forcing
  const A r45 = (A)4.5 * rho, r3 = (A)3 * rho, p9 = (A)9 * pref, p3 = (A)3 * pref;
  auto put = [&](int i, int o, A w, A eu, A eF) {
    const A se = fmac(r45 * eu, eu, eq0);      // even part of f_eq / w
    const A sf = fmac(p9 * eu, eF, fo0);       // even part of the forcing / w
    if (TAU1) {
      const A odd = fmac(r3, eu, p3 * eF);     // odd parts of f_eq and the forcing / w
      fs[i] = (C)(w * ((se + sf) + odd));
      fs[o] = (C)(w * ((se + sf) - odd));
    } else {
      const A ae = r3 * eu, af = p3 * eF;      // odd parts
      const A fi = (A)f[i], fo = (A)f[o];
      fs[i] = (C)(fmac(w * (se + ae) - fi, inv_tau, fi) + w * (sf + af));
      fs[o] = (C)(fmac(w * (se - ae) - fo, inv_tau, fo) + w * (sf - af));
    }
  };
  put(1, 3, w1, vx, Fx);
  put(2, 4, w1, vy, Fy);
  put(5, 7, w2, vx + vy, Fx + Fy);
  put(6, 8, w2, vy - vx, Fy - Fx);
  // the differences see the rounded f*_i that are stored
  const C d13 = (f[1] - fs[1]) + (f[3] - fs[3]), d24 = (f[2] - fs[2]) + (f[4] - fs[4]);
  const C d57 = (f[5] - fs[5]) + (f[7] - fs[7]), d68 = (f[6] - fs[6]) + (f[8] - fs[8]);
  fs[0] = f[0] + ((d13 + d24) + (d57 + d68));
}

// MRT collision of Eq. 15 with Lambda = diag(0, s_e, s_eps, 1, s_q, 1, s_q, 1/tau, 1/tau) (Eq. 2), the forcing
// (I - Lambda/2) S of Eq. 5-6 (last entry of S: v_x F_y + v_y F_x) and the surface-tension source C of Eq. 16
// (Q_3 = 0; the eighth entry -(1/tau)(Q_xx - Q_yy), the ninth's factor). Moments in the order of Eq. 4 (rho, e,
// eps, j_x, q_x, j_y, q_y, p_xx, p_xy). The change of every moment, dm_k = -s_k (m_k - m_eq,k) + (1 - s_k/2) S_k
// + C_k, is mapped back with M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) and added to f; the
// momentum moments change by exactly F (v = (j + F/2)/rho). With storage shifted by w_i rho0 the equilibrium
// moments of the stored populations are those of rho minus rho0 (1, -2, 1, 0, ...), i.e. delta = rho - rho0 in
// the zeroth-order parts. Opposite pairs and the moments are formed so that the rounded result is exactly
// mirror-symmetric (see sum9), and f*_0 comes from mass conservation as in collide().
template <class C>
__device__ inline void collide_mrt(const C (&f)[9], C rho, C delta, C Fx, C Fy, C irho, C s_e, C s_eps, C s_q,
                                   C s_nu, C qxx, C qyy, C qxy, C (&fs)[9]) {
#pragma clang fp contract(off)
  const C dx = (f[5] - f[7]) + (f[8] - f[6]), dy = (f[5] - f[7]) + (f[6] - f[8]);  // diagonal parts of j
  const C ax = f[1] - f[3], ay = f[2] - f[4];
  const C jx = ax + dx, jy = ay + dy;
  const C s13 = f[1] + f[3], s24 = f[2] + f[4];
  const C sax = s13 + s24, sdg = (f[5] + f[7]) + (f[6] + f[8]);
  const C m_e = (sdg + sdg) - (sax + (C)4 * f[0]);
  const C m_eps = ((C)4 * f[0] + sdg) - (sax + sax);
  const C m_qx = dx - (ax + ax), m_qy = dy - (ay + ay);
  const C m_pxx = s13 - s24, m_pxy = (f[5] + f[7]) - (f[6] + f[8]);
  const C vx = (jx + (C)0.5 * Fx) * irho, vy = (jy + (C)0.5 * Fy) * irho;
  const C rv2 = (C)3 * rho * (vx * vx + vy * vy);
  const C vF = vx * Fx + vy * Fy;
  const C ce = (C)1.5 * s_e * (qxx + qyy);
  const C de = -s_e * (m_e - (rv2 - (delta + delta))) + ((C)1 - (C)0.5 * s_e) * ((C)6 * vF) + ce;
  const C deps = -s_eps * (m_eps - (delta - rv2)) - ((C)1 - (C)0.5 * s_eps) * ((C)6 * vF);
  const C hq = (C)1 - (C)0.5 * s_q, hn = (C)1 - (C)0.5 * s_nu;
  const C dqx = -s_q * (m_qx + rho * vx) - hq * Fx;
  const C dqy = -s_q * (m_qy + rho * vy) - hq * Fy;
  const C dpxx = -s_nu * (m_pxx - rho * (vx * vx - vy * vy)) + hn * ((C)2 * (vx * Fx - vy * Fy)) - s_nu * (qxx - qyy);
  const C dpxy = -s_nu * (m_pxy - rho * (vx * vy)) + hn * (vx * Fy + vy * Fx) - s_nu * qxy;
  const C a1 = de * (C)(1.0 / 36.0), a2 = deps * (C)(1.0 / 36.0);
  const C a3 = Fx * (C)(1.0 / 6.0), a4 = dqx * (C)(1.0 / 12.0);
  const C a5 = Fy * (C)(1.0 / 6.0), a6 = dqy * (C)(1.0 / 12.0);
  const C a7 = dpxx * (C)0.25, a8 = dpxy * (C)0.25;
  const C eax = -(a1 + (a2 + a2));            // even part on the axes
  const C ox = a3 - (a4 + a4), oy = a5 - (a6 + a6);
  fs[1] = f[1] + ((eax + a7) + ox);
  fs[3] = f[3] + ((eax + a7) - ox);
  fs[2] = f[2] + ((eax - a7) + oy);
  fs[4] = f[4] + ((eax - a7) - oy);
  const C ed = (a1 + a1) + a2;                // even part on the diagonals
  const C X = a3 + a4, Y = a5 + a6;
  fs[5] = f[5] + ((ed + a8) + (X + Y));
  fs[7] = f[7] + ((ed + a8) - (X + Y));
  fs[6] = f[6] + ((ed - a8) + (Y - X));
  fs[8] = f[8] + ((ed - a8) - (Y - X));
  const C d13 = (f[1] - fs[1]) + (f[3] - fs[3]), d24 = (f[2] - fs[2]) + (f[4] - fs[4]);
  const C d57 = (f[5] - fs[5]) + (f[7] - fs[7]), d68 = (f[6] - fs[6]) + (f[8] - fs[8]);
  fs[0] = f[0] + ((d13 + d24) + (d57 + d68));
}

// Q of Eq. 17 with the factor G/2 (kq = kappa G / 2): kq [(1 - A) psi sum_a w_a (psi_a - psi) e_a e_a
// + (A/2) sum_a w_a (psi_a^2 - psi^2) e_a e_a] from the centre psi p, the row's neighbours pL, pR and the rows
// above (n) and below (m). Grouped so that Q_xx, Q_yy are even and Q_xy odd, exactly, under both mirrors.
template <class C>
__device__ inline void qtensor(C p, C pL, C pR, C pn, C pnL, C pnR, C pm, C pmL, C pmR, C A, C kq, C& qxx, C& qyy,
                               C& qxy) {
#pragma clang fp contract(off)
  const C k1 = (C)(1.0 / 3.0), k2 = (C)(1.0 / 12.0);
  const C p2 = p * p;
  const C dg1 = ((pnR + pnL) + (pmR + pmL)) - (C)4 * p;
  const C dg2 = ((pnR * pnR + pnL * pnL) + (pmR * pmR + pmL * pmL)) - (C)4 * p2;
  const C xx1 = k1 * ((pR + pL) - (p + p)) + k2 * dg1;
  const C yy1 = k1 * ((pn + pm) - (p + p)) + k2 * dg1;
  const C xy1 = k2 * ((pnR - pnL) - (pmR - pmL));
  const C xx2 = k1 * ((pR * pR + pL * pL) - (p2 + p2)) + k2 * dg2;
  const C yy2 = k1 * ((pn * pn + pm * pm) - (p2 + p2)) + k2 * dg2;
  const C xy2 = k2 * ((pnR * pnR - pnL * pnL) - (pmR * pmR - pmL * pmL));
  const C c1 = ((C)1 - A) * p, c2 = (C)0.5 * A;
  qxx = kq * (c1 * xx1 + c2 * xx2);
  qyy = kq * (c1 * yy1 + c2 * yy2);
  qxy = kq * (c1 * xy1 + c2 * xy2);
}

// Ghost density of Sec. 4 in FP64: Eq. 19 (iters == 0) or the iters-th iterate of Eq. 21 with the square root of
// Eq. 20. T is the tangential difference of the boundary row, D = rho_2 - rho_1. Clamped to [0, rho_cap_hi].
__device__ inline double ghost_density(double rL, double rR, double r1, double r2, double c, double cot, int iters,
                                       double cap_hi, bool& clamped) {
#pragma clang fp contract(off)
  const double T = rR - rL;
  double r0;
  if (iters == 0) {
    r0 = r2 + cot * fabs(T);
  } else {
    const double D = r2 - r1;
    double dd = c * sqrt(T * T + 4.0 * D * D);
    for (int k = 2; k <= iters; ++k) dd = c * sqrt(T * T + dd * dd);
    r0 = r2 + dd;
  }
  clamped = false;
  if (r0 < 0.0) { r0 = 0.0; clamped = true; }
  else if (r0 > cap_hi) { r0 = cap_hi; clamped = true; }
  return r0;
}

// Streamed populations at fluid node (x, y) (rows 1..ny-2) from the stored post-collision ones (see the file
// header): f_i(x) = g_i(x - e_i), or g_{opp(i)}(x) where x - e_i is a ghost row (halfway bounce-back). With
// periodic rows (py) the rows below row 1 and above row ny-2 are rows ny-2 and 1.
template <class S, class C>
__device__ inline void gather(const typename Gbl<S>::T* __restrict__ g, int64_t plane, int pitch, int nx, int ny,
                              int x, int y, C (&f)[9], bool py = false) {
  typedef typename Gbl<S>::T GS;
  const int xl = x == 0 ? nx - 1 : x - 1, xr = x + 1 == nx ? 0 : x + 1;
  const bool bot = !py && (y == 1), top = !py && (y == ny - 2);
  const unsigned rc = (unsigned)((y - 1) * pitch);
  // row below (unused at the bottom wall) and row above (unused at the top wall)
  const unsigned rd = bot ? rc : (y == 1 ? (unsigned)((ny - 3) * pitch) : rc - (unsigned)pitch);
  const unsigned ru = top ? rc : (y == ny - 2 ? 0u : rc + (unsigned)pitch);
  auto P = [&](int q, unsigned off) -> C { return (C)((const GS*)(g + q * plane))[off]; };
  f[0] = P(0, rc + x);
  f[1] = P(1, rc + xl);
  f[2] = bot ? P(4, rc + x) : P(2, rd + x);
  f[3] = P(3, rc + xr);
  f[4] = top ? P(2, rc + x) : P(4, ru + x);
  f[5] = bot ? P(7, rc + x) : P(5, rd + xl);
  f[6] = bot ? P(8, rc + x) : P(6, rd + xr);
  f[7] = top ? P(5, rc + x) : P(7, ru + xr);
  f[8] = top ? P(6, rc + x) : P(8, ru + xl);
}


__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

}  // namespace
}  // namespace lbm
