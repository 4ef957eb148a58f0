// Adjoint of one time step (FP64), for lbm_adjoint_step.
//
// Forward step, per fluid node x (see lbm_kernels.hip):
//   rho = sum_i f_i, j = sum_i f_i e_i, psi = sqrt(a), a = (2/G_psi)(p_EOS(rho) - rho/3) clamped at 0 (Eq. 10);
//   ghost rows rho_0 = W(rho_{c-1,1}, rho_{c+1,1}, rho_{c,1}, rho_{c,2}; theta_c) clamped, psi_0 = psi(rho_0)
//   (Sec. 4, Eq. 19 / 21);
//   F = -G_f [ (A/2) sum_a w_a psi(x+e_a)^2 e_a + (1-A) psi(x) sum_a w_a psi(x+e_a) e_a ] + F_body (Eq. 9);
//   f*_i = (1 - 1/tau) f_i + f_eq_i(rho, v)/tau + S_i(v, F), v = (j + F/2)/rho (Eq. 1-6);
//   f'_i(x + e_i) = f*_i(x), or f'_{opp(i)}(x) = f*_i(x) at a wall (halfway bounce-back).
// The reverse pass, with lambda = dL/df' given:
//   1. lambda*_i(x) = lambda_i(x + e_i) (or lambda_{opp(i)}(x) at a wall): streaming transposed, as a gather;
//   2. collision transposed node by node: direct part of dL/df(x) and F_bar(x);
//   3. force transposed as a gather over neighbours: psi_bar(y) from F_bar(y) and F_bar(y - e_a);
//      G_f_bar += F_bar . (F - F_body) / G_f;
//   4. ghost rows: psi_bar_0 -> rho_bar_0 -> wetting transposed -> theta_bar and the boundary-row densities;
//   5. psi transposed: rho_bar(y) = psi_bar dpsi/drho, G_psi_bar += psi_bar dpsi/dG_psi; dL/df_k += rho_bar.
// The same order covers the other options of the forward step: the MRT collision of Eq. 15 (transposed in moment
// space, collide_mrt_adj) with the source of Eq. 16-17, whose Q reads psi like the force does (Q_bar joins F_bar
// in step 3; G_f_bar += Q_bar : Q / G_f); Martys-Chen walls (Eq. 14: psi_bar += +-(G_w/2) F_bar_y on the boundary
// rows, no ghost rows to transpose); periodic rows (every neighbour a fluid row, no ghost rows).
// Kinks (|T| of Eq. 19, the square root at 0, the clamps) take the sub-gradient 0.
// Passes: ka_wall_fwd (forward values of the wall rows and the ghost rows), ka_fused (steps 1-3 and 5 in one
// walk over row strips), ka_ghost_adj (step 4), ka_wall_fix (step 4's boundary-row terms into lambda_n),
// ka_finalize (the G partials).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int AB = 256;          // block size
constexpr int kAdjBlocks = 4096; // largest grid of the passes that leave reduction partials (grid-stride)

__device__ inline double dp_drho(const InstDesc& d, double rho) {
  // Eq. 11: the slope of the segment that the forward pass evaluated (same comparisons)
  if (d.eos_kind == 1) return rho <= d.pw_r1 ? d.pw_t[0] : (rho <= d.pw_r2 ? d.pw_t[1] : d.pw_t[2]);
  // Carnahan-Starling: R T (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4 - 2 a rho, e = b rho / 4
  const double e = d.eos_b4 * rho, om = 1.0 - e;
  const double om2 = om * om;
  return d.RT * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) * rcp64(om2 * om2) - 2.0 * d.eos_a * rho;
}

// d psi / d rho where psi > 0 (Eq. 10): (p'(rho) - 1/3) / (G_psi psi); 0 where psi was clamped. The reciprocals are
// the hardware's refined by Newton steps (about 1 ulp): a derivative needs no correctly rounded division.
__device__ inline double dpsi_drho(const InstDesc& d, double rho, double psi) {
  if (!(psi > 0.0)) return 0.0;
  return (dp_drho(d, rho) - 1.0 / 3.0) * (0.5 * d.two_over_Gpsi) * rcp64(psi);
}

struct Field {
  double* p;
  int pitch;
  __device__ double& at(int x, int y) const { return p[(int64_t)y * pitch + x]; }
};

__device__ inline double block_sum(double v, double* sm) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sm[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < AB / 64; ++k) t += sm[k];
  __syncthreads();
  return t;
}

// psi of Eq. 10 at one density and its derivative dpsi/drho (0 where the argument is clamped at 0: the
// sub-gradient at the kink). The division and the square root are the hardware's reciprocal and reciprocal square
// root refined by Newton / Goldschmidt steps (about 1 ulp): the reverse pass linearises about these values and does
// not have to reproduce the forward step's rounding.
__device__ inline void psi_dpsi(const InstDesc& d, double rho, double& psi, double& dps) {
  double p, dp;
  if (d.eos_kind == 1) {  // Eq. 11, the segment chosen by the forward step's comparisons
    if (rho <= d.pw_r1) {
      p = rho * d.pw_t[0];
      dp = d.pw_t[0];
    } else if (rho <= d.pw_r2) {
      p = d.pw_p1 + (rho - d.pw_r1) * d.pw_t[1];
      dp = d.pw_t[1];
    } else {
      p = d.pw_p2 + (rho - d.pw_r2) * d.pw_t[2];
      dp = d.pw_t[2];
    }
  } else {  // Carnahan-Starling, e = b rho / 4: p' = R T (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4 - 2 a rho
    const double e = d.eos_b4 * rho, io = rcp64(1.0 - e), io3 = io * io * io;
    p = rho * d.RT * (1.0 + e + e * e - e * e * e) * io3 - d.eos_a * rho * rho;
    dp = d.RT * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) * (io3 * io) - 2.0 * d.eos_a * rho;
  }
  const double arg = d.two_over_Gpsi * (p - rho * (1.0 / 3.0));
  if (arg <= 0.0) {
    psi = 0.0;
    dps = 0.0;
    return;
  }
  // s -> sqrt(arg), h -> 1 / (2 sqrt(arg))
  const double y = __builtin_amdgcn_rsq(arg);
  double s = arg * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  psi = fma(fma(-s, s, arg), h, s);
  dps = (dp - 1.0 / 3.0) * d.two_over_Gpsi * h;  // (p' - 1/3) (2 / G_psi) / (2 psi)
}

// 1. forward density of a fluid node from its populations
template <class T>
__device__ inline double node_rho(const T* __restrict__ f, int64_t n, int nx, int x, int y) {
  const unsigned k = (unsigned)((y - 1) * nx + x);  // node counts are below 2^31 (lbm_create checks)
  double fl[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) fl[i] = (double)f[i * n + k];
  return sum9(fl);
}

// Forward values of the wall rows, one thread per wall and column c: density and psi of the boundary row r1 and the
// second row r2 at c into the scratch field (read by the ghost rows' adjoint), and the ghost row beside the wall:
// density (clamped), psi, and whether the clamp was active (derivative 0). The boundary row's densities at c - 1 and
// c + 1 are summed again here from the populations, in the same order, rather than read from other threads.
template <class T>
__global__ __launch_bounds__(AB) void ka_wall_fwd(const InstDesc* __restrict__ descs, int inst,
                                                  const T* __restrict__ f, AdjScratch sc) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int t = (int)(blockIdx.x * AB + threadIdx.x);
  if (t >= 2 * nx) return;
  const int wall = t / nx, c = t % nx;
  const int64_t n = (int64_t)nx * (ny - 2);
  Field R{sc.rho, d.pitch}, P{sc.psi, d.pitch};
  const int g = wall == 0 ? 0 : ny - 1, r1 = wall == 0 ? 1 : ny - 2, r2 = wall == 0 ? 2 : ny - 3;  // ny >= 4
  const double rho1 = node_rho(f, n, nx, c, r1), rho2 = node_rho(f, n, nx, c, r2);
  double dps;
  R.at(c, r1) = rho1;
  psi_dpsi(d, rho1, P.at(c, r1), dps);
  R.at(c, r2) = rho2;
  psi_dpsi(d, rho2, P.at(c, r2), dps);
  if (d.wall_mc) {  // solid wall rows (Eq. 14): psi = 0 there, no dependence on the state
    R.at(c, g) = 0.0;
    P.at(c, g) = 0.0;
    sc.gflag[wall * nx + c] = 1.0;
    return;
  }
  bool cl;
  const double r0 = ghost_density(node_rho(f, n, nx, wrapx(c - 1, nx), r1), node_rho(f, n, nx, wrapx(c + 1, nx), r1),
                                  rho1, rho2, d.cos_th[wall * nx + c], d.cot_th[wall * nx + c], d.wet_iters,
                                  d.rho_cap_hi, cl);
  R.at(c, g) = r0;
  bool dm;
  P.at(c, g) = psi_f64(d, r0, dm);
  sc.gflag[wall * nx + c] = cl ? 1.0 : 0.0;
}

// 2. streaming and collision transposed at a fluid node, BGK: given lambda* (ls), the node's forward density and
//    momentum and its total force F: F_bar and the direct part of lambda_n,
//    lam_i = (1 - 1/tau) ls_i + h + hx e_ix + hy e_iy.
__device__ inline void collide_adj(const InstDesc& d, double rho, double jx, double jy, const double (&ls)[9],
                                   double Fx, double Fy, double& h, double& hx, double& hy, double& Fbx,
                                   double& Fby) {
  const double irho = rcp64(rho);
  const double vx = (jx + 0.5 * Fx) * irho, vy = (jy + 0.5 * Fy) * irho;
  const double v2 = vx * vx + vy * vy;
  const double it = d.inv_tau, pref = d.force_pref;
  // Every sum over directions below is a weighted moment of the cotangent ls: with m = sum_i w_i ls_i (1, e_x, e_y,
  // e_x^2, e_x e_y, e_y^2),
  //   adjoint of f_eq (weight it):   rho_bar = it [m0 (1 - 1.5 v^2) + 3 v.m1 + 4.5 v.m2.v],
  //                                  v_bar  += it rho [3 m1 + 9 m2.v - 3 v m0],
  //   adjoint of the forcing (pref): v_bar  += pref [9 m2.F - 3 F m0],   F_bar = pref [3 m1 - 3 v m0 + 9 m2.v].
  const double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w2 = 1.0 / 36.0;
  const double d5 = ls[5] + ls[7], d6 = ls[6] + ls[8];   // diagonal pairs
  const double dg = d5 + d6;
  const double m0 = w0 * ls[0] + w1 * ((ls[1] + ls[3]) + (ls[2] + ls[4])) + w2 * dg;
  const double mx = w1 * (ls[1] - ls[3]) + w2 * ((ls[5] - ls[7]) + (ls[8] - ls[6]));
  const double my = w1 * (ls[2] - ls[4]) + w2 * ((ls[5] - ls[7]) + (ls[6] - ls[8]));
  const double mxx = w1 * (ls[1] + ls[3]) + w2 * dg;
  const double myy = w1 * (ls[2] + ls[4]) + w2 * dg;
  const double mxy = w2 * (d5 - d6);
  const double m2vx = mxx * vx + mxy * vy, m2vy = mxy * vx + myy * vy;  // m2 . v
  double rhob = it * (m0 * (1.0 - 1.5 * v2) + 3.0 * (vx * mx + vy * my) + 4.5 * (vx * m2vx + vy * m2vy));
  double vbx = it * rho * (3.0 * mx + 9.0 * m2vx - 3.0 * vx * m0) + pref * (9.0 * (mxx * Fx + mxy * Fy) - 3.0 * Fx * m0);
  double vby = it * rho * (3.0 * my + 9.0 * m2vy - 3.0 * vy * m0) + pref * (9.0 * (mxy * Fx + myy * Fy) - 3.0 * Fy * m0);
  Fbx = pref * (3.0 * mx - 3.0 * vx * m0 + 9.0 * m2vx);
  Fby = pref * (3.0 * my - 3.0 * vy * m0 + 9.0 * m2vy);
  // v = (j + F/2) / rho
  const double jbx = vbx * irho, jby = vby * irho;
  Fbx += 0.5 * jbx;
  Fby += 0.5 * jby;
  rhob -= (jbx * vx + jby * vy);
  h = rhob;
  hx = jbx;
  hy = jby;
}

// D2Q9 moment basis in the order of Eq. 4 (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) and its row norms.
constexpr int kMom[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},       {-4, -1, -1, -1, -1, 2, 2, 2, 2}, {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},    {0, -2, 0, 2, 0, 1, -1, -1, 1},   {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},    {0, 1, -1, 1, -1, 0, 0, 0, 0},    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
constexpr double kMomNorm[9] = {9.0, 36.0, 36.0, 6.0, 12.0, 6.0, 12.0, 4.0, 4.0};

// 2'. the MRT collision of Eq. 15 transposed. Forward: f* = f + M^-1 dm with dm_k = -s_k (m_k - m_eq,k)
//     + (1 - s_k/2) S_k + C_k on the non-conserved moments and dm = F on j. Reverse: dm_bar = D^-1 M lambda*, then
//     the relaxation (through m = M f), the equilibria and forcing moments (through rho and v = (j + F/2)/rho) and
//     the source (Q_bar, the adjoint of Q of Eq. 17, xx / yy / xy).
__device__ inline void collide_mrt_adj(const InstDesc& d, double rho, double jx, double jy, const double (&ls)[9],
                                       double Fx, double Fy, double (&lam)[9], double& Fbx, double& Fby,
                                       double (&qb)[3]) {
  const double irho = rcp64(rho);
  const double vx = (jx + 0.5 * Fx) * irho, vy = (jy + 0.5 * Fy) * irho;
  const double v2 = vx * vx + vy * vy;
  const double sn = d.inv_tau;
  double dmb[9];
#pragma unroll
  for (int k = 1; k < 9; ++k) {
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) a += kMom[k][i] * ls[i];
    dmb[k] = a / kMomNorm[k];
  }
  // a_k = s_k dm_bar_k is the adjoint of m_eq,k; the relaxation's term through m = M f is -a_k; the forcing's
  // adjoint is b_k = (1 - s_k/2) dm_bar_k = dm_bar_k - a_k / 2
  const double a1 = d.s_e * dmb[1], a2 = d.s_eps * dmb[2], a4 = d.s_q * dmb[4], a6 = d.s_q * dmb[6];
  const double a7 = sn * dmb[7], a8 = sn * dmb[8];
  const double b12 = (dmb[1] - 0.5 * a1) - (dmb[2] - 0.5 * a2), b4 = dmb[4] - 0.5 * a4, b6 = dmb[6] - 0.5 * a6;
  const double b7 = dmb[7] - 0.5 * a7, b8 = dmb[8] - 0.5 * a8;
  // m_eq / rho: (-2 + 3 v^2, 1 - 3 v^2, -v_x, -v_y, v_x^2 - v_y^2, v_x v_y) on e, eps, q_x, q_y, p_xx, p_xy
  double rhob = a1 * (-2.0 + 3.0 * v2) + a2 * (1.0 - 3.0 * v2) - a4 * vx - a6 * vy + a7 * (vx * vx - vy * vy) +
                a8 * vx * vy;
  double vbx = 6.0 * rho * vx * (a1 - a2) - rho * a4 + 2.0 * rho * vx * a7 + rho * vy * a8;
  double vby = 6.0 * rho * vy * (a1 - a2) - rho * a6 - 2.0 * rho * vy * a7 + rho * vx * a8;
  vbx += 6.0 * Fx * b12 + 2.0 * Fx * b7 + Fy * b8;
  vby += 6.0 * Fy * b12 - 2.0 * Fy * b7 + Fx * b8;
  Fbx = dmb[3] + 6.0 * vx * b12 - b4 + 2.0 * vx * b7 + vy * b8;
  Fby = dmb[5] + 6.0 * vy * b12 - b6 - 2.0 * vy * b7 + vx * b8;
  qb[0] = 1.5 * d.s_e * dmb[1] - sn * dmb[7];
  qb[1] = 1.5 * d.s_e * dmb[1] + sn * dmb[7];
  qb[2] = -sn * dmb[8];
  // v = (j + F/2) / rho
  const double jbx = vbx * irho, jby = vby * irho;
  Fbx += 0.5 * jbx;
  Fby += 0.5 * jby;
  rhob -= (jbx * vx + jby * vy);
  const double mr[9] = {0.0, -a1, -a2, 0.0, -a4, 0.0, -a6, -a7, -a8};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double m = 0.0;
#pragma unroll
    for (int k = 1; k < 9; ++k) m += kMom[k][i] * mr[k];
    lam[i] = ls[i] + m + rhob + jbx * kEX[i] + jby * kEY[i];
  }
}

// psi_bar at node y from the force of node x = y - e_a (x a fluid node): -G_f w_a (F_bar(x).e_a)(A psi(y) + (1-A) psi(x)),
// plus, with the surface-tension source, kq w_a (Q_bar(x) : e_a e_a)(A psi(y) + (1-A) psi(x)) from Q of Eq. 17
// (qwall: Q_bar of the boundary rows, or NULL).
__device__ inline double psi_bar_from(const InstDesc& d, const Field& P, const Field& FX, const Field& FY,
                                      const double* qwall, int nx, int ny, int x0, int y0) {
  double acc = 0.0;
  const double py = P.at(x0, y0);
#pragma unroll
  for (int a = 1; a < 9; ++a) {
    const int xs = wrapx(x0 - kEX[a], nx), ys = y0 - kEY[a];
    if (ys < 1 || ys > ny - 2) continue;
    const double wa = a < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
    double fe = -d.G_f * (FX.at(xs, ys) * kEX[a] + FY.at(xs, ys) * kEY[a]);
    if (qwall) {  // the source's Q at the boundary-row node xs (Eq. 17) also reads psi here
      const double* q = qwall + (ys == 1 ? 0 : 3) * nx;
      fe += d.kq * (q[xs] * kEX[a] * kEX[a] + q[nx + xs] * kEY[a] * kEY[a] + q[2 * nx + xs] * kEX[a] * kEY[a]);
    }
    acc += wa * fe * (d.A * py + (1.0 - d.A) * P.at(xs, ys));
  }
  return acc;
}

// 4. ghost rows transposed: psi_bar_0 -> rho_bar_0 -> wetting -> theta_bar, boundary-row density adjoints
//    (wet[wall][0..3][c] = d/d rho_{c-1,1}, d/d rho_{c+1,1}, d/d rho_{c,1}, d/d rho_{c,2}); partials of G_psi_bar.
__global__ __launch_bounds__(AB) void ka_ghost_adj(const InstDesc* __restrict__ descs, int inst, AdjScratch sc,
                                                   double* __restrict__ theta_bar) {
  __shared__ double sm[AB / 64];
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  Field R{sc.rho, d.pitch}, P{sc.psi, d.pitch}, FX{sc.Fbar, d.pitch}, FY{sc.Fbar + (int64_t)ny * d.pitch, d.pitch};
  const int t = (int)(blockIdx.x * AB + threadIdx.x);
  double gpsi = 0.0;
  if (t < 2 * nx) {
    const int wall = t / nx, c = t % nx;
    const int g = wall == 0 ? 0 : ny - 1, r1 = wall == 0 ? 1 : ny - 2, r2 = wall == 0 ? 2 : ny - 3;
    const double pb = psi_bar_from(d, P, FX, FY, (d.mrt && d.kq != 0.0) ? sc.qwall : nullptr, nx, ny, c, g);
    const double psi0 = P.at(c, g), rho0 = R.at(c, g);
    if (psi0 > 0.0) gpsi += pb * (-psi0 * 0.5 * d.two_over_Gpsi * 0.5);  // d psi / d G_psi = -psi / (2 G_psi)
    double rb0 = sc.gflag[wall * nx + c] != 0.0 ? 0.0 : pb * dpsi_drho(d, rho0, psi0);
    // wetting transposed (forward recomputed)
    const double rL = R.at(wrapx(c - 1, nx), r1), rR = R.at(wrapx(c + 1, nx), r1);
    const double q1 = R.at(c, r1), q2 = R.at(c, r2);
    const double cth = d.cos_th[wall * nx + c], sth = d.sin_th[wall * nx + c], cot = d.cot_th[wall * nx + c];
    const double T = rR - rL;
    double Tb = 0.0, Db = 0.0, thb = 0.0, q2b = rb0;
    const int K = d.wet_iters;
    if (K == 0) {
      // rho_0 = rho_2 + cot(theta) |T|
      const double sg = T > 0.0 ? 1.0 : (T < 0.0 ? -1.0 : 0.0);
      Tb = rb0 * cot * sg;
      thb = rb0 * fabs(T) * (-1.0 / (sth * sth));
    } else {
      // iterates d_1 = c sqrt(T^2 + 4 D^2), d_k = c sqrt(T^2 + d_{k-1}^2), rho_0 = rho_2 + d_K
      const double D = q2 - q1;
      double db = rb0;   // adjoint of d_K
      double cb = 0.0;   // adjoint of cos(theta)
      for (int k = K; k >= 1; --k) {
        // forward value d_{k-1} (k >= 2) recomputed from the start
        double dprev = 0.0;
        if (k >= 2) {
          dprev = cth * sqrt(T * T + 4.0 * D * D);
          for (int m = 2; m <= k - 1; ++m) dprev = cth * sqrt(T * T + dprev * dprev);
        }
        const double s = k >= 2 ? sqrt(T * T + dprev * dprev) : sqrt(T * T + 4.0 * D * D);
        cb += db * s;
        const double sb = db * cth;
        if (s > 0.0) {
          Tb += sb * T / s;
          if (k >= 2) db = sb * dprev / s;
          else Db += sb * 4.0 * D / s;
        } else {
          db = 0.0;
        }
      }
      thb = cb * (-sth);
    }
    q2b += Db;
    const double q1b = -Db;
    double* wet = sc.wet + wall * 4 * nx;
    wet[0 * nx + c] = -Tb;  // d / d rho_{c-1, r1}
    wet[1 * nx + c] = Tb;   // d / d rho_{c+1, r1}
    wet[2 * nx + c] = q1b;  // d / d rho_{c, r1}
    wet[3 * nx + c] = q2b;  // d / d rho_{c, r2}
    theta_bar[wall * nx + c] += thb;
  }
  const double tot = block_sum(gpsi, sm);
  if (threadIdx.x == 0) sc.part[kAdjBlocks + blockIdx.x] = tot;
}

// 3 + 5 fused: one wavefront walks a strip of rows [y0, ylast] over at most 60 columns. Row by row it transposes
// the streaming and collision one row ahead (stage C, also on one halo column at each side and on the rows y0 - 1
// and ylast + 1; a second halo column at each side only supplies psi), keeps that row's F_bar in a ring of three
// rows in LDS, and transposes the force and psi for the row behind (stage S): psi_bar from its own force and the
// eight neighbours' forces, rho_bar = psi_bar dpsi/drho, and lambda_n = direct part + rho_bar, written once.
// Per row the window keeps the forward values the two stages read (psi with its left and right neighbours,
// dpsi/drho, density and momentum), computed once from the row's populations; the populations are loaded two rows
// ahead of stage C and lambda* one row ahead, so every global load of a row iteration is for a later row. The
// ghost rows' psi comes from the scratch field. F_bar of the boundary rows 1 and ny-2 also goes to the scratch for
// the ghost rows' adjoint, whose boundary-row terms ka_wall_fix adds afterwards. Partials of G_f_bar (stage C) and
// G_psi_bar (stage S) per block, over the block's own columns and rows only.
constexpr int FL = 64;         // lanes per block (one wavefront): at most 60 own columns, two halo columns each side

// Interaction force (Eq. 9) from the 3 x 3 psi values around the node: rows below (m), own (c), above (n).
__device__ inline void force_vals(const InstDesc& d, double pmL, double pm, double pmR, double pcL, double pcR,
                                  double pc, double pnL, double pn, double pnR, double& Fx, double& Fy) {
  const double k1 = 1.0 / 3.0, k2 = 1.0 / 12.0, A = d.A, Gf = d.G_f;
  const double spx = k1 * (pcR - pcL) + k2 * ((pnR - pnL) + (pmR - pmL));
  const double spy = k1 * (pn - pm) + k2 * ((pnR + pnL) - (pmR + pmL));
  const double sux = k1 * (pcR * pcR - pcL * pcL) + k2 * ((pnR * pnR - pnL * pnL) + (pmR * pmR - pmL * pmL));
  const double suy = k1 * (pn * pn - pm * pm) + k2 * ((pnR * pnR + pnL * pnL) - (pmR * pmR + pmL * pmL));
  Fx = -Gf * (0.5 * A * sux + (1.0 - A) * pc * spx);
  Fy = -Gf * (0.5 * A * suy + (1.0 - A) * pc * spy);
}

// Left and right neighbours of a per-lane value across the wavefront: lane l receives the values of lanes l - 1
// and l + 1 (wavefront shifts by one lane, both 32-bit halves; lanes 0 and 63 receive their own value).
__device__ inline void lane_lr(double v, double& L, double& R) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  L = __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),   // wave_shr:1
                       __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
  R = __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),   // wave_shl:1
                       __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}

// EXT: the MRT collision with the source of Eq. 16-17 (Q_bar joins F_bar in the ring) and the fluid-solid force of
// Eq. 14 on the boundary rows; without it only the BGK collision with geometric walls is compiled.
// T: storage type of the state and of lambda (double, or float for lbm_adjoint_step_f32); the arithmetic is FP64.
template <bool EXT, class T>
__global__ __launch_bounds__(FL, 2) void ka_fused(const InstDesc* __restrict__ descs, int inst,
                                                  const T* __restrict__ f, const T* __restrict__ lam1,
                                                  T* __restrict__ lam0, AdjScratch sc, int bw, int ncb, int H,
                                                  int ntasks) {
  constexpr int NR = EXT ? 5 : 2;  // per node in the ring: F_bar (x, y), then Q_bar (xx, yy, xy)
  constexpr int ND = EXT ? 9 : 1;  // EXT: the direct part of lambda_n of two rows, written by C and read by S
  __shared__ double ring[3][NR][FL];
  __shared__ double ldir[2][ND][FL];
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int64_t n = (int64_t)nx * (ny - 2);
  Field P{sc.psi, d.pitch}, FX{sc.Fbar, d.pitch}, FY{sc.Fbar + (int64_t)ny * d.pitch, d.pitch};
  const int l = (int)threadIdx.x;
  const double k1 = 1.0 / 3.0, k2 = 1.0 / 12.0, Gf = d.G_f, A = d.A;
  const bool mrt = EXT && d.mrt != 0, mcw = EXT && d.wall_mc != 0;
  const bool py = d.periodic_y != 0;  // periodic rows: rows are walked as virtual rows, wrapped to 1 .. ny-2
  auto wy = [&](int y) { return y < 1 ? y + (ny - 2) : (y > ny - 2 ? y - (ny - 2) : y); };
  const double kq = mrt ? d.kq : 0.0, gwb = d.gw_half[0], gwt = d.gw_half[1];
  const double keep = 1.0 - d.inv_tau;  // BGK: the relaxed part f - (f - f_eq)/tau keeps (1 - 1/tau) of lambda*
  const bool kept = keep != 0.0;
  double gf_part = 0.0, gpsi = 0.0;
  // XCD-aware order: blocks go round-robin to the eight XCDs (the grid is a multiple of 8); XCD k takes the k-th
  // contiguous share of the task slots, so neighbouring column blocks of a strip, which read the same cache lines
  // at their common edge, share one L2
  const int nslots = (ntasks + 7) / 8 * 8, per = nslots / 8;
  for (int i = (int)blockIdx.x; i < nslots; i += (int)gridDim.x) {
    const int t = (i % 8) * per + i / 8;
    if (t >= ntasks) continue;  // uniform over the block
    const int cb = t % ncb, sb = t / ncb;
    const int x0 = cb * bw, w = min(bw, nx - x0);
    const int y0 = 1 + sb * H, ylast = min(ny - 2, y0 + H - 1);
    // lanes 0 .. w+3: columns x0-2 .. x0+w+1 (one period at most: nx >= 2); stage C is valid on lanes 1 .. w+2
    // (lanes 0 and w+3 only supply psi), stage S runs on the block's own columns, lanes 2 .. w+1. The lanes past
    // w+3 repeat column x0 and their results are not used.
    const bool own = l >= 2 && l <= w + 1;
    const int x = l <= w + 3 ? wrapx(x0 - 2 + l, nx) : x0;
    const int xl = wrapx(x - 1, nx), xr = wrapx(x + 1, nx);
    const int yc0 = py ? y0 - 1 : max(1, y0 - 1), yc1 = py ? ylast + 1 : min(ny - 2, ylast + 1);
    auto fluid = [&](int y) { return py || (y >= 1 && y <= ny - 2); };
    auto rowk = [&](int y) { return (unsigned)((wy(y) - 1) * nx); };  // node counts are below 2^31
    // populations of the node in row y: loads keep the storage type and are widened where the row is used
    auto load_f = [&](int y, T (&fl)[9]) {
      const unsigned k = rowk(y) + (unsigned)x;
#pragma unroll
      for (int i = 0; i < 9; ++i) fl[i] = f[i * n + k];
    };
    // 1. lambda*_i(x) = lambda_i(x + e_i), or lambda_opp(i)(x) where x + e_i is a wall row (bounce-back)
    auto load_lam = [&](int y, T (&ls)[9]) {
      const bool bot = !py && y == 1, top = !py && y == ny - 2;
      const unsigned r0 = rowk(y), rd = bot ? r0 : rowk(y - 1), ru = top ? r0 : rowk(y + 1);
      const unsigned xo = r0 + (unsigned)x;
      auto L = [&](int q, unsigned off) -> T { return lam1[q * n + off]; };
      ls[0] = L(0, xo);
      ls[1] = L(1, r0 + (unsigned)xr);
      ls[3] = L(3, r0 + (unsigned)xl);
      ls[2] = L(top ? 4 : 2, top ? xo : ru + (unsigned)x);
      ls[5] = L(top ? 7 : 5, top ? xo : ru + (unsigned)xr);
      ls[6] = L(top ? 8 : 6, top ? xo : ru + (unsigned)xl);
      ls[4] = L(bot ? 2 : 4, bot ? xo : rd + (unsigned)x);
      ls[7] = L(bot ? 5 : 7, bot ? xo : rd + (unsigned)xl);
      ls[8] = L(bot ? 6 : 8, bot ? xo : rd + (unsigned)xr);
    };
    auto node = [&](const T (&fl)[9], double& r, double& jx, double& jy, double& p, double& dp) {
      double v[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) v[i] = (double)fl[i];
      r = sum9(v);
      jx = mom_x(v);
      jy = mom_y(v);
      psi_dpsi(d, r, p, dp);
    };
    // window at the stage C row yc: psi (own, left, right) of rows yc-2 (a), yc-1 (b), yc (c); dpsi/drho of rows
    // b and c; density and momentum of row c; the direct part of lambda_n of row b (BGK: h + hx e_x + hy e_y, and
    // lambda* of row b where 1/tau != 1); the populations of row yc+1 (fN) and lambda* of row yc (lsA)
    double pa = 0.0, aL = 0.0, aR = 0.0, pb = 0.0, bL = 0.0, bR = 0.0, pc = 0.0, cL = 0.0, cR = 0.0;
    double db = 0.0, dc = 0.0, rc = 0.0, jxc = 0.0, jyc = 0.0, pg = 0.0, hb = 0.0, hbx = 0.0, hby = 0.0;
    T fN[9], lsA[9], lsN[9], lsB[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) lsN[i] = lsB[i] = (T)0;
    if (fluid(yc0 - 1)) {
      double r, jx, jy;
      load_f(yc0 - 1, fN);
      node(fN, r, jx, jy, pb, db);
    } else {
      pb = P.at(x, yc0 - 1);  // ghost row
    }
    lane_lr(pb, bL, bR);
    load_f(yc0, fN);
    node(fN, rc, jxc, jyc, pc, dc);
    lane_lr(pc, cL, cR);
    if (fluid(yc0 + 1)) load_f(yc0 + 1, fN);
    else pg = P.at(x, yc0 + 1);
    load_lam(yc0, lsA);
    // stage S at row ys: psi rows ys-1 (a), ys (b), ys+1 (c), dpsi/drho of row ys in db
    auto stage_s = [&](int ys) {
      const double* Ra = &ring[(ys - 1) % 3][0][0];
      const double* Rb = &ring[ys % 3][0][0];
      const double* Rc = &ring[(ys + 1) % 3][0][0];
      const double pv[3][3] = {{aL, pa, aR}, {bL, pb, bR}, {cL, pc, cR}};  // [row ys-1..ys+1][x-1..x+1]
      const double spx = k1 * (bR - bL) + k2 * ((cR - cL) + (aR - aL));
      const double spy = k1 * (pc - pa) + k2 * ((cR + cL) - (aR + aL));
      double acc = -Gf * (1.0 - A) * (Rb[l] * spx + Rb[FL + l] * spy);
      if constexpr (EXT) {
        // fluid-solid force of Eq. 14 on the boundary rows: F_s,y = +-(G_w / 2) psi
        if (mcw && ys == 1) acc += gwb * Rb[FL + l];
        if (mcw && ys == ny - 2) acc -= gwt * Rb[FL + l];
        if (kq != 0.0) {
          // own Q (Eq. 17): d Q / d psi(x) = kq [(1 - A) a - psi W], a = sum_a w_a (psi_a - psi) e_a e_a, W = I
          const double dg = ((cR + cL) + (aR + aL)) - 4.0 * pb;
          const double axx = k1 * ((bR + bL) - 2.0 * pb) + k2 * dg;
          const double ayy = k1 * ((pc + pa) - 2.0 * pb) + k2 * dg;
          const double axy = k2 * ((cR - cL) - (aR - aL));
          const double qxx = Rb[2 * FL + l], qyy = Rb[3 * FL + l], qxy = Rb[4 * FL + l];
          acc += kq * ((1.0 - A) * (qxx * axx + qyy * ayy + qxy * axy) - pb * (qxx + qyy));
        }
      }
      // the neighbour x = y - e_q lies in row ys - e_qy: rows below (e_qy = 1) and above (e_qy = -1) are skipped
      // where they are wall rows
      const bool lo_ok = py || ys > 1, hi_ok = py || ys < ny - 2;
#pragma unroll
      for (int q = 1; q < 9; ++q) {
        if ((kEY[q] == 1 && !lo_ok) || (kEY[q] == -1 && !hi_ok)) continue;
        const double* Rq = kEY[q] == 1 ? Ra : (kEY[q] == 0 ? Rb : Rc);
        const int ln = l - kEX[q];
        const double wa = q < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
        double fe = -Gf * (Rq[ln] * kEX[q] + Rq[FL + ln] * kEY[q]);
        if constexpr (EXT) {
          if (kq != 0.0)  // the neighbour's Q reads psi here (Eq. 17)
            fe += kq * (Rq[2 * FL + ln] * (kEX[q] * kEX[q]) + Rq[3 * FL + ln] * (kEY[q] * kEY[q]) +
                        Rq[4 * FL + ln] * (kEX[q] * kEY[q]));
        }
        acc += wa * fe * (A * pb + (1.0 - A) * pv[1 - kEY[q]][1 - kEX[q]]);
      }
      if (pb > 0.0) gpsi += acc * (-pb * 0.5 * d.two_over_Gpsi * 0.5);
      const double rbar = acc * db;
      const unsigned k = rowk(ys) + (unsigned)x;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        double dir;
        if constexpr (EXT) {
          dir = ldir[ys & 1][i][l];
        } else {
          dir = hb;
          if (kEX[i] != 0) dir += kEX[i] * hbx;
          if (kEY[i] != 0) dir += kEY[i] * hby;
          if (kept) dir = keep * (double)lsB[i] + dir;
        }
        lam0[i * n + k] = (T)(dir + rbar);
      }
    };
    for (int yc = yc0; yc <= yc1; ++yc) {
      // forward values of row yc+1 from its populations (loaded one iteration ago), or the ghost row's psi
      double pe, de = 0.0, re = 0.0, jxe = 0.0, jye = 0.0;
      if (fluid(yc + 1)) node(fN, re, jxe, jye, pe, de);
      else pe = pg;
      // loads for later rows: populations (or the ghost row's psi) of row yc+2, lambda* of row yc+1
      const int r2 = yc + 2;
      double pgnext = 0.0;
      if (r2 <= yc1 + 1) {
        if (fluid(r2)) load_f(r2, fN);
        else pgnext = P.at(x, r2);
      }
      if (yc < yc1) load_lam(yc + 1, lsN);
      double eL, eR;
      lane_lr(pe, eL, eR);
      // 2. stage C at row yc: psi rows yc-1 (b), yc (c), yc+1 (e)
      double Fix, Fiy;
      force_vals(d, bL, pb, bR, cL, cR, pc, eL, pe, eR, Fix, Fiy);
      double Fx = Fix + d.body_fx, Fy = Fiy + d.body_fy;
      if (mcw && yc == 1) Fy = Fy + gwb * pc;        // Eq. 14 next to the bottom wall
      if (mcw && yc == ny - 2) Fy = Fy - gwt * pc;   // and next to the top wall
      double ls[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) ls[i] = (double)lsA[i];
      double Fbx, Fby, qb[3] = {0.0, 0.0, 0.0}, gq = 0.0, hc = 0.0, hcx = 0.0, hcy = 0.0;
      if (mrt) {
        double lam[9];
        collide_mrt_adj(d, rc, jxc, jyc, ls, Fx, Fy, lam, Fbx, Fby, qb);
#pragma unroll
        for (int i = 0; i < 9; ++i) ldir[yc & 1][i % ND][l] = lam[i];
        if (kq != 0.0) {  // Q is proportional to G_f: G_f_bar += Q_bar : Q / G_f (the division once per block)
          double qxx, qyy, qxy;
          qtensor<double>(pc, cL, cR, pe, eL, eR, pb, bL, bR, A, kq, qxx, qyy, qxy);
          gq = qb[0] * qxx + qb[1] * qyy + qb[2] * qxy;
        }
      } else {
        collide_adj(d, rc, jxc, jyc, ls, Fx, Fy, hc, hcx, hcy, Fbx, Fby);
        if constexpr (EXT) {
#pragma unroll
          for (int i = 0; i < 9; ++i) {
            double dir = hc;
            if (kEX[i] != 0) dir += kEX[i] * hcx;
            if (kEY[i] != 0) dir += kEY[i] * hcy;
            ldir[yc & 1][i][l] = kept ? keep * ls[i] + dir : dir;
          }
        }
      }
      if (own) {
        if (yc >= y0 && yc <= ylast) gf_part += (Fbx * Fix + Fby * Fiy) + gq;  // halo rows belong elsewhere
        if (!py && (yc == 1 || yc == ny - 2)) {
          FX.at(x, yc) = Fbx;
          FY.at(x, yc) = Fby;
          if (kq != 0.0) {
            double* q = sc.qwall + (yc == 1 ? 0 : 3) * nx;
            q[x] = qb[0];
            q[nx + x] = qb[1];
            q[2 * nx + x] = qb[2];
          }
        }
      }
      __syncthreads();  // the slot written next was read by stage S two rows back
      double* Rw = &ring[yc % 3][0][0];
      Rw[l] = Fbx;
      Rw[FL + l] = Fby;
      if constexpr (EXT) {
        Rw[2 * FL + l] = qb[0];
        Rw[3 * FL + l] = qb[1];
        Rw[4 * FL + l] = qb[2];
      }
      __syncthreads();
      // 3, 5. stage S at row yc-1: psi rows yc-2 (a), yc-1 (b), yc (c)
      if (yc - 1 >= y0 && yc - 1 <= ylast && own) stage_s(yc - 1);
      // slide the window one row on
      pa = pb; aL = bL; aR = bR;
      pb = pc; bL = cL; bR = cR;
      pc = pe; cL = eL; cR = eR;
      db = dc; dc = de;
      rc = re; jxc = jxe; jyc = jye;
      hb = hc; hbx = hcx; hby = hcy;
      pg = pgnext;
      if (!EXT && kept) {
#pragma unroll
        for (int i = 0; i < 9; ++i) lsB[i] = lsA[i];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) lsA[i] = lsN[i];
    }
    // the top wall's boundary row: no stage C row above it (row ny-1 is the ghost row, F_bar absent there);
    // after the slide the window holds psi rows ny-3 (a), ny-2 (b), ny-1 (c)
    if (!py && ylast == ny - 2 && own) stage_s(ylast);
    __syncthreads();  // the ring is reused by the next task
  }
  const double tf = wave_sum(gf_part) / Gf;  // one wavefront per block; F (less F_body) is proportional to G_f
  const double tp = wave_sum(gpsi);
  if (threadIdx.x == 0) {
    sc.part[blockIdx.x] = tf;
    sc.part[2 * kAdjBlocks + blockIdx.x] = tp;
  }
}

// The wetting's boundary-row adjoints (from ka_ghost_adj) into lambda_n: rows 1, 2 (bottom wall) and ny-2, ny-3
// (top wall), each fluid row once, every population of the node (rho = sum_i f_i).
template <class T>
__global__ __launch_bounds__(AB) void ka_wall_fix(const InstDesc* __restrict__ descs, int inst,
                                                  T* __restrict__ lam0, AdjScratch sc) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int64_t n = (int64_t)nx * (ny - 2);
  const int t = (int)(blockIdx.x * AB + threadIdx.x);
  if (t >= 4 * nx) return;
  const int j = t / nx, x = t % nx;
  const int rows[4] = {1, 2, ny - 3, ny - 2};
  const int y = rows[j];
  for (int m = 0; m < j; ++m)
    if (rows[m] == y) return;  // a row listed twice (ny < 6) is handled by its first entry
  if (y < 1 || y > ny - 2) return;
  const int xl = wrapx(x - 1, nx), xr = wrapx(x + 1, nx);
  double rb = 0.0;
  for (int wall = 0; wall < 2; ++wall) {
    const int r1 = wall == 0 ? 1 : ny - 2, r2 = wall == 0 ? 2 : ny - 3;
    const double* wet = sc.wet + wall * 4 * nx;
    if (y == r1) rb += wet[2 * nx + x] + wet[0 * nx + xr] + wet[1 * nx + xl];
    if (y == r2) rb += wet[3 * nx + x];
  }
  const unsigned k = (unsigned)((y - 1) * nx + x);
#pragma unroll
  for (int i = 0; i < 9; ++i) lam0[i * n + k] = (T)((double)lam0[i * n + k] + rb);
}

// Fold of the partials into G_bar by one block: each thread sums a fixed strided subset in order, then a fixed
// tree over the block, so the result does not depend on timing.
__global__ __launch_bounds__(AB) void ka_finalize(AdjScratch sc, int nb_fluid, int nb_ghost,
                                                  double* __restrict__ G_bar) {
  __shared__ double sm[AB / 64];
  double gf = 0.0, gp = 0.0;
  for (int b = (int)threadIdx.x; b < nb_fluid; b += AB) {
    gf += sc.part[b];
    gp += sc.part[2 * kAdjBlocks + b];
  }
  for (int b = (int)threadIdx.x; b < nb_ghost; b += AB) gp += sc.part[kAdjBlocks + b];
  gf = block_sum(gf, sm);
  gp = block_sum(gp, sm);
  if (threadIdx.x == 0) {
    G_bar[0] += gf;
    G_bar[1] += gp;
  }
}

}  // namespace

int adjoint_partials_needed() { return 3 * kAdjBlocks; }

namespace {
// resident blocks (wavefronts) of the fused pass per compute unit, from its register and LDS use
template <bool EXT, class T>
int fused_blocks_per_cu() {
  static const int b = [] {
    int v = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, ka_fused<EXT, T>, FL, 0) == hipSuccess && v > 0 ? v : 8;
  }();
  return b;
}

template <class T>
hipError_t launch_adjoint_t(const InstDesc* d_desc, const InstDesc& h, int inst, const AdjScratch& sc, const T* f_n,
                            const T* lam_np1, T* lam_n, double* theta_bar, double* G_bar, hipStream_t s) {
  const unsigned gghost = (unsigned)((2 * h.nx + AB - 1) / AB);
  if (gghost > (unsigned)kAdjBlocks) return hipErrorInvalidValue;
  // fused pass: column blocks of at most FL - 4 columns (balanced), and row strips sized so that the tasks fit
  // in one round of resident wavefronts (as many per compute unit as the kernel's register use allows), at least
  // 4 rows
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    cus = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ? v : 256;
  }
  const bool ext = h.mrt || h.wall_mc;
  const int per_cu = ext ? fused_blocks_per_cu<true, T>() : fused_blocks_per_cu<false, T>();
  const int ncb = (h.nx + FL - 5) / (FL - 4);
  const int bw = (h.nx + ncb - 1) / ncb;
  const int nyf = h.ny - 2;
  const int strips = std::max(1, std::min(nyf, per_cu * cus / ncb));
  const int H = std::max(4, (nyf + strips - 1) / strips);
  const int ntasks = ncb * ((nyf + H - 1) / H);
  const unsigned gfused = (unsigned)std::min((ntasks + 7) / 8 * 8, kAdjBlocks);  // a multiple of 8
  const bool walls = h.periodic_y == 0;  // periodic rows have no ghost rows and no wetting
  if (walls) {
    hipLaunchKernelGGL(ka_wall_fwd<T>, dim3(gghost), dim3(AB), 0, s, d_desc, inst, f_n, sc);
  }
  if (ext)
    hipLaunchKernelGGL((ka_fused<true, T>), dim3(gfused), dim3(FL), 0, s, d_desc, inst, f_n, lam_np1, lam_n, sc, bw, ncb,
                       H, ntasks);
  else
    hipLaunchKernelGGL((ka_fused<false, T>), dim3(gfused), dim3(FL), 0, s, d_desc, inst, f_n, lam_np1, lam_n, sc, bw, ncb,
                       H, ntasks);
  if (walls) {
    hipLaunchKernelGGL(ka_ghost_adj, dim3(gghost), dim3(AB), 0, s, d_desc, inst, sc, theta_bar);
    hipLaunchKernelGGL(ka_wall_fix<T>, dim3((unsigned)((4 * h.nx + AB - 1) / AB)), dim3(AB), 0, s, d_desc, inst, lam_n,
                       sc);
  }
  hipLaunchKernelGGL(ka_finalize, dim3(1), dim3(AB), 0, s, sc, (int)gfused, walls ? (int)gghost : 0, G_bar);
  return hipGetLastError();
}

// Adjoint of the density readout rho = sum_i f_i of the streamed populations (fluid rows): every population of a
// node receives that node's dL/drho, lambda_i(x) = grad_rho(x). The accumulators theta_bar [2][nx] and G_bar [2]
// start at zero.
template <class T>
__global__ __launch_bounds__(AB) void ka_seed_rho(const double* __restrict__ grad_rho, T* __restrict__ lam,
                                                  double* __restrict__ theta_bar, double* __restrict__ G_bar,
                                                  int64_t nodes, int nx) {
  const int64_t k = (int64_t)blockIdx.x * AB + threadIdx.x;
  if (k < nodes) {
    const T g = (T)grad_rho[k];
#pragma unroll
    for (int i = 0; i < 9; ++i) lam[i * nodes + k] = g;
  }
  if (k < 2 * (int64_t)nx) theta_bar[k] = 0.0;
  if (k < 2) G_bar[k] = 0.0;
}

}  // namespace

hipError_t launch_adjoint_seed_rho(bool f32, const double* grad_rho, void* lam, double* theta_bar, double* G_bar,
                                   int nx, int nyf, hipStream_t s) {
  const int64_t nodes = (int64_t)nx * nyf;
  const int64_t work = std::max<int64_t>(nodes, 2 * (int64_t)nx);
  const dim3 grid((unsigned)((work + AB - 1) / AB));
  if (f32)
    hipLaunchKernelGGL(ka_seed_rho<float>, grid, dim3(AB), 0, s, grad_rho, (float*)lam, theta_bar, G_bar, nodes, nx);
  else
    hipLaunchKernelGGL(ka_seed_rho<double>, grid, dim3(AB), 0, s, grad_rho, (double*)lam, theta_bar, G_bar, nodes,
                       nx);
  return hipGetLastError();
}

hipError_t launch_adjoint(const InstDesc* d_desc, const InstDesc& h, int inst, const AdjScratch& sc, bool f32,
                          const void* f_n, const void* lam_np1, void* lam_n, double* theta_bar, double* G_bar,
                          hipStream_t s) {
  if (f32)
    return launch_adjoint_t<float>(d_desc, h, inst, sc, (const float*)f_n, (const float*)lam_np1, (float*)lam_n,
                                   theta_bar, G_bar, s);
  return launch_adjoint_t<double>(d_desc, h, inst, sc, (const double*)f_n, (const double*)lam_np1, (double*)lam_n,
                                  theta_bar, G_bar, s);
}

}  // namespace lbm
