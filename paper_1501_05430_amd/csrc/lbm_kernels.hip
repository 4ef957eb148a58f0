// HIP kernels of liblbm for gfx950 (MI355X): the fused pseudo-potential LB step and its diagnostics.
//
// Storage: the population buffers hold POST-COLLISION populations g_i(x) = f*_i(x) in SoA planes
// [9][ny-2][pitch]. The streamed populations of the next state are gathered on read,
// f_i(x) = g_i(x - e_i), with halfway bounce-back folded in: where x - e_i lies in a ghost row,
// f_i(x) = g_{opp(i)}(x). Every kernel that reads the state gathers this way; stores are then aligned and
// unshifted, so every wavefront writes whole 64-column runs of every plane.
//
// Step kernel (one launch per time step, no grid-wide dependency inside a step):
//  * A block of W wavefronts owns 64 W consecutive columns (aligned) x nrows rows and walks the rows upwards.
//    Each lane holds one column. A 3-row window of psi (Eq. 10) lives in registers; x-neighbours come from the
//    adjacent lanes (ds_bpermute) and, across wavefront boundaries, through a few LDS words with one barrier per
//    row. The two halo columns outside the block are gathered by the block's edge lanes.
//  * Row y is processed once row y+1 is in: the force (Eq. 9) uses the eight psi neighbours, the BGK-Guo
//    collision (Eq. 1-6 with diag(0,1,...,1)) runs in registers, and f* is stored in place.
//  * The ghost rows (Sec. 4, Eq. 19 and 21) are computed by the blocks that touch a wall, from the densities of
//    the boundary row (with its two neighbours) and of the second row.
//  * Each population is read once and written once per step (plus halo reads served by L2/MALL):
//    72 B (FP32) / 144 B (FP64) of HBM traffic per lattice update at the roofline.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lbm_internal.h"

namespace lbm {
namespace {

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

// ------------------------------------------------------------------------------------------------ EOS / psi
// Carnahan-Starling p(rho) and psi = sqrt(2 (p - rho/3) / G) (Eq. 10 with c = 1); the argument is clamped at 0
// (counted) where it is negative.

// FP64 mode: IEEE division and square root.
__device__ inline double psi_f64(const InstDesc& d, double rho, bool& clamped) {
  const double eta = d.eos_b4 * rho;
  const double om = 1.0 - eta;
  const double p = rho * d.RT * (1.0 + eta + eta * eta - eta * eta * eta) / (om * om * om) - d.eos_a * rho * rho;
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

// FP32 modes: below rho_fp64_below the EOS is evaluated in FP64 (vapour side of a large density ratio),
// elsewhere in FP32 with the hardware reciprocal and square root.
__device__ inline float psi_f32(const InstDesc& d, float rho, bool& clamped) {
  if (rho < (float)d.rho_fp64_below) {
    const double r = (double)rho;
    const double eta = d.eos_b4 * r;
    const double om = 1.0 - eta;
    const double p = r * d.RT * (1.0 + eta + eta * eta - eta * eta * eta) * rcp64(om * om * om) - d.eos_a * r * r;
    const double arg = d.two_over_Gpsi * (p - r * (1.0 / 3.0));
    clamped = arg < 0.0;
    return (float)sqrt64(arg);
  }
  const float eta = (float)d.eos_b4 * rho;
  const float om = 1.0f - eta;
  const float p = rho * (float)d.RT * (1.0f + eta + eta * eta - eta * eta * eta) * __builtin_amdgcn_rcpf(om * om * om) -
                  (float)d.eos_a * rho * rho;
  float arg = (float)d.two_over_Gpsi * (p - rho * (1.0f / 3.0f));
  clamped = arg < 0.0f;
  if (clamped) arg = 0.0f;
  return __builtin_amdgcn_sqrtf(arg);
}

__device__ inline double psi_eval(const InstDesc& d, double rho, bool& cl) { return psi_f64(d, rho, cl); }
__device__ inline float psi_eval(const InstDesc& d, float rho, bool& cl) { return psi_f32(d, rho, cl); }

// BGK collision with Guo forcing (Eq. 1-6; at tau = 1 this is the relaxation matrix diag(0,1,...,1) of Sec. 3.1):
//   v = (j + F/2)/rho, f*_i = f_i - (f_i - f_i^eq)/tau + (1 - 1/(2 tau)) w_i [3 (e_i - v) + 9 (e_i.v) e_i] . F,
// f_i^eq = w_i rho (1 + 3 e_i.v + 4.5 (e_i.v)^2 - 1.5 v^2). Populations may be stored shifted by w_i rho0:
// delta = rho - rho0 replaces rho in the zeroth-order term. Opposite directions share the even part
// (w [delta - 1.5 rho v^2 + 4.5 rho (e.v)^2 + pref (9 (e.v)(e.F) - 3 v.F)]) and differ in the sign of the odd
// part (w [3 rho e.v + 3 pref e.F]).
template <class C, bool TAU1>
__device__ inline void collide(const C (&f)[9], C rho, C delta, C Fx, C Fy, C inv_tau, C pref, C irho, C (&fs)[9]) {
  const C w0 = (C)(4.0 / 9.0), w1 = (C)(1.0 / 9.0), w2 = (C)(1.0 / 36.0);
  const C jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  const C jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  const C vx = (jx + (C)0.5 * Fx) * irho;
  const C vy = (jy + (C)0.5 * Fy) * irho;
  const C vF = vx * Fx + vy * Fy;
  const C eq0 = delta - (C)1.5 * rho * (vx * vx + vy * vy);  // zeroth + second-order isotropic part of f_eq
  const C fo0 = -(C)3 * pref * vF;                          // isotropic part of the forcing
  const C r45 = (C)4.5 * rho, r3 = (C)3 * rho, p9 = (C)9 * pref, p3 = (C)3 * pref;
  auto put = [&](int i, int o, C w, C eu, C eF) {
    const C se = eq0 + r45 * eu * eu;          // even part of f_eq / w
    const C sf = fo0 + p9 * eu * eF;           // even part of the forcing / w
    const C ae = r3 * eu, af = p3 * eF;        // odd parts
    if (TAU1) {
      fs[i] = w * ((se + sf) + (ae + af));
      fs[o] = w * ((se + sf) - (ae + af));
    } else {
      fs[i] = f[i] + (w * (se + ae) - f[i]) * inv_tau + w * (sf + af);
      fs[o] = f[o] + (w * (se - ae) - f[o]) * inv_tau + w * (sf - af);
    }
  };
  if (TAU1) fs[0] = w0 * (eq0 + fo0);
  else fs[0] = f[0] + (w0 * eq0 - f[0]) * inv_tau + w0 * fo0;
  put(1, 3, w1, vx, Fx);
  put(2, 4, w1, vy, Fy);
  put(5, 7, w2, vx + vy, Fx + Fy);
  put(6, 8, w2, vy - vx, Fy - Fx);
}

// Ghost density of Sec. 4 in FP64: Eq. 19 (iters == 0) or the iters-th iterate of Eq. 21 with the square root of
// Eq. 20. T is the tangential difference of the boundary row, D = rho_2 - rho_1. Clamped to [0, rho_cap_hi].
__device__ inline double ghost_density(double rL, double rR, double r1, double r2, double c, double cot, int iters,
                                       double cap_hi, bool& clamped) {
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
// header): f_i(x) = g_i(x - e_i), or g_{opp(i)}(x) where x - e_i is a ghost row (halfway bounce-back).
template <class S, class C>
__device__ inline void gather(const typename Gbl<S>::T* __restrict__ g, int64_t plane, int pitch, int nx, int ny,
                              int x, int y, C (&f)[9]) {
  typedef typename Gbl<S>::T GS;
  const int xl = x == 0 ? nx - 1 : x - 1, xr = x + 1 == nx ? 0 : x + 1;
  const bool bot = (y == 1), top = (y == ny - 2);
  const unsigned rc = (unsigned)((y - 1) * pitch);
  const unsigned rd = bot ? rc : rc - (unsigned)pitch;  // row below (unused at the bottom wall)
  const unsigned ru = top ? rc : rc + (unsigned)pitch;  // row above (unused at the top wall)
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

template <class C>
__device__ inline C sum9(const C (&f)[9]) {
  C s = f[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) s += f[i];
  return s;
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

// ------------------------------------------------------------------------------------------------ step kernel
template <class S, bool CHECK, bool TAU1, int W, bool PF>
__global__ __launch_bounds__(WAVE * W) void k_step(const InstDesc* __restrict__ descs,
                                                   const WaveTask* __restrict__ tasks, int ntasks, int flip,
                                                   WaveDiag* __restrict__ wdiag) {
  typedef typename ComputeOf<S>::type C;
  typedef typename Gbl<S>::T GS;
  const int task = (int)blockIdx.x;
  if (task >= ntasks) return;  // uniform over the block
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = uni((int)(threadIdx.x >> 6));
  const WaveTask t = tasks[task];
  const int inst = uni(t.inst);
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny, pitch = d.pitch, iters = d.wet_iters;
  const int64_t plane = d.plane;
  const int cur = d.cur ^ flip;
  const GS* __restrict__ gin = (const GS*)d.f[cur];
  GS* __restrict__ gout = (GS*)d.f[cur ^ 1];
  const GCD* __restrict__ cos_th = (const GCD*)d.cos_th;
  const GCD* __restrict__ cot_th = (const GCD*)d.cot_th;
  const int x0 = uni(t.x0), y0 = uni(t.y0), bw = uni(t.wh & 0xffff), nrows = uni(t.wh >> 16);
  const int ylast = y0 + nrows - 1;
  const C rho0 = (C)d.rho0;

  const int lx = wv * WAVE + lane;  // column offset inside the block
  const bool act = lx < bw;
  const int col = act ? x0 + lx : x0;
  const bool ledge = lx == 0, redge = lx == bw - 1;  // distinct lanes: blocks are at least 2 columns wide
  const bool edge = ledge || redge;
  const int hcol = wrapx(ledge ? x0 - 1 : x0 + bw, nx);      // halo column gathered by an edge lane
  const int ocol = wrapx(ledge ? x0 - 2 : x0 + bw + 1, nx);  // next column out (ghost tangential difference)
  const int srcL = lane > 0 ? lane - 1 : 0, srcR = lane < WAVE - 1 ? lane + 1 : WAVE - 1;

  // (left, right) neighbours of a per-lane value: adjacent lanes, the adjacent wavefront's edge lane through LDS,
  // or the halo value h that the block's edge lanes hold. One barrier per call when W > 1 (uniform over the block).
  __shared__ C xs[2][W][2];
  int par = 0;
  auto xchg = [&](C v, C h, C& l, C& r) {
    if (W > 1) {
      if (lane == 0) xs[par][wv][0] = v;
      if (lane == WAVE - 1) xs[par][wv][1] = v;
      __syncthreads();
    }
    const C sl = __shfl(v, srcL, WAVE), sr = __shfl(v, srcR, WAVE);
    C fromL = sl, fromR = sr;
    if (W > 1) {
      if (lane == 0) fromL = xs[par][wv > 0 ? wv - 1 : 0][1];
      if (lane == WAVE - 1) fromR = xs[par][wv < W - 1 ? wv + 1 : 0][0];
    }
    l = ledge ? h : fromL;
    r = redge ? h : fromR;
    par ^= 1;
  };

  // Row y (fluid): own column populations, density and psi; edge lanes also density and psi of the halo column.
  auto produce = [&](int y, C (&f)[9], C& rho, C& psi, C& hrho, C& hpsi, bool& cl) {
    if (act) {
      gather<S, C>(gin, plane, pitch, nx, ny, col, y, f);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = (C)0;
    }
    rho = rho0 + sum9(f);
    psi = psi_eval(d, rho, cl);
    hrho = (C)0;
    hpsi = (C)0;
    if (edge) {
      C g[9];
      gather<S, C>(gin, plane, pitch, nx, ny, hcol, y, g);
      hrho = rho0 + sum9(g);
      bool dm;
      hpsi = psi_eval(d, hrho, dm);
    }
  };

  int psi_cl = 0, ghost_cl = 0, nonfin = 0;
  double mass = 0.0;

  // Ghost row beside wall `wall` (0 bottom, 1 top), Sec. 4: from the boundary row yb (densities r1, halo hr1) and
  // the second row (r2, halo hr2). Returns the ghost density and psi of the own column and the halo psi.
  auto ghost = [&](int wall, int yb, C r1, C r2, C hr1, C hr2, C& g_rho, C& g_psi, C& gh_psi) {
    C L, R;
    xchg(r1, hr1, L, R);
    C ro = (C)0;
    if (edge) {
      C g[9];
      gather<S, C>(gin, plane, pitch, nx, ny, ocol, yb, g);
      ro = rho0 + sum9(g);
    }
    const int base = wall * nx;
    double r0 = 0.0, rh0 = 0.0;
    bool gc = false, gch = false;
    if (act)
      r0 = ghost_density((double)L, (double)R, (double)r1, (double)r2, cos_th[base + col], cot_th[base + col], iters,
                         d.rho_cap_hi, gc);
    if (edge) {
      const double hl = ledge ? (double)ro : (double)r1;  // density at (halo column - 1)
      const double hr = ledge ? (double)r1 : (double)ro;  // density at (halo column + 1)
      rh0 = ghost_density(hl, hr, (double)hr1, (double)hr2, cos_th[base + hcol], cot_th[base + hcol], iters,
                          d.rho_cap_hi, gch);
    }
    if (CHECK && act && gc) ghost_cl++;
    bool dm;
    g_rho = (C)r0;
    g_psi = (C)psi_eval(d, r0, dm);
    gh_psi = (C)psi_eval(d, rh0, dm);
  };

  const C A = (C)d.A, Gf = (C)d.G_f, inv_tau = (C)d.inv_tau, pref = (C)d.force_pref;
  const C bfx = (C)d.body_fx, bfy = (C)d.body_fy;
  const C k1 = (C)(1.0 / 3.0), k2 = (C)(1.0 / 12.0);

  // Top wall: the top strip computes the ghost row's psi (with its neighbours) up front, so that the row loop
  // itself carries no wall code.
  C tg = (C)0, tgL = (C)0, tgR = (C)0;
  if (ylast == ny - 2) {
    C f1[9], f2[9], r1, r2, h1, h2, p1, p2, hp1, hp2, g_rho, hg;
    bool dm;
    produce(ny - 2, f1, r1, p1, h1, hp1, dm);
    produce(ny - 3, f2, r2, p2, h2, hp2, dm);
    ghost(1, ny - 2, r1, r2, h1, h2, g_rho, tg, hg);
    xchg(tg, hg, tgL, tgR);
  }

  // window: rows (m, c, n) = (y-1, y, y+1) when row y is processed
  C fc[9], fn[9], fp[9];
  C rm, rc, rn, pm, pc, pn, pmL, pmR, pcL, pcR, pnL, pnR;
  bool cl_c = false, cl_n = false;
  {
    C hpm, hpc, hpn, hrm, hrc, hrn;
    if (y0 == 1) {
      produce(1, fc, rc, pc, hrc, hpc, cl_c);
      produce(2, fn, rn, pn, hrn, hpn, cl_n);
      ghost(0, 1, rc, rn, hrc, hrn, rm, pm, hpm);
    } else {
      C fm[9];
      bool dm;
      produce(y0 - 1, fm, rm, pm, hrm, hpm, dm);
      produce(y0, fc, rc, pc, hrc, hpc, cl_c);
      if (y0 + 1 <= ny - 2) produce(y0 + 1, fn, rn, pn, hrn, hpn, cl_n);
    }
    xchg(pm, hpm, pmL, pmR);
    xchg(pc, hpc, pcL, pcR);
    if (y0 + 1 <= ny - 2) {
      xchg(pn, hpn, pnL, pnR);
    } else {
      pn = tg; pnL = tgL; pnR = tgR;
      cl_n = false;
    }
  }
  // rows read by the strip: y0-1 .. min(ylast+1, ny-2); with PF the populations of row y+2 are in flight while
  // row y is processed
  const int yread = ylast + 1 <= ny - 2 ? ylast + 1 : ny - 2;
  if (PF && act && y0 + 2 <= yread) gather<S, C>(gin, plane, pitch, nx, ny, col, y0 + 2, fp);

  for (int y = y0;; ++y) {
    if (act) {
      // Interaction force, Eq. 9: F = -G_f [ (A/2) sum w psi_n^2 e + (1 - A) psi sum w psi_n e ].
      const C spx = k1 * (pcR - pcL) + k2 * ((pnR - pnL) + (pmR - pmL));
      const C spy = k1 * (pn - pm) + k2 * ((pnR + pnL) - (pmR + pmL));
      const C sux = k1 * (pcR * pcR - pcL * pcL) + k2 * ((pnR * pnR - pnL * pnL) + (pmR * pmR - pmL * pmL));
      const C suy = k1 * (pn * pn - pm * pm) + k2 * ((pnR * pnR + pnL * pnL) - (pmR * pmR + pmL * pmL));
      const C Fx = -Gf * ((C)0.5 * A * sux + ((C)1 - A) * pc * spx) + bfx;
      const C Fy = -Gf * ((C)0.5 * A * suy + ((C)1 - A) * pc * spy) + bfy;
      C fs[9];
      collide<C, TAU1>(fc, rc, rc - rho0, Fx, Fy, inv_tau, pref, (C)1 / rc, fs);
      const unsigned off = (unsigned)((y - 1) * pitch + col);
#pragma unroll
      for (int i = 0; i < 9; ++i) ((GS*)(gout + i * plane))[off] = (S)fs[i];
      if (CHECK) {
        double m = (double)fc[0];
#pragma unroll
        for (int i = 1; i < 9; ++i) m += (double)fc[i];
        mass += m + d.rho0;
        nonfin += isfinite(rc) ? 0 : 1;
        psi_cl += cl_c ? 1 : 0;
      }
    }
    if (y == ylast) break;
    // slide the window up one row
    rm = rc; pm = pc; pmL = pcL; pmR = pcR;
    rc = rn; pc = pn; pcL = pnL; pcR = pnR;
    cl_c = cl_n;
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = fn[i];
    if (y + 2 <= ny - 2) {
      if (PF) {
#pragma unroll
        for (int i = 0; i < 9; ++i) fn[i] = act ? fp[i] : (C)0;
        if (act && y + 3 <= yread) gather<S, C>(gin, plane, pitch, nx, ny, col, y + 3, fp);
      } else if (act) {
        gather<S, C>(gin, plane, pitch, nx, ny, col, y + 2, fn);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) fn[i] = (C)0;
      }
      rn = rho0 + sum9(fn);
      pn = psi_eval(d, rn, cl_n);
      C hpn = (C)0;
      if (edge) {
        C g[9];
        gather<S, C>(gin, plane, pitch, nx, ny, hcol, y + 2, g);
        bool dm;
        hpn = psi_eval(d, rho0 + sum9(g), dm);
      }
      xchg(pn, hpn, pnL, pnR);
    } else {
      pn = tg; pnL = tgL; pnR = tgR;
      cl_n = false;
    }
  }

  if (CHECK) {
    __shared__ double sm[W];
    __shared__ int si[W][3];
    mass = wave_sum(mass);
    nonfin = wave_sum(nonfin);
    psi_cl = wave_sum(psi_cl);
    ghost_cl = wave_sum(ghost_cl);
    if (lane == 0) {
      sm[wv] = mass;
      si[wv][0] = nonfin;
      si[wv][1] = psi_cl;
      si[wv][2] = ghost_cl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      WaveDiag w;
      w.mass = 0.0;
      w.nonfinite = w.psi_clamps = w.ghost_clamps = w.pad = 0;
      for (int k = 0; k < W; ++k) {
        w.mass += sm[k];
        w.nonfinite += si[k][0];
        w.psi_clamps += si[k][1];
        w.ghost_clamps += si[k][2];
      }
      wdiag[task] = w;
    }
  }
}

// One block per selected instance: fold its waves' diagnostics in a fixed order (deterministic).
__global__ __launch_bounds__(BLOCK) void k_finalize_diag(const int32_t* __restrict__ inst_first, int inst0,
                                                         const WaveDiag* __restrict__ wdiag,
                                                         InstDiag* __restrict__ idiag) {
  const int inst = inst0 + (int)blockIdx.x;
  const int a = inst_first[inst], b = inst_first[inst + 1];
  double m = 0.0;
  long long nf = 0, pcl = 0, gcl = 0;
  for (int i = a + (int)threadIdx.x; i < b; i += BLOCK) {
    const WaveDiag w = wdiag[i];
    m += w.mass;
    nf += w.nonfinite;
    pcl += w.psi_clamps;
    gcl += w.ghost_clamps;
  }
  __shared__ double sm[BLOCK];
  __shared__ long long s1[BLOCK], s2[BLOCK], s3[BLOCK];
  sm[threadIdx.x] = m;
  s1[threadIdx.x] = nf;
  s2[threadIdx.x] = pcl;
  s3[threadIdx.x] = gcl;
  __syncthreads();
  for (int o = BLOCK / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sm[threadIdx.x] += sm[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
      s3[threadIdx.x] += s3[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    InstDiag& g = idiag[inst];
    g.mass = sm[0];
    g.checks += 1;
    g.nonfinite += s1[0];
    g.psi_clamps += s2[0];
    g.ghost_clamps += s3[0];
  }
}

// ------------------------------------------------------------------------------------------------ init
// Initial density rho = rho_v + (rho_l - rho_v)(1 - tanh(2 (r - R)/W))/2, max over droplets, into scratch
// [ny][nx] (fluid rows).
__global__ __launch_bounds__(BLOCK) void k_init_rho(const InstDesc* __restrict__ descs, int inst,
                                                    const double* __restrict__ drops, int ndrops, double width,
                                                    double rho_l, double rho_v, double* __restrict__ rho) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, nyf = d.ny - 2;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= (int64_t)nx * nyf) return;
  const int x = (int)(k % nx);
  const int y = (int)(k / nx) + 1;
  double r = rho_v;
  for (int j = 0; j < ndrops; ++j) {
    double dx = (double)x - drops[3 * j];
    dx -= (double)nx * floor(dx / (double)nx + 0.5);
    const double dy = (double)y - drops[3 * j + 1];
    const double dist = sqrt(dx * dx + dy * dy);
    const double v = rho_v + (rho_l - rho_v) * 0.5 * (1.0 - tanh(2.0 * (dist - drops[3 * j + 2]) / width));
    if (v > r) r = v;
  }
  rho[(int64_t)y * nx + x] = r;
}

__device__ constexpr int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Rest state f_i = w_i rho stored as post-collision populations: g_i(x) = f_i(x + e_i), or f_{opp(i)}(x) where
// x + e_i is a ghost row (the inverse of the gather).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_init_pops(const InstDesc* __restrict__ descs, int inst,
                                                     const double* __restrict__ rho) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= (int64_t)nx * (ny - 2)) return;
  const int x = (int)(k % nx);
  const int y = (int)(k / nx) + 1;
  S* g = (S*)d.f[d.cur];
  const int64_t idx = (int64_t)(y - 1) * d.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int yd = y + kEY[i];
    const double r = (yd < 1 || yd > ny - 2) ? rho[(int64_t)y * nx + x] : rho[(int64_t)yd * nx + wrapx(x + kEX[i], nx)];
    g[i * d.plane + idx] = (S)(kW[i] * r - kW[i] * d.rho0);
  }
}

// ------------------------------------------------------------------------------------------------ wetting
// Ghost rows of the current state (the step kernel's arithmetic), into d.ghost[2][nx].
template <class S>
__global__ __launch_bounds__(BLOCK) void k_wetting(const InstDesc* __restrict__ descs, int inst) {
  typedef typename ComputeOf<S>::type C;
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int t = (int)(blockIdx.x * BLOCK + threadIdx.x);
  if (t >= 2 * nx) return;
  const int wall = t / nx, x = t % nx;
  const typename Gbl<S>::T* g = (const typename Gbl<S>::T*)d.f[d.cur];
  const C rho0 = (C)d.rho0;
  const int r1 = wall == 0 ? 1 : ny - 2, r2 = wall == 0 ? 2 : ny - 3;
  auto dens = [&](int y, int xx) -> C {
    C f[9];
    gather<S, C>(g, d.plane, d.pitch, nx, ny, xx, y, f);
    return rho0 + sum9(f);
  };
  const C rL = dens(r1, wrapx(x - 1, nx)), rR = dens(r1, wrapx(x + 1, nx));
  const C rc = dens(r1, x), rs = dens(r2, x);
  bool gc;
  d.ghost[wall * nx + x] = ghost_density((double)rL, (double)rR, (double)rc, (double)rs, d.cos_th[wall * nx + x],
                                         d.cot_th[wall * nx + x], d.wet_iters, d.rho_cap_hi, gc);
}

// ------------------------------------------------------------------------------------------------ readout
// FP64 density [ny][nx]: fluid rows sum the gathered populations, ghost rows come from d.ghost (k_wetting first).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_get_rho(const InstDesc* __restrict__ descs, int inst,
                                                   double* __restrict__ dst) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= (int64_t)nx * ny) return;
  const int x = (int)(k % nx), y = (int)(k / nx);
  if (y == 0) { dst[k] = d.ghost[x]; return; }
  if (y == ny - 1) { dst[k] = d.ghost[nx + x]; return; }
  double f[9];
  gather<S, double>((const typename Gbl<S>::T*)d.f[d.cur], d.plane, d.pitch, nx, ny, x, y, f);
  dst[k] = sum9(f) + d.rho0;
}

// Population planes [q0, q1) of the current state as FP64 [q1-q0][ny-2][nx] (unshifted).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_get_pops(const InstDesc* __restrict__ descs, int inst, int q0, int q1,
                                                    double* __restrict__ dst) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int64_t n = (int64_t)nx * (ny - 2);
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= n) return;
  const int x = (int)(k % nx), y = (int)(k / nx) + 1;
  double f[9];
  gather<S, double>((const typename Gbl<S>::T*)d.f[d.cur], d.plane, d.pitch, nx, ny, x, y, f);
  for (int i = q0; i < q1; ++i) dst[(i - q0) * n + k] = f[i] + kW[i] * d.rho0;
}

// Set stored plane q from a physical population plane p ([ny-2][nx], FP64): p == q writes the nodes whose
// destination x + e_q is a fluid node (g_q(x) = f_q(x + e_q)); p == opp(q) writes the nodes whose destination is
// a ghost row (g_q(x) = f_{opp(q)}(x)).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_set_plane(const InstDesc* __restrict__ descs, int inst, int q, int p,
                                                     const double* __restrict__ src) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, ny = d.ny;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= (int64_t)nx * (ny - 2)) return;
  const int x = (int)(k % nx), y = (int)(k / nx) + 1;
  const int yd = y + kEY[q];
  const bool wall = yd < 1 || yd > ny - 2;
  S* g = (S*)d.f[d.cur];
  const int64_t idx = (int64_t)q * d.plane + (int64_t)(y - 1) * d.pitch + x;
  if (p == q && !wall) g[idx] = (S)(src[(int64_t)(yd - 1) * nx + wrapx(x + kEX[q], nx)] - kW[q] * d.rho0);
  if (p == kOPP[q] && wall) g[idx] = (S)(src[k] - kW[q] * d.rho0);
}

// FP64 mass: every stored post-collision population is some node's population after streaming, so the mass is
// the plain sum of the stored values. Per-block partial sums (grid-stride, fixed order), reduced on the host.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_mass(const InstDesc* __restrict__ descs, int inst,
                                                double* __restrict__ partials) {
  const InstDesc& d = descs[inst];
  const int nx = d.nx, nyf = d.ny - 2;
  const int64_t n = (int64_t)nx * nyf;
  const S* g = (const S*)d.f[d.cur];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < n; k += (int64_t)gridDim.x * BLOCK) {
    const int x = (int)(k % nx), yf = (int)(k / nx);
    const int64_t idx = (int64_t)yf * d.pitch + x;
    double s = (double)g[idx];
#pragma unroll
    for (int i = 1; i < 9; ++i) s += (double)g[i * d.plane + idx];
    acc += s + d.rho0;
  }
  __shared__ double sm[BLOCK];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int o = BLOCK / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

// ------------------------------------------------------------------------------------------------ contact angle
// min / max of rho over the box (per-block partials: [2 * nblocks], min then max).
__global__ __launch_bounds__(BLOCK) void k_minmax(const double* __restrict__ rho, int nx, int bx0, int bx1,
                                                  int by0, int by1, double* __restrict__ partials) {
  const int bw = bx1 - bx0;
  const int64_t n = (int64_t)bw * (by1 - by0);
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < n; k += (int64_t)gridDim.x * BLOCK) {
    const double v = rho[(int64_t)(by0 + k / bw) * nx + bx0 + k % bw];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  __shared__ double a[BLOCK], b[BLOCK];
  a[threadIdx.x] = lo;
  b[threadIdx.x] = hi;
  __syncthreads();
  for (int o = BLOCK / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      a[threadIdx.x] = fmin(a[threadIdx.x], a[threadIdx.x + o]);
      b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = a[0];
    partials[gridDim.x + blockIdx.x] = b[0];
  }
}

// Moments of the rho_mid crossing points for the algebraic circle fit, coordinates shifted by (sx, sy):
// {n, Sx, Sy, Sxx, Syy, Sxy, Sxxx, Sxyy, Sxxy, Syyy}, per block ([10][nblocks]).
__device__ inline void add_point(double px, double py, double (&m)[kMeasureMoments]) {
  m[0] += 1.0;
  m[1] += px;
  m[2] += py;
  m[3] += px * px;
  m[4] += py * py;
  m[5] += px * py;
  m[6] += px * px * px;
  m[7] += px * py * py;
  m[8] += px * px * py;
  m[9] += py * py * py;
}

__global__ __launch_bounds__(BLOCK) void k_ca_moments(const double* __restrict__ rho, int nx, int ny, int bx0,
                                                      int bx1, int by0, int by1, int wall, double mid, double sx,
                                                      double sy, double* __restrict__ partials) {
  const int bw = bx1 - bx0;
  const int64_t n = (int64_t)bw * (by1 - by0);
  const double yw = wall == 0 ? 0.5 : (double)ny - 1.5;
  double m[kMeasureMoments];
#pragma unroll
  for (int i = 0; i < kMeasureMoments; ++i) m[i] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < n; k += (int64_t)gridDim.x * BLOCK) {
    const int x = bx0 + (int)(k % bw), y = by0 + (int)(k / bw);
    const double a = rho[(int64_t)y * nx + x];
    if (x + 1 < bx1) {
      const double b = rho[(int64_t)y * nx + x + 1];
      if ((a < mid) != (b < mid)) {
        const double px = (double)x + (mid - a) / (b - a), py = (double)y;
        if (wall == 0 ? py >= yw + 3.0 : py <= yw - 3.0) add_point(px - sx, py - sy, m);
      }
    }
    if (y + 1 < by1) {
      const double b = rho[(int64_t)(y + 1) * nx + x];
      if ((a < mid) != (b < mid)) {
        const double px = (double)x, py = (double)y + (mid - a) / (b - a);
        if (wall == 0 ? py >= yw + 3.0 : py <= yw - 3.0) add_point(px - sx, py - sy, m);
      }
    }
  }
  __shared__ double sm[BLOCK];
  for (int j = 0; j < kMeasureMoments; ++j) {
    sm[threadIdx.x] = m[j];
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) partials[j * gridDim.x + blockIdx.x] = sm[0];
    __syncthreads();
  }
}

__global__ void k_zero_diag(InstDiag* __restrict__ g, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) {
    InstDiag z = {};
    g[i] = z;
  }
}

__global__ void k_set_cur(InstDesc* __restrict__ d, int inst, int cur) {
  if (threadIdx.x == 0) d[inst].cur = cur;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

template <class S, bool CHECK, bool TAU1, bool PF>
void launch_step_w(int waves, unsigned grid, hipStream_t s, const InstDesc* d_desc, const WaveTask* d_tasks,
                   int ntasks, int flip, WaveDiag* d_wdiag) {
  switch (waves) {
    case 1: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 1, PF>), dim3(grid), dim3(WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
    case 2: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 2, PF>), dim3(grid), dim3(2 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
    case 4: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 4, PF>), dim3(grid), dim3(4 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
    default: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 8, PF>), dim3(grid), dim3(8 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
  }
}

template <class S, bool PF>
void launch_step_s(bool check, bool tau1, int waves, unsigned grid, hipStream_t s, const InstDesc* d_desc,
                   const WaveTask* d_tasks, int ntasks, int flip, WaveDiag* d_wdiag) {
  if (check) {
    if (tau1) launch_step_w<S, true, true, PF>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
    else launch_step_w<S, true, false, PF>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
  } else {
    if (tau1) launch_step_w<S, false, true, PF>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
    else launch_step_w<S, false, false, PF>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------------ launchers
hipError_t launch_step(int storage, bool check, bool tau1, int waves, bool prefetch, const InstDesc* d_desc,
                       const WaveTask* d_tasks, int ntasks, int flip, WaveDiag* d_wdiag, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  const unsigned grid = (unsigned)ntasks;
  if (storage == STORE_F64) {
    if (prefetch) launch_step_s<double, true>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
    else launch_step_s<double, false>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
  } else {
    if (prefetch) launch_step_s<float, true>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
    else launch_step_s<float, false>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
  }
  return hipGetLastError();
}

hipError_t launch_finalize_diag(const WaveTask*, const int32_t* d_inst_first, int ninst_sel, int inst0,
                                const WaveDiag* d_wdiag, InstDiag* d_idiag, const InstDesc*, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_diag, dim3(ninst_sel), dim3(BLOCK), 0, s, d_inst_first, inst0, d_wdiag, d_idiag);
  return hipGetLastError();
}

hipError_t launch_init_droplets(int storage, const InstDesc* d_desc, int inst, int ny_fluid, int nx,
                                const double* d_drops, int ndrops, double width, double rho_l, double rho_v,
                                double* d_rho_scratch, hipStream_t s) {
  const unsigned g = blocks_for((int64_t)nx * ny_fluid);
  hipLaunchKernelGGL(k_init_rho, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, d_drops, ndrops, width, rho_l, rho_v,
                     d_rho_scratch);
  if (storage == STORE_F64) hipLaunchKernelGGL(k_init_pops<double>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, d_rho_scratch);
  else hipLaunchKernelGGL(k_init_pops<float>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, d_rho_scratch);
  return hipGetLastError();
}

hipError_t launch_wetting(int storage, const InstDesc* d_desc, int inst, int nx, hipStream_t s) {
  const unsigned g = blocks_for(2 * (int64_t)nx);
  if (storage == STORE_F64) hipLaunchKernelGGL(k_wetting<double>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst);
  else hipLaunchKernelGGL(k_wetting<float>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst);
  return hipGetLastError();
}

hipError_t launch_get_rho(int storage, const InstDesc* d_desc, int inst, int nx, int ny, double* d_dst,
                          hipStream_t s) {
  const unsigned g = blocks_for((int64_t)nx * ny);
  if (storage == STORE_F64) hipLaunchKernelGGL(k_get_rho<double>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, d_dst);
  else hipLaunchKernelGGL(k_get_rho<float>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, d_dst);
  return hipGetLastError();
}

hipError_t launch_get_pops(int storage, const InstDesc* d_desc, int inst, int nx, int ny, int q0, int q1,
                           double* d_dst, hipStream_t s) {
  const unsigned g = blocks_for((int64_t)nx * (ny - 2));
  if (storage == STORE_F64)
    hipLaunchKernelGGL(k_get_pops<double>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, q0, q1, d_dst);
  else
    hipLaunchKernelGGL(k_get_pops<float>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, q0, q1, d_dst);
  return hipGetLastError();
}

hipError_t launch_set_plane(int storage, const InstDesc* d_desc, int inst, int nx, int ny, int q, int p,
                            const double* d_src, hipStream_t s) {
  const unsigned g = blocks_for((int64_t)nx * (ny - 2));
  if (storage == STORE_F64)
    hipLaunchKernelGGL(k_set_plane<double>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, q, p, d_src);
  else
    hipLaunchKernelGGL(k_set_plane<float>, dim3(g), dim3(BLOCK), 0, s, d_desc, inst, q, p, d_src);
  return hipGetLastError();
}

hipError_t launch_mass(int storage, const InstDesc* d_desc, int inst, int, int, double* d_partials, int nblocks,
                       hipStream_t s) {
  if (storage == STORE_F64) hipLaunchKernelGGL(k_mass<double>, dim3(nblocks), dim3(BLOCK), 0, s, d_desc, inst, d_partials);
  else hipLaunchKernelGGL(k_mass<float>, dim3(nblocks), dim3(BLOCK), 0, s, d_desc, inst, d_partials);
  return hipGetLastError();
}

hipError_t launch_minmax(const double* d_rho, int nx, int, const int32_t* box, double* d_partials, int nblocks,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_minmax, dim3(nblocks), dim3(BLOCK), 0, s, d_rho, nx, box[0], box[1], box[2], box[3], d_partials);
  return hipGetLastError();
}

hipError_t launch_ca_moments(const double* d_rho, int nx, int ny, const int32_t* box, int wall, double rho_mid,
                             double shift_x, double shift_y, double* d_partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_ca_moments, dim3(nblocks), dim3(BLOCK), 0, s, d_rho, nx, ny, box[0], box[1], box[2], box[3],
                     wall, rho_mid, shift_x, shift_y, d_partials);
  return hipGetLastError();
}

hipError_t launch_zero_diag(InstDiag* d_idiag, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_diag, dim3((n + 255) / 256), dim3(256), 0, s, d_idiag, n);
  return hipGetLastError();
}

hipError_t launch_set_cur(InstDesc* d_desc, int inst, int cur, hipStream_t s) {
  hipLaunchKernelGGL(k_set_cur, dim3(1), dim3(64), 0, s, d_desc, inst, cur);
  return hipGetLastError();
}

hipError_t launch_adjoint(const InstDesc*, const InstDesc&, int, const AdjScratch&, const double*, const double*,
                          double*, double*, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace lbm
