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

#include <type_traits>
#include <math.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

// ------------------------------------------------------------------------------------------------ step kernel
template <class S, bool CHECK, bool TAU1, int W, bool PF, bool DOWN, bool MIX>
__global__ __launch_bounds__(WAVE * W) void k_step(const InstDesc* __restrict__ descs,
                                                   const WaveTask* __restrict__ tasks, int ntasks, int flip,
                                                   WaveDiag* __restrict__ wdiag) {
  typedef typename ComputeOf<S>::type C;
  typedef typename Gbl<S>::T GS;
  static_assert(!MIX || std::is_same<S, float>::value, "the mixed arithmetic is a form of FP32 storage");
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
  const bool py = d.periodic_y != 0;  // rows wrap around, no walls
  const bool mcw = d.wall_mc != 0;    // Martys-Chen walls: solid rows with the fluid-solid force of Eq. 14
  auto wrapy = [&](int y) { return y < 1 ? y + (ny - 2) : (y > ny - 2 ? y - (ny - 2) : y); };

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
      gather<S, C>(gin, plane, pitch, nx, ny, col, wrapy(y), f, py);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = (C)0;
    }
    rho = rho0 + sum9(f);
    psi = node_psi<MIX>(d, rho, cl);
    hrho = (C)0;
    hpsi = (C)0;
    if (edge) {
      C g[9];
      gather<S, C>(gin, plane, pitch, nx, ny, hcol, wrapy(y), g, py);
      hrho = rho0 + sum9(g);
      bool dm;
      hpsi = node_psi<MIX>(d, hrho, dm);
    }
  };

  int psi_cl = 0, ghost_cl = 0, nonfin = 0;
  double mass = 0.0;

  // Ghost row beside wall `wall` (0 bottom, 1 top), Sec. 4: from the boundary row yb (densities r1, halo hr1) and
  // the second row (r2, halo hr2). Returns the ghost density and psi of the own column and the halo psi.
  auto ghost = [&](int wall, int yb, C r1, C r2, C hr1, C hr2, C& g_rho, C& g_psi, C& gh_psi) {
    if (mcw) {  // solid wall rows (Eq. 14 mode): absent from the fluid-fluid force; uniform over the block
      g_rho = g_psi = gh_psi = (C)0;
      return;
    }
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

  const C A = (C)d.A, inv_tau = (C)d.inv_tau, pref = (C)d.force_pref;
  // MRT collision with the surface-tension source (never in the tau = 1 BGK specialisation)
  const bool mrt = !TAU1 && d.mrt != 0, kap = mrt && d.kq != 0.0;
  const C s_e = (C)d.s_e, s_eps = (C)d.s_eps, s_q = (C)d.s_q, kq = (C)d.kq;
  const C gwb = (C)d.gw_half[0], gwt = (C)d.gw_half[1];  // G_w / 2 of the bottom and top wall

  // The strip's rows are walked upwards (DOWN = false) or downwards. Consecutive launches alternate, so each
  // launch first reads the rows that the previous one wrote last, while they are still in the memory-side cache.
  // Below, "behind", "current" and "ahead" are rows in the walking direction; the force maps them back to the rows
  // below (y - 1) and above (y + 1).
  constexpr int st = DOWN ? -1 : 1;
  const int ystart = DOWN ? ylast : y0, yend = DOWN ? y0 : ylast;
  auto fluid_row = [&](int y) { return py || (y >= 1 && y <= ny - 2); };
  const bool wall_start = !py && (DOWN ? (ylast == ny - 2) : (y0 == 1));  // a wall behind the walk's first row
  const bool wall_end = !py && (DOWN ? (y0 == 1) : (ylast == ny - 2));     // a wall ahead of the walk's last row

  // The far wall: its ghost row's psi (with its neighbours) is computed up front, so that the row loop itself
  // carries no wall code.
  C tg = (C)0, tgL = (C)0, tgR = (C)0;
  if (wall_end) {
    const int yb = DOWN ? 1 : ny - 2, y2 = DOWN ? 2 : ny - 3;  // boundary row and second row of that wall
    C f1[9], f2[9], r1, r2, h1, h2, p1, p2, hp1, hp2, g_rho, hg;
    bool dm;
    produce(yb, f1, r1, p1, h1, hp1, dm);
    produce(y2, f2, r2, p2, h2, hp2, dm);
    ghost(DOWN ? 0 : 1, yb, r1, r2, h1, h2, g_rho, tg, hg);
    xchg(tg, hg, tgL, tgR);
  }

  // window: rows (b, c, a) = (y - st, y, y + st) when row y is processed
  C fc[9], fn[9], fp[9];
  C rb, rc, ra, pb, pc, pa, pbL, pbR, pcL, pcR, paL, paR;
  bool cl_c = false, cl_a = false;
  {
    C hpb, hpc, hpa, hrb, hrc, hra;
    if (wall_start) {
      produce(ystart, fc, rc, pc, hrc, hpc, cl_c);
      produce(ystart + st, fn, ra, pa, hra, hpa, cl_a);
      ghost(DOWN ? 1 : 0, ystart, rc, ra, hrc, hra, rb, pb, hpb);
    } else {
      C fb[9];
      bool dm;
      produce(ystart - st, fb, rb, pb, hrb, hpb, dm);
      produce(ystart, fc, rc, pc, hrc, hpc, cl_c);
      if (fluid_row(ystart + st)) produce(ystart + st, fn, ra, pa, hra, hpa, cl_a);
    }
    xchg(pb, hpb, pbL, pbR);
    xchg(pc, hpc, pcL, pcR);
    if (fluid_row(ystart + st)) {
      xchg(pa, hpa, paL, paR);
    } else {
      pa = tg; paL = tgL; paR = tgR;
      cl_a = false;
    }
  }
  // rows read by the strip: ystart - st .. yend + st, clipped to the fluid rows (wrapped when periodic); with PF
  // the populations of row y + 2 st are in flight while row y is processed
  const int yread = DOWN ? (y0 - 1 >= 1 ? y0 - 1 : 1) : (ylast + 1 <= ny - 2 ? ylast + 1 : ny - 2);
  auto readable = [&](int y) {
    if (py) return (y - ystart) * st <= (yend - ystart) * st + 1;
    return DOWN ? y >= yread : y <= yread;
  };
  if (PF && act && readable(ystart + 2 * st))
    gather<S, C>(gin, plane, pitch, nx, ny, col, wrapy(ystart + 2 * st), fp, py);

  for (int y = ystart;; y += st) {
    if (act) {
      // psi of the rows below (m) and above (n) row y
      const C pm = DOWN ? pa : pb, pmL = DOWN ? paL : pbL, pmR = DOWN ? paR : pbR;
      const C pn = DOWN ? pb : pa, pnL = DOWN ? pbL : paL, pnR = DOWN ? pbR : paR;
      // Interaction force, Eq. 9: F = -G_f [ (A/2) sum w psi_n^2 e + (1 - A) psi sum w psi_n e ] (plus the body
      // force), then the collision; for MIX the force, velocity, equilibrium and forcing in FP64
      C fs[9];
      if constexpr (MIX) {
        double Fx, Fy;
        hybrid_force<double>(d, pc, pcL, pcR, pm, pmL, pmR, pn, pnL, pnR, Fx, Fy);
        // Eq. 14 next to a flat solid row: sum_a w_a S(x + e_a) e_a = (0, -1/2) below, (0, 1/2) above
        if (mcw) {
          if (y == 1) Fy = Fy + d.gw_half[0] * (double)pc;
          if (y == ny - 2) Fy = Fy - d.gw_half[1] * (double)pc;
        }
        if (mrt) {
          double fd[9], fsd[9], qxx = 0.0, qyy = 0.0, qxy = 0.0;
#pragma unroll
          for (int i = 0; i < 9; ++i) fd[i] = (double)fc[i];
          const double r = (double)rc;
          if (kap) qtensor<double>(pc, pcL, pcR, pn, pnL, pnR, pm, pmL, pmR, d.A, d.kq, qxx, qyy, qxy);
          collide_mrt<double>(fd, r, r - d.rho0, Fx, Fy, rcp64(r), d.s_e, d.s_eps, d.s_q, d.inv_tau, qxx, qyy, qxy,
                              fsd);
#pragma unroll
          for (int i = 0; i < 9; ++i) fs[i] = (C)fsd[i];
        } else {
          const double r = (double)rc;
          collide<C, double, TAU1>(fc, r, r - d.rho0, Fx, Fy, d.inv_tau, d.force_pref, rcp64(r), fs);
        }
      } else {
        C Fx, Fy;
        hybrid_force<C>(d, pc, pcL, pcR, pm, pmL, pmR, pn, pnL, pnR, Fx, Fy);
        // Eq. 14 next to a flat solid row: sum_a w_a S(x + e_a) e_a = (0, -1/2) below, (0, 1/2) above
        if (mcw) {
          if (y == 1) Fy = Fy + gwb * pc;
          if (y == ny - 2) Fy = Fy - gwt * pc;
        }
        if (mrt) {
          C qxx = (C)0, qyy = (C)0, qxy = (C)0;
          if (kap) qtensor<C>(pc, pcL, pcR, pn, pnL, pnR, pm, pmL, pmR, A, kq, qxx, qyy, qxy);
          collide_mrt<C>(fc, rc, rc - rho0, Fx, Fy, (C)1 / rc, s_e, s_eps, s_q, inv_tau, qxx, qyy, qxy, fs);
        } else {
          collide<C, C, TAU1>(fc, rc, rc - rho0, Fx, Fy, inv_tau, pref, (C)1 / rc, fs);
        }
      }
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
    if (y == yend) break;
    // slide the window one row on
    rb = rc; pb = pc; pbL = pcL; pbR = pcR;
    rc = ra; pc = pa; pcL = paL; pcR = paR;
    cl_c = cl_a;
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = fn[i];
    const int ynew = y + 2 * st;  // the row entering the window
    if (fluid_row(ynew)) {
      C g[9];  // the halo column's populations of row ynew (edge lanes)
      if (PF) {
#pragma unroll
        for (int i = 0; i < 9; ++i) fn[i] = act ? fp[i] : (C)0;
        if (act && readable(ynew + st)) gather<S, C>(gin, plane, pitch, nx, ny, col, wrapy(ynew + st), fp, py);
        if (edge) gather<S, C>(gin, plane, pitch, nx, ny, hcol, wrapy(ynew), g, py);
      } else if (act) {
        gather<S, C>(gin, plane, pitch, nx, ny, col, wrapy(ynew), fn, py);
        if (edge) gather<S, C>(gin, plane, pitch, nx, ny, hcol, wrapy(ynew), g, py);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) fn[i] = (C)0;
      }
      ra = rho0 + sum9(fn);
      pa = node_psi<MIX>(d, ra, cl_a);
      C hpa = (C)0;
      if (edge) {
        bool dm;
        hpa = node_psi<MIX>(d, rho0 + sum9(g), dm);
      }
      xchg(pa, hpa, paL, paR);
    } else {
      pa = tg; paL = tgL; paR = tgR;
      cl_a = false;
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
    double dy = (double)y - drops[3 * j + 1];
    if (d.periodic_y) dy -= (double)nyf * floor(dy / (double)nyf + 0.5);  // nearest periodic image
    const double dist = sqrt(dx * dx + dy * dy);
    const double v = rho_v + (rho_l - rho_v) * 0.5 * (1.0 - tanh(2.0 * (dist - drops[3 * j + 2]) / width));
    if (v > r) r = v;
  }
  rho[(int64_t)y * nx + x] = r;
}


// Rest state f_i = w_i rho stored as post-collision populations: g_i(x) = f_i(x + e_i), or f_{opp(i)}(x) where
// x + e_i is a ghost row (the inverse of the gather; with periodic rows x + e_i wraps instead).
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
    int yd = y + kEY[i];
    bool wall = yd < 1 || yd > ny - 2;
    if (wall && d.periodic_y) {
      yd = yd < 1 ? ny - 2 : 1;
      wall = false;
    }
    const double r = wall ? rho[(int64_t)y * nx + x] : rho[(int64_t)yd * nx + wrapx(x + kEX[i], nx)];
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
  if (d.periodic_y || d.wall_mc) {  // no walls, or solid walls without ghost densities
    d.ghost[wall * nx + x] = 0.0;
    return;
  }
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
  gather<S, double>((const typename Gbl<S>::T*)d.f[d.cur], d.plane, d.pitch, nx, ny, x, y, f, d.periodic_y != 0);
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
  gather<S, double>((const typename Gbl<S>::T*)d.f[d.cur], d.plane, d.pitch, nx, ny, x, y, f, d.periodic_y != 0);
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
  int yd = y + kEY[q];
  bool wall = yd < 1 || yd > ny - 2;
  if (wall && d.periodic_y) {
    yd = yd < 1 ? ny - 2 : 1;
    wall = false;
  }
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

template <class S, bool CHECK, bool TAU1, bool PF, bool DOWN, bool MIX>
void launch_step_d(int waves, unsigned grid, hipStream_t s, const InstDesc* d_desc, const WaveTask* d_tasks,
                   int ntasks, int flip, WaveDiag* d_wdiag) {
  switch (waves) {
    case 1: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 1, PF, DOWN, MIX>), dim3(grid), dim3(WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
    case 2: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 2, PF, DOWN, MIX>), dim3(grid), dim3(2 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
    case 4: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 4, PF, DOWN, MIX>), dim3(grid), dim3(4 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
    default: hipLaunchKernelGGL((k_step<S, CHECK, TAU1, 8, PF, DOWN, MIX>), dim3(grid), dim3(8 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, d_wdiag); break;
  }
}

// down: walk the strips downwards (see k_step)
template <class S, bool CHECK, bool TAU1, bool PF, bool MIX>
void launch_step_w(int waves, unsigned grid, hipStream_t s, const InstDesc* d_desc, const WaveTask* d_tasks,
                   int ntasks, int flip, WaveDiag* d_wdiag, bool down) {
  if (down) launch_step_d<S, CHECK, TAU1, PF, true, MIX>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
  else launch_step_d<S, CHECK, TAU1, PF, false, MIX>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag);
}

template <class S, bool PF, bool MIX>
void launch_step_s(bool check, bool tau1, int waves, unsigned grid, hipStream_t s, const InstDesc* d_desc,
                   const WaveTask* d_tasks, int ntasks, int flip, WaveDiag* d_wdiag, bool down) {
  if (check) {
    if (tau1) launch_step_w<S, true, true, PF, MIX>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, down);
    else launch_step_w<S, true, false, PF, MIX>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, down);
  } else {
    if (tau1) launch_step_w<S, false, true, PF, MIX>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, down);
    else launch_step_w<S, false, false, PF, MIX>(waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, down);
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------------ launchers
hipError_t launch_step(int storage, bool check, bool tau1, int waves, bool prefetch, const InstDesc* d_desc,
                       const WaveTask* d_tasks, int ntasks, int flip, WaveDiag* d_wdiag, hipStream_t s, int down) {
  if (ntasks <= 0) return hipSuccess;
  const unsigned grid = (unsigned)ntasks;
  const bool dn = down < 0 ? (flip & 1) != 0 : down != 0;  // consecutive steps alternate by default
  if (storage == STORE_F64) {
    if (prefetch) launch_step_s<double, true, false>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, dn);
    else launch_step_s<double, false, false>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, dn);
  } else if (storage == STORE_F32M) {
    if (prefetch) launch_step_s<float, true, true>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, dn);
    else launch_step_s<float, false, true>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, dn);
  } else {
    if (prefetch) launch_step_s<float, true, false>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, dn);
    else launch_step_s<float, false, false>(check, tau1, waves, grid, s, d_desc, d_tasks, ntasks, flip, d_wdiag, dn);
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

}  // namespace lbm
