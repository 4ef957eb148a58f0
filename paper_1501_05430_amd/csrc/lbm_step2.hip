// Two time steps per launch (temporal blocking) for the step with tau = 1 BGK-Guo collision and the geometric walls
// of Sec. 4 (the headline form of the method), in every storage precision; a general instance covers the other
// collisions (MRT with the surface-tension source, BGK at any tau) and the Martys-Chen walls of Eq. 14. Per lattice
// update it moves about half the HBM bytes of the one-step kernel (lbm_kernels.hip), whose per-node arithmetic it
// repeats exactly: the results are bit for bit those of two one-step launches.
//
// A block of W wavefronts owns a tile: output columns [x0, x0 + bw) (bw <= 64 W - 8) of output rows [y0, ylast].
// Lane l works on column x0 - 4 + l (periodic): step A collides three halo columns on each side of the outputs, and
// the outermost lane on each side only supplies psi, so every wavefront runs the same instructions (a halo column
// gathered by an edge lane on top of its own would load the two edge wavefronts, and through the barriers every
// wavefront, with one more gather and psi per row).
//  * Step A (t -> t+1) is the one-step kernel's row walk over the tile's lanes: the populations g^t are gathered from
//    HBM (pull scheme with halfway bounce-back), psi (Eq. 10) is exchanged with the neighbouring lanes, and the
//    force (Eq. 9) and the collision (Eq. 1-6 at tau = 1) produce g^{t+1} of one row per iteration. The ghost rows
//    (Eq. 19 / 21) are computed where the walk meets a wall, as in the one-step kernel. g^{t+1} does not go to HBM:
//    it goes into a three-row ring in LDS.
//  * Step B (t+1 -> t+2) trails two rows behind: it gathers f^{t+1} of row y-1 from the ring (lanes 2 .. bw + 5),
//    forms rho and psi (psi into a three-row LDS ring of its own), computes its own ghost rows from those densities
//    at a wall, and collides row y-2 on the output lanes, storing g^{t+2} to HBM.
// Reach: one step reads populations one column away and psi one more, and a ghost row reads densities one column
// further, so step B's outputs need step A on three more columns per side, and step A psi one column beyond those
// (the psi-only lanes; at a wall their ghost rows read one column further still). In y a strip reads g^t rows
// y0 - 4 .. ylast + 4.
// Per launch and output node: 36 B read (plus the halo share) and 36 B written for two updates.
// Latency: the rows of g^t are loaded one row ahead of their use; the row loop is unrolled by the three-row period
// of the window, so sliding it renames registers instead of copying them.
// Block order: consecutive tasks (tiles of one row band, then the next band) are given to the same XCD, so tiles
// that share halo rows and boundary cache lines meet in one L2.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <math.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kXcds = 8;

// FP64: at least two blocks per compute unit, which caps the registers at 256 (two wavefronts per SIMD; the ring of
// FP64 rows allows two blocks of four wavefronts per compute unit). The general FP32 instance: four wavefronts per
// SIMD (128 registers, a few spilled), which runs the paper's setting 3.6 % faster than three at 140 registers. The
// checked mixed instance is held to the four wavefronts per SIMD of the unchecked one, whose task table it runs.
template <class S, int W, bool MIX, bool GEN, bool CHK>
__global__ __launch_bounds__(WAVE * W, (std::is_same<S, double>::value
                                            ? 2
                                            : (((GEN && !MIX) || (MIX && !GEN && CHK)) ? 4 : 1))) void k_step2(const InstDesc* __restrict__ descs,
                                                    const WaveTask* __restrict__ tasks, int ntasks, int flip,
                                                    WaveDiag* __restrict__ wdiag) {
  typedef typename ComputeOf<S>::type C;
  typedef typename Gbl<S>::T GS;
  static_assert(!MIX || std::is_same<S, float>::value, "the mixed arithmetic is a form of FP32 storage");
  constexpr int L = WAVE * W;
  // XCD-aware order: blocks go round-robin to the XCDs; XCD k takes the k-th contiguous share of the task table.
  const int per = (ntasks + kXcds - 1) / kXcds;
  const int task = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
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
  // GEN: Martys-Chen walls (Eq. 14), a branch uniform over the block: solid wall rows (psi = 0 in the ghost rows, no
  // wetting) and the fluid-solid force on the boundary rows
  const bool mcw = GEN && d.wall_mc != 0;
  auto wrapc = [&](int x) { x %= nx; return x < 0 ? x + nx : x; };

  const int bwA = bw + 6;           // step A collides columns x0 - 3 .. x0 + bw + 2, on lanes 1 .. bwA
  const int lx = wv * WAVE + lane;  // position in the tile = column - (x0 - 4)
  const bool act = lx <= bwA + 1;   // gathers and psi on lanes 0 .. bwA + 1 (the outer two only supply psi)
  const bool actA = act && lx >= 1 && lx <= bwA;          // step A collides here
  const int col = wrapc(x0 - 4 + (act ? lx : 0));
  const bool ledge = lx == 0, redge = lx == bwA + 1;
  const bool edge = ledge || redge;
  const int ocol = wrapc(ledge ? x0 - 5 : x0 + bw + 4);  // one further out (a ghost row's tangential difference)
  const bool actBg = lx >= 2 && lx <= bwA - 1;            // step B gathers here
  const bool actBw = lx >= 3 && lx <= bwA - 2;            // step B ghost rows here
  const bool actBc = lx >= 4 && lx < bw + 4;              // step B output lanes

  // LDS: step A's post-collision rows (ring of 3 rows), row exchange buffers, step B's psi rows (ring of 3 rows,
  // ghost rows included) and step B's boundary-row densities (bottom, top) for its ghost rows.
  __shared__ S gA[3][9][L];
  __shared__ C xa[2][L + 2];
  __shared__ C psB[3][L];
  __shared__ C rhB[2][L];
  // CHK: a checked launch also takes the diagnostics of step B's input, the state after step A, which is what a
  // checked one-step launch of the second step reads: mass, non-finite densities, psi clamps (output nodes) and
  // ghost-row clamps (output columns). Each output lane sums its own nodes here; the block folds them at the end
  // into wdiag[task].
  __shared__ double ckm[CHK ? L : 1];
  __shared__ int ckc[3][CHK ? L : 1];
  if constexpr (CHK) {
    ckm[lx] = 0.0;
    ckc[0][lx] = ckc[1][lx] = ckc[2][lx] = 0;
  }

  // (left, right) neighbours of a per-lane value through xa: put, barrier, get (lanes 1 .. bwA read them)
  int par = 0;
  auto xput = [&](C v) {
    if (act) xa[par][lx + 1] = v;
  };
  auto xget = [&](C& l, C& r) {
    l = xa[par][lx];
    r = xa[par][lx + 2];
    par ^= 1;
  };
  auto xchg = [&](C v, C& l, C& r) {
    xput(v);
    __syncthreads();
    xget(l, r);
  };

  // ---------------------------------------------------------------------------------------------- step A
  auto produce = [&](int y, C (&f)[9], C& rho, C& psi, bool& cl) {
    if (act) {
      gather<S, C>(gin, plane, pitch, nx, ny, col, y, f);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = (C)0;
    }
    rho = rho0 + sum9(f);
    psi = node_psi<MIX>(d, rho, cl);
  };
  // ghost row beside wall `wall` from the boundary row yb (r1) and the second row (r2), Sec. 4; the outermost lanes'
  // tangential difference reads one column further out (ocol)
  auto ghostA = [&](int wall, int yb, C r1, C r2, C& g_rho, C& g_psi) {
    if (mcw) {
      g_rho = g_psi = (C)0;
      return;
    }
    C Lf, Rf;
    xchg(r1, Lf, Rf);
    C ro = (C)0;
    if (edge) {
      C g[9];
      gather<S, C>(gin, plane, pitch, nx, ny, ocol, yb, g);
      ro = rho0 + sum9(g);
    }
    const int base = wall * nx;
    double r0 = 0.0;
    bool gc = false;
    if (act)
      r0 = ghost_density(ledge ? (double)ro : (double)Lf, redge ? (double)ro : (double)Rf, (double)r1, (double)r2,
                         cos_th[base + col], cot_th[base + col], iters, d.rho_cap_hi, gc);
    bool dm;
    g_rho = (C)r0;
    g_psi = (C)psi_eval(d, r0, dm);
  };

  const C inv_tau = (C)d.inv_tau, pref = (C)d.force_pref;
  // GEN: the instance's own collision, a branch uniform over the block: MRT (Eq. 15) with the surface-tension source
  // (Eq. 16-17) where set, else BGK at any tau; otherwise the tau = 1 BGK specialisation (geometric walls only)
  const bool mrt = GEN && d.mrt != 0, kap = mrt && d.kq != 0.0;
  const C Ac = (C)d.A, s_e = (C)d.s_e, s_eps = (C)d.s_eps, s_q = (C)d.s_q, kq = (C)d.kq;
  const C gwb = (C)d.gw_half[0], gwt = (C)d.gw_half[1];  // G_w / 2 of the bottom and top wall

  // Eq. 9 (with Eq. 14 next to solid walls) and the collision of node row y, as in the one-step kernel: FP32 or
  // FP64, or for MIX the force, velocity, equilibrium and forcing in FP64 (and the whole MRT collision)
  auto force_collide = [&](int y, const C (&f)[9], C rho, C pc, C pcL, C pcR, C pm, C pmL, C pmR, C pn, C pnL,
                           C pnR, C (&fs)[9]) {
    if constexpr (MIX) {
      double Fx, Fy;
      hybrid_force<double>(d, pc, pcL, pcR, pm, pmL, pmR, pn, pnL, pnR, Fx, Fy);
      const double r = (double)rho;
      if constexpr (GEN) {
        if (mcw) {
          if (y == 1) Fy = Fy + d.gw_half[0] * (double)pc;
          if (y == ny - 2) Fy = Fy - d.gw_half[1] * (double)pc;
        }
        if (mrt) {
          double fd[9], fsd[9], qxx = 0.0, qyy = 0.0, qxy = 0.0;
#pragma unroll
          for (int i = 0; i < 9; ++i) fd[i] = (double)f[i];
          if (kap) qtensor<double>(pc, pcL, pcR, pn, pnL, pnR, pm, pmL, pmR, d.A, d.kq, qxx, qyy, qxy);
          collide_mrt<double>(fd, r, r - d.rho0, Fx, Fy, rcp64(r), d.s_e, d.s_eps, d.s_q, d.inv_tau, qxx, qyy, qxy,
                              fsd);
#pragma unroll
          for (int i = 0; i < 9; ++i) fs[i] = (C)fsd[i];
        } else {
          collide<C, double, false>(f, r, r - d.rho0, Fx, Fy, d.inv_tau, d.force_pref, rcp64(r), fs);
        }
      } else {
        collide<C, double, true>(f, r, r - d.rho0, Fx, Fy, d.inv_tau, d.force_pref, rcp64(r), fs);
      }
    } else {
      C Fx, Fy;
      hybrid_force<C>(d, pc, pcL, pcR, pm, pmL, pmR, pn, pnL, pnR, Fx, Fy);
      if constexpr (GEN) {
        if (mcw) {
          if (y == 1) Fy = Fy + gwb * pc;
          if (y == ny - 2) Fy = Fy - gwt * pc;
        }
        if (mrt) {
          C qxx = (C)0, qyy = (C)0, qxy = (C)0;
          if (kap) qtensor<C>(pc, pcL, pcR, pn, pnL, pnR, pm, pmL, pmR, Ac, kq, qxx, qyy, qxy);
          collide_mrt<C>(f, rho, rho - rho0, Fx, Fy, (C)1 / rho, s_e, s_eps, s_q, inv_tau, qxx, qyy, qxy, fs);
        } else {
          collide<C, C, false>(f, rho, rho - rho0, Fx, Fy, inv_tau, pref, (C)1 / rho, fs);
        }
      } else {
        collide<C, C, true>(f, rho, rho - rho0, Fx, Fy, inv_tau, pref, (C)1 / rho, fs);
      }
    }
  };

  // step A's rows: those step B reads, g^{t+1} of rows y0 - 2 .. ylast + 2 within the fluid rows
  const int ya0 = y0 - 2 >= 1 ? y0 - 2 : 1, ya1 = ylast + 2 <= ny - 2 ? ylast + 2 : ny - 2;
  const bool wall_start = ya0 == 1, wall_end = ya1 == ny - 2;

  C tg = (C)0;  // step A's top ghost row's psi
  if (wall_end) {
    C f1[9], f2[9], r1, r2, p1, p2, g_rho;
    bool dm;
    produce(ny - 2, f1, r1, p1, dm);
    produce(ny - 3, f2, r2, p2, dm);
    ghostA(1, ny - 2, r1, r2, g_rho, tg);
  }
  // window: rows (b, c, a) = (y - 1, y, y + 1) when step A processes row y
  C fc[9], fn[9], fp[9];
  C rb, rc, ra, pb, pc, pa, pbL, pbR, pcL, pcR, paL, paR;
  {
    bool dm;
    if (wall_start) {
      produce(ya0, fc, rc, pc, dm);
      produce(ya0 + 1, fn, ra, pa, dm);
      ghostA(0, ya0, rc, ra, rb, pb);
    } else {
      C fb[9];
      produce(ya0 - 1, fb, rb, pb, dm);
      produce(ya0, fc, rc, pc, dm);
      if (ya0 + 1 <= ny - 2) produce(ya0 + 1, fn, ra, pa, dm);
    }
    xchg(pb, pbL, pbR);
    xchg(pc, pcL, pcR);
    if (ya0 + 1 <= ny - 2) {
      xchg(pa, paL, paR);
    } else {
      pa = tg;
      xchg(tg, paL, paR);
    }
  }
  // rows gathered by step A: ya0 - 1 .. ya1 + 1 within the fluid rows; the populations of row y + 2 are in flight
  // while row y is processed
  const int yread = ya1 + 1 <= ny - 2 ? ya1 + 1 : ny - 2;
  // every lane loads (a lane past the tile's columns reads a valid column and its results are never stored), so the
  // window slides by renaming registers
#pragma unroll
  for (int i = 0; i < 9; ++i) fp[i] = (C)0;
  if (ya0 + 2 <= yread) gather<S, C>(gin, plane, pitch, nx, ny, col, ya0 + 2, fp);

  // ---------------------------------------------------------------------------------------------- step B state
  const bool wallB_bot = y0 == 1, wallB_top = ylast == ny - 2;
  const int jb0 = y0 - 1 >= 1 ? y0 - 1 : 1, jb1 = ylast + 1 <= ny - 2 ? ylast + 1 : ny - 2;  // rows B gathers
  C fBp[9], rBp = (C)0;  // step B's populations and density of the row gathered in the previous iteration
  C rBtop2 = (C)0;       // density of row ny - 3 on the own lane (top ghost row of step B)
#pragma unroll
  for (int i = 0; i < 9; ++i) fBp[i] = (C)0;

  // Iteration y: step A collides row y; step B gathers row j = y - 1 and collides row m = y - 2. The window slides
  // every iteration (past step A's last row nothing reads it), and the loop is unrolled by its period of three rows,
  // so the slide is a renaming of registers rather than copies.
  const int yend = ylast + 2;
  auto row = [&](const int y) -> bool {
    // ---- step A: collide row y into the ring, then bring row y + 2 into the window
    if (y <= ya1 && actA) {
      C fs[9];
      force_collide(y, fc, rc, pc, pcL, pcR, pb, pbL, pbR, pa, paL, paR, fs);
      const int s = y % 3;
#pragma unroll
      for (int i = 0; i < 9; ++i) gA[s][i][lx] = fs[i];
    }
    rb = rc; pb = pc; pbL = pcL; pbR = pcR;
    rc = ra; pc = pa;
#pragma unroll
    for (int i = 0; i < 9; ++i) { fc[i] = fn[i]; fn[i] = fp[i]; }
    const int ynew = y + 2;
    if (y < ya1 && ynew <= ny - 2) {
      // densities of the row prefetched an iteration ago, then the next prefetch
      ra = rho0 + sum9(fn);
      if (ynew + 1 <= yread) gather<S, C>(gin, plane, pitch, nx, ny, col, ynew + 1, fp);
      bool dm;
      pa = node_psi<MIX>(d, ra, dm);
      xput(pa);
    } else {
      // the row above the top fluid row is the ghost row (or step A is done and the window is no longer read)
      ra = (C)0;
      pa = tg;
      xput(tg);
    }
    pcL = paL; pcR = paR;
    __syncthreads();  // step A's row y is in the ring; the psi of row y + 2 is in xa
    xget(paL, paR);

    // ---- step B: gather row j = y - 1 from the ring (density, psi), ghost rows at the walls
    const int j = y - 1;
    const bool doG = j >= jb0 && j <= jb1;
    C fg[9], rj = (C)0;
    if (doG && actBg) {
      const bool bot = j == 1, top = j == ny - 2;
      const int sm = (j + 2) % 3, sc = j % 3, sp = (j + 1) % 3;  // ring slots of rows j - 1, j, j + 1
      fg[0] = gA[sc][0][lx];
      fg[1] = gA[sc][1][lx - 1];
      fg[2] = bot ? gA[sc][4][lx] : gA[sm][2][lx];
      fg[3] = gA[sc][3][lx + 1];
      fg[4] = top ? gA[sc][2][lx] : gA[sp][4][lx];
      fg[5] = bot ? gA[sc][7][lx] : gA[sm][5][lx - 1];
      fg[6] = bot ? gA[sc][8][lx] : gA[sm][6][lx + 1];
      fg[7] = top ? gA[sc][5][lx] : gA[sp][7][lx + 1];
      fg[8] = top ? gA[sc][6][lx] : gA[sp][8][lx - 1];
      rj = rho0 + sum9(fg);
      bool dm;
      psB[sc][lx] = node_psi<MIX>(d, rj, dm);
      if (bot) rhB[0][lx] = rj;
      if (top) rhB[1][lx] = rj;
      if constexpr (CHK) if (actBc && j >= y0 && j <= ylast) {
        double mm = (double)fg[0];
#pragma unroll
        for (int i = 1; i < 9; ++i) mm += (double)fg[i];
        ckm[lx] += mm + d.rho0;
        ckc[0][lx] += isfinite(rj) ? 0 : 1;
        ckc[1][lx] += dm ? 1 : 0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) fg[i] = __builtin_nondeterministic_value((C)0);  // never collided
    }
    if (doG && j == ny - 3) rBtop2 = rj;
    // bottom ghost row (row 0, ring slot 0) once rows 1 and 2 are in: row 1's densities through LDS
    if (wallB_bot && doG && j == 2 && actBw) {
      if (mcw) {
        psB[0][lx] = (C)0;
      } else {
        bool gc, dm;
        const double r0 = ghost_density((double)rhB[0][lx - 1], (double)rhB[0][lx + 1], (double)rhB[0][lx],
                                        (double)rj, cos_th[col], cot_th[col], iters, d.rho_cap_hi, gc);
        psB[0][lx] = (C)psi_eval(d, r0, dm);
        if constexpr (CHK) if (gc && actBc) ckc[2][lx] += 1;
      }
    }
    // top ghost row (row ny - 1) after the last gather: row ny - 2's densities through LDS, row ny - 3's own
    if (wallB_top && y == ny && actBw) {
      if (mcw) {
        psB[(ny - 1) % 3][lx] = (C)0;
      } else {
        bool gc, dm;
        const double r0 = ghost_density((double)rhB[1][lx - 1], (double)rhB[1][lx + 1], (double)rhB[1][lx],
                                        (double)rBtop2, cos_th[nx + col], cot_th[nx + col], iters, d.rho_cap_hi, gc);
        psB[(ny - 1) % 3][lx] = (C)psi_eval(d, r0, dm);
        if constexpr (CHK) if (gc && actBc) ckc[2][lx] += 1;
      }
    }
    __syncthreads();  // step B's psi of row j (and a ghost row) are in the ring

    // ---- step B: collide row m = y - 2 (gathered in the previous iteration) and store it
    const int m = y - 2;
    if (m >= y0 && m <= ylast && actBc) {
      C fs[9];
      const int s0 = (m + 2) % 3, s1 = m % 3, s2 = (m + 1) % 3;  // rows m - 1, m, m + 1
      force_collide(m, fBp, rBp, psB[s1][lx], psB[s1][lx - 1], psB[s1][lx + 1], psB[s0][lx], psB[s0][lx - 1],
                    psB[s0][lx + 1], psB[s2][lx], psB[s2][lx - 1], psB[s2][lx + 1], fs);
      const unsigned off = (unsigned)((m - 1) * pitch + col);
#pragma unroll
      for (int i = 0; i < 9; ++i) ((GS*)(gout + i * plane))[off] = fs[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) fBp[i] = fg[i];
    rBp = rj;
    return y == yend;
  };
  for (int y = ya0;; y += 3) {
    if (row(y)) break;
    if (row(y + 1)) break;
    if (row(y + 2)) break;
  }
  if constexpr (CHK) {  // fold in a fixed order: lanes of a wavefront, then the wavefronts
    __shared__ double sm[W];
    __shared__ int si[W][3];
    const double m = wave_sum(ckm[lx]);
    const int c0 = wave_sum(ckc[0][lx]), c1 = wave_sum(ckc[1][lx]), c2 = wave_sum(ckc[2][lx]);
    if (lane == 0) {
      sm[wv] = m;
      si[wv][0] = c0;
      si[wv][1] = c1;
      si[wv][2] = c2;
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

template <class S, int W, bool MIX, bool GEN>
int occupancy_of(int* blocks) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_step2<S, W, MIX, GEN, false>, WAVE * W, 0);
}

template <class S, bool MIX, bool GEN>
hipError_t blocks_per_cu(int waves, int* blocks) {
  switch (waves) {
    case 1: return (hipError_t)occupancy_of<S, 1, MIX, GEN>(blocks);
    case 2: return (hipError_t)occupancy_of<S, 2, MIX, GEN>(blocks);
    case 4: return (hipError_t)occupancy_of<S, 4, MIX, GEN>(blocks);
    default: return (hipError_t)occupancy_of<S, 8, MIX, GEN>(blocks);
  }
}

template <class S, bool MIX, bool GEN, bool CHK>
void launch2c(const InstDesc* d_desc, const WaveTask* d_tasks, int ntasks, int waves, int flip, WaveDiag* wd,
              unsigned grid, hipStream_t s) {
  switch (waves) {
    case 1: hipLaunchKernelGGL((k_step2<S, 1, MIX, GEN, CHK>), dim3(grid), dim3(WAVE), 0, s, d_desc, d_tasks, ntasks, flip, wd); break;
    case 2: hipLaunchKernelGGL((k_step2<S, 2, MIX, GEN, CHK>), dim3(grid), dim3(2 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, wd); break;
    case 4: hipLaunchKernelGGL((k_step2<S, 4, MIX, GEN, CHK>), dim3(grid), dim3(4 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, wd); break;
    default: hipLaunchKernelGGL((k_step2<S, 8, MIX, GEN, CHK>), dim3(grid), dim3(8 * WAVE), 0, s, d_desc, d_tasks, ntasks, flip, wd); break;
  }
}

template <class S, bool MIX, bool GEN>
void launch2(const InstDesc* d_desc, const WaveTask* d_tasks, int ntasks, int waves, int flip, WaveDiag* wd,
             unsigned grid, hipStream_t s) {
  if (wd) launch2c<S, MIX, GEN, true>(d_desc, d_tasks, ntasks, waves, flip, wd, grid, s);
  else launch2c<S, MIX, GEN, false>(d_desc, d_tasks, ntasks, waves, flip, wd, grid, s);
}

template <bool GEN>
hipError_t blocks_for(int waves, int storage, int* blocks) {
  if (storage == STORE_F64) return blocks_per_cu<double, false, GEN>(waves, blocks);
  return storage == STORE_F32M ? blocks_per_cu<float, true, GEN>(waves, blocks)
                               : blocks_per_cu<float, false, GEN>(waves, blocks);
}

template <bool GEN>
void launch_for(const InstDesc* d_desc, const WaveTask* d_tasks, int ntasks, int waves, int storage, int flip,
                WaveDiag* wd, unsigned grid, hipStream_t s) {
  if (storage == STORE_F64) launch2<double, false, GEN>(d_desc, d_tasks, ntasks, waves, flip, wd, grid, s);
  else if (storage == STORE_F32M) launch2<float, true, GEN>(d_desc, d_tasks, ntasks, waves, flip, wd, grid, s);
  else launch2<float, false, GEN>(d_desc, d_tasks, ntasks, waves, flip, wd, grid, s);
}

}  // namespace

hipError_t step2_blocks_per_cu(int waves, int storage, bool general, int* blocks) {
  *blocks = 0;
  return general ? blocks_for<true>(waves, storage, blocks) : blocks_for<false>(waves, storage, blocks);
}

hipError_t launch_step2(const InstDesc* d_desc, const WaveTask* d_tasks, int ntasks, int waves, int storage,
                        bool general, int flip, hipStream_t s, WaveDiag* d_wdiag) {
  if (ntasks <= 0) return hipSuccess;
  const unsigned grid = (unsigned)(((ntasks + kXcds - 1) / kXcds) * kXcds);
  if (general) launch_for<true>(d_desc, d_tasks, ntasks, waves, storage, flip, d_wdiag, grid, s);
  else launch_for<false>(d_desc, d_tasks, ntasks, waves, storage, flip, d_wdiag, grid, s);
  return hipGetLastError();
}

}  // namespace lbm
