// C-ABI of liblbm (include/lbm.h): context, workspace carving, host EOS solves, stepping with HIP graph replay,
// diagnostics and contact-angle measurement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// ------------------------------------------------------------------------------------------------ host EOS (FP64)
// Carnahan-Starling: p = rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2, eta = b rho/4.
struct Eos {
  double a, b, R, T;
  double p(double rho) const {
    const double e = 0.25 * b * rho, om = 1.0 - e;
    return rho * R * T * (1.0 + e * (1.0 + e * (1.0 - e))) / (om * om * om) - a * rho * rho;
  }
  // dp/drho = R T Phi'(eta) - 2 a rho with Phi = eta Z, Phi' = (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4
  double dp(double rho) const {
    const double e = 0.25 * b * rho, om = 1.0 - e;
    const double om2 = om * om;
    return R * T * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (om2 * om2) - 2.0 * a * rho;
  }
  double d2p(double rho) const {
    const double e = 0.25 * b * rho, om = 1.0 - e;
    const double om2 = om * om;
    return R * T * 0.25 * b * (8.0 + e * (20.0 - 4.0 * e)) / (om2 * om2 * om) - 2.0 * a;
  }
  // chemical potential with mu' = p'/rho: R T [ln rho + (8e - 9e^2 + 3e^3)/(1-e)^3] - 2 a rho
  double mu(double rho) const {
    const double e = 0.25 * b * rho, om = 1.0 - e;
    return R * T * (std::log(rho) + e * (8.0 + e * (-9.0 + 3.0 * e)) / (om * om * om)) - 2.0 * a * rho;
  }
};

// Newton iteration safeguarded by bisection on a bracket [lo, hi] with f(lo), f(hi) of opposite sign.
double safe_root(const std::function<double(double)>& f, const std::function<double(double)>& df, double lo,
                 double hi) {
  double flo = f(lo);
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    const double fx = f(x);
    if (fx == 0.0) return x;
    if ((fx < 0) == (flo < 0)) { lo = x; flo = fx; } else { hi = x; }
    const double d = df(x);
    double xn = (d != 0.0 && std::isfinite(d)) ? x - fx / d : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 4e-16 * std::fabs(x) || hi - lo <= 4e-16 * std::fabs(hi)) return xn;
    x = xn;
  }
  return x;
}

// Critical point from the quintic 1 - 5e - 20e^2 - 4e^3 + 5e^4 - e^5 = 0 (p' = p'' = 0 with T eliminated),
// then T_c = 8 a e_c / (b R Phi'(e_c)).
void cs_critical(double a, double b, double R, double* rho_c, double* T_c) {
  auto q = [](double e) { return 1.0 + e * (-5.0 + e * (-20.0 + e * (-4.0 + e * (5.0 - e)))); };
  auto dq = [](double e) { return -5.0 + e * (-40.0 + e * (-12.0 + e * (20.0 - 5.0 * e))); };
  const double e = safe_root(q, dq, 0.05, 0.3);
  const double om = 1.0 - e;
  const double phi1 = (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (om * om * om * om);
  *rho_c = 4.0 * e / b;
  *T_c = 8.0 * a * e / (b * R * phi1);
}

// Maxwell construction: for a pressure level P the outer branches give rho_v(P) < s1 and rho_l(P) > s2; the
// coexistence level zeroes mu(rho_l) - mu(rho_v). Regula falsi (Illinois) on P.
bool cs_maxwell(const Eos& E, double rho_c, double* rv, double* rl) {
  const double top = 0.9999 * 4.0 / E.b;
  auto dp = [&](double r) { return E.dp(r); };
  auto d2p = [&](double r) { return E.d2p(r); };
  if (!(E.dp(rho_c) < 0)) return false;
  const double s1 = safe_root(dp, d2p, 1e-12 * rho_c, rho_c);
  const double s2 = safe_root(dp, d2p, rho_c, top);
  auto branch = [&](double P, double lo, double hi) {
    return safe_root([&](double r) { return E.p(r) - P; }, dp, lo, hi);
  };
  auto g = [&](double P, double* v, double* l) {
    *v = branch(P, 1e-300, s1);
    *l = branch(P, s2, top);
    return E.mu(*l) - E.mu(*v);
  };
  double Pa = std::max(E.p(s2), 0.0) + 1e-300, Pb = E.p(s1);
  double v, l;
  double ga = g(Pa, &v, &l), gb = g(Pb, &v, &l);
  if (!((ga > 0) && (gb < 0))) {
    // mu_l - mu_v is positive at the lowest level and negative at the vapour spinodal; fall back to bisection
    // in log P if the bracket is degenerate at the low end.
    if (!(gb < 0)) return false;
  }
  int side = 0;
  double P = Pb;
  for (int it = 0; it < 300; ++it) {
    P = (Pa * gb - Pb * ga) / (gb - ga);
    if (!(P > Pa && P < Pb)) P = 0.5 * (Pa + Pb);
    const double gp = g(P, &v, &l);
    if (gp == 0.0 || (Pb - Pa) <= 1e-16 * Pb) break;
    if ((gp > 0) == (ga > 0)) {
      Pa = P; ga = gp;
      if (side == -1) gb *= 0.5;
      side = -1;
    } else {
      Pb = P; gb = gp;
      if (side == 1) ga *= 0.5;
      side = 1;
    }
  }
  g(P, &v, &l);
  *rv = v;
  *rl = l;
  return v > 0 && l > v;
}

// Largest density with real psi (Eq. 10, G < 0): the root of p(rho) - rho/3 above the liquid branch.
double cs_rho_cap(const Eos& E, double rho_c) {
  const double top = 0.9999 * 4.0 / E.b;
  double lo = rho_c;
  if (E.dp(rho_c) < 0) lo = safe_root([&](double r) { return E.dp(r); }, [&](double r) { return E.d2p(r); }, rho_c,
                                      top);
  auto h = [&](double r) { return E.p(r) - r / 3.0; };
  if (!(h(lo) < 0)) return lo;
  return safe_root(h, [&](double r) { return E.dp(r) - 1.0 / 3.0; }, lo, top);
}

// Piecewise-linear EOS (Eq. 11) with slopes t = (theta_v, theta_m, theta_l) and break points r1 < r2.
struct PwEos {
  double tv, tm, tl, r1 = 0, r2 = 0;
  double p(double rho) const {
    if (rho <= r1) return rho * tv;
    if (rho <= r2) return r1 * tv + (rho - r1) * tm;
    return r1 * tv + (r2 - r1) * tm + (rho - r2) * tl;
  }
};

// Break points for the coexistence pair (rv, rl). Eq. 12 is linear in (r1, r2): r1 = (tv rv + (tl - tm) r2 -
// tl rl) / (tv - tm). Eq. 13 is then a function of r2 alone, bisected over the r2 for which rv < r1 < r2 < rl.
bool pw_solve(PwEos* E, double rv, double rl) {
  const double tv = E->tv, tm = E->tm, tl = E->tl;
  auto r1_of = [&](double r2) { return (tv * rv + (tl - tm) * r2 - tl * rl) / (tv - tm); };
  auto eq13 = [&](double r2) {
    const double r1 = r1_of(r2);
    return tv * std::log(r1 / rv) + tm * std::log(r2 / r1) + tl * std::log(rl / r2);
  };
  double lo = (tl * rl - tm * rv) / (tl - tm);             // r1 = rv here
  if (tl < tv) lo = std::max(lo, (tv * rv - tl * rl) / (tv - tl));  // r1 = r2 here
  double hi = rl;
  if (tl > tv) hi = std::min(hi, (tl * rl - tv * rv) / (tl - tv));
  if (!(lo < hi)) return false;
  const double span = hi - lo;
  lo += 1e-14 * span;
  hi -= 1e-14 * span;
  double hl = eq13(lo), hh = eq13(hi);
  if (!std::isfinite(hl) || !std::isfinite(hh) || (hl > 0) == (hh > 0)) return false;
  for (int it = 0; it < 400 && hi - lo > 1e-16 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double hm = eq13(mid);
    if (hm == 0.0) { lo = hi = mid; break; }
    if ((hm > 0) == (hl > 0)) { lo = mid; hl = hm; } else { hi = mid; }
  }
  E->r2 = 0.5 * (lo + hi);
  E->r1 = r1_of(E->r2);
  return rv < E->r1 && E->r1 < E->r2 && E->r2 < rl;
}

// Largest density with real psi (Eq. 10, G < 0: p <= rho/3). p - rho/3 falls on the vapour and unstable branches
// (theta_v < 1/3, theta_m < 0), so only a liquid slope above 1/3 brings it back to 0.
double pw_rho_cap(const PwEos& E) {
  if (!(E.tl > 1.0 / 3.0)) return 1e300;
  return E.r2 + (E.r2 / 3.0 - E.p(E.r2)) / (E.tl - 1.0 / 3.0);
}

bool pw_from_params(const lbm_params& q, PwEos* E) {
  *E = PwEos{q.pw_theta[0], q.pw_theta[1], q.pw_theta[2]};
  return pw_solve(E, q.pw_rho[0], q.pw_rho[1]);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// MRT collision (Eq. 15) when a rate of Eq. 2 or the surface-tension parameter kappa is set.
bool uses_mrt(const lbm_params& q) {
  return q.mrt_rates[0] != 0.0 || q.mrt_rates[1] != 0.0 || q.mrt_rates[2] != 0.0 || q.kappa != 0.0;
}

// Measured defaults on MI355X (autotuning can refine them per context): FP32 8 wavefronts per block with
// prefetch, FP64 4 wavefronts without. Strip height: about two blocks per compute unit over all instances,
// rows = round(fluid nodes / (2 CUs * 64 * waves)), within [2, 32] (FP32) / [2, 64] (FP64); this matches the
// fastest measured height on 512 x 256 up to 4096 x 2048 lattices (e.g. 32 / 64 rows at 4096 x 2048, 2 / 4 rows
// at 1024 x 512).
constexpr int kDefaultStripRows = 32;
constexpr int kDefaultWaves = 8;
constexpr bool kDefaultPrefetch = true;
constexpr int kDefaultStripRows64 = 64;
constexpr int kDefaultWaves64 = 4;
constexpr bool kDefaultPrefetch64 = false;
constexpr int kMinDefaultStripRows = 2;
// Two-step kernel (lbm_step2.hip): wavefronts per block and output rows per strip.
constexpr int kDefaultWaves2 = 4;
// FP32 arithmetic on contexts of at least this many fluid nodes: eight wavefronts per two-step block (504-column
// tiles: fewer halo lanes and task prologues per output; 4096 x 2048: 107.2 against 103.2 GLUPS, 6144 x 3072 118.0
// against 107.5); below it the wider tiles leave more of the last tile empty (3072 x 1536: 98.6 against 101.2,
// 2048 x 1024: 81.9 against 86.1). The mixed form, FP64 and the general instance keep four (4096 x 2048: 87.6
// against 93.7, 44.9 against 56.7, 82.6 against 84.7).
constexpr double kWide2MinNodes = 6.0e6;
constexpr int kWide2MinNx = 2048;  // and instances at least four tiles of 504 columns wide
constexpr int kDefaultStripRows2 = 32;
constexpr int kMinStripRows2 = 8, kMaxStripRows2 = 256;  // bounds of the default from the occupancy
// FP64 storage: at most 24 output rows per strip. At two blocks per compute unit the FP64 kernel runs faster with
// several rounds of 24-row strips than with one round of taller ones (4096 x 2048: 45.7 against 34.0 GLUPS); FP32
// loses a quarter of its rate to a partial second round, so it keeps the one-round rule.
constexpr int kMaxStripRows2F64 = 24;
// Below about 5e4 fluid nodes per context the two-step kernel has too few tasks to pay for its halo: one-step
// launches are as fast (256 x 128: 2.90 against 2.86 GLUPS in FP32; FP64 2.73 against 3.00), above it two steps per
// launch in one-wavefront blocks win (362 x 181: 5.67 against 5.59, FP64 5.93 against 5.11; 600 x 300: 14.7
// against 11.4, FP64 14.8 against 10.9; 4096 x 2048 in its own shape: 109.5 against 65, FP64 57.0 against 34.9).
constexpr double kStep2MinNodes = 50000.0;
// Largest instance below this many fluid nodes: one wavefront per two-step block (56-column tiles; more, smaller
// tasks balance better and need no barrier between wavefronts). 724 x 362: 21.0 against 18.9 GLUPS with four
// (FP64 20.8 against 18.0); 2048 x 1024: 90.2 against 87.2 (FP64 54.3 against 52.3, the mixed form 74.8 against
// 73.0, the paper's setting 67.9 against 66.4). Above it the halo lanes of narrow tiles cost more: 2896 x 1448
// FP64 49.4 against 54.9, FP32 100.6 against 103.0; 4096 x 2048 FP64 52.6 against 57.6.
constexpr double kNarrow2MaxNodes = 3.0e6;
constexpr int kStep2Halo = 8;  // lanes beyond a two-step tile's outputs (three of step A and one of psi per side)
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int kMaxDrops = 4096;
static_assert(sizeof(lbm_params) == 10 * 4 + 22 * 8, "lbm_params layout: 10 int32 then 22 double, no padding");

struct Inst {
  lbm_params p;
  int pitch = 0;
  int64_t plane = 0;
  double rho_c = 0, T_c = 0, T = 0, rho_v = 0, rho_l = 0, rho_cap = 0;
  double pw_r1 = 0, pw_r2 = 0;  // piecewise-linear EOS break points
  int strip_rows = kDefaultStripRows;
  int strip_rows2 = kDefaultStripRows2;  // output rows per strip of the two-step kernel
  bool initialized = false;
  int64_t steps = 0;
  size_t off_f[2] = {0, 0}, off_th = 0, off_ghost = 0, off_adj = 0;
  std::vector<double> cos_th, cot_th, sin_th;
};

struct Layout {
  size_t desc, tasks, wdiag, first, first2, idiag, drops, rho_scratch, partials, tasks2, total;
  size_t task_cap, task2_cap;
  std::vector<size_t> inst_f[2], inst_th, inst_ghost, inst_adj;
};

size_t storage_bytes(int precision) { return precision == LBM_F64 ? 8 : 4; }

// column blocks of 64 * waves columns (at most; see build_tasks)
int blocks_x(int nx, int waves) { return (nx + 64 * waves - 1) / (64 * waves); }

size_t adj_bytes(const lbm_params& p) {
  const size_t pitch = (size_t)((p.nx + 63) / 64 * 64);
  const size_t field = align256(sizeof(double) * pitch * p.ny);
  return 4 * field + align256(sizeof(double) * 2 * p.nx) + align256(sizeof(double) * 8 * p.nx) +
         align256(sizeof(double) * 6 * p.nx) + align256(sizeof(double) * adjoint_partials_needed());
}

bool valid_params(const lbm_params* p, int32_t n, std::string* why) {
  if (!p || n < 1) { *why = "need at least one instance"; return false; }
  for (int i = 0; i < n; ++i) {
    const lbm_params& q = p[i];
    char b[256];
    auto bad = [&](const char* what) {
      snprintf(b, sizeof b, "instance %d: %s", i, what);
      *why = b;
      return false;
    };
    if (q.nx < 2 || q.ny < 4) return bad("need nx >= 2 and ny >= 4");
    if ((int64_t)q.nx * q.ny > (int64_t)1 << 34) return bad("lattice too large");
    if (q.ny - 2 > 65535) return bad("ny too large");
    if (q.precision < LBM_F64 || q.precision > LBM_F32_SHIFTED_MIXED) return bad("unknown precision");
    if (q.precision != p[0].precision) return bad("all instances must share one precision");
    if (q.wet_iters < 0 || q.wet_iters > 1000) return bad("wet_iters out of range [0, 1000]");
    if (q.check_every < 0) return bad("check_every < 0");
    if (q.strip_rows < 0) return bad("strip_rows < 0");
    if (q.step_variant < 0 || q.step_variant > 3 * kNumWaveChoices) return bad("step_variant outside [0, 12]");
    if (q.boundary != LBM_WALLS_Y && q.boundary != LBM_PERIODIC_Y && q.boundary != LBM_WALLS_MARTYS_CHEN)
      return bad("unknown boundary");
    if (!std::isfinite(q.G_w[0]) || !std::isfinite(q.G_w[1])) return bad("G_w not finite");
    if (q.eos != LBM_EOS_CARNAHAN_STARLING && q.eos != LBM_EOS_PIECEWISE_LINEAR) return bad("unknown eos");
    // offsets inside a population plane are 32-bit in the kernels (planes are 64-bit apart)
    if ((int64_t)((q.nx + 63) / 64 * 64) * (q.ny - 2) >= ((int64_t)1 << 31))
      return bad("lattice too large: pitch x (ny - 2) must stay below 2^31");
    if (!(q.tau > 0.5) || !std::isfinite(q.tau)) return bad("tau must be > 0.5");
    if (!(q.G < 0) || !std::isfinite(q.G)) return bad("G must be negative");
    if (!std::isfinite(q.A)) return bad("A not finite");
    if (q.eos == LBM_EOS_CARNAHAN_STARLING) {
      if (!(q.eos_a > 0) || !(q.eos_b > 0) || !(q.eos_R > 0)) return bad("EOS constants must be positive");
      if (!(q.T_over_Tc > 0 && q.T_over_Tc < 1)) return bad("T_over_Tc must be in (0, 1)");
    } else {
      const double* t = q.pw_theta;
      if (!(t[0] > 0 && t[0] < 1.0 / 3.0)) return bad("piecewise EOS: theta_v must be in (0, 1/3)");
      if (!(t[1] < 0) || !std::isfinite(t[1])) return bad("piecewise EOS: theta_m must be negative");
      if (!(t[2] > 0) || !std::isfinite(t[2])) return bad("piecewise EOS: theta_l must be positive");
      if (!(q.pw_rho[0] > 0 && q.pw_rho[1] > q.pw_rho[0] && std::isfinite(q.pw_rho[1])))
        return bad("piecewise EOS: need 0 < rho_v < rho_l");
      PwEos E;
      // With these signs Eq. 13 changes sign across the feasible break points (the integral of dp / rho is negative
      // where p falls first and positive where it rises first), so a failure here means degenerate input (theta_m or
      // rho_l / rho_v - 1 at round-off level). psi is then real up to rho_l: p(rho_l) = p(rho_v) = theta_v rho_v
      // < rho_l / 3.
      if (!pw_from_params(q, &E)) return bad("piecewise EOS: Eq. 12-13 have no break points rho_v < rho_1 < rho_2 < rho_l");
    }
    if (!std::isfinite(q.rho0_shift) || q.rho0_shift < 0) return bad("rho0_shift must be >= 0");
    if (q.precision != LBM_F32_SHIFTED && q.precision != LBM_F32_SHIFTED_MIXED && q.rho0_shift != 0)
      return bad("rho0_shift needs LBM_F32_SHIFTED or LBM_F32_SHIFTED_MIXED");
    if (!std::isfinite(q.rho_fp64_below)) return bad("rho_fp64_below not finite");
    if (!std::isfinite(q.body_force[0]) || !std::isfinite(q.body_force[1])) return bad("body force not finite");
    for (int k = 0; k < 3; ++k)
      if (!(q.mrt_rates[k] == 0.0 || (q.mrt_rates[k] > 0.0 && q.mrt_rates[k] < 2.0)))
        return bad("mrt_rates must be 0 (= 1/tau) or in (0, 2)");
    if (!std::isfinite(q.kappa)) return bad("kappa not finite");
  }
  return true;
}

Layout make_layout(const lbm_params* p, int32_t n) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align256(bytes);
    return r;
  };
  L.task_cap = 0;
  L.task2_cap = 0;
  size_t max_nodes = 0;
  for (int i = 0; i < n; ++i) {
    L.task_cap += (size_t)blocks_x(p[i].nx, 1) * (size_t)(p[i].ny - 2);
    L.task2_cap += (size_t)((p[i].nx + (64 - kStep2Halo) - 1) / (64 - kStep2Halo)) * (size_t)(p[i].ny - 2);
    max_nodes = std::max(max_nodes, (size_t)p[i].nx * p[i].ny);
  }
  L.desc = take(sizeof(InstDesc) * n);
  L.tasks = take(sizeof(WaveTask) * L.task_cap);
  L.wdiag = take(sizeof(WaveDiag) * std::max(L.task_cap, L.task2_cap));  // per task of either table
  L.first = take(sizeof(int32_t) * (n + 1));
  L.first2 = take(sizeof(int32_t) * (n + 1));
  L.idiag = take(sizeof(InstDiag) * n);
  L.drops = take(sizeof(double) * 3 * kMaxDrops);
  L.rho_scratch = take(sizeof(double) * max_nodes);
  L.partials = take(sizeof(double) * kMeasureBlocks * 16);
  L.tasks2 = take(sizeof(WaveTask) * L.task2_cap);
  for (int i = 0; i < n; ++i) {
    const size_t pitch = (size_t)((p[i].nx + 63) / 64 * 64);
    const size_t fbytes = storage_bytes(p[i].precision) * 9 * pitch * (size_t)(p[i].ny - 2);
    L.inst_f[0].push_back(take(fbytes));
    L.inst_f[1].push_back(take(fbytes));
    L.inst_th.push_back(take(sizeof(double) * 6 * p[i].nx));
    L.inst_ghost.push_back(take(sizeof(double) * 2 * p[i].nx));
    L.inst_adj.push_back(p[i].enable_adjoint ? take(adj_bytes(p[i])) : 0);
  }
  L.total = o;
  return L;
}

}  // namespace

namespace lbm {

int report_error(int code, const char* msg) { return fail(code, "%s", msg); }

int measure_contact_angle_field(const double* d_rho, int nx, int ny, int wall, const int32_t b[4], double* d_partials,
                                hipStream_t s, double out[5]) {
  // host copies of the partials live on the stack: the measurement allocates nothing
  double part[kMeasurePartials];
  HIP_TRY(launch_minmax(d_rho, nx, ny, b, d_partials, kMeasureBlocks, s));
  HIP_TRY(hipMemcpyAsync(part, d_partials, sizeof(double) * 2 * kMeasureBlocks, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double lo = part[0], hi = part[kMeasureBlocks];
  for (int k = 0; k < kMeasureBlocks; ++k) {
    lo = std::min(lo, part[k]);
    hi = std::max(hi, part[kMeasureBlocks + k]);
  }
  const double mid = 0.5 * (hi + lo);
  const double sx = 0.5 * (b[0] + b[1]), sy = 0.5 * (b[2] + b[3]);
  HIP_TRY(launch_ca_moments(d_rho, nx, ny, b, wall, mid, sx, sy, d_partials, kMeasureBlocks, s));
  HIP_TRY(hipMemcpyAsync(part, d_partials, sizeof(double) * kMeasurePartials, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double m[kMeasureMoments] = {0};
  for (int j = 0; j < kMeasureMoments; ++j)
    for (int k = 0; k < kMeasureBlocks; ++k) m[j] += part[j * kMeasureBlocks + k];
  if (m[0] < 3) return fail(LBM_E_INVALID, "too few interface points in the box (%g)", m[0]);
  // Kasa normal equations for x^2 + y^2 + D x + E y + F = 0.
  double M3[3][4] = {{m[3], m[5], m[1], -(m[6] + m[7])},
                     {m[5], m[4], m[2], -(m[8] + m[9])},
                     {m[1], m[2], m[0], -(m[3] + m[4])}};
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (std::fabs(M3[r][col]) > std::fabs(M3[piv][col])) piv = r;
    if (M3[piv][col] == 0.0) return fail(LBM_E_INVALID, "degenerate circle fit");
    if (piv != col)
      for (int k = 0; k < 4; ++k) std::swap(M3[piv][k], M3[col][k]);
    for (int r = col + 1; r < 3; ++r) {
      const double f = M3[r][col] / M3[col][col];
      for (int k = col; k < 4; ++k) M3[r][k] -= f * M3[col][k];
    }
  }
  double sol[3];
  for (int r = 2; r >= 0; --r) {
    double v = M3[r][3];
    for (int k = r + 1; k < 3; ++k) v -= M3[r][k] * sol[k];
    sol[r] = v / M3[r][r];
  }
  const double xc = -0.5 * sol[0], yc = -0.5 * sol[1];
  const double R = std::sqrt(xc * xc + yc * yc - sol[2]);
  const double Xc = xc + sx, Yc = yc + sy;
  const double yw = wall == 0 ? 0.5 : ny - 1.5;
  double cth = wall == 0 ? (yw - Yc) / R : (Yc - yw) / R;
  cth = std::max(-1.0, std::min(1.0, cth));
  out[0] = std::acos(cth);
  out[1] = R;
  out[2] = Xc;
  out[3] = Yc;
  out[4] = m[0];
  return LBM_OK;
}

}  // namespace lbm

struct lbm_ctx {
  std::vector<Inst> inst;
  Layout L;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int storage = STORE_F64;
  int waves = kDefaultWaves;       // wavefronts per block of the step kernel (context-wide)
  bool prefetch = kDefaultPrefetch;  // next row's populations in flight during the collision
  std::vector<InstDesc> hdesc;
  std::vector<int32_t> first;       // [n+1] task ranges per instance
  std::vector<WaveTask> tasks;
  // two steps per launch where the selection allows it (walls, not periodic rows)
  bool step2 = false;
  int waves2 = kDefaultWaves2;
  std::vector<int32_t> first2;      // [n+1] ranges of the two-step tasks
  std::vector<WaveTask> tasks2;
  struct Chunk {
    hipGraphExec_t ex;
    int64_t launches;  // kernel launches of the step kernels in the graph (each flips the buffers once)
  };
  std::map<std::tuple<int, int, int>, Chunk> graphs;  // (selection, length, final check) -> graph
  hipEvent_t ev[2] = {nullptr, nullptr};  // lbm_step_timed: around the queued steps

  InstDesc* d_desc() { return (InstDesc*)(ws + L.desc); }
  WaveTask* d_tasks() { return (WaveTask*)(ws + L.tasks); }
  WaveTask* d_tasks2() { return (WaveTask*)(ws + L.tasks2); }
  WaveDiag* d_wdiag() { return (WaveDiag*)(ws + L.wdiag); }
  int32_t* d_first() { return (int32_t*)(ws + L.first); }
  int32_t* d_first2() { return (int32_t*)(ws + L.first2); }
  InstDiag* d_idiag() { return (InstDiag*)(ws + L.idiag); }
  double* d_partials() { return (double*)(ws + L.partials); }
  double* d_rho_scratch() { return (double*)(ws + L.rho_scratch); }
  int n() const { return (int)inst.size(); }

  // the tau = 1 BGK specialisation applies when every selected instance has tau == 1 exactly, no MRT rates and no
  // Martys-Chen walls (those run the general instances of both step kernels, so that one- and two-step launches
  // round alike)
  bool tau1(int sel) const {
    for (int i = 0; i < n(); ++i)
      if ((sel < 0 || i == sel) &&
          (inst[i].p.tau != 1.0 || uses_mrt(inst[i].p) || inst[i].p.boundary == LBM_WALLS_MARTYS_CHEN))
        return false;
    return true;
  }

  bool f32() const { return storage != STORE_F64; }
  // the two-step kernel covers the selection: walls everywhere, geometric or Martys-Chen (any collision, any
  // storage); periodic rows step one at a time
  bool step2_ok(int sel) const {
    if (!step2) return false;
    for (int i = 0; i < n(); ++i)
      if ((sel < 0 || i == sel) && inst[i].p.boundary == LBM_PERIODIC_Y) return false;
    return true;
  }

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second.ex);
    graphs.clear();
  }

  // Block decomposition of every instance: columns in aligned runs of 64 * waves (the last run takes the rest;
  // a 1-column remainder is merged so every block is at least 2 columns wide), rows balanced over
  // ceil((ny-2)/strip_rows) bands. Row bands outer, column blocks inner: blocks that run at the same time cover
  // whole contiguous rows of every population plane. Tasks of one instance are contiguous.
  void build_tasks() {
    tasks.clear();
    first.assign(n() + 1, 0);
    const int bwmax = 64 * waves;
    for (int i = 0; i < n(); ++i) {
      first[i] = (int)tasks.size();
      const int nx = inst[i].p.nx, nyf = inst[i].p.ny - 2;
      std::vector<int> xs;  // block start columns, then nx
      for (int x = 0; x < nx; x += bwmax) xs.push_back(x);
      xs.push_back(nx);
      const int nb = (int)xs.size() - 1;
      if (nb >= 2 && xs[nb] - xs[nb - 1] == 1) xs[nb - 1] -= 1;  // widths >= 2 (the previous block keeps >= 63)
      const int H = std::max(1, std::min(inst[i].strip_rows, nyf));
      const int sy = (nyf + H - 1) / H;
      for (int b = 0; b < sy; ++b) {
        const int ya = 1 + (int)((int64_t)nyf * b / sy), yb = 1 + (int)((int64_t)nyf * (b + 1) / sy);
        for (int a = 0; a < nb; ++a) {
          WaveTask t;
          t.inst = i;
          t.x0 = xs[a];
          t.y0 = ya;
          t.wh = (xs[a + 1] - xs[a]) | ((yb - ya) << 16);
          tasks.push_back(t);
        }
      }
    }
    first[n()] = (int)tasks.size();
    build_tasks2();
  }

  // Two-step tiles: ceil(nx / (64 waves2 - 8)) column tiles of balanced width, rows balanced over
  // ceil((ny-2)/strip_rows2) bands; bands outer, tiles inner (the kernel hands contiguous runs of this table to
  // one XCD each).
  void build_tasks2() {
    tasks2.clear();
    first2.assign(n() + 1, 0);
    const int wmax = 64 * waves2 - kStep2Halo;
    for (int i = 0; i < n(); ++i) {
      first2[i] = (int)tasks2.size();
      const int nx = inst[i].p.nx, nyf = inst[i].p.ny - 2;
      const int nt = (nx + wmax - 1) / wmax;
      const int H = std::max(1, std::min(inst[i].strip_rows2, nyf));
      const int sy = (nyf + H - 1) / H;
      for (int b = 0; b < sy; ++b) {
        const int ya = 1 + (int)((int64_t)nyf * b / sy), yb = 1 + (int)((int64_t)nyf * (b + 1) / sy);
        for (int a = 0; a < nt; ++a) {
          const int xa = (int)((int64_t)nx * a / nt), xb = (int)((int64_t)nx * (a + 1) / nt);
          WaveTask t;
          t.inst = i;
          t.x0 = xa;
          t.y0 = ya;
          t.wh = (xb - xa) | ((yb - ya) << 16);
          tasks2.push_back(t);
        }
      }
    }
    first2[n()] = (int)tasks2.size();
  }

  int upload_tables() {
    if (tasks.size() > L.task_cap || tasks2.size() > L.task2_cap) return fail(LBM_E_INVALID, "task table overflow");
    HIP_TRY(hipMemcpyAsync(d_tasks(), tasks.data(), sizeof(WaveTask) * tasks.size(), hipMemcpyHostToDevice, stream));
    if (!tasks2.empty())
      HIP_TRY(hipMemcpyAsync(d_tasks2(), tasks2.data(), sizeof(WaveTask) * tasks2.size(), hipMemcpyHostToDevice,
                             stream));
    HIP_TRY(hipMemcpyAsync(d_first(), first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_first2(), first2.data(), sizeof(int32_t) * first2.size(), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipMemcpyAsync(d_desc(), hdesc.data(), sizeof(InstDesc) * hdesc.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return LBM_OK;
  }
};

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

size_t lbm_workspace_bytes(const lbm_params* p, int32_t n_inst) {
  std::string why;
  if (!valid_params(p, n_inst, &why)) {
    fail(LBM_E_INVALID, "%s", why.c_str());
    return 0;
  }
  return make_layout(p, n_inst).total;
}

int lbm_create(const lbm_params* p, int32_t n_inst, void* d_workspace, size_t ws_bytes, void* hip_stream,
               lbm_ctx** out) {
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!valid_params(p, n_inst, &why)) return fail(LBM_E_INVALID, "%s", why.c_str());
  Layout L = make_layout(p, n_inst);
  if (!d_workspace || ((uintptr_t)d_workspace & 255)) return fail(LBM_E_WORKSPACE, "workspace NULL or not 256-B aligned");
  if (ws_bytes < L.total) return fail(LBM_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.total);

  lbm_ctx* c = new lbm_ctx();
  c->L = L;
  c->ws = (char*)d_workspace;
  c->ws_bytes = ws_bytes;
  c->stream = (hipStream_t)hip_stream;
  c->storage = p[0].precision == LBM_F64 ? STORE_F64 : (p[0].precision == LBM_F32_SHIFTED_MIXED ? STORE_F32M : STORE_F32);
  if (c->storage == STORE_F64) {
    c->waves = kDefaultWaves64;
    c->prefetch = kDefaultPrefetch64;
  }
  // two steps per launch by default (where the selection allows it) on contexts of at least kStep2MinNodes fluid
  // nodes, in blocks of one wavefront while every instance is below kNarrow2MaxNodes; variants 1..8 choose a
  // one-step shape, 9..12 the two-step kernel with 1, 2, 4 or 8 wavefronts per block
  {
    double nodes = 0;
    for (int i = 0; i < n_inst; ++i) nodes += (double)p[i].nx * (p[i].ny - 2);
    c->step2 = nodes >= kStep2MinNodes;
    int min_nx = p[0].nx;
    double max_inst = 0;
    bool special = true;  // every instance takes the tau = 1 BGK specialisation (see tau1)
    for (int i = 0; i < n_inst; ++i) {
      min_nx = std::min(min_nx, p[i].nx);
      max_inst = std::max(max_inst, (double)p[i].nx * (p[i].ny - 2));
      special = special && p[i].tau == 1.0 && !uses_mrt(p[i]) && p[i].boundary == LBM_WALLS_Y;
    }
    if (max_inst < kNarrow2MaxNodes) c->waves2 = 1;
    else if (c->storage == STORE_F32 && special && nodes >= kWide2MinNodes && min_nx >= kWide2MinNx) c->waves2 = 8;
  }
  if (p[0].step_variant > 0 && p[0].step_variant <= 2 * kNumWaveChoices) {
    c->waves = kWaveChoices[(p[0].step_variant - 1) % kNumWaveChoices];
    c->prefetch = (p[0].step_variant - 1) / kNumWaveChoices == 1;
    c->step2 = false;
  } else if (p[0].step_variant > 2 * kNumWaveChoices) {
    c->waves2 = kWaveChoices[p[0].step_variant - 2 * kNumWaveChoices - 1];
    c->step2 = true;
  }
  c->inst.resize(n_inst);
  c->hdesc.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    Inst& I = c->inst[i];
    I.p = p[i];
    I.pitch = (p[i].nx + 63) / 64 * 64;
    I.plane = (int64_t)I.pitch * (p[i].ny - 2);
    I.strip_rows = p[i].strip_rows > 0 ? p[i].strip_rows
                                        : (p[i].precision == LBM_F64 ? kDefaultStripRows64 : kDefaultStripRows);
    I.strip_rows2 = p[i].strip_rows > 0 ? p[i].strip_rows : kDefaultStripRows2;
    PwEos pw{};
    if (p[i].eos == LBM_EOS_PIECEWISE_LINEAR) {
      pw_from_params(p[i], &pw);  // solvable: checked by valid_params
      I.rho_v = p[i].pw_rho[0];
      I.rho_l = p[i].pw_rho[1];
      I.rho_cap = pw_rho_cap(pw);
    } else {
      cs_critical(p[i].eos_a, p[i].eos_b, p[i].eos_R, &I.rho_c, &I.T_c);
      I.T = p[i].T_over_Tc * I.T_c;
      Eos E{p[i].eos_a, p[i].eos_b, p[i].eos_R, I.T};
      if (!cs_maxwell(E, I.rho_c, &I.rho_v, &I.rho_l)) {
        delete c;
        return fail(LBM_E_INVALID, "instance %d: no coexistence found", i);
      }
      I.rho_cap = cs_rho_cap(E, I.rho_c);
    }
    I.pw_r1 = pw.r1;
    I.pw_r2 = pw.r2;
    for (int k = 0; k < 2; ++k) I.off_f[k] = L.inst_f[k][i];
    I.off_th = L.inst_th[i];
    I.off_ghost = L.inst_ghost[i];
    I.off_adj = L.inst_adj[i];
    const int nx = p[i].nx;
    I.cos_th.assign(2 * nx, std::cos(M_PI / 2));
    I.cot_th.assign(2 * nx, std::cos(M_PI / 2) / std::sin(M_PI / 2));
    I.sin_th.assign(2 * nx, 1.0);

    InstDesc& d = c->hdesc[i];
    std::memset(&d, 0, sizeof d);
    d.f[0] = c->ws + I.off_f[0];
    d.f[1] = c->ws + I.off_f[1];
    double* th = (double*)(c->ws + I.off_th);
    d.cos_th = th;
    d.cot_th = th + 2 * nx;
    d.sin_th = th + 4 * nx;
    d.ghost = (double*)(c->ws + I.off_ghost);
    d.nx = nx;
    d.ny = p[i].ny;
    d.pitch = I.pitch;
    d.wet_iters = p[i].wet_iters;
    d.plane = I.plane;
    d.cur = 0;
    d.periodic_y = p[i].boundary == LBM_PERIODIC_Y ? 1 : 0;
    d.wall_mc = p[i].boundary == LBM_WALLS_MARTYS_CHEN ? 1 : 0;
    d.gw_half[0] = d.wall_mc ? 0.5 * p[i].G_w[0] : 0.0;
    d.gw_half[1] = d.wall_mc ? 0.5 * p[i].G_w[1] : 0.0;
    d.RT = p[i].eos_R * I.T;
    d.eos_a = p[i].eos_a;
    d.eos_b4 = 0.25 * p[i].eos_b;
    d.two_over_Gpsi = 2.0 / p[i].G;
    d.G_f = p[i].G;
    d.A = p[i].A;
    d.inv_tau = 1.0 / p[i].tau;
    d.force_pref = 1.0 - 0.5 / p[i].tau;
    d.body_fx = p[i].body_force[0];
    d.body_fy = p[i].body_force[1];
    d.rho0 = (p[i].precision == LBM_F32_SHIFTED || p[i].precision == LBM_F32_SHIFTED_MIXED) ? p[i].rho0_shift : 0.0;
    d.rho_fp64_below = p[i].precision == LBM_F64 ? 0.0 : p[i].rho_fp64_below;
    d.rho_cap_hi = I.rho_cap * (1.0 - 1e-6);
    d.eos_kind = p[i].eos;
    d.mrt = uses_mrt(p[i]) ? 1 : 0;
    d.s_e = p[i].mrt_rates[0] != 0.0 ? p[i].mrt_rates[0] : 1.0 / p[i].tau;
    d.s_eps = p[i].mrt_rates[1] != 0.0 ? p[i].mrt_rates[1] : 1.0 / p[i].tau;
    d.s_q = p[i].mrt_rates[2] != 0.0 ? p[i].mrt_rates[2] : 1.0 / p[i].tau;
    d.kq = 0.5 * p[i].kappa * p[i].G;
    if (p[i].eos == LBM_EOS_PIECEWISE_LINEAR) {
      for (int k = 0; k < 3; ++k) d.pw_t[k] = p[i].pw_theta[k];
      d.pw_r1 = pw.r1;
      d.pw_r2 = pw.r2;
      d.pw_p1 = pw.p(pw.r1);
      d.pw_p2 = pw.p(pw.r2);
    }
  }
  {
    // default strip height from the total work (see kDefaultStripRows)
    int cus = 256, dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    double nodes = 0;
    for (int i = 0; i < n_inst; ++i) nodes += (double)p[i].nx * (p[i].ny - 2);
    const int hmax = c->storage == STORE_F64 ? kDefaultStripRows64 : kDefaultStripRows;
    const int h = (int)std::max<long>(kMinDefaultStripRows,
                                      std::min<long>(hmax, std::lround(nodes / (2.0 * cus * 64 * c->waves))));
    for (int i = 0; i < n_inst; ++i)
      if (p[i].strip_rows <= 0) c->inst[i].strip_rows = h;
    // two-step kernel: one round of resident blocks over all instances, each task a tile of a strip; fewer, taller
    // strips than that leave compute units idle, more add a partial second round and more halo rows
    int per_cu = 0;
    if (step2_blocks_per_cu(c->waves2, c->storage, !c->tau1(-1), &per_cu) == hipSuccess &&
        per_cu > 0) {
      const int wmax = 64 * c->waves2 - kStep2Halo;
      double tile_rows = 0;
      for (int i = 0; i < n_inst; ++i) tile_rows += (double)((p[i].nx + wmax - 1) / wmax) * (p[i].ny - 2);
      const long hcap = c->storage == STORE_F64 ? kMaxStripRows2F64 : kMaxStripRows2;
      int h2 = (int)std::max<long>(kMinStripRows2, std::min<long>(hcap,
                                   (long)std::ceil(tile_rows / ((double)cus * per_cu))));
      // whole strips per instance can add tasks beyond one round: raise the height until they fit
      auto ntasks2 = [&](int h) {
        double n = 0;
        for (int i = 0; i < n_inst; ++i)
          n += (double)((p[i].nx + wmax - 1) / wmax) * (double)((p[i].ny - 2 + h - 1) / h);
        return n;
      };
      while (h2 < hcap && ntasks2(h2) > (double)cus * per_cu) ++h2;
      for (int i = 0; i < n_inst; ++i)
        if (p[i].strip_rows <= 0) c->inst[i].strip_rows2 = h2;
    }
  }
  c->build_tasks();
  int rc = c->upload_tables();
  if (rc == LBM_OK) {
    for (int i = 0; i < n_inst; ++i) {
      Inst& I = c->inst[i];
      std::vector<double> th(6 * (size_t)I.p.nx);
      std::copy(I.cos_th.begin(), I.cos_th.end(), th.begin());
      std::copy(I.cot_th.begin(), I.cot_th.end(), th.begin() + 2 * I.p.nx);
      std::copy(I.sin_th.begin(), I.sin_th.end(), th.begin() + 4 * I.p.nx);
      hipError_t e = hipMemcpyAsync(c->ws + I.off_th, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice,
                                    c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) { rc = fail(LBM_E_HIP, "theta upload: %s", hipGetErrorString(e)); break; }
    }
  }
  if (rc == LBM_OK) {
    hipError_t e = launch_zero_diag(c->d_idiag(), n_inst, c->stream);
    if (e != hipSuccess) rc = fail(LBM_E_HIP, "zero diag: %s", hipGetErrorString(e));
  }
  if (rc != LBM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return fail(LBM_E_INVALID, "NULL context");
  c->drop_graphs();
  for (hipEvent_t& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return LBM_OK;
}

#define CHECK_INST(c, i)                                                                       \
  do {                                                                                         \
    if (!(c)) return fail(LBM_E_INVALID, "NULL context");                                      \
    if ((i) < 0 || (i) >= (c)->n()) return fail(LBM_E_INVALID, "instance %d out of range", (i)); \
  } while (0)

int lbm_eos_info(const lbm_ctx* c, int32_t inst, double out[6]) {
  if (!c) return fail(LBM_E_INVALID, "NULL context");
  if (inst < 0 || inst >= (int)c->inst.size()) return fail(LBM_E_INVALID, "instance out of range");
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  const Inst& I = c->inst[inst];
  out[0] = I.rho_v;
  out[1] = I.rho_l;
  const bool pw = I.p.eos == LBM_EOS_PIECEWISE_LINEAR;
  out[2] = pw ? I.pw_r1 : I.T;
  out[3] = pw ? I.pw_r2 : I.T_c;
  out[4] = pw ? 0.0 : I.rho_c;
  out[5] = I.rho_cap;
  return LBM_OK;
}

int lbm_coexistence(const lbm_ctx* c, int32_t inst, double out[2]) {
  if (!c) return fail(LBM_E_INVALID, "NULL context");
  if (inst < 0 || inst >= (int)c->inst.size()) return fail(LBM_E_INVALID, "instance out of range");
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  out[0] = c->inst[inst].rho_v;
  out[1] = c->inst[inst].rho_l;
  return LBM_OK;
}

int lbm_init_droplet(lbm_ctx* c, int32_t inst, int32_t n, const double* xc, const double* yc, const double* R,
                     double width, double rho_l, double rho_v) {
  CHECK_INST(c, inst);
  if (n < 0 || n > kMaxDrops) return fail(LBM_E_INVALID, "droplet count %d outside [0, %d]", n, kMaxDrops);
  if (n > 0 && (!xc || !yc || !R)) return fail(LBM_E_INVALID, "droplet arrays NULL");
  if (!(width > 0) || !std::isfinite(width)) return fail(LBM_E_INVALID, "width must be > 0");
  Inst& I = c->inst[inst];
  if (!(rho_l > 0)) rho_l = I.rho_l;
  if (!(rho_v > 0)) rho_v = I.rho_v;
  if (!std::isfinite(rho_l) || !std::isfinite(rho_v)) return fail(LBM_E_INVALID, "densities not finite");
  std::vector<double> drops(3 * (size_t)std::max(n, 1));
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(xc[k]) || !std::isfinite(yc[k]) || !std::isfinite(R[k]))
      return fail(LBM_E_INVALID, "droplet %d not finite", k);
    drops[3 * k] = xc[k];
    drops[3 * k + 1] = yc[k];
    drops[3 * k + 2] = R[k];
  }
  double* dd = (double*)(c->ws + c->L.drops);
  if (n > 0) HIP_TRY(hipMemcpyAsync(dd, drops.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(launch_init_droplets(c->storage, c->d_desc(), inst, I.p.ny - 2, I.p.nx, dd, n, width, rho_l, rho_v,
                               c->d_rho_scratch(), c->stream));
  HIP_TRY(launch_wetting(c->storage, c->d_desc(), inst, I.p.nx, c->stream));
  HIP_TRY(launch_zero_diag(c->d_idiag() + inst, 1, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  I.initialized = true;
  I.steps = 0;
  return LBM_OK;
}

int lbm_apply_wetting(lbm_ctx* c, int32_t inst, const double* theta_bottom, const double* theta_top) {
  CHECK_INST(c, inst);
  Inst& I = c->inst[inst];
  const int nx = I.p.nx;
  const double* src[2] = {theta_bottom, theta_top};
  for (int w = 0; w < 2; ++w) {
    if (!src[w]) continue;
    for (int x = 0; x < nx; ++x) {
      const double th = src[w][x];
      if (!(th > 0 && th < M_PI)) return fail(LBM_E_INVALID, "theta[%d][%d] = %g outside (0, pi)", w, x, th);
    }
  }
  for (int w = 0; w < 2; ++w) {
    if (!src[w]) continue;
    for (int x = 0; x < nx; ++x) {
      const double th = src[w][x];
      I.cos_th[w * nx + x] = std::cos(th);
      I.sin_th[w * nx + x] = std::sin(th);
      I.cot_th[w * nx + x] = std::cos(th) / std::sin(th);
    }
  }
  std::vector<double> th(6 * (size_t)nx);
  std::copy(I.cos_th.begin(), I.cos_th.end(), th.begin());
  std::copy(I.cot_th.begin(), I.cot_th.end(), th.begin() + 2 * nx);
  std::copy(I.sin_th.begin(), I.sin_th.end(), th.begin() + 4 * nx);
  HIP_TRY(hipMemcpyAsync(c->ws + I.off_th, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice, c->stream));
  if (I.initialized) HIP_TRY(launch_wetting(c->storage, c->d_desc(), inst, nx, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

namespace {

// Queue `count` steps for the selection (task range), buffer flips starting at 0, checks every K (0 = none)
// counting from the first queued step, plus one after the last step if final_check. A check reads the input state
// of its step. Where the selection allows it, an unchecked step and the step after it go into one two-step launch,
// which takes the second step's check if it has one (its input is the state after the first); a checked step not
// paired that way is a one-step launch. Each launch flips the buffers once. *launches receives the launch count;
// dry = true only counts.
int queue_steps(lbm_ctx* c, int sel, int64_t count, int K, bool final_check, int64_t* launches, bool dry = false) {
  const int a = sel < 0 ? 0 : c->first[sel];
  const int b = sel < 0 ? c->first[c->n()] : c->first[sel + 1];
  const int a2 = sel < 0 ? 0 : c->first2[sel];
  const int b2 = sel < 0 ? c->first2[c->n()] : c->first2[sel + 1];
  const int ninst = sel < 0 ? c->n() : 1;
  const int inst0 = sel < 0 ? 0 : sel;
  const bool two = c->step2_ok(sel);
  auto chk_at = [&](int64_t i) { return (K > 0 && (i + 1) % K == 0) || (final_check && i == count - 1); };
  int64_t nl = 0;
  for (int64_t i = 0; i < count; ++nl) {
    const bool chk = chk_at(i);
    if (two && !chk && i + 1 < count) {
      const bool chk2 = chk_at(i + 1);
      if (!dry) {
        HIP_TRY(launch_step2(c->d_desc(), c->d_tasks2() + a2, b2 - a2, c->waves2, c->storage, !c->tau1(sel),
                             (int)(nl & 1), c->stream, chk2 ? c->d_wdiag() + a2 : nullptr));
        if (chk2)
          HIP_TRY(launch_finalize_diag(c->d_tasks2(), c->d_first2(), ninst, inst0, c->d_wdiag(), c->d_idiag(),
                                       c->d_desc(), c->stream));
      }
      i += 2;
      continue;
    }
    if (!dry) {
      HIP_TRY(launch_step(c->storage, chk, c->tau1(sel), c->waves, c->prefetch, c->d_desc(), c->d_tasks() + a, b - a,
                          (int)(nl & 1), c->d_wdiag() + a, c->stream));
      if (chk)
        HIP_TRY(launch_finalize_diag(c->d_tasks(), c->d_first(), ninst, inst0, c->d_wdiag(), c->d_idiag(),
                                     c->d_desc(), c->stream));
    }
    i += 1;
  }
  *launches = nl;
  return LBM_OK;
}

// Cached graphs: one per (selection, length, final check); lengths other than the chunk length come from the
// remainder of a call, so a bounded number of them is kept.
constexpr size_t kMaxGraphs = 64;

int get_graph(lbm_ctx* c, int sel, int len, int K, bool final_check, lbm_ctx::Chunk* out) {
  auto key = std::make_tuple(sel, len, final_check ? 1 : 0);
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return LBM_OK;
  }
  if (c->graphs.size() >= kMaxGraphs) {
    *out = lbm_ctx::Chunk{nullptr, 0};  // the caller queues plain launches
    return LBM_OK;
  }
  hipGraph_t g = nullptr;
  int64_t nl = 0;
  HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = queue_steps(c, sel, len, K, final_check, &nl);
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(LBM_E_HIP, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(LBM_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
  c->graphs[key] = lbm_ctx::Chunk{ex, nl};
  *out = c->graphs[key];
  return LBM_OK;
}

}  // namespace

namespace {

// lbm_step; with ev (two events) the first is recorded before the first queued launch and the second after the
// last one, ahead of the closing host synchronization.
int step_impl(lbm_ctx* c, int32_t inst, int64_t nsteps, hipEvent_t* ev) {
  if (!c) return fail(LBM_E_INVALID, "NULL context");
  if (inst < -1 || inst >= c->n()) return fail(LBM_E_INVALID, "instance %d out of range", inst);
  if (nsteps < 0) return fail(LBM_E_INVALID, "nsteps < 0");
  for (int i = 0; i < c->n(); ++i)
    if ((inst < 0 || i == inst) && !c->inst[i].initialized)
      return fail(LBM_E_STATE, "instance %d has no state (call lbm_init_droplet or lbm_set_populations)", i);
  if (ev) HIP_TRY(hipEventRecord(ev[0], c->stream));
  if (nsteps > 0) {
    const int K = c->inst[inst < 0 ? 0 : inst].p.check_every;
    // chunk length: whole check periods with an even number of launches, so that every replay starts from the
    // same buffer with the same check positions
    int len = K > 0 ? (K % 2 == 0 ? K : 2 * K) : 64;
    int64_t nl_len = 0;
    queue_steps(c, inst, len, K, false, &nl_len, true);
    if (nl_len & 1) len *= 2;
    int64_t left = nsteps, launches = 0;
    const bool graphs = c->stream != nullptr && len <= 4096;
    if (graphs && nsteps >= len) {
      lbm_ctx::Chunk ch;
      int rc = get_graph(c, inst, len, K, false, &ch);
      if (rc != LBM_OK) return rc;
      while (ch.ex && left >= len) {
        HIP_TRY(hipGraphLaunch(ch.ex, c->stream));
        left -= len;
        launches += ch.launches;
      }
    }
    // The rest (fewer steps than a chunk): one graph of exactly that length, or plain launches once the cache is
    // full. Chunk replays end on the starting buffer, so its flips restart at 0 and check positions stay aligned.
    if (left > 0 && graphs && left < len) {
      lbm_ctx::Chunk ch;
      int rc = get_graph(c, inst, (int)left, K, K > 0, &ch);
      if (rc != LBM_OK) return rc;
      if (ch.ex) {
        HIP_TRY(hipGraphLaunch(ch.ex, c->stream));
        launches += ch.launches;
        left = 0;
      }
    }
    if (left > 0) {
      int64_t nl = 0;
      int rc = queue_steps(c, inst, left, K, K > 0, &nl);
      if (rc != LBM_OK) return rc;
      launches += nl;
    }
    if (launches & 1) {
      for (int i = 0; i < c->n(); ++i) {
        if (inst >= 0 && i != inst) continue;
        c->hdesc[i].cur ^= 1;
        HIP_TRY(launch_set_cur(c->d_desc(), i, c->hdesc[i].cur, c->stream));
      }
    }
    for (int i = 0; i < c->n(); ++i)
      if (inst < 0 || i == inst) c->inst[i].steps += nsteps;
  }
  if (ev) HIP_TRY(hipEventRecord(ev[1], c->stream));
  const int K = c->inst[inst < 0 ? 0 : inst].p.check_every;
  if (K > 0 && nsteps > 0) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<InstDiag> g(c->n());
    HIP_TRY(hipMemcpy(g.data(), c->d_idiag(), sizeof(InstDiag) * c->n(), hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n(); ++i)
      if ((inst < 0 || i == inst) && g[i].nonfinite > 0)
        return fail(LBM_E_UNSTABLE, "instance %d: non-finite density at a check (%lld nodes)", i,
                    (long long)g[i].nonfinite);
  }
  return LBM_OK;
}

}  // namespace

int lbm_step(lbm_ctx* c, int32_t inst, int64_t nsteps) { return step_impl(c, inst, nsteps, nullptr); }

int lbm_step_timed(lbm_ctx* c, int32_t inst, int64_t nsteps, double* ms) {
  if (!c || !ms) return fail(LBM_E_INVALID, "NULL context or ms");
  for (hipEvent_t& e : c->ev)
    if (!e) HIP_TRY(hipEventCreate(&e));
  const int rc = step_impl(c, inst, nsteps, c->ev);
  if (rc != LBM_OK && rc != LBM_E_UNSTABLE) return rc;
  HIP_TRY(hipEventSynchronize(c->ev[1]));
  float t = 0.0f;
  HIP_TRY(hipEventElapsedTime(&t, c->ev[0], c->ev[1]));
  *ms = t;
  return rc;
}

int lbm_get_diag(lbm_ctx* c, int32_t inst, lbm_diag* out) {
  CHECK_INST(c, inst);
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  InstDiag g;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&g, c->d_idiag() + inst, sizeof g, hipMemcpyDeviceToHost));
  out->mass = g.mass;
  out->checks = g.checks;
  out->nonfinite = g.nonfinite;
  out->psi_clamps = g.psi_clamps;
  out->ghost_clamps = g.ghost_clamps;
  out->steps = c->inst[inst].steps;
  return LBM_OK;
}

int lbm_mass(lbm_ctx* c, int32_t inst, double* out) {
  CHECK_INST(c, inst);
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  if (!c->inst[inst].initialized) return fail(LBM_E_STATE, "no state");
  const Inst& I = c->inst[inst];
  HIP_TRY(launch_mass(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, c->d_partials(), kMeasureBlocks, c->stream));
  std::vector<double> part(kMeasureBlocks);
  HIP_TRY(hipMemcpyAsync(part.data(), c->d_partials(), sizeof(double) * kMeasureBlocks, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double m = 0.0;
  for (double v : part) m += v;
  *out = m;
  return LBM_OK;
}

int lbm_get_rho(lbm_ctx* c, int32_t inst, double* dst, int32_t dst_on_device) {
  CHECK_INST(c, inst);
  if (!dst) return fail(LBM_E_INVALID, "dst is NULL");
  if (!c->inst[inst].initialized) return fail(LBM_E_STATE, "no state");
  const Inst& I = c->inst[inst];
  const size_t n = (size_t)I.p.nx * I.p.ny;
  double* target = dst_on_device ? dst : c->d_rho_scratch();
  HIP_TRY(launch_wetting(c->storage, c->d_desc(), inst, I.p.nx, c->stream));
  HIP_TRY(launch_get_rho(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, target, c->stream));
  if (!dst_on_device) {
    HIP_TRY(hipMemcpyAsync(dst, target, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

int lbm_get_populations(lbm_ctx* c, int32_t inst, double* dst, int32_t dst_on_device) {
  CHECK_INST(c, inst);
  if (!dst) return fail(LBM_E_INVALID, "dst is NULL");
  if (!c->inst[inst].initialized) return fail(LBM_E_STATE, "no state");
  const Inst& I = c->inst[inst];
  const size_t n = (size_t)I.p.nx * (I.p.ny - 2);
  if (dst_on_device) {
    HIP_TRY(launch_get_pops(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, 0, 9, dst, c->stream));
    return LBM_OK;
  }
  // host destination: one population plane at a time through the density scratch ([nx][ny] doubles)
  for (int q = 0; q < 9; ++q) {
    HIP_TRY(launch_get_pops(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, q, q + 1, c->d_rho_scratch(), c->stream));
    HIP_TRY(hipMemcpyAsync(dst + q * n, c->d_rho_scratch(), sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

int lbm_set_populations(lbm_ctx* c, int32_t inst, const double* src, int32_t src_on_device) {
  CHECK_INST(c, inst);
  if (!src) return fail(LBM_E_INVALID, "src is NULL");
  Inst& I = c->inst[inst];
  const size_t n = (size_t)I.p.nx * (I.p.ny - 2);
  // stored plane q takes physical plane q (nodes streaming into the fluid) and plane opp(q) (wall bounce-back)
  for (int p = 0; p < 9; ++p) {
    const double* plane = src + p * n;
    if (!src_on_device) {
      HIP_TRY(hipMemcpyAsync(c->d_rho_scratch(), plane, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
      plane = c->d_rho_scratch();
    }
    HIP_TRY(launch_set_plane(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, p, p, plane, c->stream));
    if (kOpp[p] != p)
      HIP_TRY(launch_set_plane(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, kOpp[p], p, plane, c->stream));
    if (!src_on_device) HIP_TRY(hipStreamSynchronize(c->stream));
  }
  HIP_TRY(launch_wetting(c->storage, c->d_desc(), inst, I.p.nx, c->stream));
  HIP_TRY(launch_zero_diag(c->d_idiag() + inst, 1, c->stream));
  I.initialized = true;
  I.steps = 0;
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx* c, int32_t inst) {
  if (!c || inst < 0 || inst >= (int)c->inst.size()) {
    fail(LBM_E_INVALID, "bad context or instance");
    return 0;
  }
  const Inst& I = c->inst[inst];
  return storage_bytes(I.p.precision) * 9 * (size_t)I.pitch * (I.p.ny - 2);
}

int lbm_get_state(lbm_ctx* c, int32_t inst, void* d_dst) {
  CHECK_INST(c, inst);
  if (!d_dst) return fail(LBM_E_INVALID, "dst is NULL");
  if (!c->inst[inst].initialized) return fail(LBM_E_STATE, "no state");
  HIP_TRY(hipMemcpyAsync(d_dst, c->hdesc[inst].f[c->hdesc[inst].cur], lbm_state_bytes(c, inst),
                         hipMemcpyDeviceToDevice, c->stream));
  return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, int32_t inst, const void* d_src) {
  CHECK_INST(c, inst);
  if (!d_src) return fail(LBM_E_INVALID, "src is NULL");
  HIP_TRY(hipMemcpyAsync(c->hdesc[inst].f[c->hdesc[inst].cur], d_src, lbm_state_bytes(c, inst),
                         hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(launch_wetting(c->storage, c->d_desc(), inst, c->inst[inst].p.nx, c->stream));
  c->inst[inst].initialized = true;
  return LBM_OK;
}

int lbm_measure_contact_angle(lbm_ctx* c, int32_t inst, int32_t wall, const int32_t box[4], double out[5]) {
  CHECK_INST(c, inst);
  if (!box || !out) return fail(LBM_E_INVALID, "box/out NULL");
  if (wall != 0 && wall != 1) return fail(LBM_E_INVALID, "wall must be 0 or 1");
  if (!c->inst[inst].initialized) return fail(LBM_E_STATE, "no state");
  const Inst& I = c->inst[inst];
  int32_t b[4] = {std::max(box[0], 0), std::min(box[1], I.p.nx), std::max(box[2], 1), std::min(box[3], I.p.ny - 1)};
  if (b[1] - b[0] < 2 || b[3] - b[2] < 2) return fail(LBM_E_INVALID, "box too small after clipping");
  double* rho = c->d_rho_scratch();
  HIP_TRY(launch_wetting(c->storage, c->d_desc(), inst, I.p.nx, c->stream));
  HIP_TRY(launch_get_rho(c->storage, c->d_desc(), inst, I.p.nx, I.p.ny, rho, c->stream));
  return measure_contact_angle_field(rho, I.p.nx, I.p.ny, wall, b, c->d_partials(), c->stream, out);
}

int lbm_autotune(lbm_ctx* c, int32_t inst, int32_t trial_steps, int32_t* chosen) {
  if (!c) return fail(LBM_E_INVALID, "NULL context");
  if (inst < -1 || inst >= c->n()) return fail(LBM_E_INVALID, "instance out of range");
  if (trial_steps <= 0 || !chosen) return fail(LBM_E_INVALID, "trial_steps must be > 0 and chosen non-NULL");
  for (int i = 0; i < c->n(); ++i)
    if ((inst < 0 || i == inst) && !c->inst[i].initialized) return fail(LBM_E_STATE, "instance %d has no state", i);
  // The selection is timed as it runs: one launch over all its tasks. Trial launches read the state buffer and
  // write the spare one (flip 0), walking up and down alternately, so the state is not modified. Times are compared
  // per time step (a two-step launch counts twice).
  std::vector<int> sel;
  int max_nx = 0, max_nyf = 0;
  for (int i = 0; i < c->n(); ++i)
    if (inst < 0 || i == inst) {
      sel.push_back(i);
      max_nx = std::max(max_nx, c->inst[i].p.nx);
      max_nyf = std::max(max_nyf, c->inst[i].p.ny - 2);
    }
  std::map<std::pair<int, int>, std::vector<int>> shapes;  // shape classes of the selection
  for (int i : sel) shapes[{c->inst[i].p.nx, c->inst[i].p.ny}].push_back(i);
  const int cand[] = {2, 4, 8, 12, 16, 24, 32, 48, 64, 128};
  const int cand2[] = {8, 12, 16, 24, 32, 40, 48, 56, 64, 96, 128};
  std::vector<int> saved(c->n()), saved2(c->n());
  for (int i = 0; i < c->n(); ++i) {
    saved[i] = c->inst[i].strip_rows;
    saved2[i] = c->inst[i].strip_rows2;
  }
  // On every exit: the events are destroyed, and unless the search completed the saved shapes come back with their
  // task tables (the trials uploaded theirs) and no graph of a trial shape survives.
  struct Guard {
    lbm_ctx* c;
    const std::vector<int>& saved;
    const std::vector<int>& saved2;
    int waves, waves2;
    bool pf, step2;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool done = false;
    ~Guard() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (done) return;
      c->waves = waves;
      c->prefetch = pf;
      c->waves2 = waves2;
      c->step2 = step2;
      for (int i = 0; i < c->n(); ++i) {
        c->inst[i].strip_rows = saved[i];
        c->inst[i].strip_rows2 = saved2[i];
      }
      c->build_tasks();
      (void)c->upload_tables();
      c->drop_graphs();
    }
  } guard{c, saved, saved2, c->waves, c->waves2, c->prefetch, c->step2};
  HIP_TRY(hipEventCreate(&guard.e0));
  HIP_TRY(hipEventCreate(&guard.e1));
  hipEvent_t e0 = guard.e0, e1 = guard.e1;
  // ms per time step of the current shape: one-step launches, or (two = true) two-step launches
  auto trial = [&](bool two, float* ms) -> int {
    c->build_tasks();
    int rc = c->upload_tables();
    if (rc != LBM_OK) return rc;
    const int a = c->first[sel.front()], b = c->first[sel.back() + 1];
    const int a2 = c->first2[sel.front()], b2 = c->first2[sel.back() + 1];
    const int launches = two ? std::max(1, trial_steps / 2) : trial_steps;
    for (int k = 0; k <= launches; ++k) {
      if (k == 1) HIP_TRY(hipEventRecord(e0, c->stream));  // launch 0 warms up
      if (two)
        HIP_TRY(launch_step2(c->d_desc(), c->d_tasks2() + a2, b2 - a2, c->waves2, c->storage, !c->tau1(inst), 0,
                             c->stream));
      else
        HIP_TRY(launch_step(c->storage, false, c->tau1(inst), c->waves, c->prefetch, c->d_desc(), c->d_tasks() + a,
                            b - a, 0, c->d_wdiag() + a, c->stream, k & 1));
    }
    HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(hipEventSynchronize(e1));
    *ms = 0;
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    *ms /= (float)(two ? 2 * launches : launches);
    return LBM_OK;
  };
  // 1. one-step kernel: wavefronts per block, prefetch and one strip height for the whole selection
  float best = 1e30f;
  int best_w = c->waves, best_h = saved[sel.front()];
  bool best_pf = c->prefetch;
  for (int pf = 0; pf < 2; ++pf)
    for (int wi = 0; wi < kNumWaveChoices; ++wi) {
      const int w = kWaveChoices[wi];
      if (w > 1 && 64 * (w / 2) >= max_nx) continue;  // more waves than columns
      for (int h : cand) {
        if (h > max_nyf && h != cand[0]) continue;
        c->waves = w;
        c->prefetch = pf == 1;
        for (int i : sel) c->inst[i].strip_rows = h;
        float ms;
        int rc = trial(false, &ms);
        if (rc != LBM_OK) return rc;
        if (ms < best) { best = ms; best_w = w; best_pf = pf == 1; best_h = h; }
      }
    }
  c->waves = best_w;
  c->prefetch = best_pf;
  for (int i : sel) c->inst[i].strip_rows = best_h;
  // 1b. two-step kernel where the selection allows it: wavefronts per block and one strip height
  bool use2 = false;
  c->step2 = true;
  if (c->step2_ok(inst)) {
    float best2 = 1e30f;
    int bw2 = c->waves2, bh2 = saved2[sel.front()];
    for (int wi = 0; wi < kNumWaveChoices; ++wi) {
      const int w = kWaveChoices[wi];
      if (w > 1 && 64 * (w / 2) - kStep2Halo >= max_nx) continue;
      for (int h : cand2) {
        if (h > max_nyf && h != cand2[0]) continue;
        c->waves2 = w;
        for (int i : sel) c->inst[i].strip_rows2 = h;
        float ms;
        int rc = trial(true, &ms);
        if (rc != LBM_OK) return rc;
        if (ms < best2) { best2 = ms; bw2 = w; bh2 = h; }
      }
    }
    c->waves2 = bw2;
    for (int i : sel) c->inst[i].strip_rows2 = bh2;
    use2 = best2 < best;
    if (use2) best = best2;
  }
  c->step2 = use2 || (guard.step2 && !c->step2_ok(inst));
  // 2. with several shape classes, refine each class's strip height in turn (the others held)
  if (shapes.size() > 1) {
    for (auto& kv : shapes) {
      const int nyf = kv.first.second - 2;
      int keep = use2 ? c->inst[kv.second.front()].strip_rows2 : c->inst[kv.second.front()].strip_rows;
      for (int h : use2 ? std::vector<int>(std::begin(cand2), std::end(cand2))
                        : std::vector<int>(std::begin(cand), std::end(cand))) {
        if ((h > nyf && h != (use2 ? cand2[0] : cand[0])) || h == keep) continue;
        for (int i : kv.second) (use2 ? c->inst[i].strip_rows2 : c->inst[i].strip_rows) = h;
        float ms;
        int rc = trial(use2, &ms);
        if (rc != LBM_OK) return rc;
        if (ms < best) { best = ms; keep = h; }
      }
      for (int i : kv.second) (use2 ? c->inst[i].strip_rows2 : c->inst[i].strip_rows) = keep;
    }
  }
  c->build_tasks();
  int rc = c->upload_tables();
  if (rc != LBM_OK) return rc;
  c->drop_graphs();
  guard.done = true;
  const int i0 = inst >= 0 ? inst : sel.front();
  *chosen = use2 ? c->inst[i0].strip_rows2 : c->inst[i0].strip_rows;
  return LBM_OK;
}

int lbm_get_tuning(const lbm_ctx* c, lbm_tuning* t, int32_t* strip_rows, int32_t* strip_rows2) {
  if (!c || !t) return fail(LBM_E_INVALID, "NULL argument");
  t->two_step = c->step2 ? 1 : 0;
  t->waves = c->waves;
  t->prefetch = c->prefetch ? 1 : 0;
  t->waves2 = c->waves2;
  for (int i = 0; i < c->n(); ++i) {
    if (strip_rows) strip_rows[i] = c->inst[i].strip_rows;
    if (strip_rows2) strip_rows2[i] = c->inst[i].strip_rows2;
  }
  return LBM_OK;
}

int lbm_set_tuning(lbm_ctx* c, const lbm_tuning* t, const int32_t* strip_rows, const int32_t* strip_rows2) {
  if (!c || !t) return fail(LBM_E_INVALID, "NULL argument");
  auto wave_ok = [](int w) {
    for (int k = 0; k < kNumWaveChoices; ++k)
      if (kWaveChoices[k] == w) return true;
    return false;
  };
  if (!wave_ok(t->waves) || !wave_ok(t->waves2)) return fail(LBM_E_INVALID, "wavefronts per block not in {1,2,4,8}");
  if ((t->prefetch != 0 && t->prefetch != 1) || (t->two_step != 0 && t->two_step != 1))
    return fail(LBM_E_INVALID, "prefetch and two_step must be 0 or 1");
  for (int i = 0; i < c->n(); ++i)
    if ((strip_rows && strip_rows[i] < 1) || (strip_rows2 && strip_rows2[i] < 1))
      return fail(LBM_E_INVALID, "instance %d: rows per strip must be >= 1", i);
  c->waves = t->waves;
  c->prefetch = t->prefetch != 0;
  c->waves2 = t->waves2;
  c->step2 = t->two_step != 0;
  for (int i = 0; i < c->n(); ++i) {
    if (strip_rows) c->inst[i].strip_rows = strip_rows[i];
    if (strip_rows2) c->inst[i].strip_rows2 = strip_rows2[i];
  }
  c->build_tasks();
  const int rc = c->upload_tables();
  if (rc != LBM_OK) return rc;
  c->drop_graphs();
  return LBM_OK;
}

}  // extern "C"

namespace {
int adjoint_step(lbm_ctx* c, int32_t inst, bool f32, const void* d_state_n, const void* d_lambda_np1,
                 void* d_lambda_n, double* d_theta_bar, double* d_G_bar) {
  CHECK_INST(c, inst);
  if (!d_state_n || !d_lambda_np1 || !d_lambda_n || !d_theta_bar || !d_G_bar)
    return fail(LBM_E_INVALID, "NULL buffer");
  const Inst& I = c->inst[inst];
  if (!I.p.enable_adjoint)
    return fail(LBM_E_STATE, "instance %d was created without enable_adjoint", inst);
  const int nx = I.p.nx, ny = I.p.ny;
  const size_t pitch = (size_t)I.pitch;
  const size_t field = align256(sizeof(double) * pitch * ny);
  char* base = c->ws + I.off_adj;
  AdjScratch sc;
  sc.rho = (double*)base;
  sc.psi = (double*)(base + field);
  sc.Fbar = (double*)(base + 2 * field);
  sc.gflag = (double*)(base + 4 * field);
  sc.wet = (double*)(base + 4 * field + align256(sizeof(double) * 2 * nx));
  sc.qwall = (double*)(base + 4 * field + align256(sizeof(double) * 2 * nx) + align256(sizeof(double) * 8 * nx));
  sc.part = (double*)(base + 4 * field + align256(sizeof(double) * 2 * nx) + align256(sizeof(double) * 8 * nx) +
                      align256(sizeof(double) * 6 * nx));
  if (2 * nx > 1024 * 256) return fail(LBM_E_UNSUPPORTED, "adjoint: nx too large");
  HIP_TRY(launch_adjoint(c->d_desc(), c->hdesc[inst], inst, sc, f32, d_state_n, d_lambda_np1, d_lambda_n,
                         d_theta_bar, d_G_bar, c->stream));
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_adjoint_step(lbm_ctx* c, int32_t inst, const double* d_state_n, const double* d_lambda_np1,
                     double* d_lambda_n, double* d_theta_bar, double* d_G_bar) {
  return adjoint_step(c, inst, false, d_state_n, d_lambda_np1, d_lambda_n, d_theta_bar, d_G_bar);
}

int lbm_adjoint_step_f32(lbm_ctx* c, int32_t inst, const float* d_state_n, const float* d_lambda_np1,
                         float* d_lambda_n, double* d_theta_bar, double* d_G_bar) {
  return adjoint_step(c, inst, true, d_state_n, d_lambda_np1, d_lambda_n, d_theta_bar, d_G_bar);
}

namespace {
int seed_rho(lbm_ctx* c, int32_t inst, bool f32, const double* d_grad_rho, void* d_lambda, double* d_theta_bar,
             double* d_G_bar) {
  CHECK_INST(c, inst);
  if (!d_grad_rho || !d_lambda || !d_theta_bar || !d_G_bar) return fail(LBM_E_INVALID, "NULL buffer");
  const Inst& I = c->inst[inst];
  HIP_TRY(launch_adjoint_seed_rho(f32, d_grad_rho, d_lambda, d_theta_bar, d_G_bar, I.p.nx, I.p.ny - 2, c->stream));
  return LBM_OK;
}
}  // namespace

int lbm_adjoint_seed_rho(lbm_ctx* c, int32_t inst, const double* d_grad_rho, double* d_lambda, double* d_theta_bar,
                         double* d_G_bar) {
  return seed_rho(c, inst, false, d_grad_rho, d_lambda, d_theta_bar, d_G_bar);
}

int lbm_adjoint_seed_rho_f32(lbm_ctx* c, int32_t inst, const double* d_grad_rho, float* d_lambda,
                             double* d_theta_bar, double* d_G_bar) {
  return seed_rho(c, inst, true, d_grad_rho, d_lambda, d_theta_bar, d_G_bar);
}

}  // extern "C"
