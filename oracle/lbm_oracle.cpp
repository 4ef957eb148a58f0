// Plain reference of the EOS-based single-component pseudo-potential lattice Boltzmann step with the geometric
// contact-angle wall (Hu, Li & Uddin, "Contact Angle Adjustment in Equation of States Based Pseudo-Potential
// Model", arXiv:1501.05430).
//
// TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's CPU-baseline leg load this library;
// the GPU library neither links nor includes it, and it shares no source with the GPU library.
//
// Written for readability, not speed: array-of-structures populations f[(y*nx + x)*9 + i] over all ny rows, one
// loop nest per stage, double precision throughout. Every stage is templated on the scalar type so that the same
// code runs on std::complex<double> for complex-step derivatives (the adjoint's reference).
//
// Readings of the paper that this file takes (each also listed in the design notes):
//  * Lattice: D2Q9 in the moment order of Eq. (4): e0=(0,0), e1..e4=(1,0),(0,1),(-1,0),(0,-1),
//    e5..e8=(1,1),(-1,1),(-1,-1),(1,-1); lattice weights 4/9, 1/9, 1/36, c_s^2 = 1/3.
//  * Collision: Eq. (1)-(6) with the relaxation matrix of Sec. 3.1, diag(0,1,...,1), equal BGK with tau = 1 and
//    Guo forcing; tau is kept general (BGK), with v = (j + F/2)/rho. The last entry of Eq. (6) is the forcing's
//    second moment, v_x F_y + v_y F_x.
//  * MRT (mrt = 1): Eq. (15) in moment space with Lambda of Eq. (2) = diag(0, s_e, s_eps, 1, s_q, 1, s_q, 1/tau,
//    1/tau) and the surface-tension source C of Eq. (16) with Q_3 = 0; the eighth entry of C is
//    -(1/tau)(Q_xx - Q_yy), the factor of the ninth (the two entries are the deviatoric parts of one tensor). Q of
//    Eq. (17) carries the factor G/2: with it the source scales the anisotropic part of the pressure tensor by
//    1 - kappa and keeps its normal part, so the surface tension goes as 1 - kappa as the paper states (as printed,
//    without G/2, it would go as 1 + 2 kappa at G = -1).
//  * Force: Eq. (9) (Kupershtokh hybrid, parameter A) with the weights of Eq. (7), w(1)=1/3, w(2)=1/12, and
//    U = G psi^2 / 2 (Eq. 8). A = 0 is the plain Shan-Chen force of Eq. (7).
//  * psi from Eq. (10) with c = 1: psi = sqrt(2 (p_EOS(rho) - rho/3) / G); p_EOS is Carnahan-Starling, or the
//    piecewise-linear EOS of Eq. (11) with break points from Eq. (12)-(13).
//  * Wall: rows 0 and ny-1 are the ghost layer (index 0 of Sec. 4), rows 1 and ny-2 the boundary nodes (index 1),
//    rows 2 and ny-3 index 2. Ghost rows carry density and psi only. Populations use halfway bounce-back.
//  * Ghost density: Eq. (19) when wet_iters == 0; otherwise the iteration of Eq. (21) with the square root of
//    Eq. (20) restored, stopped after exactly wet_iters iterates (the first line of Eq. (21) is iterate 1).
//  * Martys-Chen walls (wall_mode = 1, the method the paper compares against): the wall rows are solid nodes,
//    S = 1 in Eq. (14), F_s = -G_w psi(x) sum_a w_a S(x + e_a) e_a with one G_w per wall. Solid nodes take no part
//    in the fluid-fluid force or in Q (their psi is 0, as if absent); the paper does not say, and its G_w range
//    (about -0.8 to -2.8 spanning 180 to 0 deg at a density ratio of 10) brackets -psi_v .. -psi_l, which fits
//    walls that attract through F_s alone. No geometric wetting then.
//  * Ghost density is clamped to [0, rho_cap (1 - 1e-6)], rho_cap the largest density with real psi (psi at the
//    clamp is then ~1e-3, not a square root of round-off, so two independent rho_cap solves agree there);
//    psi^2 is clamped at 0 on fluid nodes. Every clamp is counted.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

typedef std::complex<double> cplx;

inline double re(double x) { return x; }
inline double re(const cplx& z) { return z.real(); }

// |x| for the complex-step: x * sign(Re x); the derivative at an exact kink is taken as 0.
inline double absval(double x) { return std::fabs(x); }
inline cplx absval(const cplx& z) { return z.real() < 0.0 ? -z : z; }

inline double sqrt_s(double x) { return std::sqrt(x); }
inline cplx sqrt_s(const cplx& z) {
  if (z.real() == 0.0) return cplx(0.0, 0.0);  // sqrt at 0: value 0, derivative taken as 0
  return std::sqrt(z);
}

// D2Q9 velocities in the moment order of Eq. (4).
const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
const double WLB[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
// Interaction weights of Eq. (7): w(|e|^2 = 1) = 1/3, w(|e|^2 = 2) = 1/12.
const double WF[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};

int wrap(int i, int n) { return ((i % n) + n) % n; }

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------------------------------------------
// Parameters (the oracle's own definition; it is not the GPU library's struct).
// ---------------------------------------------------------------------------------------------------------------
typedef struct {
  int32_t nx, ny;        // ny counts every row, the two ghost rows included when walls are on
  int32_t periodic_y;    // 0: walls at rows 0 and ny-1; 1: periodic in y, every row is fluid
  int32_t wet_iters;     // 0: Eq. (19); k >= 1: k-th iterate of Eq. (21)
  double tau;            // BGK relaxation time
  double G;              // interaction strength (Eq. 7-10); used both as force prefactor and inside psi
  double A;              // hybrid-force parameter of Eq. (9)
  double eos_a, eos_b, eos_R;
  double T;              // absolute temperature of the Carnahan-Starling EOS
  double body_fx, body_fy;  // constant body force F_g of Eq. (7), per unit volume
  int32_t eos_kind;      // 0: Carnahan-Starling (eos_a, eos_b, eos_R, T); 1: piecewise-linear EOS of Eq. (11)
  int32_t pad;
  double pw_theta_v, pw_theta_m, pw_theta_l;  // Eq. (11): slopes of the vapour, unstable and liquid branches
  double pw_rho1, pw_rho2;                    // Eq. (11): break points (from Eq. 12-13, ora_pw_breakpoints)
  int32_t mrt;           // 0: BGK (above); 1: MRT collision of Eq. (15) with the rates below and 1/tau for the stress
  int32_t pad2;
  double s_e, s_eps, s_q;  // Eq. (2): tau_e^-1, tau_xi^-1, tau_q^-1 (MRT only)
  double kappa;            // Eq. (17): surface-tension parameter (MRT only; 0 = no source C)
  int32_t wall_mode;       // 0: geometric wetting (Sec. 4); 1: Martys-Chen fluid-solid force (Eq. 14)
  int32_t pad3;
  double G_w[2];           // Eq. (14): wall interaction strength of the bottom (row 0) and top (row ny-1) wall
} ora_params;

// ---------------------------------------------------------------------------------------------------------------
// Carnahan-Starling equation of state.
// p(rho) = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2,  eta = b rho / 4.
// ---------------------------------------------------------------------------------------------------------------
double ora_cs_pressure(double a, double b, double R, double T, double rho) {
  double eta = b * rho / 4.0;
  double num = 1.0 + eta + eta * eta - eta * eta * eta;
  double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
  return rho * R * T * num / den - a * rho * rho;
}

// dp/drho, written from d(eta Z)/d eta = (1 + 4 eta + 4 eta^2 - 4 eta^3 + eta^4) / (1 - eta)^4.
double ora_cs_dpdrho(double a, double b, double R, double T, double rho) {
  double eta = b * rho / 4.0;
  double om = 1.0 - eta;
  double n = 1.0 + 4.0 * eta + 4.0 * eta * eta - 4.0 * eta * eta * eta + eta * eta * eta * eta;
  return R * T * n / (om * om * om * om) - 2.0 * a * rho;
}

// d2p/drho2, written from d^2(eta Z)/d eta^2 = (8 + 20 eta - 4 eta^2) / (1 - eta)^5.
double ora_cs_d2pdrho2(double a, double b, double R, double T, double rho) {
  double eta = b * rho / 4.0;
  double om = 1.0 - eta;
  double n = 8.0 + 20.0 * eta - 4.0 * eta * eta;
  return R * T * (b / 4.0) * n / (om * om * om * om * om) - 2.0 * a;
}

// Chemical potential (up to a T-dependent constant): mu = R T [ln rho + (8 eta - 9 eta^2 + 3 eta^3)/(1-eta)^3]
// - 2 a rho. It satisfies d mu / d rho = (dp/drho) / rho, the Gibbs-Duhem relation at fixed T.
double ora_cs_mu(double a, double b, double R, double T, double rho) {
  double eta = b * rho / 4.0;
  double om = 1.0 - eta;
  return R * T * (std::log(rho) + (8.0 * eta - 9.0 * eta * eta + 3.0 * eta * eta * eta) / (om * om * om)) -
         2.0 * a * rho;
}

// Critical point: dp/drho = d2p/drho2 = 0. p is linear in T, p = T P1(rho) - a rho^2, so T_c = 2 a rho / P1'(rho)
// = 2 a / P1''(rho) at rho_c; rho_c is the root of g(rho) = rho P1''(rho) - P1'(rho) on (0, 4/b), by bisection.
int ora_cs_critical(double a, double b, double R, double* rho_c, double* T_c, double* p_c) {
  if (!(a > 0) || !(b > 0) || !(R > 0)) return 1;
  auto P1d = [&](double rho) { return ora_cs_dpdrho(0.0, b, R, 1.0, rho); };
  auto P1dd = [&](double rho) { return ora_cs_d2pdrho2(0.0, b, R, 1.0, rho); };
  auto g = [&](double rho) { return rho * P1dd(rho) - P1d(rho); };
  double lo = 1e-9 * 4.0 / b, hi = 0.5 * 4.0 / b;  // eta in (1e-9, 0.5)
  double glo = g(lo);
  if (glo * g(hi) > 0) return 2;
  for (int it = 0; it < 300; ++it) {
    double mid = 0.5 * (lo + hi);
    double gm = g(mid);
    if ((gm < 0) == (glo < 0)) { lo = mid; glo = gm; } else { hi = mid; }
  }
  double rc = 0.5 * (lo + hi);
  double tc = 2.0 * a / P1dd(rc);
  *rho_c = rc;
  *T_c = tc;
  *p_c = ora_cs_pressure(a, b, R, tc, rc);
  return 0;
}

// Spinodal densities (dp/drho = 0) below T_c: rho_s1 < rho_c < rho_s2, by bisection on each side of rho_c.
static int cs_spinodals(double a, double b, double R, double T, double rc, double* s1, double* s2) {
  auto d = [&](double rho) { return ora_cs_dpdrho(a, b, R, T, rho); };
  if (!(d(rc) < 0)) return 1;
  double lo = 1e-300, hi = rc;  // d > 0 at lo, < 0 at hi
  for (int it = 0; it < 2000 && hi - lo > 0; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (d(mid) > 0) lo = mid; else hi = mid;
  }
  *s1 = 0.5 * (lo + hi);
  lo = rc; hi = 0.999999 * 4.0 / b;  // d < 0 at lo, > 0 at hi
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (d(mid) < 0) lo = mid; else hi = mid;
  }
  *s2 = 0.5 * (lo + hi);
  return 0;
}

// The density on the branch [lo, hi] (p monotone there) where p(rho) = P, by bisection.
static double cs_invert(double a, double b, double R, double T, double P, double lo, double hi) {
  double plo = ora_cs_pressure(a, b, R, T, lo);
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    double pm = ora_cs_pressure(a, b, R, T, mid);
    if ((pm < P) == (plo < P)) { lo = mid; plo = pm; } else { hi = mid; }
  }
  return 0.5 * (lo + hi);
}

// Maxwell coexistence (equal pressure and equal chemical potential), the Carnahan-Starling counterpart of the
// two-phase equilibrium conditions written for the piecewise EOS in Eq. (12)-(13). Nested bisection: for a
// pressure level P between the spinodal pressures, rho_v(P) and rho_l(P) lie on the outer branches; bisect P on
// mu(rho_l) - mu(rho_v) = 0.
int ora_cs_maxwell(double a, double b, double R, double T, double* rho_v, double* rho_l) {
  double rc, tc, pc;
  if (ora_cs_critical(a, b, R, &rc, &tc, &pc)) return 1;
  if (!(T > 0) || !(T < tc)) return 2;
  double s1, s2;
  if (cs_spinodals(a, b, R, T, rc, &s1, &s2)) return 3;
  double p_hi = ora_cs_pressure(a, b, R, T, s1);
  double p_lo = ora_cs_pressure(a, b, R, T, s2);
  if (p_lo < 0) p_lo = 0;
  double rho_max = 0.999999 * 4.0 / b;
  auto dmu = [&](double P, double* rv, double* rl) {
    *rv = cs_invert(a, b, R, T, P, 1e-300, s1);
    *rl = cs_invert(a, b, R, T, P, s2, rho_max);
    return ora_cs_mu(a, b, R, T, *rl) - ora_cs_mu(a, b, R, T, *rv);
  };
  double rv, rl;
  double lo = p_lo, hi = p_hi;
  if (lo == 0) lo = 1e-300;
  double flo = dmu(lo, &rv, &rl);
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    double fm = dmu(mid, &rv, &rl);
    if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
  }
  dmu(0.5 * (lo + hi), &rv, &rl);
  *rho_v = rv;
  *rho_l = rl;
  return 0;
}

// Largest density with real psi: psi^2 = 2 (p - rho/3) / G with G < 0 needs p <= rho/3. Returns the smallest
// root of p(rho) - rho/3 = 0 above the liquid spinodal (or above rho_c when there is none), by bisection.
double ora_cs_rho_cap(double a, double b, double R, double T, double G) {
  (void)G;
  double rc, tc, pc;
  ora_cs_critical(a, b, R, &rc, &tc, &pc);
  auto h = [&](double rho) { return ora_cs_pressure(a, b, R, T, rho) - rho / 3.0; };
  // h < 0 at rc (sub-critical pressures are small), h > 0 near rho = 4/b where p diverges. Step outwards until
  // the sign changes, then bisect.
  double lo = rc, hi = rc;
  const double top = 0.999999 * 4.0 / b;
  while (h(hi) < 0 && hi < top) hi = std::fmin(top, hi + 1e-3);
  lo = hi - 1e-3 < rc ? rc : hi - 1e-3;
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (h(mid) < 0) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------------------------------------------
// Piecewise-linear EOS of Eq. (11) (the self-tuning EOS the paper adopts): slope theta_v up to rho_1, theta_m
// between rho_1 and rho_2, theta_l above rho_2, continuous, p(0) = 0.
// ---------------------------------------------------------------------------------------------------------------
double ora_pw_pressure(double tv, double tm, double tl, double r1, double r2, double rho) {
  if (rho <= r1) return rho * tv;
  if (rho <= r2) return r1 * tv + (rho - r1) * tm;
  return r1 * tv + (r2 - r1) * tm + (rho - r2) * tl;
}

// Break points rho_1 < rho_2 for given coexistence densities rho_v < rho_l and slopes: Eq. (12) (equal pressure,
// the integral of dp) and Eq. (13) (equal chemical potential, the integral of dp / rho) written out. Eq. (12) gives
// rho_2 as a linear function of rho_1; Eq. (13) is then one equation in rho_1, solved by bisection over the rho_1
// for which rho_v <= rho_1 < rho_2 <= rho_l. Returns 0 on success.
int ora_pw_breakpoints(double tv, double tm, double tl, double rv, double rl, double* r1, double* r2) {
  if (!(rv > 0 && rl > rv && tv > 0 && tl > 0 && tm < 0)) return 1;
  auto rho2_of = [&](double x) { return (rv * tv - x * tv + x * tm - rl * tl) / (tm - tl); };  // Eq. (12)
  auto eq13 = [&](double x) {
    const double y = rho2_of(x);
    return std::log(x / rv) * tv + std::log(y / x) * tm + std::log(rl / y) * tl;
  };
  // feasible rho_1: the segment order of Eq. (11), rho_v <= rho_1 < rho_2(rho_1) <= rho_l. rho_2(rho_1) increases
  // with rho_1 and reaches rho_l at rho_1 = (rv tv - rl tm) / (tv - tm); rho_2 - rho_1 is proportional to
  // rho_1 (tv - tl) + rl tl - rv tv, which vanishes at (rl tl - rv tv) / (tl - tv).
  double lo = rv, hi = (rv * tv - rl * tm) / (tv - tm);
  if (tv > tl) lo = std::max(lo, (rl * tl - rv * tv) / (tl - tv));
  if (tv < tl) hi = std::min(hi, (rl * tl - rv * tv) / (tl - tv));
  if (!(lo < hi)) return 2;
  double flo = eq13(lo), fhi = eq13(hi);
  if (!std::isfinite(flo) || !std::isfinite(fhi) || (flo < 0) == (fhi < 0)) return 2;
  for (int it = 0; it < 300; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    const double fm = eq13(mid);
    if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
  }
  *r1 = 0.5 * (lo + hi);
  *r2 = rho2_of(*r1);
  return 0;
}

// Largest density with real psi for the piecewise EOS: the root of p(rho) = rho/3 on the liquid branch when its
// slope exceeds 1/3, else unbounded.
double ora_pw_rho_cap(double tv, double tm, double tl, double r1, double r2) {
  const double h2 = ora_pw_pressure(tv, tm, tl, r1, r2, r2) - r2 / 3.0;
  if (tl > 1.0 / 3.0) return r2 - h2 / (tl - 1.0 / 3.0);
  return 1e300;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------------------------
// The time step (templated on the scalar type).
// ---------------------------------------------------------------------------------------------------------------
namespace {

// Orthogonal D2Q9 moment matrix in the moment order of Eq. (4): rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy.
const int MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

// Q of Eq. (17) at node (x, y) from a psi field [ny][nx] (neighbours wrap in x, and in y when periodic), with the
// factor G/2 (see the file header): Q = kappa (G/2) [(1 - A) psi(x) sum_a w_a (psi(x+e_a) - psi(x)) e_a e_a
//                                                 + (A/2) sum_a w_a (psi(x+e_a)^2 - psi(x)^2) e_a e_a].
template <class S>
void qtensor_at(const ora_params& p, const S& G, const S* psi, int nx, int ny, int x, int y, S* qxx, S* qyy,
                S* qxy) {
  S pc = psi[(size_t)y * nx + x];
  S a_xx = 0.0, a_yy = 0.0, a_xy = 0.0, b_xx = 0.0, b_yy = 0.0, b_xy = 0.0;
  for (int a = 1; a < 9; ++a) {
    int xn = wrap(x + EX[a], nx);
    int yn = p.periodic_y ? wrap(y + EY[a], ny) : y + EY[a];
    S pn = psi[(size_t)yn * nx + xn];
    S d1 = WF[a] * (pn - pc);
    S d2 = WF[a] * (pn * pn - pc * pc);
    a_xx += d1 * (double)(EX[a] * EX[a]);
    a_yy += d1 * (double)(EY[a] * EY[a]);
    a_xy += d1 * (double)(EX[a] * EY[a]);
    b_xx += d2 * (double)(EX[a] * EX[a]);
    b_yy += d2 * (double)(EY[a] * EY[a]);
    b_xy += d2 * (double)(EX[a] * EY[a]);
  }
  S k = p.kappa * G / 2.0;
  *qxx = k * ((1.0 - p.A) * pc * a_xx + p.A / 2.0 * b_xx);
  *qyy = k * ((1.0 - p.A) * pc * a_yy + p.A / 2.0 * b_yy);
  *qxy = k * ((1.0 - p.A) * pc * a_xy + p.A / 2.0 * b_xy);
}

struct Counters {
  int64_t ghost_clamps = 0;
  int64_t psi_clamps = 0;
};

template <class S>
S cs_pressure_t(const ora_params& p, const S& rho) {
  if (p.eos_kind == 1) {  // Eq. (11); the branch follows the real part
    const double r = re(rho);
    if (r <= p.pw_rho1) return rho * p.pw_theta_v;
    if (r <= p.pw_rho2) return p.pw_rho1 * p.pw_theta_v + (rho - p.pw_rho1) * p.pw_theta_m;
    return p.pw_rho1 * p.pw_theta_v + (p.pw_rho2 - p.pw_rho1) * p.pw_theta_m + (rho - p.pw_rho2) * p.pw_theta_l;
  }
  S eta = p.eos_b * rho / 4.0;
  S num = 1.0 + eta + eta * eta - eta * eta * eta;
  S om = 1.0 - eta;
  return rho * p.eos_R * p.T * num / (om * om * om) - p.eos_a * rho * rho;
}

// Eq. (10) with c = 1: G psi^2 / 2 = p_EOS - rho/3.
template <class S>
S psi_of_rho(const ora_params& p, const S& G_psi, const S& rho, Counters* cnt) {
  S arg = 2.0 * (cs_pressure_t(p, rho) - rho / 3.0) / G_psi;
  if (re(arg) < 0.0) {
    if (cnt) cnt->psi_clamps++;
    return S(0.0);
  }
  return sqrt_s(arg);
}

// Ghost density of Sec. 4: rho_{i,0} from rho_{i-1,1}, rho_{i+1,1}, rho_{i,1}, rho_{i,2} and theta.
//  wet_iters == 0:  Eq. (19), rho_0 = rho_2 + tan(pi/2 - theta) |rho_{i+1,1} - rho_{i-1,1}|.
//  wet_iters >= 1:  Eq. (21) with the square root of Eq. (20): the first iterate uses 2 (rho_2 - rho_1) in place
//                   of (rho_2 - rho_0); each later iterate uses the previous rho_0.
template <class S>
S ghost_density(const S& r_im1_1, const S& r_ip1_1, const S& r_i_1, const S& r_i_2, const S& theta, int iters) {
  S T = r_ip1_1 - r_im1_1;
  if (iters == 0) {
    return r_i_2 + std::tan(M_PI / 2 - theta) * absval(T);
  }
  S s = std::sin(M_PI / 2 - theta);
  S r0 = r_i_2 + s * sqrt_s(T * T + 4.0 * (r_i_2 - r_i_1) * (r_i_2 - r_i_1));
  for (int k = 2; k <= iters; ++k) {
    r0 = r_i_2 + s * sqrt_s(T * T + (r_i_2 - r0) * (r_i_2 - r0));
  }
  return r0;
}

// Specialisation helpers: std::tan/std::sin are overloaded for both double and complex.

template <class S>
struct Oracle {
  const ora_params& p;
  S G_f, G_psi;        // force prefactor and the G inside the psi inversion (equal in the model; split for gradients)
  double rho_cap;
  Counters cnt;
  int nx, ny;
  std::vector<S> rho, jx, jy, psi;

  Oracle(const ora_params& pp, S gf, S gpsi) : p(pp), G_f(gf), G_psi(gpsi), nx(pp.nx), ny(pp.ny) {
    rho_cap = p.eos_kind == 1 ? ora_pw_rho_cap(p.pw_theta_v, p.pw_theta_m, p.pw_theta_l, p.pw_rho1, p.pw_rho2)
                              : ora_cs_rho_cap(p.eos_a, p.eos_b, p.eos_R, p.T, re(G_psi));
    rho.assign((size_t)nx * ny, S(0.0));
    jx.assign((size_t)nx * ny, S(0.0));
    jy.assign((size_t)nx * ny, S(0.0));
    psi.assign((size_t)nx * ny, S(0.0));
  }

  bool fluid_row(int y) const { return p.periodic_y || (y >= 1 && y <= ny - 2); }

  // Step 1-3 of a time step: moments of the streamed populations, psi on fluid rows, then the ghost rows.
  void moments(const S* f, const S* th_bot, const S* th_top) {
    int64_t psi_clamps = 0;
#pragma omp parallel for schedule(static) reduction(+ : psi_clamps)
    for (int y = 0; y < ny; ++y) {
      if (!fluid_row(y)) continue;
      Counters local;
      for (int x = 0; x < nx; ++x) {
        const S* fn = f + ((size_t)y * nx + x) * 9;
        S r = 0.0, mx = 0.0, my = 0.0;
        for (int i = 0; i < 9; ++i) {
          r += fn[i];
          mx += fn[i] * (double)EX[i];
          my += fn[i] * (double)EY[i];
        }
        size_t k = (size_t)y * nx + x;
        rho[k] = r;
        jx[k] = mx;
        jy[k] = my;
        psi[k] = psi_of_rho(p, G_psi, r, &local);
      }
      psi_clamps += local.psi_clamps;
    }
    cnt.psi_clamps += psi_clamps;
    if (p.periodic_y) return;
    if (p.wall_mode == 1) {  // solid wall rows: absent from the fluid-fluid force
      for (int x = 0; x < nx; ++x) {
        rho[x] = psi[x] = S(0.0);
        rho[(size_t)(ny - 1) * nx + x] = psi[(size_t)(ny - 1) * nx + x] = S(0.0);
      }
      return;
    }
    // Ghost rows: bottom uses rows 1 (index 1) and 2 (index 2); top mirrors with rows ny-2 and ny-3.
    for (int wall = 0; wall < 2; ++wall) {
      int g = wall == 0 ? 0 : ny - 1;
      int r1 = wall == 0 ? 1 : ny - 2;
      int r2 = wall == 0 ? 2 : ny - 3;
      const S* th = wall == 0 ? th_bot : th_top;
      for (int x = 0; x < nx; ++x) {
        S r0 = ghost_density(rho[(size_t)r1 * nx + wrap(x - 1, nx)], rho[(size_t)r1 * nx + wrap(x + 1, nx)],
                             rho[(size_t)r1 * nx + x], rho[(size_t)r2 * nx + x], th[x], p.wet_iters);
        double hi = rho_cap * (1.0 - 1e-6);
        if (re(r0) < 0.0) { r0 = S(0.0); cnt.ghost_clamps++; }
        else if (re(r0) > hi) { r0 = S(hi); cnt.ghost_clamps++; }
        rho[(size_t)g * nx + x] = r0;
        psi[(size_t)g * nx + x] = psi_of_rho(p, G_psi, r0, nullptr);
      }
    }
  }

  // Step 4: the interaction force of Eq. (9) at fluid node (x, y); neighbours in ghost rows use the ghost psi.
  void force(int x, int y, S* Fx, S* Fy) const {
    S pc = psi[(size_t)y * nx + x];
    S su_x = 0.0, su_y = 0.0, sp_x = 0.0, sp_y = 0.0;
    for (int a = 1; a < 9; ++a) {
      int xn = wrap(x + EX[a], nx);
      int yn = p.periodic_y ? wrap(y + EY[a], ny) : y + EY[a];
      S pn = psi[(size_t)yn * nx + xn];
      S U = G_f * pn * pn / 2.0;  // potential of Eq. (8)
      su_x += WF[a] * U * (double)EX[a];
      su_y += WF[a] * U * (double)EY[a];
      sp_x += WF[a] * pn * (double)EX[a];
      sp_y += WF[a] * pn * (double)EY[a];
    }
    *Fx = -p.A * su_x - (1.0 - p.A) * G_f * pc * sp_x;
    *Fy = -p.A * su_y - (1.0 - p.A) * G_f * pc * sp_y;
    if (p.wall_mode == 1 && !p.periodic_y) {
      // Eq. (14): F_s = -G_w psi(x) sum_a w_a S(x + e_a) e_a over the solid (wall-row) neighbours
      for (int a = 1; a < 9; ++a) {
        int yn = y + EY[a];
        if (yn != 0 && yn != ny - 1) continue;
        double gw = yn == 0 ? p.G_w[0] : p.G_w[1];
        *Fx -= gw * pc * (WF[a] * (double)EX[a]);
        *Fy -= gw * pc * (WF[a] * (double)EY[a]);
      }
    }
  }

  // Steps 5-6: collision with forcing at every fluid node, then streaming (halfway bounce-back at the walls).
  void collide_stream(const S* f, S* fout) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
      if (!fluid_row(y)) continue;
      for (int x = 0; x < nx; ++x) {
        size_t k = (size_t)y * nx + x;
        S Fx, Fy;
        force(x, y, &Fx, &Fy);
        Fx += p.body_fx;
        Fy += p.body_fy;
        S fstar[9];
        if (p.mrt) {
          S qxx, qyy, qxy;
          qtensor_at(p, G_f, psi.data(), nx, ny, x, y, &qxx, &qyy, &qxy);
          collide_mrt(f + k * 9, rho[k], jx[k], jy[k], Fx, Fy, qxx, qyy, qxy, fstar);
        } else {
          collide_node(f + k * 9, rho[k], jx[k], jy[k], Fx, Fy, fstar);
        }
        for (int i = 0; i < 9; ++i) {
          int xd = wrap(x + EX[i], nx);
          int yd = y + EY[i];
          if (p.periodic_y) yd = wrap(yd, ny);
          if (!fluid_row(yd)) {
            fout[k * 9 + OPP[i]] = fstar[i];  // halfway bounce-back
          } else {
            fout[((size_t)yd * nx + xd) * 9 + i] = fstar[i];
          }
        }
      }
    }
  }

  // BGK collision with Guo forcing: v = (j + F/2)/rho; f* = f - (f - f_eq(rho, v))/tau
  //   + (1 - 1/(2 tau)) w_i [3 (e_i - v) + 9 (e_i . v) e_i] . F.
  void collide_node(const S* fn, const S& r, const S& mx, const S& my, const S& Fx, const S& Fy, S* fstar) const {
    S vx = (mx + Fx / 2.0) / r;
    S vy = (my + Fy / 2.0) / r;
    S vv = vx * vx + vy * vy;
    for (int i = 0; i < 9; ++i) {
      S ev = (double)EX[i] * vx + (double)EY[i] * vy;
      S feq = WLB[i] * r * (1.0 + 3.0 * ev + 4.5 * ev * ev - 1.5 * vv);
      S gx = 3.0 * ((double)EX[i] - vx) + 9.0 * ev * (double)EX[i];
      S gy = 3.0 * ((double)EY[i] - vy) + 9.0 * ev * (double)EY[i];
      S Fi = (1.0 - 1.0 / (2.0 * p.tau)) * WLB[i] * (gx * Fx + gy * Fy);
      fstar[i] = fn[i] - (fn[i] - feq) / p.tau + Fi;
    }
  }

  // MRT collision of Eq. (15): m = M f; m* = m - Lambda (m - m_eq) + (I - Lambda/2) S + C; f* = M^-1 m*, with
  // m_eq of Eq. (4) at v = (j + F/2)/rho, S of Eq. (6), C of Eq. (16) and M^-1 = M^T diag(1 / |row|^2).
  void collide_mrt(const S* fn, const S& r, const S& mx, const S& my, const S& Fx, const S& Fy, const S& qxx,
                   const S& qyy, const S& qxy, S* fstar) const {
    S m[9];
    for (int k = 0; k < 9; ++k) {
      m[k] = 0.0;
      for (int i = 0; i < 9; ++i) m[k] += (double)MM[k][i] * fn[i];
    }
    S vx = (mx + Fx / 2.0) / r;
    S vy = (my + Fy / 2.0) / r;
    S vv = vx * vx + vy * vy;
    S meq[9] = {r, r * (-2.0 + 3.0 * vv), r * (1.0 - 3.0 * vv), r * vx, -r * vx, r * vy, -r * vy,
                r * (vx * vx - vy * vy), r * vx * vy};
    S vf = vx * Fx + vy * Fy;
    S src[9] = {S(0.0), 6.0 * vf, -6.0 * vf, Fx, -Fx, Fy, -Fy, 2.0 * (vx * Fx - vy * Fy), vx * Fy + vy * Fx};
    const double s_nu = 1.0 / p.tau;
    const double lam[9] = {0.0, p.s_e, p.s_eps, 1.0, p.s_q, 1.0, p.s_q, s_nu, s_nu};
    S C[9] = {S(0.0), 1.5 * p.s_e * (qxx + qyy), S(0.0), S(0.0), S(0.0), S(0.0), S(0.0), -s_nu * (qxx - qyy),
              -s_nu * qxy};
    S ms[9];
    for (int k = 0; k < 9; ++k) ms[k] = m[k] - lam[k] * (m[k] - meq[k]) + (1.0 - lam[k] / 2.0) * src[k] + C[k];
    for (int i = 0; i < 9; ++i) {
      S v = 0.0;
      for (int k = 0; k < 9; ++k) {
        int nk = 0;
        for (int j = 0; j < 9; ++j) nk += MM[k][j] * MM[k][j];
        v += (double)MM[k][i] * ms[k] / (double)nk;
      }
      fstar[i] = v;
    }
  }
};

template <class S>
void run_steps(const ora_params& p, S G_f, S G_psi, S* f, int64_t nsteps, const S* th_bot, const S* th_top,
               int64_t* counters) {
  Oracle<S> o(p, G_f, G_psi);
  std::vector<S> tmp((size_t)p.nx * p.ny * 9, S(0.0));
  for (int64_t n = 0; n < nsteps; ++n) {
    o.moments(f, th_bot, th_top);
    o.collide_stream(f, tmp.data());
    std::memcpy((void*)f, (const void*)tmp.data(), sizeof(S) * tmp.size());
  }
  if (counters) {
    counters[0] += o.cnt.ghost_clamps;
    counters[1] += o.cnt.psi_clamps;
  }
}

bool params_ok(const ora_params* p) {
  if (!p || p->nx < 1 || p->ny < (p->periodic_y ? 1 : 4) || p->wet_iters < 0) return false;
  if (!(p->tau > 0.5) || !(p->G < 0)) return false;
  if (p->mrt && !(p->s_e > 0 && p->s_e < 2 && p->s_eps > 0 && p->s_eps < 2 && p->s_q > 0 && p->s_q < 2)) return false;
  if (!p->mrt && p->kappa != 0.0) return false;
  if (p->wall_mode != 0 && p->wall_mode != 1) return false;
  if (p->eos_kind == 1)
    return p->pw_theta_v > 0 && p->pw_theta_m < 0 && p->pw_theta_l > 0 && p->pw_rho1 > 0 && p->pw_rho2 > p->pw_rho1;
  return p->eos_kind == 0 && p->T > 0;
}

}  // namespace

extern "C" {

// Advance the populations f (layout [ny][nx][9], ghost rows ignored) by nsteps time steps in place.
// theta_bot/theta_top: per-column contact angles in radians ([nx] each; unused when periodic_y).
// counters (may be NULL): [0] += ghost-density clamps, [1] += fluid psi clamps.
int ora_run(const ora_params* p, double* f, int64_t nsteps, const double* theta_bot, const double* theta_top,
            int64_t* counters) {
  if (!params_ok(p)) return 1;
  run_steps<double>(*p, p->G, p->G, f, nsteps, theta_bot, theta_top, counters);
  return 0;
}

// Complex-step variant: every input is complex (interleaved re, im), with G split into the force prefactor G_f
// and the G inside the psi inversion G_psi. Used for directional derivatives of the step.
int ora_run_cplx(const ora_params* p, double* f_ri, int64_t nsteps, const double* theta_bot_ri,
                 const double* theta_top_ri, const double* G_f_ri, const double* G_psi_ri) {
  if (!params_ok(p)) return 1;
  cplx* f = reinterpret_cast<cplx*>(f_ri);
  cplx gf(G_f_ri[0], G_f_ri[1]), gp(G_psi_ri[0], G_psi_ri[1]);
  run_steps<cplx>(*p, gf, gp, f, nsteps, reinterpret_cast<const cplx*>(theta_bot_ri),
                  reinterpret_cast<const cplx*>(theta_top_ri), nullptr);
  return 0;
}

// Density field of the populations, with the ghost rows filled by the wetting rule ([ny][nx]), and psi.
int ora_density(const ora_params* p, const double* f, const double* theta_bot, const double* theta_top,
                double* rho_out, double* psi_out) {
  if (!params_ok(p)) return 1;
  Oracle<double> o(*p, p->G, p->G);
  o.moments(f, theta_bot, theta_top);
  std::memcpy(rho_out, o.rho.data(), sizeof(double) * o.rho.size());
  if (psi_out) std::memcpy(psi_out, o.psi.data(), sizeof(double) * o.psi.size());
  return 0;
}

// The interaction force (Eq. 9, without the body force) at every fluid node of the current populations,
// [ny][nx] each; ghost rows are left at zero.
int ora_force(const ora_params* p, const double* f, const double* theta_bot, const double* theta_top, double* Fx,
              double* Fy) {
  if (!params_ok(p)) return 1;
  Oracle<double> o(*p, p->G, p->G);
  o.moments(f, theta_bot, theta_top);
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      Fx[k] = 0.0;
      Fy[k] = 0.0;
      if (o.fluid_row(y)) o.force(x, y, &Fx[k], &Fy[k]);
    }
  }
  return 0;
}

// The interaction force of Eq. (9) (Martys-Chen wall term of Eq. 14 included when wall_mode = 1, no body force) on
// a given psi field [ny][nx] (every row read as given, the ghost rows too), at every fluid node; other rows are
// left at zero. It evaluates Oracle::force, the step's own force, on psi values chosen by the caller.
int ora_force_psi(const ora_params* p, const double* psi, double* Fx, double* Fy) {
  if (!params_ok(p)) return 1;
  Oracle<double> o(*p, p->G, p->G);
  std::memcpy(o.psi.data(), psi, sizeof(double) * o.psi.size());
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      size_t k = (size_t)y * p->nx + x;
      Fx[k] = 0.0;
      Fy[k] = 0.0;
      if (o.fluid_row(y)) o.force(x, y, &Fx[k], &Fy[k]);
    }
  }
  return 0;
}

// One BGK-Guo collision of a single node (no streaming); f_in[9] -> f_out[9], given the total force.
int ora_collide_node(const ora_params* p, const double* f_in, double Fx, double Fy, double* f_out) {
  if (!params_ok(p)) return 1;
  Oracle<double> o(*p, p->G, p->G);
  double r = 0, mx = 0, my = 0;
  for (int i = 0; i < 9; ++i) {
    r += f_in[i];
    mx += f_in[i] * EX[i];
    my += f_in[i] * EY[i];
  }
  o.collide_node(f_in, r, mx, my, Fx, Fy, f_out);
  return 0;
}

// One MRT collision of a single node (Eq. 15) given the total force and the tensor Q of Eq. (17).
int ora_collide_mrt_node(const ora_params* p, const double* f_in, double Fx, double Fy, const double* Q,
                         double* f_out) {
  if (!params_ok(p) || !p->mrt) return 1;
  Oracle<double> o(*p, p->G, p->G);
  double r = 0, mx = 0, my = 0;
  for (int i = 0; i < 9; ++i) {
    r += f_in[i];
    mx += f_in[i] * EX[i];
    my += f_in[i] * EY[i];
  }
  o.collide_mrt(f_in, r, mx, my, Fx, Fy, Q[0], Q[1], Q[2], f_out);
  return 0;
}

// Q of Eq. (17) (with G/2, see the header) at every node of a psi field [ny][nx]: q[3][ny][nx] = Q_xx, Q_yy, Q_xy.
// Rows 0 and ny-1 are skipped unless periodic_y (they are ghost rows).
int ora_qtensor(const ora_params* p, const double* psi, double* q) {
  if (!params_ok(p)) return 1;
  const int nx = p->nx, ny = p->ny;
  const size_t n = (size_t)nx * ny;
  for (int y = 0; y < ny; ++y) {
    if (!p->periodic_y && (y == 0 || y == ny - 1)) continue;
    for (int x = 0; x < nx; ++x) {
      const size_t k = (size_t)y * nx + x;
      qtensor_at<double>(*p, p->G, psi, nx, ny, x, y, &q[k], &q[n + k], &q[2 * n + k]);
    }
  }
  return 0;
}

// Ghost density of one wall node (Eq. 19 / Eq. 21), unclamped.
double ora_ghost_density(double r_im1_1, double r_ip1_1, double r_i_1, double r_i_2, double theta, int32_t iters) {
  return ghost_density<double>(r_im1_1, r_ip1_1, r_i_1, r_i_2, theta, iters);
}

double ora_psi(const ora_params* p, double rho) { return psi_of_rho<double>(*p, p->G, rho, nullptr); }

// Initial state: density profile rho = rho_v + (rho_l - rho_v) (1 - tanh(2 (r - R)/W)) / 2 around each droplet
// (the largest value over droplets), node (x, y) at coordinates (x, y); x distances use the nearest periodic
// image, dx - nx floor(dx/nx + 1/2) (and y likewise when periodic). Populations at rest: f_i = w_i rho.
int ora_init_droplets(const ora_params* p, double* f, int32_t n, const double* xc, const double* yc,
                      const double* R, double W, double rho_l, double rho_v) {
  if (!params_ok(p) || n < 0 || !(W > 0)) return 1;
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      double r = rho_v;
      for (int d = 0; d < n; ++d) {
        double dx = x - xc[d];
        dx -= p->nx * std::floor(dx / p->nx + 0.5);
        double dy = y - yc[d];
        if (p->periodic_y) dy -= p->ny * std::floor(dy / p->ny + 0.5);
        double dist = std::sqrt(dx * dx + dy * dy);
        double v = rho_v + (rho_l - rho_v) * 0.5 * (1.0 - std::tanh(2.0 * (dist - R[d]) / W));
        if (v > r) r = v;
      }
      bool fluid = p->periodic_y || (y >= 1 && y <= p->ny - 2);
      for (int i = 0; i < 9; ++i) f[((size_t)y * p->nx + x) * 9 + i] = fluid ? WLB[i] * r : 0.0;
    }
  }
  return 0;
}

// Total mass over fluid nodes.
double ora_mass(const ora_params* p, const double* f) {
  double m = 0.0;
  for (int y = 0; y < p->ny; ++y) {
    if (!(p->periodic_y || (y >= 1 && y <= p->ny - 2))) continue;
    for (int x = 0; x < p->nx; ++x)
      for (int i = 0; i < 9; ++i) m += f[((size_t)y * p->nx + x) * 9 + i];
  }
  return m;
}

}  // extern "C"

#include <omp.h>
extern "C" int32_t ora_num_threads(void) { return (int32_t)omp_get_max_threads(); }
