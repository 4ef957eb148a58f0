// Internal structures shared by the host part (lbm_api.cpp) and the kernels (lbm_kernels.hip) of liblbm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Per-instance constants read by every kernel (one table in device memory, indexed by instance).
struct InstDesc {
  void* f[2];               // population buffers, SoA [9][ny-2][pitch] of the storage type
  const double* cos_th;     // [2][nx]: bottom row then top row
  const double* cot_th;     // [2][nx]
  const double* sin_th;     // [2][nx]
  double* ghost;            // [2][nx] ghost densities written by the wetting kernel (inspection only)
  int32_t nx, ny, pitch, wet_iters;
  int64_t plane;            // (ny-2) * pitch elements per population
  int32_t cur;              // buffer holding the state before a launch with flip s = 0
  int32_t periodic_y;       // 1: fluid rows 1..ny-2 wrap around, no walls (LBM_PERIODIC_Y)
  double RT;                // R * T
  double eos_a, eos_b4;     // a, b/4
  double two_over_Gpsi;     // 2 / G (G inside psi, Eq. 10)
  double G_f, A;            // force prefactor and hybrid parameter (Eq. 9)
  double inv_tau, force_pref;  // 1/tau and 1 - 1/(2 tau)
  double body_fx, body_fy;
  double rho0;              // storage shift (0 unless shifted FP32)
  double rho_fp64_below;    // FP32 modes: FP64 EOS below this density
  double rho_cap_hi;        // ghost density upper clamp, rho_cap (1 - 1e-6)
  int32_t eos_kind, pad1;   // lbm_eos: 0 Carnahan-Starling (RT, eos_a, eos_b4), 1 piecewise linear (pw_*)
  double pw_t[3];           // Eq. 11 slopes theta_v, theta_m, theta_l
  double pw_r1, pw_r2;      // break points rho_1 < rho_2 (Eq. 12-13)
  double pw_p1, pw_p2;      // p(rho_1) = rho_1 theta_v and p(rho_2) = p(rho_1) + (rho_2 - rho_1) theta_m
  int32_t mrt, pad2;        // 1: MRT collision (Eq. 15) with the rates below, else BGK
  double s_e, s_eps, s_q;   // Eq. 2 relaxation rates (the stress relaxes at inv_tau)
  double kq;                // kappa G / 2 of Eq. 17 (0: no surface-tension source)
  int32_t wall_mc, pad3;    // 1: Martys-Chen walls (Eq. 14): solid rows, psi = 0 there, no geometric wetting
  double gw_half[2];        // G_w / 2 of the bottom and top wall
};

// One block's share of a step: columns [x0, x0+width) of rows [y0, y0+nrows) of instance inst
// (width <= 64 * waves per block, width >= 2).
struct WaveTask {
  int32_t inst, x0, y0, wh;  // wh = width | (nrows << 16)
};

// Per-block results of a checked step.
struct WaveDiag {
  double mass;
  int32_t nonfinite, psi_clamps, ghost_clamps, pad;
};

// Per-instance accumulated diagnostics (device).
struct InstDiag {
  double mass;
  long long checks, nonfinite, psi_clamps, ghost_clamps, pad;
};

// state storage: FP64, FP32 (FP32 arithmetic), FP32 with the mixed arithmetic of LBM_F32_SHIFTED_MIXED
enum { STORE_F64 = 0, STORE_F32 = 1, STORE_F32M = 2 };

// Launch helpers implemented in lbm_kernels.hip. All return the hipError_t of the launch.
// waves: wavefronts per block (1, 2, 4 or 8; the tasks must have been built for it); tau1: specialised collision
// for tau = 1 (every instance of the launch must have tau = 1).
constexpr int kWaveChoices[] = {1, 2, 4, 8};
constexpr int kNumWaveChoices = 4;
// prefetch: the populations of row y+2 are loaded while row y is processed.
// down < 0: odd flips walk the strips downwards (consecutive steps alternate); 0 / 1 force up / down.
hipError_t launch_step(int storage, bool check, bool tau1, int waves, bool prefetch, const InstDesc* d_desc,
                       const WaveTask* d_tasks, int ntasks, int flip, WaveDiag* d_wdiag, hipStream_t s,
                       int down = -1);
// Two steps per launch (lbm_step2.hip): geometric walls (every instance of the launch); general = false for the
// tau = 1 BGK collision everywhere, true for each instance's own (MRT with the surface-tension source, or BGK at
// any tau). Tasks are tiles: output columns [x0, x0 + width) with width <= 64 waves - 8 (the kernel adds four halo
// lanes per side), output rows [y0, y0 + nrows). Reads buffer cur ^ flip, writes the other one (as one one-step
// launch). storage: STORE_F64, STORE_F32 or STORE_F32M (the mixed arithmetic of LBM_F32_SHIFTED_MIXED).
// d_wdiag (one entry per task) makes it a checked launch: the diagnostics of the second step's input state, which
// k_finalize_diag then folds per instance over the two-step task ranges.
hipError_t launch_step2(const InstDesc* d_desc, const WaveTask* d_tasks, int ntasks, int waves, int storage,
                        bool general, int flip, hipStream_t s, WaveDiag* d_wdiag = nullptr);
// Resident blocks of the two-step kernel per compute unit (hipOccupancyMaxActiveBlocksPerMultiprocessor).
hipError_t step2_blocks_per_cu(int waves, int storage, bool general, int* blocks);
hipError_t launch_finalize_diag(const WaveTask* d_tasks, const int32_t* d_inst_first, int ninst_sel, int inst0,
                                const WaveDiag* d_wdiag, InstDiag* d_idiag, const InstDesc* d_desc,
                                hipStream_t s);
hipError_t launch_init_droplets(int storage, const InstDesc* d_desc, int inst, int ny_fluid, int nx,
                                const double* d_drops, int ndrops, double width, double rho_l, double rho_v,
                                double* d_rho_scratch, hipStream_t s);
hipError_t launch_wetting(int storage, const InstDesc* d_desc, int inst, int nx, hipStream_t s);
hipError_t launch_get_rho(int storage, const InstDesc* d_desc, int inst, int nx, int ny, double* d_dst,
                          hipStream_t s);
// Population planes [q0, q1) as FP64 [q1-q0][ny-2][nx] (unshifted), and the reverse.
hipError_t launch_get_pops(int storage, const InstDesc* d_desc, int inst, int nx, int ny, int q0, int q1,
                           double* d_dst, hipStream_t s);
// Stored plane q from physical plane p ([ny-2][nx] FP64): p == q fills nodes streaming into the fluid,
// p == opp(q) the nodes bouncing back at a wall.
hipError_t launch_set_plane(int storage, const InstDesc* d_desc, int inst, int nx, int ny, int q, int p,
                            const double* d_src, hipStream_t s);
hipError_t launch_mass(int storage, const InstDesc* d_desc, int inst, int nx, int ny, double* d_partials,
                       int nblocks, hipStream_t s);
hipError_t launch_minmax(const double* d_rho, int nx, int ny, const int32_t* box, double* d_partials,
                         int nblocks, hipStream_t s);
hipError_t launch_ca_moments(const double* d_rho, int nx, int ny, const int32_t* box, int wall, double rho_mid,
                             double shift_x, double shift_y, double* d_partials, int nblocks, hipStream_t s);
hipError_t launch_zero_diag(InstDiag* d_idiag, int n, hipStream_t s);
hipError_t launch_set_cur(InstDesc* d_desc, int inst, int cur, hipStream_t s);

// Adjoint (FP64 only): scratch carved from the workspace of an instance created with enable_adjoint.
struct AdjScratch {
  double* rho;    // [ny][pitch]  densities, ghost rows included
  double* psi;    // [ny][pitch]
  double* Fbar;   // [2][ny][pitch]  adjoint of the force at fluid nodes (x then y component)
  double* gflag;  // [2][nx]  1 where the forward ghost density was clamped
  double* wet;    // [2][4][nx]  adjoints of the densities feeding each ghost column
  double* qwall;  // [2][3][nx]  adjoint of Q (Eq. 17: xx, yy, xy) on the boundary rows 1 and ny-2
  double* part;   // [adjoint_partials_needed()] reduction partials for G_bar
};
int adjoint_partials_needed();
// f32: the state and lambda are FP32 (else FP64); theta_bar and G_bar are FP64 either way
hipError_t launch_adjoint(const InstDesc* d_desc, const InstDesc& h, int inst, const AdjScratch& sc, bool f32,
                          const void* f_n, const void* lam_np1, void* lam_n, double* theta_bar, double* G_bar,
                          hipStream_t s);

// lambda_N [9][nyf][nx] (FP32 if f32, else FP64) = grad_rho [nyf][nx] on every plane; theta_bar [2][nx] and G_bar[2]
// set to zero.
hipError_t launch_adjoint_seed_rho(bool f32, const double* grad_rho, void* lam, double* theta_bar, double* G_bar,
                                   int nx, int nyf, hipStream_t s);

constexpr int kMeasureBlocks = 512;
constexpr int kMeasureMoments = 10;
// Doubles of reduction partials one contact-angle measurement needs (min/max pass, then the moments pass).
constexpr int kMeasurePartials = kMeasureBlocks * kMeasureMoments;

// Host part of the contact-angle measurement on a device density field rho [ny][nx] (FP64, ghost rows included),
// box already clipped to the fluid rows: min/max and moment passes with their partials in d_partials
// (kMeasurePartials doubles), folded on the host in a fixed order, Kasa fit. Returns an lbm_status and sets
// lbm_last_error on failure. Synchronizes the stream. Implemented in lbm_api.cpp.
int measure_contact_angle_field(const double* d_rho, int nx, int ny, int wall, const int32_t box[4],
                                double* d_partials, hipStream_t s, double out[5]);
// Sets the message lbm_last_error() returns and passes the status through (lbm_api.cpp).
int report_error(int code, const char* msg);

}  // namespace lbm
