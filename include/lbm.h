/* liblbm — EOS-based single-component pseudo-potential lattice Boltzmann method with the geometric
 * contact-angle wall, for AMD Instinct MI355X (gfx950).
 *
 * Method: Hu, Li & Uddin, "Contact Angle Adjustment in Equation of States Based Pseudo-Potential Model",
 * arXiv:1501.05430. One time step is
 *   streamed populations f -> density rho, momentum j            (Sec. 2, Eq. 1)
 *   -> effective density psi(rho), Carnahan-Starling EOS          (Eq. 10, c = 1)
 *   -> ghost-layer density at each wall from theta                (Sec. 4, Eq. 19-21)
 *   -> interaction force, hybrid form with parameter A            (Eq. 9, weights of Eq. 7)
 *   -> BGK collision with Guo forcing, v = (j + F/2)/rho          (Eq. 1-6 with diag(0,1,...,1), Sec. 3.1)
 *   -> streaming with halfway bounce-back at the walls.
 * Per instance (lbm_params) the EOS may instead be the piecewise-linear one of Eq. 11-13, the collision the MRT
 * form of Eq. 15 with general rates and the surface-tension source of Eq. 16-17, and the walls those of the
 * comparison method (the fluid-solid force of Eq. 14) or none (periodic rows).
 *
 * Lattice: D2Q9, velocities e0=(0,0), e1..e4=(1,0),(0,1),(-1,0),(0,-1), e5..e8=(1,1),(-1,1),(-1,-1),(1,-1)
 * (the moment order of Eq. 4). Grid nx x ny with x periodic; rows 0 and ny-1 are the ghost layer beside the
 * walls (Sec. 4 index 0) and carry only density and psi; rows 1..ny-2 are fluid. The wall planes sit at
 * y = 0.5 and y = ny - 1.5.
 *
 * Conventions for every entry point:
 *  - The return value is a status (lbm_status); 0 = LBM_OK. No C++ exception or abort crosses this boundary.
 *    On failure lbm_last_error() returns a thread-local message.
 *  - Device memory is owned by the caller: one workspace of lbm_workspace_bytes() bytes, passed to lbm_create.
 *    The library never allocates or frees device memory. lbm_destroy frees only host memory.
 *  - Work is queued asynchronously on the HIP stream given to lbm_create, except where a function says it
 *    synchronizes that stream. A context is not thread-safe; use one context per stream.
 *  - Pointers named d_* are device pointers; all others are host pointers. Angles are in radians.
 *  - Invalid arguments return LBM_E_INVALID before any work is queued.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_API_VERSION 1

typedef enum {
  LBM_OK = 0,
  LBM_E_INVALID = 1,     /* bad argument or parameter */
  LBM_E_WORKSPACE = 2,   /* workspace too small or misaligned (256 B) */
  LBM_E_HIP = 3,         /* a HIP runtime call failed; message has the HIP error text */
  LBM_E_UNSTABLE = 4,    /* a non-finite density was seen by a periodic check; state stays readable */
  LBM_E_STATE = 5,       /* call out of order (e.g. stepping before lbm_init_droplet / lbm_set_populations) */
  LBM_E_UNSUPPORTED = 6  /* valid request this build does not provide */
} lbm_status;

typedef enum {
  LBM_F64 = 0,         /* populations stored and computed in FP64 */
  LBM_F32 = 1,         /* populations stored and computed in FP32 */
  LBM_F32_SHIFTED = 2, /* FP32 storage of f_i - w_i rho0 (rho0 = rho0_shift), computed in FP32 */
  LBM_F32_SHIFTED_MIXED = 3  /* FP32 storage of f_i - w_i rho0 (rho0 = rho0_shift, 0 = unshifted) as in
                          LBM_F32_SHIFTED, and the same FP32 sums (density, momentum, the rest population from the
                          mass balance), but psi from the FP64 EOS (Eq. 10, rounded to FP32) at every density and
                          the force (Eq. 9), velocity, equilibrium and forcing terms (Eq. 1-6) in FP64; MRT (Eq. 15)
                          is evaluated in FP64 throughout. Same memory traffic as the other FP32 modes; holds the
                          density to the FP64 result over long runs where FP32 arithmetic drifts (the FP32 rounding of
                          the force and the equilibrium accumulates over thousands of steps). rho_fp64_below is not
                          used. */
} lbm_precision;

typedef enum {
  LBM_WALLS_Y = 0,     /* rows 0 and ny-1 are the walls' ghost rows (Sec. 4 wetting, halfway bounce-back) */
  LBM_PERIODIC_Y = 1,  /* no walls: fluid rows 1..ny-2 wrap around (a periodic lattice of ny-2 rows; the ghost
                          rows are unused and read back as 0). x is periodic in all cases. */
  LBM_WALLS_MARTYS_CHEN = 2  /* the comparison method of Sec. 3: rows 0 and ny-1 are solid walls that attract the
                          fluid through the force of Eq. 14 (strength G_w per wall) and take no part in the
                          fluid-fluid force (psi = 0 there; they read back as 0); halfway bounce-back as for
                          LBM_WALLS_Y, no geometric wetting (contact angles unused; theta_bar stays 0). */
} lbm_boundary;

typedef enum {
  LBM_EOS_CARNAHAN_STARLING = 0,  /* p = rho R T (1 + e + e^2 - e^3) / (1 - e)^3 - a rho^2, e = b rho / 4, at
                                     T = T_over_Tc T_c; coexistence from the equal-area construction */
  LBM_EOS_PIECEWISE_LINEAR = 1    /* Eq. 11: slopes theta_v, theta_m, theta_l (pw_theta) on [0, rho_1],
                                     [rho_1, rho_2], [rho_2, inf); the break points solve Eq. 12 (equal pressure)
                                     and Eq. 13 (equal chemical potential) for the coexistence pair pw_rho. Needs
                                     0 < theta_v < 1/3, theta_m < 0, theta_l > 0 and 0 < rho_v < rho_l, with psi
                                     real up to rho_l; eos_a/b/R and T_over_Tc are ignored */
} lbm_eos;

typedef struct lbm_ctx lbm_ctx; /* opaque; holds host memory only */

/* Parameters of one lattice instance. Defaults in brackets are the paper's / the workloads' values. */
typedef struct {
  int32_t nx, ny;         /* columns (periodic) and rows including both ghost rows; nx >= 2, ny >= 4,
                             ny - 2 <= 65535, and pitch x (ny - 2) < 2^31 with pitch = nx rounded up to 64 (about
                             2.1e9 fluid nodes: 155 GB of FP32 populations) */
  int32_t precision;      /* lbm_precision; every instance of a context must use the same one */
  int32_t wet_iters;      /* 0: Eq. 19; k >= 1: k-th iterate of Eq. 21 (first line = iterate 1) [4] */
  int32_t check_every;    /* steps between device checks of mass, non-finite density and clamps; 0 = none */
  int32_t strip_rows;     /* rows per block strip of the step kernels; 0 = library default: for the one-step
                             kernel about two blocks per compute unit over all instances, 2..32 rows (FP32) / 2..64
                             (FP64); for the two-step kernel one round of resident blocks */
  int32_t enable_adjoint; /* 1: reserve workspace for lbm_adjoint_step (any precision) */
  int32_t step_variant;   /* step kernel shape: k = 1..4 selects the one-step kernel with 1, 2, 4 or 8 wavefronts
                             (64, 128, 256 or 512 aligned columns) per block, 5..8 the same with the next row's
                             loads in flight; 9..12 the two-step kernel (two time steps per launch, geometric or
                             Martys-Chen walls, any collision and precision; periodic rows step one at a time) with
                             1, 2, 4 or 8 wavefronts per block; 0 = library default (two-step where it applies on
                             contexts of at least 50 000 fluid nodes, one-step below; one wavefront per two-step
                             block while every instance has fewer than 3 000 000 fluid nodes).
                             Instance 0's value applies to the whole context (lbm_autotune may change it). Results
                             do not depend on it (bitwise). */
  int32_t boundary;       /* lbm_boundary [LBM_WALLS_Y] */
  int32_t eos;            /* lbm_eos [LBM_EOS_CARNAHAN_STARLING] */
  double tau;             /* BGK relaxation time (> 0.5) [1.0] */
  double G;               /* interaction strength, < 0 [-1.0] */
  double A;               /* hybrid-force parameter of Eq. 9 [-0.6]; 0 = plain Shan-Chen force (Eq. 7) */
  double eos_a, eos_b, eos_R; /* Carnahan-Starling constants [1, 4, 1] */
  double T_over_Tc;       /* temperature as a fraction of the EOS critical temperature, in (0, 1) */
  double rho0_shift;      /* LBM_F32_SHIFTED: reference density rho0 of the stored f_i - w_i rho0 */
  double rho_fp64_below;  /* FP32 modes: the EOS / psi is evaluated in FP64 where rho < this; 0 = never */
  double body_force[2];   /* constant body force per unit volume (F_g of Eq. 7) [0, 0] */
  double pw_theta[3];     /* LBM_EOS_PIECEWISE_LINEAR: theta_v, theta_m, theta_l of Eq. 11 (Table 1: e.g.
                             0.25, -0.02, 0.3 for a density ratio of 10) */
  double pw_rho[2];       /* LBM_EOS_PIECEWISE_LINEAR: rho_v, rho_l (Eq. 12-13), e.g. 1 and 10 */
  double mrt_rates[3];    /* s_e, s_eps, s_q of Eq. 2 (tau_e^-1, tau_xi^-1, tau_q^-1), each 0 (= 1/tau) or in
                             (0, 2). Any non-zero rate, or kappa != 0, selects the MRT collision of Eq. 15 (stress
                             relaxed at 1/tau; the conserved moments' rates do not enter); all 0 with kappa = 0 is
                             BGK, the same scheme up to rounding. [0, 0, 0] */
  double kappa;           /* surface-tension parameter of Eq. 16-17: the source C with Q = kappa (G/2)[...] scales
                             the surface tension by 1 - kappa and leaves flat-interface densities unchanged. [0] */
  double G_w[2];          /* LBM_WALLS_MARTYS_CHEN: G_w of Eq. 14 for the bottom and top wall (more negative
                             attracts more: smaller contact angle); ignored otherwise [0, 0] */
} lbm_params;

/* Device diagnostics of one instance, accumulated by the periodic checks (check_every) of lbm_step. */
typedef struct {
  double mass;            /* FP64 sum of the populations over fluid nodes at the last check */
  int64_t checks;         /* number of checks run since lbm_create / lbm_init_droplet */
  int64_t nonfinite;      /* fluid nodes with a non-finite density, summed over checks */
  int64_t psi_clamps;     /* fluid nodes where p_EOS - rho/3 had the wrong sign (psi set to 0), summed */
  int64_t ghost_clamps;   /* ghost densities clamped into [0, rho_cap), summed over checks */
  int64_t steps;          /* time steps taken since the last initialization */
} lbm_diag;

/* Bytes of device workspace for n_inst instances described by p[0..n_inst-1]; 0 if the parameters are
 * invalid (lbm_last_error says why). */
size_t lbm_workspace_bytes(const lbm_params* p, int32_t n_inst);

/* Create a context over n_inst instances. d_workspace: caller-owned device memory, 256-byte aligned, at least
 * lbm_workspace_bytes(p, n_inst) bytes, kept alive until lbm_destroy. hip_stream: a hipStream_t (NULL = the
 * null stream; graph replay of lbm_step then falls back to plain launches). The EOS critical point, Maxwell
 * coexistence densities and the largest density with real psi are solved on the host in FP64 here. The
 * populations start undefined: call lbm_init_droplet or lbm_set_populations before lbm_step. */
int lbm_create(const lbm_params* p, int32_t n_inst, void* d_workspace, size_t ws_bytes, void* hip_stream,
               lbm_ctx** out);

/* Free the context (host memory only; the workspace and the stream stay the caller's). NULL: LBM_E_INVALID. Work
 * already queued on the stream is not waited for: synchronize the stream before reusing the workspace. */
int lbm_destroy(lbm_ctx* c);

/* Host FP64 EOS data of instance inst. Carnahan-Starling: out[0] = rho_v, out[1] = rho_l (Maxwell equal-area
 * coexistence), out[2] = T (absolute), out[3] = T_c, out[4] = rho_c. Piecewise linear: out[0], out[1] = pw_rho,
 * out[2] = rho_1, out[3] = rho_2 (the break points of Eq. 12-13), out[4] = 0. Both: out[5] = rho_cap, the largest
 * density with real psi (Eq. 10), or 1e300 where psi is real at every density above the vapour. */
int lbm_eos_info(const lbm_ctx* c, int32_t inst, double out[6]);

/* Coexistence densities of instance inst (host FP64, solved at lbm_create): out[0] = rho_v, out[1] = rho_l. For
 * Carnahan-Starling the Maxwell equal-area pair at T_over_Tc T_c (the counterpart of the two-phase conditions the
 * paper writes for Eq. 11 as Eq. 12-13); for the piecewise-linear EOS the pair pw_rho that Eq. 12-13 were solved
 * for. lbm_eos_info reports these with the rest of the EOS data. */
int lbm_coexistence(const lbm_ctx* c, int32_t inst, double out[2]);

/* Initial state (droplets at rest): rho(x, y) = rho_v + (rho_l - rho_v) (1 - tanh(2 (r - R_k)/width)) / 2,
 * the maximum over the n droplets, r the distance from node (x, y) to (xc[k], yc[k]) with the nearest periodic
 * image in x; f_i = w_i rho. rho_l <= 0 or rho_v <= 0 selects the Maxwell value. The setup of Sec. 3.1 is one
 * semicircle on the bottom wall: yc = 0.5. Resets the step counter and diagnostics. Host arrays [n]. */
int lbm_init_droplet(lbm_ctx* c, int32_t inst, int32_t n, const double* xc, const double* yc, const double* R,
                     double width, double rho_l, double rho_v);

/* Set the wall contact angles (Sec. 4): theta_bottom / theta_top are host arrays of nx angles in (0, pi),
 * one per wall column; NULL keeps the current values (initially pi/2). Then recomputes the ghost-row densities
 * of the current state (Eq. 19 or Eq. 21) into the context, readable with lbm_get_rho. The ghost rows are also
 * recomputed inside every lbm_step. Synchronizes the stream (the host arrays may be reused on return). */
int lbm_apply_wetting(lbm_ctx* c, int32_t inst, const double* theta_bottom, const double* theta_top);

/* Advance nsteps time steps. inst >= 0 steps one instance; inst = -1 steps every instance, each kernel launch
 * covering all of them (two time steps per launch where step_variant allows it, see above). Steps are replayed from
 * a captured HIP graph in chunks when the stream is not the null stream. With check_every > 0 a device check runs
 * every check_every steps and after the last step, on the state its step starts from (inside a two-step launch when
 * the step before it is unchecked); the call then synchronizes the stream once at its end and returns
 * LBM_E_UNSTABLE if a check saw a non-finite density. */
int lbm_step(lbm_ctx* c, int32_t inst, int64_t nsteps);

/* lbm_step with device timing: HIP events on the context's stream bracket the queued steps (recorded before the
 * first launch and after the last, ahead of the closing synchronization of the checks), and *ms receives the
 * elapsed time between them. Synchronizes the stream. Same status as lbm_step (LBM_E_UNSTABLE still sets *ms). */
int lbm_step_timed(lbm_ctx* c, int32_t inst, int64_t nsteps, double* ms);

/* Contact angle of the droplet inside box = {x_lo, x_hi, y_lo, y_hi} (half-open node ranges; rows are clipped
 * to the fluid rows) on wall 0 (bottom) or 1 (top). Reading of the method (the paper quotes angles without the
 * procedure): rho_mid = (max + min)/2 over the box; rho_mid crossings on horizontal and vertical links by linear
 * interpolation; points within 3 nodes of the wall plane dropped; algebraic (Kasa) circle fit from FP64 moments;
 * theta = acos((y_w - y_c)/R) (bottom) or acos((y_c - y_w)/R) (top). out = {theta, R, x_c, y_c, n_points}.
 * Synchronizes the stream. */
int lbm_measure_contact_angle(lbm_ctx* c, int32_t inst, int32_t wall, const int32_t box[4], double out[5]);

/* lbm_measure_contact_angle for callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same measurement on a density field the caller holds, with no
 * context and no workspace. d_rho: device FP64 field [ny][nx] (row 0 and ny-1 the ghost rows, as lbm_get_rho
 * writes it), read only; box, wall and out[5] as for lbm_measure_contact_angle (results identical to it on the same
 * field). The reduction partials live in a library-owned device array of 512 x 10 doubles (40 KiB) per GPU, held
 * until the process ends; the measurement's grid is fixed, so any field size fits (nx >= 2, ny >= 4,
 * nx ny <= 2^34). Nothing is allocated. Runs on the current device on hip_stream and synchronizes it. Calls that
 * overlap on one GPU share that array and race: serialize them. */
int lbm_measure_contact_angle_noalloc(const double* d_rho, int32_t nx, int32_t ny, int32_t wall,
                                      const int32_t box[4], void* hip_stream, double out[5]);

/* FP64 total mass (sum of all populations over fluid nodes) of the current state. Synchronizes the stream. */
int lbm_mass(lbm_ctx* c, int32_t inst, double* out);

/* Diagnostics accumulated by the periodic checks. Synchronizes the stream. */
int lbm_get_diag(lbm_ctx* c, int32_t inst, lbm_diag* out);

/* Density of the current state as FP64 [ny][nx]: fluid rows sum the populations (FP64 sum of the stored values
 * plus 9 w_i rho0 when shifted); rows 0 and ny-1 hold the ghost densities the next step will use (clamped).
 * dst_on_device != 0: dst is a device pointer (stream-ordered); otherwise host (synchronizes). */
int lbm_get_rho(lbm_ctx* c, int32_t inst, double* dst, int32_t dst_on_device);

/* Populations of the current state as FP64 [9][ny-2][nx] (unshifted f_i, fluid rows 1..ny-2), to a device or
 * host buffer; and the reverse (rounded to the storage precision). */
int lbm_get_populations(lbm_ctx* c, int32_t inst, double* dst, int32_t dst_on_device);
int lbm_set_populations(lbm_ctx* c, int32_t inst, const double* src, int32_t src_on_device);

/* Raw state (the stored populations, lbm_state_bytes bytes) for checkpoint / resume, device to device. */
size_t lbm_state_bytes(const lbm_ctx* c, int32_t inst);
int lbm_get_state(lbm_ctx* c, int32_t inst, void* d_dst);
int lbm_set_state(lbm_ctx* c, int32_t inst, const void* d_src);

/* Choose the step kernel's shape (wavefronts per block, prefetch: context-wide) and the rows per strip by timing
 * the launch that lbm_step(inst) runs on the current state, for every candidate: first one strip height for the
 * whole selection, then, with several lattice shapes in the selection (inst = -1), each shape's height in turn.
 * The state is not modified (trials read the current buffer and write the spare one). trial_steps > 0 timed
 * launches per candidate. *chosen receives the rows per strip of inst (of instance 0 for inst = -1).
 * Synchronizes. */
int lbm_autotune(lbm_ctx* c, int32_t inst, int32_t trial_steps, int32_t* chosen);

/* The step shape of a context: what lbm_autotune chose (or the defaults), to keep and re-apply later without the
 * trials (the Python binding keeps a JSON cache of these records, keyed by the device and the instances). */
typedef struct {
  int32_t two_step;  /* 1: two time steps per launch wherever the selection allows it (walls, not periodic rows:
                        any collision and precision); 0: one step per launch */
  int32_t waves;     /* one-step kernel: wavefronts per block, 1, 2, 4 or 8 */
  int32_t prefetch;  /* one-step kernel: 1 = the next row's loads in flight, 0 = not */
  int32_t waves2;    /* two-step kernel: wavefronts per block, 1, 2, 4 or 8 */
} lbm_tuning;

/* Reads the context's shape into *t and, when the arrays are non-NULL, every instance's rows per strip of the
 * one-step and the two-step kernel (n_inst entries each, the count lbm_create was given). Host only. */
int lbm_get_tuning(const lbm_ctx* c, lbm_tuning* t, int32_t* strip_rows, int32_t* strip_rows2);

/* Applies a shape read by lbm_get_tuning (from this or another context with the same instances): wavefronts in
 * {1, 2, 4, 8}, prefetch and two_step 0 or 1, rows per strip >= 1 (NULL arrays keep the current rows; two_step
 * is ignored for FP64 storage). LBM_E_INVALID on any other value, with nothing changed. Results do not depend on
 * the shape (bitwise); the context's captured graphs are dropped. Stream-ordered: uploads the task tables. */
int lbm_set_tuning(lbm_ctx* c, const lbm_tuning* t, const int32_t* strip_rows, const int32_t* strip_rows2);

/* Adjoint of one time step (the reverse of streaming, collision, force, wetting and psi, in that order).
 * Given the FP64 populations f_n of step n (d_state_n, [9][ny-2][nx], unshifted) and the adjoint
 * lambda_{n+1} = dL/df_{n+1} (same layout), writes lambda_n = (d f_{n+1} / d f_n)^T lambda_{n+1} to d_lambda_n
 * and ACCUMULATES d_theta_bar[2][nx] += (d f_{n+1}/d theta)^T lambda_{n+1} (bottom row then top row) and
 * d_G_bar[2] += {dL/dG_f, dL/dG_psi}, G_f being the prefactor of the force of Eq. 9 and of Q in Eq. 17 and G_psi
 * the G inside Eq. 10 (equal in the forward model, so their sum is the total derivative: zero with geometric walls,
 * where every term depends on G_f / G_psi only; the fluid-solid force of Eq. 14 scales with psi alone). Covers the
 * BGK and MRT collisions with the source of Eq. 16-17, both EOS, geometric and Martys-Chen walls and periodic rows
 * (theta_bar stays 0 without geometric walls). Needs enable_adjoint = 1. The adjoint is evaluated in FP64 at the given state for every precision: for an FP32
 * instance it differentiates the FP32 trajectory (pass its populations from lbm_get_populations). Runs on the
 * context's stream; sub-gradient 0 at exact kinks (|T| of Eq. 19, the square root at 0, the clamps). Does not
 * change the context's state. */
int lbm_adjoint_step(lbm_ctx* c, int32_t inst, const double* d_state_n, const double* d_lambda_np1,
                     double* d_lambda_n, double* d_theta_bar, double* d_G_bar);

/* lbm_adjoint_step with the state and the adjoints in FP32 (device arrays of the same [9][ny-2][nx] layout): the
 * arithmetic is the same FP64 evaluation, only the state is read from and lambda_n written to FP32, which halves
 * the reverse step's unavoidable traffic (108 B per fluid node). d_theta_bar and d_G_bar stay FP64 and accumulate
 * as above. Same preconditions and errors as lbm_adjoint_step. */
int lbm_adjoint_step_f32(lbm_ctx* c, int32_t inst, const float* d_state_n, const float* d_lambda_np1,
                         float* d_lambda_n, double* d_theta_bar, double* d_G_bar);

/* Adjoint of the density readout rho = sum_i f_i (the fluid rows of lbm_get_rho, Eq. 1's zeroth moment): given
 * d_grad_rho = dL/drho_N [ny-2][nx] (FP64, device), writes lambda_N = dL/df_N [9][ny-2][nx] (every population of a
 * node receives that node's dL/drho; FP64, or FP32 for the _f32 form that lbm_adjoint_step_f32 takes) and sets the
 * accumulators d_theta_bar [2][nx] and d_G_bar [2] to zero: the start of a reverse sweep of lbm_adjoint_step calls.
 * Stream-ordered; needs no enable_adjoint. */
int lbm_adjoint_seed_rho(lbm_ctx* c, int32_t inst, const double* d_grad_rho, double* d_lambda, double* d_theta_bar,
                         double* d_G_bar);
int lbm_adjoint_seed_rho_f32(lbm_ctx* c, int32_t inst, const double* d_grad_rho, float* d_lambda,
                             double* d_theta_bar, double* d_G_bar);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
