/*
 * lbm.h - C ABI of the MI355X (gfx950) free-energy lattice Boltzmann library.
 *
 * The library advances the forcing-based free-energy multiphase lattice
 * Boltzmann method of Li, Yu & Huang (arXiv:2008.01473) on periodic D2Q9 and
 * D3Q19 lattices, in the paper's standard scheme (force of Eq. 13, equilibrium
 * of Eq. 11, collision of Eq. 9) and in its improved scheme (p_m = (1 + mu)/3,
 * force of Eq. 24, equilibrium of Eq. 27, correction term of Eqs. 28-29), with
 * the BGK special case Lambda = I / tau of the relaxation matrix (Eq. 8) or,
 * on D2Q9, the full relaxation matrix of Eq. 8 (optionally with a per-node
 * shear rate that holds the kinematic viscosity constant).
 * The chemical potential is Eq. 2 with the van der Waals free energy of Eq. 30
 * or a Carnahan-Starling free energy; gradients use the isotropic stencil of
 * Eq. 17 and the Laplacian its isotropic counterpart with the same weights.
 *
 * Conventions shared by every entry point
 *   - Return value: LBM_OK (0) or a negative LBM_ERR_* code; no C++ exception
 *     crosses this boundary.  lbm_error_string() describes a code, and
 *     lbm_last_error() the most recent failure of the calling thread in words.
 *   - Device memory: every large buffer (distributions, workspace, input and
 *     output fields) is allocated and owned by the caller.  The library owns
 *     only the handle, a few small host tables and the HIP graphs it captures.
 *   - Streams: work is enqueued, asynchronously, on the hipStream_t given to
 *     lbm_create / lbm_create_batch (NULL = the null stream).  Only
 *     lbm_diagnostics, lbm_maxwell and the size queries block the host.
 *   - Field layout across the boundary: float64, structure of arrays, row-major
 *     with x fastest.  A scalar field of one lattice has nz*ny*nx entries
 *     indexed (z*ny + y)*nx + x (nz = 1 in 2D); a vector field has D such
 *     blocks (component x first).  In a batch the lattices follow one another
 *     in creation order, each starting at its node offset (lbm_node_offset).
 *   - Distribution layout (lbm_get_f / lbm_set_f): Q blocks of one scalar
 *     field each, population a at block a.  Velocity order
 *       D2Q9 : rest; E, N, W, S; NE, NW, SW, SE
 *              (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *       D3Q19: rest; +x, -x, +y, -y, +z, -z;
 *              (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1)
 *              (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *     These are the populations f_a(x, t) after streaming (Eq. 10) and before
 *     the next collision, i.e. those from which Eq. 12 computes rho and u.
 *   - Time level: a handle holds one time level t (0 after lbm_init); each
 *     lbm_step advances it by one.  lbm_moments returns the fields at t.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_status_code {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,          /* invalid argument or parameter combination        */
    LBM_ERR_UNSUPPORTED = -2,  /* valid request the library does not implement    */
    LBM_ERR_HIP = -3,          /* a HIP runtime call failed                        */
    LBM_ERR_BLOWUP = -4,       /* a lattice produced NaN/Inf or left the EOS domain */
    LBM_ERR_DOMAIN = -5,       /* no liquid-gas coexistence (e.g. T >= T_c)        */
    LBM_ERR_STATE = -6         /* call out of order (e.g. step before bind/init)   */
};

enum lbm_lattice   { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
enum lbm_eos       { LBM_EOS_VDW = 0, LBM_EOS_CS = 1 };
enum lbm_scheme    { LBM_STANDARD = 0, LBM_IMPROVED = 1 };
enum lbm_force     { LBM_FORCE_CHEMPOT = 0, LBM_FORCE_PTENSOR = 1 };
enum lbm_precision { LBM_FP64 = 0, LBM_FP32_DEV = 1 };
enum lbm_collision { LBM_BGK = 0, LBM_MRT = 1 };

/* Per-lattice blow-up flags, OR-ed into lbm_diag.status. */
enum lbm_blowup_bits {
    LBM_BLOWUP_NONFINITE = 1,  /* rho, u or a population is NaN or Inf      */
    LBM_BLOWUP_RHO_NONPOS = 2, /* rho <= 0                                  */
    LBM_BLOWUP_RHO_MAX = 4     /* rho >= packing limit (1/b vdW, 4/b CS)    */
};

/*
 * Physical and numerical parameters of one lattice.
 *   lattice      LBM_D2Q9 or LBM_D3Q19 (nz must be 1 for D2Q9)
 *   nx, ny, nz   lattice extent, periodic in every direction, each >= 1
 *   eos          LBM_EOS_VDW: E_f = rho R T ln[rho/(1 - b rho)] - a rho^2 (Eq. 30)
 *                LBM_EOS_CS : E_f = rho R T [ln rho + (4h - 3h^2)/(1-h)^2] - a rho^2,
 *                             h = b rho / 4 (Carnahan-Starling; not in the paper)
 *   a, b, R      EOS constants (the paper: a = 9/392, b = 2/21, R = 1)
 *   T_over_Tc    reduced temperature; T_c is 8a/(27Rb) for vdW and the numerical
 *                critical point of the CS free energy
 *   kappa        interfacial coefficient of Eq. 1 (> 0)
 *   tau          BGK relaxation time, Lambda = I/tau (> 0.5)
 *   scheme       LBM_STANDARD (Eq. 13) or LBM_IMPROVED (Eq. 24, 27, 28-29)
 *   force_form   LBM_FORCE_CHEMPOT (rho grad mu) or LBM_FORCE_PTENSOR (div P of
 *                Eqs. 4-5); PTENSOR requires LBM_STANDARD
 *   precision    LBM_FP64: float64 storage and arithmetic.
 *                LBM_FP32_DEV: float32 storage of f - fbar and float32 arithmetic,
 *                fbar the rest equilibrium at (rho_ref, u = 0, p_m = pm_ref);
 *                mass sums stay float64.
 *   rho_ref, pm_ref  FP32_DEV reference state; values <= 0 select the defaults
 *                rho_ref = (rho_g + rho_l)/2 of the Maxwell construction and
 *                pm_ref = (1 + mu_sat)/3 (improved) or rho_ref/3 (standard).
 *   collision    LBM_BGK (zero, the default): Lambda = I/tau.
 *                LBM_MRT (D2Q9 only): the relaxation matrix of Eq. 8 in the
 *                moment basis (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy),
 *                Lambda = diag(1, 1/tau_e, 1/tau_s, 1, 1/tau_q, 1, 1/tau_q,
 *                1/tau_v, 1/tau_v) (tau_c = 1 for the conserved moments), applied
 *                as in Eq. 9 (standard) and Eq. 28 (improved).
 *   tau_e, tau_s, tau_q  MRT relaxation times of e (bulk viscosity), eps and q
 *                (each > 0.5); the paper leaves them free.
 *   nu           MRT shear relaxation: nu <= 0 gives tau_v = tau; nu > 0 holds the
 *                kinematic viscosity nu = eta/rho constant, i.e. tau_v = 3 nu + 1/2
 *                in the standard scheme (eta = rho c_s^2 (tau_v - 1/2), Sec. II A) and
 *                tau_v = nu rho / p_m + 1/2 per node in the improved scheme
 *                (eta = p_m (tau_v - 1/2), Sec. III).
 *   walls        0: periodic in y.  1 (D2Q9, chemical-potential force, ny >= 4):
 *                the lattice is bounded in y by two plates, halfway between rows
 *                -1 / 0 and ny-1 / ny, moving along x at wall_u_bottom / wall_u_top
 *                (the channel of Sec. IV B).  A population that would stream in
 *                from beyond a plate is the node's own reversed population plus
 *                feq_b - feq_-b of the scheme's equilibrium (Eq. 11 or Eq. 27) at the
 *                node's rho, p_m and the plate velocity (halfway bounce-back; the
 *                paper cites its no-slip scheme without stating it).  The stencils
 *                see beyond a plate the mirror image of the fluid (rho, mu, phi u_x
 *                even; phi u_y odd).  x stays periodic.
 *   wall_u_bottom, wall_u_top  plate velocities along x (lattice units)
 *   c0           improved scheme: p_m = (c0 + mu)/3.  0 selects the paper's c0 = 1
 *                (Sec. III); another value (> 0) is an extension, not the paper's
 *                method: the force of Eq. 24 depends on grad p_m only and the
 *                uniform-mu rest state stays a fixed point, while a smaller c0 keeps
 *                the gas rest population rho - 5 p_m/3 of Eq. 27 positive at lower
 *                T/T_c.
 * A zero-initialised tail (collision, tau_e, tau_s, tau_q, nu, walls, c0 all 0)
 * is the paper's method with BGK on a periodic lattice.
 * All lattices of one batch must share lattice, scheme, force_form, precision;
 * collision and its rates may differ between lattices.
 */
typedef struct {
    int lattice, nx, ny, nz;
    int eos;
    double a, b, R;
    double T_over_Tc, kappa, tau;
    int scheme, force_form, precision;
    double rho_ref, pm_ref;
    int collision, reserved;
    double tau_e, tau_s, tau_q, nu;
    int walls, reserved2;
    double wall_u_bottom, wall_u_top;
    double c0;
} lbm_params;

/*
 * Diagnostics of one lattice at one time level (float64 sums over the nodes in
 * a fixed order, so repeated runs give identical values):
 *   mass = sum rho,  mom = sum (j + F/2) = sum rho u (mom[2] = 0 in 2D),
 *   max_u = max |u|, mu_min / mu_max over the lattice, step = time level,
 *   status = OR of lbm_blowup_bits seen since lbm_init (0 = healthy).
 */
typedef struct {
    double mass, mom[3], max_u, mu_min, mu_max;
    long long step;
    int status, reserved;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Create a handle for one lattice.  Checks the parameters, solves the Maxwell
 * construction on the host (for the FP32_DEV defaults) and plans the tiling.
 * No device memory is allocated.  *out receives the handle.
 * The parameters are those of the paper's experiments (Sec. IV A: the van der
 * Waals free energy of Eq. 30 with a, b, R, the temperature as T/T_c, kappa of
 * Eq. 1 and the relaxation rates of Eq. 8); T_c = 8a/(27Rb) for vdW (Sec. IV A).
 * Errors: LBM_ERR_ARG for an invalid parameter (the message names it),
 * LBM_ERR_UNSUPPORTED for a valid combination the library does not implement
 * (e.g. MRT or plates on D3Q19, or a population array beyond 4 GB: more than
 * 2^30 nodes in one float32 lattice, 2^29 in float64; the kernels address each
 * array with unsigned 32-bit byte offsets). */
int lbm_create(const lbm_params* p, void* hip_stream, lbm_ctx** out);

/* Create a handle for `count` independent lattices advanced together by one
 * kernel launch per step (sizes, EOS constants, T, kappa and tau may differ). */
int lbm_create_batch(const lbm_params* p, int count, void* hip_stream, lbm_ctx** out);

/* Bytes of one distribution buffer (all lattices) and of the workspace the
 * caller must allocate; alignment of both: 256 bytes. */
size_t lbm_state_bytes(const lbm_ctx* h);
size_t lbm_workspace_bytes(const lbm_ctx* h);

/* Total nodes of the handle and the node offset of lattice i in field arrays. */
long long lbm_num_nodes(const lbm_ctx* h);
long long lbm_node_offset(const lbm_ctx* h, int i);
int lbm_count(const lbm_ctx* h);

/* Attach caller-owned device memory: two distribution buffers of
 * lbm_state_bytes each and one workspace of lbm_workspace_bytes.  Uploads the
 * small parameter and tile tables into the workspace (asynchronously). */
int lbm_bind(lbm_ctx* h, void* f_a, void* f_b, void* workspace);

/* Set time level 0: f = f_eq(rho0, u0) with the scheme's equilibrium (Eq. 11
 * or Eq. 27; p_m from mu(rho0) including -kappa lap(rho0)).  rho0: device,
 * float64, lbm_num_nodes entries; u0: device, float64, D blocks, or NULL for
 * u0 = 0.  Clears the blow-up flags. */
int lbm_init(lbm_ctx* h, const double* rho0, const double* u0);

/* Advance n >= 0 steps (Eqs. 7-10 with the scheme's force and sources), one
 * fused kernel per step; n >= 2 steps are replayed from a captured HIP graph.
 * Every step checks its input for blow-up; lattices whose blow-up flags are
 * set are skipped from then on.  The steps reduce no diagnostics: see
 * lbm_diagnostics. */
int lbm_step(lbm_ctx* h, int n);

/* Capture, without running them, the HIP graphs that lbm_step(h, n) will replay
 * from the current buffer parity, so that a later lbm_step(h, n) launches only
 * (e.g. outside a timed region).  Enqueues no work. */
int lbm_prepare_steps(lbm_ctx* h, int n);

/* Fields at the current time level (Eq. 12, Eq. 2): rho [N], u [D][N], mu [N];
 * device float64 pointers, any may be NULL.  Also refreshes the diagnostics. */
int lbm_moments(lbm_ctx* h, double* rho, double* u, double* mu);

/* Copy the diagnostics of every lattice (count entries) to host memory.  They
 * refer to the time level of the most recent lbm_step input or lbm_moments
 * call (lbm_diag.step).  After lbm_step they are reduced here, by one read-out
 * launch over the last step's input, which the second population buffer holds
 * until the next step.  Blocks until the stream has finished.  Returns
 * LBM_ERR_BLOWUP if any lattice has its status set (out is still filled).
 * The sums describe the state as it is, NaNs of a blown-up state included.
 * Lattices it reports blown up leave the launch plan (their populations stay
 * frozen and no work group is spent on them; captured graphs are re-captured
 * on the next lbm_step) until lbm_init, lbm_set_f or lbm_set_state clears the
 * flags; repeated calls before the next step return the same values, and a
 * lattice out of the plan keeps reporting the diagnostics (and step) it had
 * when it was reported. */
int lbm_diagnostics(lbm_ctx* h, lbm_diag* out_host);

/* Populations f_a(x, t) at the current time level as float64 (layout above),
 * and the inverse: replace the state by the given populations. */
int lbm_get_f(lbm_ctx* h, double* f_dev);
int lbm_set_f(lbm_ctx* h, const double* f_dev);

/* Raw checkpoint of the current state (lbm_state_bytes, device to device) and
 * its restore; the time level is saved/restored through *step. */
int lbm_get_state(lbm_ctx* h, void* dst_dev, long long* step);
int lbm_set_state(lbm_ctx* h, const void* src_dev, long long step);

/* Time level of the handle. */
long long lbm_time(const lbm_ctx* h);

/* Change kappa and T/T_c of lattice i (e.g. for finite-difference checks);
 * synchronises the stream and re-uploads the parameter table. */
int lbm_set_physics(lbm_ctx* h, int i, double kappa, double T_over_Tc);

/*
 * Adjoint (vector-Jacobian products) of the D2Q9 step, for one lattice per
 * handle with the improved scheme or the standard chemical-potential scheme.
 * The step is Eqs. 7-14 (standard) or Eqs. 24-29 (improved) with
 * Lambda = I/tau; its transpose runs the streaming backwards, applies the
 * transposed stencils (the Eq. 17 gradient is antisymmetric and the Laplacian
 * symmetric on a periodic lattice) and the local derivatives of the
 * equilibrium, forcing and correction terms.  Arithmetic is float64.
 *   state_t   raw state of time level t in this handle's storage format, as
 *             returned by lbm_get_state (device, lbm_state_bytes)
 *   lam_next  dL/df(t+1), device float64, layout of lbm_get_f ([9][N])
 *   lam_out   dL/df(t), same layout (must not alias lam_next)
 *   ws        device workspace of lbm_adjoint_workspace_bytes, caller-owned
 *   grad      device float64[2], incremented by dL/dkappa and dL/d(T/Tc)
 *             contributed by this step (fixed-order, deterministic sums)
 * lbm_adjoint_fields: dL/df(t) for given cotangents of the fields of Eq. 12,
 *   rho_bar [N] and u_bar [2][N] (either may be NULL = zero), plus the
 *   parameter terms through mu.
 * lbm_adjoint_init: dL/drho0 of the initialisation f = f_eq(rho0, u0 = 0) from
 *   lam0 = dL/df(0); grad_rho0 [N] is overwritten, grad incremented.
 * Returns LBM_ERR_UNSUPPORTED for D3Q19, batches, the pressure-tensor force,
 * the MRT collision or plates (lbm_adjoint_workspace_bytes then returns 0).
 */
size_t lbm_adjoint_workspace_bytes(const lbm_ctx* h);
int lbm_adjoint_step(lbm_ctx* h, const void* state_t, const double* lam_next, double* lam_out, void* ws,
                     double* grad);
int lbm_adjoint_fields(lbm_ctx* h, const void* state_t, const double* rho_bar, const double* u_bar,
                       double* lam_out, void* ws, double* grad);
/* lbm_adjoint_step_noalloc: lbm_adjoint_step for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and the same result, bit for bit, with
 * the workspace taken from a fixed array in each GPU's global memory instead of
 * the caller's `ws`.  The array holds lbm_adjoint_noalloc_max_bytes() bytes (24
 * MiB: D2Q9 lattices up to about 120 000 nodes, e.g. 256 x 256 or 345 x 345) on
 * every GPU the library runs on, until the process ends; a lattice whose
 * workspace (lbm_adjoint_workspace_bytes) is larger gets LBM_ERR_UNSUPPORTED.
 * The first call on a device resolves the array's address (hipGetSymbolAddress);
 * no call allocates.  Every call on one GPU uses the same array, and each call
 * overwrites what the previous one left there (nothing in it needs to start at
 * zero): calls that overlap in time on one GPU (two streams, two host threads)
 * race on it and must be serialised by the caller.  Arguments, errors and the
 * increment of grad as for lbm_adjoint_step. */
int lbm_adjoint_step_noalloc(lbm_ctx* h, const void* state_t, const double* lam_next, double* lam_out,
                             double* grad);
size_t lbm_adjoint_noalloc_max_bytes(void);

/* lbm_adjoint_segment: one checkpoint segment of a checkpointed backward pass.
 * Copies `checkpoint` (raw state of time level t0, lbm_get_state layout) into
 * the first of the m >= 1 slots of `states` (device, m * lbm_state_bytes,
 * caller-owned, overwritten), recomputes the states of time levels t0+1 ..
 * t0+m-1 into the next slots, then runs lbm_adjoint_step from t0+m-1 down to
 * t0.  checkpoint, states, lam and lam2 must be 16-byte aligned.  With graphs
 * on (lbm_set_use_graphs) the segment's launches are captured once per segment
 * length and buffer set and replayed.  On entry lam holds dL/df(t0+m), on
 * exit dL/df(t0) (layout of lbm_get_f); lam2 is device scratch of the same size
 * (must not alias lam); grad is incremented as by lbm_adjoint_step.  The handle is
 * left at time level t0 + m with no diagnostics.  Same support as the calls above. */
int lbm_adjoint_segment(lbm_ctx* h, const void* checkpoint, long long t0, int m, void* states, double* lam,
                        double* lam2, void* ws, double* grad);

/* lbm_adjoint_sweep: every segment of a checkpointed backward pass in one call,
 * the recomputation of a segment overlapped with the adjoint steps of the one
 * after it.  Segment i (0 <= i < nseg, nseg >= 1) starts from checkpoints[i], the
 * raw state of time level t0[i] (device pointer, lbm_get_state layout, 16-byte
 * aligned), and covers m[i] >= 1 steps; the segments must be consecutive
 * (t0[i+1] = t0[i] + m[i]).  checkpoints, t0 and m are host arrays of nseg
 * entries.  `states` (device, caller-owned, overwritten, 16-byte aligned) holds
 * two arenas of kmax = max m[i] slots: 2 * kmax * lbm_state_bytes.  From the last
 * segment to the first, each segment's states t0[i] .. t0[i]+m[i]-1 are recomputed
 * into arena i % 2 on a second stream of the library's own (default priority)
 * while the adjoint steps of segment i+1 run on the handle's stream over the
 * other arena; events order the two streams, and the second stream starts after
 * the work already queued on the handle's stream.  lam, lam2, ws and grad as in
 * lbm_adjoint_segment: on entry lam holds dL/df(t0[nseg-1] + m[nseg-1]), on exit
 * dL/df(t0[0]); the results equal those of lbm_adjoint_segment called for
 * i = nseg-1 .. 0 bit for bit.  When the call returns, all its work is queued on
 * the handle's stream (synchronising that stream covers the second one).  The
 * handle's own state and time level are not changed; blow-up flags are cleared.
 * Graphs (lbm_set_use_graphs) are captured per (kind, segment length, arena,
 * buffers) and replayed.  Same support as the calls above. */
int lbm_adjoint_sweep(lbm_ctx* h, const void* const* checkpoints, const long long* t0, const int* m, int nseg,
                      void* states, double* lam, double* lam2, void* ws, double* grad);
int lbm_adjoint_init(lbm_ctx* h, const double* rho0, const double* lam0, double* grad_rho0, void* ws,
                     double* grad);

/* Maxwell construction of the chosen EOS at T/T_c, on the host in float64: the
 * gas and liquid densities with equal bulk chemical potential (Eq. 2 without the
 * gradient term) and equal bulk pressure (Eq. 3), which are the analytical
 * coexistence densities of Sec. IV A and Table II and the uniform mu of Appendix
 * A.  Outputs are host pointers (none may be NULL).  Returns LBM_ERR_ARG for
 * non-positive constants or T/T_c, LBM_ERR_DOMAIN when there is no coexistence
 * (T/T_c >= 1). */
int lbm_maxwell(int eos, double a, double b, double R, double T_over_Tc,
                double* rho_g, double* rho_l, double* mu_sat, double* p_sat);

/* Critical temperature of the chosen EOS (host, float64). */
double lbm_critical_temperature(int eos, double a, double b, double R);

/* Kernel tuning: tile shape index and whether lbm_step replays HIP graphs
 * (1, default) or launches one kernel per step (0).  An index in
 * [0, lbm_num_tile_shapes) names the output tile of one work group, bx x by
 * nodes; for D3Q19 it also fixes the z-chunk bz each work group sweeps (the same
 * xy tile appears with several chunk lengths).  lbm_describe_tile_shape reports
 * (bx, by, bz); for D2Q9, bz > 0 is the number of nodes each thread owns (1 or
 * 2, rows by / bz apart; work groups of bx * by / bz threads), and bz = -2 marks
 * work groups of 2 * bx * by threads, one owning each node and the others taking
 * halo pulls and a share of the ring stages (shorter stages for lattices that fill
 * the chip with a single wave of work groups).  The 2048-node D2Q9
 * tile exists in float32 only; it and some D3Q19 float64 shapes return
 * LBM_ERR_UNSUPPORTED in float64 (LDS), and lbm_autotune skips them.  Re-tiling
 * synchronises the handle's stream. */
int lbm_set_tile_shape(lbm_ctx* h, int shape_index);
int lbm_get_tile_shape(const lbm_ctx* h);
int lbm_num_tile_shapes(const lbm_ctx* h);
int lbm_describe_tile_shape(const lbm_ctx* h, int shape_index, int* bx, int* by, int* bz);
int lbm_set_use_graphs(lbm_ctx* h, int on);

/* D3Q19 z-chunk length: bz = 0 (default) takes it from the tuning index (chunks
 * aimed at a work-group count); bz >= 16 fixes the number of z-slices each work
 * group sweeps for every tile shape (the last chunk of a lattice may be shorter).
 * D2Q9 handles accept only 0.  Re-plans like lbm_set_tile_shape (synchronises
 * the stream, drops captured graphs).  LBM_ERR_ARG for 0 < bz < 16.
 * lbm_get_zchunk returns the fixed length, 0 when automatic, -1 for a null handle. */
int lbm_set_zchunk(lbm_ctx* h, int bz);
int lbm_get_zchunk(const lbm_ctx* h);

/* How the step kernels store the new populations (Eq. 10's f*):
 *   LBM_STORES_STREAMING  non-temporal stores (default; the choice for lattices
 *                         streamed through HBM)
 *   LBM_STORES_DEVICE     device-scope stores, written through the L2 during the
 *                         kernel: nothing is left for the end-of-kernel
 *                         write-back, which pays when the state buffers stay
 *                         (mostly) in the last-level cache between steps (e.g.
 *                         D2Q9 512^2 float64, D3Q19 256 x 256 x 32 float32)
 * The results are identical.  A change drops the captured graphs.
 * lbm_get_store_mode returns the mode, -1 for a null handle. */
enum lbm_store_mode { LBM_STORES_STREAMING = 0, LBM_STORES_DEVICE = 1 };
int lbm_set_store_mode(lbm_ctx* h, int mode);
int lbm_get_store_mode(const lbm_ctx* h);

/* Pick the fastest tile shape and store mode by timing `steps` steps of
 * each pair, twice, on the current state (the state, the time level and the
 * blow-up flags are restored afterwards); returns the chosen shape index and
 * leaves both selected. */
int lbm_autotune(lbm_ctx* h, int steps, void* scratch_state);

/* Measurement helper: copy `bytes` from src to dst (device, 16-byte aligned,
 * not overlapping) on the stream `hip_stream` with a plain copy kernel, one
 * 16-byte vector per thread; the reference of known size for the traffic
 * counters and the streaming ceiling.  LBM_ERR_ARG for null or misaligned
 * pointers. */
int lbm_copy_kernel(void* dst, const void* src, size_t bytes, void* hip_stream);

const char* lbm_error_string(int code);
const char* lbm_last_error(void);
void lbm_destroy(lbm_ctx* h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
