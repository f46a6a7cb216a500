/*
 * rsl.h -- C ABI of librsl, an MI355X (gfx950) implementation of the time step
 * of the quadrature-based relativistic lattice Boltzmann method for massless
 * particles, R-SLB(N_Omega; Q_xi) (Ambrus & Blaga, arXiv:1612.01287).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: RSL_OK (0) or a negative RSL_E*
 *    code; rsl_last_error() then returns a thread-local message.  No C++
 *    exception crosses this boundary.
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors on ROCm).  The caller owns all device buffers and the HIP stream
 *    (hipStream_t passed as void*, NULL = legacy default stream).  Work is
 *    enqueued on that stream and the call returns without synchronising;
 *    argument validation is synchronous.
 *  - The library owns rsl_quad handles; they are immutable after creation and
 *    may be shared by calls on several streams of one device.
 *  - rsl_step never allocates device memory.
 *
 * Distribution layout in device memory (one instance):
 *    f[v * pitch + s],  v = k * Q_xi + j   (radial node k outer, angle node j
 *    inner, as the velocity grouping of App. B), s = cell index 0..nz-1,
 *    pitch = rsl_pitch(nz) >= nz elements; element type double (RSL_F64) or
 *    float (RSL_F32).  Ghost cells are not stored: they are generated from the
 *    boundary rule inside the kernels.  For Bjorken flow nz = 1.
 *  f_jk is the paper's scaled population  f_jk = 2 pi T0^3 e^{pbar_k}
 *  w_j w_k f(p_k, xi_j)  (Sec. III E, eq. fjk), so that moments are plain sums
 *  (eq. macro_jk).
 */
#ifndef RSL_H
#define RSL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define RSL_OK            0
#define RSL_EINVAL       (-1)  /* bad argument: sizes, states, null pointers          */
#define RSL_EUNSUPPORTED (-2)  /* outside the model family built here                 */
#define RSL_EUNSTABLE    (-3)  /* time step beyond the CFL or stiffness limit         */
#define RSL_EDEVICE      (-4)  /* a HIP runtime error (message has the HIP text)      */
#define RSL_ENONFINITE   (-5)  /* a cell reached an unphysical or non-finite state    */

/* ------------------------------------------------------------ enumerations */
#define RSL_SOD        0   /* 1D shock tube, Sec. IV, operator eq. L_Sod            */
#define RSL_BJORKEN    1   /* 0+1D Bjorken flow, Sec. V, operator eq. L_Bjorken     */

#define RSL_TAU_CONST  0   /* tau_AW = tau_r in every cell                          */
#define RSL_TAU_ETAS   1   /* constant eta/s: tau_AW = tau_AW0 / T * (1 - ln(lambda_bar lambda_ref)/4)
                              (eq. Sod:tau); Bjorken ideal gas eq. bjorken_tauAW_mu;
                              parton gas tau_AW = tau_AW0 / T                     */
#define RSL_TAU_INF    2   /* collisionless (ballistic) limit                       */

#define RSL_GAS_IDEAL  0   /* P = n T, n conserved                                  */
#define RSL_GAS_PARTON 1   /* mu = 0: T = P^{1/4}, n_eq = T^3 (Sec. V D); Bjorken only */

#define RSL_BC_EQ      0   /* 3 ghost cells per side fixed to f^eq of the initial
                              left / right states (Sec. IV A)                      */
#define RSL_BC_OUTFLOW 1   /* zero-gradient: ghosts copy the first / last cell      */

#define RSL_F64        0   /* f stored in binary64                                  */
#define RSL_F32        1   /* f stored in binary32; all per-cell work (moments,
                              Landau frame, tau, f^eq coefficients) stays binary64 */

#define RSL_FLAG_FORCE_UNSTABLE 1  /* rsl_step: skip the stiffness guard          */
#define RSL_FLAG_IMEX           2  /* rsl_batch_create: the instance is stepped   */
                                   /* implicit-explicit (CFL bound only); the     */
                                   /* batch then refuses the explicit steps       */
#define RSL_QUAD_HOST_ONLY      1  /* rsl_make_quadrature: build host tables only  */

/* Fields of rsl_moments output, per cell, in this order. */
#define RSL_NMOM 13
/* N^0, N^z, T^00, T^0z, T^zz  (eq. macro_jk)
 * n, E, P, T, beta            (Landau frame, eqs. E_landau, u_landau; P = E/3, T = P/n)
 * lambda_bar = n / T^3        (relative fugacity)
 * q  = -4 T (N^z - n beta gamma)        (eq. q_val)
 * Pi = 2E/3 - T^00 + T^zz               (eq. pi_val)
 * For Bjorken flow (u = (1,0,0,0)): N^z = T^0z = 0 slots hold 0, T^zz holds
 * P_L = T^{eta eta}, Pi = P_L - P, q = 0. */

typedef struct rsl_quad rsl_quad;

/* Problem description (Sod: Sec. IV A; Bjorken: Sec. V A).  Plain data. */
typedef struct rsl_problem {
    int problem;      /* RSL_SOD | RSL_BJORKEN                                      */
    int nz;           /* cells; Sod: >= 5; Bjorken: must be 1                       */
    int dtype;        /* RSL_F64 | RSL_F32                                          */
    int bc;           /* RSL_BC_EQ | RSL_BC_OUTFLOW (Sod)                           */
    int tau_mode;     /* RSL_TAU_*                                                  */
    int gas;          /* RSL_GAS_* (Bjorken; Sod is always ideal)                   */
    int flags;        /* RSL_FLAG_*                                                 */
    int reserved;
    double z_lo, z_hi;        /* Sod domain, cell centres z_s = z_lo + (s + 1/2) dz    */
    double n_L, T_L;          /* Sod left state at rest; Bjorken initial state at tau0 */
    double n_R, T_R;          /* Sod right state at rest                               */
    double tau_r;             /* RSL_TAU_CONST relaxation time                          */
    double tau_aw0;           /* RSL_TAU_ETAS: tau_{A-W;0}                              */
    double lambda_ref;        /* RSL_TAU_ETAS: lambda_ref (1 in the paper's setups)     */
    double kappa;             /* stiffness guard: dt gamma (1 + |beta|) / tau_AW <= kappa
                                 at the states of the inviscid Riemann solution (the
                                 initial states and the two plateaus, Sec. IV B 1);
                                 0 -> 2.0 (RK3 is stable on the real axis to 2.51)  */
} rsl_problem;

/* Build the velocity set R-SLB(N_Omega; Q_xi) with Q_L radial nodes
 * (Sec. III E): Gauss-Legendre nodes/weights in xi = cos(theta) (eq. quad_xi),
 * generalised Gauss-Laguerre (alpha = 2) radial nodes p_k = T0 pbar_k and
 * weights (eq. wL, Table I), Legendre tables P_m(xi_j), the momentum-space
 * kernels K^L (eq. K_lag_disc) and K^P (eq. K_leg_disc), and the tables the
 * kernels use for the equilibrium coefficients (Sec. III D, eq. feq_trunc).
 * Tables are built in host extended precision and uploaded to the current
 * HIP device unless flags has RSL_QUAD_HOST_ONLY.
 * Limits: 2 <= Q_L <= 8, N_L = 1, 0 <= N_Omega <= 6, N_Omega < Q_xi <= 1024,
 * T0 > 0.  Errors: RSL_EINVAL, RSL_EUNSUPPORTED (N_L != 1, N_Omega > 6),
 * RSL_EDEVICE.  *out is NULL on error. */
int rsl_make_quadrature(int Q_L, int Q_xi, int N_L, int N_Omega, double T0, int flags,
                        rsl_quad** out);
void rsl_free_quadrature(rsl_quad* q);

/* Host copies of the tables, for inspection.  which: */
#define RSL_TAB_XI   0   /* xi_j,      Q_xi values, ascending                         */
#define RSL_TAB_WXI  1   /* w_j,       Q_xi values                                    */
#define RSL_TAB_PBAR 2   /* pbar_k,    Q_L values, ascending                          */
#define RSL_TAB_WL   3   /* w_k,       Q_L values                                     */
#define RSL_TAB_KL   4   /* K^L_{k,k'}, Q_L x Q_L row-major                           */
#define RSL_TAB_KP   5   /* K^P_{j,j'}, Q_xi x Q_xi row-major                          */
/* Copies up to n doubles; *count (if not NULL) receives the table length. */
int rsl_quad_table(const rsl_quad* q, int which, double* host_out, int n, int* count);

/* Elements per velocity plane for nz cells (multiple of 64, >= nz). */
int rsl_pitch(int nz);

/* Limits of the time step that rsl_step's guards apply (host only, no device
 * work; q may be RSL_QUAD_HOST_ONLY): dt must be < *cfl_dt (dt max|xi|/dz < 1,
 * Sec. III F) and <= *stiff_dt (kappa over the largest relaxation rate
 * gamma (1 + |beta|) / tau_AW at the states of the inviscid Riemann solution,
 * Sec. IV B 1; eq. L_Sod).  HUGE_VAL where no bound applies (no advection in
 * Bjorken flow, tau = infinity).  RSL_EINVAL for NULL pointers or a bad problem. */
int rsl_max_dt(const rsl_quad* q, const rsl_problem* p, double* cfl_dt, double* stiff_dt);

/* Sizes of the caller-owned buffers for one instance: f (the state) and work
 * (two RK stage copies of f, the boundary states and a status word). */
int rsl_sizes(const rsl_quad* q, const rsl_problem* p, size_t* f_bytes, size_t* work_bytes);

/* Initial state.  Sod: f = f^eq(n_L, T_L, u = 0) for z_s < centre and
 * f^eq(n_R, T_R, 0) beyond, the cell centred on the membrane (odd nz) taking
 * the mean (Sec. IV A); the f^eq used is the truncated expansion at the nodes.
 * Bjorken: f = f^eq(n_L, T_L, 0) (eq. bjorken_f0 with n_L = T_L = 1).
 * Also clears the status word in work. */
int rsl_init(const rsl_quad* q, const rsl_problem* p, void* f_dev, void* work_dev,
             void* hip_stream);

/* Advance f by nsteps steps of the TVD RK3 scheme (eq. rk3, stage times of
 * Table II) applied to L_Sod (eq. L_Sod: WENO5 advection, Sec. III F, plus the
 * Anderson-Witting term) or L_Bjorken (eq. L_Bjorken).  *t (host) is the
 * time (Sod) or proper time tau (Bjorken) and advances by nsteps*dt.
 * Errors: RSL_EINVAL; RSL_EUNSTABLE if dt*max|xi|/dz >= 1 (CFL, eq. CFL) or
 * dt gamma (1 + |beta|) / tau_AW > kappa at a state of the inviscid Riemann
 * solution (see rsl_problem.kappa), unless RSL_FLAG_FORCE_UNSTABLE.
 * Unphysical cell states are reported by the next rsl_moments / rsl_status. */
int rsl_step(const rsl_quad* q, const rsl_problem* p, void* f_dev, void* work_dev,
             double* t, double dt, int nsteps, void* hip_stream);

/* Advance a Sod instance by nsteps implicit-explicit steps, for time steps
 * not bound by the relaxation time (Sec. I names the option; Sec. III F):
 * the WENO5 advection explicit and the Anderson-Witting term implicit in the
 * IMEX-SSP2(2,2,2) scheme (second order, L-stable implicit part;
 * g = 1 - 1/sqrt(2)):
 *   F1 = f + g dt Q(F1),  F2 = f + dt A(F1) + (1 - 2g) dt Q(F1) + g dt Q(F2),
 *   f' = f + dt/2 (A(F1) + A(F2)) + dt/2 (Q(F1) + Q(F2)).
 * Each implicit stage is solved per cell: the collision keeps N^0, T^00,
 * T^0z, and Broyden's method finds the N^z, T^zz whose Landau frame, tau
 * and f^eq reproduce them (its Jacobian from finite differences in the first
 * stage of a call, then carried per cell from stage to stage in the work
 * buffer's per-cell rows).  Binary64 or
 * binary32 storage (f and the stages stored in the instance's dtype; the
 * arithmetic in binary64 except the WENO5 stencil of binary32 storage, which
 * takes binary32 weights as rsl_step does).  Uses the work buffer of rsl_sizes after rsl_init
 * (the two stage slots, the ghost states, the status word).  Only the CFL
 * bound applies (RSL_EUNSTABLE if dt max|xi| / dz >= 1); no stiffness guard.
 * A cell whose stage has no Landau frame or does not converge gets NaN and
 * sets the status word (rsl_status).  Errors: RSL_EINVAL, RSL_EUNSUPPORTED
 * (Bjorken), RSL_EUNSTABLE. */
int rsl_step_imex(const rsl_quad* q, const rsl_problem* p, void* f_dev, void* work_dev, double* t, double dt,
                  int nsteps, void* hip_stream);

/* Per-cell fields written to out_dev on the stream, cell-major:
 * out[s*fields + field], in the order listed at RSL_NMOM.  fields is
 * RSL_MOM_RAW5 (the five moments of eq. macro_jk) or RSL_MOM_ALL (those and the
 * derived fields; the derived ones are NaN in a cell whose Landau frame does
 * not exist, which also sets the status word).  Bjorken writes one row.
 * Stream-ordered and asynchronous like rsl_step (so it can be captured in a
 * graph); an unphysical or non-finite state met by earlier calls is reported
 * by rsl_status, which synchronises.  RSL_EINVAL for other fields values. */
#define RSL_MOM_RAW5  5
#define RSL_MOM_ALL   13   /* = RSL_NMOM */
int rsl_moments(const rsl_quad* q, const rsl_problem* p, const void* f_dev, void* work_dev,
                double* out_dev, int fields, void* hip_stream);

/* Synchronises the stream and reads the status word: RSL_OK, or
 * RSL_ENONFINITE if any kernel since rsl_init met an unphysical state. */
int rsl_status(const rsl_quad* q, const rsl_problem* p, void* work_dev, void* hip_stream);

const char* rsl_last_error(void);

/* ---------------------------------------------------------------- batches
 * Many instances of one problem kind and one dtype, of uneven nz, velocity
 * set and relaxation law, advanced together.  Sod batches sort their
 * instances into velocity classes (see the stage-kernel variants below); per
 * RK stage each class runs one launch (fused form) or two (two-kernel form)
 * over all its instances (work items = (instance, tile), ordered per XCD,
 * costliest first), each class on a stream of its own forked from and joined
 * back into the caller's stream once per call.  Bjorken batches run one
 * launch per call (one workgroup per instance or per group of 16 instances
 * with one velocity set, all steps inside).  Each instance has its own time
 * step dt[i].  The batch copies the problem structs and keeps pointers to the
 * quads, which must outlive it.  Device memory of the batch (descriptor and
 * work-item tables) is allocated at creation; stepping allocates nothing and
 * may be captured into a HIP graph.
 * Buffers: one f buffer and one work buffer for the whole batch
 * (rsl_batch_sizes); instance i's f starts rsl_batch_offset(i) bytes into f,
 * with the single-instance layout.  rsl_batch_create applies rsl_step's CFL
 * and stiffness guards to every (problem, dt[i]) and fails with
 * RSL_EUNSTABLE when one of them fails (rsl_last_error names the instance). */
typedef struct rsl_batch rsl_batch;
int rsl_batch_create(const rsl_quad* const* quads, const rsl_problem* problems, const double* dt, int n,
                     rsl_batch** out);
void rsl_batch_free(rsl_batch* b);
int rsl_batch_sizes(const rsl_batch* b, size_t* f_bytes, size_t* work_bytes);
int rsl_batch_offset(const rsl_batch* b, int i, size_t* f_offset);
/* Host-side time of instance i (advanced by rsl_batch_step). */
int rsl_batch_time(const rsl_batch* b, int i, double* t);
int rsl_batch_init(rsl_batch* b, void* f_dev, void* work_dev, void* hip_stream);
/* nsteps RK3 steps of every instance (eq. rk3 with L_Sod or L_Bjorken). */
int rsl_batch_step(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream);
/* The same nsteps steps replayed from a HIP graph: captured on the first call
 * (and again whenever f_dev, work_dev, nsteps or the stream change), then
 * launched with one hipGraphLaunch per call.  Needs an explicit stream; the
 * graph holds kernel launches and event waits only.  Results are bitwise
 * those of rsl_batch_step. */
int rsl_batch_graph_step(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream);
/* nsteps implicit-explicit steps (as rsl_step_imex) of every instance of a Sod
 * batch, each with its own dt: per step four launches over the batch (two
 * implicit stages, each one launch per class of velocity-set size, and two
 * explicit passes).  Instances created with RSL_FLAG_IMEX were checked
 * against the CFL bound only; such a batch refuses rsl_batch_step,
 * rsl_batch_graph_step, rsl_batch_stage and rsl_batch_autotune
 * (RSL_EUNSTABLE).  Builds its work-item lists (device memory owned by the
 * batch, freed by rsl_batch_free) on the first call with nsteps > 0, so make
 * that call outside HIP graph capture; later calls allocate nothing.
 * Errors: RSL_EINVAL, RSL_EUNSUPPORTED (Bjorken), RSL_EUNSTABLE (CFL). */
int rsl_batch_step_imex(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream);
/* One RK3 stage (1, 2 or 3) of every Sod instance, without advancing the
 * host-side times: stage s reads f_n and the stage field s-1 and writes stage
 * field s (stage 3 writes f_{n+1} over f_n).  For custom drivers and timing. */
int rsl_batch_stage(rsl_batch* b, void* f_dev, void* work_dev, int stage, void* hip_stream);
/* Per-cell fields of every instance, rows concatenated in instance order
 * (nz rows per Sod instance, one per Bjorken instance), `fields` per row
 * (RSL_MOM_RAW5 or RSL_MOM_ALL, as for rsl_moments). */
int rsl_batch_moments(rsl_batch* b, const void* f_dev, void* work_dev, double* out_dev, int fields,
                      void* hip_stream);
/* Kernel path of a Bjorken batch: -1 automatic (matrix cores when every
 * instance fits: Q_L <= 4 and a padded Q_xi x 16 Q_L stage field within the
 * LDS), 0 one workgroup per instance on the vector units, 1 matrix cores
 * (RSL_EUNSUPPORTED if not available).  The two paths agree to rounding. */
int rsl_batch_set_path(rsl_batch* b, int path);
/* Matrix-core groups of a Bjorken batch, in launch order: *ngroups receives
 * their number (0 when the batch has no matrix-core path) and, when sizes is
 * not NULL, sizes[g] for g < min(*ngroups, cap) the number of instances in
 * group g (1..16, all sharing one velocity set).  Groups are sized so that
 * their estimated costs balance over the GPU's compute units: a group of fewer
 * instances fills fewer 16-column tiles of the K^P F product (eq. K_leg_disc)
 * and finishes sooner.  RSL_EINVAL for a NULL batch or ngroups, or cap < 0. */
int rsl_batch_groups(const rsl_batch* b, int* ngroups, int* sizes, int cap);
/* Stage-kernel variants.  One Sod RK3 stage (Sec. III F-G: moments, Landau
 * frame, f^eq, AW relaxation, WENO5 fluxes, RK combination) runs in one of
 * three forms (*form): 0, one fused kernel per tile of cells; 1, a two-kernel
 * form (a per-cell kernel for the moments and equilibrium coefficients, then
 * a kernel per (cell, velocity slice) for fluxes, relaxation and the RK
 * combination); 2, a loop form for batches (one workgroup per tile walks
 * all velocities and, from the output it writes, computes the next stage's
 * coefficients; the per-cell kernel runs only before the first stage of a
 * call).  The
 * fused kernel has launch shapes of W waves per workgroup, NV velocities per
 * lane and 64/TW velocity slots per wave of TW lanes (tiles of TW - 1 cells)
 * and covers V <= W (64/TW) NV; the other two take any V (up to 65536) with W
 * waves of NV velocities at a time, and cell_waves waves per 64 cells in the
 * per-cell kernel.  Variants differ only in the order of the per-cell moment
 * sums, so results agree to rounding.
 * rsl_stage_variant returns the shape of variant id var, *max_v its largest
 * V, *cell_waves the per-cell kernel's waves (0 for the fused kernel) and
 * *form its form (each pointer may be NULL); RSL_EINVAL past the last id.
 * A Sod batch sorts its instances into seven classes by V (V <= 32, 64, 128,
 * 256, 320, 384 and V > 384), each launched on a stream of its own;
 * rsl_batch_variant reports a class's variant (-1 if the class is empty) and
 * its largest V; rsl_batch_set_variant selects one (var < 0: the default;
 * RSL_EINVAL if it holds fewer than the class's largest V).  Class index 7
 * stands for every instance at once: setting a variant there runs the whole
 * batch as one class (one launch per kernel and stage, on the caller's
 * stream), var < 0 returns to the seven classes; rsl_batch_variant(b, 7)
 * reports -1 unless the batch runs that way.
 * rsl_batch_autotune times every variant that fits each class on stage 2 as
 * it runs inside a multi-step call (reps launches each, after one stage-1
 * launch), keeps the fastest per class and writes the ids to chosen[7] (if not
 * NULL; -1 for empty classes); it then times 2 reps whole steps of the
 * batch (graph-replayed when hip_stream is not the default stream) with those
 * classes on their streams against the whole batch as one class in every
 * variant that fits, and keeps the fastest (rsl_batch_variant(b, 7) tells
 * which).  For those steps it saves f to a temporary device copy (allocated
 * and freed here) and restores it after: f is left unchanged, the work
 * buffer's contents are overwritten, the instances' times do not advance.
 * It synchronises the stream.  Changing a variant drops the captured graph. */
int rsl_stage_variant(int var, int* waves, int* vel_per_slot, int* lanes_per_vel, int* max_v, int* cell_waves,
                      int* form);
int rsl_batch_variant(const rsl_batch* b, int cls, int* var, int* max_v);
int rsl_batch_set_variant(rsl_batch* b, int cls, int var);
int rsl_batch_autotune(rsl_batch* b, void* f_dev, void* work_dev, int reps, void* hip_stream, int* chosen);
/* Synchronises and reads every instance's status word; *first_bad (if not
 * NULL) receives the first failing instance or -1. */
int rsl_batch_status(rsl_batch* b, void* work_dev, void* hip_stream, int* first_bad);
/* Synchronises and writes every instance's status to status[0..n-1]
 * (RSL_OK or RSL_ENONFINITE), so that a failing instance can be told from the
 * others of its launch group.  RSL_EINVAL for NULL arguments, RSL_EDEVICE on
 * a HIP error. */
int rsl_batch_instance_status(rsl_batch* b, void* work_dev, void* hip_stream, int* status);

/* ------------------------------------------------------------ diagnostics
 * Reductions of per-cell (or per-sample) field rows on the device, one
 * workgroup in a fixed summation order; results are written to out_dev on
 * the stream (asynchronous).  RSL_EINVAL for NULL pointers or bad sizes. */

/* out_dev[c] = dz * sum_{r = row_lo}^{row_hi - 1} m_dev[r * ncols + c] for
 * c < ncols: the integral over a window of cells (midpoint rule).  With
 * rsl_moments rows (ncols = RSL_MOM_ALL) columns 11 and 12 give the integrated
 * heat flux q and shear pressure Pi around a discontinuity (Sec. IV B 3,
 * eqs. intq, intpi). */
int rsl_window_integral(const double* m_dev, int nrows, int ncols, double dz, int row_lo, int row_hi, double* out_dev,
                        void* hip_stream);
/* Error measure of the Sod convergence test (Sec. IV E, eq. eps_def) between
 * two RSL_MOM_ALL moment tables of nz cells on the same grid:
 * eps_j = max_z |d_j - d_j,ref| / (max_z d_j - min_z d_j) for d_j = n, T, gamma;
 * out_dev = {eps_n, eps_T, eps_gamma, max_j eps_j}. */
int rsl_sod_eps(const double* m_dev, const double* ref_dev, int nz, double* out_dev, void* hip_stream);
/* L2 norm of the Bjorken convergence test (Sec. V E, eq. bjork_L2) between two
 * histories of RSL_MOM_ALL rows sampled at tau = 1 + i dtau, i < nsamples:
 * L2(A) = sqrt(int dtau' (A - A_ref)^2 / (tau_f - 1)) by the trapezoid rule,
 * tau_f = 1 + (nsamples - 1) dtau, for A = n, T, P, Pi;
 * out_dev = {L2(n), L2(T), L2(P), L2(Pi), max_A L2(A)}. */
int rsl_bjorken_l2(const double* hist_dev, const double* ref_dev, int nsamples, double dtau, double* out_dev,
                   void* hip_stream);

/* ------------------------------------------------ learned T^{mu nu} correction
 * Not part of the paper: a per-cell network that maps the local moments of a
 * low-order velocity set to the difference between a high-order and the
 * low-order T^{00}, T^{0z}, T^{zz}.  Features of cell s: M_{a,r} =
 * sum_jk f_jk p_k^a xi_j^r (a in {0,1}, r in 0..7; eq. macro_jk extended to
 * r <= 7) of cells s-2..s+2 (end cells repeated), the a = 0 ones divided by the
 * centre's N^0, the a = 1 ones by its T^00, then log tau_r: 81 floats.
 * Network: 81 -> 128 -> 128 -> 3, ReLU, parameters W1 [81][128], b1, W2
 * [128][128], b2, W3 [128][3], b3 (27395 values) in an fp32 master copy and a
 * bf16 compute copy; matrix products in bf16 with fp32 accumulation.
 * Output y = (T_hi - T_lo) / T^00_lo for (T^00, T^0z, T^zz). */
#define RSL_MLP_IN      81
#define RSL_MLP_HIDDEN  128
#define RSL_MLP_OUT     3
#define RSL_MLP_NPARAM  27395

/* feat_dev[nz][81] (fp32) from one Sod instance's f.  With shift_dev and
 * scale_dev (device [81], both or neither) each feature x is stored as
 * (x - shift) / scale in fp32 (the standardisation a trained network expects). */
int rsl_mlp_features(const rsl_quad* q, const rsl_problem* p, const void* f_dev, double log_tau,
                     const float* shift_dev, const float* scale_dev, float* feat_dev, void* hip_stream);
/* bf16 (round to nearest even) copy of fp32 parameters. */
int rsl_mlp_to_bf16(const float* params, unsigned short* params_bf16, void* hip_stream);
/* y[n][3] = net(x[n][81]).  h1, h2 ([n][128] bf16 each) receive the hidden
 * activations for rsl_mlp_backward, or are both NULL. */
int rsl_mlp_forward(const unsigned short* params_bf16, const float* x, int n, float* y, unsigned short* h1,
                    unsigned short* h2, void* hip_stream);
/* grad[27395] = d/dparams of mean((y - t)^2) over the n x 3 outputs, from the
 * activations of the matching forward call (grad is overwritten).  work is a
 * device buffer of rsl_mlp_backward_work(n) floats owned by the caller
 * (partial gradients of up to 256 workgroups, added in a fixed order, so the
 * result does not depend on scheduling); calls that share it must not
 * overlap.  RSL_EINVAL for NULL pointers or n <= 0. */
size_t rsl_mlp_backward_work(int n);
int rsl_mlp_backward(const unsigned short* params_bf16, const float* x, const unsigned short* h1,
                     const unsigned short* h2, const float* y, const float* t, int n, float* grad, float* work,
                     void* hip_stream);
/* rsl_mlp_backward without the caller's workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc).  The partial gradients go to a
 * scratch array inside the library: 256 x 27395 floats (28 MB) per device,
 * enough for any n, held until the process ends.  Allocates nothing (the
 * array's device address is looked up once per device, at the first call).
 * Results are bitwise those of rsl_mlp_backward.  Calls on one device share
 * the array: calls that overlap on one GPU (several streams, threads) race,
 * so serialise them.  RSL_EINVAL for NULL pointers or n <= 0. */
int rsl_mlp_backward_noalloc(const unsigned short* params_bf16, const float* x, const unsigned short* h1,
                             const unsigned short* h2, const float* y, const float* t, int n, float* grad,
                             void* hip_stream);
/* One Adam step (step >= 1, bias-corrected) on the fp32 parameters; refreshes
 * the bf16 copy. */
int rsl_mlp_adam(float* params, const float* grad, float* m, float* v, unsigned short* params_bf16, int step, float lr,
                 float beta1, float beta2, float eps, void* hip_stream);
/* Moment rows m_lo, m_hi: RSL_NMOM doubles per cell (rsl_moments output).
 * mode 0: t_out[n][3] = (T_hi - T_lo) / T^00_lo (training targets);
 * mode 1: t_corr[n][3] = T_lo + y T^00_lo (corrected T^00, T^0z, T^zz). */
int rsl_mlp_tmunu(const double* m_lo, const double* m_hi, const float* y, int n, int mode, float* t_out,
                  double* t_corr, void* hip_stream);
/* In-loop feedback of the correction: adds to every cell s of one Sod
 * instance's f the population change
 *   df_jk = w_j w_k L_1^(2)(pbar_k) (a0 + a1 xi_j + a2 xi_j^2),
 * which leaves N^0 and N^z unchanged (the Laguerre rule gives
 * sum_k w_k L_1(pbar_k) = 0) and moves (T^00, T^0z, T^zz) by y[s][0..2] times
 * the cell's T^00 (the network's output convention); (a0, a1, a2) solve the
 * three moment equations.  In place, stream-ordered.  RSL_EINVAL for NULL
 * pointers or a non-Sod problem; RSL_EUNSUPPORTED when Q_xi < 3 (the three
 * moment equations are then singular). */
int rsl_mlp_inject(const rsl_quad* q, const rsl_problem* p, void* f_dev, const float* y, void* hip_stream);
/* Projection of a high-order Sod state onto a low-order velocity set over the
 * same cells: f_lo = the low-order equilibrium (eq. feq_trunc) of f_hi's
 * Landau frame (eqs. E_landau, u_landau), plus the change along the basis
 * above and along w_j w_k (4 - pbar_k) xi_j^c (c = 0, 1; no T^{mu nu}) that
 * gives f_lo the N^0, N^z, T^00, T^0z, T^zz of f_hi.  A cell without a
 * Landau frame gets NaN populations.  Either dtype on either side.
 * Stream-ordered.  RSL_EINVAL for NULL pointers, non-Sod problems or
 * different nz; RSL_EUNSUPPORTED as rsl_mlp_inject for q_lo. */
int rsl_project(const rsl_quad* q_hi, const rsl_problem* p_hi, const void* f_hi, const rsl_quad* q_lo,
                const rsl_problem* p_lo, void* f_lo, void* hip_stream);
/* Sets *flag_dev (atomic OR 1) if any feature lies outside [lo[c], hi[c]]
 * (the range seen in training): the caller then falls back to the high-order
 * solve. */
int rsl_mlp_guard(const float* x, int n, const float* lo, const float* hi, unsigned* flag_dev, void* hip_stream);

/* ------------------------------------------- velocity sets with azimuthal nodes
 * For flows whose velocity is not along z (Sec. III D: the addition theorem
 * of eq. leg_product and the azimuthal quadrature).  The set adds Q_phi
 * equally spaced azimuths phi_l = 2 pi l / Q_phi with weights 2 pi / Q_phi to
 * the Q_L radial and Q_xi polar nodes of rsl_make_quadrature; node
 * v = (k Q_phi + l) Q_xi + j, direction Omega_v = (sin theta_j cos phi_l,
 * sin theta_j sin phi_l, xi_j), momentum p_k = T0 pbar_k.  The equal-weight
 * rule integrates trigonometric polynomials of degree below Q_phi exactly, so
 * with Q_phi >= N_Omega + 3 the moments N^mu, T^{mu nu} of the truncated
 * equilibrium are exact (the addition theorem makes P_m(cos gamma_u) a
 * trigonometric polynomial of degree m in phi).  Q_phi = 1 is the aligned
 * set of the paper (eq. pjk).  Tables live on the current HIP device. */
typedef struct rsl_quad3 rsl_quad3;
/* Limits: those of rsl_make_quadrature (N_L = 1) and 1 <= Q_phi <= 256.
 * Errors: RSL_EINVAL, RSL_EUNSUPPORTED, RSL_EDEVICE; *out is NULL on error. */
int rsl_make_quadrature3(int Q_L, int Q_xi, int Q_phi, int N_Omega, double T0, rsl_quad3** out);
void rsl_free_quadrature3(rsl_quad3* q);
/* Number of nodes V = Q_L Q_xi Q_phi, or RSL_EINVAL for a NULL set. */
int rsl_quad3_velocities(const rsl_quad3* q);

/* Discrete equilibrium of the truncated expansion (eq. feq_trunc, N_L = 1)
 * for ncell cells at state_dev[c][5] = (n, T, u^x, u^y, u^z), u the spatial
 * part of the four-velocity (gamma v), mapped by eq. fjk with the azimuthal
 * weight 2 pi / Q_phi:
 *   f_v = (w_j w_k / Q_phi) sum_m P_m(Omega_v . u_hat) (c0_m + L_1(pbar_k) c1_m)
 * with the coefficients of the aligned flow at |u|.  Output f_dev[v][pitch]
 * (binary64 or binary32 per dtype; cells c < ncell written, the rest of each
 * row untouched).  Stream-ordered, asynchronous.  Errors: RSL_EINVAL (NULL
 * buffers with ncell > 0, pitch < ncell, bad dtype, another device),
 * RSL_EDEVICE.  ncell = 0 does nothing. */
int rsl_feq3(const rsl_quad3* q, const double* state_dev, int ncell, int dtype, void* f_dev, int pitch,
             void* hip_stream);

/* Moments of f_dev[v][pitch] (eq. macro_jk over the set's nodes) and the
 * Landau frame of T^{mu nu} (Sec. II E: T^{mu nu} u_nu = E u^mu, the timelike
 * eigenvector; n = u_mu N^mu, P = E / 3, T = P / n).  Output
 * out_dev[c][RSL_NMOM3] in the order below; the derived fields are NaN for a
 * cell whose T^{mu nu} has no timelike eigenvector with E > 0 and n > 0.
 * Stream-ordered, asynchronous.  Errors as rsl_feq3. */
#define RSL_NMOM3 22   /* N^0..N^3, T^00 T^01 T^02 T^03 T^11 T^12 T^13 T^22 T^23 T^33,
                          n, E, P, T, u^0, u^1, u^2, u^3 */
int rsl_moments3(const rsl_quad3* q, const void* f_dev, int dtype, int ncell, int pitch, double* out_dev,
                 void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* RSL_H */
