// Internal definitions shared by the host side and the kernels of librsl.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rsl.h"

namespace rsl {

// Stage-3 weights of the TVD RK3 scheme (eq. rk3), as products instead of divisions.
constexpr double kThird = 1.0 / 3.0;
constexpr double kTwoThirds = 2.0 / 3.0;
// Largest N_Omega with equilibrium coefficients (App. A gives m <= 6).
constexpr int kMaxNOm = 6;
// Terms kept in the Maclaurin tables of K_{3,m}, K_{4,m} (see rsl_math.h):
// enough for |beta| up to the largest series switch, 0.7 (67 terms carry every
// (k, m) series there to 2^-58; build_quadrature checks it).
constexpr int kSeriesTerms = 72;
// Doubles per velocity record (QuadDev::vrec): 4 + kMaxNOm + 1 used, padded to 16.
constexpr int kVrec = 16;
// slots of the per-velocity record past P_0..P_kMaxNOm (entries 4..10)
constexpr int kVrecXi2 = 11;   // xi_j^2
constexpr int kVrecXi6 = 12;   // xi_j / 6 (WENO5 candidates are formed six times larger)
constexpr int kVrecF32 = 13;   // 16 bytes: binary32 xi_j, xi_j / 6, p_k, then int sign(xi_j)
static_assert(4 + kMaxNOm < kVrecXi2 && kVrecF32 + 2 <= kVrec, "velocity record layout");
// Cells per wavefront tile: 64 lanes carry 64 interface fluxes, 63 cells are updated.
constexpr int kLanes = 64;
constexpr int kTileCells = kLanes - 1;
// Cells per tile of the per-cell kernel (no stencil there: one lane per cell).
constexpr int kCellTile = kLanes;
// LDS window per velocity plane: cells z0-3 .. z0+65 (69 values), padded.
constexpr int kWin = 72;

// Device-side tables of one velocity set.  All pointers are device memory
// owned by the rsl_quad that carries this struct.
struct QuadDev {
    const double* xi;    // [Q]      Gauss-Legendre nodes
    const double* wxw;   // [V]      w_j * w_k, v = k*Q + j
    const double* pk;    // [QL]     p_k = T0 * pbar_k
    const double* L1;    // [QL]     L_1^(2)(pbar_k) = 3 - pbar_k
    const double* Pm;    // [(NOm+1)*Q]  P_m(xi_j), row m
    const double* ser;   // [kSeriesTerms][2][kMaxNOm+1]  Maclaurin coefficients of K_{3,m}, K_{4,m}
    const double* thr;   // [kSeriesTerms]  beta^2 below which i terms suffice
    const double* KL;    // [QL*QL]
    const double* KP;    // [Q*Q]
    // per-velocity copies, v = k*Q + j, read with uniform (scalar) loads
    const double* xv;    // [V]      xi_j
    const double* pv;    // [V]      p_k
    const double* l1v;   // [V]      L_1(pbar_k)
    const double* Pv;    // [(NOm+1)*V]  P_m(xi_j), row m
    const int* vperm;    // [V] velocities ordered by the sign of xi (negative, zero, positive):
                         // the 32-lane stage kernels pair vperm[2p], vperm[2p+1]
    const double* vrec;  // [V][kVrec] per-velocity record: xi_j, p_k, L_1(pbar_k), w_j w_k, P_0..P_6(xi_j)
    const double* KPt;   // K^P zero-padded to Qp = 16 ceil(Q/16), in MFMA A-operand order:
                         // [rt][kk][lane] = K^P[16 rt + lane % 16][4 kk + lane / 16]
};

// Velocity sets with azimuthal nodes (vel3d.hip): device tables of one set.
struct Quad3Dev {
    const double* arec;   // [A][4]  Omega_x, Omega_y, Omega_z, w_j / Q_phi of angular node a = l Q_xi + j
    const double* rrec;   // [QL][4] p_k, w_k, L_1(pbar_k), 0
    const double* ser;    // the base set's Maclaurin tables
    const double* thr;
    int A, QL, NOm;
    double T0, beta_series;
};

// Everything a kernel needs about one problem instance.  Passed by value as a
// kernel argument for single-instance calls and stored in device arrays by
// the batched path.
struct InstDesc {
    int nz, pitch, Q, QL, V, NOm, bc, tau_mode;
    int gas, dtype, pad0, pad1;
    double dz_inv, dt, tau_r, tau_aw0, lambda_ref, T0, beta_series;
    double z_lo, dz;
    QuadDev tab;
    void* f;             // state  f_n       [V][pitch]
    void* f1;            // stage  f^(1)
    void* f2;            // stage  f^(2)
    const double* feqL;  // [V] ghost state left  (RSL_BC_EQ)
    const double* feqR;  // [V] ghost state right
    unsigned* status;    // bit 0: unphysical cell state; bit 1: non-finite f
    double* clock;       // Bjorken batches: current proper time of the instance
    double* cell;        // Sod: per-cell relaxation and equilibrium coefficients
                         // [kCellPar][pitch] of the current stage (two-kernel stage form)
};

// Per-cell coefficients stored by the two-kernel stage form: gamma/tau,
// gamma beta/tau, c0[0..kMaxNOm], c1[0..kMaxNOm].
constexpr int kCellPar = 2 + 2 * (kMaxNOm + 1);

// Descriptors stored by a batch hold byte offsets (f relative to the batch's f
// buffer, the rest relative to its work buffer); kernels add the bases.
__host__ __device__ inline void rebase(InstDesc& d, char* fbase, char* wbase) {
    d.f = fbase + (size_t)d.f;
    d.f1 = wbase + (size_t)d.f1;
    d.f2 = wbase + (size_t)d.f2;
    d.feqL = (const double*)(wbase + (size_t)d.feqL);
    d.feqR = (const double*)(wbase + (size_t)d.feqR);
    d.status = (unsigned*)(wbase + (size_t)d.status);
    d.clock = (double*)(wbase + (size_t)d.clock);
    d.cell = (double*)(wbase + (size_t)d.cell);
}

// Work items of one velocity-set class (see stage_class_of) in a batch.  The
// class runs one kernel variant (sod_stage.h); items exist for both tile
// widths (63 and 31 cells) so that the autotuner can switch variants, and
// for the 64-cell tiles of the two-kernel form's cell kernel.
struct StageClass {
    int var;                 // kernel variant in use
    int maxV;                // largest velocity set of the class
    const InstDesc* descs;   // device [n]
    const int2* items;       // device items of the current tile width, (instance, tile) or (-1, -1)
    int nitems;
    const int2* items_tw[3]; // [0]: 63-cell tiles, [1]: 31-cell tiles, [2]: 64-cell tiles
    int nitems_tw[3];
};

// Velocity-set classes of a Sod batch: V <= 32, 64, 128, 256, 320, 384 (the
// capacities of the fused stage kernel's shapes) and V > 384.
constexpr int kClasses = 7;
// Largest velocity set accepted by the Sod stage kernels.
constexpr int kMaxVelocities = 1 << 16;
struct BatchLaunch {
    StageClass cl[kClasses];
    StageClass all;          // every instance in one class (one launch per kernel and stage)
};

}  // namespace rsl

struct rsl_quad3 {
    rsl_quad* base = nullptr;   // the polar and radial nodes, Maclaurin tables
    int Qphi = 1, A = 0, V = 0;
    int device = -1;
    void* dmem = nullptr;       // angular and radial records
    rsl::Quad3Dev dev{};
};

struct rsl_quad {
    int QL, Q, NOm, V;
    double T0;
    double beta_series;        // |beta| below which the Maclaurin branch is used
    std::vector<double> xi, wxi, pbar, wL, KL, KP, Pm, ser, thr;
    bool on_device = false;
    int device = -1;
    void* dmem = nullptr;      // one allocation holding every table
    rsl::QuadDev dev{};
};

namespace rsl {

int set_error(int code, const std::string& msg);
int hip_check(hipError_t e, const char* what);

// Work-buffer layout for one instance.
struct WorkLayout {
    size_t f_bytes, f1_off, f2_off, feqL_off, feqR_off, status_off, cell_off, total;
};
WorkLayout work_layout(const rsl_quad* q, const rsl_problem* p);
InstDesc make_desc(const rsl_quad* q, const rsl_problem* p, void* f, void* work, double dt);
// CFL and relaxation-stiffness guards of one step of size dt (RSL_EUNSTABLE
// unless RSL_FLAG_FORCE_UNSTABLE is set).
int check_stability(const rsl_quad* q, const rsl_problem* p, double dt);
// Default bound on dt gamma (1 + |beta|) / tau_AW: the explicit RK3 scheme is
// stable on the negative real axis up to 2.51.
constexpr double kDefaultKappa = 2.0;
// Plateau of the inviscid Riemann problem of two ideal gases at rest
// (pressure, signed velocity, densities left and right of the contact).
struct RiemannPlateau {
    double PC, betaC, nI, nII;
};
RiemannPlateau riemann_plateau(double nL, double PL, double nR, double PR);

// Kernel launchers (sod.hip, bjorken.hip).
int launch_boundary_states(const InstDesc& d, double nL, double TL, double nR, double TR,
                           hipStream_t s);
int launch_sod_init(const InstDesc& d, hipStream_t s);
// Initial state of every instance of a Sod batch in two launches: states
// [n][4] = (n_L, T_L, n_R, T_R) per instance, items = (instance, 64-cell tile).
int launch_sod_batch_init(const InstDesc* descs, const double* states, int n, const int2* items, int nitems,
                          int dtype, char* fbase, char* wbase, hipStream_t s);
// `seq`: the stage's index within a call (0: the first, where the loop form
// computes the stage field's coefficients with the per-cell kernel first).
int launch_sod_stage(const InstDesc& d, int stage, hipStream_t s, int seq);
int launch_sod_moments(const InstDesc& d, const void* f, double* out, int nf, hipStream_t s);
int launch_sod_class_stage(const StageClass& cl, int dtype, int stage, char* fbase, char* wbase, hipStream_t s,
                           int seq);
int stage_class_of(int V);
int stage_default_variant(int cls);
// Stage kernel forms: fused (sod_stage.h), two-kernel and loop (sod_split.h).
constexpr int kFormFused = 0, kFormSplit = 1, kFormLoop = 2;
bool stage_variant_shape(int var, int* W, int* NV, int* TW, int* form, int* WC);
int stage_variant_count();
int stage_variant_capacity(int var);
int stage_variant_tile_cells(int var);
int launch_bj_batch_steps(const InstDesc* descs, int n, size_t lds, int dtype, char* fbase, char* wbase,
                          double tau0, double dtau, int nsteps, hipStream_t s);
int launch_bj_init(const InstDesc& d, double n0, double T0s, double tau0, hipStream_t s);
size_t bj_lds_bytes(int V);
size_t bj_mfma_lds_bytes(int Q, int QL);
bool bj_mfma_fits(int Q, int QL);
int launch_bj_mfma(const InstDesc* descs, const int* groups, int ngroups, int QL, size_t lds, int dtype, char* fbase,
                   char* wbase, int nsteps, hipStream_t s);
int launch_bj_steps(const InstDesc& d, double tau0, double dtau, int nsteps, hipStream_t s);
int launch_bj_moments(const InstDesc& d, const void* f, double* out, int nf, hipStream_t s);

int launch_feq3(const Quad3Dev& q, const double* state, int ncell, int dtype, void* f, int pitch, hipStream_t s);
int launch_moments3(const Quad3Dev& q, const void* f, int dtype, int ncell, int pitch, double* out, hipStream_t s);

}  // namespace rsl
