#pragma once
// Two-kernel form of one Sod RK3 stage (same operator as sod_stage.h).
//
// The fused stage kernel keeps every velocity of a tile in one workgroup so
// that the moments never leave the chip; for large velocity sets that pins
// many registers per lane and few waves per SIMD.  Here the stage is split
// at the only coupling between velocities, the moments:
//
//   cell kernel    per cell: the five moments of the stage field (eq. macro_jk
//                  in discrete form), the Landau frame (eqs. E_landau,
//                  u_landau), tau (eq. Sod:tau) and the equilibrium
//                  coefficients c0[m], c1[m], stored as kCellPar rows of the
//                  work buffer;
//   stream kernel  per (cell, velocity): the WENO5 fluxes (Sec. III F), the
//                  advective update, f^eq_jk from the stored coefficients, the
//                  AW relaxation and the RK combination (eq. rk3).
//
// Velocities are independent in the stream kernel, so its workgroups take
// any slice of the velocity set: W waves x NV velocities each, over the
// 63-cell tiles of the fused kernel; the cell kernel splits each cell's
// velocity sum over WC waves.  The price is a second read of the stage
// field (by then mostly in the last-level cache) and kCellPar doubles per cell.
#include "sod_stage.h"

namespace rsl {

namespace {

constexpr int kCellUnroll = 16;  // stage-field loads per wave in flight in the cell kernel

constexpr int kSerLen = kSeriesTerms * 2 * (kMaxNOm + 1);

// Shared memory of the cell kernel: partial moments of the waves, and copies
// of the Maclaurin tables (read by wave 0 with uniform addresses; staging
// them once per workgroup keeps table misses off the per-cell chain).
template <int WC>
struct CellLds {
    double red[WC * 5 * kLanes];
    double ser[kSerLen];
    double thr[kSeriesTerms];
};

// The per-cell chain on one wave, from the five moments of the stage field
// (eq. macro_jk in discrete form): the Landau frame (eqs. E_landau, u_landau),
// tau (eq. Sod:tau) and the equilibrium coefficients, stored as kCellPar rows
// (stride apart) at out when live.  Lanes without a cell carry a rest state so
// that the series term count stays wave-uniform.
template <typename TP>
__device__ __forceinline__ void cell_chain(const InstDesc& d, const double (&M)[5], bool live, double* out,
                                           size_t stride, TP ser, TP thr) {
    CellState cs = landau(M[0], M[1], M[2], M[3], M[4]);
    if (live && !cs.ok) atomicOr(d.status, 1u);
    if (!live || !cs.ok) {
        cs.n = 1.0; cs.T = 1.0; cs.beta = 0.0; cs.gamma = 1.0;
    }
    // terms for the lanes on the series branch (|beta| < beta_s); the others
    // take the recurrence and do not count
    const int nt = series_terms_uniform(wave_max_uniform(fmin(cs.beta * cs.beta, d.beta_series * d.beta_series)), thr);
    double tau = d.tau_r;
    if (d.tau_mode == RSL_TAU_ETAS) {
        const double lam = cs.n / (cs.T * cs.T * cs.T);
        tau = d.tau_aw0 / cs.T * (1.0 - 0.25 * log(lam * d.lambda_ref));
    }
    const double it = 1.0 / tau;
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
    feq_coef(cs.n, cs.T, cs.beta, cs.gamma, d.T0, d.NOm, d.beta_series, ser, nt, c0, c1);
    if (!live) return;
    out[0] = cs.gamma * it;
    out[stride] = cs.gamma * cs.beta * it;
#pragma unroll
    for (int m = 0; m <= kMaxNOm; ++m)      // the rows in use (the readers skip the rest)
        if (m <= d.NOm) {
            out[(2 + m) * stride] = c0[m];
            out[(3 + kMaxNOm + m) * stride] = c1[m];
        }
}

// WC waves split the velocity sum of 64 cells (one lane per cell).
template <typename Tf, int STAGE, int WC>
__device__ __forceinline__ void cell_tile(const InstDesc& d, int tile, CellLds<WC>& sh) {
    constexpr int W = WC, U = kCellUnroll;
    double* red = sh.red;
    for (int e = threadIdx.x; e < kSerLen; e += WC * kLanes) sh.ser[e] = d.tab.ser[e];
    for (int e = threadIdx.x; e < kSeriesTerms; e += WC * kLanes) sh.thr[e] = d.tab.thr[e];
    const int lane = threadIdx.x & (kLanes - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int c = tile * kCellTile + lane;
    const bool live = c < d.nz;
    const int cc = min(c, d.nz - 1);
    const Tf* __restrict__ fcur = (const Tf*)(STAGE == 1 ? d.f : (STAGE == 2 ? d.f1 : d.f2));
    const size_t pitch = (size_t)d.pitch;
    const int V = d.V;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
    for (int v0 = w; v0 < V; v0 += U * W) {
        Tf r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = fcur[(size_t)min(v0 + u * W, V - 1) * pitch + cc];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * W;
            if (v < V) {
                const double x = ldc(d.tab.xv, v), pk = ldc(d.tab.pv, v);
                const double fo = (double)r[u];
                const double p = pk * fo;
                m0 += fo;
                m1 += x * fo;
                m2 += p;
                m3 += x * p;
                m4 += x * x * p;
            }
        }
    }
    red[(w * 5 + 0) * kLanes + lane] = m0;
    red[(w * 5 + 1) * kLanes + lane] = m1;
    red[(w * 5 + 2) * kLanes + lane] = m2;
    red[(w * 5 + 3) * kLanes + lane] = m3;
    red[(w * 5 + 4) * kLanes + lane] = m4;
    __syncthreads();
    if (w != 0) return;
    // wave 0, all 64 lanes: per-cell coefficients
    double M[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double sum = red[q * kLanes + lane];
#pragma unroll
        for (int ww = 1; ww < W; ++ww) sum += red[(ww * 5 + q) * kLanes + lane];
        M[q] = sum;
    }
    cell_chain(d, M, live, d.cell + c, (size_t)d.pitch, (const double*)sh.ser, (const double*)sh.thr);
}

// The W waves of a workgroup share one tile: its cells' coefficients are
// loaded once into LDS (cf, kCellPar rows of 64) and read from there.
template <typename Tf, int STAGE, int W, int NV>
__device__ __forceinline__ void stream_tile(const InstDesc& d, int tile, int grp, char* lds, double* cf) {
    constexpr int G = kGroup;
    constexpr int WN = kWin;
    const int vbase = grp * (W * NV);
    if (vbase >= d.V) return;            // no workgroup-wide barrier below
    const int lane = threadIdx.x & (kLanes - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int z0 = tile * kTileCells;
    const int c = z0 - 1 + lane;
    const bool ghost = (c < 0) || (c >= d.nz);
    const int cc = min(max(c, 0), d.nz - 1);
    const int hc = lane < 2 ? z0 - 3 + lane : z0 + kLanes - 3 + lane;
    const bool hghost = (hc < 0) || (hc >= d.nz);
    const int hcc = min(max(hc, 0), d.nz - 1);
    const bool eqbc = d.bc == RSL_BC_EQ;
    const int V = d.V;
    Tf* win = (Tf*)lds + w * G * WN;          // one window per wave, reused group after group

    const Tf* __restrict__ fcur = (const Tf*)(STAGE == 1 ? d.f : (STAGE == 2 ? d.f1 : d.f2));
    Tf* __restrict__ fout = (Tf*)(STAGE == 1 ? d.f1 : (STAGE == 2 ? d.f2 : d.f));
    const Tf* __restrict__ fn = (const Tf*)d.f;
    const size_t pitch = (size_t)d.pitch;
    const double dt = d.dt, dzi = d.dz_inv;

    // stage-field and f_n loads of all NV velocities in flight at once
    Tf ra[NV], rh[NV], rn[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int v = min(vbase + w + i * W, V - 1);
        const Tf* row = fcur + (size_t)v * pitch;
        ra[i] = row[cc];
        rh[i] = lane < 5 ? row[hcc] : Tf(0);
        if (STAGE > 1) rn[i] = fn[(size_t)v * pitch + cc];
    }
    // the tile's cell coefficients: the rows in use (gamma/tau, gamma beta/tau,
    // c0[0..N_Omega], c1[0..N_Omega]) spread over the waves, through LDS
    // (c0, c1 stay in LDS and are read per velocity: fewer registers, more
    // waves per SIMD)
    const bool collide = d.tau_mode != RSL_TAU_INF;
    double cA = 0.0, cB = 0.0;
    const double* cfl = cf + lane;
    if (collide) {
        const int nrow = 2 + 2 * (d.NOm + 1);
        for (int r = w; r < nrow; r += W) {
            const int row = r < 2 + d.NOm + 1 ? r : r - (2 + d.NOm + 1) + 3 + kMaxNOm;
            cf[row * kLanes + lane] = d.cell[(size_t)row * pitch + cc];
        }
        __syncthreads();
        cA = cfl[0];
        cB = cfl[kLanes];
    }

    const bool out_lane = !ghost && lane >= 1;
    // stencil arithmetic in the storage type (per-cell coefficients stay binary64)
    using Tc = Tf;
    const Tc dtc = (Tc)dt, dzic = (Tc)dzi, cAc = (Tc)cA, cBc = (Tc)cB;
    unsigned bad = 0;
#pragma unroll
    for (int i0 = 0; i0 < NV; i0 += G) {
        if (vbase + w + i0 * W >= V) break;
#pragma unroll
        for (int i = i0; i < i0 + G && i < NV; ++i) {
            const int v = vbase + w + i * W;
            if (v < V) {
                double fc = (double)ra[i], h = (double)rh[i];
                if (eqbc) {
                    const double gl = ldc(d.feqL, v), gr = ldc(d.feqR, v);
                    fc = ghost ? (c < 0 ? gl : gr) : fc;
                    h = hghost ? (hc < 0 ? gl : gr) : h;
                }
                Tf* wb = win + (i - i0) * WN;
                wb[lane + 2] = (Tf)fc;
                if (lane < 2) wb[lane] = (Tf)h;
                else if (lane < 5) wb[kLanes + lane] = (Tf)h;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int i = i0; i < i0 + G && i < NV; ++i) {
            const int v = vbase + w + i * W;
            if (v < V) {
                // the velocity's constants: one contiguous record, scalar loads
                const __attribute__((address_space(4))) double* vr =
                    (const __attribute__((address_space(4))) double*)d.tab.vrec + (size_t)v * kVrec;
                const double x = vr[0];
                const Tc xc = (Tc)x;
                const Tf* wb = win + (i - i0) * WN;
                Tc sv[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) sv[q] = wb[lane + q];
                Tc F = 0;
                if (x > 0.0) F = xc * weno5(sv[0], sv[1], sv[2], sv[3], sv[4]);
                else if (x < 0.0) F = xc * weno5(sv[5], sv[4], sv[3], sv[2], sv[1]);
                const Tc Fm = shift_up(F);
                Tc y = sv[2] + dtc * (-(F - Fm) * dzic);
                if (collide) {
                    const double l1 = vr[2], wx = vr[3];
                    double gsum = 0.0;
#pragma unroll
                    for (int m = 0; m <= kMaxNOm; ++m)
                        if (m <= d.NOm)
                            gsum = fma(vr[4 + m], fma(l1, cfl[(3 + kMaxNOm + m) * kLanes], cfl[(2 + m) * kLanes]),
                                       gsum);
                    y += dtc * (cAc - cBc * xc) * ((Tc)(wx * gsum) - sv[2]);
                }
                Tc out;
                if (STAGE == 1) out = y;
                else if (STAGE == 2) out = Tc(0.75) * rn[i] + Tc(0.25) * y;
                else out = fma(Tc(kTwoThirds), y, Tc(kThird) * rn[i]);
                if (out_lane) {
                    const Tf o = (Tf)out;
                    if (!isfinite(o)) bad |= 2u;
                    fout[(size_t)v * pitch + c] = o;
                }
            }
        }
        wave_lds_sync();   // the group's window reads are done before the next group writes
    }
    if (bad) atomicOr(d.status, bad);
}

template <typename Tf, int STAGE, int WC>
__global__ void __launch_bounds__(WC * 64) cell_single_kernel(InstDesc d, int ntiles) {
    __shared__ CellLds<WC> sh;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles || d.tau_mode == RSL_TAU_INF) return;
    cell_tile<Tf, STAGE, WC>(d, tile, sh);
}

template <typename Tf, int STAGE, int WC>
__global__ void __launch_bounds__(WC * 64) cell_batch_kernel(const InstDesc* __restrict__ descs,
                                                            const int2* __restrict__ items, char* fbase,
                                                            char* wbase) {
    __shared__ CellLds<WC> sh;
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    InstDesc d = descs[it.x];
    if (d.tau_mode == RSL_TAU_INF) return;
    rebase(d, fbase, wbase);
    cell_tile<Tf, STAGE, WC>(d, it.y, sh);
}

template <typename Tf, int W>
struct StreamLds {
    Tf win[W * kGroup * kWin];
    double cf[kCellPar * kLanes];
};

template <typename Tf, int STAGE, int W, int NV>
__global__ void __launch_bounds__(W * 64) stream_single_kernel(InstDesc d, int ntiles) {
    __shared__ StreamLds<Tf, W> sh;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    stream_tile<Tf, STAGE, W, NV>(d, tile, blockIdx.y, (char*)sh.win, sh.cf);
}

template <typename Tf, int STAGE, int W, int NV>
__global__ void __launch_bounds__(W * 64) stream_batch_kernel(const InstDesc* __restrict__ descs,
                                                             const int2* __restrict__ items, char* fbase,
                                                             char* wbase) {
    __shared__ StreamLds<Tf, W> sh;
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    stream_tile<Tf, STAGE, W, NV>(d, it.y, blockIdx.y, (char*)sh.win, sh.cf);
}

// ---------------------------------------------------------------------------
// Loop form: one workgroup per 63-cell tile walks the whole velocity set (W
// waves x NV velocities per round, K rounds of loads in flight) and, as it
// writes the stage's output, sums that output's five moments per cell; at the
// end wave 0 runs the per-cell chain on the sums and stores the NEXT stage's
// coefficients over the ones this stage read (each tile reads and writes only
// its own cells).  The stage field is then read once per stage instead of
// twice, and the per-cell kernel runs only before the first stage of a call.
template <typename Tf, int W>
struct LoopLds {
    union {
        struct {
            Tf win[W * kGroup * kWin];
            double cf[kCellPar * kLanes];
        } s;
        double red[W * 5 * kLanes];   // moment sums of the waves (outside the velocity walk)
    } u;
};

// A buffer resource over one velocity plane of a field (gfx9 resource word:
// raw byte addressing, no format conversion, offsets range-checked against
// the plane size), and binary32 / binary64 loads and stores through it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* plane, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(plane), (short)0, bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T plane_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void plane_store(__amdgpu_buffer_rsrc_t r, uint32_t off, T x) {
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
    else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, off, 0, 0);
}

// Legendre sums of the equilibrium coefficients at one angular node for
// N_Omega = N: sum_m P_m(xi_J) c0_m and sum_m P_m(xi_J) c1_m, the record's
// P_m and the cell's coefficient rows read in one batch.
template <int N>
__device__ __forceinline__ void legendre_sums(const __attribute__((address_space(4))) double* vr, const double* cfl,
                                              double& g, double& hs) {
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        g = fma(vr[4 + m], cfl[(2 + m) * kLanes], g);
        hs = fma(vr[4 + m], cfl[(3 + kMaxNOm + m) * kLanes], hs);
    }
}

template <typename Tf, int STAGE, int W, int NV, int K>
__device__ __forceinline__ void loop_tile(const InstDesc& d, int tile, LoopLds<Tf, W>& sh) {
    constexpr int G = kGroup;
    constexpr int WN = kWin;
    constexpr int step = W * NV;
    const int lane = threadIdx.x & (kLanes - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int z0 = tile * kTileCells;
    const int c = z0 - 1 + lane;
    const bool ghost = (c < 0) || (c >= d.nz);
    const int cc = min(max(c, 0), d.nz - 1);
    const int hc = lane < 2 ? z0 - 3 + lane : z0 + kLanes - 3 + lane;
    const bool hghost = (hc < 0) || (hc >= d.nz);
    const int hcc = min(max(hc, 0), d.nz - 1);
    const bool eqbc = d.bc == RSL_BC_EQ;
    Tf* win = sh.u.s.win + w * G * WN;       // one window per wave, reused group after group
    double* cf = sh.u.s.cf;

    const Tf* __restrict__ fcur = (const Tf*)(STAGE == 1 ? d.f : (STAGE == 2 ? d.f1 : d.f2));
    Tf* __restrict__ fout = (Tf*)(STAGE == 1 ? d.f1 : (STAGE == 2 ? d.f2 : d.f));
    const Tf* __restrict__ fn = (const Tf*)d.f;
    const size_t pitch = (size_t)d.pitch;
    const double dt = d.dt, dzi = d.dz_inv;
    const bool collide = d.tau_mode != RSL_TAU_INF;
    const bool out_lane = !ghost && lane >= 1;   // the tile's cells (lane 0: the left neighbour's)

    // this stage's coefficients of the tile's cells (written by the previous
    // stage's workgroup of this tile; lane 0 reads the tile's first cell
    // instead of its neighbour's, which another workgroup rewrites, and its
    // result is never stored)
    double cA = 0.0, cB = 0.0;
    const double* cfl = cf + lane;
    if (collide) {
        const int ccf = lane == 0 ? min(z0, d.nz - 1) : cc;
        const int nrow = 2 + 2 * (d.NOm + 1);
        for (int r = w; r < nrow; r += W) {
            const int row = r < 2 + d.NOm + 1 ? r : r - (2 + d.NOm + 1) + 3 + kMaxNOm;
            cf[row * kLanes + lane] = d.cell[(size_t)row * pitch + ccf];
        }
        __syncthreads();
        cA = cfl[0];
        cB = cfl[kLanes];
    }

    // stencil arithmetic in the storage type (per-cell coefficients and the
    // moment sums stay binary64); the relaxation rate is taken with dt folded
    // in, dt gamma (1 - beta xi) / tau = dtA - dtB xi
    using Tc = Tf;
    const Tc dtdz = (Tc)(dt * dzi), dtA = (Tc)(dt * cA), dtB = (Tc)(dt * cB);
    unsigned bad = 0;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
    // Rounds of W NV velocities, angular-node blocks outer and radial nodes
    // inner: round (J-block jb, radial node k) gives wave w the velocities
    // v = k Q_xi + J, J = jb + w + i W, so that a wave meets each angular node
    // J in Q_L consecutive rounds and forms the Legendre sums of f^eq over m
    // (which depend on J only) once for all of them.  The loads of rounds
    // r + 1 .. r + K - 1 are issued before round r is computed, into other
    // register sets (no copies between them, so nothing waits for the loads
    // in flight).  Loads are unconditional (indices clamped into the field) so
    // that the compiler's wait counts stay exact; the halo lanes' second load
    // is, on other lanes, a repeat of their own cell.
    const int Q = d.Q, QL = d.QL;
    const int nrounds = (Q + step - 1) / step * QL;
    struct Pos {
        int jb, k;
    };
    auto advance = [&](Pos& p) {
        if (++p.k == QL) {
            p.k = 0;
            p.jb += step;
        }
    };
    const int hcl = lane < 5 ? hcc : cc;
    // Loads and stores through a buffer resource per velocity plane (uniform
    // base and size): per-lane 32-bit byte offsets, no 64-bit per-lane
    // address arithmetic
    // (a lane that stores owns cell c = cc, so its store offset is occ too)
    const uint32_t occ = (uint32_t)cc * (uint32_t)sizeof(Tf), ohc = (uint32_t)hcl * (uint32_t)sizeof(Tf);
    const int plane_bytes = (int)(pitch * sizeof(Tf));
    auto load_round = [&](const Pos& p, Tf (&a)[NV], Tf (&h)[NV], Tf (&n)[NV]) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int v = p.k * Q + min(p.jb + w + i * W, Q - 1);
            const auto row = plane_rsrc(fcur + (size_t)v * pitch, plane_bytes);
            a[i] = plane_load<Tf>(row, occ);
            h[i] = plane_load<Tf>(row, ohc);
            if (STAGE > 1) n[i] = plane_load<Tf>(plane_rsrc(fn + (size_t)v * pitch, plane_bytes), occ);
        }
    };
    double gJ[NV], hJ[NV];   // Legendre sums of the coefficients at the wave's angular nodes
#pragma unroll
    for (int i = 0; i < NV; ++i) gJ[i] = hJ[i] = 0.0;
    auto round = [&](const Pos& p, const Tf (&ra)[NV], const Tf (&rh)[NV], const Tf (&rn)[NV]) {
#pragma unroll
        for (int i0 = 0; i0 < NV; i0 += G) {
            if (p.jb + w + i0 * W >= Q) break;
#pragma unroll
            for (int i = i0; i < i0 + G && i < NV; ++i) {
                const int J = p.jb + w + i * W;
                if (J < Q) {
                    const int v = p.k * Q + J;
                    double fc = (double)ra[i], h = (double)rh[i];
                    if (eqbc) {
                        const double gl = ldc(d.feqL, v), gr = ldc(d.feqR, v);
                        fc = ghost ? (c < 0 ? gl : gr) : fc;
                        h = hghost ? (hc < 0 ? gl : gr) : h;
                    }
                    Tf* wb = win + (i - i0) * WN;
                    wb[lane + 2] = (Tf)fc;
                    if (lane < 2) wb[lane] = (Tf)h;
                    else if (lane < 5) wb[kLanes + lane] = (Tf)h;
                }
            }
            wave_lds_sync();
#pragma unroll
            for (int i = i0; i < i0 + G && i < NV; ++i) {
                const int J = p.jb + w + i * W;
                if (J < Q) {
                    const int v = p.k * Q + J;
                    const __attribute__((address_space(4))) double* vr =
                        (const __attribute__((address_space(4))) double*)d.tab.vrec + (size_t)v * kVrec;
                    const __attribute__((address_space(4))) float* vf =
                        (const __attribute__((address_space(4))) float*)(vr + kVrecF32);
                    // the record's fields, loaded together ahead of the branches
                    const int sgn = ((const __attribute__((address_space(4))) int*)vf)[3];
                    const Tc xc = sizeof(Tc) == 4 ? (Tc)vf[0] : (Tc)vr[0];
                    const Tc x6 = sizeof(Tc) == 4 ? (Tc)vf[1] : (Tc)vr[kVrecXi6];
                    const double x = vr[0], pk = vr[1], l1 = vr[2], wx = vr[3], x2 = vr[kVrecXi2];
                    const Tf* wb = win + (i - i0) * WN;
                    Tc sv[6];
#pragma unroll
                    for (int q = 0; q < 6; ++q) sv[q] = wb[lane + q];
                    Tc F = 0;
                    if (sgn > 0) F = x6 * weno5_6(sv[0], sv[1], sv[2], sv[3], sv[4]);
                    else if (sgn < 0) F = x6 * weno5_6(sv[5], sv[4], sv[3], sv[2], sv[1]);
                    const Tc Fm = shift_up(F);
                    Tc y = fma(Fm - F, dtdz, sv[2]);
                    if (collide) {
                        if (p.k == 0) {   // first radial node of this J: its sums over m
                            double g = 0.0, hs = 0.0;
                            switch (d.NOm) {   // branch-free sums for the usual orders
                                case 3: legendre_sums<3>(vr, cfl, g, hs); break;
                                case 4: legendre_sums<4>(vr, cfl, g, hs); break;
                                case 5: legendre_sums<5>(vr, cfl, g, hs); break;
                                case 6: legendre_sums<6>(vr, cfl, g, hs); break;
                                default:
#pragma unroll
                                    for (int m = 0; m <= kMaxNOm; ++m)
                                        if (m <= d.NOm) {
                                            g = fma(vr[4 + m], cfl[(2 + m) * kLanes], g);
                                            hs = fma(vr[4 + m], cfl[(3 + kMaxNOm + m) * kLanes], hs);
                                        }
                            }
                            gJ[i] = g;
                            hJ[i] = hs;
                        }
                        // f^eq in binary64 (its Legendre terms grow like gamma^4 at high
                        // |beta| and partly cancel), rounded once to the stencil type
                        const Tc fe = (Tc)(wx * fma(l1, hJ[i], gJ[i]));
                        y = fma(fma(-dtB, xc, dtA), fe - sv[2], y);
                    }
                    Tc out;
                    if (STAGE == 1) out = y;
                    else if (STAGE == 2) out = Tc(0.75) * rn[i] + Tc(0.25) * y;
                    else out = fma(Tc(kTwoThirds), y, Tc(kThird) * rn[i]);
                    if (out_lane) {
                        const Tf o = (Tf)out;
                        if (!isfinite(o)) bad |= 2u;
                        plane_store<Tf>(plane_rsrc(fout + (size_t)v * pitch, plane_bytes), occ, o);
                        // moments of the stored output (the next stage's field)
                        const double fo = (double)o, pw = pk * fo;
                        m0 += fo;
                        m1 = fma(x, fo, m1);
                        m2 += pw;
                        m3 = fma(x, pw, m3);
                        m4 = fma(x2, pw, m4);
                    }
                }
            }
            wave_lds_sync();   // the group's window reads are done before the next group writes
        }
    };
    // a ring of K register sets: round r is computed while rounds r + 1 ..
    // r + K - 1 are in flight
    Tf A[K][NV], H[K][NV], N[K][NV];
    Pos lp{0, 0}, cp{0, 0};
#pragma unroll
    for (int k = 0; k < K - 1; ++k) {
        load_round(lp, A[k], H[k], N[k]);
        advance(lp);
    }
    for (int r0 = 0; r0 < nrounds; r0 += K) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (r0 + k >= nrounds) break;
            load_round(lp, A[(k + K - 1) % K], H[(k + K - 1) % K], N[(k + K - 1) % K]);
            advance(lp);
            round(cp, A[k], H[k], N[k]);
            advance(cp);
        }
    }
    if (bad) atomicOr(d.status, bad);
    if (!collide) return;                 // uniform: nobody reaches the barriers below
    __syncthreads();                      // windows and coefficients are dead: red overlays them
    double* red = sh.u.red;
    red[(w * 5 + 0) * kLanes + lane] = m0;
    red[(w * 5 + 1) * kLanes + lane] = m1;
    red[(w * 5 + 2) * kLanes + lane] = m2;
    red[(w * 5 + 3) * kLanes + lane] = m3;
    red[(w * 5 + 4) * kLanes + lane] = m4;
    __syncthreads();
    if (w != 0) return;
    double M[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double sum = red[q * kLanes + lane];
#pragma unroll
        for (int ww = 1; ww < W; ++ww) sum += red[(ww * 5 + q) * kLanes + lane];
        M[q] = sum;
    }
    // the Maclaurin tables through scalar loads (uniform addresses, shared by
    // every workgroup through the scalar cache)
    using CP = const __attribute__((address_space(4))) double*;
    cell_chain(d, M, out_lane, d.cell + c, pitch, (CP)d.tab.ser, (CP)d.tab.thr);
}

template <typename Tf, int STAGE, int W, int NV, int K>
__global__ void __launch_bounds__(W * 64) loop_batch_kernel(const InstDesc* __restrict__ descs,
                                                           const int2* __restrict__ items, char* fbase,
                                                           char* wbase) {
    __shared__ LoopLds<Tf, W> sh;
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    InstDesc d = descs[it.x];
    rebase(d, fbase, wbase);
    loop_tile<Tf, STAGE, W, NV, K>(d, it.y, sh);
}

// The loop kernel, preceded by the per-cell kernel (WC waves, 64-cell tiles)
// at the first stage of a call (seq == 0).  Batches only: one instance has too
// few tiles for one workgroup per tile to fill the GPU.
template <typename Tf, int STAGE, int W, int NV, int WC, int K>
int launch_loop_t(const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s, int seq) {
    if (d) return set_error(RSL_EUNSUPPORTED, "the loop form of the Sod stage runs in batches only");
    if (seq == 0)
        hipLaunchKernelGGL((cell_batch_kernel<Tf, STAGE, WC>), dim3(cl->nitems_tw[2]), dim3(WC * 64), 0, s, cl->descs,
                           cl->items_tw[2], fb, wb);
    hipLaunchKernelGGL((loop_batch_kernel<Tf, STAGE, W, NV, K>), dim3(cl->nitems), dim3(W * 64), 0, s, cl->descs,
                       cl->items, fb, wb);
    return hip_check(hipGetLastError(), "sod loop-form stage launch");
}

// Two launches on one stream: the cell kernel (WC waves) over 64-cell tiles,
// then the stream kernel (W waves of NV velocities) over (63-cell tile,
// velocity slice).  A batch class sizes the slice dimension by its largest V.
template <typename Tf, int STAGE, int W, int NV, int WC>
int launch_split_t(const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s) {
    if (d) {
        const int ntiles = (d->nz + kTileCells - 1) / kTileCells;
        const int nb = (ntiles + 7) / 8 * 8;
        const int ng = (d->V + W * NV - 1) / (W * NV);
        const int nct = (d->nz + kCellTile - 1) / kCellTile;
        hipLaunchKernelGGL((cell_single_kernel<Tf, STAGE, WC>), dim3((nct + 7) / 8 * 8), dim3(WC * 64), 0, s, *d,
                           nct);
        hipLaunchKernelGGL((stream_single_kernel<Tf, STAGE, W, NV>), dim3(nb, ng), dim3(W * 64), 0, s, *d, ntiles);
    } else {
        const int ng = (cl->maxV + W * NV - 1) / (W * NV);
        hipLaunchKernelGGL((cell_batch_kernel<Tf, STAGE, WC>), dim3(cl->nitems_tw[2]), dim3(WC * 64), 0, s,
                           cl->descs, cl->items_tw[2], fb, wb);
        hipLaunchKernelGGL((stream_batch_kernel<Tf, STAGE, W, NV>), dim3(cl->nitems, ng), dim3(W * 64), 0, s,
                           cl->descs, cl->items, fb, wb);
    }
    return hip_check(hipGetLastError(), "sod two-kernel stage launch");
}

template <typename Tf, int STAGE>
int launch_cls(int var, const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s, int seq) {
    switch (var) {
#define RSL_CASE(id, W, NV, TW) \
    case id: return launch_t<Tf, STAGE, W, NV, TW>(d, cl, fb, wb, s);
        RSL_STAGE_VARIANTS(RSL_CASE)
#undef RSL_CASE
#define RSL_CASE(id, W, NV, WC) \
    case id: return launch_split_t<Tf, STAGE, W, NV, WC>(d, cl, fb, wb, s);
        RSL_SPLIT_VARIANTS(RSL_CASE)
#undef RSL_CASE
#define RSL_CASE(id, W, NV, WC, K) \
    case id: return launch_loop_t<Tf, STAGE, W, NV, WC, K>(d, cl, fb, wb, s, seq);
        RSL_LOOP_VARIANTS(RSL_CASE)
#undef RSL_CASE
        default: return set_error(RSL_EINVAL, "unknown stage kernel variant");
    }
}

template <typename Tf>
int launch_stage_any(int stage, int var, const InstDesc* d, const StageClass* cl, char* fb, char* wb,
                     hipStream_t s, int seq) {
    if (stage == 1) return launch_cls<Tf, 1>(var, d, cl, fb, wb, s, seq);
    if (stage == 2) return launch_cls<Tf, 2>(var, d, cl, fb, wb, s, seq);
    return launch_cls<Tf, 3>(var, d, cl, fb, wb, s, seq);
}

}  // namespace

}  // namespace rsl
