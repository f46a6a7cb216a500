// C ABI of librsl: argument validation, table upload, kernel sequencing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "imex.h"
#include "rsl_impl.h"

namespace rsl {

int build_quadrature(int QL, int Q, int NOm, double T0, rsl_quad* q);

namespace {
thread_local std::string g_err;
}

int set_error(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return RSL_OK;
    return set_error(RSL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

WorkLayout work_layout(const rsl_quad* q, const rsl_problem* p) {
    WorkLayout L{};
    const size_t es = p->dtype == RSL_F32 ? 4 : 8;
    const size_t pitch = p->problem == RSL_SOD ? (size_t)rsl_pitch(p->nz) : 1;
    L.f_bytes = align_up(es * pitch * q->V, 256);
    L.f1_off = 0;
    L.f2_off = L.f_bytes;
    L.feqL_off = 2 * L.f_bytes;
    L.feqR_off = L.feqL_off + align_up(sizeof(double) * q->V, 256);
    L.status_off = L.feqR_off + align_up(sizeof(double) * q->V, 256);
    L.cell_off = L.status_off + 256;
    L.total = L.cell_off + (p->problem == RSL_SOD ? sizeof(double) * kCellPar * pitch : 0);
    return L;
}

InstDesc make_desc(const rsl_quad* q, const rsl_problem* p, void* f, void* work, double dt) {
    InstDesc d{};
    const WorkLayout L = work_layout(q, p);
    d.nz = p->problem == RSL_SOD ? p->nz : 1;
    d.pitch = p->problem == RSL_SOD ? rsl_pitch(p->nz) : 1;
    d.Q = q->Q;
    d.QL = q->QL;
    d.V = q->V;
    d.NOm = q->NOm;
    d.bc = p->bc;
    d.tau_mode = p->tau_mode;
    d.gas = p->gas;
    d.dtype = p->dtype;
    d.dz = p->problem == RSL_SOD ? (p->z_hi - p->z_lo) / p->nz : 1.0;
    d.dz_inv = 1.0 / d.dz;
    d.z_lo = p->z_lo;
    d.dt = dt;
    d.tau_r = p->tau_r;
    d.tau_aw0 = p->tau_aw0;
    d.lambda_ref = p->lambda_ref > 0 ? p->lambda_ref : 1.0;
    d.T0 = q->T0;
    d.beta_series = q->beta_series;
    d.tab = q->dev;
    char* w = (char*)work;
    d.f = f;
    d.f1 = w + L.f1_off;
    d.f2 = w + L.f2_off;
    d.feqL = (const double*)(w + L.feqL_off);
    d.feqR = (const double*)(w + L.feqR_off);
    d.status = (unsigned*)(w + L.status_off);
    d.clock = (double*)(w + L.status_off + 8);
    d.cell = (double*)(w + L.cell_off);
    return d;
}

// Plateau of the inviscid Riemann problem between two ideal gases at rest with
// P = E/3 (Sec. IV B 1): P_C is the root of eq. Sod:PC, beta_C follows from eq.
// Sod:uplateau, n_I from eq. Sod:nI and n_II from eq. Sod:nII.  The
// higher-pressure side plays the left state (the problem mirrors otherwise);
// equal pressures give no flow.
RiemannPlateau riemann_plateau(double nL, double PL, double nR, double PR) {
    RiemannPlateau r{};
    const bool mirror = PR > PL;
    if (mirror) {
        std::swap(nL, nR);
        std::swap(PL, PR);
    }
    if (!(PL > PR)) {
        r.PC = PL;
        r.betaC = 0.0;
        r.nI = nL;
        r.nII = nR;
    } else {
        const double h = std::sqrt(3.0) / 2.0;
        auto resid = [&](double P) {
            const double a = std::pow(PL / P, h);
            const double d = P - PR;
            return (a - 1.0) / (a + 1.0) - std::sqrt(3.0 * d * d / ((P + 3.0 * PR) * (3.0 * P + PR)));
        };
        double lo = PR, hi = PL;      // resid(PR) > 0 > resid(PL)
        for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
            const double mid = 0.5 * (lo + hi);
            (resid(mid) > 0.0 ? lo : hi) = mid;
        }
        const double PC = 0.5 * (lo + hi), d = PC - PR;
        r.PC = PC;
        r.betaC = std::sqrt(3.0 * d * d / ((PC + 3.0 * PR) * (3.0 * PC + PR)));
        r.nI = nL * std::pow(PC / PL, 0.75);
        r.nII = nR * std::sqrt(PC * (PR + 3.0 * PC) / (PR * (PC + 3.0 * PR)));
    }
    if (mirror) {
        std::swap(r.nI, r.nII);
        r.betaC = -r.betaC;
    }
    return r;
}

// Largest dt allowed by the CFL condition (dt max|xi| / dz < 1, Sec. III F)
// and by the stiffness of the AW term, whose rate for population j is
// gamma (1 - beta xi_j) / tau <= gamma (1 + |beta|) / tau.  The largest rate
// over the flow is taken over the states of the inviscid Riemann solution
// (the two initial states and the two plateaus, whose speed |beta_C| is the
// largest in the flow); Bjorken flow is at rest.  Infinite where no bound
// applies.
void stability_limits(const rsl_quad* q, const rsl_problem* p, double* cfl_dt, double* stiff_dt) {
    *cfl_dt = *stiff_dt = HUGE_VAL;
    if (p->problem == RSL_SOD) *cfl_dt = (p->z_hi - p->z_lo) / p->nz / std::fabs(q->xi.back());
    if (p->tau_mode == RSL_TAU_INF) return;
    const double kappa = p->kappa > 0 ? p->kappa : kDefaultKappa;
    const double lref = p->lambda_ref > 0 ? p->lambda_ref : 1.0;
    auto tau_of = [&](double n, double T) {
        if (p->tau_mode == RSL_TAU_CONST) return p->tau_r;
        return p->tau_aw0 / T * (1.0 - 0.25 * std::log(n / (T * T * T) * lref));
    };
    double rate = 1.0 / tau_of(p->n_L, p->T_L);
    if (p->problem == RSL_SOD) {
        const RiemannPlateau r = riemann_plateau(p->n_L, p->n_L * p->T_L, p->n_R, p->n_R * p->T_R);
        const double b = std::fabs(r.betaC);
        const double speed = std::sqrt((1.0 + b) / (1.0 - b));     // gamma (1 + |beta|)
        rate = std::max(rate, 1.0 / tau_of(p->n_R, p->T_R));
        rate = std::max(rate, speed / tau_of(r.nI, r.PC / r.nI));
        rate = std::max(rate, speed / tau_of(r.nII, r.PC / r.nII));
    }
    *stiff_dt = rate > 0.0 ? kappa / rate : 0.0;    // a non-positive tau leaves no stable step
}

int check_cfl(const rsl_quad* q, const rsl_problem* p, double dt) {
    if (!(dt > 0.0 && std::isfinite(dt))) return set_error(RSL_EINVAL, "dt must be > 0");
    double cfl_dt, stiff_dt;
    stability_limits(q, p, &cfl_dt, &stiff_dt);
    if (!(dt < cfl_dt)) return set_error(RSL_EUNSTABLE, "CFL number dt*max|xi|/dz >= 1");
    return RSL_OK;
}

int check_stability(const rsl_quad* q, const rsl_problem* p, double dt) {
    if (!(dt > 0.0 && std::isfinite(dt))) return set_error(RSL_EINVAL, "dt must be > 0");
    if (p->flags & RSL_FLAG_FORCE_UNSTABLE) return RSL_OK;
    double cfl_dt, stiff_dt;
    stability_limits(q, p, &cfl_dt, &stiff_dt);
    if (!(dt < cfl_dt)) return set_error(RSL_EUNSTABLE, "CFL number dt*max|xi|/dz >= 1");
    if (!(dt <= stiff_dt))
        return set_error(RSL_EUNSTABLE, "dt * gamma (1 + |beta|) / tau_AW exceeds kappa (stiff relaxation); set "
                                        "RSL_FLAG_FORCE_UNSTABLE to override");
    return RSL_OK;
}

}  // namespace rsl

using namespace rsl;

namespace {

int check_quad(const rsl_quad* q) {
    if (!q) return set_error(RSL_EINVAL, "null rsl_quad");
    if (!q->on_device) return set_error(RSL_EINVAL, "rsl_quad was built with RSL_QUAD_HOST_ONLY");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != q->device)
        return set_error(RSL_EINVAL, "rsl_quad belongs to another HIP device than the current one");
    return RSL_OK;
}

bool pos(double x) { return x > 0.0 && std::isfinite(x); }

int check_problem(const rsl_quad* q, const rsl_problem* p) {
    if (!p) return set_error(RSL_EINVAL, "null rsl_problem");
    if (p->problem != RSL_SOD && p->problem != RSL_BJORKEN) return set_error(RSL_EINVAL, "unknown problem kind");
    if (p->dtype != RSL_F64 && p->dtype != RSL_F32) return set_error(RSL_EINVAL, "dtype must be RSL_F64 or RSL_F32");
    if (p->tau_mode < RSL_TAU_CONST || p->tau_mode > RSL_TAU_INF) return set_error(RSL_EINVAL, "unknown tau_mode");
    if (p->tau_mode == RSL_TAU_CONST && !pos(p->tau_r)) return set_error(RSL_EINVAL, "tau_r must be > 0");
    if (p->tau_mode == RSL_TAU_ETAS && !pos(p->tau_aw0)) return set_error(RSL_EINVAL, "tau_aw0 must be > 0");
    if (!pos(p->n_L) || !pos(p->T_L)) return set_error(RSL_EINVAL, "left/initial state needs n > 0, T > 0");
    if (p->problem == RSL_SOD) {
        if (p->nz < 5 || p->nz > (1 << 28)) return set_error(RSL_EINVAL, "Sod needs 5 <= nz <= 2^28");
        if (!(p->z_hi > p->z_lo)) return set_error(RSL_EINVAL, "Sod needs z_hi > z_lo");
        if (!pos(p->n_R) || !pos(p->T_R)) return set_error(RSL_EINVAL, "right state needs n > 0, T > 0");
        if (p->bc != RSL_BC_EQ && p->bc != RSL_BC_OUTFLOW) return set_error(RSL_EINVAL, "unknown bc");
        if (p->gas != RSL_GAS_IDEAL) return set_error(RSL_EUNSUPPORTED, "the Sod problem is built for the ideal gas");
    } else {
        if (p->nz != 1) return set_error(RSL_EINVAL, "Bjorken flow needs nz = 1");
        if (p->gas != RSL_GAS_IDEAL && p->gas != RSL_GAS_PARTON) return set_error(RSL_EINVAL, "unknown gas");
    }
    (void)q;
    return RSL_OK;
}

}  // namespace

extern "C" {

const char* rsl_last_error(void) { return g_err.c_str(); }

int rsl_pitch(int nz) { return nz <= 0 ? 0 : (nz + 63) / 64 * 64; }

int rsl_make_quadrature(int Q_L, int Q_xi, int N_L, int N_Omega, double T0, int flags, rsl_quad** out) {
    if (!out) return set_error(RSL_EINVAL, "null output pointer");
    *out = nullptr;
    if (N_L != 1) return set_error(RSL_EUNSUPPORTED, "only N_L = 1 is built (the paper's radial truncation)");
    if (N_Omega > kMaxNOm) return set_error(RSL_EUNSUPPORTED, "N_Omega > 6: no equilibrium coefficients (App. A)");
    if (Q_L < 2 || Q_L > 8) return set_error(RSL_EINVAL, "need 2 <= Q_L <= 8");
    if (N_Omega < 0 || Q_xi <= N_Omega || Q_xi > 1024) return set_error(RSL_EINVAL, "need 0 <= N_Omega < Q_xi <= 1024");
    if (!pos(T0)) return set_error(RSL_EINVAL, "T0 must be > 0");
    rsl_quad* q = new (std::nothrow) rsl_quad();
    if (!q) return set_error(RSL_EINVAL, "out of host memory");
    int rc = build_quadrature(Q_L, Q_xi, N_Omega, T0, q);
    if (rc != RSL_OK) { delete q; return rc; }
    if (!(flags & RSL_QUAD_HOST_ONLY)) {
        const int V = q->V, Q = q->Q, QL = q->QL;
        std::vector<double> wxw(V), pk(QL), L1(QL), xv(V), pv(V), l1v(V), Pv((size_t)(q->NOm + 1) * V);
        for (int k = 0; k < QL; ++k) {
            pk[k] = T0 * q->pbar[k];
            L1[k] = 3.0 - q->pbar[k];
            for (int j = 0; j < Q; ++j) {
                const int v = k * Q + j;
                wxw[v] = q->wxi[j] * q->wL[k];
                xv[v] = q->xi[j];
                pv[v] = pk[k];
                l1v[v] = L1[k];
                for (int m = 0; m <= q->NOm; ++m) Pv[(size_t)m * V + v] = q->Pm[(size_t)m * Q + j];
            }
        }
        const int Qp = (Q + 15) / 16 * 16, RT = Qp / 16, KT = Qp / 4;
        std::vector<double> KPt((size_t)Qp * Qp, 0.0);
        for (int rt = 0; rt < RT; ++rt)
            for (int kk = 0; kk < KT; ++kk)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * rt + l % 16, col = 4 * kk + l / 16;
                    if (row < Q && col < Q) KPt[((size_t)rt * KT + kk) * 64 + l] = q->KP[(size_t)row * Q + col];
                }
        // velocity order by ascending xi_j (so by its sign), radial node inner; as
        // doubles in the table block, converted to int below
        std::vector<double> vpd(V);
        {
            int o = 0;
            for (int j = 0; j < Q; ++j)
                for (int k = 0; k < QL; ++k) vpd[o++] = (double)(k * Q + j);
        }
        // one record of kVrec doubles per velocity (read with scalar loads):
        // xi_j, p_k, L_1(pbar_k), w_j w_k, P_0..P_kMaxNOm(xi_j), xi_j^2,
        // xi_j / 6, then binary32 xi_j and xi_j / 6, binary32 p_k and the sign
        // of xi_j as an int (the layout of kVrec* in rsl_impl.h)
        std::vector<double> vrec((size_t)V * kVrec, 0.0);
        for (int v = 0; v < V; ++v) {
            double* r = vrec.data() + (size_t)v * kVrec;
            r[0] = xv[v];
            r[1] = pv[v];
            r[2] = l1v[v];
            r[3] = wxw[v];
            for (int m = 0; m <= q->NOm; ++m) r[4 + m] = Pv[(size_t)m * V + v];
            r[kVrecXi2] = xv[v] * xv[v];
            r[kVrecXi6] = xv[v] / 6.0;
            const float f32[4] = {(float)xv[v], (float)(xv[v] / 6.0), (float)pv[v], 0.0f};
            std::memcpy(&r[kVrecF32], f32, 3 * sizeof(float));
            const int sgn = xv[v] > 0.0 ? 1 : (xv[v] < 0.0 ? -1 : 0);
            std::memcpy(reinterpret_cast<char*>(&r[kVrecF32]) + 3 * sizeof(float), &sgn, sizeof(int));
        }
        const std::vector<double>* parts[] = {&q->xi, &wxw, &pk, &L1, &q->Pm, &q->ser, &q->thr, &q->KL, &q->KP,
                                              &xv, &pv, &l1v, &Pv, &KPt, &vrec, &vpd};
        constexpr int NP = 16;
        size_t off[NP], total = 0;
        for (int i = 0; i < NP; ++i) {
            off[i] = total;
            total += align_up(parts[i]->size() * sizeof(double), 256);
        }
        if ((rc = hip_check(hipGetDevice(&q->device), "hipGetDevice")) != RSL_OK) { delete q; return rc; }
        if ((rc = hip_check(hipMalloc(&q->dmem, total), "hipMalloc(tables)")) != RSL_OK) { delete q; return rc; }
        std::vector<char> host(total, 0);
        for (int i = 0; i < NP - 1; ++i)
            std::memcpy(host.data() + off[i], parts[i]->data(), parts[i]->size() * sizeof(double));
        for (int v = 0; v < V; ++v) ((int*)(host.data() + off[NP - 1]))[v] = (int)vpd[v];
        rc = hip_check(hipMemcpy(q->dmem, host.data(), total, hipMemcpyHostToDevice), "hipMemcpy(tables)");
        if (rc != RSL_OK) { (void)hipFree(q->dmem); delete q; return rc; }
        char* b = (char*)q->dmem;
        q->dev.xi = (const double*)(b + off[0]);
        q->dev.wxw = (const double*)(b + off[1]);
        q->dev.pk = (const double*)(b + off[2]);
        q->dev.L1 = (const double*)(b + off[3]);
        q->dev.Pm = (const double*)(b + off[4]);
        q->dev.ser = (const double*)(b + off[5]);
        q->dev.thr = (const double*)(b + off[6]);
        q->dev.KL = (const double*)(b + off[7]);
        q->dev.KP = (const double*)(b + off[8]);
        q->dev.xv = (const double*)(b + off[9]);
        q->dev.pv = (const double*)(b + off[10]);
        q->dev.l1v = (const double*)(b + off[11]);
        q->dev.Pv = (const double*)(b + off[12]);
        q->dev.KPt = (const double*)(b + off[13]);
        q->dev.vrec = (const double*)(b + off[14]);
        q->dev.vperm = (const int*)(b + off[15]);
        q->on_device = true;
    }
    *out = q;
    return RSL_OK;
}

void rsl_free_quadrature(rsl_quad* q) {
    if (!q) return;
    if (q->dmem) (void)hipFree(q->dmem);
    delete q;
}

int rsl_quad_table(const rsl_quad* q, int which, double* host_out, int n, int* count) {
    if (!q) return set_error(RSL_EINVAL, "null rsl_quad");
    const std::vector<double>* t = nullptr;
    switch (which) {
        case RSL_TAB_XI: t = &q->xi; break;
        case RSL_TAB_WXI: t = &q->wxi; break;
        case RSL_TAB_PBAR: t = &q->pbar; break;
        case RSL_TAB_WL: t = &q->wL; break;
        case RSL_TAB_KL: t = &q->KL; break;
        case RSL_TAB_KP: t = &q->KP; break;
        default: return set_error(RSL_EINVAL, "unknown table");
    }
    if (count) *count = (int)t->size();
    if (host_out && n > 0) std::memcpy(host_out, t->data(), sizeof(double) * std::min((size_t)n, t->size()));
    return RSL_OK;
}

int rsl_max_dt(const rsl_quad* q, const rsl_problem* p, double* cfl_dt, double* stiff_dt) {
    if (!q || !cfl_dt || !stiff_dt) return set_error(RSL_EINVAL, "null argument");
    int rc = check_problem(q, p);
    if (rc) return rc;
    stability_limits(q, p, cfl_dt, stiff_dt);
    return RSL_OK;
}

int rsl_sizes(const rsl_quad* q, const rsl_problem* p, size_t* f_bytes, size_t* work_bytes) {
    if (!q) return set_error(RSL_EINVAL, "null rsl_quad");
    int rc = check_problem(q, p);
    if (rc) return rc;
    const WorkLayout L = work_layout(q, p);
    if (f_bytes) *f_bytes = L.f_bytes;
    if (work_bytes) *work_bytes = L.total;
    return RSL_OK;
}

int rsl_init(const rsl_quad* q, const rsl_problem* p, void* f_dev, void* work_dev, void* hip_stream) {
    int rc = check_quad(q);
    if (rc || (rc = check_problem(q, p))) return rc;
    if (!f_dev || !work_dev) return set_error(RSL_EINVAL, "null device buffer");
    hipStream_t s = (hipStream_t)hip_stream;
    const WorkLayout L = work_layout(q, p);
    InstDesc d = make_desc(q, p, f_dev, work_dev, 0.0);
    if ((rc = hip_check(hipMemsetAsync((char*)work_dev + L.status_off, 0, 256, s), "clear status"))) return rc;
    if (p->problem == RSL_SOD) {
        if ((rc = launch_boundary_states(d, p->n_L, p->T_L, p->n_R, p->T_R, s))) return rc;
        return launch_sod_init(d, s);
    }
    return launch_bj_init(d, p->n_L, p->T_L, 1.0, s);
}

int rsl_step(const rsl_quad* q, const rsl_problem* p, void* f_dev, void* work_dev, double* t, double dt,
             int nsteps, void* hip_stream) {
    int rc = check_quad(q);
    if (rc || (rc = check_problem(q, p))) return rc;
    if (!f_dev || !work_dev || !t) return set_error(RSL_EINVAL, "null argument");
    if (nsteps < 0) return set_error(RSL_EINVAL, "nsteps < 0");
    if ((rc = check_stability(q, p, dt))) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    InstDesc d = make_desc(q, p, f_dev, work_dev, dt);
    if (p->problem == RSL_SOD) {
        for (int it = 0; it < nsteps; ++it)
            for (int st = 1; st <= 3; ++st)
                if ((rc = launch_sod_stage(d, st, s, 3 * it + st - 1))) return rc;
    } else if (nsteps > 0) {
        if ((rc = launch_bj_steps(d, *t, dt, nsteps, s))) return rc;
    }
    *t += nsteps * dt;
    return RSL_OK;
}

int rsl_step_imex(const rsl_quad* q, const rsl_problem* p, void* f_dev, void* work_dev, double* t, double dt,
                  int nsteps, void* hip_stream) {
    int rc = check_quad(q);
    if (rc || (rc = check_problem(q, p))) return rc;
    if (p->problem != RSL_SOD) return set_error(RSL_EUNSUPPORTED, "IMEX steps are built for the Sod problem");
    if (!f_dev || !work_dev || !t) return set_error(RSL_EINVAL, "null argument");
    if (nsteps < 0) return set_error(RSL_EINVAL, "nsteps < 0");
    if ((rc = check_cfl(q, p, dt))) return rc;
    InstDesc d = make_desc(q, p, f_dev, work_dev, dt);
    if (nsteps > 0 && (rc = launch_imex_steps(d, p->dtype, nsteps, (hipStream_t)hip_stream))) return rc;
    *t += nsteps * dt;
    return RSL_OK;
}

int rsl_moments(const rsl_quad* q, const rsl_problem* p, const void* f_dev, void* work_dev, double* out_dev,
                int fields, void* hip_stream) {
    int rc = check_quad(q);
    if (rc || (rc = check_problem(q, p))) return rc;
    if (!f_dev || !work_dev || !out_dev) return set_error(RSL_EINVAL, "null device buffer");
    if (fields != RSL_MOM_RAW5 && fields != RSL_MOM_ALL) return set_error(RSL_EINVAL, "fields must be RSL_MOM_RAW5 or RSL_MOM_ALL");
    InstDesc d = make_desc(q, p, (void*)f_dev, work_dev, 0.0);
    if (p->problem == RSL_SOD) return launch_sod_moments(d, f_dev, out_dev, fields, (hipStream_t)hip_stream);
    return launch_bj_moments(d, f_dev, out_dev, fields, (hipStream_t)hip_stream);
}

int rsl_status(const rsl_quad* q, const rsl_problem* p, void* work_dev, void* hip_stream) {
    int rc = check_quad(q);
    if (rc || (rc = check_problem(q, p))) return rc;
    if (!work_dev) return set_error(RSL_EINVAL, "null work buffer");
    hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    unsigned word = 0;
    const WorkLayout L = work_layout(q, p);
    if ((rc = hip_check(hipMemcpy(&word, (char*)work_dev + L.status_off, sizeof(word), hipMemcpyDeviceToHost),
                        "read status")))
        return rc;
    if (word & 1u) return set_error(RSL_ENONFINITE, "a cell reached an unphysical state (Landau frame undefined)");
    if (word & 2u) return set_error(RSL_ENONFINITE, "a population became non-finite");
    return RSL_OK;
}

}  // extern "C"
