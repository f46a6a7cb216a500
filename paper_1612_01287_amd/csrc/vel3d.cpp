// Host side of the velocity sets with azimuthal nodes: building the node
// records and the rsl_feq3 / rsl_moments3 entry points (include/rsl.h).
#include <cmath>
#include <new>
#include <vector>

#include "rsl_impl.h"

using namespace rsl;

namespace {

constexpr int kMaxQphi = 256;

int check_device(const rsl_quad3* q) {
    int dev = -1;
    const int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc != RSL_OK) return rc;
    if (dev != q->device) return set_error(RSL_EINVAL, "the velocity set lives on another HIP device");
    return RSL_OK;
}

}  // namespace

extern "C" {

int rsl_make_quadrature3(int Q_L, int Q_xi, int Q_phi, int N_Omega, double T0, rsl_quad3** out) {
    if (!out) return set_error(RSL_EINVAL, "null output pointer");
    *out = nullptr;
    if (Q_phi < 1 || Q_phi > kMaxQphi) return set_error(RSL_EINVAL, "need 1 <= Q_phi <= 256");
    rsl_quad* base = nullptr;
    int rc = rsl_make_quadrature(Q_L, Q_xi, 1, N_Omega, T0, 0, &base);
    if (rc != RSL_OK) return rc;
    rsl_quad3* q = new (std::nothrow) rsl_quad3();
    if (!q) {
        rsl_free_quadrature(base);
        return set_error(RSL_EINVAL, "out of host memory");
    }
    q->base = base;
    q->Qphi = Q_phi;
    q->A = Q_xi * Q_phi;
    q->V = Q_L * q->A;
    q->device = base->device;
    // angular records: unit direction (sin theta_j cos phi_l, sin theta_j sin
    // phi_l, xi_j) and w_j / Q_phi, phi_l = 2 pi l / Q_phi (equal weights)
    std::vector<double> rec((size_t)4 * q->A + 4 * Q_L, 0.0);
    const double twopi = 6.283185307179586476925286766559;
    for (int l = 0; l < Q_phi; ++l) {
        const double ph = twopi * l / Q_phi;
        const double cph = std::cos(ph), sph = std::sin(ph);
        for (int j = 0; j < Q_xi; ++j) {
            const double xi = base->xi[j], s = std::sqrt(1.0 - xi * xi);
            double* r = rec.data() + 4 * ((size_t)l * Q_xi + j);
            r[0] = s * cph;
            r[1] = s * sph;
            r[2] = xi;
            r[3] = base->wxi[j] / Q_phi;
        }
    }
    for (int k = 0; k < Q_L; ++k) {
        double* r = rec.data() + 4 * (size_t)q->A + 4 * k;
        r[0] = T0 * base->pbar[k];
        r[1] = base->wL[k];
        r[2] = 3.0 - base->pbar[k];
    }
    rc = hip_check(hipMalloc(&q->dmem, rec.size() * sizeof(double)), "hipMalloc(velocity set 3)");
    if (rc == RSL_OK)
        rc = hip_check(hipMemcpy(q->dmem, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice),
                       "hipMemcpy(velocity set 3)");
    if (rc != RSL_OK) {
        rsl_free_quadrature3(q);
        return rc;
    }
    q->dev.arec = (const double*)q->dmem;
    q->dev.rrec = q->dev.arec + 4 * (size_t)q->A;
    q->dev.ser = base->dev.ser;
    q->dev.thr = base->dev.thr;
    q->dev.A = q->A;
    q->dev.QL = Q_L;
    q->dev.NOm = base->NOm;
    q->dev.T0 = base->T0;
    q->dev.beta_series = base->beta_series;
    *out = q;
    return RSL_OK;
}

void rsl_free_quadrature3(rsl_quad3* q) {
    if (!q) return;
    if (q->dmem) (void)hipFree(q->dmem);
    rsl_free_quadrature(q->base);
    delete q;
}

int rsl_quad3_velocities(const rsl_quad3* q) {
    if (!q) return set_error(RSL_EINVAL, "null velocity set");
    return q->V;
}

int rsl_feq3(const rsl_quad3* q, const double* state_dev, int ncell, int dtype, void* f_dev, int pitch,
             void* hip_stream) {
    if (!q) return set_error(RSL_EINVAL, "null velocity set");
    if (ncell < 0 || pitch < ncell) return set_error(RSL_EINVAL, "need 0 <= ncell <= pitch");
    if (dtype != RSL_F64 && dtype != RSL_F32) return set_error(RSL_EINVAL, "dtype must be RSL_F64 or RSL_F32");
    if (ncell == 0) return RSL_OK;
    if (!state_dev || !f_dev) return set_error(RSL_EINVAL, "null device buffer");
    const int rc = check_device(q);
    if (rc != RSL_OK) return rc;
    return launch_feq3(q->dev, state_dev, ncell, dtype, f_dev, pitch, (hipStream_t)hip_stream);
}

int rsl_moments3(const rsl_quad3* q, const void* f_dev, int dtype, int ncell, int pitch, double* out_dev,
                 void* hip_stream) {
    if (!q) return set_error(RSL_EINVAL, "null velocity set");
    if (ncell < 0 || pitch < ncell) return set_error(RSL_EINVAL, "need 0 <= ncell <= pitch");
    if (dtype != RSL_F64 && dtype != RSL_F32) return set_error(RSL_EINVAL, "dtype must be RSL_F64 or RSL_F32");
    if (ncell == 0) return RSL_OK;
    if (!f_dev || !out_dev) return set_error(RSL_EINVAL, "null device buffer");
    const int rc = check_device(q);
    if (rc != RSL_OK) return rc;
    return launch_moments3(q->dev, f_dev, dtype, ncell, pitch, out_dev, (hipStream_t)hip_stream);
}

}  // extern "C"
