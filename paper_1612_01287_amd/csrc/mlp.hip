// Learned T^{mu nu} correction for low-order velocity sets (not part of the
// paper): per-cell features, a 81 -> 128 -> 128 -> 3 ReLU network in bf16 with
// fp32 accumulation on the matrix cores (v_mfma_f32_16x16x16bf16_1k), its
// backward pass, Adam, and the application of the correction.
//
// Parameter layout (fp32 master copy and bf16 compute copy alike):
//   W1 [81][128], b1 [128], W2 [128][128], b2 [128], W3 [128][3], b3 [3]
// (row = input index), 27395 values.
//
// MFMA operand layout (16x16x16, wave64), with l the lane:
//   A (16 x 16, row-major M x K): lane l holds A[l % 16][4 (l / 16) + e], e = 0..3
//   B (16 x 16, K x N):           lane l holds B[4 (l / 16) + e][l % 16]
//   D (16 x 16, f32):             lane l holds D[4 (l / 16) + r][l % 16], r = 0..3
#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <mutex>

#include "rsl_math.h"

namespace rsl {

namespace {

constexpr int NI = RSL_MLP_IN, NH = RSL_MLP_HIDDEN, NO = RSL_MLP_OUT;
constexpr int KI = 96;                 // NI padded to a multiple of 16
constexpr int OP = 16;                 // NO padded to one tile
constexpr int OFF_W1 = 0, OFF_B1 = NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NO, NPARAM = OFF_B3 + NO;
static_assert(NPARAM == RSL_MLP_NPARAM, "parameter count");
constexpr int ROWS = 64;               // samples per workgroup tile
constexpr int TPB = 256;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
    // round to nearest even (finite inputs)
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Row (within the 16 x 16 tile) of accumulator element r of lane l.
__device__ __forceinline__ int drow(int lane, int r) { return 4 * (lane >> 4) + r; }

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// A fragment from a row-major bf16 matrix in LDS (ld = row stride in elements).
__device__ __forceinline__ s4 frag_a(const unsigned short* m, int ld, int r0, int k0, int lane) {
    const unsigned short* p = m + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
    s4 v;
    v[0] = (short)p[0]; v[1] = (short)p[1]; v[2] = (short)p[2]; v[3] = (short)p[3];
    return v;
}
// A fragment of the transpose of a row-major matrix: A[i][k] = m[k][i].
__device__ __forceinline__ s4 frag_at(const unsigned short* m, int ld, int r0, int k0, int lane) {
    s4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (short)m[(k0 + 4 * (lane >> 4) + e) * ld + r0 + (lane & 15)];
    return v;
}
// B fragment from a row-major (K x N) matrix.
__device__ __forceinline__ s4 frag_b(const unsigned short* m, int ld, int k0, int c0, int lane) {
    s4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (short)m[(k0 + 4 * (lane >> 4) + e) * ld + c0 + (lane & 15)];
    return v;
}
// B fragment of the transpose of a row-major (N x K) matrix: B[k][n] = m[n][k].
__device__ __forceinline__ s4 frag_bt(const unsigned short* m, int ld, int k0, int c0, int lane) {
    const unsigned short* p = m + (c0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
    s4 v;
    v[0] = (short)p[0]; v[1] = (short)p[1]; v[2] = (short)p[2]; v[3] = (short)p[3];
    return v;
}

// Weights in LDS as bf16: W1 [KI][NH] (rows >= NI zero), W2 [NH][NH], W3 [NH][OP] (cols >= NO zero)
struct WL {
    unsigned short w1[KI * NH];
    unsigned short w2[NH * NH];
    unsigned short w3[NH * OP];
    float b1[NH], b2[NH], b3[OP];
};
struct AL {                       // one tile of activations
    unsigned short x[ROWS * KI];
    unsigned short h1[ROWS * NH];
    unsigned short h2[ROWS * NH];
};

__device__ void load_weights(WL& W, const unsigned short* pb) {
    for (int e = threadIdx.x; e < KI * NH; e += blockDim.x) {
        const int r = e / NH, c = e - r * NH;
        W.w1[e] = r < NI ? pb[OFF_W1 + r * NH + c] : 0;
    }
    for (int e = threadIdx.x; e < NH * NH; e += blockDim.x) W.w2[e] = pb[OFF_W2 + e];
    for (int e = threadIdx.x; e < NH * OP; e += blockDim.x) {
        const int r = e / OP, c = e - r * OP;
        W.w3[e] = c < NO ? pb[OFF_W3 + r * NO + c] : 0;
    }
    for (int e = threadIdx.x; e < NH; e += blockDim.x) {
        W.b1[e] = from_bf16(pb[OFF_B1 + e]);
        W.b2[e] = from_bf16(pb[OFF_B2 + e]);
    }
    for (int e = threadIdx.x; e < OP; e += blockDim.x) W.b3[e] = e < NO ? from_bf16(pb[OFF_B3 + e]) : 0.f;
}

// Forward pass over rows [r0, r0 + ROWS): every wave owns 16 rows.
__device__ void forward_tile(const WL& W, AL& A, const float* __restrict__ x, int n, int r0, float* __restrict__ y,
                             unsigned short* __restrict__ h1g, unsigned short* __restrict__ h2g) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < ROWS * KI; e += blockDim.x) {
        const int r = e / KI, c = e - r * KI;
        A.x[e] = (r0 + r < n && c < NI) ? to_bf16(x[(size_t)(r0 + r) * NI + c]) : 0;
    }
    __syncthreads();
    const int rw = 16 * w;
    // layer 1
    for (int ct = 0; ct < NH / 16; ++ct) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < KI / 16; ++kt)
            acc = mfma(frag_a(A.x, KI, rw, 16 * kt, lane), frag_b(W.w1, NH, 16 * kt, 16 * ct, lane), acc);
        const int col = 16 * ct + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rw + drow(lane, r);
            A.h1[row * NH + col] = to_bf16(fmaxf(acc[r] + W.b1[col], 0.f));
        }
    }
    __syncthreads();
    // layer 2
    for (int ct = 0; ct < NH / 16; ++ct) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < NH / 16; ++kt)
            acc = mfma(frag_a(A.h1, NH, rw, 16 * kt, lane), frag_b(W.w2, NH, 16 * kt, 16 * ct, lane), acc);
        const int col = 16 * ct + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rw + drow(lane, r);
            A.h2[row * NH + col] = to_bf16(fmaxf(acc[r] + W.b2[col], 0.f));
        }
    }
    __syncthreads();
    // layer 3
    {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < NH / 16; ++kt)
            acc = mfma(frag_a(A.h2, NH, rw, 16 * kt, lane), frag_b(W.w3, OP, 16 * kt, 0, lane), acc);
        const int col = lane & 15;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + rw + drow(lane, r);
            if (col < NO && row < n) y[(size_t)row * NO + col] = acc[r] + W.b3[col];
        }
    }
    if (h1g)
        for (int e = threadIdx.x; e < ROWS * NH; e += blockDim.x) {
            const int r = e / NH;
            if (r0 + r < n) {
                h1g[(size_t)r0 * NH + e] = A.h1[e];
                h2g[(size_t)r0 * NH + e] = A.h2[e];
            }
        }
    __syncthreads();
}

__global__ void __launch_bounds__(TPB) mlp_forward_kernel(const unsigned short* __restrict__ pb,
                                                          const float* __restrict__ x, int n, float* __restrict__ y,
                                                          unsigned short* __restrict__ h1g,
                                                          unsigned short* __restrict__ h2g) {
    extern __shared__ char smem[];
    WL& W = *(WL*)smem;
    AL& A = *(AL*)(smem + sizeof(WL));
    load_weights(W, pb);
    __syncthreads();
    for (int r0 = blockIdx.x * ROWS; r0 < n; r0 += gridDim.x * ROWS) forward_tile(W, A, x, n, r0, y, h1g, h2g);
}

// Backward for loss = mean over n samples and 3 outputs of (y - t)^2.
// Per tile: dY, dZ2 = (dY W3^T) .* [h2 > 0], dZ1 = (dZ2 W2^T) .* [h1 > 0].
// Workgroup b sums the gradient of its tiles (b, b + G, ...) into its own
// fp32 row part[b][NPARAM] (every entry owned by one lane: no atomics); a
// second kernel adds the G rows in a fixed order.
struct BL {
    unsigned short x[ROWS * KI];
    unsigned short h1[ROWS * NH];
    unsigned short h2[ROWS * NH];
    unsigned short dy[ROWS * OP];
    unsigned short dz2[ROWS * NH];
    unsigned short dz1[ROWS * NH];
    float dyf[ROWS * OP];          // dY in fp32 (the output bias gradient)
};

// Workgroups of the backward kernel (rows of partial gradients).
constexpr int kBwdGroups = 256;
int bwd_groups(int n) { return std::max(1, std::min(kBwdGroups, (n + ROWS - 1) / ROWS)); }

__global__ void __launch_bounds__(TPB) mlp_backward_kernel(const unsigned short* __restrict__ pb,
                                                           const float* __restrict__ x,
                                                           const unsigned short* __restrict__ h1g,
                                                           const unsigned short* __restrict__ h2g,
                                                           const float* __restrict__ y, const float* __restrict__ t,
                                                           int n, float* __restrict__ part) {
    extern __shared__ char smem[];
    WL& W = *(WL*)smem;
    BL& B = *(BL*)(smem + sizeof(WL));
    load_weights(W, pb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const float scale = 2.0f / ((float)n * NO);
    float* __restrict__ g = part + (size_t)blockIdx.x * NPARAM;
    for (int r0 = blockIdx.x * ROWS; r0 < n; r0 += gridDim.x * ROWS) {
        const bool first = r0 == blockIdx.x * ROWS;     // the row starts from this tile's values
        auto put = [&](int i, float v) { g[i] = first ? v : g[i] + v; };
        __syncthreads();
        for (int e = threadIdx.x; e < ROWS * KI; e += blockDim.x) {
            const int r = e / KI, c = e - r * KI;
            B.x[e] = (r0 + r < n && c < NI) ? to_bf16(x[(size_t)(r0 + r) * NI + c]) : 0;
        }
        for (int e = threadIdx.x; e < ROWS * NH; e += blockDim.x) {
            const bool in = r0 + e / NH < n;
            B.h1[e] = in ? h1g[(size_t)r0 * NH + e] : 0;
            B.h2[e] = in ? h2g[(size_t)r0 * NH + e] : 0;
        }
        for (int e = threadIdx.x; e < ROWS * OP; e += blockDim.x) {
            const int r = e / OP, c = e - r * OP;
            float v = 0.f;
            if (r0 + r < n && c < NO) v = scale * (y[(size_t)(r0 + r) * NO + c] - t[(size_t)(r0 + r) * NO + c]);
            B.dy[e] = to_bf16(v);
            B.dyf[e] = v;
        }
        __syncthreads();
        const int rw = 16 * w;
        // dZ2 = dY W3^T .* [h2 > 0]   (rows rw.., K = OP, N = NH)
        for (int ct = 0; ct < NH / 16; ++ct) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(frag_a(B.dy, OP, rw, 0, lane), frag_bt(W.w3, OP, 0, 16 * ct, lane), acc);
            const int col = 16 * ct + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rw + drow(lane, r);
                const float v = B.h2[row * NH + col] != 0 ? acc[r] : 0.f;
                B.dz2[row * NH + col] = to_bf16(v);
            }
        }
        __syncthreads();
        // dZ1 = dZ2 W2^T .* [h1 > 0]
        for (int ct = 0; ct < NH / 16; ++ct) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int kt = 0; kt < NH / 16; ++kt)
                acc = mfma(frag_a(B.dz2, NH, rw, 16 * kt, lane), frag_bt(W.w2, NH, 16 * kt, 16 * ct, lane), acc);
            const int col = 16 * ct + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rw + drow(lane, r);
                const float v = B.h1[row * NH + col] != 0 ? acc[r] : 0.f;
                B.dz1[row * NH + col] = to_bf16(v);
            }
        }
        __syncthreads();
        // weight gradients: dW = act^T dZ over the ROWS samples of the tile
        // (M = fan-in, N = fan-out, K = ROWS); tiles dealt round-robin to waves
        const int nt3 = NH / 16, nt2 = (NH / 16) * (NH / 16), nt1 = (KI / 16) * (NH / 16);
        for (int tt = w; tt < nt3 + nt2 + nt1; tt += TPB / 64) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            const unsigned short *act, *dz;
            int lda, ldz, mi, nj, goff, fan_in, fan_out, ldw;
            if (tt < nt3) { act = B.h2; lda = NH; dz = B.dy; ldz = OP; mi = tt; nj = 0; goff = OFF_W3; fan_in = NH; fan_out = NO; ldw = NO; }
            else if (tt < nt3 + nt2) { const int q = tt - nt3; act = B.h1; lda = NH; dz = B.dz2; ldz = NH; mi = q / (NH / 16); nj = q % (NH / 16); goff = OFF_W2; fan_in = NH; fan_out = NH; ldw = NH; }
            else { const int q = tt - nt3 - nt2; act = B.x; lda = KI; dz = B.dz1; ldz = NH; mi = q / (NH / 16); nj = q % (NH / 16); goff = OFF_W1; fan_in = NI; fan_out = NH; ldw = NH; }
            for (int kt = 0; kt < ROWS / 16; ++kt)
                acc = mfma(frag_at(act, lda, 16 * mi, 16 * kt, lane), frag_b(dz, ldz, 16 * kt, 16 * nj, lane), acc);
            const int col = 16 * nj + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * mi + drow(lane, r);
                if (row < fan_in && col < fan_out) put(goff + row * ldw + col, acc[r]);
            }
        }
        // bias gradients: hidden layers from the bf16 dZ, the output layer from dY in fp32
        for (int c = threadIdx.x; c < 2 * NH + NO; c += blockDim.x) {
            float s = 0.f;
            if (c < 2 * NH) {
                const unsigned short* dz = c < NH ? B.dz1 : B.dz2;
                const int cc = c % NH;
                for (int r = 0; r < ROWS; ++r) s += from_bf16(dz[r * NH + cc]);
                put((c < NH ? OFF_B1 : OFF_B2) + cc, s);
            } else {
                const int cc = c - 2 * NH;
                for (int r = 0; r < ROWS; ++r) s += B.dyf[r * OP + cc];
                put(OFF_B3 + cc, s);
            }
        }
    }
}

// grad[p] = sum over the G partial rows, in row order.
__global__ void grad_reduce_kernel(const float* __restrict__ part, int G, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float s = 0.f;
    for (int b = 0; b < G; ++b) s += part[(size_t)b * NPARAM + p];
    grad[p] = s;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, unsigned short* __restrict__ pb, int np, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = to_bf16(pi);
}

__global__ void to_bf16_kernel(const float* __restrict__ p, unsigned short* __restrict__ pb, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) pb[i] = to_bf16(p[i]);
}

// Features: moments M_{a,r} (a in {0,1}, r in 0..7) of cells s-2..s+2 (ghosts
// copy the end cells), normalised by the centre cell's N^0 (a = 0) and T^00
// (a = 1), then log tau.  One thread per cell; the block's cells and halo
// have their moments computed once into LDS.
template <typename Tf>
__global__ void __launch_bounds__(TPB) features_kernel(InstDesc d, const Tf* __restrict__ f, double log_tau,
                                                       const float* __restrict__ shift,
                                                       const float* __restrict__ scale, float* __restrict__ out) {
    __shared__ double Ms[(TPB + 4) * 16];
    const int s0 = blockIdx.x * TPB;
    for (int t = threadIdx.x; t < TPB + 4; t += blockDim.x) {
        const int s = min(max(s0 - 2 + t, 0), d.nz - 1);
        double M[16];
        for (int q = 0; q < 16; ++q) M[q] = 0.0;
        for (int v = 0; v < d.V; ++v) {
            const double fv = (double)f[(size_t)v * d.pitch + s];
            const double x = d.tab.xv[v], p = d.tab.pv[v];
            double xr = 1.0;
            for (int r = 0; r < 8; ++r) {
                M[r] += xr * fv;
                M[8 + r] += p * xr * fv;
                xr *= x;
            }
        }
        for (int q = 0; q < 16; ++q) Ms[t * 16 + q] = M[q];
    }
    __syncthreads();
    const int s = s0 + threadIdx.x;
    if (s >= d.nz) return;
    const double* c = Ms + (threadIdx.x + 2) * 16;
    const double n0 = c[0], e0 = c[8];
    float* o = out + (size_t)s * NI;
    float x[NI];
    for (int off = 0; off < 5; ++off) {
        const double* m = Ms + (threadIdx.x + off) * 16;
        for (int r = 0; r < 8; ++r) {
            x[off * 16 + r] = (float)(m[r] / n0);
            x[off * 16 + 8 + r] = (float)(m[8 + r] / e0);
        }
    }
    x[80] = (float)log_tau;
    for (int i = 0; i < NI; ++i) o[i] = shift ? (x[i] - shift[i]) / scale[i] : x[i];
}

// mode 0: t = (T_hi - T_lo) / T^00_lo; mode 1: T_corr = T_lo + y T^00_lo.
// Moment rows are RSL_NMOM doubles (T^00, T^0z, T^zz at 2, 3, 4).
__global__ void tmunu_kernel(const double* __restrict__ mlo, const double* __restrict__ mhi,
                             const float* __restrict__ y, int n, int mode, float* __restrict__ tout,
                             double* __restrict__ tcorr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* a = mlo + (size_t)i * RSL_NMOM;
    const double e = a[2];
    for (int q = 0; q < NO; ++q) {
        if (mode == 0) tout[(size_t)i * NO + q] = (float)((mhi[(size_t)i * RSL_NMOM + 2 + q] - a[2 + q]) / e);
        else tcorr[(size_t)i * NO + q] = a[2 + q] + (double)y[(size_t)i * NO + q] * e;
    }
}

// Out-of-range guard: flag |x_c - mu_c| > k sigma_c for any feature c of any row.
__global__ void guard_kernel(const float* __restrict__ x, int n, const float* __restrict__ lo,
                             const float* __restrict__ hi, unsigned* __restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool out = false;
    for (int c = 0; c < NI; ++c) {
        const float v = x[(size_t)i * NI + c];
        out |= !(v >= lo[c] && v <= hi[c]);
    }
    if (out) atomicOr(flag, 1u);
}

// In-loop feedback.  A change of (T^00, T^0z, T^zz) goes along
//   b_c[v] = w_j w_k L_1(pbar_k) xi_j^c (c = 0, 1, 2), which carries no N^0, N^z,
// a change of (N^0, N^z) along
//   b'_c[v] = w_j w_k (4 - pbar_k) xi_j^c (c = 0, 1), which carries no T^{mu nu};
// tinv, ninv invert the moment matrices of the two families (per velocity set).
struct InjectConst {
    double tinv[9], ninv[4];
};

// f += df with (dT^00, dT^0z, dT^zz) = y T^00 per cell (the network's output
// convention), T^00 the cell's own.
template <typename Tf>
__global__ void __launch_bounds__(TPB) inject_kernel(InstDesc d, Tf* __restrict__ f, const float* __restrict__ y,
                                                     InjectConst K) {
    const int s = blockIdx.x * TPB + threadIdx.x;
    if (s >= d.nz) return;
    double e = 0.0;
    for (int v = 0; v < d.V; ++v) e = fma(d.tab.pv[v], (double)f[(size_t)v * d.pitch + s], e);
    const double dT[3] = {y[3 * (size_t)s] * e, y[3 * (size_t)s + 1] * e, y[3 * (size_t)s + 2] * e};
    double a[3];
    for (int r = 0; r < 3; ++r) a[r] = K.tinv[3 * r] * dT[0] + K.tinv[3 * r + 1] * dT[1] + K.tinv[3 * r + 2] * dT[2];
    for (int v = 0; v < d.V; ++v) {
        const double x = d.tab.xv[v];
        const double df = d.tab.wxw[v] * d.tab.l1v[v] * fma(fma(a[2], x, a[1]), x, a[0]);
        Tf& fv = f[(size_t)v * d.pitch + s];
        fv = (Tf)((double)fv + df);
    }
}

// Low-order populations fl with the N^mu, T^{mu nu} of the high-order fh (same
// cells): the low-order equilibrium of fh's Landau frame (eqs. E_landau,
// u_landau, feq_trunc) as stored, plus the change along b and b' that carries
// the rest of both.  NaN populations for a cell without a Landau frame.
template <typename Th, typename Tl>
__global__ void __launch_bounds__(TPB) project_kernel(InstDesc dh, const Th* __restrict__ fh, InstDesc dl,
                                                      Tl* __restrict__ fl, InjectConst K) {
    const int s = blockIdx.x * TPB + threadIdx.x;
    if (s >= dl.nz) return;
    double M[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < dh.V; ++v) {
        const double fv = (double)fh[(size_t)v * dh.pitch + s];
        const double x = dh.tab.xv[v], pf = dh.tab.pv[v] * fv;
        M[0] += fv;
        M[1] = fma(x, fv, M[1]);
        M[2] += pf;
        M[3] = fma(x, pf, M[3]);
        M[4] = fma(x * x, pf, M[4]);
    }
    const CellState cs = landau(M[0], M[1], M[2], M[3], M[4]);
    if (!cs.ok) {
        for (int v = 0; v < dl.V; ++v) fl[(size_t)v * dl.pitch + s] = (Tl)__builtin_nan("");
        return;
    }
    const int nt = series_terms(fmin(cs.beta * cs.beta, dl.beta_series * dl.beta_series), dl.tab.thr);
    double c0[kMaxNOm + 1], c1[kMaxNOm + 1];
    feq_coef(cs.n, cs.T, cs.beta, cs.gamma, dl.T0, dl.NOm, dl.beta_series, dl.tab.ser, nt, c0, c1);
    double E[5] = {0.0, 0.0, 0.0, 0.0, 0.0};     // moments of the stored equilibrium
    for (int v = 0; v < dl.V; ++v) {
        double g = 0.0, h = 0.0;
        for (int m = 0; m <= dl.NOm; ++m) {
            const double P = dl.tab.Pv[(size_t)m * dl.V + v];
            g = fma(P, c0[m], g);
            h = fma(P, c1[m], h);
        }
        const Tl fe = (Tl)(dl.tab.wxw[v] * fma(dl.tab.l1v[v], h, g));
        fl[(size_t)v * dl.pitch + s] = fe;
        const double fd = (double)fe, x = dl.tab.xv[v], pf = dl.tab.pv[v] * fd;
        E[0] += fd;
        E[1] = fma(x, fd, E[1]);
        E[2] += pf;
        E[3] = fma(x, pf, E[3]);
        E[4] = fma(x * x, pf, E[4]);
    }
    const double dN[2] = {M[0] - E[0], M[1] - E[1]}, dT[3] = {M[2] - E[2], M[3] - E[3], M[4] - E[4]};
    double a[3], b[2];
    for (int r = 0; r < 3; ++r) a[r] = K.tinv[3 * r] * dT[0] + K.tinv[3 * r + 1] * dT[1] + K.tinv[3 * r + 2] * dT[2];
    for (int r = 0; r < 2; ++r) b[r] = K.ninv[2 * r] * dN[0] + K.ninv[2 * r + 1] * dN[1];
    for (int v = 0; v < dl.V; ++v) {
        const double x = dl.tab.xv[v], pb = dl.tab.pv[v] / dl.T0;
        const double df = dl.tab.wxw[v] * (dl.tab.l1v[v] * fma(fma(a[2], x, a[1]), x, a[0]) +
                                           (4.0 - pb) * fma(b[1], x, b[0]));
        Tl& fv = fl[(size_t)v * dl.pitch + s];
        fv = (Tl)((double)fv + df);
    }
}

// The two moment matrices of a velocity set (from its host tables), inverted.
int inject_const(const rsl_quad* q, InjectConst* K) {
    double S[5] = {0.0, 0.0, 0.0, 0.0, 0.0};          // sum_j w_j xi_j^r, r = 0..4
    for (int j = 0; j < q->Q; ++j) {
        double xr = 1.0;
        for (int r = 0; r < 5; ++r) {
            S[r] += q->wxi[j] * xr;
            xr *= q->xi[j];
        }
    }
    double G1 = 0.0, H0 = 0.0;                        // sum_k w_k p_k L_1, sum_k w_k (4 - pbar_k)
    for (int k = 0; k < q->QL; ++k) {
        G1 += q->wL[k] * q->T0 * q->pbar[k] * (3.0 - q->pbar[k]);
        H0 += q->wL[k] * (4.0 - q->pbar[k]);
    }
    // T block: rows (T^00, T^0z, T^zz) = G1 (S_c, S_{c+1}, S_{c+2}) for b_c
    double A[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) A[r][c] = G1 * S[r + c];
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    // N block: rows (N^0, N^z) = H0 (S_c, S_{c+1}) for b'_c
    const double n00 = H0 * S[0], n01 = H0 * S[1], n11 = H0 * S[2];
    const double detn = n00 * n11 - n01 * n01;
    // singular when the polar rule cannot tell 1, xi, xi^2 apart (Q_xi < 3):
    // the determinants vanish to rounding relative to their diagonals
    if (!(fabs(det) > 1e-9 * fabs(A[0][0] * A[1][1] * A[2][2])) || !(fabs(detn) > 1e-9 * fabs(n00 * n11)) ||
        !std::isfinite(det) || !std::isfinite(detn))
        return set_error(RSL_EUNSUPPORTED, "the feedback basis is singular for this velocity set (need Q_xi >= 3)");
    const double id = 1.0 / det;
    K->tinv[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * id;
    K->tinv[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    K->tinv[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    K->tinv[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * id;
    K->tinv[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    K->tinv[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    K->tinv[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * id;
    K->tinv[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    K->tinv[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    K->ninv[0] = n11 / detn;
    K->ninv[1] = -n01 / detn;
    K->ninv[2] = -n01 / detn;
    K->ninv[3] = n00 / detn;
    return RSL_OK;
}

constexpr size_t kFwdLds = sizeof(WL) + sizeof(AL);
constexpr size_t kBwdLds = sizeof(WL) + sizeof(BL);

int grid_rows(int n) { return std::max(1, std::min(1024, (n + ROWS - 1) / ROWS)); }

// Scratch of rsl_mlp_backward_noalloc: the partial-gradient rows of the
// backward kernel's workgroups.  bwd_groups() never exceeds kBwdGroups, so
// this holds what any sample count needs (28 MB).  Each device holds its own
// copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchFloats = (size_t)kBwdGroups * NPARAM;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per device.
int scratch_address(float** out) {
    int dev = -1;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return set_error(RSL_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if ((rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return rc;
        g_scratch_dev[dev] = (float*)p;
    }
    *out = g_scratch_dev[dev];
    return RSL_OK;
}

// The backward pass with partial-gradient rows in `work` (bwd_groups(n) x NPARAM floats).
int launch_backward(const unsigned short* params_bf16, const float* x, const unsigned short* h1,
                    const unsigned short* h2, const float* y, const float* t, int n, float* grad, float* work,
                    hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)mlp_backward_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBwdLds);
    if (attr != hipSuccess) return hip_check(attr, "hipFuncSetAttribute(mlp_backward_kernel)");
    const int G = bwd_groups(n);
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(G), dim3(TPB), kBwdLds, s, params_bf16, x, h1, h2, y, t, n, work);
    int rc = hip_check(hipGetLastError(), "mlp_backward_kernel launch");
    if (rc) return rc;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, work, G, grad);
    return hip_check(hipGetLastError(), "grad_reduce_kernel launch");
}

}  // namespace

}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_mlp_features(const rsl_quad* q, const rsl_problem* p, const void* f_dev, double log_tau,
                     const float* shift_dev, const float* scale_dev, float* feat_dev,
                     void* hip_stream) {
    if (!q || !p || !f_dev || !feat_dev) return set_error(RSL_EINVAL, "null argument");
    if (!q->on_device) return set_error(RSL_EINVAL, "rsl_quad was built with RSL_QUAD_HOST_ONLY");
    if (p->problem != RSL_SOD) return set_error(RSL_EINVAL, "features are defined for Sod instances");
    if (!shift_dev != !scale_dev) return set_error(RSL_EINVAL, "shift and scale go together");
    InstDesc d = make_desc(q, p, (void*)f_dev, (void*)f_dev, 0.0);
    hipStream_t s = (hipStream_t)hip_stream;
    const dim3 grid((p->nz + TPB - 1) / TPB);
    if (p->dtype == RSL_F64)
        hipLaunchKernelGGL(features_kernel<double>, grid, dim3(TPB), 0, s, d, (const double*)f_dev, log_tau,
                           shift_dev, scale_dev, feat_dev);
    else
        hipLaunchKernelGGL(features_kernel<float>, grid, dim3(TPB), 0, s, d, (const float*)f_dev, log_tau,
                           shift_dev, scale_dev, feat_dev);
    return hip_check(hipGetLastError(), "features_kernel launch");
}

int rsl_mlp_inject(const rsl_quad* q, const rsl_problem* p, void* f_dev, const float* y, void* hip_stream) {
    if (!q || !p || !f_dev || !y) return set_error(RSL_EINVAL, "null argument");
    if (!q->on_device) return set_error(RSL_EINVAL, "rsl_quad was built with RSL_QUAD_HOST_ONLY");
    if (p->problem != RSL_SOD) return set_error(RSL_EINVAL, "the feedback is defined for Sod instances");
    InjectConst K;
    int rc = inject_const(q, &K);
    if (rc) return rc;
    InstDesc d = make_desc(q, p, f_dev, f_dev, 0.0);
    hipStream_t s = (hipStream_t)hip_stream;
    const dim3 grid((p->nz + TPB - 1) / TPB);
    if (p->dtype == RSL_F64)
        hipLaunchKernelGGL(inject_kernel<double>, grid, dim3(TPB), 0, s, d, (double*)f_dev, y, K);
    else
        hipLaunchKernelGGL(inject_kernel<float>, grid, dim3(TPB), 0, s, d, (float*)f_dev, y, K);
    return hip_check(hipGetLastError(), "inject_kernel launch");
}

int rsl_project(const rsl_quad* q_hi, const rsl_problem* p_hi, const void* f_hi, const rsl_quad* q_lo,
                const rsl_problem* p_lo, void* f_lo, void* hip_stream) {
    if (!q_hi || !p_hi || !f_hi || !q_lo || !p_lo || !f_lo) return set_error(RSL_EINVAL, "null argument");
    if (!q_hi->on_device || !q_lo->on_device) return set_error(RSL_EINVAL, "rsl_quad was built with RSL_QUAD_HOST_ONLY");
    if (p_hi->problem != RSL_SOD || p_lo->problem != RSL_SOD)
        return set_error(RSL_EINVAL, "the projection is defined for Sod instances");
    if (p_hi->nz != p_lo->nz) return set_error(RSL_EINVAL, "the two instances must have the same cells");
    InjectConst K;
    int rc = inject_const(q_lo, &K);
    if (rc) return rc;
    InstDesc dh = make_desc(q_hi, p_hi, (void*)f_hi, (void*)f_hi, 0.0);
    InstDesc dl = make_desc(q_lo, p_lo, f_lo, f_lo, 0.0);
    hipStream_t s = (hipStream_t)hip_stream;
    const dim3 grid((p_lo->nz + TPB - 1) / TPB);
    const bool h64 = p_hi->dtype == RSL_F64, l64 = p_lo->dtype == RSL_F64;
    if (h64 && l64)
        hipLaunchKernelGGL((project_kernel<double, double>), grid, dim3(TPB), 0, s, dh, (const double*)f_hi, dl,
                           (double*)f_lo, K);
    else if (h64)
        hipLaunchKernelGGL((project_kernel<double, float>), grid, dim3(TPB), 0, s, dh, (const double*)f_hi, dl,
                           (float*)f_lo, K);
    else if (l64)
        hipLaunchKernelGGL((project_kernel<float, double>), grid, dim3(TPB), 0, s, dh, (const float*)f_hi, dl,
                           (double*)f_lo, K);
    else
        hipLaunchKernelGGL((project_kernel<float, float>), grid, dim3(TPB), 0, s, dh, (const float*)f_hi, dl,
                           (float*)f_lo, K);
    return hip_check(hipGetLastError(), "project_kernel launch");
}

int rsl_mlp_to_bf16(const float* params, unsigned short* params_bf16, void* hip_stream) {
    if (!params || !params_bf16) return set_error(RSL_EINVAL, "null argument");
    hipLaunchKernelGGL(to_bf16_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, params,
                       params_bf16, NPARAM);
    return hip_check(hipGetLastError(), "to_bf16_kernel launch");
}

int rsl_mlp_forward(const unsigned short* params_bf16, const float* x, int n, float* y, unsigned short* h1,
                    unsigned short* h2, void* hip_stream) {
    if (!params_bf16 || !x || !y || n < 0 || (!h1) != (!h2)) return set_error(RSL_EINVAL, "bad argument");
    if (n == 0) return RSL_OK;
    static const hipError_t attr = hipFuncSetAttribute((const void*)mlp_forward_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFwdLds);
    if (attr != hipSuccess) return hip_check(attr, "hipFuncSetAttribute(mlp_forward_kernel)");
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid_rows(n)), dim3(TPB), kFwdLds, (hipStream_t)hip_stream, params_bf16,
                       x, n, y, h1, h2);
    return hip_check(hipGetLastError(), "mlp_forward_kernel launch");
}

size_t rsl_mlp_backward_work(int n) { return n > 0 ? (size_t)bwd_groups(n) * NPARAM : 0; }

int rsl_mlp_backward(const unsigned short* params_bf16, const float* x, const unsigned short* h1,
                     const unsigned short* h2, const float* y, const float* t, int n, float* grad, float* work,
                     void* hip_stream) {
    if (!params_bf16 || !x || !h1 || !h2 || !y || !t || !grad || !work || n <= 0)
        return set_error(RSL_EINVAL, "bad argument");
    return launch_backward(params_bf16, x, h1, h2, y, t, n, grad, work, (hipStream_t)hip_stream);
}

int rsl_mlp_backward_noalloc(const unsigned short* params_bf16, const float* x, const unsigned short* h1,
                             const unsigned short* h2, const float* y, const float* t, int n, float* grad,
                             void* hip_stream) {
    if (!params_bf16 || !x || !h1 || !h2 || !y || !t || !grad || n <= 0)
        return set_error(RSL_EINVAL, "bad argument");
    if ((size_t)bwd_groups(n) * NPARAM > kScratchFloats)
        return set_error(RSL_EINVAL, "partial gradients exceed the library's scratch");
    float* work = nullptr;
    const int rc = scratch_address(&work);
    if (rc) return rc;
    return launch_backward(params_bf16, x, h1, h2, y, t, n, grad, work, (hipStream_t)hip_stream);
}

int rsl_mlp_adam(float* params, const float* grad, float* m, float* v, unsigned short* params_bf16, int step, float lr,
                 float beta1, float beta2, float eps, void* hip_stream) {
    if (!params || !grad || !m || !v || !params_bf16 || step < 1) return set_error(RSL_EINVAL, "bad argument");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, params, grad, m,
                       v, params_bf16, NPARAM, lr, beta1, beta2, eps, c1, c2);
    return hip_check(hipGetLastError(), "adam_kernel launch");
}

int rsl_mlp_tmunu(const double* m_lo, const double* m_hi, const float* y, int n, int mode, float* t_out,
                  double* t_corr, void* hip_stream) {
    if (!m_lo || n < 0 || (mode == 0 && (!m_hi || !t_out)) || (mode == 1 && (!y || !t_corr)) || mode < 0 || mode > 1)
        return set_error(RSL_EINVAL, "bad argument");
    if (n == 0) return RSL_OK;
    hipLaunchKernelGGL(tmunu_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, m_lo, m_hi, y, n, mode,
                       t_out, t_corr);
    return hip_check(hipGetLastError(), "tmunu_kernel launch");
}

int rsl_mlp_guard(const float* x, int n, const float* lo, const float* hi, unsigned* flag_dev, void* hip_stream) {
    if (!x || !lo || !hi || !flag_dev || n < 0) return set_error(RSL_EINVAL, "bad argument");
    if (n == 0) return RSL_OK;
    hipLaunchKernelGGL(guard_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, x, n, lo, hi,
                       flag_dev);
    return hip_check(hipGetLastError(), "guard_kernel launch");
}

}  // extern "C"
