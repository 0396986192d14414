// Amortised encoder of a group's Gaussian proposal factor (not in the paper):
// features [1, mean y, mean x (D), mean y*x (D)] -> 64 -> 64 -> (mean, log var),
// exact GELU x*Phi(x), BF16 weights, FP32 accumulation.  Trained on the
// posterior moments QEM produces with the KL objective of appendix B
// (maximum likelihood of the proposal under the estimated posterior).
//
// Parameter layout (5506 floats): W1[64][18] b1[64] W2[64][64] b2[64] W3[2][64] b3[2].
// Forward: one thread per group, weights staged in LDS as FP32 (every thread
// of a wave reads the same weight at once, an LDS broadcast).
// Backward: a workgroup per chunk of 32 groups keeps inputs, activations and
// deltas in LDS and writes its partial parameter gradient; a second kernel
// adds the partials in chunk order (deterministic, no atomics).
#include <mutex>

#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

constexpr int IN = 18, HID = 64, OUT = 2;
constexpr int O_W1 = 0, O_B1 = O_W1 + HID * IN, O_W2 = O_B1 + HID, O_B2 = O_W2 + HID * HID,
              O_W3 = O_B2 + HID, O_B3 = O_W3 + OUT * HID, NPARAM = O_B3 + OUT;
constexpr int CHUNK = 32;
constexpr int EBLOCK = 256;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// Round to nearest even (NaN payloads are not special-cased: weights are finite).
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    const uint32_t b = __float_as_uint(x);
    return static_cast<uint16_t>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float a) {
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * __expf(-0.5f * a * a);
}

__device__ void stage_weights(const uint16_t* __restrict__ w, float* s_w) {
    for (int p = threadIdx.x; p < NPARAM; p += blockDim.x) s_w[p] = bf16_to_f32(w[p]);
    __syncthreads();
}

__global__ void __launch_bounds__(EBLOCK) k_enc_features(const double* __restrict__ y, const double* __restrict__ cov,
                                                         int n, int J, int D, float* __restrict__ feat) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int nf = 2 + 2 * D;
    if (t >= static_cast<long>(n) * nf) return;
    const long i = t / nf;
    const int f = static_cast<int>(t % nf);
    double s = 0.0;
    if (f == 0) s = J;
    else if (f == 1) for (int o = 0; o < J; ++o) s += y[i * J + o];
    else if (f < 2 + D) for (int o = 0; o < J; ++o) s += cov[(i * J + o) * D + (f - 2)];
    else for (int o = 0; o < J; ++o) s += y[i * J + o] * cov[(i * J + o) * D + (f - 2 - D)];
    feat[t] = static_cast<float>(s / J);
}

__global__ void __launch_bounds__(64) k_enc_fwd(const uint16_t* __restrict__ w, const float* __restrict__ x, int n,
                                                float* __restrict__ out, float* __restrict__ act) {
    __shared__ float s_w[NPARAM];
    stage_weights(w, s_w);
    const long s = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float xi[IN];
#pragma unroll
    for (int i = 0; i < IN; ++i) xi[i] = x[s * IN + i];
    float h1[HID];
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        float a = s_w[O_B1 + j];
#pragma unroll
        for (int i = 0; i < IN; ++i) a += s_w[O_W1 + j * IN + i] * xi[i];
        if (act) act[s * 2 * HID + j] = a;
        h1[j] = gelu(a);
    }
    float o0 = s_w[O_B3], o1 = s_w[O_B3 + 1];
    for (int j = 0; j < HID; ++j) {
        float a = s_w[O_B2 + j];
#pragma unroll
        for (int k = 0; k < HID; ++k) a += s_w[O_W2 + j * HID + k] * h1[k];
        if (act) act[s * 2 * HID + HID + j] = a;
        const float g = gelu(a);
        o0 += s_w[O_W3 + j] * g;
        o1 += s_w[O_W3 + HID + j] * g;
    }
    out[s * 2] = o0;
    out[s * 2 + 1] = o1;
}

// Per-group KL(N(m_t, v_t) || N(mu, exp(s))) and its gradient / n.
__global__ void __launch_bounds__(EBLOCK) k_enc_kl(const float* __restrict__ out, const double* __restrict__ target,
                                                   int n, float* __restrict__ dout, double* __restrict__ kl) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double mu = out[i * 2], sv = out[i * 2 + 1];
    const double mt = target[i * 2], vt = target[i * 2 + 1];
    const double es = exp(-sv);
    const double d2 = (mt - mu) * (mt - mu);
    kl[i] = 0.5 * (sv - log(vt)) + 0.5 * (vt + d2) * es - 0.5;
    dout[i * 2] = static_cast<float>(-(mt - mu) * es / n);
    dout[i * 2 + 1] = static_cast<float>((0.5 - 0.5 * (vt + d2) * es) / n);
}

__global__ void __launch_bounds__(EBLOCK) k_mean_f64(const double* __restrict__ v, int n, double* __restrict__ out) {
    __shared__ double red[EBLOCK];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += EBLOCK) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = EBLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / n;
}

__global__ void __launch_bounds__(EBLOCK) k_enc_bwd_partial(const uint16_t* __restrict__ w, const float* __restrict__ x,
                                                            const float* __restrict__ act, const float* __restrict__ dout,
                                                            int n, float* __restrict__ part) {
    extern __shared__ float smem_f[];
    float* s_w = smem_f;                        // [NPARAM]
    float* X = s_w + NPARAM;                    // [CHUNK][IN]
    float* H1 = X + CHUNK * IN;                 // [CHUNK][HID]
    float* H2 = H1 + CHUNK * HID;
    float* DZ1 = H2 + CHUNK * HID;
    float* DZ2 = DZ1 + CHUNK * HID;
    float* DO = DZ2 + CHUNK * HID;              // [CHUNK][OUT]
    stage_weights(w, s_w);
    const long s0 = static_cast<long>(blockIdx.x) * CHUNK;
    // inputs, activations and output deltas of the chunk (zero past n)
    for (int e = threadIdx.x; e < CHUNK * IN; e += EBLOCK) {
        const long s = s0 + e / IN;
        X[e] = s < n ? x[s * IN + e % IN] : 0.f;
    }
    for (int e = threadIdx.x; e < CHUNK * OUT; e += EBLOCK) {
        const long s = s0 + e / OUT;
        DO[e] = s < n ? dout[s * OUT + e % OUT] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < CHUNK * HID; e += EBLOCK) {
        const int sl = e / HID, j = e % HID;
        const long s = s0 + sl;
        const float a1 = s < n ? act[s * 2 * HID + j] : 0.f;
        const float a2 = s < n ? act[s * 2 * HID + HID + j] : 0.f;
        H1[e] = s < n ? gelu(a1) : 0.f;
        H2[e] = s < n ? gelu(a2) : 0.f;
        const float dh2 = s_w[O_W3 + j] * DO[sl * OUT] + s_w[O_W3 + HID + j] * DO[sl * OUT + 1];
        DZ2[e] = dh2 * gelu_grad(a2);
        DZ1[e] = a1;   // pre-activation kept until the next pass
    }
    __syncthreads();
    for (int e = threadIdx.x; e < CHUNK * HID; e += EBLOCK) {
        const int sl = e / HID, k = e % HID;
        float dh1 = 0.f;
        for (int j = 0; j < HID; ++j) dh1 += s_w[O_W2 + j * HID + k] * DZ2[sl * HID + j];
        DZ1[e] = dh1 * gelu_grad(DZ1[e]);   // each thread rewrites only its own entry
    }
    __syncthreads();
    float* g = part + static_cast<long>(blockIdx.x) * NPARAM;
    for (int p = threadIdx.x; p < NPARAM; p += EBLOCK) {
        float acc = 0.f;
        if (p < O_B1) {
            const int j = p / IN, i = p % IN;
            for (int sl = 0; sl < CHUNK; ++sl) acc += DZ1[sl * HID + j] * X[sl * IN + i];
        } else if (p < O_W2) {
            const int j = p - O_B1;
            for (int sl = 0; sl < CHUNK; ++sl) acc += DZ1[sl * HID + j];
        } else if (p < O_B2) {
            const int j = (p - O_W2) / HID, k = (p - O_W2) % HID;
            for (int sl = 0; sl < CHUNK; ++sl) acc += DZ2[sl * HID + j] * H1[sl * HID + k];
        } else if (p < O_W3) {
            const int j = p - O_B2;
            for (int sl = 0; sl < CHUNK; ++sl) acc += DZ2[sl * HID + j];
        } else if (p < O_B3) {
            const int o = (p - O_W3) / HID, j = (p - O_W3) % HID;
            for (int sl = 0; sl < CHUNK; ++sl) acc += DO[sl * OUT + o] * H2[sl * HID + j];
        } else {
            const int o = p - O_B3;
            for (int sl = 0; sl < CHUNK; ++sl) acc += DO[sl * OUT + o];
        }
        g[p] = acc;
    }
}

__global__ void __launch_bounds__(EBLOCK) k_enc_grad_sum(const float* __restrict__ part, int nchunks,
                                                         float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float acc = 0.f;
    for (int c = 0; c < nchunks; ++c) acc += part[static_cast<long>(c) * NPARAM + p];
    grad[p] = acc;
}

__global__ void __launch_bounds__(EBLOCK) k_enc_adam(float* __restrict__ master, uint16_t* __restrict__ w,
                                                     const float* __restrict__ grad, float* __restrict__ m1,
                                                     float* __restrict__ m2, float c1, float c2, float lr, float b1,
                                                     float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.f - b1) * g;
    const float b = b2 * m2[p] + (1.f - b2) * g * g;
    m1[p] = a;
    m2[p] = b;
    const float upd = master[p] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    master[p] = upd;
    w[p] = f32_to_bf16(upd);
}

__global__ void __launch_bounds__(EBLOCK) k_enc_to_bf16(const float* __restrict__ master, uint16_t* __restrict__ w) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) w[p] = f32_to_bf16(master[p]);
}

// Empirical logit of a group mean of J Bernoulli outcomes (+1/2 counts); yc
// is the corrected mean.
__device__ __forceinline__ double elogit(double ybar, int J, double& yc) {
    yc = (ybar * J + 0.5) / (J + 1.0);
    return log(yc / (1.0 - yc));
}

// Fixed-order sums of NV values per thread over one workgroup (tree in LDS).
template <int NV>
__device__ void block_sums(double (&acc)[NV], double (*red)[EBLOCK]) {
#pragma unroll
    for (int f = 0; f < NV; ++f) red[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int h = EBLOCK / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h)
#pragma unroll
            for (int f = 0; f < NV; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + h];
        __syncthreads();
    }
#pragma unroll
    for (int f = 0; f < NV; ++f) acc[f] = red[f][0];
    __syncthreads();
}

// c(s) = E[sigma'(s Z)], Z ~ N(0, 1), by the trapezoid rule on [-10, 10]
// (nodes z = -10 + 0.05 i, i < 401), summed over the workgroup in a fixed
// order; every thread gets it.  red: LDS of EBLOCK doubles.
constexpr int QUAD_N = 401;
constexpr double QUAD_H = 0.05;
__device__ double block_slope(double s, double* red) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < QUAD_N; i += EBLOCK) {
        const double z = -10.0 + QUAD_H * i;
        const double w = (i == 0 || i == QUAD_N - 1) ? 0.5 * QUAD_H : QUAD_H;
        const double t = exp(-fabs(s * z));
        acc += w * exp(-0.5 * z * z) * 0.39894228040143267794 * t / ((1.0 + t) * (1.0 + t));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = EBLOCK / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double c = red[0];
    __syncthreads();
    return c;
}

// Input rows of the global head, pooled over one dataset's n groups of J
// observations (single workgroup, FP64, fixed-order sums).
// Pass 1: P = mean feature, V = variance of the group means of y,
//   u = P_yx / |P_yx|; B = |beta| solves c(sqrt(B^2 + sigma^2)) B = |P_yx|
//   (Stein's lemma; bisection on [0, 50]).
// Pass 2: kappa = 4 c(B), a_i = e_i - kappa xbar_i . (u B) (e = empirical
//   logit), noise_i = 1 / (J yc_i (1 - yc_i)),
//   sigma^2 = max((Var(a) - kappa mean noise) / kappa^2, 1e-4).
// B starts at sigma = 0 and the two alternate POOL_FIXED_POINT times.
//   row j < 8 (beta_j):  [1, u_j B,          u_j, B, 5|P_yx|, 4 sqrt V, 0, 5 P[2+j], P[1], kappa, 0, 0, 0...]
//   row 8 (log sigma):   [1, log(sigma^2)/2, 0,   B, 5|P_yx|, 4 sqrt V, 1, 0,        P[1], kappa, Var(a), mean noise, 0...]
constexpr int NPOOL = IN + 1;
constexpr int POOL_FIXED_POINT = 3;
constexpr int BISECT_STEPS = 60;
constexpr double B_MAX = 50.0;
__global__ void __launch_bounds__(EBLOCK) k_enc_pool(const float* __restrict__ feat, int n, int J,
                                                     float* __restrict__ rows) {
    __shared__ double red[NPOOL][EBLOCK];
    double acc[NPOOL];
#pragma unroll
    for (int f = 0; f < NPOOL; ++f) acc[f] = 0.0;
    for (int i = threadIdx.x; i < n; i += EBLOCK) {
#pragma unroll
        for (int f = 0; f < IN; ++f) acc[f] += static_cast<double>(feat[static_cast<long>(i) * IN + f]);
        const double y = static_cast<double>(feat[static_cast<long>(i) * IN + 1]);
        acc[IN] += y * y;
    }
    block_sums(acc, red);
    double P[IN];
    for (int f = 0; f < IN; ++f) P[f] = acc[f] / n;
    const double V = fmax(acc[IN] / n - P[1] * P[1], 0.0);
    double nyx2 = 0.0;
    for (int j = 0; j < 8; ++j) nyx2 += P[10 + j] * P[10 + j];
    const double nyx = sqrt(nyx2);
    double u[8];
    for (int j = 0; j < 8; ++j) u[j] = nyx > 0.0 ? P[10 + j] / nyx : 0.0;
    // the noise of the groups' empirical logits does not depend on B
    double accn[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += EBLOCK) {
        double yc;
        elogit(static_cast<double>(feat[static_cast<long>(i) * IN + 1]), J, yc);
        accn[0] += 1.0 / (J * yc * (1.0 - yc));
    }
    block_sums(accn, red);
    const double mnoise = accn[0] / n;
    double s2 = 0.0, B = 0.0, kappa = 1.0, var_a = 0.0;
    for (int it = 0; it < POOL_FIXED_POINT; ++it) {
        double lo = 0.0, hi = B_MAX;
        for (int b = 0; b < BISECT_STEPS; ++b) {
            const double mid = 0.5 * (lo + hi);
            if (block_slope(sqrt(mid * mid + s2), red[0]) * mid < nyx) lo = mid;
            else hi = mid;
        }
        B = 0.5 * (lo + hi);
        kappa = 4.0 * block_slope(B, red[0]);
        double acc2[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += EBLOCK) {
            const float* fi = feat + static_cast<long>(i) * IN;
            double yc;
            const double e = elogit(static_cast<double>(fi[1]), J, yc);
            double o = 0.0;
            for (int j = 0; j < 8; ++j) o += static_cast<double>(fi[2 + j]) * (u[j] * B);
            const double a = e - kappa * o;
            acc2[0] += a;
            acc2[1] += a * a;
        }
        block_sums(acc2, red);
        var_a = fmax(acc2[1] / n - (acc2[0] / n) * (acc2[0] / n), 0.0);
        s2 = fmax((var_a - kappa * mnoise) / (kappa * kappa), 1e-4);
    }
    if (threadIdx.x != 0) return;
    for (int r = 0; r < 9; ++r) {
        double row[IN];
        for (int f = 0; f < IN; ++f) row[f] = 0.0;
        row[0] = 1.0;
        row[3] = B;
        row[4] = 5.0 * nyx;
        row[5] = 4.0 * sqrt(V);
        row[8] = P[1];
        row[9] = kappa;
        if (r < 8) {
            row[1] = u[r] * B;
            row[2] = u[r];
            row[7] = 5.0 * P[2 + r];
        } else {
            row[1] = 0.5 * log(s2);
            row[6] = 1.0;
            row[10] = var_a;
            row[11] = mnoise;
        }
        for (int f = 0; f < IN; ++f) rows[r * IN + f] = static_cast<float>(row[f]);
    }
}

// Group features with the dataset context of the global head's plug-ins
// (rows from k_enc_pool): for group i,
//   [1, ybar, o = xbar . beta^, m = mean(y x) . beta^, e (empirical logit),
//    e / kappa - o, sigma^, B, kappa, 1 / (J yc (1 - yc) kappa), 0 ...]
__global__ void __launch_bounds__(EBLOCK) k_enc_features_ctx(const float* __restrict__ feat,
                                                             const float* __restrict__ rows, int n, int J,
                                                             float* __restrict__ out) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* fi = feat + i * IN;
    double o = 0.0, m = 0.0;
    for (int j = 0; j < 8; ++j) {
        const double bj = static_cast<double>(rows[j * IN + 1]);
        o += static_cast<double>(fi[2 + j]) * bj;
        m += static_cast<double>(fi[10 + j]) * bj;
    }
    const double kappa = static_cast<double>(rows[9]);
    double yc;
    const double e = elogit(static_cast<double>(fi[1]), J, yc);
    double g[IN];
    for (int f = 0; f < IN; ++f) g[f] = 0.0;
    g[0] = 1.0;
    g[1] = static_cast<double>(fi[1]);
    g[2] = o;
    g[3] = m;
    g[4] = e;
    g[5] = e / kappa - o;
    g[6] = exp(static_cast<double>(rows[8 * IN + 1]));
    g[7] = static_cast<double>(rows[3]);
    g[8] = kappa;
    g[9] = 1.0 / (J * yc * (1.0 - yc) * kappa);
    for (int f = 0; f < IN; ++f) out[i * IN + f] = static_cast<float>(g[f]);
}

// Training targets from EMA mean parameters m[n][2] = (E z, E z^2):
// target[i] = (E z - rows[i, 1] (when rows is set), max(E z^2 - (E z)^2, floor)).
__global__ void __launch_bounds__(EBLOCK) k_enc_targets(const double* __restrict__ m, int n, double floor_v,
                                                        const float* __restrict__ rows, double* __restrict__ target) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m1 = m[i * 2], m2 = m[i * 2 + 1];
    target[i * 2] = rows ? m1 - static_cast<double>(rows[i * IN + 1]) : m1;
    target[i * 2 + 1] = fmax(m2 - m1 * m1, floor_v);
}

__global__ void __launch_bounds__(EBLOCK) k_enc_apply(const float* __restrict__ out, int n, double* __restrict__ qp) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    qp[i * 2] = out[i * 2];
    qp[i * 2 + 1] = exp(static_cast<double>(out[i * 2 + 1]));
}

// As k_enc_apply with the mean predicted as a residual of the input feature
// rows[i, 1] (the global head's plug-in estimate).
__global__ void __launch_bounds__(EBLOCK) k_enc_apply_res(const float* __restrict__ out,
                                                          const float* __restrict__ rows, int n,
                                                          double* __restrict__ qp) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    qp[i * 2] = static_cast<double>(rows[i * IN + 1]) + static_cast<double>(out[i * 2]);
    qp[i * 2 + 1] = exp(static_cast<double>(out[i * 2 + 1]));
}

}  // namespace

int enc_nparam() { return NPARAM; }
size_t enc_scratch_bytes(int n) { return static_cast<size_t>((n + CHUNK - 1) / CHUNK) * NPARAM * sizeof(float); }

hipError_t enc_features(hipStream_t s, const double* y, const double* cov, int n, int J, int D, float* feat) {
    const long total = static_cast<long>(n) * (2 + 2 * D);
    hipLaunchKernelGGL(k_enc_features, dim3((total + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, y, cov, n, J, D, feat);
    return hipGetLastError();
}

hipError_t enc_apply_res(hipStream_t s, const float* out, const float* rows, int n, double* qp) {
    hipLaunchKernelGGL(k_enc_apply_res, dim3((n + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, out, rows, n, qp);
    return hipGetLastError();
}

hipError_t enc_pool(hipStream_t s, const float* feat, int n, int J, float* rows) {
    hipLaunchKernelGGL(k_enc_pool, dim3(1), dim3(EBLOCK), 0, s, feat, n, J, rows);
    return hipGetLastError();
}

hipError_t enc_features_ctx(hipStream_t s, const float* feat, const float* rows, int n, int J, float* out) {
    hipLaunchKernelGGL(k_enc_features_ctx, dim3((n + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, feat, rows, n, J, out);
    return hipGetLastError();
}

hipError_t enc_fwd(hipStream_t s, const uint16_t* w, const float* x, int n, float* out, float* act) {
    hipLaunchKernelGGL(k_enc_fwd, dim3((n + 63) / 64), dim3(64), 0, s, w, x, n, out, act);
    return hipGetLastError();
}

hipError_t enc_kl(hipStream_t s, const float* out, const double* target, int n, float* dout, double* kl,
                  double* loss) {
    hipLaunchKernelGGL(k_enc_kl, dim3((n + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, out, target, n, dout, kl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(k_mean_f64, dim3(1), dim3(EBLOCK), 0, s, kl, n, loss);
    return hipGetLastError();
}

hipError_t enc_bwd(hipStream_t s, const uint16_t* w, const float* x, const float* act, const float* dout, int n,
                   float* grad, float* scratch) {
    const int nchunks = (n + CHUNK - 1) / CHUNK;
    const size_t sm = (NPARAM + CHUNK * (IN + 4 * HID + OUT)) * sizeof(float);
    hipLaunchKernelGGL(k_enc_bwd_partial, dim3(nchunks), dim3(EBLOCK), sm, s, w, x, act, dout, n, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_enc_grad_sum, dim3((NPARAM + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, scratch, nchunks, grad);
    return hipGetLastError();
}

}  // namespace qemk

// Library-owned scratch of enc_bwd_noalloc: the per-chunk partial gradients
// of up to ENC_NOALLOC_MAX_N groups (512 chunks x 5506 floats, 11.3 MB).
// Every GPU the library runs on holds its own copy until the process ends.
// In host code this name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, taken once per device below.
static __device__ __align__(256) float scratch[static_cast<size_t>(qemk::ENC_NOALLOC_MAX_N / qemk::CHUNK) *
                                              qemk::NPARAM];

namespace qemk {

static_assert(ENC_NOALLOC_MAX_N % CHUNK == 0, "the no-alloc scratch holds whole chunks");

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
float* g_noalloc_scratch[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device (with that device current) and kept.
hipError_t noalloc_scratch(int dev, float** out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_noalloc_scratch[dev] = static_cast<float*>(p);
    }
    *out = g_noalloc_scratch[dev];
    return hipSuccess;
}
}  // namespace

hipError_t enc_bwd_noalloc(hipStream_t s, const uint16_t* w, const float* x, const float* act, const float* dout,
                           int n, float* grad) {
    if (n < 1 || n > ENC_NOALLOC_MAX_N) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (s) {
        int sdev = -1;
        e = hipStreamGetDevice(s, &sdev);
        if (e != hipSuccess) return e;
        // the symbol address is per device: the stream must run on the current one
        if (sdev != dev) return hipErrorInvalidDevice;
    }
    float* part = nullptr;
    e = noalloc_scratch(dev, &part);
    if (e != hipSuccess) return e;
    return enc_bwd(s, w, x, act, dout, n, grad, part);
}

hipError_t enc_adam(hipStream_t s, float* master, uint16_t* w, const float* grad, float* m1, float* m2, int step,
                    float lr, float b1, float b2, float eps) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(k_enc_adam, dim3((NPARAM + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, master, w, grad, m1, m2,
                       c1, c2, lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t enc_to_bf16(hipStream_t s, const float* master, uint16_t* w) {
    hipLaunchKernelGGL(k_enc_to_bf16, dim3((NPARAM + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, master, w);
    return hipGetLastError();
}

hipError_t enc_targets(hipStream_t s, const double* m, int n, double floor_v, const float* rows, double* target) {
    hipLaunchKernelGGL(k_enc_targets, dim3((n + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, m, n, floor_v, rows, target);
    return hipGetLastError();
}

hipError_t enc_apply(hipStream_t s, const float* out, int n, double* qp) {
    hipLaunchKernelGGL(k_enc_apply, dim3((n + EBLOCK - 1) / EBLOCK), dim3(EBLOCK), 0, s, out, n, qp);
    return hipGetLastError();
}

}  // namespace qemk
