// su2_learned.hip -- the learned proposal for x0: targets, network, training.
//
//   k_cdf          knots y_j = F_alpha^{-1}(j/32) of the x0 density
//                  sqrt(1 - x^2) exp(alpha x) (the heat-bath's local
//                  conditional, Eqs. (2), (3), (6)), integrated in FP64 on the
//                  device: theta = arccos(x) cut into 2048 panels, 8-point
//                  Gauss-Legendre per panel, a fixed-order block scan, then
//                  bisection-safeguarded Newton inside the bracketing panel.
//   k_l1..k_head   forward of the 1 -> 64 -> 64 -> 33 network (SiLU), BF16
//                  weights, FP32 accumulation; the head turns outputs 0..31
//                  into segment widths 2 softmax(z) and knots, and (training)
//                  the log-width loss and its gradient.
//   k_bwd3, k_bwd2 backward signals per sample.
//   k_wgrad_part, k_wgrad_reduce   weight gradients: the batch contractions on
//                  the matrix cores (MFMA, FP32), chunk partials added in a
//                  fixed order (FP64), so they are deterministic.
//   k_adam         Adam on the FP32 master weights, then RNE rounding to BF16.
// Parameters are one flat vector: W1 (64x1), b1 (64), W2 (64x64), b2 (64),
// W3 (33x64), b3 (33) -- 6433 numbers.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "su2.h"
#include "su2_learned.hpp"
#include "su2_pass.hpp"

namespace su2 {

constexpr int kH = 64, kOut = 33, kSeg = 32;
constexpr int kW1 = 0, kB1 = 64, kW2 = 128, kB2 = 128 + 4096, kW3 = kB2 + 64, kB3 = kW3 + 33 * 64;
constexpr int kNParam = kB3 + 33;  // 6433
static_assert(kNParam == kLearnedParams, "parameter count");
constexpr float kAlphaMax = 40.0f;

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // round to nearest, ties to even
}

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }

// ---------------------------------------------------------------------------
// Gauss-Legendre 8-point rule on [-1, 1] (Abramowitz & Stegun, Table 25.4).
__constant__ double kGLx[4] = { 0.1834346424956498049394761, 0.5255324099163289858177390,
                                0.7966664774136267395915539, 0.9602898564975362316835609 };
__constant__ double kGLw[4] = { 0.3626837833783619829651504, 0.3137066458778872873379622,
                                0.2223810344533744705443560, 0.1012285362903762591525314 };

__device__ __forceinline__ double dens_theta(double th, double alpha)
{
    const double sn = sin(th);
    return sn * sn * exp(alpha * (cos(th) - 1.0));  // sqrt(1 - x^2) dx, x = cos(theta)
}

__device__ double gl8(double a, double b, double alpha)
{
    const double c = 0.5 * (a + b), r = 0.5 * (b - a);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        s += kGLw[i] * (dens_theta(c - r * kGLx[i], alpha) + dens_theta(c + r * kGLx[i], alpha));
    return s * r;
}

constexpr int kPanels = 2048;  // 8 per thread

__global__ __launch_bounds__(kBlock) void k_cdf(const double *__restrict__ alphas,
                                                double *__restrict__ knots)
{
    __shared__ double cum[kPanels + 1];  // mass above x = cos(theta_i), theta_i = i * pi / kPanels
    __shared__ double tot[kBlock];
    const double alpha = alphas[blockIdx.x];
    const double h = M_PI / kPanels;
    const int t = threadIdx.x;
    double part[8], run = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int p = 8 * t + i;
        part[i] = gl8(p * h, (p + 1) * h, alpha);
        run += part[i];
    }
    tot[t] = run;
    __syncthreads();
    if (t == 0) {  // exclusive scan of the 256 thread totals, in order
        double acc = 0.0;
        for (int i = 0; i < kBlock; ++i) {
            const double v = tot[i];
            tot[i] = acc;
            acc += v;
        }
        cum[kPanels] = acc;
    }
    __syncthreads();
    double acc = tot[t];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        cum[8 * t + i] = acc;
        acc += part[i];
    }
    __syncthreads();
    double *out = knots + (size_t)33 * blockIdx.x;
    const double Z = cum[kPanels];
    if (t == 0) out[0] = -1.0;
    if (t == kSeg) out[kSeg] = 1.0;
    if (t >= 1 && t < kSeg) {
        const double target = (1.0 - (double)t / kSeg) * Z;  // mass above knot t
        int lo = 0, hi = kPanels;  // cum[lo] <= target < cum[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cum[mid] <= target) lo = mid; else hi = mid;
        }
        const double a = lo * h, b = (lo + 1) * h, need = target - cum[lo];
        const double seg = cum[lo + 1] - cum[lo];
        double x = a + (seg > 0.0 ? h * need / seg : 0.5 * h), blo = a, bhi = b;
        for (int it = 0; it < 40; ++it) {
            const double F = gl8(a, x, alpha) - need;
            if (F > 0.0) bhi = x; else blo = x;
            const double d = dens_theta(x, alpha);
            double xn = d > 0.0 ? x - F / d : 0.5 * (blo + bhi);
            if (!(xn > blo && xn < bhi)) xn = 0.5 * (blo + bhi);  // keep the bracket
            if (fabs(xn - x) <= 1e-15 * (1.0 + fabs(x))) {
                x = xn;
                break;
            }
            x = xn;
        }
        out[t] = cos(x);
    }
}

// log segment widths of knot rows (training targets)
__global__ void k_logw(const double *__restrict__ knots, uint32_t n, float *__restrict__ logw)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kSeg) return;
    const uint32_t r = i / kSeg, j = i - r * kSeg;
    logw[i] = (float)log(knots[33 * r + j + 1] - knots[33 * r + j]);
}

// ---------------------------------------------------------------------------
// Network.  One thread per (sample, unit).
__global__ void k_l1(const uint16_t *__restrict__ P, const float *__restrict__ alpha, uint32_t B,
                     float *__restrict__ a1, float *__restrict__ h1)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kH) return;
    const uint32_t b = i / kH, u = i - b * kH;
    const float a = bf16_to_f32(P[kW1 + u]) * (alpha[b] / kAlphaMax) + bf16_to_f32(P[kB1 + u]);
    a1[i] = a;
    h1[i] = a * sigm(a);
}

__global__ void k_l2(const uint16_t *__restrict__ P, const float *__restrict__ h1, uint32_t B,
                     float *__restrict__ a2, float *__restrict__ h2)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kH) return;
    const uint32_t b = i / kH, u = i - b * kH;
    float a = bf16_to_f32(P[kB2 + u]);
    for (int j = 0; j < kH; ++j) a += bf16_to_f32(P[kW2 + kH * u + j]) * h1[kH * b + j];
    a2[i] = a;
    h2[i] = a * sigm(a);
}

__global__ void k_l3(const uint16_t *__restrict__ P, const float *__restrict__ h2, uint32_t B,
                     float *__restrict__ z)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kOut) return;
    const uint32_t b = i / kOut, o = i - b * kOut;
    float a = bf16_to_f32(P[kB3 + o]);
    for (int j = 0; j < kH; ++j) a += bf16_to_f32(P[kW3 + kH * o + j]) * h2[kH * b + j];
    z[i] = a;
}

// One thread per sample: widths, knots (optional), loss term and dL/dz (optional).
__global__ void k_head(const float *__restrict__ z, uint32_t B, const float *__restrict__ target,
                       float *__restrict__ knots, float *__restrict__ dz,
                       float *__restrict__ loss_terms)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float *zb = z + (size_t)kOut * b;
    float m = zb[0];
    for (int j = 1; j < kSeg; ++j) m = fmaxf(m, zb[j]);
    float se = 0.0f;
    for (int j = 0; j < kSeg; ++j) se += expf(zb[j] - m);
    const float lse = m + logf(se);
    if (knots) {
        float *y = knots + (size_t)33 * b;
        float acc = -1.0f;
        y[0] = -1.0f;
        for (int j = 0; j < kSeg - 1; ++j) {
            acc += 2.0f * expf(zb[j] - lse);
            y[j + 1] = acc;
        }
        y[kSeg] = 1.0f;
    }
    if (target) {
        const float *tg = target + (size_t)kSeg * b;
        const float scale = 2.0f / ((float)B * kSeg);
        float loss = 0.0f, gsum = 0.0f, g[kSeg];
        for (int j = 0; j < kSeg; ++j) {
            const float e = (0.69314718055994531f + zb[j] - lse) - tg[j];
            loss += e * e;
            g[j] = scale * e;
            gsum += g[j];
        }
        float *d = dz + (size_t)kOut * b;
        for (int j = 0; j < kSeg; ++j) d[j] = g[j] - expf(zb[j] - lse) * gsum;
        d[kSeg] = 0.0f;  // output 32 is reserved
        loss_terms[b] = loss;
    }
}

__global__ void k_bwd3(const uint16_t *__restrict__ P, const float *__restrict__ dz,
                       const float *__restrict__ a2, uint32_t B, float *__restrict__ da2)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kH) return;
    const uint32_t b = i / kH, j = i - b * kH;
    float d = 0.0f;
    for (int o = 0; o < kOut; ++o) d += dz[kOut * b + o] * bf16_to_f32(P[kW3 + kH * o + j]);
    const float a = a2[i], s = sigm(a);
    da2[i] = d * s * (1.0f + a * (1.0f - s));
}

__global__ void k_bwd2(const uint16_t *__restrict__ P, const float *__restrict__ da2,
                       const float *__restrict__ a1, uint32_t B, float *__restrict__ da1)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kH) return;
    const uint32_t b = i / kH, j = i - b * kH;
    float d = 0.0f;
    for (int u = 0; u < kH; ++u) d += da2[kH * b + u] * bf16_to_f32(P[kW2 + kH * u + j]);
    const float a = a1[i], s = sigm(a);
    da1[i] = d * s * (1.0f + a * (1.0f - s));
}

// Weight gradients: sums over the batch of products of a backward signal and
// a forward activation -- dense contractions with the batch as the inner
// dimension, done on the matrix cores.  Workgroup c takes samples
// [c * kChunk, (c + 1) * kChunk) and writes its partial of every parameter to
// part[c][.]; k_wgrad_reduce then adds the partials in chunk order (FP64), so
// the result does not depend on scheduling.
//   dW2[u][j] = sum_b da2[b][u] h1[b][j]   four 32 x 32 tiles (waves 0..3)
//   dW3[o][j] = sum_b dz[b][o]  h2[b][j]   o < 32: two tiles (waves 0, 1);
//                                          o = 32 (reserved output) is zero
// with v_mfma_f32_32x32x2f32: per instruction lane l supplies A[i][k] and
// B[k][j] for i = j = l mod 32, k = l / 32 (two samples per instruction), and
// holds D[8 (r / 4) + 4 (l / 32) + r mod 4][l mod 32] in accumulator r.  The
// first- and last-layer bias and W1 sums (225 of them) run on plain lanes.
constexpr uint32_t kChunk = 64;
typedef float mfma_acc16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void mfma_tile(const float *__restrict__ A, uint32_t lda, uint32_t a0,
                                          const float *__restrict__ Bm, uint32_t ldb, uint32_t b0,
                                          uint32_t s0, uint32_t s1, float *__restrict__ out,
                                          uint32_t ldo)
{
    const uint32_t l = threadIdx.x % kWave, i = l % 32u, kk = l / 32u;
    mfma_acc16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint32_t b = s0; b < s1; b += 2u) {
        const uint32_t bs = b + kk;
        const float av = bs < s1 ? A[(size_t)lda * bs + a0 + i] : 0.f;
        const float bv = bs < s1 ? Bm[(size_t)ldb * bs + b0 + i] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (uint32_t r = 0; r < 16u; ++r) {
        const uint32_t row = 8u * (r / 4u) + 4u * kk + (r % 4u);
        out[(size_t)ldo * row + i] = acc[r];
    }
}

__global__ __launch_bounds__(kBlock) void k_wgrad_part(const float *__restrict__ alpha,
                                                       const float *__restrict__ h1,
                                                       const float *__restrict__ h2,
                                                       const float *__restrict__ dz,
                                                       const float *__restrict__ da2,
                                                       const float *__restrict__ da1, uint32_t B,
                                                       float *__restrict__ part)
{
    const uint32_t c = blockIdx.x, s0 = c * kChunk, s1 = min(B, s0 + kChunk);
    float *pc = part + (size_t)c * kNParam;
    const uint32_t w = threadIdx.x / kWave;
    // dW2 tile (u0, j0) = (32 (w / 2), 32 (w % 2))
    mfma_tile(da2, kH, 32u * (w / 2u), h1, kH, 32u * (w % 2u), s0, s1,
              pc + kW2 + kH * (32u * (w / 2u)) + 32u * (w % 2u), kH);
    if (w < 2u)  // dW3 tile (o0, j0) = (0, 32 w)
        mfma_tile(dz, kOut, 0u, h2, kH, 32u * w, s0, s1, pc + kW3 + 32u * w, kH);
    // plain sums: W1 and b1 (64 each), b2 (64), b3 (33); the reserved row of W3
    const uint32_t t = threadIdx.x;
    if (t < 64u) {
        float gw = 0.f, gb = 0.f;
        for (uint32_t b = s0; b < s1; ++b) {
            const float d = da1[(size_t)kH * b + t];
            gw += d * (alpha[b] / kAlphaMax);
            gb += d;
        }
        pc[kW1 + t] = gw;
        pc[kB1 + t] = gb;
    } else if (t < 128u) {
        const uint32_t u = t - 64u;
        float g = 0.f;
        for (uint32_t b = s0; b < s1; ++b) g += da2[(size_t)kH * b + u];
        pc[kB2 + u] = g;
    } else if (t < 128u + (uint32_t)kOut) {
        const uint32_t o = t - 128u;
        float g = 0.f;
        for (uint32_t b = s0; b < s1; ++b) g += dz[(size_t)kOut * b + o];
        pc[kB3 + o] = g;
        pc[kW3 + kH * 32 + (o % 32u) * 2u] = 0.f;  // reserved output 32: zero gradient
        pc[kW3 + kH * 32 + (o % 32u) * 2u + 1u] = 0.f;
    }
}

__global__ void k_wgrad_reduce(const float *__restrict__ part, uint32_t nchunk,
                               float *__restrict__ grad)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (uint32_t)kNParam) return;
    double acc = 0.0;
    for (uint32_t c = 0; c < nchunk; ++c) acc += part[(size_t)c * kNParam + q];
    grad[q] = (float)acc;
}

// Single workgroup: loss = sum of per-sample terms / (B * 32), fixed order.
__global__ __launch_bounds__(kBlock) void k_loss(const float *__restrict__ terms, uint32_t B,
                                                 float *__restrict__ out,
                                                 const int32_t *__restrict__ step)
{
    double a = 0.0;
    for (uint32_t j = threadIdx.x; j < B; j += kBlock) a += terms[j];
    const double r = block_sum(a);
    if (threadIdx.x == 0) out[step ? *step : 0] = (float)(r / ((double)B * kSeg));
}

// Adam (Kingma & Ba) with bias correction and a cosine learning-rate decay
// from lr0 to lr_min over `total` steps; the step number lives on the device.
__global__ void k_adam(float *__restrict__ master, uint16_t *__restrict__ P,
                       const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, const int32_t *__restrict__ step, float lr0,
                       float lr_min, int32_t total)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (uint32_t)kNParam) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int32_t t = *step + 1;
    const float frac = fminf(1.0f, (float)(t - 1) / (float)max(1, total));
    const float lr = lr_min + 0.5f * (lr0 - lr_min) * (1.0f + cospif(frac));
    const float g = grad[q];
    const float mq = b1 * m[q] + (1.0f - b1) * g;
    const float vq = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.0f - powf(b1, (float)t)), vh = vq / (1.0f - powf(b2, (float)t));
    const float w = master[q] - lr * mh / (sqrtf(vh) + eps);
    master[q] = w;
    P[q] = f32_to_bf16(w);
}

__global__ void k_step_tick(int32_t *step)
{
    if (threadIdx.x == 0) *step += 1;
}

__global__ void k_to_bf16(const float *__restrict__ master, uint16_t *__restrict__ P)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < (uint32_t)kNParam) P[q] = f32_to_bf16(master[q]);
}

__global__ void k_f64_to_f32(const double *__restrict__ a, uint32_t n, float *__restrict__ b)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

}  // namespace su2

// ---------------------------------------------------------------------------
// Host side: one global network (and knot table), independent of the lattice.
// ---------------------------------------------------------------------------
using namespace su2;

namespace {

struct Learn {
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *P = nullptr;
    bool have_params = false;
    uint32_t cap = 0;  // batch capacity of the work buffers
    float *alpha = nullptr, *a1 = nullptr, *h1 = nullptr, *a2 = nullptr, *h2 = nullptr,
          *z = nullptr, *dz = nullptr, *da2 = nullptr, *da1 = nullptr, *terms = nullptr,
          *target = nullptr, *knots = nullptr;
    int32_t *step = nullptr;
    float *loss1 = nullptr;  // one loss value
    float *table = nullptr;  // [G][33]
    uint32_t G = 0;
    float *part = nullptr;   // [ceil(cap / kChunk)][kNParam] weight-gradient partials
};

Learn LN;
char lerr[512] = "no error";

int lfail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(lerr, sizeof lerr, fmt, ap);
    va_end(ap);
    return code;
}

#define LTRY(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return lfail(SU2_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

inline uint32_t nb(size_t n, uint32_t t = 256) { return (uint32_t)((n + t - 1) / t); }
inline uint32_t nchunks(uint32_t B) { return (B + kChunk - 1) / kChunk; }

int ensure_params()
{
    if (LN.master) return SU2_OK;
    if (hipMalloc(&LN.master, kNParam * sizeof(float)) != hipSuccess ||
        hipMalloc(&LN.m, kNParam * sizeof(float)) != hipSuccess ||
        hipMalloc(&LN.v, kNParam * sizeof(float)) != hipSuccess ||
        hipMalloc(&LN.grad, kNParam * sizeof(float)) != hipSuccess ||
        hipMalloc(&LN.P, kNParam * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&LN.step, sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&LN.loss1, sizeof(float)) != hipSuccess) {
        hipGetLastError();
        return lfail(SU2_ENOMEM, "cannot allocate the network");
    }
    return SU2_OK;
}

int ensure_batch(uint32_t B)
{
    if (B <= LN.cap) return SU2_OK;
    float **bufs[] = { &LN.alpha, &LN.a1, &LN.h1, &LN.a2, &LN.h2, &LN.z, &LN.dz, &LN.da2,
                       &LN.da1, &LN.terms, &LN.target, &LN.knots };
    const size_t sizes[] = { 1, kH, kH, kH, kH, kOut, kOut, kH, kH, 1, kSeg, 33 };
    for (int i = 0; i < 12; ++i) {
        if (*bufs[i]) hipFree(*bufs[i]);
        *bufs[i] = nullptr;
    }
    if (LN.part) hipFree(LN.part);
    LN.part = nullptr;
    for (int i = 0; i < 12; ++i)
        if (hipMalloc(bufs[i], (size_t)B * sizes[i] * sizeof(float)) != hipSuccess) {
            hipGetLastError();
            LN.cap = 0;
            return lfail(SU2_ENOMEM, "cannot allocate network buffers for %u samples", B);
        }
    if (hipMalloc(&LN.part, (size_t)nchunks(B) * kNParam * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        LN.cap = 0;
        return lfail(SU2_ENOMEM, "cannot allocate gradient partials for %u samples", B);
    }
    LN.cap = B;
    return SU2_OK;
}

hipError_t forward(uint32_t B, bool knots_out, bool with_target)
{
    hipLaunchKernelGGL(k_l1, dim3(nb((size_t)B * kH)), dim3(256), 0, nullptr, LN.P, LN.alpha, B,
                       LN.a1, LN.h1);
    hipLaunchKernelGGL(k_l2, dim3(nb((size_t)B * kH)), dim3(256), 0, nullptr, LN.P, LN.h1, B,
                       LN.a2, LN.h2);
    hipLaunchKernelGGL(k_l3, dim3(nb((size_t)B * kOut)), dim3(256), 0, nullptr, LN.P, LN.h2, B,
                       LN.z);
    hipLaunchKernelGGL(k_head, dim3(nb(B)), dim3(256), 0, nullptr, LN.z, B,
                       with_target ? LN.target : nullptr, knots_out ? LN.knots : nullptr, LN.dz,
                       LN.terms);
    return hipGetLastError();
}

hipError_t backward(uint32_t B)
{
    hipLaunchKernelGGL(k_bwd3, dim3(nb((size_t)B * kH)), dim3(256), 0, nullptr, LN.P, LN.dz, LN.a2,
                       B, LN.da2);
    hipLaunchKernelGGL(k_bwd2, dim3(nb((size_t)B * kH)), dim3(256), 0, nullptr, LN.P, LN.da2, LN.a1,
                       B, LN.da1);
    hipLaunchKernelGGL(k_wgrad_part, dim3(nchunks(B)), dim3(kBlock), 0, nullptr, LN.alpha, LN.h1,
                       LN.h2, LN.dz, LN.da2, LN.da1, B, LN.part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(kNParam)), dim3(256), 0, nullptr, LN.part,
                       nchunks(B), LN.grad);
    return hipGetLastError();
}

int need_params()
{
    if (!LN.have_params) return lfail(SU2_ESTATE, "no network parameters: call su2_mlp_set_params");
    return SU2_OK;
}

}  // namespace

// internal: the current knot table for the lattice context
bool su2_learned_table(const float **knots, uint32_t *G, float *alpha_max)
{
    if (!LN.table || LN.G < 2) return false;
    *knots = LN.table;
    *G = LN.G;
    *alpha_max = kAlphaMax;
    return true;
}

const char *su2_learned_error() { return lerr; }

extern "C" {

int su2_cdf_knots(const double *alphas, int32_t n, double *knots)
{
    if (n < 0 || (n > 0 && (!alphas || !knots))) return lfail(SU2_EINVAL, "bad arguments");
    if (n == 0) return SU2_OK;
    for (int32_t i = 0; i < n; ++i)
        if (!(alphas[i] >= 0.0) || !std::isfinite(alphas[i]))
            return lfail(SU2_EINVAL, "alpha must be finite and >= 0");
    double *d_a = nullptr, *d_k = nullptr;
    if (hipMalloc(&d_a, (size_t)n * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_k, (size_t)n * 33 * sizeof(double)) != hipSuccess) {
        hipGetLastError();
        if (d_a) hipFree(d_a);
        return lfail(SU2_ENOMEM, "cannot allocate");
    }
    hipError_t e = hipMemcpy(d_a, alphas, (size_t)n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cdf, dim3((uint32_t)n), dim3(kBlock), 0, nullptr, d_a, d_k);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(knots, d_k, (size_t)n * 33 * sizeof(double), hipMemcpyDeviceToHost);
    hipFree(d_a);
    hipFree(d_k);
    if (e != hipSuccess) return lfail(SU2_EDEVICE, "su2_cdf_knots: %s", hipGetErrorString(e));
    return SU2_OK;
}

int su2_mlp_set_params(const float *params, size_t n)
{
    if (!params || n != (size_t)kNParam) return lfail(SU2_EINVAL, "expected %d parameters", kNParam);
    int rc = ensure_params();
    if (rc) return rc;
    LTRY(hipMemcpy(LN.master, params, kNParam * sizeof(float), hipMemcpyHostToDevice));
    LTRY(hipMemset(LN.m, 0, kNParam * sizeof(float)));
    LTRY(hipMemset(LN.v, 0, kNParam * sizeof(float)));
    LTRY(hipMemset(LN.step, 0, sizeof(int32_t)));
    hipLaunchKernelGGL(k_to_bf16, dim3(nb(kNParam)), dim3(256), 0, nullptr, LN.master, LN.P);
    LTRY(hipGetLastError());
    LTRY(hipDeviceSynchronize());
    LN.have_params = true;
    return SU2_OK;
}

int su2_mlp_get_params(float *master, uint16_t *bf16, size_t n)
{
    int rc = need_params();
    if (rc) return rc;
    if (n != (size_t)kNParam) return lfail(SU2_EINVAL, "expected %d parameters", kNParam);
    if (master) LTRY(hipMemcpy(master, LN.master, kNParam * sizeof(float), hipMemcpyDeviceToHost));
    if (bf16) LTRY(hipMemcpy(bf16, LN.P, kNParam * sizeof(uint16_t), hipMemcpyDeviceToHost));
    return SU2_OK;
}

int su2_mlp_forward(const float *alphas, int32_t n, float *knots)
{
    int rc = need_params();
    if (rc) return rc;
    if (n < 1 || !alphas || !knots) return lfail(SU2_EINVAL, "bad arguments");
    rc = ensure_batch((uint32_t)n);
    if (rc) return rc;
    LTRY(hipMemcpy(LN.alpha, alphas, (size_t)n * sizeof(float), hipMemcpyHostToDevice));
    LTRY(forward((uint32_t)n, true, false));
    LTRY(hipMemcpy(knots, LN.knots, (size_t)n * 33 * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
}

int su2_mlp_loss_grad(const float *alphas, const float *target_logw, int32_t n, float *loss,
                      float *grad)
{
    int rc = need_params();
    if (rc) return rc;
    if (n < 1 || !alphas || !target_logw || !loss || !grad) return lfail(SU2_EINVAL, "bad arguments");
    rc = ensure_batch((uint32_t)n);
    if (rc) return rc;
    LTRY(hipMemcpy(LN.alpha, alphas, (size_t)n * sizeof(float), hipMemcpyHostToDevice));
    LTRY(hipMemcpy(LN.target, target_logw, (size_t)n * kSeg * sizeof(float), hipMemcpyHostToDevice));
    LTRY(forward((uint32_t)n, false, true));
    LTRY(backward((uint32_t)n));
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kBlock), 0, nullptr, LN.terms, (uint32_t)n, LN.loss1,
                       nullptr);
    LTRY(hipGetLastError());
    float l = 0.f;
    LTRY(hipMemcpy(&l, LN.loss1, sizeof(float), hipMemcpyDeviceToHost));
    LTRY(hipMemcpy(grad, LN.grad, kNParam * sizeof(float), hipMemcpyDeviceToHost));
    *loss = l;
    return SU2_OK;
}

int su2_mlp_train(const double *alphas, int32_t n, int32_t steps, float lr0, float lr_min,
                  float *loss_hist)
{
    int rc = need_params();
    if (rc) return rc;
    if (n < 1 || steps < 0 || !alphas || !(lr0 > 0.f) || !(lr_min >= 0.f))
        return lfail(SU2_EINVAL, "bad arguments");
    for (int32_t i = 0; i < n; ++i)
        if (!(alphas[i] >= 0.0) || alphas[i] > (double)kAlphaMax)
            return lfail(SU2_EINVAL, "training alphas must lie in [0, %g]", (double)kAlphaMax);
    rc = ensure_batch((uint32_t)n);
    if (rc) return rc;
    const uint32_t B = (uint32_t)n;
    double *d_a = nullptr, *d_k = nullptr;
    float *d_hist = nullptr;
    if (hipMalloc(&d_a, B * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_k, (size_t)B * 33 * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_hist, (size_t)std::max(1, steps) * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        if (d_a) hipFree(d_a);
        if (d_k) hipFree(d_k);
        return lfail(SU2_ENOMEM, "cannot allocate training buffers");
    }
    // everything below runs in order on one stream of its own: the targets,
    // the optimiser reset, then the replayed training steps
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    // targets: the method's own numerically integrated CDF knots, on the device
    if (e == hipSuccess) e = hipMemcpyAsync(d_a, alphas, B * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cdf, dim3(B), dim3(kBlock), 0, st, d_a, d_k);
        hipLaunchKernelGGL(k_logw, dim3(nb((size_t)B * kSeg)), dim3(256), 0, st, d_k, B, LN.target);
        hipLaunchKernelGGL(k_f64_to_f32, dim3(nb(B)), dim3(256), 0, st, d_a, B, LN.alpha);
        e = hipGetLastError();
    }
    // each call is a fresh run of Adam from the current parameters: step
    // counter and both moment estimates start at zero
    if (e == hipSuccess) e = hipMemsetAsync(LN.step, 0, sizeof(int32_t), st);
    if (e == hipSuccess) e = hipMemsetAsync(LN.m, 0, kNParam * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(LN.v, 0, kNParam * sizeof(float), st);
    // one training step as a graph: forward, loss, backward, Adam, step tick
    if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_l1, dim3(nb((size_t)B * kH)), dim3(256), 0, st, LN.P, LN.alpha, B, LN.a1, LN.h1);
        hipLaunchKernelGGL(k_l2, dim3(nb((size_t)B * kH)), dim3(256), 0, st, LN.P, LN.h1, B, LN.a2, LN.h2);
        hipLaunchKernelGGL(k_l3, dim3(nb((size_t)B * kOut)), dim3(256), 0, st, LN.P, LN.h2, B, LN.z);
        hipLaunchKernelGGL(k_head, dim3(nb(B)), dim3(256), 0, st, LN.z, B, LN.target, nullptr, LN.dz,
                           LN.terms);
        hipLaunchKernelGGL(k_loss, dim3(1), dim3(kBlock), 0, st, LN.terms, B, d_hist, LN.step);
        hipLaunchKernelGGL(k_bwd3, dim3(nb((size_t)B * kH)), dim3(256), 0, st, LN.P, LN.dz, LN.a2, B, LN.da2);
        hipLaunchKernelGGL(k_bwd2, dim3(nb((size_t)B * kH)), dim3(256), 0, st, LN.P, LN.da2, LN.a1, B, LN.da1);
        hipLaunchKernelGGL(k_wgrad_part, dim3(nchunks(B)), dim3(kBlock), 0, st, LN.alpha, LN.h1, LN.h2,
                           LN.dz, LN.da2, LN.da1, B, LN.part);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(kNParam)), dim3(256), 0, st, LN.part, nchunks(B),
                           LN.grad);
        hipLaunchKernelGGL(k_adam, dim3(nb(kNParam)), dim3(256), 0, st, LN.master, LN.P, LN.grad, LN.m,
                           LN.v, LN.step, lr0, lr_min, steps);
        hipLaunchKernelGGL(k_step_tick, dim3(1), dim3(1), 0, st, LN.step);
        e = hipStreamEndCapture(st, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int32_t i = 0; i < steps && e == hipSuccess; ++i) e = hipGraphLaunch(exec, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && loss_hist && steps > 0)
        e = hipMemcpy(loss_hist, d_hist, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost);
    if (st) hipStreamSynchronize(st);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (st) hipStreamDestroy(st);
    hipFree(d_a);
    hipFree(d_k);
    hipFree(d_hist);
    if (e != hipSuccess) return lfail(SU2_EDEVICE, "su2_mlp_train: %s", hipGetErrorString(e));
    return SU2_OK;
}

int su2_mlp_tabulate(int32_t points)
{
    int rc = need_params();
    if (rc) return rc;
    if (points < 2 || points > (1 << 20)) return lfail(SU2_EINVAL, "points must be in 2..2^20");
    const uint32_t G = (uint32_t)points;
    rc = ensure_batch(G);
    if (rc) return rc;
    std::vector<float> a(G);
    for (uint32_t g = 0; g < G; ++g) a[g] = (float)((double)g * kAlphaMax / (double)(G - 1));
    LTRY(hipMemcpy(LN.alpha, a.data(), G * sizeof(float), hipMemcpyHostToDevice));
    LTRY(forward(G, true, false));
    if (LN.table && LN.G != G) {
        hipFree(LN.table);
        LN.table = nullptr;
    }
    if (!LN.table && hipMalloc(&LN.table, (size_t)G * 33 * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        return lfail(SU2_ENOMEM, "cannot allocate the knot table");
    }
    LTRY(hipMemcpy(LN.table, LN.knots, (size_t)G * 33 * sizeof(float), hipMemcpyDeviceToDevice));
    LTRY(hipDeviceSynchronize());
    LN.G = G;
    return SU2_OK;
}

int su2_cdf_tabulate(int32_t points)
{
    if (points < 2 || points > (1 << 16)) return lfail(SU2_EINVAL, "points must be in 2..65536");
    const uint32_t G = (uint32_t)points, n = G * 33u;
    std::vector<double> a(G);
    for (uint32_t g = 0; g < G; ++g) a[g] = (double)g * (double)kAlphaMax / (double)(G - 1);
    double *d_a = nullptr, *d_k = nullptr;
    if (hipMalloc(&d_a, G * sizeof(double)) != hipSuccess || hipMalloc(&d_k, n * sizeof(double)) != hipSuccess) {
        hipGetLastError();
        if (d_a) hipFree(d_a);
        return lfail(SU2_ENOMEM, "cannot allocate");
    }
    if (LN.table && LN.G != G) {
        hipFree(LN.table);
        LN.table = nullptr;
        LN.G = 0;
    }
    hipError_t e = hipSuccess;
    if (!LN.table && hipMalloc(&LN.table, (size_t)n * sizeof(float)) != hipSuccess) {
        hipGetLastError();
        LN.table = nullptr;
        e = hipErrorOutOfMemory;
    }
    if (e == hipSuccess) e = hipMemcpy(d_a, a.data(), G * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cdf, dim3(G), dim3(kBlock), 0, nullptr, d_a, d_k);
        hipLaunchKernelGGL(k_f64_to_f32, dim3(nb(n)), dim3(256), 0, nullptr, d_k, n, LN.table);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hipFree(d_a);
    hipFree(d_k);
    if (e != hipSuccess) {
        LN.G = 0;
        return lfail(e == hipErrorOutOfMemory ? SU2_ENOMEM : SU2_EDEVICE, "su2_cdf_tabulate: %s",
                     hipGetErrorString(e));
    }
    LN.G = G;
    return SU2_OK;
}

int su2_mlp_table(float *host_out, size_t n_floats)
{
    if (!LN.table) return lfail(SU2_ESTATE, "no table: call su2_mlp_tabulate");
    if (!host_out || n_floats != (size_t)LN.G * 33) return lfail(SU2_EINVAL, "n_floats must be 33*G");
    LTRY(hipMemcpy(host_out, LN.table, n_floats * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
}

const char *su2_mlp_last_error(void) { return lerr; }

}  // extern "C"
