// su2_pass.hpp -- one tile of a heat-bath pass (Sec. 2.4, Eqs. (5)-(7)): the
// Eq. (6) staple from 18 gathered links, the capped Kennedy-Pendleton draw,
// the direction, rotation, FP64-normed reunitarisation and the store; shared by
// the single-lattice pass kernel and the batched-replica kernels.
#pragma once

#include "su2_device.hpp"

namespace su2 {

constexpr int kBlock = 256;
constexpr int kWave = 64;

// Knot table of the learned proposal: rows g = 0..G-1 hold the 33 knots
// y_0 = -1 < ... < y_32 = +1 of the 32 equal-probability segments of x0 at
// alpha_g = g * alpha_max / (G - 1).  Knots at other alpha <= alpha_max are the
// linear mix of the two neighbouring rows (still monotone with the same ends).
// The descriptor travels by value as a kernel argument, so its fields are at
// hand with the other arguments when a wave starts.
struct ImhTable {
    const float *knots = nullptr;          // [G][33], zero-padded to >= kImhLdsVec4 float4
    uint32_t G = 0;
    float alpha_max = 0.0f;
    float inv_step = 0.0f;                 // (G - 1) / alpha_max
    // not part of the table: the plain heat-bath's switch to Creutz's draw
    // (alpha below it; 0 = Kennedy-Pendleton throughout), carried here
    // because every pass kernel receives this descriptor
    float creutz_below = 0.0f;
    unsigned long long *stats = nullptr;   // per wave: (proposals, accepts)
};

// Tables of at most kImhLdsRows rows are read from LDS, larger ones from global
// memory.  Every workgroup copies the first kImhLdsVec4 float4 of the table
// (31 rows of 33 knots fill 1023 of its 1024 floats) straight from global
// memory into LDS: one 16-byte copy per lane, issued right behind the staple
// gathers, with no branch and no register held (the table buffer is padded to
// at least that size).  The launch provides kImhLdsBytes of dynamic LDS.
constexpr uint32_t kImhLdsVec4 = kBlock;
constexpr uint32_t kImhLdsRows = kImhLdsVec4 * 4u / 33u;  // 31
constexpr uint32_t kImhLdsBytes = kImhLdsVec4 * 16u;

// ---------------------------------------------------------------------------
// The three directions nu != mu, as compile-time constants.
template <uint32_t MU, int I>
constexpr uint32_t other_dir()
{
    return (uint32_t)(I < (int)MU ? I : I + 1);
}

// The six gathered links of the two staples of U_mu(x) in the plane (mu, nu)
// (Eq. (6)): forward U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag and backward
// U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu).
struct StapleLinks {
    float4 a, b, c, d, e, f;
};

template <uint32_t MU, uint32_t NU, bool OFF32>
__device__ __forceinline__ StapleLinks gather(const float4 *L, const Geo &g, uint32_t p,
                                              uint32_t h, uint32_t h_pm, const Site &x)
{
    const uint32_t q = p ^ 1u;
    const uint32_t h_pn = h_plus<NU>(g, h, x.x[NU]);
    const uint32_t h_mn = h_minus<NU>(g, h, x.x[NU]);
    const uint32_t h_pm_mn = h_minus<NU>(g, h_pm, x.x[NU]);  // x+mu has the same x_nu
    const float4 *Lnp = L + arr(g, NU, p), *Lnq = L + arr(g, NU, q), *Lmq = L + arr(g, MU, q);
    StapleLinks s;
    s.a = ld4<OFF32>(Lnp, h);         // U_nu(x)
    s.b = ld4<OFF32>(Lmq, h_pn);      // U_mu(x+nu)
    s.c = ld4<OFF32>(Lnq, h_pm);      // U_nu(x+mu)
    s.d = ld4<OFF32>(Lnq, h_mn);      // U_nu(x-nu)
    s.e = ld4<OFF32>(Lmq, h_mn);      // U_mu(x-nu)
    s.f = ld4<OFF32>(Lnp, h_pm_mn);   // U_nu(x+mu-nu)
    return s;
}

__device__ __forceinline__ float4 staple_sum(const StapleLinks &s)
{
    return qadd(qmul(qmul(s.a, s.b), qdag(s.c)), qmul(qmul(qdag(s.d), s.e), s.f));
}

// ln u for a uniform u in [2^-24, 1] (never denormal, never 0): the hardware
// base-2 logarithm times ln 2 carried in two parts -- the steps the library
// logf takes for normal arguments, without its denormal and infinity cases.
__device__ __forceinline__ float ln_unit(float u)
{
#pragma clang fp contract(off)
    constexpr float kLn2Hi = 0x1.62e42ep-1f, kLn2Lo = 0x1.efa39ep-25f;
    const float l = __builtin_amdgcn_logf(u);
    const float r = l * kLn2Hi;
    float e = __builtin_fmaf(l, kLn2Hi, -r);
    e = __builtin_fmaf(l, kLn2Lo, e);
    return __builtin_fmaf(l, kLn2Hi, e);
}

// cos^2(2 pi u) for a uniform u = k 2^-24 in (0, 1]: with x = 2u - rint(2u) in
// [-1/2, 1/2] and y = 1/2 - |x| (both exact), cos^2(2 pi u) = sin^2(pi y) =
// s R(s), s = y^2, where R(s) = sin^2(pi y) / y^2 is a degree-5 polynomial in s
// fitted on [0, 1/4] for relative error (1.4e-8 in exact arithmetic, within
// 2e-7 of the true value once evaluated in FP32 -- checked on all 2^24
// uniforms).  A dozen instructions, where the library's cospif and a square
// take about thirty; the result only feeds the Gaussian part of lambda^2.
__device__ __forceinline__ float cos2_2pi(float u)
{
#pragma clang fp contract(off)
    const float t = 2.0f * u;
    const float x = t - __builtin_rintf(t);
    const float y = 0.5f - __builtin_fabsf(x);
    const float s = y * y;
    float r = -0x1.ab08f6p+1f;
    r = __builtin_fmaf(r, s, 0x1.a13006p+3f);
    r = __builtin_fmaf(r, s, -0x1.e193acp+4f);
    r = __builtin_fmaf(r, s, 0x1.55d0cp+5f);
    r = __builtin_fmaf(r, s, -0x1.03c1dep+5f);
    r = __builtin_fmaf(r, s, 0x1.3bd3ccp+3f);
    return s * r;
}

// One Kennedy-Pendleton attempt from uniforms u0..u3 at coupling alpha:
// lambda^2 = -(ln u0 + cos^2(2 pi u1) ln u2) / (2 alpha), accepted iff
// u3^2 <= 1 - lambda^2.  The test is taken multiplied through by 2 alpha > 0,
// 2 alpha (1 - u3^2) + num >= 0 with num = ln u0 + cos^2 ln u2 = -2 alpha
// lambda^2, so an attempt needs no division; lambda^2 itself is formed once,
// for the accepted attempt (kp_lambda2).  Every operation rounds as written:
// the decision is taken in FP32.
__device__ __forceinline__ float kp_num(float u0, float u1, float u2)
{
#pragma clang fp contract(off)
    return ln_unit(u0) + cos2_2pi(u1) * ln_unit(u2);
}

__device__ __forceinline__ bool kp_accept(float u3, float num, float two_alpha)
{
#pragma clang fp contract(off)
    return __builtin_fmaf(two_alpha, 1.0f - u3 * u3, num) >= 0.0f;
}

__device__ __forceinline__ float kp_lambda2(float num, float two_alpha)
{
#pragma clang fp contract(off)
    return -num / two_alpha;
}

// Creutz's draw (Phys. Rev. D 21 (1980) 2308), the better heat-bath at small
// alpha: y uniform on [exp(-2 alpha), 1] makes x0 = 1 + ln(y) / alpha
// distributed as exp(alpha x0) on [-1, 1], and the attempt is accepted with
// probability sqrt(1 - x0^2).  With m = 1 - x0 = -ln(y) / alpha (so m / 2
// plays the part of lambda^2) and y = 1 + z, z = -(1 - u) d, d = 1 - exp(-2
// alpha) (formed once per update, with expm1), this returns L = alpha m =
// -ln(1 + z); the test and m need only one division, for the accepted attempt.
// ln(1 + z) is Kahan's ln(y) z / (y - 1) with y the rounded 1 + z: the factor
// undoes the rounding of y, so L keeps a few ulps as z -> 0 (m accurate as
// alpha -> 0) with the hardware log2, which is within one ulp of its result
// also next to 1.
__device__ __forceinline__ float creutz_l(float u, float d)
{
#pragma clang fp contract(off)
    const float z = -(1.0f - u) * d;  // in (-1, 0]
    const float y = 1.0f + z;
    const float l = -(ln_unit(y) * (z * __builtin_amdgcn_rcpf(y - 1.0f)));
    return y == 1.0f ? -z : l;
}

// u1 <= sqrt(1 - x0^2) with 1 - x0^2 = m (2 - m) = L (2 alpha - L) / alpha^2,
// taken multiplied by alpha^2: L (2 alpha - L) - (alpha u1)^2 >= 0
__device__ __forceinline__ bool creutz_accept(float u1, float l, float alpha, float two_alpha)
{
#pragma clang fp contract(off)
    const float au = alpha * u1;
    return __builtin_fmaf(l, two_alpha - l, -(au * au)) >= 0.0f;
}

// A double moved across lanes by a DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum of v over the 64 lanes of a wave (every lane active), the same value in
// every lane, in a fixed order: DPP moves inside each row of 16 lanes (quad
// permutations xor 1 and xor 2, half-row mirror, row mirror; each step adds
// the partner's partial, so every lane of a row ends with the row's sum) and
// the four row sums read out and added as (0 + 1) + (2 + 3).  Register moves,
// where shuffles through LDS would cost a dependent round trip per step.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Block-level FP64 sum of two values: wave sums, then waves in order (fixed
// structure, so the result does not depend on scheduling).
__device__ __forceinline__ double2 block_sum2(double a, double b)
{
    __shared__ double sh[2][kBlock / kWave];
    a = wave_sum(a);
    b = wave_sum(b);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
    }
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
        for (int i = 0; i < kBlock / kWave; ++i) {
            r.x += sh[0][i];
            r.y += sh[1][i];
        }
    }
    return r;
}

// The same for one value (the result in thread 0).
__device__ __forceinline__ double block_sum(double a)
{
    __shared__ double sh1[kBlock / kWave];
    a = wave_sum(a);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) sh1[wv] = a;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / kWave; ++i) r += sh1[i];
    return r;
}

// (e^z - 1) / z for z >= 0 to a few units in the last place: the Taylor
// series to z^4 below 1/16 (the remainder, about z^5/720, is below 2^-29),
// hardware exp2 above (where e^z - 1 >= e^z / 17 keeps the subtraction's
// relative error near 2e-6 at worst).
// z <= 80 in use, so e^z stays finite.
__device__ __forceinline__ float expm1_over(float z)
{
#pragma clang fp contract(off)
    if (z < 0.0625f)
        return __builtin_fmaf(z, __builtin_fmaf(z, __builtin_fmaf(z, __builtin_fmaf(z, 0x1.111112p-7f, 0x1.555556p-5f),
                                                                   0x1.555556p-3f), 0.5f), 1.0f);
    return (__builtin_amdgcn_exp2f(z * 1.44269504f) - 1.0f) * __builtin_amdgcn_rcpf(z);
}

// ln(1 + t) / t for t >= 0: the series to t^6 below 1/16 (remainder below
// t^7/8 < 2^-31), hardware log2 of the rounded 1 + t above (relative error
// below 1e-6 there)
__device__ __forceinline__ float log1p_over(float t)
{
#pragma clang fp contract(off)
    if (t < 0.0625f) {
        float q = __builtin_fmaf(t, 0x1.24924ap-3f, -0x1.555556p-3f);
        q = __builtin_fmaf(t, q, 0.2f);
        q = __builtin_fmaf(t, q, -0.25f);
        q = __builtin_fmaf(t, q, 0x1.555556p-2f);
        q = __builtin_fmaf(t, q, -0.5f);
        return __builtin_fmaf(t, q, 1.0f);
    }
    return __builtin_amdgcn_logf(1.0f + t) * 0.693147181f * __builtin_amdgcn_rcpf(t);
}

// Independence-Metropolis decision of the learned proposal at one link.  r0
// points at row g0 of the knot table (row g0 + 1 follows at r0 + 33); the
// proposal's knots are the rows' linear mix with weight f (y_0 = -1 and
// y_32 = +1 in every row).  Segment j = floor(32 u0) is chosen with
// probability 1/32 and x0 drawn inside it from the density proportional to
// exp(alpha x) -- the exponential factor of the target, so that only the
// slowly varying sqrt(1 - x^2) is left for the accept step to correct.  u1
// decides; xc is the current link's x0.  Returns whether the proposal is
// accepted and sets xp (the proposed x0) and num = 1 - xp^2.  Ptr is an LDS
// or a global pointer type, so each table location gets its own load
// instructions.
//
// With w = y_{j+1} - y_j, E = e^{alpha w} - 1 and s = E / alpha (which stays
// finite as alpha -> 0), the draw is x = y_j + ln(1 + v E) / alpha for
// v = 32 u0 - j, and the proposal density is q(x) = e^{alpha (x - y_j)} / (32 s).
// The target pi(x) = sqrt(1 - x^2) e^{alpha x} over q is then
// 32 sqrt(1 - x^2) e^{alpha y_j} s, and the acceptance ratio
// r = sqrt((1 - x'^2) / (1 - xc^2)) e^{alpha (y_j' - y_jc)} s_j' / s_jc.
template <typename Ptr>
__device__ __forceinline__ bool imh_decide(Ptr r0, float f, float u0, float u1, float alpha,
                                           float xc, float &xp, float &num)
{
#pragma clang fp contract(off)
    auto knot = [&](uint32_t j) { return r0[j] + f * (r0[33u + j] - r0[j]); };
    // the proposal's segment and its two knots
    const uint32_t jp = min((uint32_t)(32.0f * u0), 31u);
    const float ya = knot(jp), yb = knot(jp + 1u);
    // segment [y_lo, y_lo+1) of the current value: for non-decreasing knots
    // the largest lo in 0..31 with y_lo <= xc (y_0 = -1), by a five-step
    // binary search -- few registers live, which keeps more waves resident
    uint32_t lo = 0u;
#pragma unroll
    for (uint32_t step = 16u; step >= 1u; step >>= 1)
        if (xc >= knot(lo + step)) lo += step;
    const float ylo = lo == 0u ? -1.0f : knot(lo);
    const float yhi = lo == 31u ? 1.0f : knot(lo + 1u);
    const float wp = yb - ya, wc = yhi - ylo;
    const float v = 32.0f * u0 - (float)jp;  // exact
    const float zp = alpha * wp, zc = alpha * wc;
    // x' and the ratio E_j' / E_jc (= s_j' / s_jc).  With alpha >= 1/8 and both
    // z = alpha w >= 1/256 (segments of a table near the integrated one are
    // wider than 1/30 at small alpha, so that is nearly every update), e^z - 1
    // and ln(1 + v E) straight from hardware exp2 and log2 (absolute error
    // ~1.2e-7 in e^z and ~6e-8 in 1 + v E) move x' by about 2e-7 / alpha at
    // most and the ratio by 1.2e-7 / z <= 3e-5 relative; otherwise the series
    // forms keep a few ulps down to alpha -> 0.
    float e_ratio;
    if (alpha >= 0.125f && zp >= 0x1p-8f && zc >= 0x1p-8f) {
        const float Ep = __builtin_amdgcn_exp2f(zp * 1.44269504f) - 1.0f;
        const float Ec = __builtin_amdgcn_exp2f(zc * 1.44269504f) - 1.0f;
        xp = ya + __builtin_amdgcn_logf(__builtin_fmaf(v, Ep, 1.0f)) *
                      (0.693147181f * __builtin_amdgcn_rcpf(alpha));
        e_ratio = Ep * __builtin_amdgcn_rcpf(Ec);
    } else {
        // ln(1 + v E) / alpha = v s Q(v E), Q(t) = ln(1 + t) / t
        const float sp = wp * expm1_over(zp), sc = wc * expm1_over(zc);
        const float vs = v * sp;
        xp = ya + vs * log1p_over(alpha * vs);
        e_ratio = sp * __builtin_amdgcn_rcpf(sc);
    }
    num = 1.0f - xp * xp;
    const float den = 1.0f - xc * xc;
    // the target density vanishes at the proposal, or the proposal sits on a
    // segment of zero (or, from rounding, negative) width, an atom of q:
    // reject; else if it vanishes at the current value, or the current value
    // sits on such a segment: accept
    if (num <= 0.0f || !(wp > 0.0f)) return false;
    if (den <= 0.0f || !(wc > 0.0f)) return true;
    // alpha <= 40 keeps alpha (y_j' - y_jc) within +-80.  Overflow to +inf
    // needs a true ratio far above 1 (accept), underflow to 0 one far below
    // u1 >= 2^-24 (reject).
    // Hardware exp2, rcp and sqrt carry relative errors of order 1e-6, far
    // inside the statistical slack of an accept decision.
    const float e = __builtin_amdgcn_exp2f(alpha * (ya - ylo) * 1.44269504f);
    const float ratio = __builtin_amdgcn_sqrtf(num * __builtin_amdgcn_rcpf(den)) * (e * e_ratio);
    return u1 <= ratio;
}

// The links one tile's updates read before any arithmetic: the 18 staple
// links of every lane and, for the learned proposal, the lane's old link; lex
// is the lane's lexicographic site index (the Philox counter's first word).
struct TileLoad {
    StapleLinks s0, s1, s2;
    float4 uold;
    uint32_t lex;
};

// The loads of the update of U_MU(x) at the site x of parity p with half index
// hh (any lane may call it with a valid site).
template <uint32_t MU, bool OFF32, bool IMH>
__device__ __forceinline__ TileLoad load_site(const float4 *__restrict__ L, const Geo &g, uint32_t p,
                                              uint32_t hh, const Site &x)
{
    constexpr uint32_t N0 = other_dir<MU, 0>(), N1 = other_dir<MU, 1>(), N2 = other_dir<MU, 2>();
    const uint32_t h_pm = h_plus<MU>(g, hh, x.x[MU]);
    TileLoad t;
    t.lex = 2u * hh + (x.x[0] & 1u);  // L0 = 2*H0, so lex = 2h + (x0 mod 2)
    t.s0 = gather<MU, N0, OFF32>(L, g, p, hh, h_pm, x);
    t.s1 = gather<MU, N1, OFF32>(L, g, p, hh, h_pm, x);
    t.s2 = gather<MU, N2, OFF32>(L, g, p, hh, h_pm, x);
    // the old link does not depend on the staple, so its load goes out with
    // the gathers
    t.uold = IMH ? ld4<OFF32>(L + arr(g, MU, p), hh) : make_float4(0.f, 0.f, 0.f, 0.f);
    return t;
}

template <uint32_t MU, bool OFF32, bool IMH>
__device__ __forceinline__ TileLoad load_tile(const float4 *__restrict__ L, const Geo &g, uint32_t p,
                                              uint32_t tile)
{
    const uint32_t h = tile * kBlock + threadIdx.x;
    const uint32_t hh = h < g.half ? h : 0u;
    return load_site<MU, OFF32, IMH>(L, g, p, hh, site_of(g, hh, p));
}

// Learned proposal: every workgroup copies the first kImhLdsVec4 float4 of the
// knot table into LDS, one 16-byte global-to-LDS load per lane (lane l of
// wave v lands at float4 64 v + l); update_tile waits for it at a barrier.
__device__ __forceinline__ void stage_table(const ImhTable &imh)
{
    extern __shared__ float4 imh_lds[];
    const uint32_t wv = threadIdx.x / kWave;
    __builtin_amdgcn_global_load_lds(
        (const __attribute__((address_space(1))) void *)(reinterpret_cast<const float4 *>(imh.knots) + threadIdx.x),
        (__attribute__((address_space(3))) void *)(imh_lds + wv * kWave), 16u, 0, 0);
}

// What an update needs of its loads once the staples are formed: the three
// plane staples (the plaquette measurement uses those with nu < MU), their sum
// w (Eq. (6)), the old link (learned proposal) and lex.
struct TileStaples {
    float4 w0, w1, w2, w;
    float4 uold;
    uint32_t lex;
};

__device__ __forceinline__ TileStaples staples_of(const TileLoad &in)
{
    TileStaples t;
    t.w0 = staple_sum(in.s0);
    t.w1 = staple_sum(in.s1);
    t.w2 = staple_sum(in.s2);
    t.w = qadd(qadd(t.w0, t.w1), t.w2);
    t.uold = in.uold;
    t.lex = in.lex;
    return t;
}

// The update of one link U_MU(x), parity(x) = p, half index h, at sweep index
// s, from the staples in `in`, by every lane of a wave (lanes with !valid take
// part in the wave-wide steps only); counter_slot names the wave's pair of
// counters.  Returns the link's value after the update when KEEP is set (a
// lane whose heat-bath hit the cap re-reads its unchanged link).  With MEASURE
// (even passes MU >= 1 of a measured sweep), meas receives dot(U_new,
// staple_nu) summed over nu < MU: over the three even passes this counts every
// plaquette of the final configuration exactly once (planes (nu, MU), nu < MU),
// so the plaquette of the sweep's result comes out of the sweep itself.  With
// IMH the caller has made the staged knot table visible (a barrier).  With
// CREUTZ, lanes whose alpha is below imh.creutz_below draw Creutz's way.
template <uint32_t MU, bool OFF32, bool MEASURE, bool IMH, bool KEEP, bool CREUTZ = false>
__device__ __forceinline__ float4 update_link(float4 *__restrict__ L, const Geo &g, Key key,
                                              float beta, uint32_t p, uint32_t s, uint32_t h,
                                              bool valid, uint32_t counter_slot,
                                              const TileStaples &in,
                                              unsigned long long *__restrict__ counters,
                                              const ImhTable &imh, double &meas)
{
    // every operation rounds as written, whatever kernel inlines this
#pragma clang fp contract(off)
    constexpr uint32_t N0 = other_dir<MU, 0>(), N1 = other_dir<MU, 1>(), N2 = other_dir<MU, 2>();
    const uint32_t lex = in.lex;
    float4 *Lout = L + arr(g, MU, p);
    [[maybe_unused]] const float4 uold = in.uold;
    const float4 w0 = in.w0, w1 = in.w1, w2 = in.w2;
    const float4 w = in.w;
    const float k = sqrtf(qdot(w, w));
    const float alpha = beta * k;
    const bool haar_branch = valid && alpha == 0.0f;
    // learned proposal: one independence-Metropolis step for alpha in the
    // table's range; the plain heat-bath stays the fallback outside it
    bool imh_lane = false;
    if constexpr (IMH) imh_lane = valid && !haar_branch && alpha <= imh.alpha_max;
    bool done = !valid || haar_branch || imh_lane;
    // below the switch the attempts draw Creutz's way (same cap, same slots)
    const bool creutz = CREUTZ && alpha < imh.creutz_below;
    const float two_alpha = 2.0f * alpha;
    float creutz_d = 0.0f;  // 1 - exp(-2 alpha), for the Creutz lanes
    if constexpr (CREUTZ)
        if (creutz) creutz_d = -expm1f(-two_alpha);
    float lam2 = 0.0f, num_acc = 0.0f;
    unsigned long long attempts = 0;
    for (uint32_t t = 0; t < 8u; ++t) {
        const unsigned long long pending = __ballot(!done);
        if (pending == 0ull) break;
        attempts += __popcll(pending);
        if (!done) {
            const uint4 r = draw(key, lex, MU, kPurposeUpdate, s, t);
            if (creutz) {
                const float l = creutz_l(unit24(r.x), creutz_d);
                if (creutz_accept(unit24(r.y), l, alpha, two_alpha)) {
                    done = true;
                    num_acc = l;
                }
            } else {
                const float num = kp_num(unit24(r.x), unit24(r.y), unit24(r.z));
                if (kp_accept(unit24(r.w), num, two_alpha)) {
                    done = true;
                    num_acc = num;
                }
            }
        }
    }
    // lambda^2 of the accepted attempt: -num / (2 alpha) (Kennedy-Pendleton) or
    // m / 2 = L / (2 alpha) (Creutz)
    lam2 = kp_lambda2(creutz ? -num_acc : num_acc, two_alpha);
    const bool failed = valid && !done;
    const unsigned long long failures = __popcll(__ballot(failed));
    float4 un = make_float4(0.f, 0.f, 0.f, 0.f);
    // a new link X V with X = (x0n, amag * direction); the direction comes from
    // two uniforms (cos theta = 2 u - 1, phi = 2 pi u') of the lane's draw
    bool rotate = false;
    float x0n = 0.0f, amag = 0.0f;
    uint32_t rz = 0u, rphi = 0u;
    if constexpr (IMH) {
        bool rejected = false;
        const bool staged = imh.G <= kImhLdsRows;
        if (imh_lane) {
            const float tpos = alpha * imh.inv_step;
            const uint32_t g0 = min((uint32_t)tpos, imh.G - 2u);
            const float f = tpos - (float)g0;
            const uint4 r = draw(key, lex, MU, kPurposeImh, s, 0u);
            const float ik = __builtin_amdgcn_rcpf(k);
            const float xc = fminf(1.0f, fmaxf(-1.0f, qdot(uold, w) * ik));
            float xp, num;
            bool acc;
            if (staged) {
                extern __shared__ float4 imh_lds[];
                acc = imh_decide((const __attribute__((address_space(3))) float *)imh_lds + 33u * g0, f,
                                 unit24(r.x), unit24(r.y), alpha, xc, xp, num);
            } else {
                acc = imh_decide((const __attribute__((address_space(1))) float *)imh.knots + 33u * g0, f,
                                 unit24(r.x), unit24(r.y), alpha, xc, xp, num);
            }
            // accepted: x0 = x'; rejected: x0 keeps the current value xc but the
            // direction about V is drawn afresh all the same (the target's
            // conditional of the direction given x0 is uniform, so this Gibbs
            // step costs nothing in exactness and refreshes the rejected link)
            rotate = true;
            x0n = acc ? xp : xc;
            amag = __builtin_amdgcn_sqrtf(acc ? num : fmaxf(0.0f, 1.0f - xc * xc));
            rz = r.z;
            rphi = r.w;
            rejected = !acc;
        }
        const unsigned long long nprop = __popcll(__ballot(imh_lane));
        const unsigned long long nacc = __popcll(__ballot(imh_lane && !rejected));
        if ((threadIdx.x & (kWave - 1)) == 0 && nprop != 0ull) {
            atomicAdd(&imh.stats[2 * counter_slot], nprop);
            atomicAdd(&imh.stats[2 * counter_slot + 1], nacc);
        }
    }
    if (valid && !failed && !imh_lane) {
        if (haar_branch) {
            un = unitize(haar(draw(key, lex, MU, kPurposeUpdate, s, kSlotHaar)));
            st4_stream<OFF32>(Lout, h, un);
        } else {
            const uint4 r = draw(key, lex, MU, kPurposeUpdate, s, kSlotDirection);
            rotate = true;
            x0n = 1.0f - 2.0f * lam2;
            amag = 2.0f * __builtin_amdgcn_sqrtf(lam2 * (1.0f - lam2));
            rz = r.x;
            rphi = r.y;
        }
    }
    if (rotate) {
        // the direction and the rotation feed only the link's value (checked to
        // 1e-5), not a decision: hardware sin/cos of 2 pi u (their argument in
        // revolutions), reciprocal and square root, each within a few ulp
        const float cz = 2.0f * unit24(rz) - 1.0f;
        const float sphi = __builtin_amdgcn_sinf(unit24(rphi));
        const float cphi = __builtin_amdgcn_cosf(unit24(rphi));
        const float sn = __builtin_amdgcn_sqrtf(1.0f - cz * cz);
        const float4 X = make_float4(x0n, amag * sn * cphi, amag * sn * sphi, amag * cz);
        const float ik = __builtin_amdgcn_rcpf(k);
        const float4 V = make_float4(w.x * ik, w.y * ik, w.z * ik, w.w * ik);
        un = unitize(qmul(X, V));
        st4_stream<OFF32>(Lout, h, un);
    }
    // each wave owns its two counters; the adds return nothing, so the wave
    // does not wait on a read-modify-write before it retires
    if ((threadIdx.x & (kWave - 1)) == 0 && attempts != 0ull) {
        atomicAdd(&counters[2 * counter_slot], attempts);
        if (failures != 0ull) atomicAdd(&counters[2 * counter_slot + 1], failures);
    }
    if constexpr (MEASURE || KEEP) {
        if (failed) un = ld4<OFF32>(Lout, h);  // the link kept its value
    }
    if constexpr (MEASURE) {
        double acc = 0.0;
        if (valid) {
            if (N0 < MU) acc += (double)qdot(un, w0);
            if (N1 < MU) acc += (double)qdot(un, w1);
            if (N2 < MU) acc += (double)qdot(un, w2);
        }
        meas = acc;
    }
    return un;
}

// The updates of one tile (256 half-sites) of a pass; meas_out receives the
// tile's FP64 plaquette partial (spatial planes, MU = 1, 2, in .x; temporal
// planes, MU = 3, in .y).  CREUTZ as in update_link.
template <uint32_t MU, bool OFF32, bool MEASURE, bool IMH, bool CREUTZ = false>
__device__ __forceinline__ void update_tile(float4 *__restrict__ L, const Geo &g, Key key,
                                            float beta, uint32_t p, uint32_t s, uint32_t tile,
                                            const TileStaples &in,
                                            unsigned long long *__restrict__ counters,
                                            double2 *__restrict__ meas_out, const ImhTable &imh)
{
    const uint32_t h = tile * kBlock + threadIdx.x;
    if constexpr (IMH) __syncthreads();  // the staged table is complete
    double acc = 0.0;
    update_link<MU, OFF32, MEASURE, IMH, false, CREUTZ>(L, g, key, beta, p, s, h, h < g.half, h / kWave,
                                                        in, counters, imh, acc);
    if constexpr (MEASURE) {
        const double r = block_sum(acc);
        if (threadIdx.x == 0)
            meas_out[tile] = MU == 3u ? make_double2(0.0, r) : make_double2(r, 0.0);
    }
}


// One tile of a pass: its loads, then its updates (the single-tile kernels and
// the batched-replica kernels, which take the heat-bath without the Creutz
// switch).
template <uint32_t MU, bool OFF32, bool MEASURE, bool IMH = false, bool CREUTZ = false>
__device__ __forceinline__ void pass_tile(float4 *__restrict__ L, const Geo &g, Key key,
                                          float beta, uint32_t p, uint32_t s, uint32_t tile,
                                          unsigned long long *__restrict__ counters,
                                          double2 *__restrict__ meas_out,
                                          const ImhTable &imh = ImhTable{})
{
    const TileLoad in = load_tile<MU, OFF32, IMH>(L, g, p, tile);
    if constexpr (IMH) stage_table(imh);
    update_tile<MU, OFF32, MEASURE, IMH, CREUTZ>(L, g, key, beta, p, s, tile, staples_of(in), counters,
                                                 meas_out, imh);
}

}  // namespace su2
