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
// y_0 = -1 < ... < y_32 = +1 of the piecewise-linear inverse CDF of x0 at
// alpha_g = g * alpha_max / (G - 1).  Knots at other alpha <= alpha_max are the
// linear mix of the two neighbouring rows (still monotone with the same ends).
struct ImhTable {
    const float *knots;          // [G][33]
    uint32_t G;
    float alpha_max;
    float inv_step;              // (G - 1) / alpha_max
    unsigned long long *stats;   // per wave: (proposals, accepts)
};

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

// lambda^2 of one Kennedy-Pendleton attempt; evaluated without contraction so
// each operation rounds as written (the accept decision is taken in FP32)
__device__ __forceinline__ float kp_lambda2(float u0, float u1, float u2, float alpha)
{
#pragma clang fp contract(off)
    const float c = cospif(2.0f * u1);
    const float num = logf(u0) + c * c * logf(u2);
    return -num / (2.0f * alpha);
}

__device__ __forceinline__ bool kp_accept(float u3, float lam2)
{
#pragma clang fp contract(off)
    return u3 * u3 <= 1.0f - lam2;
}

// Block-level FP64 sum of two values: wave butterflies, then waves in order
// (fixed structure, so the result does not depend on scheduling).
__device__ __forceinline__ double2 block_sum2(double a, double b)
{
    __shared__ double sh[2][kBlock / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
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

// One tile (256 half-sites) of a heat-bath pass over the links U_MU(x),
// parity(x) = p, at sweep index s.  All 18 gathers
// are issued before any arithmetic (MU is a template parameter so the three
// staple directions unroll).  With MEASURE (even passes MU >= 1 of a measured
// sweep), each lane also adds dot(U_new, staple_nu) for nu < MU: over the
// three even passes this counts every plaquette of the final configuration
// exactly once (planes (nu, MU), nu < MU), so the plaquette of the sweep's
// result comes out of the sweep itself.  meas_out receives one FP64 partial
// per tile.
template <uint32_t MU, bool OFF32, bool MEASURE, bool IMH = false>
__device__ __forceinline__ void pass_tile(float4 *__restrict__ L, const Geo &g, Key key,
                                          float beta, uint32_t p, uint32_t s, uint32_t tile,
                                          unsigned long long *__restrict__ counters,
                                          double2 *__restrict__ meas_out,
                                          const ImhTable *__restrict__ imh = nullptr)
{
    constexpr uint32_t N0 = other_dir<MU, 0>(), N1 = other_dir<MU, 1>(), N2 = other_dir<MU, 2>();
    const uint32_t h = tile * kBlock + threadIdx.x;
    const bool valid = h < g.half;
    const uint32_t hh = valid ? h : 0u;
    const Site x = site_of(g, hh, p);
    const uint32_t lex = 2u * hh + (x.x[0] & 1u);  // L0 = 2*H0, so lex = 2h + (x0 mod 2)
    const uint32_t h_pm = h_plus<MU>(g, hh, x.x[MU]);
    const StapleLinks s0 = gather<MU, N0, OFF32>(L, g, p, hh, h_pm, x);
    const StapleLinks s1 = gather<MU, N1, OFF32>(L, g, p, hh, h_pm, x);
    const StapleLinks s2 = gather<MU, N2, OFF32>(L, g, p, hh, h_pm, x);
    const float4 w0 = staple_sum(s0), w1 = staple_sum(s1), w2 = staple_sum(s2);
    const float4 w = qadd(qadd(w0, w1), w2);
    const float k = sqrtf(qdot(w, w));
    const float alpha = beta * k;
    const bool haar_branch = valid && alpha == 0.0f;
    // learned proposal: one independence-Metropolis step for alpha in the
    // table's range; the plain heat-bath stays the fallback outside it
    bool imh_lane = false;
    if constexpr (IMH) imh_lane = valid && !haar_branch && alpha <= imh->alpha_max;
    bool done = !valid || haar_branch || imh_lane;
    float lam2 = 0.0f;
    unsigned long long attempts = 0;
    for (uint32_t t = 0; t < 8u; ++t) {
        const unsigned long long pending = __ballot(!done);
        if (pending == 0ull) break;
        attempts += __popcll(pending);
        if (!done) {
            const uint4 r = draw(key, lex, MU, kPurposeUpdate, s, t);
            const float l = kp_lambda2(unit24(r.x), unit24(r.y), unit24(r.z), alpha);
            if (kp_accept(unit24(r.w), l)) {
                done = true;
                lam2 = l;
            }
        }
    }
    const bool failed = valid && !done;
    const unsigned long long failures = __popcll(__ballot(failed));
    float4 *Lout = L + arr(g, MU, p);
    float4 un = make_float4(0.f, 0.f, 0.f, 0.f);
    bool rejected = false;
    if constexpr (IMH) {
        if (imh_lane) {
            const float tpos = alpha * imh->inv_step;
            const uint32_t g0 = min((uint32_t)tpos, imh->G - 2u);
            const float f = tpos - (float)g0;
            const float *r0 = imh->knots + 33u * g0;
            const float *r1 = r0 + 33;
            auto knot = [&](uint32_t j) { return r0[j] + f * (r1[j] - r0[j]); };
            const uint4 r = draw(key, lex, MU, kPurposeImh, s, 0u);
            const float u0 = unit24(r.x);
            const uint32_t jp = min((uint32_t)(32.0f * u0), 31u);
            const float ya = knot(jp), yb = knot(jp + 1u);
            const float xp = ya + (32.0f * u0 - (float)jp) * (yb - ya);
            const float4 uold = ld4<OFF32>(Lout, h);
            const float ik = 1.0f / k;
            const float4 V = make_float4(w.x * ik, w.y * ik, w.z * ik, w.w * ik);
            const float xc = fminf(1.0f, fmaxf(-1.0f, qdot(uold, V)));
            uint32_t lo = 0u, hi = 32u;  // y_lo <= xc < y_hi
            while (hi - lo > 1u) {
                const uint32_t mid = (lo + hi) >> 1;
                if (xc >= knot(mid)) lo = mid; else hi = mid;
            }
            const float wc = knot(lo + 1u) - knot(lo);
            const float num = 1.0f - xp * xp, den = 1.0f - xc * xc;
            bool acc;
            if (num <= 0.0f) {
                acc = false;  // target density vanishes at the proposal
            } else if (den <= 0.0f) {
                acc = true;   // ... or at the current value
            } else {
                // log of [pi(x') / q(x')] / [pi(x) / q(x)], q = (1/32) / width
                const float lr = 0.5f * logf(num / den) + alpha * (xp - xc) + logf((yb - ya) / wc);
                acc = logf(unit24(r.y)) <= lr;
            }
            if (acc) {
                const float cz = 2.0f * unit24(r.z) - 1.0f;
                float sphi, cphi;
                sincospif(2.0f * unit24(r.w), &sphi, &cphi);
                const float sn = sqrtf(1.0f - cz * cz), am = sqrtf(num);
                const float4 X = make_float4(xp, am * sn * cphi, am * sn * sphi, am * cz);
                un = unitize(qmul(X, V));
                st4_stream<OFF32>(Lout, h, un);
            } else {
                un = uold;
                rejected = true;
            }
        }
        const unsigned long long nprop = __popcll(__ballot(imh_lane));
        const unsigned long long nacc = __popcll(__ballot(imh_lane && !rejected));
        if ((threadIdx.x & (kWave - 1)) == 0) {
            const uint32_t wave = h / kWave;
            imh->stats[2 * wave] += nprop;
            imh->stats[2 * wave + 1] += nacc;
        }
    }
    if (valid && !failed && !imh_lane) {
        if (haar_branch) {
            un = unitize(haar(draw(key, lex, MU, kPurposeUpdate, s, kSlotHaar)));
        } else {
            const uint4 r = draw(key, lex, MU, kPurposeUpdate, s, kSlotDirection);
            const float cz = 2.0f * unit24(r.x) - 1.0f;
            float sphi, cphi;
            sincospif(2.0f * unit24(r.y), &sphi, &cphi);
            const float sn = sqrtf(1.0f - cz * cz);
            const float a0 = 1.0f - 2.0f * lam2;
            const float am = 2.0f * sqrtf(lam2 * (1.0f - lam2));
            const float4 X = make_float4(a0, am * sn * cphi, am * sn * sphi, am * cz);
            const float ik = 1.0f / k;
            const float4 V = make_float4(w.x * ik, w.y * ik, w.z * ik, w.w * ik);
            un = unitize(qmul(X, V));
        }
        st4_stream<OFF32>(Lout, h, un);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const uint32_t wave = h / kWave;
        counters[2 * wave] += attempts;
        counters[2 * wave + 1] += failures;
    }
    if constexpr (MEASURE) {
        if (failed) un = ld4<OFF32>(Lout, h);  // the link kept its value
        double acc = 0.0;
        if (valid) {
            if (N0 < MU) acc += (double)qdot(un, w0);
            if (N1 < MU) acc += (double)qdot(un, w1);
            if (N2 < MU) acc += (double)qdot(un, w2);
        }
        const double2 r = block_sum2(acc, 0.0);
        // spatial planes (MU = 1, 2) in .x, temporal planes (MU = 3) in .y
        if (threadIdx.x == 0)
            meas_out[tile] = MU == 3u ? make_double2(0.0, r.x) : make_double2(r.x, 0.0);
    }
}

}  // namespace su2
