// su2_pair.hpp -- two consecutive passes of one parity in one launch: the
// updates of U_MU and then of U_NU on the sites of parity p, (MU, NU) = (0, 1)
// or (2, 3) (Sec. 2.4: within a parity the directions are updated in turn).
//
// Why this is exact and needs no grid-wide ordering.  The update of U_NU(x)
// reads the freshly updated U_MU only at x and at y = x - MU + NU (both of
// parity p: the forward and backward staples of the plane (NU, MU), Eq. (6));
// every other link it reads is left alone by both passes.  The update of
// U_MU(x') reads U_NU of parity p only at x' and x' + MU - NU.  So if each
// workgroup takes a set T of parity-p sites that the shift x -> x - MU + NU
// maps onto itself, a workgroup reads U_MU and U_NU of parity p only inside
// its own T, and other workgroups write only outside it: the workgroup can
// run the U_MU updates of T, keep their results in LDS, and run the U_NU
// updates of T from them, while other workgroups do the same elsewhere.  Every
// update sees exactly the links it sees in the two separate passes, with the
// same Philox counter, so the links come out bit for bit the same.
//
//   (0, 1): T = the parity-p sites of one (x0, x1) plane (fixed x2, x3);
//           position pos = x1 * H0 + x0 / 2, a contiguous range of half indices.
//   (2, 3): T = the parity-p sites with fixed x1 and (x2, x3) on one orbit of
//           the step (-1, +1): points t = 0 .. lcm(L2, L3) - 1 at
//           (x2, x3) = (-t mod L2, (o + t) mod L3), o < gcd(L2, L3); position
//           pos = t * H0 + x0 / 2, whole x0 rows of 16-byte links.  Set j is
//           (x1, o) = (j / gcd, j mod gcd): the sets of one XCD's chunk take
//           every orbit of a few x1 rows, so the x2 and x3 neighbours of a set
//           (the next orbits) are mostly that XCD's own.
//
// A set of at most 1024 sites gets one lane per site (k_pair_small): every
// U_MU update, one barrier, every U_NU update, the first pass's results in
// LDS.  Larger sets go block by block with 256 lanes (k_pair), the second pass
// trailing the first by `lag` positions (the largest forward distance from x
// to y in position order), so both read nearly the same links at nearly the
// same time; LDS then keeps the first pass's results for the current and the
// previous block of positions, and for block 0 (the y of the last positions
// wrap around to it).
#pragma once

#include "su2_pass.hpp"

namespace su2 {

struct PairGeo {
    uint32_t n_t = 0;         // sites (positions) per workgroup
    uint32_t n_wg = 0;        // workgroups
    uint32_t lag = 0;         // positions by which the NU pass trails the MU pass
    uint32_t nblk = 0;        // blocks of kBlock positions of the MU pass
    uint32_t orbit = 0;       // (2, 3): orbit length lcm(L2, L3)
    uint32_t xcd_chunk = 0;   // != 0: workgroup w takes T number (w % 8) * xcd_chunk + w / 8
    uint32_t counter_slots = 0;
    FastDiv dL3;
    FastDiv dGC;              // (2, 3): gcd(L2, L3), the orbits per x1
};

// Half index and site of position pos of the set T number j.
template <uint32_t MU>
__device__ __forceinline__ uint32_t pair_site(const Geo &g, const PairGeo &pg, uint32_t j,
                                              uint32_t p, uint32_t pos, Site &x)
{
    if constexpr (MU == 0u) {
        const uint32_t h = j * (g.H0 * g.L[1]) + pos;
        x = site_of(g, h, p);
        return h;
    } else {
        const uint32_t x1 = fdiv(j, pg.dGC);
        const uint32_t o = j - x1 * (pg.n_wg / g.L[1]);
        const uint32_t t = fdiv(pos, g.dH0);
        const uint32_t h0 = pos - t * g.H0;
        const uint32_t t2 = t - fdiv(t, g.dL2) * g.L[2];
        const uint32_t ot = o + t;
        x.x[1] = x1;
        x.x[2] = t2 == 0u ? 0u : g.L[2] - t2;
        x.x[3] = ot - fdiv(ot, pg.dL3) * g.L[3];
        x.x[0] = 2u * h0 + ((p + x1 + x.x[2] + x.x[3]) & 1u);
        return h0 + x1 * g.st[1] + x.x[2] * g.st[2] + x.x[3] * g.st[3];
    }
}

// Position of y = x - MU + NU for the site x at position pos (half index h).
template <uint32_t MU>
__device__ __forceinline__ uint32_t pair_shift(const Geo &g, const PairGeo &pg, uint32_t j,
                                               uint32_t pos, uint32_t h, const Site &x)
{
    if constexpr (MU == 0u) {
        return h_minus<0>(g, h_plus<1>(g, h, x.x[1]), x.x[0]) - j * (g.H0 * g.L[1]);
    } else {
        const uint32_t t = fdiv(pos, g.dH0);
        return t + 1u == pg.orbit ? pos - t * g.H0 : pos + g.H0;
    }
}

// The staple links of U_NU(x) in the plane (NU, MU) whose U_MU(x) (a) and
// U_MU(x + NU - MU) (f) come from the first pass; the other four from memory.
template <uint32_t NU, uint32_t MU, bool OFF32>
__device__ __forceinline__ StapleLinks gather_fresh(const float4 *L, const Geo &g, uint32_t p,
                                                    uint32_t h, uint32_t h_pn, const Site &x,
                                                    float4 a, float4 f)
{
    const uint32_t q = p ^ 1u;
    const uint32_t h_pm = h_plus<MU>(g, h, x.x[MU]);
    const uint32_t h_mm = h_minus<MU>(g, h, x.x[MU]);
    const float4 *Lmq = L + arr(g, MU, q), *Lnq = L + arr(g, NU, q);
    StapleLinks s;
    s.a = a;                          // U_MU(x)
    s.b = ld4<OFF32>(Lnq, h_pm);      // U_NU(x+MU)
    s.c = ld4<OFF32>(Lmq, h_pn);      // U_MU(x+NU)
    s.d = ld4<OFF32>(Lmq, h_mm);      // U_MU(x-MU)
    s.e = ld4<OFF32>(Lnq, h_mm);      // U_NU(x-MU)
    s.f = f;                          // U_MU(x+NU-MU)
    return s;
}

// Arguments every pair kernel passes to the per-site updates.
struct PairCtx {
    float4 *L;
    Geo g;
    PairGeo pg;
    Key key;
    float beta;
    uint32_t p, s, j, slot;
    unsigned long long *counters;
    ImhTable imh;
};

// Links the U_MU update at x loads that the U_NU update at the same x reads
// again (one lane per site): U_rho(x) and U_rho(x - rho) for the two other
// directions rho, U_NU(x + MU), U_MU(x + NU), and U_NU(x) (not yet updated).
struct PairCarry {
    float4 ra[2], rd[2];
    float4 nu_pm, mu_pn, nu_old;
};

// slot of the direction RHO (not MU, NU) in PairCarry: the smaller one first
template <uint32_t MU, uint32_t NU, uint32_t RHO>
constexpr int rho_slot()
{
    return RHO == (MU == 0u ? 2u : 0u) ? 0 : 1;
}

template <uint32_t MU, uint32_t NU, uint32_t NUI>
__device__ __forceinline__ void carry_plane(const StapleLinks &sl, PairCarry &cr)
{
    if constexpr (NUI == NU) {
        cr.nu_old = sl.a;
        cr.mu_pn = sl.b;
        cr.nu_pm = sl.c;
    } else {
        cr.ra[rho_slot<MU, NU, NUI>()] = sl.a;
        cr.rd[rho_slot<MU, NU, NUI>()] = sl.d;
    }
}

template <uint32_t MU, uint32_t NU>
__device__ __forceinline__ void carry_of(const TileLoad &ld, PairCarry &cr)
{
    carry_plane<MU, NU, other_dir<MU, 0>()>(ld.s0, cr);
    carry_plane<MU, NU, other_dir<MU, 1>()>(ld.s1, cr);
    carry_plane<MU, NU, other_dir<MU, 2>()>(ld.s2, cr);
}

// The U_MU update at position pos (lanes with !valid join the wave-wide steps);
// returns the new link and adds the plaquette terms it measures to acc_s.
// before_update(), called by every lane once the staples are formed from the
// update's loads (so the loaded links no longer hold registers), may wait at
// a barrier for the knot table, whose copy the caller issued first.
template <uint32_t MU, bool OFF32, bool MEAS, bool IMH, bool CARRY, bool CREUTZ, typename Hook>
__device__ __forceinline__ float4 pair_update1(const PairCtx &c, uint32_t pos, bool valid, double &acc_s,
                                               Hook before_update, PairCarry &carry)
{
    constexpr uint32_t NU = MU + 1u;
    Site x;
    const uint32_t h = pair_site<MU>(c.g, c.pg, c.j, c.p, valid ? pos : 0u, x);
    const TileLoad ld = load_site<MU, OFF32, IMH>(c.L, c.g, c.p, h, x);
    if constexpr (CARRY) carry_of<MU, NU>(ld, carry);
    const TileStaples in = staples_of(ld);
    before_update();
    double m = 0.0;
    const float4 un = update_link<MU, OFF32, MEAS, IMH, true, CREUTZ>(c.L, c.g, c.key, c.beta, c.p, c.s, h, valid,
                                                              c.slot, in, c.counters, c.imh, m);
    acc_s += m;  // MU = 2: spatial planes (0, 2), (1, 2)
    return un;
}

// The staple links of U_NU(x) in the plane (NU, RHO) when U_RHO(x) (a) and
// U_RHO(x - RHO) (d) are at hand; the other four from memory.
template <uint32_t NU, uint32_t RHO, bool OFF32>
__device__ __forceinline__ StapleLinks gather_carried(const float4 *L, const Geo &g, uint32_t p,
                                                      uint32_t h, uint32_t h_pn, const Site &x,
                                                      float4 a, float4 d)
{
    const uint32_t q = p ^ 1u;
    const uint32_t h_pr = h_plus<RHO>(g, h, x.x[RHO]);
    const uint32_t h_mr = h_minus<RHO>(g, h, x.x[RHO]);
    const uint32_t h_pn_mr = h_minus<RHO>(g, h_pn, x.x[RHO]);  // x+NU has the same x_RHO
    const float4 *Lrp = L + arr(g, RHO, p), *Lrq = L + arr(g, RHO, q), *Lnq = L + arr(g, NU, q);
    StapleLinks s;
    s.a = a;                             // U_RHO(x)
    s.b = ld4<OFF32>(Lnq, h_pr);         // U_NU(x+RHO)
    s.c = ld4<OFF32>(Lrq, h_pn);         // U_RHO(x+NU)
    s.d = d;                             // U_RHO(x-RHO)
    s.e = ld4<OFF32>(Lnq, h_mr);         // U_NU(x-RHO)
    s.f = ld4<OFF32>(Lrp, h_pn_mr);      // U_RHO(x+NU-RHO)
    return s;
}

// The staple links of U_NU(x) in the plane (NU, RHO) with the carried links
// in place of loads (RHO = MU: the plane of the fresh U_MU).
template <uint32_t MU, uint32_t NU, uint32_t RHO, bool OFF32>
__device__ __forceinline__ StapleLinks plane_carried(const PairCtx &c, uint32_t h, uint32_t h_pn,
                                                     const Site &x, float4 a, float4 f,
                                                     const PairCarry &cr)
{
    if constexpr (RHO == MU) {
        // as gather_fresh, with U_NU(x+MU) and U_MU(x+NU) carried
        const uint32_t h_mm = h_minus<MU>(c.g, h, x.x[MU]);
        const uint32_t q = c.p ^ 1u;
        StapleLinks sl;
        sl.a = a;                                          // U_MU(x)
        sl.b = cr.nu_pm;                                   // U_NU(x+MU)
        sl.c = cr.mu_pn;                                   // U_MU(x+NU)
        sl.d = ld4<OFF32>(c.L + arr(c.g, MU, q), h_mm);    // U_MU(x-MU)
        sl.e = ld4<OFF32>(c.L + arr(c.g, NU, q), h_mm);    // U_NU(x-MU)
        sl.f = f;                                          // U_MU(x+NU-MU)
        return sl;
    } else {
        return gather_carried<NU, RHO, OFF32>(c.L, c.g, c.p, h, h_pn, x, cr.ra[rho_slot<MU, NU, RHO>()],
                                              cr.rd[rho_slot<MU, NU, RHO>()]);
    }
}

// The U_NU update at position pos; fresh(q) is the new U_MU at position q;
// carry (one lane per site) holds the links the U_MU update at pos loaded
// that this one reads again.
template <uint32_t MU, uint32_t NU, bool OFF32, bool MEAS, bool IMH, bool CARRY, bool CREUTZ, typename Fresh>
__device__ __forceinline__ void pair_update2(const PairCtx &c, uint32_t pos, bool valid, Fresh fresh,
                                             double &acc_s, double &acc_t, const PairCarry &carry)
{
    const Geo &g = c.g;
    Site x;
    const uint32_t h = pair_site<MU>(g, c.pg, c.j, c.p, pos, x);
    const uint32_t posy = pair_shift<MU>(g, c.pg, c.j, pos, h, x);
    const float4 a = fresh(pos), f = fresh(posy);
    constexpr uint32_t N0 = other_dir<NU, 0>(), N1 = other_dir<NU, 1>(), N2 = other_dir<NU, 2>();
    const uint32_t h_pn = h_plus<NU>(g, h, x.x[NU]);
    TileLoad t;
    t.lex = 2u * h + (x.x[0] & 1u);
    if constexpr (CARRY) {
        t.s0 = plane_carried<MU, NU, N0, OFF32>(c, h, h_pn, x, a, f, carry);
        t.s1 = plane_carried<MU, NU, N1, OFF32>(c, h, h_pn, x, a, f, carry);
        t.s2 = plane_carried<MU, NU, N2, OFF32>(c, h, h_pn, x, a, f, carry);
        t.uold = IMH ? carry.nu_old : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        if constexpr (N0 == MU) t.s0 = gather_fresh<NU, MU, OFF32>(c.L, g, c.p, h, h_pn, x, a, f);
        else t.s0 = gather<NU, N0, OFF32>(c.L, g, c.p, h, h_pn, x);
        if constexpr (N1 == MU) t.s1 = gather_fresh<NU, MU, OFF32>(c.L, g, c.p, h, h_pn, x, a, f);
        else t.s1 = gather<NU, N1, OFF32>(c.L, g, c.p, h, h_pn, x);
        if constexpr (N2 == MU) t.s2 = gather_fresh<NU, MU, OFF32>(c.L, g, c.p, h, h_pn, x, a, f);
        else t.s2 = gather<NU, N2, OFF32>(c.L, g, c.p, h, h_pn, x);
        t.uold = IMH ? ld4<OFF32>(c.L + arr(g, NU, c.p), h) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    double m = 0.0;
    update_link<NU, OFF32, MEAS, IMH, false, CREUTZ>(c.L, g, c.key, c.beta, c.p, c.s, h, valid, c.slot,
                                             staples_of(t), c.counters, c.imh, m);
    if (NU == 3u) acc_t += m; else acc_s += m;
}

// FP64 sum of two values over a workgroup of any multiple of 64 threads (at
// most 1024): wave butterflies, then the waves in order.
__device__ __forceinline__ double2 block_sum2_any(double a, double b)
{
    __shared__ double sh[2][16];
    a = wave_sum(a);
    b = wave_sum(b);
    const uint32_t wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
    }
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
        for (uint32_t i = 0; i < nw; ++i) {
            r.x += sh[0][i];
            r.y += sh[1][i];
        }
    }
    return r;
}

// The learned proposal's knot table copied into LDS by a workgroup of any
// multiple of 64 threads: the same kImhLdsVec4 float4 as stage_table, wave v
// copying the 64-float4 chunks v, v + waves, ...
__device__ __forceinline__ void stage_table_any(const ImhTable &imh)
{
    extern __shared__ float4 imh_lds[];
    const uint32_t wv = threadIdx.x / kWave, nw = blockDim.x / kWave, lane = threadIdx.x % kWave;
    for (uint32_t c = wv; c < kImhLdsVec4 / kWave; c += nw)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(reinterpret_cast<const float4 *>(imh.knots) +
                                                             c * kWave + lane),
            (__attribute__((address_space(3))) void *)(imh_lds + c * kWave), 16u, 0, 0);
}

// Sets of at most kPairLanes sites: one lane per site (the launch has
// n_t rounded up to a multiple of 64 threads), so each pass is one phase --
// every U_MU update, one barrier, every U_NU update.
constexpr uint32_t kPairLanes = 1024;

template <uint32_t MU, uint32_t NU, bool OFF32, bool MEAS1, bool MEAS2, bool IMH, bool CREUTZ>
__global__ __launch_bounds__(kPairLanes) void k_pair_small(
    float4 *__restrict__ L, Geo g, PairGeo pg, Key key, float beta, uint32_t p,
    const uint32_t *__restrict__ sweep_ptr, unsigned long long *__restrict__ counters,
    double2 *__restrict__ meas_out, ImhTable imh)
{
    static_assert((MU == 0u && NU == 1u) || (MU == 2u && NU == 3u), "pairs (0,1) and (2,3)");
    __shared__ float4 buf[kPairLanes];  // the new U_MU of the set
    const uint32_t w = blockIdx.x;
    const PairCtx c{ L, g, pg, key, beta, p, *sweep_ptr,
                     pg.xcd_chunk ? (w % 8u) * pg.xcd_chunk + w / 8u : w,
                     (w * (blockDim.x / kWave) + threadIdx.x / kWave) % pg.counter_slots, counters, imh };
    double acc_s = 0.0, acc_t = 0.0;
    const uint32_t pos = threadIdx.x;
    const bool valid = pos < pg.n_t;
    // the knot table's copy goes out ahead of the first pass's loads and is
    // waited for once their staples are formed; the links both updates of a
    // site read stay in registers
    if constexpr (IMH) stage_table_any(imh);
    PairCarry carry;
    const float4 un = pair_update1<MU, OFF32, MEAS1, IMH, true, CREUTZ>(c, pos, valid, acc_s, [&] {
        if constexpr (IMH) __syncthreads();
    }, carry);
    if (valid) buf[pos] = un;
    __syncthreads();
    pair_update2<MU, NU, OFF32, MEAS2, IMH, true, CREUTZ>(c, valid ? pos : 0u, valid,
                                                          [&](uint32_t q) { return buf[q]; }, acc_s, acc_t, carry);
    if constexpr (MEAS1 || MEAS2) {
        const double2 r = block_sum2_any(acc_s, acc_t);
        if (threadIdx.x == 0) meas_out[w] = r;
    }
}

// Larger sets, block by block with 256 threads: the U_NU updates trail the
// U_MU updates by `lag` positions.
template <uint32_t MU, uint32_t NU, bool OFF32, bool MEAS1, bool MEAS2, bool IMH, bool CREUTZ>
__global__ __launch_bounds__(kBlock) void k_pair(
    float4 *__restrict__ L, Geo g, PairGeo pg, Key key, float beta, uint32_t p,
    const uint32_t *__restrict__ sweep_ptr, unsigned long long *__restrict__ counters,
    double2 *__restrict__ meas_out, ImhTable imh)
{
    static_assert((MU == 0u && NU == 1u) || (MU == 2u && NU == 3u), "pairs (0,1) and (2,3)");
    // MU-pass results: blocks b - 1 and b in buf[0 .. 2 kBlock), block 0 in
    // buf[2 kBlock .. 3 kBlock)
    __shared__ float4 buf[3 * kBlock];
    const uint32_t w = blockIdx.x;
    const PairCtx c{ L, g, pg, key, beta, p, *sweep_ptr,
                     pg.xcd_chunk ? (w % 8u) * pg.xcd_chunk + w / 8u : w,
                     (w * (kBlock / kWave) + threadIdx.x / kWave) % pg.counter_slots, counters, imh };
    double acc_s = 0.0, acc_t = 0.0;
    PairCarry unused;  // (the two passes of a site run on different lanes here)
    for (uint32_t b = 0; b <= pg.nblk; ++b) {
        // the MU pass on positions [b * kBlock, (b + 1) * kBlock)
        if (b < pg.nblk) {
            const uint32_t pos = b * kBlock + threadIdx.x;
            // block 0: the knot table's copy goes out ahead of its loads and is
            // waited for once their staples are formed
            if constexpr (IMH) {
                if (b == 0u) stage_table(imh);
            }
            const float4 un = pair_update1<MU, OFF32, MEAS1, IMH, false, CREUTZ>(c, pos, pos < pg.n_t, acc_s, [&] {
                if constexpr (IMH) {
                    if (b == 0u) __syncthreads();
                }
            }, unused);
            buf[(b & 1u) * kBlock + threadIdx.x] = un;
            if (b == 0u) buf[2u * kBlock + threadIdx.x] = un;
        }
        __syncthreads();
        // the NU pass on positions [b * kBlock - lag, (b + 1) * kBlock - lag)
        const int ipos = (int)(b * kBlock + threadIdx.x) - (int)pg.lag;
        const bool valid = ipos >= 0 && (uint32_t)ipos < pg.n_t;
        pair_update2<MU, NU, OFF32, MEAS2, IMH, false, CREUTZ>(c, valid ? (uint32_t)ipos : 0u, valid, [&](uint32_t q) {
            const uint32_t blk = q / kBlock;
            return buf[(blk == b || blk + 1u == b) ? (blk & 1u) * kBlock + q % kBlock
                                                   : 2u * kBlock + q % kBlock];
        }, acc_s, acc_t, unused);
        __syncthreads();  // before the next block's MU results replace block b - 1
    }
    if constexpr (MEAS1 || MEAS2) {
        const double2 r = block_sum2(acc_s, acc_t);
        if (threadIdx.x == 0) meas_out[w] = r;
    }
}

}  // namespace su2
