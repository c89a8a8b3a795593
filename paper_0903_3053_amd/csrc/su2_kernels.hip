// su2_kernels.hip -- gfx950 kernels of the SU(2) heat-bath sweep.
//
//   k_init       cold / hot lattice (Sec. 2.1: initialisation on the GPU)
//   k_pass       one (parity, mu) pass: staple, Kennedy-Pendleton x0, direction,
//                rotation, FP64-normed reunitarisation, store (Eqs. (5)-(7)).
//                The paper's separate staple and update kernels and its staple
//                buffer (Sec. 2.4) are fused: the staple stays in registers.
//   k_pair       the passes of U_0 and U_1 (or U_2 and U_3) of one parity in
//                one launch (su2_pair.hpp)
//   k_or         one overrelaxation pass (U -> V U^dag V about the staple)
//   k_tick       advances the device-resident sweep index words (graph-friendly)
//   k_plaquette  per-workgroup FP64 partial sums of spatial / temporal
//                plaquettes (Sec. 2.4, Eq. (3))
//   k_polyakov   per-workgroup FP64 partial sums of the Polyakov loop
//   k_reduce     fixed-order FP64 reduction of the partials (deterministic)
//   k_pack / k_unpack   device checkerboard layout <-> host [V][4][4]
//   k_philox     raw generator blocks, for bit-exact checks
#include <algorithm>
#include <numeric>

#include "su2_kernels.hpp"
#include "su2_pass.hpp"

namespace su2 {


// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init(float4 *__restrict__ links, Geo g, Key key,
                                                 int hot)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;  // half-site index
    const uint32_t mu = blockIdx.y >> 1, p = blockIdx.y & 1u;  // one (mu, p) array per grid row
    if (i >= g.half) return;
    float4 q = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
    if (hot) {
        const Site s = site_of(g, i, p);
        q = haar(draw(key, lex_of(g, s), mu, kPurposeHot, 0u, 0u));
    }
    links[arr(g, mu, p) + i] = q;
}

// One heat-bath pass over U_MU(x), parity(x) = p; each workgroup runs one tile.
// A table can reorder tiles so that the workgroups the hardware sends to one
// XCD share their neighbour data in L2.  CREUTZ: the heat-bath with the
// small-alpha switch (its own kernels, so the plain ones stay as they are).
template <uint32_t MU, bool OFF32, bool MEASURE, bool IMH, bool CREUTZ>
__global__ __launch_bounds__(kBlock) void k_pass(
    float4 *__restrict__ L, Geo g, Key key, float beta, uint32_t p,
    const uint32_t *__restrict__ sweep_ptr, unsigned long long *__restrict__ counters,
    double2 *__restrict__ meas_out, const uint32_t *__restrict__ order,
    ImhTable imh)
{
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    pass_tile<MU, OFF32, MEASURE, IMH, CREUTZ>(L, g, key, beta, p, *sweep_ptr, tile, counters, meas_out,
                                               imh);
}

// One overrelaxation pass over U_MU(x), parity(x) = p: U -> V U^dag V with
// V = w/|w| (w the Eq. (6) staple sum), the standard SU(2) reflection that
// keeps the local weight exp(beta dot(U, w)) and needs no random number;
// links with w = 0 are kept.  The pass reads the old link (144 B per update).
template <uint32_t MU, bool OFF32>
__global__ __launch_bounds__(kBlock) void k_or(float4 *__restrict__ L, Geo g, uint32_t p,
                                               const uint32_t *__restrict__ order)
{
#pragma clang fp contract(off)
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const TileStaples t = staples_of(load_tile<MU, OFF32, true>(L, g, p, tile));
    const uint32_t h = tile * kBlock + threadIdx.x;
    if (h >= g.half) return;
    const float k = sqrtf(qdot(t.w, t.w));
    if (k == 0.0f) return;
    const float ik = __builtin_amdgcn_rcpf(k);
    const float4 V = make_float4(t.w.x * ik, t.w.y * ik, t.w.z * ik, t.w.w * ik);
    st4_stream<OFF32>(L + arr(g, MU, p), h, unitize(qmul(qmul(V, qdag(t.uold)), V)));
}

// The sweep index lives in kSweepSlots consecutive words, word j holding
// index + j, so that sweep j of a graph of several sweeps reads word j and a
// single tick per graph advances all of them by the graph's sweeps.
__global__ void k_tick(uint32_t *sweep_ptr, uint32_t n)
{
    if (threadIdx.x < kSweepSlots) sweep_ptr[threadIdx.x] += n;
}

// ---------------------------------------------------------------------------
// One site per lane (index over both parities); the six plaquettes whose
// corner is x, split spatial (nu < 3) / temporal (nu == 3).
__global__ __launch_bounds__(kBlock) void k_plaquette(const float4 *__restrict__ L, Geo g,
                                                      double2 *__restrict__ partials)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    double ps = 0.0, pt = 0.0;
    if (i < 2u * g.half) {
        const uint32_t p = i >= g.half ? 1u : 0u;
        const uint32_t h = i - p * g.half;
        const uint32_t q = p ^ 1u;
        const Site x = site_of(g, h, p);
        const uint32_t hn[4] = { h_plus<0>(g, h, x.x[0]), h_plus<1>(g, h, x.x[1]),
                                 h_plus<2>(g, h, x.x[2]), h_plus<3>(g, h, x.x[3]) };
        float4 u[4], nb[4][4];
#pragma unroll
        for (uint32_t mu = 0; mu < 4; ++mu) u[mu] = L[arr(g, mu, p) + h];
#pragma unroll
        for (uint32_t mu = 0; mu < 4; ++mu)
#pragma unroll
            for (uint32_t nu = 0; nu < 4; ++nu)
                if (nu != mu) nb[mu][nu] = L[arr(g, nu, q) + hn[mu]];  // U_nu(x + mu)
#pragma unroll
        for (uint32_t mu = 0; mu < 4; ++mu) {
#pragma unroll
            for (uint32_t nu = mu + 1; nu < 4; ++nu) {
                // U_mu(x) U_nu(x+mu) . [U_nu(x) U_mu(x+nu)]^dag
                const float4 a = qmul(u[mu], nb[mu][nu]);
                const float4 b = qmul(u[nu], nb[nu][mu]);
                const double v = (double)qdot(a, b);
                if (nu == 3) pt += v; else ps += v;
            }
        }
    }
    const double2 r = block_sum2(ps, pt);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// One spatial site per lane: ordered product of U_3(x, t), t = 0..L3-1.
__global__ __launch_bounds__(kBlock) void k_polyakov(const float4 *__restrict__ L, Geo g,
                                                     uint32_t vs, double2 *__restrict__ partials)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    if (i < vs) {
        const uint32_t x0 = i % g.L[0];
        const uint32_t r = i / g.L[0];
        const uint32_t x1 = r % g.L[1];
        const uint32_t x2 = r / g.L[1];
        float4 P = make_float4(1.f, 0.f, 0.f, 0.f);
        for (uint32_t t = 0; t < g.L[3]; ++t) {
            const uint32_t p = (x0 + x1 + x2 + t) & 1u;
            const uint32_t h = (x0 >> 1) + x1 * g.st[1] + x2 * g.st[2] + t * g.st[3];
            P = qmul(P, L[arr(g, 3, p) + h]);
        }
        acc = (double)P.x;
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(r, 0.0);
}

// First level of the deterministic reduction: workgroup b sums the partials
// [b*chunk, (b+1)*chunk) -- thread j takes j, j+256, ... in order, then the
// fixed block tree.
__global__ __launch_bounds__(kBlock) void k_reduce_chunks(const double2 *__restrict__ in,
                                                          uint32_t n, uint32_t chunk,
                                                          double2 *__restrict__ out)
{
    const uint32_t lo = blockIdx.x * chunk;
    const uint32_t hi = min(n, lo + chunk);
    double a = 0.0, b = 0.0;
    for (uint32_t j = lo + threadIdx.x; j < hi; j += kBlock) {
        a += in[j].x;
        b += in[j].y;
    }
    const double2 r = block_sum2(a, b);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// Final level, one workgroup: thread j sums j, j+256, ... in order, then a
// fixed tree.  Mode 0 (plaquette): out[0] = (a*sa + b*sb)/2, out[1] = a*sa,
// out[2] = b*sb.  Mode 1 (single value): out[0] = a*sa.  With a cursor the
// results go to entry *cursor of a history (out + 3 * *cursor in mode 0) and
// the cursor advances by one, so a graph of measured sweeps fills a history
// in place.
__global__ __launch_bounds__(kBlock) void k_reduce(const double2 *__restrict__ partials,
                                                   uint32_t n, double sa, double sb, int mode,
                                                   double *__restrict__ out,
                                                   uint32_t *__restrict__ cursor)
{
    __shared__ double sh[2][kBlock];
    double a = 0.0, b = 0.0;
    for (uint32_t j = threadIdx.x; j < n; j += kBlock) {
        a += partials[j].x;
        b += partials[j].y;
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (cursor) {
            out += (size_t)(mode == 0 ? 3u : 1u) * *cursor;
            *cursor += 1u;
        }
        const double A = sh[0][0] * sa, B = sh[1][0] * sb;
        if (mode == 0) {
            out[0] = 0.5 * (A + B);
            out[1] = A;
            out[2] = B;
        } else {
            out[0] = A;
        }
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pack(const float4 *__restrict__ L, Geo g,
                                                 float4 *__restrict__ host_layout)
{
    const uint32_t lex = blockIdx.x * kBlock + threadIdx.x;
    if (lex >= 2u * g.half) return;
    Site s;
    uint32_t r = lex;
    s.x[0] = r % g.L[0]; r /= g.L[0];
    s.x[1] = r % g.L[1]; r /= g.L[1];
    s.x[2] = r % g.L[2];
    s.x[3] = r / g.L[2];
    const uint32_t p = (s.x[0] + s.x[1] + s.x[2] + s.x[3]) & 1u;
    const uint32_t h = half_of(g, s);
#pragma unroll
    for (uint32_t mu = 0; mu < 4; ++mu) host_layout[(size_t)lex * 4 + mu] = L[arr(g, mu, p) + h];
}

__global__ __launch_bounds__(kBlock) void k_unpack(float4 *__restrict__ L, Geo g,
                                                   const float4 *__restrict__ host_layout)
{
    const uint32_t lex = blockIdx.x * kBlock + threadIdx.x;
    if (lex >= 2u * g.half) return;
    Site s;
    uint32_t r = lex;
    s.x[0] = r % g.L[0]; r /= g.L[0];
    s.x[1] = r % g.L[1]; r /= g.L[1];
    s.x[2] = r % g.L[2];
    s.x[3] = r / g.L[2];
    const uint32_t p = (s.x[0] + s.x[1] + s.x[2] + s.x[3]) & 1u;
    const uint32_t h = half_of(g, s);
#pragma unroll
    for (uint32_t mu = 0; mu < 4; ++mu) L[arr(g, mu, p) + h] = host_layout[(size_t)lex * 4 + mu];
}

__global__ __launch_bounds__(kBlock) void k_philox(const uint4 *__restrict__ ctr, uint32_t n,
                                                   Key key, uint4 *__restrict__ out)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = philox(ctr[i], key);
}

// ---------------------------------------------------------------------------
// Launchers (host side)
// ---------------------------------------------------------------------------
static inline uint32_t blocks_for(size_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

hipError_t launch_init(float4 *links, const Geo &g, Key key, int hot, hipStream_t st)
{
    dim3 grid(blocks_for(g.half), 8);
    hipLaunchKernelGGL(k_init, grid, dim3(kBlock), 0, st, links, g, key, hot);
    return hipGetLastError();
}

bool use_off32(const Geo &g) { return (uint64_t)g.half * 16u <= 0xffffffffull; }

template <uint32_t MU, bool MEASURE, bool IMH, bool CREUTZ>
static const void *pass_func_4(bool off32)
{
    return off32 ? reinterpret_cast<const void *>(&k_pass<MU, true, MEASURE, IMH, CREUTZ>)
                 : reinterpret_cast<const void *>(&k_pass<MU, false, MEASURE, IMH, CREUTZ>);
}

// the learned proposal runs with the Creutz switch off
template <uint32_t MU>
static const void *pass_func_mu(bool off32, bool measure, bool imh, bool creutz)
{
    if (imh)
        return measure ? pass_func_4<MU, true, true, false>(off32) : pass_func_4<MU, false, true, false>(off32);
    if (creutz)
        return measure ? pass_func_4<MU, true, false, true>(off32) : pass_func_4<MU, false, false, true>(off32);
    return measure ? pass_func_4<MU, true, false, false>(off32) : pass_func_4<MU, false, false, false>(off32);
}

const void *pass_func(uint32_t mu, bool off32, bool measure, bool imh, bool creutz)
{
    switch (mu) {
    case 0: return pass_func_mu<0>(off32, false, imh, creutz);  // no plaquette plane has nu < 0
    case 1: return pass_func_mu<1>(off32, measure, imh, creutz);
    case 2: return pass_func_mu<2>(off32, measure, imh, creutz);
    default: return pass_func_mu<3>(off32, measure, imh, creutz);
    }
}

uint32_t pass_blocks(const Geo &g) { return blocks_for(g.half); }

// Tile orders (workgroup w runs tile order[w]; the hardware deals workgroups
// to the 8 XCDs round-robin, w mod 8).  kind 0: identity.  kind T (1..99):
// when a (x2, x3) plane holds a multiple of 8 tiles, XCD k takes the k-th
// eighth of every plane (a band of x1 rows) and walks the planes in T x T
// squares of (x2, x3), so that the planes whose rows a tile's staples read
// were fetched into the same L2 shortly before.  kind 100 + T: the same with
// squares and the planes inside them walked back and forth (consecutive
// squares share an edge).  kind 200 + T: four XCDs share each plane (bands
// twice as thick, so fewer rows are fetched by two XCDs), XCDs 0-3 taking the
// planes with x2 < L2/2 and XCDs 4-7 the rest, walked as kind 100 + T.
// Returns false if the geometry does not fit the scheme (the identity is then
// used).
bool make_order(const Geo &g, int kind, std::vector<uint32_t> &order)
{
    const uint32_t n = pass_blocks(g);
    if (kind >= kAlternate) {
        // order kind - kAlternate, then the same backwards for the odd passes
        if (kind - kAlternate >= kAlternate || !make_order(g, kind - kAlternate, order)) return false;
        order.resize(2u * (size_t)n);
        for (uint32_t w = 0; w < n; ++w) order[n + w] = order[n - 1u - w];
        return true;
    }
    order.resize(n);
    for (uint32_t w = 0; w < n; ++w) order[w] = w;
    if (kind <= 0) return true;
    const uint32_t T = (uint32_t)(kind % 100), variant = (uint32_t)(kind / 100);
    if (T == 0 || variant > 2) return false;
    const bool serp = variant >= 1;
    const uint32_t share = variant == 2 ? 4u : 8u;  // XCDs per plane
    const uint32_t groups2 = 8u / share;            // plane groups along x2
    const uint64_t per_plane = (uint64_t)g.H0 * g.L[1];
    if (per_plane % ((uint64_t)share * kBlock) || n % 8u) return false;
    const uint32_t P2 = g.L[2] / groups2;  // planes per group along x2
    if (g.L[2] % groups2 || P2 % T || g.L[3] % T) return false;
    const uint32_t bpp = (uint32_t)(per_plane / kBlock);  // tiles per plane
    const uint32_t band = bpp / share;                    // tiles per plane per XCD
    const uint32_t nt2 = P2 / T;
    for (uint32_t w = 0; w < n; ++w) {
        const uint32_t k = w % 8u, j = w / 8u;
        const uint32_t bi = k % share, gi2 = k / share;
        const uint32_t in_band = j % band, pj = j / band;  // pj-th plane of this XCD
        const uint32_t sq = pj / (T * T), in_sq = pj % (T * T);
        const uint32_t s3 = sq / nt2, i3 = in_sq / T;
        uint32_t s2 = sq % nt2, i2 = in_sq % T;
        if (serp && (s3 & 1u)) s2 = nt2 - 1u - s2;
        if (serp && (i3 & 1u)) i2 = T - 1u - i2;
        const uint32_t x2 = gi2 * P2 + s2 * T + i2;
        const uint32_t x3 = s3 * T + i3;
        order[w] = (x2 + g.L[2] * x3) * bpp + bi * band + in_band;
    }
    return true;
}

PassLaunch pass_launch(float4 *links, const Geo &g, Key key, float beta, uint32_t p, uint32_t mu,
                       const uint32_t *sweep_ptr, unsigned long long *counters,
                       double2 *meas_out, const PassPlan &plan)
{
    PassLaunch pl;
    pl.lds = plan.learned ? std::max(plan.lds_bytes, plan.imh_lds_bytes) : plan.lds_bytes;
    pl.order = plan.order;
    const bool measure = meas_out != nullptr && p == 0u && mu >= 1u;
    pl.func = pass_func(mu, use_off32(g) && !plan.wide, measure, plan.learned,
                        !plan.learned && plan.imh.creutz_below > 0.0f);
    pl.imh = plan.imh;
    pl.grid = dim3(pass_blocks(g));
    pl.block = dim3(kBlock);
    pl.links = links;
    pl.g = g;
    pl.key = key;
    pl.beta = beta;
    pl.p = p;
    pl.sweep_ptr = sweep_ptr;
    pl.counters = counters;
    pl.meas_out = measure ? meas_out + (size_t)(mu - 1u) * pass_blocks(g) : nullptr;
    pl.bind();
    return pl;
}

bool make_pair_geo(const Geo &g, uint32_t counter_slots, PairGeo &pg01, PairGeo &pg23)
{
    if (g.L[0] > (uint32_t)kBlock) return false;  // both lags (2 H0 - 1 and H0) within one block
    const uint32_t gc = std::gcd(g.L[2], g.L[3]);
    pg01 = PairGeo{};
    pg01.n_t = g.H0 * g.L[1];
    pg01.n_wg = g.L[2] * g.L[3];
    pg01.lag = 2u * g.H0 - 1u;
    pg23 = PairGeo{};
    pg23.orbit = g.L[2] / gc * g.L[3];
    pg23.n_t = pg23.orbit * g.H0;
    pg23.n_wg = gc * g.L[1];
    pg23.lag = g.H0;
    for (PairGeo *pg : { &pg01, &pg23 }) {
        pg->nblk = (pg->n_t + kBlock - 1u) / kBlock;
        pg->xcd_chunk = pg->n_wg % 8u == 0u ? pg->n_wg / 8u : 0u;
        pg->counter_slots = counter_slots;
        pg->dL3 = make_fastdiv(g.L[3]);
        pg->dGC = make_fastdiv(gc);
    }
    return true;
}

template <uint32_t MU, uint32_t NU, bool MEAS1, bool MEAS2, bool OFF32, bool IMH, bool CREUTZ>
static const void *pair_func_7(bool small)
{
    return small ? reinterpret_cast<const void *>(&k_pair_small<MU, NU, OFF32, MEAS1, MEAS2, IMH, CREUTZ>)
                 : reinterpret_cast<const void *>(&k_pair<MU, NU, OFF32, MEAS1, MEAS2, IMH, CREUTZ>);
}

// The Creutz draw costs the pair kernels registers (their carried links are
// live across the first update's attempts), so it gets kernels of its own:
// the heat-bath ones without it stay as they are.  The learned proposal runs
// with the switch off.
template <uint32_t MU, uint32_t NU, bool MEAS1, bool MEAS2>
static const void *pair_func_4(bool off32, bool imh, bool creutz, bool small)
{
    if (imh)
        return off32 ? pair_func_7<MU, NU, MEAS1, MEAS2, true, true, false>(small)
                     : pair_func_7<MU, NU, MEAS1, MEAS2, false, true, false>(small);
    if (creutz)
        return off32 ? pair_func_7<MU, NU, MEAS1, MEAS2, true, false, true>(small)
                     : pair_func_7<MU, NU, MEAS1, MEAS2, false, false, true>(small);
    return off32 ? pair_func_7<MU, NU, MEAS1, MEAS2, true, false, false>(small)
                 : pair_func_7<MU, NU, MEAS1, MEAS2, false, false, false>(small);
}

// (0, 1) measures through its U_1 updates; (2, 3) through both passes
static const void *pair_func(uint32_t mu, bool off32, bool measure, bool imh, bool creutz, bool small)
{
    if (mu == 0u)
        return measure ? pair_func_4<0, 1, false, true>(off32, imh, creutz, small)
                       : pair_func_4<0, 1, false, false>(off32, imh, creutz, small);
    return measure ? pair_func_4<2, 3, true, true>(off32, imh, creutz, small)
                   : pair_func_4<2, 3, false, false>(off32, imh, creutz, small);
}

uint32_t meas_partials(const Geo &g, const PassPlan &plan)
{
    return plan.fused ? plan.pg01.n_wg + plan.pg23.n_wg : 3u * pass_blocks(g);
}

std::vector<PassLaunch> sweep_launches(float4 *links, const Geo &g, Key key, float beta,
                                       const uint32_t *sweep_ptr, unsigned long long *counters,
                                       double2 *meas_out, const PassPlan &plan)
{
    std::vector<PassLaunch> out;
    // Sec. 2.4: odd sites for every direction, then even sites
    for (int p = 1; p >= 0; --p) {
        if (!plan.fused) {
            for (uint32_t mu = 0; mu < 4; ++mu) {
                PassLaunch pl = pass_launch(links, g, key, beta, (uint32_t)p, mu, sweep_ptr, counters,
                                            meas_out, plan);
                // odd passes of the sweep walk the tiles backwards: a pass starts
                // where the previous one ended, on data still in the Infinity Cache
                if (plan.alternate && (mu & 1u)) pl.order = plan.order + pass_blocks(g);
                pl.bind();
                out.push_back(pl);
            }
            continue;
        }
        for (uint32_t mu = 0; mu < 4; mu += 2) {
            const PairGeo &pg = mu == 0u ? plan.pg01 : plan.pg23;
            const bool measure = meas_out != nullptr && p == 0;
            PassLaunch pl;
            pl.pair = true;
            pl.pg = pg;
            pl.lds = plan.learned ? std::max(plan.lds_bytes, plan.imh_lds_bytes) : plan.lds_bytes;
            pl.order = nullptr;
            const bool small = pg.n_t <= kPairLanes;
            pl.func = pair_func(mu, use_off32(g) && !plan.wide, measure, plan.learned,
                                !plan.learned && plan.imh.creutz_below > 0.0f, small);
            pl.imh = plan.imh;
            pl.grid = dim3(pg.n_wg);
            pl.block = dim3(small ? (pg.n_t + kWave - 1u) / kWave * kWave : kBlock);
            pl.links = links;
            pl.g = g;
            pl.key = key;
            pl.beta = beta;
            pl.p = (uint32_t)p;
            pl.sweep_ptr = sweep_ptr;
            pl.counters = counters;
            pl.meas_out = measure ? meas_out + (mu == 0u ? 0u : plan.pg01.n_wg) : nullptr;
            pl.bind();
            out.push_back(pl);
        }
    }
    return out;
}

hipError_t launch(PassLaunch &pl, hipStream_t st)
{
    pl.bind();
    return hipLaunchKernel(pl.func, pl.grid, pl.block, pl.args, pl.lds, st);
}

const void *tick_func() { return reinterpret_cast<const void *>(&k_tick); }

template <uint32_t MU>
static const void *or_func_mu(bool off32)
{
    return off32 ? reinterpret_cast<const void *>(&k_or<MU, true>)
                 : reinterpret_cast<const void *>(&k_or<MU, false>);
}

PassLaunch or_launch(float4 *links, const Geo &g, uint32_t p, uint32_t mu, const PassPlan &plan)
{
    PassLaunch pl{};
    const bool off32 = use_off32(g) && !plan.wide;
    pl.func = mu == 0u ? or_func_mu<0>(off32) : mu == 1u ? or_func_mu<1>(off32)
            : mu == 2u ? or_func_mu<2>(off32) : or_func_mu<3>(off32);
    pl.grid = dim3(pass_blocks(g));
    pl.block = dim3(kBlock);
    pl.lds = plan.lds_bytes;
    pl.links = links;
    pl.g = g;
    pl.p = p;
    pl.order = plan.fused ? nullptr : plan.order;
    pl.or_pass = true;
    pl.bind();
    return pl;
}

hipError_t launch_tick(uint32_t *sweep_ptr, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(kWave), 0, st, sweep_ptr, n);
    return hipGetLastError();
}

uint32_t plaquette_blocks(const Geo &g) { return blocks_for(2ull * g.half); }
uint32_t polyakov_blocks(const Geo &g)
{
    return blocks_for((size_t)g.L[0] * g.L[1] * g.L[2]);
}
uint32_t counter_waves(const Geo &g) { return blocks_for(g.half) * (kBlock / kWave); }
uint32_t reduce_scratch() { return kBlock; }

// Deterministic sum of n double2 partials into out (mode as k_reduce): one
// workgroup straight over the partials up to kReduceOneLevel of them, else a
// first level of up to 256 workgroups over fixed chunks and a second over their
// results.
static hipError_t reduce2(const double2 *partials, uint32_t n, double2 *scratch, double sa,
                          double sb, int mode, double *out, hipStream_t st)
{
    uint32_t *no_cursor = nullptr;
    if (n <= kReduceOneLevel) {
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, partials, n, sa, sb, mode, out,
                           no_cursor);
        return hipGetLastError();
    }
    const uint32_t nb1 = std::min<uint32_t>(kBlock, std::max<uint32_t>(1u, (n + 1023u) / 1024u));
    const uint32_t chunk = (n + nb1 - 1) / nb1;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nb1), dim3(kBlock), 0, st, partials, n, chunk,
                       scratch);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, scratch, nb1, sa, sb, mode, out,
                       no_cursor);
    return hipGetLastError();
}

static double plaquette_scale(const Geo &g) { return 1.0 / (3.0 * 2.0 * (double)g.half); }

bool measure_reduce_launch(const double2 *meas_partials, uint32_t n, const Geo &g, double *hist,
                           uint32_t *cursor, ReduceLaunch &rl)
{
    if (n > kReduceOneLevel) return false;
    rl = ReduceLaunch{};
    rl.func = reinterpret_cast<const void *>(&k_reduce);
    rl.partials = meas_partials;
    rl.n = n;
    rl.sa = rl.sb = plaquette_scale(g);
    rl.mode = 0;
    rl.out = hist;
    rl.cursor = cursor;
    rl.bind();
    return true;
}

hipError_t launch_plaquette(const float4 *links, const Geo &g, double2 *partials,
                            double2 *scratch, double *out, hipStream_t st)
{
    const uint32_t nb = plaquette_blocks(g);
    hipLaunchKernelGGL(k_plaquette, dim3(nb), dim3(kBlock), 0, st, links, g, partials);
    return reduce2(partials, nb, scratch, plaquette_scale(g), plaquette_scale(g), 0, out, st);
}

hipError_t launch_measure_reduce(const double2 *meas_partials, uint32_t n, const Geo &g,
                                 double2 *scratch, double *out, hipStream_t st)
{
    // spatial planes from the mu = 1, 2 updates (x), temporal from mu = 3 (y)
    return reduce2(meas_partials, n, scratch, plaquette_scale(g), plaquette_scale(g), 0, out, st);
}

hipError_t launch_polyakov(const float4 *links, const Geo &g, double2 *partials,
                           double2 *scratch, double *out, hipStream_t st)
{
    const uint32_t vs = g.L[0] * g.L[1] * g.L[2];
    const uint32_t nb = polyakov_blocks(g);
    hipLaunchKernelGGL(k_polyakov, dim3(nb), dim3(kBlock), 0, st, links, g, vs, partials);
    return reduce2(partials, nb, scratch, 1.0 / (double)vs, 0.0, 1, out, st);
}

hipError_t launch_pack(const float4 *links, const Geo &g, float4 *stage, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(2ull * g.half)), dim3(kBlock), 0, st, links, g,
                       stage);
    return hipGetLastError();
}

hipError_t launch_unpack(float4 *links, const Geo &g, const float4 *stage, hipStream_t st)
{
    hipLaunchKernelGGL(k_unpack, dim3(blocks_for(2ull * g.half)), dim3(kBlock), 0, st, links, g,
                       stage);
    return hipGetLastError();
}

hipError_t launch_philox(const uint4 *ctr, uint32_t n, Key key, uint4 *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n)), dim3(kBlock), 0, st, ctr, n, key, out);
    return hipGetLastError();
}

}  // namespace su2
