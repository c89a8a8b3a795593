// su2_ising.hip -- the 2-D Ising workload (Sec. 2.3, Eq. (1)): Metropolis on a
// red-black partition of an L0 x L1 periodic lattice, behind include/ising.h.
//
// Two layouts, chosen at init.  Bytes: one int8 array per colour, N/2 bytes
// each, indexed by the half index h = x/2 + (L0/2) y (a row of one colour is
// contiguous); each lane updates four consecutive half-sites from one
// Philox-4x32-10 call (one 32-bit word each).  Bits (L0 a multiple of 64): the
// paper's 1-bit spins (Sec. 2.3), 32 same-colour spins of a row per 32-bit
// word, bit b of word w of a colour holding half index h = 32 w + b (set = spin
// -1); a lane updates a word with bitwise arithmetic -- the four neighbour
// words, the anti-aligned count per bit as bit masks -- and eight Philox calls.
// Both layouts draw the same words for the same sites, so they give the same
// chain bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "ising.h"
#include "su2.h"
#include "su2_device.hpp"

namespace su2 {
namespace {

constexpr int kIsingBlock = 256;
constexpr int kIsingWave = 64;
constexpr uint32_t kPurposeIsing = 4u, kPurposeIsingHot = 5u;
// accepted-flip counters, one per slot of waves: a single counter for every
// wave of a pass serialises in L2 (one address), 4096 spread the adds
constexpr uint32_t kAccSlots = 4096;

struct IsingGeo {
    uint32_t L0, L1, H0, half;  // H0 = L0/2, half = N/2
    uint32_t W, nw;             // bit layout: words per row of one colour (H0/32), words per colour
    FastDiv dH0, dW;
};

// site (x, y) of colour c at half index h
__device__ __forceinline__ void ising_site(const IsingGeo &g, uint32_t c, uint32_t h, uint32_t &x,
                                           uint32_t &y)
{
    y = fdiv(h, g.dH0);
    x = 2u * (h - y * g.H0) + ((c + y) & 1u);
}

__global__ __launch_bounds__(kIsingBlock) void k_ising_init(int8_t *__restrict__ S, IsingGeo g, Key key,
                                                            int hot)
{
    const uint32_t grp = blockIdx.x * kIsingBlock + threadIdx.x;  // four half-sites of colour c
    const uint32_t c = blockIdx.y;
    if (4u * grp >= g.half) return;
    const uint4 r = hot ? philox(make_uint4(grp, c | (kPurposeIsingHot << 8), 0u, 0u), key)
                        : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t w[4] = { r.x, r.y, r.z, r.w };
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) {
        const uint32_t h = 4u * grp + k;
        if (h < g.half) S[(size_t)c * g.half + h] = (w[k] >> 31) ? (int8_t)-1 : (int8_t)1;
    }
}

// One colour: every site of colour c tries a flip.  T4, T8: the integer
// Metropolis thresholds for dE = 4 and 8.
__global__ __launch_bounds__(kIsingBlock) void k_ising_pass(int8_t *__restrict__ S, IsingGeo g, Key key,
                                                            uint32_t c, const uint32_t *__restrict__ sweep_ptr,
                                                            uint32_t T4, uint32_t T8,
                                                            unsigned long long *__restrict__ accepted)
{
    const uint32_t grp = blockIdx.x * kIsingBlock + threadIdx.x;
    uint32_t flips = 0;
    if (4u * grp < g.half) {
        int8_t *own = S + (size_t)c * g.half;
        const int8_t *oth = S + (size_t)(c ^ 1u) * g.half;
        // every load of the four sites goes out before any store (a store
        // could otherwise be taken to alias a later load and serialise them)
        int sv[4], nb[4];
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) {
            const uint32_t h = min(4u * grp + k, g.half - 1u);
            uint32_t x, y;
            ising_site(g, c, h, x, y);
            const uint32_t xp = x + 1u == g.L0 ? 0u : x + 1u, xm = x == 0u ? g.L0 - 1u : x - 1u;
            const uint32_t yp = y + 1u == g.L1 ? 0u : y + 1u, ym = y == 0u ? g.L1 - 1u : y - 1u;
            nb[k] = oth[(xp >> 1) + g.H0 * y] + oth[(xm >> 1) + g.H0 * y] + oth[(x >> 1) + g.H0 * yp] +
                    oth[(x >> 1) + g.H0 * ym];
            sv[k] = own[h];
        }
        const uint4 r = philox(make_uint4(grp, c | (kPurposeIsing << 8), *sweep_ptr, 0u), key);
        const uint32_t w[4] = { r.x, r.y, r.z, r.w };
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) {
            const uint32_t h = 4u * grp + k;
            const int dE = 2 * sv[k] * nb[k];
            const bool flip = dE <= 0 || (w[k] >> 8) < (dE == 4 ? T4 : T8);
            if (h < g.half && flip) {
                own[h] = (int8_t)-sv[k];  // same-colour sites are never neighbours
                ++flips;
            }
        }
    }
    // one counter add per wave
    unsigned long long n = flips;
#pragma unroll
    for (int off = kIsingWave / 2; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & (kIsingWave - 1)) == 0 && n)
        atomicAdd(&accepted[(blockIdx.x * (kIsingBlock / kIsingWave) + threadIdx.x / kIsingWave) % kAccSlots], n);
}

// ---------------------------------------------------------------------------
// Bit layout
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kIsingBlock) void k_ising_init_bits(uint32_t *__restrict__ P, IsingGeo g, Key key,
                                                                 int hot)
{
    const uint32_t w = blockIdx.x * kIsingBlock + threadIdx.x;  // word of colour c: half indices 32 w ..
    const uint32_t c = blockIdx.y;
    if (w >= g.nw) return;
    uint32_t bits = 0u;
    if (hot) {
#pragma unroll
        for (uint32_t q = 0; q < 8u; ++q) {
            const uint4 r = philox(make_uint4(8u * w + q, c | (kPurposeIsingHot << 8), 0u, 0u), key);
            bits |= ((r.x >> 31) | ((r.y >> 31) << 1) | ((r.z >> 31) << 2) | ((r.w >> 31) << 3)) << (4u * q);
        }
    }
    P[(size_t)c * g.nw + w] = bits;
}

// The four neighbour words of word w of colour c (row y, word k of the row):
// the other colour's spins at the same half index in rows y - 1, y, y + 1,
// and the row's other horizontal neighbour, one half index to the left
// ((c + y) even: x = 2 j, neighbours x +- 1 at j and j - 1) or to the right
// ((c + y) odd: at j and j + 1), shifted in from the next word.
struct BitNbrs {
    uint32_t mid, side, up, dn;
};

__device__ __forceinline__ BitNbrs bit_neighbours(const uint32_t *__restrict__ oth, const IsingGeo &g,
                                                  uint32_t c, uint32_t w)
{
    const uint32_t y = fdiv(w, g.dW), k = w - y * g.W;
    const uint32_t yp = y + 1u == g.L1 ? 0u : y + 1u, ym = y == 0u ? g.L1 - 1u : y - 1u;
    const bool right = ((c + y) & 1u) != 0u;
    const uint32_t kn = right ? (k + 1u == g.W ? 0u : k + 1u) : (k == 0u ? g.W - 1u : k - 1u);
    BitNbrs n;
    n.mid = oth[w];
    const uint32_t nb = oth[y * g.W + kn];
    n.up = oth[yp * g.W + k];
    n.dn = oth[ym * g.W + k];
    n.side = right ? (n.mid >> 1) | (nb << 31) : (n.mid << 1) | (nb >> 31);
    return n;
}

// One colour, one word (32 sites) per lane.  With n the number of
// anti-aligned neighbours of a site, dE = 8 - 4 n: n >= 2 always flips, n = 1
// flips iff its word is below T4, n = 0 iff below T8.
__global__ __launch_bounds__(kIsingBlock) void k_ising_pass_bits(uint32_t *__restrict__ P, IsingGeo g, Key key,
                                                                 uint32_t c, const uint32_t *__restrict__ sweep_ptr,
                                                                 uint32_t T4, uint32_t T8,
                                                                 unsigned long long *__restrict__ accepted)
{
    const uint32_t w = blockIdx.x * kIsingBlock + threadIdx.x;
    uint32_t flips = 0;
    if (w < g.nw) {
        uint32_t *own = P + (size_t)c * g.nw;
        const uint32_t *oth = P + (size_t)(c ^ 1u) * g.nw;
        const BitNbrs n = bit_neighbours(oth, g, c, w);
        const uint32_t s = own[w];
        const uint32_t a1 = s ^ n.mid, a2 = s ^ n.side, a3 = s ^ n.up, a4 = s ^ n.dn;
        const uint32_t any = a1 | a2 | a3 | a4;
        const uint32_t ge2 = (a1 & a2) | (a3 & a4) | ((a1 | a2) & (a3 | a4));
        const uint32_t one = any & ~ge2, zero = ~any;
        const uint32_t sweep = *sweep_ptr;
        uint32_t m4 = 0u, m8 = 0u;
#pragma unroll
        for (uint32_t q = 0; q < 8u; ++q) {
            const uint4 r = philox(make_uint4(8u * w + q, c | (kPurposeIsing << 8), sweep, 0u), key);
            const uint32_t u[4] = { r.x >> 8, r.y >> 8, r.z >> 8, r.w >> 8 };
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) {
                m4 |= (uint32_t)(u[i] < T4) << (4u * q + i);
                m8 |= (uint32_t)(u[i] < T8) << (4u * q + i);
            }
        }
        const uint32_t flip = ge2 | (one & m4) | (zero & m8);
        if (flip) own[w] = s ^ flip;  // same-colour sites are never neighbours
        flips = __popc(flip);
    }
    unsigned long long cnt = flips;
#pragma unroll
    for (int off = kIsingWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & (kIsingWave - 1)) == 0 && cnt)
        atomicAdd(&accepted[(blockIdx.x * (kIsingBlock / kIsingWave) + threadIdx.x / kIsingWave) % kAccSlots], cnt);
}

// Exact integer sums: every bond has one end of colour 0, so the bond sum is
// the sum over colour-0 sites of s times its four neighbours, 4 - 2 n per
// site; the magnetisation counts the set bits of both colours.
__global__ __launch_bounds__(kIsingBlock) void k_ising_obs_bits(const uint32_t *__restrict__ P, IsingGeo g,
                                                                unsigned long long *__restrict__ sums)
{
    const uint32_t w = blockIdx.x * kIsingBlock + threadIdx.x;
    long long bonds = 0, mag = 0;
    if (w < g.nw) {
        const uint32_t *oth = P + g.nw;
        const BitNbrs n = bit_neighbours(oth, g, 0u, w);
        const uint32_t s = P[w];
        // (__popc is unsigned: take the counts as signed before subtracting)
        const int anti = (int)(__popc(s ^ n.mid) + __popc(s ^ n.side) + __popc(s ^ n.up) + __popc(s ^ n.dn));
        const int down = (int)(__popc(s) + __popc(n.mid));
        bonds = 128 - 2 * anti;
        mag = 64 - 2 * down;
    }
#pragma unroll
    for (int off = kIsingWave / 2; off > 0; off >>= 1) {
        bonds += __shfl_xor(bonds, off);
        mag += __shfl_xor(mag, off);
    }
    if ((threadIdx.x & (kIsingWave - 1)) == 0) {
        const uint32_t slot = (blockIdx.x * (kIsingBlock / kIsingWave) + threadIdx.x / kIsingWave) % kAccSlots;
        atomicAdd(&sums[2 * slot], (unsigned long long)bonds);
        atomicAdd(&sums[2 * slot + 1], (unsigned long long)mag);
    }
}

// lex order <-> bit layout: one lane per site out, one lane per word in
__global__ __launch_bounds__(kIsingBlock) void k_ising_pack_bits(const uint32_t *__restrict__ P, IsingGeo g,
                                                                 int8_t *__restrict__ out)
{
    const uint32_t lex = blockIdx.x * kIsingBlock + threadIdx.x;
    if (lex >= 2u * g.half) return;
    const uint32_t y = lex / g.L0, x = lex - y * g.L0;
    const uint32_t h = (x >> 1) + g.H0 * y;
    const uint32_t word = P[(size_t)((x + y) & 1u) * g.nw + h / 32u];
    out[lex] = ((word >> (h % 32u)) & 1u) ? (int8_t)-1 : (int8_t)1;
}

__global__ __launch_bounds__(kIsingBlock) void k_ising_unpack_bits(uint32_t *__restrict__ P, IsingGeo g,
                                                                   const int8_t *__restrict__ in)
{
    const uint32_t w = blockIdx.x * kIsingBlock + threadIdx.x;  // over both colours
    if (w >= 2u * g.nw) return;
    const uint32_t c = w >= g.nw ? 1u : 0u, wc = w - c * g.nw;
    const uint32_t y = fdiv(wc, g.dW), k = wc - y * g.W;
    const uint32_t x0 = (c + y) & 1u;
    uint32_t bits = 0u;
    for (uint32_t b = 0; b < 32u; ++b) {
        const uint32_t x = 2u * (32u * k + b) + x0;
        bits |= (uint32_t)(in[x + g.L0 * y] < 0) << b;
    }
    P[w] = bits;
}

// The sweep index lives in kIsingSweepSlots consecutive words, word j holding
// index + j: sweep j of a graph of several sweeps reads word j, and one tick
// at the end of the graph advances all of them by the graph's sweeps.
constexpr uint32_t kIsingSweepSlots = 32;

__global__ void k_ising_tick(uint32_t *sweep_ptr, uint32_t n)
{
    if (threadIdx.x < kIsingSweepSlots) sweep_ptr[threadIdx.x] += n;
}

// Exact integer sums over all sites: bonds to the +x and +y neighbours, spins.
__global__ __launch_bounds__(kIsingBlock) void k_ising_obs(const int8_t *__restrict__ S, IsingGeo g,
                                                           unsigned long long *__restrict__ sums)
{
    const uint32_t i = blockIdx.x * kIsingBlock + threadIdx.x;  // over both colours
    long long bonds = 0, mag = 0;
    if (i < 2u * g.half) {
        const uint32_t c = i >= g.half ? 1u : 0u, h = i - c * g.half;
        uint32_t x, y;
        ising_site(g, c, h, x, y);
        const int8_t *oth = S + (size_t)(c ^ 1u) * g.half;
        const uint32_t xp = x + 1u == g.L0 ? 0u : x + 1u, yp = y + 1u == g.L1 ? 0u : y + 1u;
        const int s = S[(size_t)c * g.half + h];
        bonds = s * (oth[(xp >> 1) + g.H0 * y] + oth[(x >> 1) + g.H0 * yp]);
        mag = s;
    }
#pragma unroll
    for (int off = kIsingWave / 2; off > 0; off >>= 1) {
        bonds += __shfl_xor(bonds, off);
        mag += __shfl_xor(mag, off);
    }
    if ((threadIdx.x & (kIsingWave - 1)) == 0) {
        // two's complement adds: exact modulo 2^64; spread over kAccSlots pairs
        const uint32_t slot = (blockIdx.x * (kIsingBlock / kIsingWave) + threadIdx.x / kIsingWave) % kAccSlots;
        atomicAdd(&sums[2 * slot], (unsigned long long)bonds);
        atomicAdd(&sums[2 * slot + 1], (unsigned long long)mag);
    }
}

// lex order <-> colour arrays
__global__ __launch_bounds__(kIsingBlock) void k_ising_pack(const int8_t *__restrict__ S, IsingGeo g,
                                                            int8_t *__restrict__ out)
{
    const uint32_t lex = blockIdx.x * kIsingBlock + threadIdx.x;
    if (lex >= 2u * g.half) return;
    const uint32_t y = lex / g.L0, x = lex - y * g.L0;
    out[lex] = S[(size_t)((x + y) & 1u) * g.half + (x >> 1) + g.H0 * y];
}

__global__ __launch_bounds__(kIsingBlock) void k_ising_unpack(int8_t *__restrict__ S, IsingGeo g,
                                                              const int8_t *__restrict__ in)
{
    const uint32_t lex = blockIdx.x * kIsingBlock + threadIdx.x;
    if (lex >= 2u * g.half) return;
    const uint32_t y = lex / g.L0, x = lex - y * g.L0;
    S[(size_t)((x + y) & 1u) * g.half + (x >> 1) + g.H0 * y] = in[lex];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr int kIsingGraphSweeps = (int)kIsingSweepSlots;

struct IsingCtx {
    bool ready = false;
    IsingGeo g{};
    Key key{};
    double beta = 0.0;
    uint32_t T4 = 0, T8 = 0;
    bool bits = false;        // layout: 1-bit words (P) or bytes (S)
    int8_t *S = nullptr;
    uint32_t *P = nullptr;
    uint32_t *d_sweep = nullptr;
    unsigned long long *d_acc = nullptr;   // accepted flips, kAccSlots partial counts
    unsigned long long *d_sums = nullptr;  // observables, kAccSlots (bonds, spins) partial sums
    uint64_t sweep = 0;
    // graphS[k]: k = 1..kIsingGraphSweeps sweeps and one tick (built on first use)
    hipGraphExec_t graphS[kIsingGraphSweeps + 1] = {};
};

IsingCtx I;
char ierr[512] = "no error";

int ifail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ierr, sizeof ierr, fmt, ap);
    va_end(ap);
    return code;
}

#define ITRY(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ifail(SU2_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

void ising_release()
{
    if (I.ready) hipDeviceSynchronize();
    for (hipGraphExec_t gr : I.graphS)
        if (gr) hipGraphExecDestroy(gr);
    void *ptrs[] = { I.S, I.P, I.d_sweep, I.d_acc, I.d_sums };
    for (void *p : ptrs)
        if (p) hipFree(p);
    I = IsingCtx{};
}

// Sets the device sweep-index words to index + j.
hipError_t write_sweep_words(uint32_t index)
{
    uint32_t w[kIsingSweepSlots];
    for (uint32_t j = 0; j < kIsingSweepSlots; ++j) w[j] = index + j;
    return hipMemcpy(I.d_sweep, w, sizeof w, hipMemcpyHostToDevice);
}

uint32_t groups() { return (I.g.half + 3u) / 4u; }
uint32_t blocks_of(uint64_t n) { return (uint32_t)((n + kIsingBlock - 1) / kIsingBlock); }

int build_sweep_graph(int nsweeps, hipGraphExec_t *out)
{
    hipGraph_t graph;
    ITRY(hipGraphCreate(&graph, 0));
    hipGraphNode_t prev = nullptr;
    int rc = SU2_OK;
    int8_t *S = I.S;
    uint32_t *P = I.P;
    IsingGeo g = I.g;
    Key key = I.key;
    uint32_t *spw = I.d_sweep;
    uint32_t nadv = (uint32_t)nsweeps;
    uint32_t T4 = I.T4, T8 = I.T8;
    unsigned long long *acc = I.d_acc;
    uint32_t colours[2] = { 0u, 1u };
    auto add = [&](const void *func, dim3 grid, void **args) -> int {
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(func);
        kp.gridDim = grid;
        kp.blockDim = dim3(func == reinterpret_cast<const void *>(&k_ising_tick) ? 64 : kIsingBlock);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) return ifail(SU2_EDEVICE, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
        prev = node;
        return (int)SU2_OK;
    };
    for (int s = 0; s < nsweeps && rc == SU2_OK; ++s) {
        const uint32_t *sp = I.d_sweep + s;  // sweep s of the graph reads word s (= index + s)
        for (int c = 0; c < 2 && rc == SU2_OK; ++c) {
            if (I.bits) {
                void *args[] = { &P, &g, &key, &colours[c], &sp, &T4, &T8, &acc };
                rc = add(reinterpret_cast<const void *>(&k_ising_pass_bits), dim3(blocks_of(g.nw)), args);
            } else {
                void *args[] = { &S, &g, &key, &colours[c], &sp, &T4, &T8, &acc };
                rc = add(reinterpret_cast<const void *>(&k_ising_pass), dim3(blocks_of(groups())), args);
            }
        }
    }
    // one tick after the graph's sweeps advances every sweep-index word by them
    if (rc == SU2_OK) {
        void *targs[] = { &spw, &nadv };
        rc = add(reinterpret_cast<const void *>(&k_ising_tick), dim3(1), targs);
    }
    if (rc == SU2_OK) {
        hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = ifail(SU2_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    hipGraphDestroy(graph);
    return rc;
}

int ising_ready()
{
    if (!I.ready) return ifail(SU2_ESTATE, "no Ising lattice: call ising_init first");
    return SU2_OK;
}

}  // namespace
}  // namespace su2

using namespace su2;

extern "C" {

int ising_init_ex(const int32_t dims[2], double beta, uint64_t seed, int32_t start, int32_t layout)
{
    if (!dims) return ifail(SU2_EINVAL, "dims is NULL");
    if (dims[0] < 2 || dims[1] < 2 || (dims[0] & 1) || (dims[1] & 1))
        return ifail(SU2_EINVAL, "extents must be even and >= 2");
    const uint64_t N = (uint64_t)dims[0] * (uint64_t)dims[1];
    if (N >= (1ull << 32)) return ifail(SU2_EINVAL, "lattice volume must be below 2^32");
    if (!std::isfinite(beta) || beta < 0.0) return ifail(SU2_EINVAL, "beta must be finite and >= 0");
    if (start != SU2_COLD && start != SU2_HOT) return ifail(SU2_EINVAL, "start must be 0 or 1");
    if (layout < ISING_LAYOUT_AUTO || layout > ISING_LAYOUT_BITS)
        return ifail(SU2_EINVAL, "layout must be 0 (auto), 1 (bytes) or 2 (bits)");
    const bool bits_fit = dims[0] % 64 == 0;
    if (layout == ISING_LAYOUT_BITS && !bits_fit) return ifail(SU2_EINVAL, "the bit layout needs L0 % 64 == 0");
    ising_release();
    // below 2^20 spins both layouts run at the launch floor (~9 us per sweep)
    // and the byte layout's four sites per lane fill the device better
    I.bits = layout == ISING_LAYOUT_BITS || (layout == ISING_LAYOUT_AUTO && bits_fit && N >= (1ull << 20));
    I.g.L0 = (uint32_t)dims[0];
    I.g.L1 = (uint32_t)dims[1];
    I.g.H0 = I.g.L0 / 2u;
    I.g.half = (uint32_t)(N / 2);
    I.g.dH0 = make_fastdiv(I.g.H0);
    I.g.W = I.g.H0 / 32u;
    I.g.nw = I.g.half / 32u;
    I.g.dW = make_fastdiv(I.bits ? I.g.W : 1u);
    I.key = Key{ (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    I.beta = beta;
    I.T4 = (uint32_t)std::floor(std::exp(-4.0 * beta) * 16777216.0);
    I.T8 = (uint32_t)std::floor(std::exp(-8.0 * beta) * 16777216.0);
    const hipError_t ea = I.bits ? hipMalloc(&I.P, (size_t)N / 8) : hipMalloc(&I.S, (size_t)N);
    if (ea != hipSuccess || hipMalloc(&I.d_sweep, kIsingSweepSlots * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&I.d_acc, kAccSlots * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&I.d_sums, 2 * kAccSlots * sizeof(unsigned long long)) != hipSuccess) {
        hipGetLastError();
        ising_release();
        return ifail(SU2_ENOMEM, "cannot allocate the Ising lattice");
    }
    I.ready = true;
    ITRY(write_sweep_words(0u));
    ITRY(hipMemset(I.d_acc, 0, kAccSlots * sizeof(unsigned long long)));
    if (I.bits)
        hipLaunchKernelGGL(k_ising_init_bits, dim3(blocks_of(I.g.nw), 2), dim3(kIsingBlock), 0, nullptr, I.P, I.g,
                           I.key, start == SU2_HOT);
    else
        hipLaunchKernelGGL(k_ising_init, dim3(blocks_of(groups()), 2), dim3(kIsingBlock), 0, nullptr, I.S, I.g,
                           I.key, start == SU2_HOT);
    ITRY(hipGetLastError());
    ITRY(hipDeviceSynchronize());
    return SU2_OK;
}

int ising_init(const int32_t dims[2], double beta, uint64_t seed, int32_t start)
{
    return ising_init_ex(dims, beta, seed, start, ISING_LAYOUT_AUTO);
}

int ising_layout(int32_t *out)
{
    int rc = ising_ready();
    if (rc) return rc;
    if (!out) return ifail(SU2_EINVAL, "out is NULL");
    *out = I.bits ? ISING_LAYOUT_BITS : ISING_LAYOUT_BYTES;
    return SU2_OK;
}

int ising_sweep(int32_t n)
{
    int rc = ising_ready();
    if (rc) return rc;
    if (n < 0) return ifail(SU2_EINVAL, "n must be >= 0");
    if (I.sweep + (uint64_t)n > 0xffffffffull) return ifail(SU2_EINVAL, "sweep index would pass 2^32 - 1");
    // graphs of kIsingGraphSweeps sweeps, then one graph for the rest
    for (int32_t left = n; left > 0;) {
        const int32_t k = std::min<int32_t>(left, kIsingGraphSweeps);
        if (!I.graphS[k]) {
            rc = build_sweep_graph(k, &I.graphS[k]);
            if (rc) return rc;
        }
        ITRY(hipGraphLaunch(I.graphS[k], nullptr));
        left -= k;
    }
    I.sweep += (uint64_t)n;
    return SU2_OK;
}

int ising_observables(double out[2])
{
    int rc = ising_ready();
    if (rc) return rc;
    if (!out) return ifail(SU2_EINVAL, "out is NULL");
    ITRY(hipMemsetAsync(I.d_sums, 0, 2 * kAccSlots * sizeof(unsigned long long), nullptr));
    if (I.bits)
        hipLaunchKernelGGL(k_ising_obs_bits, dim3(blocks_of(I.g.nw)), dim3(kIsingBlock), 0, nullptr, I.P, I.g,
                           I.d_sums);
    else
        hipLaunchKernelGGL(k_ising_obs, dim3(blocks_of(2ull * I.g.half)), dim3(kIsingBlock), 0, nullptr, I.S, I.g,
                           I.d_sums);
    ITRY(hipGetLastError());
    std::vector<unsigned long long> h(2 * kAccSlots);
    ITRY(hipMemcpy(h.data(), I.d_sums, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    unsigned long long bonds = 0, mag = 0;
    for (uint32_t i = 0; i < kAccSlots; ++i) {
        bonds += h[2 * i];
        mag += h[2 * i + 1];
    }
    const double N = 2.0 * (double)I.g.half;
    out[0] = -(double)(long long)bonds / N;
    out[1] = (double)(long long)mag / N;
    return SU2_OK;
}

int ising_spins(int8_t *host_out, size_t n)
{
    int rc = ising_ready();
    if (rc) return rc;
    if (!host_out || n != 2ull * I.g.half) return ifail(SU2_EINVAL, "n must be L0 * L1");
    int8_t *stage = nullptr;
    if (hipMalloc(&stage, n) != hipSuccess) {
        hipGetLastError();
        return ifail(SU2_ENOMEM, "cannot allocate the staging buffer");
    }
    if (I.bits)
        hipLaunchKernelGGL(k_ising_pack_bits, dim3(blocks_of(n)), dim3(kIsingBlock), 0, nullptr, I.P, I.g, stage);
    else
        hipLaunchKernelGGL(k_ising_pack, dim3(blocks_of(n)), dim3(kIsingBlock), 0, nullptr, I.S, I.g, stage);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(host_out, stage, n, hipMemcpyDeviceToHost);
    hipFree(stage);
    if (e != hipSuccess) return ifail(SU2_EDEVICE, "ising_spins: %s", hipGetErrorString(e));
    return SU2_OK;
}

int ising_set_spins(const int8_t *host_in, size_t n, uint64_t sweep_index)
{
    int rc = ising_ready();
    if (rc) return rc;
    if (!host_in || n != 2ull * I.g.half) return ifail(SU2_EINVAL, "n must be L0 * L1");
    if (sweep_index > 0xffffffffull) return ifail(SU2_EINVAL, "sweep index must be below 2^32");
    for (size_t i = 0; i < n; ++i)
        if (host_in[i] != 1 && host_in[i] != -1) return ifail(SU2_EINVAL, "spin %zu is not +1 or -1", i);
    int8_t *stage = nullptr;
    if (hipMalloc(&stage, n) != hipSuccess) {
        hipGetLastError();
        return ifail(SU2_ENOMEM, "cannot allocate the staging buffer");
    }
    hipError_t e = hipMemcpy(stage, host_in, n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        if (I.bits)
            hipLaunchKernelGGL(k_ising_unpack_bits, dim3(blocks_of(2ull * I.g.nw)), dim3(kIsingBlock), 0, nullptr,
                               I.P, I.g, stage);
        else
            hipLaunchKernelGGL(k_ising_unpack, dim3(blocks_of(n)), dim3(kIsingBlock), 0, nullptr, I.S, I.g, stage);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hipFree(stage);
    if (e != hipSuccess) return ifail(SU2_EDEVICE, "ising_set_spins: %s", hipGetErrorString(e));
    ITRY(write_sweep_words((uint32_t)sweep_index));
    I.sweep = sweep_index;
    return SU2_OK;
}

int ising_sweep_index(uint64_t *out)
{
    int rc = ising_ready();
    if (rc) return rc;
    if (!out) return ifail(SU2_EINVAL, "out is NULL");
    *out = I.sweep;
    return SU2_OK;
}

int ising_accepted(uint64_t *out)
{
    int rc = ising_ready();
    if (rc) return rc;
    if (!out) return ifail(SU2_EINVAL, "out is NULL");
    std::vector<unsigned long long> h(kAccSlots);
    ITRY(hipMemcpy(h.data(), I.d_acc, kAccSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    uint64_t total = 0;
    for (unsigned long long v : h) total += v;
    *out = total;
    return SU2_OK;
}

const char *ising_last_error(void) { return ierr; }

void ising_finalize(void) { ising_release(); }

}  // extern "C"
