// su2_device.hpp -- device-side building blocks of the SU(2) heat-bath path on
// gfx950: Philox-4x32-10, quaternion algebra of Eq. (4), checkerboard lattice
// geometry, and the uniform / Haar / direction draws the update needs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace su2 {

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon et al., SC'11).  Counter-based: nothing is stored,
// each draw is a pure function of (key, counter) -- the paper's Sec. 2.2 point
// that generating numbers inside the consumer, never storing them, is what
// makes the generator fast.  The key words are wave-uniform, so the Weyl key
// schedule stays on the scalar unit.
// ---------------------------------------------------------------------------
struct Key {
    uint32_t lo, hi;
};

__device__ __forceinline__ uint4 philox(uint4 c, Key k)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
    uint32_t ka = k.lo, kb = k.hi;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c.x;  // one v_mad_u64_u32 each
        const uint64_t pb = (uint64_t)kMulB * c.z;
        c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ ka, (uint32_t)pb,
                       (uint32_t)(pa >> 32) ^ c.w ^ kb, (uint32_t)pa);
        ka += kWeylA;
        kb += kWeylB;
    }
    return c;
}

// top 24 bits of a word, as a uniform in (0, 1] -- exact in FP32:
// ((w >> 8) + 1) 2^-24 as one fused multiply-add of exact terms
__device__ __forceinline__ float unit24(uint32_t w)
{
    return __builtin_fmaf((float)(w >> 8), 0x1p-24f, 0x1p-24f);
}

enum : uint32_t { kPurposeUpdate = 0u, kPurposeHot = 1u, kPurposeImh = 2u };
enum : uint32_t { kSlotDirection = 8u, kSlotHaar = 9u };

__device__ __forceinline__ uint4 draw(Key k, uint32_t site, uint32_t mu, uint32_t purpose,
                                      uint32_t sweep, uint32_t slot)
{
    return philox(make_uint4(site, mu | (purpose << 8), sweep, slot), k);
}

// ---------------------------------------------------------------------------
// Quaternions U = u0 I + i sigma.u, Eq. (4), held in a float4 (x = u0).
// ---------------------------------------------------------------------------
// The quaternion arithmetic spells out every fused multiply-add, so the
// rounding is the same in every kernel that inlines it (the compiler may not
// fuse or split anything here).
__device__ __forceinline__ float4 qmul(float4 a, float4 b)  // a b
{
    return make_float4(__builtin_fmaf(a.x, b.x, -__builtin_fmaf(a.y, b.y, __builtin_fmaf(a.z, b.z, a.w * b.w))),
                       __builtin_fmaf(a.x, b.y, __builtin_fmaf(b.x, a.y, __builtin_fmaf(-a.z, b.w, a.w * b.z))),
                       __builtin_fmaf(a.x, b.z, __builtin_fmaf(b.x, a.z, __builtin_fmaf(-a.w, b.y, a.y * b.w))),
                       __builtin_fmaf(a.x, b.w, __builtin_fmaf(b.x, a.w, __builtin_fmaf(-a.y, b.z, a.z * b.y))));
}

__device__ __forceinline__ float4 qdag(float4 a) { return make_float4(a.x, -a.y, -a.z, -a.w); }

__device__ __forceinline__ float4 qadd(float4 a, float4 b)
{
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

__device__ __forceinline__ float qdot(float4 a, float4 b)  // (1/2) Re Tr(a b^dag)
{
    return __builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, __builtin_fmaf(a.z, b.z, a.w * b.w)));
}

// Reunitarisation, Eq. (7): divide by the norm, summed in FP64.  A product
// of two unit quaternions held in FP32 has n2 = |q|^2 within ~1e-6 of 1, where
// 1/sqrt(1 + d) = 1 - d/2 + 3d^2/8 - 5d^3/16 + O(d^4) reaches FP64 precision
// for |d| < 2^-14 (the next term is below 2^-57): three FP64 fused
// multiply-adds instead of a square root and a division.  Larger d (never
// produced by the update) takes the square root and the division.
__device__ __forceinline__ float4 unitize(float4 q)
{
    const double x = q.x, y = q.y, z = q.z, w = q.w;
    const double n2 = __builtin_fma(x, x, __builtin_fma(y, y, __builtin_fma(z, z, w * w)));
    const double d = n2 - 1.0;
    double inv;
    if (__builtin_fabs(d) < 0x1p-14)
        inv = __builtin_fma(d, __builtin_fma(d, __builtin_fma(d, -0.3125, 0.375), -0.5), 1.0);
    else
        inv = 1.0 / sqrt(n2);
    return make_float4((float)(x * inv), (float)(y * inv), (float)(z * inv), (float)(w * inv));
}

// Haar-uniform unit quaternion from three uniforms (Shoemake 1992).
__device__ __forceinline__ float4 haar(uint4 r)
{
    const float u0 = unit24(r.x), u1 = unit24(r.y), u2 = unit24(r.z);
    const float ra = sqrtf(1.0f - u0), rb = sqrtf(u0);
    float s1, c1, s2, c2;
    sincospif(2.0f * u1, &s1, &c1);
    sincospif(2.0f * u2, &s2, &c2);
    return make_float4(ra * s1, ra * c1, rb * s2, rb * c2);
}

// ---------------------------------------------------------------------------
// Unsigned division by a runtime-invariant divisor via a multiply-high
// (Granlund & Montgomery, PLDI'94, the round-up method with a 33-bit
// multiplier split as 2^32 + m): q = (t + ((n - t) >> s1)) >> s2.
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;  // l = ceil(log2 d)
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1ull);
    f.s1 = l < 1 ? l : 1u;
    f.s2 = l > 1 ? l - 1u : 0u;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    const uint32_t t = __umulhi(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// ---------------------------------------------------------------------------
// Checkerboard geometry.  Links of direction mu on sites of parity p form one
// contiguous array of V/2 float4, indexed by the half-site index
// h = (x0 >> 1) + H0*(x1 + L1*(x2 + L2*x3)), H0 = L0/2: coalesced 16-byte
// accesses along x0, and a pass touches whole arrays.  Array (mu, p) starts at
// (2*mu + p) * V/2.
// ---------------------------------------------------------------------------
struct Geo {
    uint32_t L[4];
    uint32_t H0;       // L0 / 2
    uint32_t half;     // V / 2
    uint32_t st[4];    // half-index strides of x0 (pairs), x1, x2, x3: 1, H0, H0*L1, H0*L1*L2
    uint32_t wrap[4];  // (L_d - 1) * st[d]: the jump back across the periodic boundary
    FastDiv dH0, dL1, dL2, dL0;
};

struct Site {
    uint32_t x[4];
};

// site of parity p with half index h
__device__ __forceinline__ Site site_of(const Geo &g, uint32_t h, uint32_t p)
{
    Site s;
    const uint32_t r = fdiv(h, g.dH0);
    const uint32_t hx = h - r * g.H0;
    const uint32_t r2 = fdiv(r, g.dL1);
    s.x[1] = r - r2 * g.L[1];
    s.x[3] = fdiv(r2, g.dL2);
    s.x[2] = r2 - s.x[3] * g.L[2];
    s.x[0] = 2u * hx + ((p + s.x[1] + s.x[2] + s.x[3]) & 1u);
    return s;
}

__device__ __forceinline__ uint32_t lex_of(const Geo &g, const Site &s)
{
    return s.x[0] + g.L[0] * (s.x[1] + g.L[1] * (s.x[2] + g.L[2] * s.x[3]));
}

__device__ __forceinline__ uint32_t half_of(const Geo &g, const Site &s)
{
    return (s.x[0] >> 1) + s.x[1] * g.st[1] + s.x[2] * g.st[2] + s.x[3] * g.st[3];
}

__device__ __forceinline__ Site step(const Geo &g, Site s, int d, int dir)
{
    if (dir > 0)
        s.x[d] = (s.x[d] + 1u == g.L[d]) ? 0u : s.x[d] + 1u;
    else
        s.x[d] = (s.x[d] == 0u) ? g.L[d] - 1u : s.x[d] - 1u;
    return s;
}

__device__ __forceinline__ size_t arr(const Geo &g, uint32_t mu, uint32_t p)
{
    return (size_t)(2u * mu + p) * g.half;
}

// Half index of the neighbour x + e_D (plus) or x - e_D (minus) of a site with
// half index h and coordinate xd along D, by additions only.  Along x0 the
// half index changes only when the step crosses a pair boundary.
template <int D>
__device__ __forceinline__ uint32_t h_plus(const Geo &g, uint32_t h, uint32_t xd)
{
    if constexpr (D == 0)
        return (xd & 1u) ? ((xd + 1u == g.L[0]) ? h - (g.H0 - 1u) : h + 1u) : h;
    else
        return (xd + 1u == g.L[D]) ? h - g.wrap[D] : h + g.st[D];
}

template <int D>
__device__ __forceinline__ uint32_t h_minus(const Geo &g, uint32_t h, uint32_t xd)
{
    if constexpr (D == 0)
        return (xd & 1u) ? h : ((xd == 0u) ? h + (g.H0 - 1u) : h - 1u);
    else
        return (xd == 0u) ? h + g.wrap[D] : h - g.st[D];
}

// 16-byte load of element idx of an array: with OFF32 the byte offset is
// formed in 32 bits (valid while an array is below 4 GiB), which lets the
// load use a scalar base address plus a 32-bit lane offset.
template <bool OFF32>
__device__ __forceinline__ float4 ld4(const float4 *base, uint32_t idx)
{
    if constexpr (OFF32)
        return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + idx * 16u);
    else
        return base[idx];
}

template <bool OFF32>
__device__ __forceinline__ void st4_stream(float4 *base, uint32_t idx, float4 v)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 *ptr;
    if constexpr (OFF32)
        ptr = reinterpret_cast<f4 *>(reinterpret_cast<char *>(base) + idx * 16u);
    else
        ptr = reinterpret_cast<f4 *>(base + idx);
    const f4 val = { v.x, v.y, v.z, v.w };
    __builtin_nontemporal_store(val, ptr);  // written links are not re-read in this pass
}

}  // namespace su2
