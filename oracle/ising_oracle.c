/*
 * ising_oracle.c -- plain CPU oracle for the paper's other workload: the 2-D
 * Ising model, H = -sum_<ij> s_i s_j (Sec. 2.3, Eq. (1)), updated by the
 * Metropolis algorithm on a red-black (checkerboard) partition (Sec. 2.3).
 *
 * TEST INFRASTRUCTURE ONLY, like su2_oracle.c (whose Philox-4x32-10 it calls):
 * only the tests and the benchmark's CPU-baseline legs use it, and it shares
 * no code with the HIP library.
 *
 * Conventions (the paper fixes the model and the algorithm, not these):
 *   - lattice L0 x L1, both even, periodic; site (x, y), lex = x + L0 y;
 *     colour c = (x + y) mod 2; a sweep updates colour 0, then colour 1;
 *   - random numbers: a site of colour c has half index h = x/2 + (L0/2) y;
 *     word h mod 4 of Philox(counter = (h/4, c | 4 << 8, sweep, 0), key =
 *     seed) gives its uniform w (top 24 bits);
 *   - Metropolis: dE = 2 s (sum of the four neighbours); the flip is accepted
 *     if dE <= 0, or if (w >> 8) < T(dE) with T(dE) = floor(exp(-beta dE) 2^24)
 *     evaluated in FP64 -- the same test as u <= exp(-beta dE) for the uniform
 *     u = ((w >> 8) + 1) 2^-24, taken on integers so that both sides decide
 *     identically;
 *   - hot start: word h mod 4 of Philox((h/4, c | 5 << 8, 0, 0)), spin -1 if
 *     its top bit is set, else +1; cold start: every spin +1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

static int dims_ok(const int dims[2])
{
    return dims[0] >= 2 && dims[1] >= 2 && dims[0] % 2 == 0 && dims[1] % 2 == 0 &&
           (uint64_t)dims[0] * (uint64_t)dims[1] < (1ull << 32);
}

/* the uniform word of site (x, y) for the given purpose and sweep */
static uint32_t site_word(const int dims[2], uint64_t seed, int x, int y, uint32_t purpose,
                          uint32_t sweep)
{
    const uint32_t c = (uint32_t)((x + y) & 1);
    const uint32_t h = (uint32_t)(x / 2) + (uint32_t)(dims[0] / 2) * (uint32_t)y;
    const uint32_t ctr[4] = { h / 4u, c | (purpose << 8), sweep, 0u };
    const uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[h % 4u];
}

int oracle_ising_init(const int dims[2], uint64_t seed, int start, int8_t *s)
{
    if (!dims_ok(dims) || (start != 0 && start != 1)) return -1;
    for (int y = 0; y < dims[1]; ++y)
        for (int x = 0; x < dims[0]; ++x)
            s[x + dims[0] * y] =
                start ? ((site_word(dims, seed, x, y, 5u, 0u) >> 31) ? -1 : 1) : 1;
    return 0;
}

/* n sweeps starting at sweep index sweep0; accepted[0] += flips accepted */
int oracle_ising_sweep(const int dims[2], double beta, uint64_t seed, uint32_t sweep0, int n,
                       int8_t *s, uint64_t *accepted)
{
    if (!dims_ok(dims) || !(beta >= 0.0) || n < 0) return -1;
    const int L0 = dims[0], L1 = dims[1];
    /* thresholds for dE = 4 and dE = 8 (J = 1) */
    const uint32_t T4 = (uint32_t)floor(exp(-4.0 * beta) * 16777216.0);
    const uint32_t T8 = (uint32_t)floor(exp(-8.0 * beta) * 16777216.0);
    uint64_t acc = 0;
    for (int k = 0; k < n; ++k) {
        const uint32_t sweep = sweep0 + (uint32_t)k;
        for (int c = 0; c < 2; ++c) {
#pragma omp parallel for schedule(static) reduction(+ : acc)
            for (int y = 0; y < L1; ++y)
                for (int x = 0; x < L0; ++x) {
                    if (((x + y) & 1) != c) continue;
                    const int8_t si = s[x + L0 * y];
                    const int nb = s[(x + 1) % L0 + L0 * y] + s[(x + L0 - 1) % L0 + L0 * y] +
                                   s[x + L0 * ((y + 1) % L1)] + s[x + L0 * ((y + L1 - 1) % L1)];
                    const int dE = 2 * si * nb;
                    int flip = dE <= 0;
                    if (!flip) {
                        const uint32_t w = site_word(dims, seed, x, y, 4u, sweep) >> 8;
                        flip = w < (dE == 4 ? T4 : T8);
                    }
                    if (flip) {
                        /* same-colour sites are never neighbours: in place is safe */
                        s[x + L0 * y] = (int8_t)-si;
                        acc += 1;
                    }
                }
        }
    }
    if (accepted) *accepted += acc;
    return 0;
}

/* out[0] = energy per site -(1/N) sum_<ij> s_i s_j, out[1] = magnetisation
 * per site (1/N) sum_i s_i; integer sums, exact. */
int oracle_ising_observables(const int dims[2], const int8_t *s, double out[2])
{
    if (!dims_ok(dims)) return -1;
    const int L0 = dims[0], L1 = dims[1];
    long long bonds = 0, mag = 0;
    for (int y = 0; y < L1; ++y)
        for (int x = 0; x < L0; ++x) {
            const int si = s[x + L0 * y];
            bonds += si * (s[(x + 1) % L0 + L0 * y] + s[x + L0 * ((y + 1) % L1)]);
            mag += si;
        }
    const double N = (double)L0 * (double)L1;
    out[0] = -(double)bonds / N;
    out[1] = (double)mag / N;
    return 0;
}
