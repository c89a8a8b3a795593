/* ising.h -- C ABI of the 2-D Ising workload in libsu2.so: the paper's other
 * model (Sec. 2.3), H = -sum_<ij> s_i s_j (Eq. (1)) on an L0 x L1 periodic
 * lattice, updated by the Metropolis algorithm on a red-black (checkerboard)
 * partition, with the same counter-based random numbers as the SU(2) path.
 *
 * Conventions: site (x, y), lex = x + L0 y, colour c = (x + y) mod 2; a sweep
 * updates colour 0, then colour 1.  A site of colour c has half index
 * h = x/2 + (L0/2) y; word h mod 4 of Philox-4x32-10(counter = (h/4, c | 4 << 8,
 * sweep, 0), key = (seed mod 2^32, seed >> 32)) is its random word w, and a
 * flip with energy change dE > 0 is accepted iff (w >> 8) < floor(exp(-beta dE)
 * 2^24) (FP64 on the host), i.e. u <= exp(-beta dE) for u = ((w >> 8) + 1)
 * 2^-24; dE <= 0 is always accepted.  Hot start: word h mod 4 of
 * Philox((h/4, c | 5 << 8, 0, 0)), spin -1 if its top bit is set; cold: all +1.
 *
 * One global Ising context, independent of the SU(2) one; calls are not
 * thread-safe; the null stream is used.  Every function except the getters
 * returns 0 or a negative SU2_* code (su2.h) and ising_last_error() explains
 * it.  Spins cross the boundary as int8 (+1 / -1) in lex order; the library
 * owns its device memory. */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Device layout of the spins (results do not depend on it): bytes = one int8
 * per spin, one array per colour indexed by h; bits = the paper's 1-bit spins
 * (Sec. 2.3), bit b of word w of a colour holding half index h = 32 w + b
 * (set = spin -1), 16x less memory, updated 32 sites per lane with bitwise
 * arithmetic; needs L0 a multiple of 64.  Auto takes bits where they fit
 * and the lattice holds at least 2^20 spins (below that both run at the
 * ~9 us launch floor per sweep and bytes fill the device better). */
enum { ISING_LAYOUT_AUTO = 0, ISING_LAYOUT_BYTES = 1, ISING_LAYOUT_BITS = 2 };

/* dims = {L0, L1}: each even and >= 2, L0 * L1 < 2^32; beta finite and >= 0;
 * start 0 = cold, 1 = hot.  Sweep index 0, acceptance counter 0.  Layout
 * auto. */
int ising_init(const int32_t dims[2], double beta, uint64_t seed, int32_t start);

/* ising_init with a chosen layout (SU2_EINVAL for bits unless L0 % 64 == 0). */
int ising_init_ex(const int32_t dims[2], double beta, uint64_t seed, int32_t start, int32_t layout);

/* The layout in use (ISING_LAYOUT_BYTES or ISING_LAYOUT_BITS). */
int ising_layout(int32_t *out);

/* n >= 0 Metropolis sweeps (replayed from a hipGraph); the sweep index
 * advances by n (SU2_EINVAL if it would pass 2^32 - 1). */
int ising_sweep(int32_t n);

/* out[0] = energy per site -(1/N) sum_<ij> s_i s_j, out[1] = magnetisation per
 * site (1/N) sum_i s_i, from exact integer sums on the device.  Synchronises. */
int ising_observables(double out[2]);

/* Copy the spins (n = L0 * L1 int8, lex order) to / from a caller buffer;
 * ising_set_spins also sets the sweep index (entries must be +1 or -1). */
int ising_spins(int8_t *host_out, size_t n);
int ising_set_spins(const int8_t *host_in, size_t n, uint64_t sweep_index);

/* Sweeps done since init (or the index set by ising_set_spins). */
int ising_sweep_index(uint64_t *out);

/* Accepted flips since init. */
int ising_accepted(uint64_t *out);

const char *ising_last_error(void);
void ising_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
