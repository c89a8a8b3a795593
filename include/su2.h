/*
 * su2.h -- C ABI of libsu2.so: the SU(2) pure-gauge Wilson-action heat-bath
 * sweep on a periodic 4-D lattice, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Demchik & Strelchenko, "Monte Carlo simulations on Graphics
 * Processing Units" (arXiv:0903.3053), Sec. 2.4: links U_mu(x) in SU(2) as unit
 * quaternions (Eq. (4)), Wilson action (Eqs. (2)-(3)), heat-bath link update
 * towards the staple sum (Eqs. (5)-(7)), odd sites then even sites for each
 * direction, at most 8 attempts per update, FP64 plaquette averages.
 *
 * Conventions shared by every entry point:
 *   - dims = {L0, L1, L2, L3}: extents, each even and >= 2, direction 3 is
 *     time; the product V must be below 2^32.  lex = x0 + L0*(x1 + L1*(x2 +
 *     L2*x3)); parity p(x) = (x0+x1+x2+x3) mod 2, odd = 1.
 *   - Host link layout: float32 [V][4][4] = (lex, direction mu, component),
 *     component 0 the identity part, 1..3 the i*sigma_j parts (Eq. (4)).
 *   - Random numbers: Philox-4x32-10, key = (seed mod 2^32, seed >> 32),
 *     counter = (lex, mu | purpose << 8, sweep index, slot); purpose 0 = heat
 *     bath (slots 0..7 attempts -- Kennedy-Pendleton, or Creutz below the
 *     su2_set_creutz switch -- 8 direction, 9 Haar draw at alpha = 0),
 *     1 = hot start, 2 = learned independence-Metropolis proposal.
 *
 * State: one global lattice context (no handle), created by su2_init /
 * su2_init_ex and released by su2_finalize or the next init.  Calls are not
 * thread-safe.  All work is enqueued on the library's stream (the null stream
 * unless su2_set_stream was called); entry points that return host data
 * synchronise that stream.
 *
 * Errors: every int-returning function returns SU2_OK (0) or a negative code;
 * su2_last_error() gives a message.  Nothing aborts and no C++ exception
 * crosses the ABI.  Functions returning double return NaN on error.
 * Ownership: the library owns the device memory it allocates; host buffers
 * always belong to the caller and are not retained after the call returns.
 */
#ifndef SU2_H
#define SU2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SU2_OK = 0,
    SU2_EINVAL = -1,  /* argument out of range / wrong size */
    SU2_ESTATE = -2,  /* no lattice initialised, or wrong call order */
    SU2_ENOMEM = -3,  /* device allocation failed */
    SU2_EDEVICE = -4  /* a HIP runtime call or kernel launch failed */
};

enum { SU2_COLD = 0, SU2_HOT = 1 };

/* Lattice initialisation (Sec. 2.1: done on the GPU; Sec. 2.4: cold or hot).
 * Allocates the links on the device and fills them: SU2_COLD = identity on
 * every link, SU2_HOT = a Haar-random unit quaternion per link from Philox
 * purpose 1 (Shoemake's three-uniform construction).  beta = 4/g^2 (Sec. 2.4)
 * must be finite and >= 0; start must be SU2_COLD or SU2_HOT.  Resets the
 * sweep counter and the update counters to 0.  Replaces any previous lattice. */
int su2_init(const int32_t dims[4], double beta, uint64_t seed, int32_t start);

/* As su2_init, but the links live in a caller-owned device buffer (e.g. a
 * torch tensor) of at least 64*V bytes, 16-byte aligned; the caller keeps it
 * alive until su2_finalize or the next init.  dev_links == NULL allocates.
 * Layout: eight arrays of V/2 float4, array 2*mu + parity; the link U_mu of
 * site lex sits at element lex / 2 (integer division) of its parity's array.
 * (Sec. 2.1: the lattice lives in one buffer of GPU memory for the whole run.) */
int su2_init_ex(const int32_t dims[4], double beta, uint64_t seed, int32_t start,
                void *dev_links, size_t bytes);

/* Move the current lattice's links into a caller-owned device buffer (e.g. a
 * torch tensor) of at least 64*V bytes, 16-byte aligned, that must not
 * overlap the current link storage: the links are copied there (device to
 * device, on the library's stream, which is then synchronised), the library's
 * own link allocation, if any, is released, and all later work reads and
 * writes the caller's buffer, which the caller keeps alive until su2_finalize
 * or the next init.  Links, sweep index and counters are unchanged.  Layout:
 * as su2_init_ex (eight arrays [mu][parity] of V/2 float4).
 * (Sec. 2.1: the lattice stays in GPU memory; here in memory the caller
 * manages.)  SU2_ESTATE without a lattice; SU2_EINVAL for NULL, a short,
 * misaligned or overlapping buffer. */
int su2_bind(void *dev_links, size_t bytes);

/* n >= 0 full sweeps (Sec. 2.4: for each direction mu = 0..3 the odd sites,
 * then for each mu the even sites; each link update draws its staple, Eq. (6),
 * a Kennedy-Pendleton x0 with at most 8 attempts, a direction, rotates, and
 * reunitarises with an FP64 norm, Eqs. (5)-(7)).  The sweep index used in the
 * Philox counters advances by one per sweep.  Asynchronous. */
int su2_sweep(int32_t n);

/* As su2_sweep (n >= 1), and the last sweep also measures: its even-parity
 * passes for mu = 1, 2, 3 add dot(U_new, staple_nu) for nu < mu, which over
 * the three passes is every plaquette (Eq. (3)) of the resulting
 * configuration exactly once.  The next su2_plaquette / su2_plaquette_st /
 * su2_measure_device then only reduces those partials instead of re-reading
 * the lattice (any call that changes the links discards them).  This is the
 * paper's working sweep with its measuring kernel (Sec. 2.1, Sec. 2.4) with
 * the measurement folded into the update. */
int su2_sweep_measured(int32_t n);

/* One pass: the links U_mu(x) with parity(x) == parity (0 or 1), mu in 0..3,
 * at the current sweep index (which does not advance) -- one of the eight
 * per-direction, per-parity updates of a sweep (Sec. 2.4, Eqs. (5)-(7)).
 * SU2_EINVAL for parity or mu out of range. */
int su2_pass(int32_t parity, int32_t mu);

/* n >= 0 overrelaxation sweeps (Sec. 2.4 names the heat-bath "with
 * overrelaxation" without a formula; this is the standard SU(2) reflection):
 * in the heat-bath sweep's pass order, every link U_mu(x) becomes V U^dag V
 * with V = w/|w| (w the Eq. (6) staple sum) and is renormalised as in Eq. (7);
 * links with w = 0 are kept.  The move keeps each link's local weight
 * exp(beta dot(U, w)), so the plaquette is conserved up to rounding; it draws
 * no random numbers, so the sweep index and the counters do not change.
 * Interleave with su2_sweep (e.g. 1 heat-bath : 3 overrelaxation sweeps) for
 * an ergodic chain.  Uses the launch plan's tile order (identity under order
 * 300). */
int su2_overrelax(int32_t n);

/* One overrelaxation pass: U_mu(x), parity(x) == parity (0 or 1), mu in 0..3
 * (the reflection of su2_overrelax, Sec. 2.4).  SU2_EINVAL for parity or mu
 * out of range. */
int su2_overrelax_pass(int32_t parity, int32_t mu);

/* Mean plaquette P = (P_s + P_t)/2 of (1/2)Tr U_mu,nu(x) (Eq. (3)), FP64
 * reduction.  Synchronises.  NaN on error. */
double su2_plaquette(void);

/* out[0] = P, out[1] = P_s (planes 01, 02, 12), out[2] = P_t (planes 03, 13,
 * 23) -- the spatial/temporal split of Sec. 2.4.  Synchronises. */
int su2_plaquette_st(double out[3]);

/* Polyakov loop: mean over spatial sites of (1/2)Tr of the ordered product of
 * U_3(x, t), t = 0..L3-1.  FP32 products, FP64 reduction.  Synchronises. */
int su2_polyakov(double *out);

/* Polyakov-loop correlator for finite-temperature lattices (L3 = L_t the time
 * extent, Sec. 2.4 and Table 1): out[r] (r = 0 .. rmax, rmax <= min(L0, L1,
 * L2) / 2) = mean over spatial sites xs and the three spatial directions i of
 * L(xs) L(xs + r e_i), L(xs) = (1/2)Tr of the ordered product of U_3(xs, t)
 * over t (FP32 products, FP64 sums in a fixed order).  Synchronises. */
int su2_polyakov_correlator(int32_t rmax, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * correlator as su2_polyakov_correlator, computed by the same kernels in the
 * same order (bit-identical results), but enqueued on the library's stream
 * without waiting and without allocating or freeing anything.  dev_out is
 * caller-owned DEVICE memory of rmax + 1 doubles, 8-byte aligned; it holds
 * C(0..rmax) once the stream reaches this work.  The field and partial sums
 * live in a fixed scratch array of 2^19 doubles (4 MiB) per GPU, held until
 * the process ends: the call needs L0 L1 L2 + ceil(L0 L1 L2 / 256) (rmax + 1)
 * doubles of it (e.g. a 64^3 spatial volume with rmax = 32) and returns
 * SU2_EINVAL beyond that, as for a bad rmax or dev_out.  Every scratch value
 * it reads it has written first in the same call, but all calls on one GPU
 * share the array: calls that can overlap in time (other streams, other
 * threads) race and must be serialised by the caller. */
int su2_polyakov_correlator_noalloc(int32_t rmax, double *dev_out);

/* Enqueue the measurements of the current configuration without waiting:
 * dev_out[0..2] = (P, P_s, P_t) as su2_plaquette_st, dev_out[3] = the
 * Polyakov loop.  dev_out is caller-owned DEVICE memory (4 doubles, 8-byte
 * aligned, e.g. a row of a torch tensor): the averages stay on the GPU until
 * the caller copies them (Sec. 2.4). */
int su2_measure_device(double *dev_out);

/* n sweeps, with (P, P_s, P_t) measured after every `every`-th sweep into a
 * device history that is copied once, at the end, to host_hist
 * [n / every][3] (Sec. 2.4: averages stay on the GPU until the run ends).
 * every >= 1; n must be a multiple of every.  The history buffer stays with
 * the lattice (grown as needed, SU2_ENOMEM if it cannot be); with every <= 16
 * the sweeps run as graphs of 16 / every measurements, each measured sweep
 * reducing into the next history entry, with the same values as one call
 * per measurement.  Synchronises. */
int su2_sweep_measure(int32_t n, int32_t every, double *host_hist);

/* Copy the links to host_out (float32 [V][4][4], caller-owned); n_floats must
 * be 16*V, else SU2_EINVAL.  Synchronises.  (Sec. 2.1: results cross to the
 * host only when asked for; Sec. 2.4: each link is four FP32 numbers.) */
int su2_links(float *host_out, size_t n_floats);

/* Replace the links from host_in (float32 [V][4][4], n_floats = 16*V, values
 * taken as given -- not renormalised) and set the sweep index (below 2^32).
 * With the same seed and sweep index, a run resumed this way is bit-identical
 * to an uninterrupted one.  (Sec. 2.1: a configuration is loaded into GPU
 * memory once, as a hot or cold start or a stored configuration.)  SU2_EINVAL
 * for a wrong size or sweep index.  Synchronises. */
int su2_set_links(const float *host_in, size_t n_floats, uint64_t sweep_index);

/* Current sweep index: the number of sweeps since init or the value last set
 * by su2_set_links (Sec. 2.4: the sweep counts are fixed before a run; here
 * the index is also the third word of every Philox counter). */
int su2_sweep_index(uint64_t *out);

/* Update statistics summed since init (Sec. 2.4: at most 8 heat-bath
 * attempts per update): out[0] = heat-bath attempts evaluated, out[1] =
 * updates whose 8 attempts all failed (the link is kept), out[2] = learned
 * proposals made and out[3] = learned proposals accepted since the last
 * su2_set_proposal(1, ...) (both 0 under the heat-bath).  Synchronises. */
int su2_counters(uint64_t out[4]);

/* Enqueue all later work on this HIP stream (hipStream_t, e.g. a torch
 * stream); NULL selects the null stream.  Synchronises the previous stream.
 * The stream must have the default priority.  (Sec. 2.1: the host enqueues
 * kernels and does not wait for them.) */
int su2_set_stream(void *hip_stream);

/* Launch plan of the pass kernel (no passage of the paper: a launch
 * configuration for this GPU, which changes no result; the paper's own kernels
 * simply cover the lattice, Sec. 2.1): order_kind 0 = workgroups in lattice order;
 * T in 1..99 = each XCD takes a band of x1 rows of every (x2, x3) plane and
 * walks the planes in T x T squares (only where a plane holds a multiple of 8
 * tiles of 256 half-sites and T divides L2 and L3, else SU2_EINVAL);
 * 100 + T = the same with squares and planes walked back and forth;
 * 200 + T = four XCDs share each plane (bands twice as thick), XCDs 0-3 on
 * the planes with x2 < L2/2, walked as 100 + T;
 * 300 = fused pairs: each parity's four passes run as two launches, U_0 then
 * U_1 and U_2 then U_3, each workgroup taking a set of sites that the shift
 * x -> x - mu + nu maps onto itself (an (x0, x1) plane, or an orbit of the
 * (x2, x3) step (-1, +1) times one x0 row), so the second pass reads the
 * first one's results from LDS (only for L0 <= 256, else SU2_EINVAL; the
 * single-pass entry su2_pass is unaffected);
 * 1000 + K (K one of the kinds 0..299 above) = order K for the passes mu = 0
 * and 2 of each parity and the same order backwards for mu = 1 and 3, so a pass
 * starts on the tiles the previous one finished with, whose data is still in
 * the Infinity Cache;
 * lds_bytes (0..65536) of local memory reserved per workgroup to cap the
 * workgroups resident on a compute unit.  Links and counters are
 * bit-identical for every plan, only the speed changes; the plaquette of a
 * measured sweep is summed in another order under plan 300 (rounding-level
 * differences). */
int su2_set_plan(int32_t order_kind, int32_t lds_bytes);

/* Launch-plan tuner (no passage of the paper; speed only).
 * Time each plan in {order 0, 4, 8, 16, 108, 208, 1000, 1008, 1104, 1108, 1116,
 * 1204, 1208, 300}
 * x {LDS 0, 16, 24, 32, 40 KiB} on a scratch copy of the links (reps measured
 * sweeps each, in three rounds over
 * all plans; the lattice, sweep index and all counters are untouched) and
 * install the plan with the smallest median; out (nullable) receives
 * {order_kind, lds_bytes}.  The plan is timed with the proposal installed at
 * the time of the call.  Synchronises. */
int su2_tune(int32_t reps, int32_t out[2]);

/* ---- Learned proposal ---------------------------------------------------
 * An extension of the method (the paper has no learned part; it names the
 * rejection loop's cost on a SIMD machine, Sec. 2.4 and Sec. 3, which this
 * removes).  The heat-bath's x0 has density ~ sqrt(1 - x^2) exp(alpha x), alpha = beta |W|
 * (the local conditional of Eqs. (2), (3), (6)).  A small network maps alpha to
 * the 33 knots of 32 equal-probability segments of x0; the proposal picks a
 * segment with probability 1/32 and draws x0 inside it from the density ~
 * exp(alpha x0) (the conditional's exponential factor, so that the accept
 * step corrects only sqrt(1 - x0^2) and the knots' errors).  Used as an
 * independence-Metropolis proposal with the exact acceptance ratio it leaves
 * that conditional invariant, with the Kennedy-Pendleton draw as the fallback
 * outside the network's range.  A rejected proposal keeps the link's x0 and
 * still redraws its direction about the staple (a Gibbs step: the direction
 * is uniform given x0).  Network: 1 -> 64 -> 64 -> 33 on alpha / 40,
 * SiLU, BF16 weights with FP32 accumulation; outputs 0..31 give segment widths
 * 2 softmax(z), output 32 is reserved.  Parameters: 6433 float32 in the order
 * W1 (64x1), b1 (64), W2 (64x64), b2 (64), W3 (33x64), b3 (33), row-major.
 * The network and its knot table are one global state, independent of the
 * lattice context; su2_mlp_last_error() explains a failed su2_mlp_* /
 * su2_cdf_knots call. */

/* knots[33*i + j] = F^{-1}(j / 32) for alpha = alphas[i] >= 0, the CDF of the
 * x0 density integrated numerically on the device (FP64). */
int su2_cdf_knots(const double *alphas, int32_t n, double *knots);

/* Load the FP32 master parameters (n = 6433); the BF16 copy is their
 * round-to-nearest-even rounding.  Resets the optimiser state. */
int su2_mlp_set_params(const float *params, size_t n);

/* Read back the FP32 master (nullable) and BF16 (nullable) parameters. */
int su2_mlp_get_params(float *master, uint16_t *bf16, size_t n);

/* knots[33*i + j] from the network at alphas[i] (BF16 weights). */
int su2_mlp_forward(const float *alphas, int32_t n, float *knots);

/* Loss (mean over samples and 32 segments of (log w_j - target_logw_j)^2)
 * and its gradient with respect to the 6433 parameters (at the BF16 values),
 * from the device's forward and backward kernels. */
int su2_mlp_loss_grad(const float *alphas, const float *target_logw, int32_t n, float *loss,
                      float *grad);

/* Train on the device: targets are the CDF knots of the n alphas (in
 * [0, 40]) integrated by su2_cdf_knots' kernel, then `steps` full-batch Adam
 * steps (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master
 * parameters, each step's gradient taken at their BF16 rounding, with the
 * learning rate of step t = 1..steps falling from lr0 along half a cosine
 * period towards lr_min (lr_min + (lr0 - lr_min)(1 + cos(pi (t-1)/steps))/2).
 * Every call starts Adam afresh: step counter and both moment estimates are
 * zeroed first.  loss_hist (nullable) receives the loss before each step. */
int su2_mlp_train(const double *alphas, int32_t n, int32_t steps, float lr0, float lr_min,
                  float *loss_hist);

/* Evaluate the network on `points` alphas evenly spaced on [0, 40] into the
 * knot table the sweep uses (knots at other alphas: linear in alpha between
 * rows -- the same table serves proposal and correction, so the step stays
 * exact). */
int su2_mlp_tabulate(int32_t points);

/* Copy the current knot table (n_floats = 33 * points). */
int su2_mlp_table(float *host_out, size_t n_floats);

/* Fill the same knot table with the integrated CDF knots instead of the
 * network's: `points` alphas evenly spaced on [0, 40], knots from
 * su2_cdf_knots' kernel (FP64) rounded to FP32.  The proposal without the
 * network's approximation, to measure what the network costs; needs no
 * parameters.  points in 2..65536, else SU2_EINVAL. */
int su2_cdf_tabulate(int32_t points);

const char *su2_mlp_last_error(void);

/* Proposal of the lattice context's passes: 0 = Kennedy-Pendleton heat-bath
 * (Sec. 2.4; bf16_weights is ignored); 1 = the learned independence-
 * Metropolis step (Philox purpose 2, one call per update) with the heat-bath
 * for alpha = 0 and alpha above 40.  With kind 1 and bf16_weights != NULL,
 * the network first takes those n_weights = 6433 BF16 parameters (bit
 * patterns, the order of su2_mlp_set_params; its FP32 master becomes their
 * exact values and the optimiser state is reset) and is tabulated at the
 * current table size (31 rows if none was made yet); with NULL the current
 * table is used (SU2_ESTATE if there is none).  Kind 1 copies the table into
 * the lattice context and zeroes the proposal counters.  su2_init resets the
 * proposal to 0.  SU2_EINVAL for another kind or a wrong n_weights. */
int su2_set_proposal(int32_t kind, const uint16_t *bf16_weights, size_t n_weights);

/* Element offsets of the pass, pair and overrelaxation kernels: on = 1 forms
 * them in 64 bits even where 32-bit ones suffice (a link array below 4 GiB,
 * i.e. V below 2^29, where they are used by default); 0 = automatic.  The
 * 64-bit forms are what lattices of 2^29 sites and more run; this lets a
 * small lattice exercise them.  Results are identical either way.  su2_init
 * resets it to 0.  SU2_EINVAL for another value, SU2_ESTATE before init. */
int su2_set_wide_offsets(int32_t on);

/* Small-alpha switch of the heat-bath (proposal 0): an update with 0 < alpha <
 * alpha_below draws x0 by Creutz's method (Phys. Rev. D 21 (1980) 2308)
 * instead of Kennedy-Pendleton's, with the same cap of 8 attempts and the same
 * Philox slots: attempt t uses words (u0, u1) of slot t, m = -ln(1 - (1 - u0)
 * (1 - exp(-2 alpha))) / alpha, x0 = 1 - m, accepted iff u1^2 <= m (2 - m);
 * direction and rotation as before.  Kennedy-Pendleton's acceptance falls
 * towards 0 as alpha -> 0 (at alpha = 0.25 about 35% of updates hit the cap
 * and keep their link), Creutz's rises towards pi/4; the two accept equally
 * often at alpha = 1.6847 (71%), the suggested switch.  alpha_below in [0, 4]
 * (0 = off); su2_init resets it to 0; it applies to proposal 0 only (the
 * learned proposal covers small alpha itself) and to every launch plan except
 * the batched replicas'.  Results stay a pure function of the inputs. */
int su2_set_creutz(double alpha_below);

/* Learned-proposal updates proposed and accepted since su2_set_proposal(1, ...)
 * (out[2], out[3] of su2_counters). */
int su2_imh_counters(uint64_t out[2]);

/* ---- Batched replicas ---------------------------------------------------
 * A second, independent context: n lattices, each with its own extents
 * dims[4*r .. 4*r+3] (even, >= 2, V/2 * 16 bytes below 4 GiB), coupling
 * betas[r] and seed seeds[r], all started cold or hot.  Every replica evolves
 * exactly as a single lattice with the same (dims, beta, seed, start) would
 * under su2_init + su2_sweep: the same Philox counters, the same sweep order
 * (Sec. 2.4), bit-identical links.  The paper runs one parameter point per GPU
 * (Sec. 3); here many share one device.  Replaces any previous batch. */
int su2_batch_init(int32_t n, const int32_t *dims, const double *betas, const uint64_t *seeds,
                   int32_t start);

/* n >= 0 sweeps of every replica, each the sweep of Sec. 2.4 (synchronises in
 * persistent mode). */
int su2_batch_sweep(int32_t n);

/* How su2_batch_sweep runs: mode 0 = one launch per (parity, mu) pass over
 * the tiles of all replicas, replayed from hipGraphs of up to 16 sweeps
 * (each XCD takes a contiguous chunk of the tiles); mode 1 = one
 * persistent launch per call (graph-captured with a counter reset and a
 * completion check), in which each replica is pinned to one XCD (replicas
 * balanced over the XCDs by size) and the workgroups running on an XCD take
 * (sweep, pass, replica, tiles) items of its replicas from that XCD's queue in
 * order; an item waits for its replica's previous pass (per-replica
 * completion counters).  SU2_EDEVICE if a wait exceeds the spin limit or an
 * XCD's queue was left unfinished.  tiles_per_item (1..64) tiles of 256
 * half-sites form one work item; lds_bytes (0..65536) caps resident
 * workgroups.  Results do not depend on any of these. */
int su2_batch_set_mode(int32_t mode, int32_t tiles_per_item, int32_t lds_bytes);

/* Time every {mode 0, 1} x {1, 2, 4, 8, 16 tiles per item} x {0, 24 KiB LDS} over
 * `sweeps` sweeps, in three rounds over all candidates, on a saved copy of the
 * state (restored afterwards) and install the one with the smallest median;
 * out (nullable) receives {mode, tiles_per_item, lds_bytes}. */
int su2_batch_tune(int32_t sweeps, int32_t out[3]);

/* Bound, in wall-clock ticks, on any single dependency wait of the
 * persistent kernel (default: 2 s).  A wait that exceeds it makes the launch
 * stop early and su2_batch_sweep return SU2_EDEVICE; the replicas are then in
 * an undefined intermediate state and must be re-initialised. */
int su2_batch_set_spin_limit(uint64_t ticks);

/* out[3*r .. 3*r+2] = (P, P_s, P_t) of replica r (as su2_plaquette_st: the
 * Eq. (3) averages of Sec. 2.4 in FP64).  out holds 3n doubles.  Synchronises. */
int su2_batch_plaquette(double *out);

/* Links of replica r, float32 [V][4][4] (n_floats = 16*V of that replica,
 * else SU2_EINVAL), as su2_links.  Synchronises. */
int su2_batch_links(int32_t r, float *host_out, size_t n_floats);

/* Heat-bath attempts and cap failures of replica r since su2_batch_init
 * (Sec. 2.4: at most 8 attempts per update), as out[0..1] of su2_counters. */
int su2_batch_counters(int32_t r, uint64_t out[2]);

/* Sweeps done since su2_batch_init (the same for every replica; the Philox
 * sweep word of each replica's counters). */
int su2_batch_sweep_index(uint64_t *out);

/* Message for the last error of a su2_batch_* call (static storage). */
const char *su2_batch_last_error(void);

/* Release the batch and its device memory; safe to call twice. */
void su2_batch_finalize(void);

/* Device Philox-4x32-10 blocks for n host counters ctr[n][4] and key = (seed
 * mod 2^32, seed >> 32), written to host out[n][4] (both caller-owned, n <=
 * 2^28); for bit-exact checks of the generator the sweep uses.  It replaces
 * the paper's RANMAR (Sec. 2.2) by a counter-based generator, so numbers are
 * computed where they are used and never stored -- the property Sec. 2.2
 * credits for its speed.  Needs no lattice.  Synchronises. */
int su2_philox(uint64_t seed, const uint32_t *ctr, size_t n, uint32_t *out);

/* Wait for all enqueued work on the library's stream (Sec. 2.1: the host
 * waits only where it needs results). */
int su2_synchronize(void);

/* Message for the last error of a lattice-context call (static storage,
 * never NULL). */
const char *su2_last_error(void);

/* Release the lattice and every device resource the library allocated
 * (caller-owned buffers are left alone); safe to call twice. */
void su2_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* SU2_H */
