/*
 * su2_oracle.c -- plain CPU oracle for the SU(2) Wilson-action heat-bath sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the tests, the package's smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library; both are written from the same written conventions.
 *
 * Arithmetic is FP64 throughout, with two exceptions the paper or the parity
 * rule fixes:
 *   - link storage: with prec32 != 0 every written link is rounded to FP32,
 *     because the paper stores each link as four single-precision numbers in one
 *     128-bit cell (Sec. 2.4, the paragraph after Eq. (4));
 *   - the accept tests of the Kennedy-Pendleton and Creutz draws: with
 *     prec32 != 0 each is taken in FP32 (each FP32 operand is the rounding of
 *     its FP64 value), because a floating point decision that picks an integer
 *     outcome is taken in the same precision on both sides of a parity
 *     comparison.  Only the decision is FP32: the accepted draw's x0 and |a|
 *     are built from the FP64 value of lambda^2 (or of m).
 * With prec32 == 0 the whole chain runs in FP64 (used to state errors against
 * FP64).
 *
 * Nothing here is blocked, fused or reordered: every site of a pass is visited
 * in lexicographic order (OpenMP only splits that loop; each update is a pure
 * function of the links of the other parity/directions and of its own Philox
 * counter, so the result does not depend on the split).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  The paper's own generator is RANMAR (Sec. 2.2); */
/* it is replaced by this counter-based generator so that random numbers are  */
/* never stored, which is the property Sec. 2.2 credits for the speed-up.     */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        /* one Philox round: two 32x32->64 products, halves mixed with the key */
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        /* Weyl key schedule */
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 32-bit word -> uniform in (0, 1]: the top 24 bits, shifted up by one step so
 * that log(u) is always finite.  Exact in FP32 and in FP64. */
double oracle_uniform(uint32_t w)
{
    return (double)((w >> 8) + 1u) * (1.0 / 16777216.0);
}

/* Counter layout of one Philox call: (site, mu | purpose<<8, sweep, slot). */
enum { PURPOSE_UPDATE = 0, PURPOSE_HOT = 1, PURPOSE_IMH = 2 };
enum { SLOT_DIRECTION = 8, SLOT_HAAR = 9 };

static void draw4(uint64_t seed, uint32_t site, int mu, int purpose, uint32_t sweep,
                  uint32_t slot, double u[4])
{
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { site, (uint32_t)mu | ((uint32_t)purpose << 8), sweep, slot };
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = oracle_uniform(w[i]);
}

/* ------------------------------------------------------------------------- */
/* Quaternion algebra of Eq. (4): U = u0*I + i*sigma_j*u_j.                   */
/* ------------------------------------------------------------------------- */

/* c = a*b.  From (i s.a)(i s.b) = -(a.b) I - i s.(a x b):
 *   c0 = a0 b0 - a.b,   c_vec = a0 b_vec + b0 a_vec - a_vec x b_vec. */
void oracle_qmul(const double a[4], const double b[4], double c[4])
{
    double r0 = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double r1 = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    double r2 = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    double r3 = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
    c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}

static void qdag(const double a[4], double c[4])
{
    c[0] = a[0]; c[1] = -a[1]; c[2] = -a[2]; c[3] = -a[3];
}

/* ------------------------------------------------------------------------- */
/* Geometry: extents L[0..3] (x0 fastest, direction 3 is time), periodic.     */
/* lex = x0 + L0*(x1 + L1*(x2 + L2*x3)); parity = (x0+x1+x2+x3) mod 2.        */
/* ------------------------------------------------------------------------- */
typedef struct { int L[4]; long V; } geom_t;

static void coords(const geom_t *g, long lex, int x[4])
{
    for (int d = 0; d < 4; ++d) { x[d] = (int)(lex % g->L[d]); lex /= g->L[d]; }
}

static long lex_of(const geom_t *g, const int x[4])
{
    return x[0] + (long)g->L[0] * (x[1] + (long)g->L[1] * (x[2] + (long)g->L[2] * x[3]));
}

/* lex of x + step*e_d with periodic wrap */
static long shifted(const geom_t *g, const int x[4], int d, int step)
{
    int y[4] = { x[0], x[1], x[2], x[3] };
    y[d] = ((y[d] + step) % g->L[d] + g->L[d]) % g->L[d];
    return lex_of(g, y);
}

/* links: double[V][4][4] = (site, direction, quaternion component) */
static const double *link(const double *U, long lex, int mu) { return U + (lex * 4 + mu) * 4; }

static int geom_init(geom_t *g, const int dims[4])
{
    g->V = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2 || (dims[d] & 1)) return -1;
        g->L[d] = dims[d];
        g->V *= dims[d];
    }
    if (g->V > 0xffffffffL) return -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Staple sum, Eq. (6), over the six plaquettes that contain U_mu(x)          */
/* (nu != mu: the "mu < nu" under the sum would leave direction 3 without     */
/* staples).  Each term is the product of the other three links of one        */
/* plaquette, oriented so that (1/2)Tr(U_mu(x) W_mu(x)^dag) is the sum of the */
/* (1/2)Tr of those plaquettes, Eq. (3).                                       */
/* ------------------------------------------------------------------------- */
void oracle_staple(const int dims[4], const double *U, long lex, int mu, double w[4])
{
    geom_t g;
    geom_init(&g, dims);
    int x[4];
    coords(&g, lex, x);
    long x_pmu = shifted(&g, x, mu, +1);
    int xpm[4];
    coords(&g, x_pmu, xpm);
    w[0] = w[1] = w[2] = w[3] = 0.0;
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        long x_pnu = shifted(&g, x, nu, +1);
        long x_mnu = shifted(&g, x, nu, -1);
        long x_pmu_mnu = shifted(&g, xpm, nu, -1);
        double t[4], d[4], s[4];
        /* U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag */
        oracle_qmul(link(U, lex, nu), link(U, x_pnu, mu), t);
        qdag(link(U, x_pmu, nu), d);
        oracle_qmul(t, d, s);
        for (int c = 0; c < 4; ++c) w[c] += s[c];
        /* U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) */
        qdag(link(U, x_mnu, nu), d);
        oracle_qmul(d, link(U, x_mnu, mu), t);
        oracle_qmul(t, link(U, x_pmu_mnu, nu), s);
        for (int c = 0; c < 4; ++c) w[c] += s[c];
    }
}

/* ------------------------------------------------------------------------- */
/* Haar-uniform unit quaternion from three uniforms (Shoemake, "Uniform       */
/* random rotations", Graphics Gems III, 1992).                               */
/* ------------------------------------------------------------------------- */
static void haar_from_uniforms(const double u[4], double q[4])
{
    double r1 = sqrt(1.0 - u[0]), r2 = sqrt(u[0]);
    double t1 = 2.0 * M_PI * u[1], t2 = 2.0 * M_PI * u[2];
    q[0] = r1 * sin(t1);
    q[1] = r1 * cos(t1);
    q[2] = r2 * sin(t2);
    q[3] = r2 * cos(t2);
}

/* ------------------------------------------------------------------------- */
/* Kennedy-Pendleton draw of x0 from sqrt(1-x0^2) exp(alpha x0) on [-1, 1]    */
/* (the heat-bath of Sec. 2.4, Eqs. (5)-(7), with at most 8 attempts per     */
/* update, Sec. 2.4).                                                         */
/*   lambda^2 = -(ln u0 + cos^2(2 pi u1) ln u2) / (2 alpha)  (a Gamma(3/2)    */
/*   variate over 2 alpha); accept iff u3^2 <= 1 - lambda^2; x0 = 1-2lambda^2.*/
/* Returns the attempt index that accepted (0..7) or -1 when all 8 failed.   */
/* *margin receives min |u3^2 - (1 - lambda^2)| over the attempts evaluated.  */
/* With prec32 the test is taken in FP32 in the form it has multiplied by    */
/* 2 alpha > 0: 2 alpha (1 - u3^2) + num >= 0, num = ln u0 + cos^2 ln u2      */
/* (= -2 alpha lambda^2), with one rounding for the last multiply-add.       */
/* ------------------------------------------------------------------------- */
int oracle_kp_draw(double alpha, uint64_t seed, uint32_t site, int mu, uint32_t sweep,
                   int prec32, double *a0_out, double *amag_out, double *margin)
{
    double m = INFINITY;
    for (uint32_t t = 0; t < 8; ++t) {
        double u[4];
        draw4(seed, site, mu, PURPOSE_UPDATE, sweep, t, u);
        /* the draw itself, in FP64 */
        double c = cos(2.0 * M_PI * u[1]);
        double lam2 = -(log(u[0]) + c * c * log(u[2])) / (2.0 * alpha);
        double lhs, rhs;
        if (prec32) {
            /* the decision in FP32, from the FP32 roundings of its inputs */
            float lu0 = (float)log(u[0]);
            float cf = (float)c;
            float lu2 = (float)log(u[2]);
            float af = (float)alpha;
            float numf = lu0 + cf * cf * lu2;
            float u3f = (float)u[3];
            float tf = 1.0f - u3f * u3f;
            float df = fmaf(2.0f * af, tf, numf);
            /* accept iff df >= 0; the margin in the units of lambda^2 */
            lhs = 0.0;
            rhs = (double)df / (2.0 * (double)af);
        } else {
            lhs = u[3] * u[3];
            rhs = 1.0 - lam2;
        }
        double dm = fabs(lhs - rhs);
        if (dm < m) m = dm;
        if (lhs <= rhs) {
            *a0_out = 1.0 - 2.0 * lam2;
            *amag_out = 2.0 * sqrt(lam2 * (1.0 - lam2));
            if (margin) *margin = m;
            return (int)t;
        }
    }
    if (margin) *margin = m;
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Creutz's draw of x0 from the same density (M. Creutz, Phys. Rev. D 21       */
/* (1980) 2308), used below a switch in alpha where Kennedy-Pendleton's        */
/* acceptance collapses; same cap of 8 attempts and same slots, words u0, u1:  */
/*   y = 1 - (1 - u0)(1 - exp(-2 alpha)) is uniform on [exp(-2 alpha), 1], so  */
/*   x0 = 1 + ln(y) / alpha has density proportional to exp(alpha x0) on       */
/*   [-1, 1]; accept iff u1 <= sqrt(1 - x0^2), i.e. u1^2 <= 1 - x0^2.          */
/* (log1p and expm1 evaluate ln y and 1 - exp(-2 alpha) without cancellation.) */
/* prec32 takes the decision in FP32, on L = alpha m = -ln y, multiplied       */
/* through by alpha^2: L (2 alpha - L) - (alpha u1)^2 >= 0 (last multiply-add  */
/* rounded once); x0 and |a| come from the FP64 m.                            */
/* Returns the accepting attempt (0..7) or -1; *margin as in oracle_kp_draw.   */
/* ------------------------------------------------------------------------- */
int oracle_creutz_draw(double alpha, uint64_t seed, uint32_t site, int mu, uint32_t sweep,
                       int prec32, double *a0_out, double *amag_out, double *margin)
{
    double mg = INFINITY;
    for (uint32_t t = 0; t < 8; ++t) {
        double u[4];
        draw4(seed, site, mu, PURPOSE_UPDATE, sweep, t, u);
        /* the draw itself, in FP64 */
        const double d = -expm1(-2.0 * alpha);  /* 1 - exp(-2 alpha) */
        double m = -log1p(-(1.0 - u[0]) * d) / alpha;
        double lhs, rhs;
        if (prec32) {
            /* the decision in FP32, from the FP32 roundings of its inputs */
            float af = (float)alpha;
            float df = (float)(-expm1(-2.0 * (double)af));
            float z = -(1.0f - (float)u[0]) * df;
            float lf = -(float)log1p((double)z);
            float au = af * (float)u[1];
            float tf = fmaf(lf, 2.0f * af - lf, -(au * au));
            /* accept iff tf >= 0; the margin in the units of 1 - x0^2 */
            lhs = 0.0;
            rhs = (double)tf / ((double)af * (double)af);
        } else {
            double x0 = 1.0 - m;
            lhs = u[1] * u[1];
            rhs = 1.0 - x0 * x0;
        }
        double dm = fabs(lhs - rhs);
        if (dm < mg) mg = dm;
        if (lhs <= rhs) {
            *a0_out = 1.0 - m;
            *amag_out = sqrt(m * (2.0 - m));
            if (margin) *margin = mg;
            return (int)t;
        }
    }
    if (margin) *margin = mg;
    return -1;
}

/* Uniform direction on S^2 from (u0, u1) of the direction slot
 * (Archimedes: cos(theta) uniform in [-1, 1]). */
static void direction(uint64_t seed, uint32_t site, int mu, uint32_t sweep, double n[3])
{
    double u[4];
    draw4(seed, site, mu, PURPOSE_UPDATE, sweep, SLOT_DIRECTION, u);
    double c = 2.0 * u[0] - 1.0;
    double phi = 2.0 * M_PI * u[1];
    double s = sqrt(1.0 - c * c);
    n[0] = s * cos(phi);
    n[1] = s * sin(phi);
    n[2] = c;
}

static void store(double *dst, const double q[4], int prec32)
{
    for (int c = 0; c < 4; ++c) dst[c] = prec32 ? (double)(float)q[c] : q[c];
}

/* Normalise to the unit sphere, Eq. (7) (reunitarisation), then store. */
static void store_unit(double *dst, const double q[4], int prec32)
{
    double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    double inv = 1.0 / sqrt(n2);
    double r[4] = { q[0] * inv, q[1] * inv, q[2] * inv, q[3] * inv };
    store(dst, r, prec32);
}

/* ------------------------------------------------------------------------- */
/* Lattice initialisation (Sec. 2.1 and Sec. 2.4): cold = identity on every   */
/* link; hot = a Haar-random SU(2) element per link from a predefined seed.   */
/* ------------------------------------------------------------------------- */
static void init_link(uint64_t seed, int start, int prec32, long lex, int mu, double out[4])
{
    double q[4] = { 1.0, 0.0, 0.0, 0.0 };
    if (start == 1) {
        double u[4];
        draw4(seed, (uint32_t)lex, mu, PURPOSE_HOT, 0u, 0u, u);
        haar_from_uniforms(u, q);
    }
    store(out, q, prec32);
}

int oracle_init(const int dims[4], uint64_t seed, int start, int prec32, double *U)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    if (start != 0 && start != 1) return -1;
#pragma omp parallel for schedule(static)
    for (long lex = 0; lex < g.V; ++lex)
        for (int mu = 0; mu < 4; ++mu) init_link(seed, start, prec32, lex, mu, U + (lex * 4 + mu) * 4);
    return 0;
}

/* The links oracle_init would write at the listed sites: out[(i*4 + mu)*4 ..]
 * for sites[i], mu = 0..3 (no lattice of V sites is formed). */
int oracle_init_sites(const int dims[4], uint64_t seed, int start, int prec32, const int64_t *sites,
                      long n, double *out)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    if (start != 0 && start != 1) return -1;
    for (long i = 0; i < n; ++i)
        if (sites[i] < 0 || sites[i] >= g.V) return -1;
    for (long i = 0; i < n; ++i)
        for (int mu = 0; mu < 4; ++mu) init_link(seed, start, prec32, (long)sites[i], mu, out + (i * 4 + mu) * 4);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* One link update U_mu(x), written to out[4] (U itself is not modified):     */
/*   w = staple sum; alpha = beta |w|;                                        */
/*   alpha == 0: the conditional is Haar, draw it (slot 9);                   */
/*   else KP for x0 (Creutz's draw when alpha < creutz_below); after 8        */
/*   failures the link is kept;                                               */
/*   X = (x0, |a| n), V = w/|w|, U' = X V, normalised (Eqs. (5)-(7)).         */
/* *tries = attempt that accepted (0..7), 8 after a cap failure, 9 for the    */
/* Haar branch; *margin = the smallest margin of the decisions taken (the     */
/* accept tests and, with the switch on, |alpha - creutz_below|).             */
/* diag (nullable) receives |w| and the accepted x0 (NaN when no draw was     */
/* accepted): the two numbers that set how strongly rounding in the staple    */
/* and in the draw can move the new link.                                     */
/* ------------------------------------------------------------------------- */
static void update_one(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int mu,
                       int prec32, double creutz_below, const double *U, long lex, double out[4],
                       int *tries, double *margin, double diag[2])
{
    double w[4];
    oracle_staple(dims, U, lex, mu, w);
    double k = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    double alpha = beta * k;
    if (diag) { diag[0] = k; diag[1] = NAN; }
    if (alpha == 0.0) {
        double u[4], q[4];
        draw4(seed, (uint32_t)lex, mu, PURPOSE_UPDATE, sweep, SLOT_HAAR, u);
        haar_from_uniforms(u, q);
        store_unit(out, q, prec32);
        *tries = 9;
        *margin = INFINITY;
        return;
    }
    double a0, amag;
    const int creutz = prec32 ? (float)alpha < (float)creutz_below : alpha < creutz_below;
    int t = creutz ? oracle_creutz_draw(alpha, seed, (uint32_t)lex, mu, sweep, prec32, &a0, &amag, margin)
                   : oracle_kp_draw(alpha, seed, (uint32_t)lex, mu, sweep, prec32, &a0, &amag, margin);
    if (creutz_below > 0.0 && fabs(alpha - creutz_below) < *margin) *margin = fabs(alpha - creutz_below);
    if (t < 0) {
        memcpy(out, link(U, lex, mu), 4 * sizeof(double));
        *tries = 8;
        return;
    }
    *tries = t;
    if (diag) diag[1] = a0;
    double n[3];
    direction(seed, (uint32_t)lex, mu, sweep, n);
    double X[4] = { a0, amag * n[0], amag * n[1], amag * n[2] };
    double V[4] = { w[0] / k, w[1] / k, w[2] / k, w[3] / k };
    double Un[4];
    oracle_qmul(X, V, Un);
    store_unit(out, Un, prec32);
}

/* One heat-bath pass: every link U_mu(x) with parity(x) == parity, in place.
 * Per-site outputs (optional, indexed by lex): tries[lex], margin[lex] and
 * diag[2 lex .. 2 lex + 1] as in update_one.  stats[0] += KP attempts
 * evaluated, stats[1] += cap failures. */
int oracle_pass(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int parity,
                int mu, int prec32, double creutz_below, double *U, int8_t *tries, double *margin,
                double *diag, uint64_t stats[2])
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    if (parity < 0 || parity > 1 || mu < 0 || mu > 3 || !(beta >= 0.0) || !(creutz_below >= 0.0))
        return -1;
    uint64_t attempts = 0, failures = 0;
#pragma omp parallel for schedule(static) reduction(+ : attempts, failures)
    for (long lex = 0; lex < g.V; ++lex) {
        int x[4];
        coords(&g, lex, x);
        if (((x[0] + x[1] + x[2] + x[3]) & 1) != parity) continue;
        double out[4], m;
        int t;
        update_one(dims, beta, seed, sweep, mu, prec32, creutz_below, U, lex, out, &t, &m,
                   diag ? diag + 2 * lex : NULL);
        /* the staples of this pass never read the links it writes (they are
         * U_mu at the other parity, and U_nu with nu != mu), so writing in
         * place is the same as writing to a copy */
        memcpy(U + (lex * 4 + mu) * 4, out, sizeof out);
        if (tries) tries[lex] = (int8_t)t;
        if (margin) margin[lex] = m;
        if (t <= 7) attempts += (uint64_t)t + 1;
        else if (t == 8) { attempts += 8; failures += 1; }
    }
    if (stats) { stats[0] += attempts; stats[1] += failures; }
    return 0;
}

/* The update a pass would give the listed sites (all of one parity), without
 * modifying U: out[i*4 .. i*4+3] for sites[i]; tries/margin optional. */
int oracle_update_sites(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int mu,
                        int prec32, double creutz_below, const double *U, const int64_t *sites,
                        long n, double *out, int8_t *tries, double *margin)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    if (mu < 0 || mu > 3 || !(beta >= 0.0) || !(creutz_below >= 0.0)) return -1;
    for (long i = 0; i < n; ++i)
        if (sites[i] < 0 || sites[i] >= g.V) return -1;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double m;
        int t;
        update_one(dims, beta, seed, sweep, mu, prec32, creutz_below, U, (long)sites[i], out + 4 * i,
                   &t, &m, NULL);
        if (tries) tries[i] = (int8_t)t;
        if (margin) margin[i] = m;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Learned-proposal variant: an independence-Metropolis step for x0.          */
/* The proposal q(x0 | alpha) puts probability 1/32 on each of 32 segments    */
/* between knots y_0 = -1 < ... < y_32 = 1 and, inside segment j, density     */
/* proportional to exp(alpha x0): with w_j = y_{j+1} - y_j and                */
/* E_j = exp(alpha w_j) - 1, q(x) = alpha exp(alpha (x - y_j)) / (32 E_j),     */
/* drawn as x = y_j + ln(1 + v E_j) / alpha for v uniform on [0, 1).  The     */
/* knots at alpha come from `table` (G rows of 33 knots at alpha_g = g *      */
/* alpha_max / (G - 1)) by linear interpolation in alpha.  One Philox call    */
/* (purpose 2, slot 0): u0 -> segment j = floor(32 u0) and v = 32 u0 - j,     */
/* u1 -> accept, (u2, u3) -> direction.                                        */
/* The target for x0 is pi(x) ~ sqrt(1 - x^2) exp(alpha x) (the same local     */
/* conditional the heat-bath samples); the step accepts with probability      */
/* min(1, [pi(x') / q(x')] / [pi(x) / q(x)]), x = dot(U_old, V), so it leaves */
/* that conditional invariant.  On rejection x0 keeps its value and the      */
/* direction is drawn afresh (a Gibbs step on the uniform direction).         */
/* alpha = 0 takes the Haar draw and alpha above alpha_max the capped         */
/* Kennedy-Pendleton draw, as in the plain pass.                              */
/* ------------------------------------------------------------------------- */
static void knots_at(const double *table, int G, double alpha_max, double alpha, double y[33])
{
    double t = alpha / (alpha_max / (double)(G - 1));
    int g0 = (int)floor(t);
    if (g0 > G - 2) g0 = G - 2;
    if (g0 < 0) g0 = 0;
    double f = t - (double)g0;
    for (int j = 0; j < 33; ++j)
        y[j] = (1.0 - f) * table[g0 * 33 + j] + f * table[(g0 + 1) * 33 + j];
}

static int segment_of(const double y[33], double x)
{
    int j = 0;
    while (j < 31 && x >= y[j + 1]) ++j;
    return j;
}

/* *res: 10 = proposal accepted, 11 = rejected (x0 kept, direction redrawn), or the plain-pass
 * codes (0..9) when the plain heat-bath handled the update. */
static void update_one_imh(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int mu,
                           int prec32, const double *U, long lex, const double *table, int G,
                           double alpha_max, double out[4], int *res, double *margin)
{
    double w[4];
    oracle_staple(dims, U, lex, mu, w);
    double k = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    double alpha = beta * k;
    if (alpha == 0.0 || alpha > alpha_max) {
        update_one(dims, beta, seed, sweep, mu, prec32, 0.0, U, lex, out, res, margin, NULL);
        return;
    }
    double y[33];
    knots_at(table, G, alpha_max, alpha, y);
    double u[4];
    draw4(seed, (uint32_t)lex, mu, PURPOSE_IMH, sweep, 0u, u);
    int jp = (int)floor(32.0 * u[0]);
    if (jp > 31) jp = 31;
    double v = 32.0 * u[0] - (double)jp;
    double Ep = expm1(alpha * (y[jp + 1] - y[jp]));
    double xp = y[jp] + log1p(v * Ep) / alpha;
    double V[4] = { w[0] / k, w[1] / k, w[2] / k, w[3] / k };
    const double *uo = link(U, lex, mu);
    double xc = uo[0] * V[0] + uo[1] * V[1] + uo[2] * V[2] + uo[3] * V[3];
    if (xc > 1.0) xc = 1.0;
    if (xc < -1.0) xc = -1.0;
    int jc = segment_of(y, xc);
    double Ec = expm1(alpha * (y[jc + 1] - y[jc]));
    /* log of the acceptance ratio: pi(x) / q(x) = 32 sqrt(1 - x^2)        */
    /* exp(alpha y_j) E_j / alpha on segment j, so                         */
    /* r = sqrt((1 - x'^2) / (1 - x^2)) exp(alpha (y_jp - y_jc)) E_jp / E_jc */
    double lr_terms[3];
    double num = 1.0 - xp * xp, den = 1.0 - xc * xc;
    /* a proposal on a segment of zero (or, from rounding, negative) width is
     * an atom of q: reject it; a current value on such a segment, or where
     * pi vanishes, accepts any proposal */
    double wp = y[jp + 1] - y[jp], wc = y[jc + 1] - y[jc];
    int accept_always = 0, reject_always = 0;
    if (num <= 0.0 || !(wp > 0.0)) reject_always = 1;
    else if (den <= 0.0 || !(wc > 0.0)) accept_always = 1;
    lr_terms[0] = (num > 0.0 && den > 0.0) ? 0.5 * log(num / den) : 0.0;
    lr_terms[1] = alpha * (y[jp] - y[jc]);
    lr_terms[2] = (Ep > 0.0 && Ec > 0.0) ? log(Ep / Ec) : 0.0;
    int acc;
    double m;
    if (reject_always) { acc = 0; m = INFINITY; }
    else if (accept_always) { acc = 1; m = INFINITY; }
    else if (prec32) {
        float lr = (float)lr_terms[0] + (float)lr_terms[1] + (float)lr_terms[2];
        float lu = (float)log(u[1]);
        acc = lu <= lr;
        m = fabs((double)lu - (double)lr);
    } else {
        double lr = lr_terms[0] + lr_terms[1] + lr_terms[2];
        double lu = log(u[1]);
        acc = lu <= lr;
        m = fabs(lu - lr);
    }
    *margin = m;
    /* accepted: x0 = x'; rejected: x0 stays x (the current value) and the  */
    /* direction about V is drawn afresh from (u2, u3) all the same -- the  */
    /* conditional of the direction given x0 is uniform, so this Gibbs step */
    /* keeps the target invariant                                           */
    double x0 = acc ? xp : xc;
    double c = 2.0 * u[2] - 1.0, phi = 2.0 * M_PI * u[3];
    double sn = sqrt(1.0 - c * c), am = sqrt(fmax(0.0, 1.0 - x0 * x0));
    double X[4] = { x0, am * sn * cos(phi), am * sn * sin(phi), am * c };
    double Un[4];
    oracle_qmul(X, V, Un);
    store_unit(out, Un, prec32);
    *res = acc ? 10 : 11;
}

/* One pass with the learned proposal; stats[0] += independence-Metropolis
 * proposals, stats[1] += accepted ones (updates outside the table's alpha
 * range go to the plain heat-bath and are not counted). */
int oracle_pass_imh(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int parity,
                    int mu, int prec32, double *U, const double *table, int G, double alpha_max,
                    int8_t *res_out, double *margin, uint64_t stats[2])
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    if (parity < 0 || parity > 1 || mu < 0 || mu > 3 || !(beta >= 0.0) || G < 2 ||
        !(alpha_max > 0.0))
        return -1;
    uint64_t prop = 0, acc = 0;
#pragma omp parallel for schedule(static) reduction(+ : prop, acc)
    for (long lex = 0; lex < g.V; ++lex) {
        int x[4];
        coords(&g, lex, x);
        if (((x[0] + x[1] + x[2] + x[3]) & 1) != parity) continue;
        double out[4], m = NAN;
        int r;
        update_one_imh(dims, beta, seed, sweep, mu, prec32, U, lex, table, G, alpha_max, out, &r, &m);
        memcpy(U + (lex * 4 + mu) * 4, out, sizeof out);
        if (res_out) res_out[lex] = (int8_t)r;
        if (margin) margin[lex] = m;
        if (r >= 10) prop += 1;
        if (r == 10) acc += 1;
    }
    if (stats) { stats[0] += prop; stats[1] += acc; }
    return 0;
}

/* A sweep with the learned proposal (same pass order as oracle_sweep). */
int oracle_sweep_imh(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int prec32,
                     double *U, const double *table, int G, double alpha_max, uint64_t stats[2])
{
    for (int parity = 1; parity >= 0; --parity)
        for (int mu = 0; mu < 4; ++mu)
            if (oracle_pass_imh(dims, beta, seed, sweep, parity, mu, prec32, U, table, G,
                                alpha_max, NULL, NULL, stats))
                return -1;
    return 0;
}

/* One sweep (Sec. 2.4): odd sites for mu = 0..3, then even sites for
 * mu = 0..3; the Philox sweep index is `sweep` for all eight passes. */
int oracle_sweep(const int dims[4], double beta, uint64_t seed, uint32_t sweep, int prec32,
                 double creutz_below, double *U, uint64_t stats[2])
{
    for (int parity = 1; parity >= 0; --parity)
        for (int mu = 0; mu < 4; ++mu)
            if (oracle_pass(dims, beta, seed, sweep, parity, mu, prec32, creutz_below, U, NULL, NULL,
                            NULL, stats))
                return -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Overrelaxation (Sec. 2.4 names "heat-bath with overrelaxation" without a    */
/* formula; this is the standard SU(2) reflection, Adler 1981, Creutz 1987,   */
/* Brown & Woch 1987).  With the staple sum w of the link, k = |w| and        */
/* V = w/k, the local weight exp(beta dot(U, w)) depends on U only through     */
/* dot(U, V) = (1/2)Re Tr(U V^dag); the move U -> V U^dag V keeps it, maps     */
/* the Haar measure onto itself and undoes itself, so it leaves the local      */
/* conditional invariant without a random number.  A link with w == 0 is      */
/* kept.  The result is normalised (Eq. (7)) and stored like a heat-bath link.  */
/* knorm (nullable) receives |w| per updated site, indexed by lex.             */
/* ------------------------------------------------------------------------- */
int oracle_or_pass(const int dims[4], int parity, int mu, int prec32, double *U, double *knorm)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    if (parity < 0 || parity > 1 || mu < 0 || mu > 3) return -1;
#pragma omp parallel for schedule(static)
    for (long lex = 0; lex < g.V; ++lex) {
        int x[4];
        coords(&g, lex, x);
        if (((x[0] + x[1] + x[2] + x[3]) & 1) != parity) continue;
        double w[4];
        oracle_staple(dims, U, lex, mu, w);
        double k = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
        if (knorm) knorm[lex] = k;
        if (k == 0.0) continue;
        double V[4] = { w[0] / k, w[1] / k, w[2] / k, w[3] / k };
        double ud[4], t[4], Un[4];
        qdag(link(U, lex, mu), ud);
        oracle_qmul(V, ud, t);
        oracle_qmul(t, V, Un);
        /* as in oracle_pass, the pass never reads the links it writes */
        store_unit(U + (lex * 4 + mu) * 4, Un, prec32);
    }
    return 0;
}

/* One overrelaxation sweep, in the heat-bath sweep's pass order. */
int oracle_or_sweep(const int dims[4], int prec32, double *U)
{
    for (int parity = 1; parity >= 0; --parity)
        for (int mu = 0; mu < 4; ++mu)
            if (oracle_or_pass(dims, parity, mu, prec32, U, NULL)) return -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Plaquette, Eq. (3): U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag; its     */
/* (1/2)Tr is the scalar component.  Sec. 2.4 keeps spatial and temporal      */
/* averages apart, in double precision.                                       */
/* out[0] = (Ps + Pt)/2, out[1] = Ps (planes 01, 02, 12), out[2] = Pt (planes */
/* 03, 13, 23); each a mean over sites and its three planes.                  */
/* ------------------------------------------------------------------------- */
int oracle_plaquette(const int dims[4], const double *U, double out[3])
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    double ss = 0.0, st = 0.0;
    for (long lex = 0; lex < g.V; ++lex) {
        int x[4];
        coords(&g, lex, x);
        for (int mu = 0; mu < 4; ++mu) {
            for (int nu = mu + 1; nu < 4; ++nu) {
                long xpm = shifted(&g, x, mu, +1), xpn = shifted(&g, x, nu, +1);
                double a[4], b[4], d1[4], d2[4], c[4];
                oracle_qmul(link(U, lex, mu), link(U, xpm, nu), a);
                qdag(link(U, xpn, mu), d1);
                oracle_qmul(a, d1, b);
                qdag(link(U, lex, nu), d2);
                oracle_qmul(b, d2, c);
                if (nu == 3) st += c[0]; else ss += c[0];
            }
        }
    }
    double ps = ss / (3.0 * (double)g.V), pt = st / (3.0 * (double)g.V);
    out[0] = 0.5 * (ps + pt);
    out[1] = ps;
    out[2] = pt;
    return 0;
}

/* Polyakov loop: mean over spatial sites of (1/2)Tr of the ordered product of
 * the time-direction links U_3(x, t), t = 0 .. L3-1. */
int oracle_polyakov(const int dims[4], const double *U, double *out)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    long Vs = (long)g.L[0] * g.L[1] * g.L[2];
    double sum = 0.0;
    for (long xs = 0; xs < Vs; ++xs) {
        double P[4] = { 1.0, 0.0, 0.0, 0.0 };
        for (int t = 0; t < g.L[3]; ++t) {
            double r[4];
            oracle_qmul(P, link(U, xs + Vs * t, 3), r);
            memcpy(P, r, sizeof P);
        }
        sum += P[0];
    }
    *out = sum / (double)Vs;
    return 0;
}

/* The Polyakov loop at every spatial site: out[xs] = (1/2)Tr of the ordered
 * product of U_3(xs, t), t = 0 .. L3-1, xs = x0 + L0 (x1 + L1 x2). */
int oracle_polyakov_field(const int dims[4], const double *U, double *out)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    long Vs = (long)g.L[0] * g.L[1] * g.L[2];
    for (long xs = 0; xs < Vs; ++xs) {
        double P[4] = { 1.0, 0.0, 0.0, 0.0 };
        for (int t = 0; t < g.L[3]; ++t) {
            double r[4];
            oracle_qmul(P, link(U, xs + Vs * t, 3), r);
            memcpy(P, r, sizeof P);
        }
        out[xs] = P[0];
    }
    return 0;
}

/* Sum over all links of dot(U_mu(x), W_mu(x)) = (1/2)Tr(U W^dag); equals
 * 4 * 6V * plaquette on any configuration (each plaquette has four links). */
int oracle_staple_action(const int dims[4], const double *U, double *out)
{
    geom_t g;
    if (geom_init(&g, dims)) return -1;
    double s = 0.0;
    for (long lex = 0; lex < g.V; ++lex)
        for (int mu = 0; mu < 4; ++mu) {
            double w[4];
            oracle_staple(dims, U, lex, mu, w);
            const double *u = link(U, lex, mu);
            s += u[0] * w[0] + u[1] * w[1] + u[2] * w[2] + u[3] * w[3];
        }
    *out = s;
    return 0;
}

/* Threads the OpenMP loops of this file use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
