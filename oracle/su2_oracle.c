/*
 * su2_oracle.c -- plain FP64 CPU reference for the pure-gauge SU(2) heat bath.
 *
 * TEST INFRASTRUCTURE ONLY: compiled and called by the tests, the smoke check
 * and the benchmark's CPU-baseline leg, never by the product path.  It shares
 * no code with the GPU library.  Written for clarity, not speed: every step is
 * the definition from the paper, in FP64, in the paper's order.
 *
 * Paper: Cardoso & Bicudo, "Lattice SU(2) on GPU's" (LAT2010).
 *   Sec. 2, SU(2) parametrisation   U = a0 + i a.sigma, a0^2 + |a|^2 = 1
 *   Sec. 2, heat-bath weight        dP(U) ~ exp[(beta/2) Tr(U V)], V = six staples
 *   Sec. 2, normalisation           U~ = V / sqrt(det V) = V / k
 *   Sec. 2, a0 distribution         P(a0) ~ sqrt(1 - a0^2) exp(beta k a0)
 *   Sec. 2, new link                U' = X U~^{-1}  (X the sampled element)
 *   Sec. 4 / Fig. 3 caption         per direction: even sites, then odd sites
 *   Sec. 4, kernel list             cold/hot start, plaquette, Polyakov loop, sums
 *
 * Readings where the paper is silent (the same readings the GPU library takes):
 *   - a0 sampler: Kennedy-Pendleton for alpha = beta k >= 1; below that the
 *     exact rejection from the Haar (semicircle) marginal with acceptance
 *     exp(alpha (a0 - 1)); both capped at SAMPLER_TRIAL_CAP trials (the cap is
 *     unreachable in practice: acceptance is >= 0.41 for every alpha).
 *   - direction of a: uniform on the sphere, |a| = sqrt(delta (2 - delta)),
 *     its two uniforms taken from the unused low 9 bits of the words of the
 *     first trial's block (18-bit uniforms).
 *   - randoms: Philox4x32-10 keyed by the seed, counter (site, sweep,
 *     mu | tag<<2 | replica<<6, draw), words mapped to (2*(w>>9)+1) 2^-24.
 */
#include "su2_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SAMPLER_TRIAL_CAP 1000
#define KP_MIN_ALPHA 1.0

/* ------------------------------------------------------------------ Philox */
/* Salmon et al., "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
 * Philox4x32 with multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments
 * 0x9E3779B9, 0xBB67AE85; ten rounds, key bumped between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_batch(int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

double orc_uniform(uint32_t w)
{
    return (2.0 * (double)(w >> 9) + 1.0) * ldexp(1.0, -24);
}

double orc_uniform18(uint32_t m)
{
    return (2.0 * (double)(m & 0x3FFFFu) + 1.0) * ldexp(1.0, -19);
}

static void block(uint64_t seed, uint32_t site, uint32_t sweep, uint32_t word2,
                  uint32_t draw, double u[4], uint32_t w_out[4])
{
    uint32_t ctr[4] = {site, sweep, word2, draw};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    for (int i = 0; i < 4; ++i) {
        if (u) u[i] = orc_uniform(w[i]);
        if (w_out) w_out[i] = w[i];
    }
}

static uint32_t word2_of(uint32_t mu, uint32_t tag, uint32_t replica)
{
    return mu | (tag << 2) | (replica << 6);
}

/* -------------------------------------------------------------- quaternions */
/* (a0 + i a.s)(b0 + i b.s) = (a0 b0 - a.b) + i (a0 b + b0 a - a x b).s */
void orc_qmul(const double a[4], const double b[4], double c[4])
{
    double r0 = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    double r1 = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    double r2 = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    double r3 = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
    c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}

void orc_qdag(const double a[4], double c[4])
{
    c[0] = a[0]; c[1] = -a[1]; c[2] = -a[2]; c[3] = -a[3];
}

void orc_qmul_batch(int64_t n, const double *a, const double *b, double *c)
{
    for (int64_t i = 0; i < n; ++i) orc_qmul(a + 4 * i, b + 4 * i, c + 4 * i);
}

static double qnorm(const double a[4])
{
    return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
}

/* ----------------------------------------------------------------- lattice */
int orc_check_dims(const int32_t dims[4])
{
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || (dims[i] & 1)) return -1;
    return 0;
}

int64_t orc_volume(const int32_t dims[4])
{
    return (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
}

static void coords(const int32_t dims[4], int64_t s, int c[4])
{
    for (int i = 0; i < 4; ++i) {
        c[i] = (int)(s % dims[i]);
        s /= dims[i];
    }
}

static int64_t site_of(const int32_t dims[4], const int c[4])
{
    return c[0] + (int64_t)dims[0] * (c[1] + (int64_t)dims[1] * (c[2] + (int64_t)dims[2] * c[3]));
}

int orc_parity(const int32_t dims[4], int64_t s)
{
    int c[4];
    coords(dims, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

int64_t orc_shift(const int32_t dims[4], int64_t s, int mu, int step)
{
    int c[4];
    coords(dims, s, c);
    c[mu] = ((c[mu] + step) % dims[mu] + dims[mu]) % dims[mu];
    return site_of(dims, c);
}

static const double *link(const double *U, int64_t s, int mu)
{
    return U + (s * 4 + mu) * 4;
}

/* Six staples around U_mu(s) (Sec. 2), oriented so that (1/2) Tr(U_mu(s) V)
 * is the sum of the six plaquettes containing U_mu(s):
 *   forward  U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+
 *   backward U_nu(s+mu-nu)^+ U_mu(s-nu)^+ U_nu(s-nu)                        */
/* The staple sum with the links supplied by `get` (a stored lattice, or the
 * hot start computed link by link). */
typedef void (*link_fn)(const void *ctx, int64_t s, int mu, double out[4]);

static void staple_with(const int32_t dims[4], link_fn get, const void *ctx, int64_t s, int mu,
                        double V[4])
{
    V[0] = V[1] = V[2] = V[3] = 0.0;
    int64_t s_pmu = orc_shift(dims, s, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int64_t s_pnu = orc_shift(dims, s, nu, +1);
        int64_t s_mnu = orc_shift(dims, s, nu, -1);
        int64_t s_pmu_mnu = orc_shift(dims, s_pmu, nu, -1);
        double a[4], b[4], t[4], f[4], l[4];

        get(ctx, s_pnu, mu, l);
        orc_qdag(l, b);
        get(ctx, s_pmu, nu, l);
        orc_qmul(l, b, t);
        get(ctx, s, nu, l);
        orc_qdag(l, a);
        orc_qmul(t, a, f);
        for (int c = 0; c < 4; ++c) V[c] += f[c];

        get(ctx, s_pmu_mnu, nu, l);
        orc_qdag(l, a);
        get(ctx, s_mnu, mu, l);
        orc_qdag(l, b);
        orc_qmul(a, b, t);
        get(ctx, s_mnu, nu, l);
        orc_qmul(t, l, f);
        for (int c = 0; c < 4; ++c) V[c] += f[c];
    }
}

static void stored_link(const void *ctx, int64_t s, int mu, double out[4])
{
    memcpy(out, link((const double *)ctx, s, mu), 4 * sizeof(double));
}

void orc_staple(const int32_t dims[4], const double *U, int64_t s, int mu, double V[4])
{
    staple_with(dims, stored_link, U, s, mu, V);
}

/* ----------------------------------------------------------------- sampler */
/* Draw a0 with density ~ sqrt(1 - a0^2) exp(alpha a0) on [-1, 1] (Sec. 2) and
 * return delta = 1 - a0.
 *   alpha >= 1: Kennedy-Pendleton.  With uniforms r1..r4 of trial t,
 *     delta = -(ln r1 + cos^2(2 pi r2) ln r3) / alpha is Gamma(3/2, alpha)
 *     distributed; accepting when r4^2 <= 1 - delta/2 supplies the missing
 *     factor sqrt(1 - delta/2) of sqrt(delta (2 - delta)).
 *   alpha < 1: a0 = sqrt(r1) cos(2 pi r2) is the first coordinate of a
 *     uniform point in the unit disc, i.e. the Haar marginal
 *     (2/pi) sqrt(1 - a0^2); accept when r3 <= exp(alpha (a0 - 1)).      */
double orc_sample_delta(double alpha, uint64_t seed, uint32_t site, uint32_t sweep,
                        uint32_t mu, uint32_t replica, int32_t *ntrials, double *margin)
{
    return orc_sample_delta_w2(alpha, seed, site, sweep, word2_of(mu, ORC_TAG_TRIAL, replica),
                               ntrials, margin);
}

double orc_sample_delta_w2(double alpha, uint64_t seed, uint32_t site, uint32_t sweep,
                           uint32_t w2, int32_t *ntrials, double *margin)
{
    double min_margin = fabs(alpha - KP_MIN_ALPHA);
    double delta = 0.0;
    int accepted = 0;
    int t;
    for (t = 0; t < SAMPLER_TRIAL_CAP; ++t) {
        double r[4];
        block(seed, site, sweep, w2, (uint32_t)t, r, NULL);
        double m;
        if (alpha >= KP_MIN_ALPHA) {
            double c = cos(2.0 * M_PI * r[1]);
            delta = -(log(r[0]) + c * c * log(r[2])) / alpha;
            m = (1.0 - 0.5 * delta) - r[3] * r[3];
        } else {
            double a0 = sqrt(r[0]) * cos(2.0 * M_PI * r[1]);
            delta = 1.0 - a0;
            m = exp(alpha * (a0 - 1.0)) - r[2];
        }
        if (fabs(m) < min_margin) min_margin = fabs(m);
        if (m >= 0.0) {
            accepted = 1;
            break;
        }
    }
    if (!accepted) delta = 0.0; /* unreachable in practice; fixed, documented value */
    if (ntrials) *ntrials = accepted ? t + 1 : SAMPLER_TRIAL_CAP;
    if (margin) *margin = min_margin;
    return delta;
}

void orc_sample_delta_batch(int64_t n, const double *alpha, uint64_t seed,
                            const uint32_t *site, uint32_t sweep, uint32_t mu,
                            uint32_t replica, double *delta, int32_t *ntrials,
                            double *margin)
{
    for (int64_t i = 0; i < n; ++i)
        delta[i] = orc_sample_delta(alpha[i], seed, site[i], sweep, mu, replica,
                                    ntrials ? ntrials + i : NULL, margin ? margin + i : NULL);
}

/* X = (1 - delta, |a| n) with n uniform on the 2-sphere from (r5, r6):
 * cos(theta) = 1 - 2 r5, sin(theta) = 2 sqrt(r5 (1 - r5)), phi = 2 pi r6,
 * |a| = sqrt(delta (2 - delta)) = sqrt(1 - a0^2). */
static void element_from_delta(double delta, const double rdir[2], double X[4])
{
    double amag = sqrt(delta * (2.0 - delta));
    double cth = 1.0 - 2.0 * rdir[0];
    double sth = 2.0 * sqrt(rdir[0] * (1.0 - rdir[0]));
    double phi = 2.0 * M_PI * rdir[1];
    X[0] = 1.0 - delta;
    X[1] = amag * sth * cos(phi);
    X[2] = amag * sth * sin(phi);
    X[3] = amag * cth;
}

void orc_heatbath_link(const double V[4], double beta, uint64_t seed, uint32_t site,
                       uint32_t sweep, uint32_t mu, uint32_t replica, double out[4],
                       double *margin)
{
    orc_heatbath_link_w2(V, beta, seed, site, sweep, word2_of(mu, ORC_TAG_TRIAL, replica), out,
                         margin);
}

void orc_heatbath_link_w2(const double V[4], double beta, uint64_t seed, uint32_t site,
                          uint32_t sweep, uint32_t w2, double out[4], double *margin)
{
    /* k = sqrt(det V); for a quaternion sum det V = |V|^2 (Sec. 2). */
    double k = qnorm(V);
    double Ut[4] = {1.0, 0.0, 0.0, 0.0};
    if (k > 0.0)
        for (int c = 0; c < 4; ++c) Ut[c] = V[c] / k;
    double alpha = beta * k;
    double delta = orc_sample_delta_w2(alpha, seed, site, sweep, w2, NULL, margin);
    /* Direction uniforms: the 9 low bits of each word of the first trial's
     * block are not used by the a0 uniforms (which take bits 9..31); they give
     * two independent 18-bit uniforms (2m+1) 2^-19. */
    uint32_t w[4];
    block(seed, site, sweep, w2, 0u, NULL, w);
    double rd[2];
    rd[0] = orc_uniform18((w[0] & 511u) | ((w[1] & 511u) << 9));
    rd[1] = orc_uniform18((w[2] & 511u) | ((w[3] & 511u) << 9));
    double X[4], Utd[4];
    element_from_delta(delta, rd, X);
    /* U' = X U~^{-1} = X U~^+ */
    orc_qdag(Ut, Utd);
    orc_qmul(X, Utd, out);
}

/* ------------------------------------------------------------------ passes */
static void update_site(const int32_t dims[4], double *U, int64_t s, int mu, uint32_t sweep,
                        double beta, uint64_t seed, uint32_t replica, double *margin)
{
    double V[4], out[4], m;
    orc_staple(dims, U, s, mu, V);
    orc_heatbath_link(V, beta, seed, (uint32_t)s, sweep, (uint32_t)mu, replica, out, &m);
    memcpy(U + (s * 4 + mu) * 4, out, sizeof(out));
    if (margin) margin[s] = m;
}

static uint64_t splitmix(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_pass(const int32_t dims[4], double *U, int mu, int parity, uint32_t sweep,
              double beta, uint64_t seed, uint32_t replica, int order, uint64_t order_seed,
              double *margin)
{
    int64_t V = orc_volume(dims);
    if (order == 3) {
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < V; ++s)
            if (orc_parity(dims, s) == parity)
                update_site(dims, U, s, mu, sweep, beta, seed, replica, margin);
        return;
    }
    int64_t *sites = (int64_t *)malloc(sizeof(int64_t) * (size_t)V);
    int64_t n = 0;
    for (int64_t s = 0; s < V; ++s)
        if (orc_parity(dims, s) == parity) sites[n++] = s;
    if (order == 1) {
        for (int64_t i = 0; i < n / 2; ++i) {
            int64_t tmp = sites[i];
            sites[i] = sites[n - 1 - i];
            sites[n - 1 - i] = tmp;
        }
    } else if (order == 2) {
        uint64_t st = order_seed;
        for (int64_t i = n - 1; i > 0; --i) {
            int64_t j = (int64_t)(splitmix(&st) % (uint64_t)(i + 1));
            int64_t tmp = sites[i];
            sites[i] = sites[j];
            sites[j] = tmp;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        update_site(dims, U, sites[i], mu, sweep, beta, seed, replica, margin);
    free(sites);
}

void orc_sweeps(const int32_t dims[4], double *U, int32_t nsweeps, uint32_t sweep0,
                double beta, uint64_t seed, uint32_t replica, int32_t reunit_every,
                int nthreads, double *plaq_hist, double *poly_hist, double *margin)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int order = nthreads > 1 ? 3 : 0;
    const int64_t Vol = orc_volume(dims);
    double *pm = NULL;
    if (margin) {
        pm = (double *)malloc(sizeof(double) * (size_t)Vol);
        if (!pm) abort();
    }
    for (int32_t i = 0; i < nsweeps; ++i) {
        uint32_t sw = sweep0 + (uint32_t)i;
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p) {
                if (pm)
                    for (int64_t s = 0; s < Vol; ++s) pm[s] = INFINITY;
                orc_pass(dims, U, mu, p, sw, beta, seed, replica, order, 0, pm);
                if (pm)
                    for (int64_t s = 0; s < Vol; ++s)
                        if (pm[s] < margin[s * 4 + mu]) margin[s * 4 + mu] = pm[s];
            }
        if (reunit_every > 0 && ((sw + 1u) % (uint32_t)reunit_every) == 0u)
            orc_reunitarize(dims, U);
        if (plaq_hist) plaq_hist[i] = orc_plaquette(dims, U);
        if (poly_hist) {
            double ls, la;
            orc_polyakov(dims, U, &ls, &la);
            poly_hist[i] = ls;
        }
    }
    free(pm);
}

/* ------------------------------------------------------- over-relaxation */
void orc_overrelax_link(const double V[4], const double U[4], double out[4])
{
    double k = qnorm(V);
    if (!(k > 0.0)) {
        memcpy(out, U, 4 * sizeof(double));
        return;
    }
    double Utd[4] = {V[0] / k, -V[1] / k, -V[2] / k, -V[3] / k}; /* U~^+ */
    double Ud[4], T[4];
    orc_qdag(U, Ud);
    orc_qmul(Utd, Ud, T);
    orc_qmul(T, Utd, out);
}

void orc_or_pass(const int32_t dims[4], double *U, int mu, int parity)
{
    const int64_t Vol = orc_volume(dims);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < Vol; ++s) {
        if (orc_parity(dims, s) != parity) continue;
        double V[4], out[4];
        orc_staple(dims, U, s, mu, V);
        orc_overrelax_link(V, U + (s * 4 + mu) * 4, out);
        memcpy(U + (s * 4 + mu) * 4, out, sizeof(out));
    }
}

void orc_sweeps_or(const int32_t dims[4], double *U, int32_t nsweeps, int32_t n_or,
                   uint32_t sweep0, double beta, uint64_t seed, uint32_t replica,
                   int32_t reunit_every, int nthreads, double *plaq_hist, double *poly_hist)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int order = nthreads > 1 ? 3 : 0;
    for (int32_t i = 0; i < nsweeps; ++i) {
        uint32_t sw = sweep0 + (uint32_t)i;
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                orc_pass(dims, U, mu, p, sw, beta, seed, replica, order, 0, NULL);
        for (int32_t k = 0; k < n_or; ++k)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p) orc_or_pass(dims, U, mu, p);
        if (reunit_every > 0 && ((sw + 1u) % (uint32_t)reunit_every) == 0u)
            orc_reunitarize(dims, U);
        if (plaq_hist) plaq_hist[i] = orc_plaquette(dims, U);
        if (poly_hist) {
            double ls, la;
            orc_polyakov(dims, U, &ls, &la);
            poly_hist[i] = ls;
        }
    }
}

/* ------------------------------------------------------------ init / misc */
void orc_haar_from_block(const uint32_t w[4], double out[4])
{
    double u[4];
    for (int i = 0; i < 4; ++i) u[i] = orc_uniform(w[i]);
    double r01 = sqrt(-2.0 * log(u[0]));
    double r23 = sqrt(-2.0 * log(u[2]));
    double g[4] = {r01 * cos(2.0 * M_PI * u[1]), r01 * sin(2.0 * M_PI * u[1]),
                   r23 * cos(2.0 * M_PI * u[3]), r23 * sin(2.0 * M_PI * u[3])};
    double n = qnorm(g);
    for (int i = 0; i < 4; ++i) out[i] = g[i] / n;
}

void orc_hot_link(int64_t s, int mu, uint64_t seed, uint32_t replica, double out[4])
{
    uint32_t w[4];
    block(seed, (uint32_t)s, 0u, word2_of((uint32_t)mu, ORC_TAG_HOT, replica), 0u, NULL, w);
    orc_haar_from_block(w, out);
}

void orc_init(const int32_t dims[4], double *U, int start, uint64_t seed, uint32_t replica)
{
    int64_t V = orc_volume(dims);
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            double *l = U + (s * 4 + mu) * 4;
            if (start == 0) {
                l[0] = 1.0; l[1] = l[2] = l[3] = 0.0;
            } else {
                orc_hot_link(s, mu, seed, replica, l);
            }
        }
}

struct hot_key {
    uint64_t seed;
    uint32_t replica;
};

static void hot_link_of(const void *ctx, int64_t s, int mu, double out[4])
{
    const struct hot_key *k = (const struct hot_key *)ctx;
    orc_hot_link(s, mu, k->seed, k->replica, out);
}

void orc_hot_staple(const int32_t dims[4], int64_t s, int mu, uint64_t seed, uint32_t replica,
                    double V[4])
{
    struct hot_key k = {seed, replica};
    staple_with(dims, hot_link_of, &k, s, mu, V);
}

void orc_reunitarize(const int32_t dims[4], double *U)
{
    int64_t n = orc_volume(dims) * 4;
    for (int64_t i = 0; i < n; ++i) {
        double *l = U + 4 * i;
        double nn = qnorm(l);
        for (int c = 0; c < 4; ++c) l[c] /= nn;
    }
}

/* Mean plaquette: (1/6V) sum_s sum_{mu<nu} (1/2) Tr U_mu(s) U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+ */
double orc_plaquette(const int32_t dims[4], const double *U)
{
    int64_t V = orc_volume(dims);
    double sum = 0.0;
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                double a[4], b[4], t1[4], t2[4], t3[4];
                orc_qmul(link(U, s, mu), link(U, orc_shift(dims, s, mu, 1), nu), t1);
                orc_qdag(link(U, orc_shift(dims, s, nu, 1), mu), a);
                orc_qmul(t1, a, t2);
                orc_qdag(link(U, s, nu), b);
                orc_qmul(t2, b, t3);
                sum += t3[0];
            }
    return sum / (6.0 * (double)V);
}

double orc_staple_action(const int32_t dims[4], const double *U)
{
    int64_t V = orc_volume(dims);
    double sum = 0.0;
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            double St[4], t[4];
            orc_staple(dims, U, s, mu, St);
            orc_qmul(link(U, s, mu), St, t);
            sum += t[0];
        }
    return sum;
}

/* L(x) = (1/2) Tr prod_{t=0}^{Nt-1} U_3(x, t), t = 0 leftmost; mean over x. */
/* Rectangular Wilson loops: W(R, T) = (1/(12 V)) sum_s sum_{mu != nu}
 * (1/2) Tr[ L_mu(s, R) L_nu(s + R mu, T) L_mu(s + T nu, R)^+ L_nu(s, T)^+ ],
 * L_mu(s, n) = U_mu(s) U_mu(s + mu) ... U_mu(s + (n - 1) mu), for
 * R = 1..rmax, T = 1..tmax; out[(R - 1) tmax + (T - 1)].  The loop is built
 * link by link around the rectangle (no line products are reused). */
void orc_wilson_loops(const int32_t dims[4], const double *U, int rmax, int tmax, double *out)
{
    const int64_t V = orc_volume(dims);
    for (int i = 0; i < rmax * tmax; ++i) out[i] = 0.0;
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                if (nu == mu) continue;
                for (int R = 1; R <= rmax; ++R)
                    for (int T = 1; T <= tmax; ++T) {
                        double W[4] = {1.0, 0.0, 0.0, 0.0}, t[4], d[4];
                        int64_t x = s;
                        for (int i = 0; i < R; ++i) { /* forward along mu */
                            orc_qmul(W, link(U, x, mu), t);
                            memcpy(W, t, sizeof(t));
                            x = orc_shift(dims, x, mu, 1);
                        }
                        for (int i = 0; i < T; ++i) { /* forward along nu */
                            orc_qmul(W, link(U, x, nu), t);
                            memcpy(W, t, sizeof(t));
                            x = orc_shift(dims, x, nu, 1);
                        }
                        for (int i = 0; i < R; ++i) { /* back along mu */
                            x = orc_shift(dims, x, mu, -1);
                            orc_qdag(link(U, x, mu), d);
                            orc_qmul(W, d, t);
                            memcpy(W, t, sizeof(t));
                        }
                        for (int i = 0; i < T; ++i) { /* back along nu */
                            x = orc_shift(dims, x, nu, -1);
                            orc_qdag(link(U, x, nu), d);
                            orc_qmul(W, d, t);
                            memcpy(W, t, sizeof(t));
                        }
                        out[(R - 1) * tmax + (T - 1)] += W[0];
                    }
            }
    for (int i = 0; i < rmax * tmax; ++i) out[i] /= 12.0 * (double)V;
}

void orc_polyakov(const int32_t dims[4], const double *U, double *mean_signed, double *abs_mean)
{
    int64_t Ns3 = (int64_t)dims[0] * dims[1] * dims[2];
    double sum = 0.0;
    for (int64_t xs = 0; xs < Ns3; ++xs) {
        double P[4] = {1.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < dims[3]; ++t) {
            double tmp[4];
            orc_qmul(P, link(U, xs + Ns3 * t, 3), tmp);
            memcpy(P, tmp, sizeof(P));
        }
        sum += P[0];
    }
    double m = sum / (double)Ns3;
    if (mean_signed) *mean_signed = m;
    if (abs_mean) *abs_mean = fabs(m);
}

/* U_mu(s) -> G(s) U_mu(s) G(s+mu)^+ with G Haar from Philox tag 3. */
void orc_gauge_transform(const int32_t dims[4], double *U, uint64_t seed, uint32_t replica)
{
    int64_t V = orc_volume(dims);
    double *G = (double *)malloc(sizeof(double) * 4 * (size_t)V);
    for (int64_t s = 0; s < V; ++s) {
        uint32_t w[4];
        block(seed, (uint32_t)s, 0u, word2_of(0u, ORC_TAG_GAUGE, replica), 0u, NULL, w);
        orc_haar_from_block(w, G + 4 * s);
    }
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            double *l = U + (s * 4 + mu) * 4;
            double gd[4], t[4];
            orc_qdag(G + 4 * orc_shift(dims, s, mu, 1), gd);
            orc_qmul(G + 4 * s, l, t);
            orc_qmul(t, gd, l);
        }
    free(G);
}

/* ======================================================= learned proposal */
/* The proposal for a0 is a monotone rational-quadratic spline flow (Durkan,
 * Bekasov, Murray, Papamakarios 2019) whose 47 parameters come from a small
 * MLP of alpha; the Metropolis step with weight w(x) = exp(alpha x)
 * sqrt(1 - x^2) / q(x) keeps the heat-bath distribution of Sec. 2 exact. */
#define NN_MIN_BIN 1e-3
#define NN_MIN_DERIV 1e-3

double orc_nn_feature(double alpha)
{
    return 2.0 * (log(alpha) - log(ORC_NN_ALPHA_LO)) / (log(ORC_NN_ALPHA_HI) - log(ORC_NN_ALPHA_LO)) -
           1.0;
}

void orc_nn_forward(const float *prm, double f, double out[ORC_NN_OUT])
{
    const float *W1 = prm, *b1 = prm + 32, *W2 = prm + 64, *b2 = prm + 64 + 1024;
    const float *W3 = prm + 64 + 1024 + 32, *b3 = W3 + 47 * 32;
    double h1[ORC_NN_H], h2[ORC_NN_H];
    for (int i = 0; i < ORC_NN_H; ++i) h1[i] = tanh((double)W1[i] * f + (double)b1[i]);
    for (int i = 0; i < ORC_NN_H; ++i) {
        double a = b2[i];
        for (int j = 0; j < ORC_NN_H; ++j) a += (double)W2[i * ORC_NN_H + j] * h1[j];
        h2[i] = tanh(a);
    }
    for (int i = 0; i < ORC_NN_OUT; ++i) {
        double a = b3[i];
        for (int j = 0; j < ORC_NN_H; ++j) a += (double)W3[i * ORC_NN_H + j] * h2[j];
        out[i] = a;
    }
}

static void knots_from_logits(const double *logit, double *k)
{
    double mx = logit[0], sum = 0.0, p[ORC_NN_BINS];
    for (int i = 1; i < ORC_NN_BINS; ++i) mx = logit[i] > mx ? logit[i] : mx;
    for (int i = 0; i < ORC_NN_BINS; ++i) sum += (p[i] = exp(logit[i] - mx));
    k[0] = -1.0;
    for (int i = 0; i < ORC_NN_BINS; ++i)
        k[i + 1] = k[i] + 2.0 * (NN_MIN_BIN + (1.0 - ORC_NN_BINS * NN_MIN_BIN) * p[i] / sum);
    k[ORC_NN_BINS] = 1.0;
}

static double softplus(double t) { return t > 30.0 ? t : log1p(exp(t)); }

void orc_spline_from_raw(const double raw[ORC_NN_OUT], double x[17], double y[17], double d[17])
{
    knots_from_logits(raw, x);
    knots_from_logits(raw + ORC_NN_BINS, y);
    d[0] = d[ORC_NN_BINS] = 1.0;
    for (int k = 1; k < ORC_NN_BINS; ++k) d[k] = NN_MIN_DERIV + softplus(raw[2 * ORC_NN_BINS + k - 1]);
}

static int find_bin(const double *knots, double v)
{
    int k = 0;
    for (int i = 1; i < ORC_NN_BINS; ++i)
        if (v >= knots[i]) k = i;
    return k;
}

/* In bin k, with xi = (x - x_k)/W, s = H/W:
 *   g  = y_k + H [s xi^2 + d_k xi (1-xi)] / [s + (d_{k+1} + d_k - 2s) xi (1-xi)]
 *   g' = s^2 [d_{k+1} xi^2 + 2 s xi (1-xi) + d_k (1-xi)^2] / [ ... ]^2        */
static double rq_eval(const double x[17], const double y[17], const double d[17], int k,
                      double xi, double *logderiv)
{
    const double W = x[k + 1] - x[k], H = y[k + 1] - y[k], s = H / W;
    const double om = xi * (1.0 - xi);
    const double den = s + (d[k + 1] + d[k] - 2.0 * s) * om;
    const double g = y[k] + H * (s * xi * xi + d[k] * om) / den;
    const double num = d[k + 1] * xi * xi + 2.0 * s * om + d[k] * (1.0 - xi) * (1.0 - xi);
    if (logderiv) *logderiv = 2.0 * log(s) + log(num) - 2.0 * log(den);
    return g;
}

double orc_spline_fwd(const double x[17], const double y[17], const double d[17], double xv,
                      double *logderiv)
{
    const int k = find_bin(x, xv);
    const double xi = (xv - x[k]) / (x[k + 1] - x[k]);
    return rq_eval(x, y, d, k, xi, logderiv);
}

/* Inverse in bin k: xi is the root in [0, 1] of a xi^2 + b xi + c = 0 with
 *   a = H (s - d_k) + (u - y_k)(d_{k+1} + d_k - 2s)
 *   b = H d_k - (u - y_k)(d_{k+1} + d_k - 2s)
 *   c = -s (u - y_k)
 * taken in the cancellation-free form xi = 2c / (-b - sqrt(b^2 - 4ac)).     */
double orc_spline_inv(const double x[17], const double y[17], const double d[17], double u,
                      double *logderiv)
{
    const int k = find_bin(y, u);
    const double W = x[k + 1] - x[k], H = y[k + 1] - y[k], s = H / W;
    const double dy = u - y[k], t = d[k + 1] + d[k] - 2.0 * s;
    const double a = H * (s - d[k]) + dy * t;
    const double b = H * d[k] - dy * t;
    const double c = -s * dy;
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) disc = 0.0;
    const double xi = 2.0 * c / (-b - sqrt(disc));
    rq_eval(x, y, d, k, xi, logderiv);
    return x[k] + xi * W;
}

void orc_nn_table(const float *params, double *table)
{
    for (int j = 0; j < ORC_NN_TABLE_ROWS; ++j) {
        const double f = -1.0 + 2.0 * j / (ORC_NN_TABLE_ROWS - 1);
        double raw[ORC_NN_OUT], x[17], y[17], d[17];
        orc_nn_forward(params, f, raw);
        orc_spline_from_raw(raw, x, y, d);
        double *row = table + (size_t)j * ORC_NN_ROW;
        for (int k = 1; k <= ORC_NN_BINS; ++k) {
            row[k - 1] = x[k];
            row[16 + k - 1] = y[k];
            row[32 + k - 1] = d[k];
        }
    }
}

int orc_table_row(double alpha, double *margin)
{
    const double p = (orc_nn_feature(alpha) + 1.0) * 0.5 * (ORC_NN_TABLE_ROWS - 1);
    int j = (int)floor(p + 0.5);
    if (j < 0) j = 0;
    if (j > ORC_NN_TABLE_ROWS - 1) j = ORC_NN_TABLE_ROWS - 1;
    if (margin) *margin = fabs((p - floor(p)) - 0.5) * 2.0 / (ORC_NN_TABLE_ROWS - 1);
    return j;
}

void orc_table_knots(const double *table, int row, double x[17], double y[17], double d[17])
{
    const double *r = table + (size_t)row * ORC_NN_ROW;
    x[0] = y[0] = -1.0;
    d[0] = 1.0;
    for (int k = 1; k <= ORC_NN_BINS; ++k) {
        x[k] = r[k - 1];
        y[k] = r[16 + k - 1];
        d[k] = r[32 + k - 1];
    }
}

/* log w(x) = alpha x + (1/2) ln(1 - x^2) - ln g'(x)  (the constant ln 1/2 of
 * q cancels in the Metropolis ratio). */
static double log_weight(double alpha, double xv, double logderiv)
{
    const double one_m_x2 = (1.0 - xv) * (1.0 + xv);
    if (!(one_m_x2 > 0.0)) return -INFINITY;
    return alpha * xv + 0.5 * log(one_m_x2) - logderiv;
}

void orc_learned_link(const double V[4], const double Uold[4], const double *table, double beta,
                      uint64_t seed, uint32_t site, uint32_t sweep, uint32_t mu, uint32_t replica,
                      double or_width, double out[4], double margin[3], int *accepted)
{
    const double k = qnorm(V);
    const double alpha = beta * k;
    /* margins: [0] Metropolis log-ratio (or the exact sampler's decisions),
     * [1] distance of the table position to the nearest rounding boundary in
     * rows, [2] distance of alpha to the ends of the table range */
    double m3[3] = {INFINITY, INFINITY,
                    fmin(fabs(alpha - ORC_NN_ALPHA_LO), fabs(alpha - ORC_NN_ALPHA_HI))};
    if (!(alpha >= ORC_NN_ALPHA_LO && alpha <= ORC_NN_ALPHA_HI)) {
        orc_heatbath_link(V, beta, seed, site, sweep, mu, replica, out, &m3[0]);
        if (margin) memcpy(margin, m3, sizeof(m3));
        if (accepted) *accepted = -1;
        return;
    }
    double Ut[4], Utd[4];
    for (int c = 0; c < 4; ++c) Ut[c] = V[c] / k;
    double mrow;
    const int row = orc_table_row(alpha, &mrow);
    m3[1] = mrow * 0.5 * (ORC_NN_TABLE_ROWS - 1);
    double x[17], y[17], d[17];
    orc_table_knots(table, row, x, y, d);
    double r[4];
    block(seed, site, sweep, word2_of(mu, ORC_TAG_LEARN, replica), 0u, r, NULL);
    double ld_new, ld_old, t[4];
    /* the old link in the frame of the staple: x_old = (U_old U~)_0 */
    orc_qmul(Uold, Ut, t);
    double xo = t[0];
    if (xo > 1.0) xo = 1.0;
    if (xo < -1.0) xo = -1.0;
    const double u_old = orc_spline_fwd(x, y, d, xo, &ld_old);
    /* proposal in the flow coordinate u = g(a0): independent and uniform, or
     * (over-relaxed) the reflection -u_old plus uniform noise of half-width
     * or_width, taken modulo 2 into [-1, 1).  Both proposal densities are
     * symmetric in (u_old, u), so the Metropolis ratio is w(a0')/w(x_old) with
     * w = p / q, q = g'/2 the flow's density of a0. */
    double u = 2.0 * r[0] - 1.0, wrap_margin = INFINITY;
    if (or_width >= 0.0) {
        u = or_width * u - u_old;
        wrap_margin = fmin(fabs(u - 1.0), fabs(u + 1.0));
        if (u >= 1.0) u -= 2.0;
        else if (u < -1.0) u += 2.0;
    }
    const double a0n = orc_spline_inv(x, y, d, u, &ld_new);
    const double lw = log_weight(alpha, a0n, ld_new) - log_weight(alpha, xo, ld_old);
    const double dm = lw - log(r[1]);
    m3[0] = fmin(fabs(dm), wrap_margin);
    if (dm > 0.0) {
        const double amag = sqrt((1.0 - a0n) * (1.0 + a0n));
        const double cth = 1.0 - 2.0 * r[2], sth = 2.0 * sqrt(r[2] * (1.0 - r[2]));
        const double phi = 2.0 * M_PI * r[3];
        const double X[4] = {a0n, amag * sth * cos(phi), amag * sth * sin(phi), amag * cth};
        orc_qdag(Ut, Utd);
        orc_qmul(X, Utd, out);
        if (accepted) *accepted = 1;
    } else {
        memcpy(out, Uold, 4 * sizeof(double));
        if (accepted) *accepted = 0;
    }
    if (margin) memcpy(margin, m3, sizeof(m3));
}

void orc_learned_pass(const int32_t dims[4], double *U, const double *table, int mu, int parity,
                      uint32_t sweep, double beta, uint64_t seed, uint32_t replica,
                      double or_width, double *margin, int32_t *accepted)
{
    const int64_t Vol = orc_volume(dims);
    for (int64_t s = 0; s < Vol; ++s) {
        if (orc_parity(dims, s) != parity) continue;
        double St[4], out[4], m[3];
        int acc;
        orc_staple(dims, U, s, mu, St);
        orc_learned_link(St, U + (s * 4 + mu) * 4, table, beta, seed, (uint32_t)s, sweep,
                         (uint32_t)mu, replica, or_width, out, m, &acc);
        memcpy(U + (s * 4 + mu) * 4, out, sizeof(out));
        if (margin) memcpy(margin + 3 * s, m, sizeof(m));
        if (accepted) accepted[s] = acc;
    }
}

/* Training data: sample i has alpha = lo (hi/lo)^u with u the first uniform of
 * block (i, 0, 0 | 5<<2, 0) (log-uniform on [lo, hi]), and a0 = 1 - delta from
 * the exact sampler with trial blocks (i, 0, 1 | 5<<2, t). */
void orc_nn_data(int64_t n, double lo, double hi, uint64_t seed, double *alpha, double *a0)
{
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        block(seed, (uint32_t)i, 0u, word2_of(0u, ORC_TAG_TRAIN, 0u), 0u, u, NULL);
        alpha[i] = lo * pow(hi / lo, u[0]);
        a0[i] = 1.0 - orc_sample_delta_w2(alpha[i], seed, (uint32_t)i, 0u,
                                          word2_of(1u, ORC_TAG_TRAIN, 0u), NULL, NULL);
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
