/*
 * su3_oracle.c -- plain FP64 CPU reference for the SU(3) pure-gauge heat bath
 * by Cabibbo-Marinari SU(2) subgroups.
 *
 * TEST INFRASTRUCTURE ONLY: compiled and called by the tests, the smoke check
 * and the benchmark's CPU-baseline leg, never by the product path.  It shares
 * no code with the GPU library.  Written for clarity, not speed.
 *
 * The paper's heat bath is for SU(2) (Sec. 2: links a0 + i a.sigma, staple sum
 * V, k = sqrt(det V), a0 drawn from sqrt(1 - a0^2) exp(beta k a0), new link
 * X V~^{-1}).  SU(3) reuses it on SU(2) subgroups (Cabibbo & Marinari 1982):
 *   weight of U_mu(s)      exp[(beta/3) Re Tr(U A)], A the sum of six staples
 *   subgroup (i, j)        U -> R U, R = 1 except the rows/columns i, j, which
 *                          hold r in SU(2)
 *   reduction to SU(2)     with W = U A and w its (i, j) block,
 *                          Re Tr(R W) = Re Tr(r w) + const, and Re Tr(r w)
 *                          only sees the quaternion part of w: writing
 *                          w = M(a) + i M(c) with M(a) = a0 + i a.sigma,
 *                          a0 = Re(w_ii + w_jj)/2, a1 = Im(w_ij + w_ji)/2,
 *                          a2 = Re(w_ij - w_ji)/2, a3 = Im(w_ii - w_jj)/2,
 *                          Re Tr(r w) = 2 |a| (r v)_0 with v = a/|a|.
 *   SU(2) step             so r v is drawn exactly as the SU(2) heat bath with
 *                          beta -> 2 beta / 3 and staple a; r = X v^+ (the
 *                          SU(2) oracle's orc_heatbath_link_w2 does exactly this).
 * Readings (the method fixes none of them; the GPU library takes the same):
 *   - subgroup order (0,1), (1,2), (0,2), one heat-bath draw each per update;
 *   - Philox tag 7 + g for subgroup g, so that the three draws are independent;
 *   - hot start: rows 0 and 1 from Gram-Schmidt of complex Gaussian vectors
 *     (Box-Muller on three Philox blocks, tag 10), row 2 = conj(row0 x row1),
 *     which is Haar on SU(3) because the map commutes with right
 *     multiplication by SU(3);
 *   - reunitarisation: Gram-Schmidt of rows 0 and 1, row 2 as above.
 */
#include "su3_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "su2_oracle.h"

typedef double complex cplx;

static const int SUBGROUP[3][2] = {{0, 1}, {1, 2}, {0, 2}};

/* ------------------------------------------------------------- 3x3 algebra */
static void m3_mul(const cplx *a, const cplx *b, cplx *c) /* c = a b, no aliasing */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx t = 0.0;
            for (int k = 0; k < 3; ++k) t += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = t;
        }
}

static void m3_adj(const cplx *a, cplx *c) /* c = a^+, no aliasing */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[3 * i + j] = conj(a[3 * j + i]);
}

static double m3_retr(const cplx *a) { return creal(a[0] + a[4] + a[8]); }

static const cplx *clink(const double *U, int64_t s, int mu)
{
    return (const cplx *)(U + ((size_t)s * 4 + (size_t)mu) * 18);
}

static cplx *mlink(double *U, int64_t s, int mu)
{
    return (cplx *)(U + ((size_t)s * 4 + (size_t)mu) * 18);
}

/* row 2 = conj(row0 x row1) */
static void third_row(cplx *m)
{
    const cplx *a = m, *b = m + 3;
    m[6] = conj(a[1] * b[2] - a[2] * b[1]);
    m[7] = conj(a[2] * b[0] - a[0] * b[2]);
    m[8] = conj(a[0] * b[1] - a[1] * b[0]);
}

/* rows 0, 1 orthonormalised (Gram-Schmidt), row 2 completed */
static void gram_schmidt(cplx *m)
{
    double n0 = 0.0;
    for (int c = 0; c < 3; ++c) n0 += creal(m[c] * conj(m[c]));
    n0 = sqrt(n0);
    for (int c = 0; c < 3; ++c) m[c] /= n0;
    cplx p = 0.0; /* <row0, row1> = sum conj(row0) row1 */
    for (int c = 0; c < 3; ++c) p += conj(m[c]) * m[3 + c];
    for (int c = 0; c < 3; ++c) m[3 + c] -= p * m[c];
    double n1 = 0.0;
    for (int c = 0; c < 3; ++c) n1 += creal(m[3 + c] * conj(m[3 + c]));
    n1 = sqrt(n1);
    for (int c = 0; c < 3; ++c) m[3 + c] /= n1;
    third_row(m);
}

/* Haar SU(3) from three Philox blocks at (site, 0, w2, draw 0..2). */
static void haar3(uint64_t seed, uint32_t site, uint32_t w2, cplx *m)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double g[12];
    for (uint32_t d = 0; d < 3; ++d) {
        uint32_t ctr[4] = {site, 0u, w2, d}, w[4];
        orc_philox4x32_10(ctr, key, w);
        double u[4];
        for (int i = 0; i < 4; ++i) u[i] = orc_uniform(w[i]);
        double r01 = sqrt(-2.0 * log(u[0])), r23 = sqrt(-2.0 * log(u[2]));
        g[4 * d + 0] = r01 * cos(2.0 * M_PI * u[1]);
        g[4 * d + 1] = r01 * sin(2.0 * M_PI * u[1]);
        g[4 * d + 2] = r23 * cos(2.0 * M_PI * u[3]);
        g[4 * d + 3] = r23 * sin(2.0 * M_PI * u[3]);
    }
    for (int c = 0; c < 6; ++c) m[c] = g[2 * c] + I * g[2 * c + 1];
    gram_schmidt(m);
}

static uint32_t word2(uint32_t mu, uint32_t tag, uint32_t replica)
{
    return mu | (tag << 2) | (replica << 6);
}

/* ----------------------------------------------------------------- staples */
/* The staple sum with the links supplied by `get` (a stored lattice, or the
 * hot start computed link by link). */
typedef void (*link3_fn)(const void *ctx, int64_t s, int mu, cplx out[9]);

static void staple_with(const int32_t dims[4], link3_fn get, const void *ctx, int64_t s, int mu,
                        cplx A[9])
{
    for (int e = 0; e < 9; ++e) A[e] = 0.0;
    int64_t sp = orc_shift(dims, s, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int64_t snp = orc_shift(dims, s, nu, +1);
        int64_t snm = orc_shift(dims, s, nu, -1);
        int64_t spnm = orc_shift(dims, sp, nu, -1);
        cplx l[9], d1[9], d2[9], t[9], st[9];
        /* forward: U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+ */
        get(ctx, snp, mu, l);
        m3_adj(l, d1);
        get(ctx, sp, nu, l);
        m3_mul(l, d1, t);
        get(ctx, s, nu, l);
        m3_adj(l, d2);
        m3_mul(t, d2, st);
        for (int e = 0; e < 9; ++e) A[e] += st[e];
        /* backward: U_nu(s+mu-nu)^+ U_mu(s-nu)^+ U_nu(s-nu) */
        get(ctx, spnm, nu, l);
        m3_adj(l, d1);
        get(ctx, snm, mu, l);
        m3_adj(l, d2);
        m3_mul(d1, d2, t);
        get(ctx, snm, nu, l);
        m3_mul(t, l, st);
        for (int e = 0; e < 9; ++e) A[e] += st[e];
    }
}

static void stored_link3(const void *ctx, int64_t s, int mu, cplx out[9])
{
    memcpy(out, clink((const double *)ctx, s, mu), 9 * sizeof(cplx));
}

void orc3_staple(const int32_t dims[4], const double *U, int64_t s, int mu, double *Aout)
{
    staple_with(dims, stored_link3, U, s, mu, (cplx *)Aout);
}

/* ---------------------------------------------------------- link update */
void orc3_heatbath_link(const double *Uin, const double *Ain, double beta, uint64_t seed,
                        uint32_t site, uint32_t sweep, uint32_t mu, uint32_t replica,
                        double *out, double *margin)
{
    cplx U[9], A[9];
    memcpy(U, Uin, sizeof(U));
    memcpy(A, Ain, sizeof(A));
    double mmin = INFINITY;
    for (int g = 0; g < 3; ++g) {
        const int i = SUBGROUP[g][0], j = SUBGROUP[g][1];
        cplx W[9];
        m3_mul(U, A, W);
        const cplx wii = W[3 * i + i], wij = W[3 * i + j], wji = W[3 * j + i], wjj = W[3 * j + j];
        double a[4] = {0.5 * creal(wii + wjj), 0.5 * cimag(wij + wji), 0.5 * creal(wij - wji),
                       0.5 * cimag(wii - wjj)};
        double r[4], m;
        orc_heatbath_link_w2(a, 2.0 * beta / 3.0, seed, site, sweep,
                             word2(mu, ORC_TAG_SU3_SUB + (uint32_t)g, replica), r, &m);
        if (m < mmin) mmin = m;
        /* M(r) = [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]] acting on rows i, j */
        const cplx r00 = r[0] + I * r[3], r01 = r[2] + I * r[1];
        const cplx r10 = -r[2] + I * r[1], r11 = r[0] - I * r[3];
        for (int c = 0; c < 3; ++c) {
            const cplx ui = U[3 * i + c], uj = U[3 * j + c];
            U[3 * i + c] = r00 * ui + r01 * uj;
            U[3 * j + c] = r10 * ui + r11 * uj;
        }
    }
    memcpy(out, U, sizeof(U));
    if (margin) *margin = mmin;
}

/* Microcanonical over-relaxation of a link (Brown & Woch, Phys. Rev. Lett. 58
 * (1987) 2394; Creutz, Phys. Rev. D 36 (1987) 515) in the same subgroups and
 * order: with v = a/|a| the subgroup element r = (v^+)^2 reflects the link
 * about the direction the staple prefers, so Re Tr(R W) = Re Tr(W) (the
 * action is unchanged) and applying it twice gives the identity.  |a| = 0
 * leaves the link alone.  No randoms. */
void orc3_overrelax_link(const double *Uin, const double *Ain, double *out)
{
    cplx U[9], A[9];
    memcpy(U, Uin, sizeof(U));
    memcpy(A, Ain, sizeof(A));
    for (int g = 0; g < 3; ++g) {
        const int i = SUBGROUP[g][0], j = SUBGROUP[g][1];
        cplx W[9];
        m3_mul(U, A, W);
        const cplx wii = W[3 * i + i], wij = W[3 * i + j], wji = W[3 * j + i], wjj = W[3 * j + j];
        double a[4] = {0.5 * creal(wii + wjj), 0.5 * cimag(wij + wji), 0.5 * creal(wij - wji),
                       0.5 * cimag(wii - wjj)};
        double k = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
        if (!(k > 0.0)) continue;
        double vd[4] = {a[0] / k, -a[1] / k, -a[2] / k, -a[3] / k}, r[4];
        orc_qmul(vd, vd, r);
        const cplx r00 = r[0] + I * r[3], r01 = r[2] + I * r[1];
        const cplx r10 = -r[2] + I * r[1], r11 = r[0] - I * r[3];
        for (int c = 0; c < 3; ++c) {
            const cplx ui = U[3 * i + c], uj = U[3 * j + c];
            U[3 * i + c] = r00 * ui + r01 * uj;
            U[3 * j + c] = r10 * ui + r11 * uj;
        }
    }
    memcpy(out, U, sizeof(U));
}

void orc3_or_pass(const int32_t dims[4], double *U, int mu, int parity, int nthreads)
{
    int64_t V = orc_volume(dims);
#ifdef _OPENMP
    if (nthreads > 1) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static) if (nthreads > 1)
    for (int64_t s = 0; s < V; ++s) {
        if (orc_parity(dims, s) != parity) continue;
        double A[18];
        orc3_staple(dims, U, s, mu, A);
        orc3_overrelax_link((const double *)clink(U, s, mu), A, (double *)mlink(U, s, mu));
    }
}

/* ------------------------------------------------------------------ passes */
static void update_site(const int32_t dims[4], double *U, int64_t s, int mu, uint32_t sweep,
                        double beta, uint64_t seed, uint32_t replica, double *margin)
{
    double A[18], m;
    orc3_staple(dims, U, s, mu, A);
    orc3_heatbath_link((const double *)clink(U, s, mu), A, beta, seed, (uint32_t)s, sweep,
                       (uint32_t)mu, replica, (double *)mlink(U, s, mu), &m);
    if (margin) margin[s] = m;
}

void orc3_pass(const int32_t dims[4], double *U, int mu, int parity, uint32_t sweep,
               double beta, uint64_t seed, uint32_t replica, int nthreads, double *margin)
{
    int64_t V = orc_volume(dims);
    if (nthreads > 1) {
#ifdef _OPENMP
        omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < V; ++s)
            if (orc_parity(dims, s) == parity)
                update_site(dims, U, s, mu, sweep, beta, seed, replica, margin);
        return;
    }
    for (int64_t s = 0; s < V; ++s)
        if (orc_parity(dims, s) == parity)
            update_site(dims, U, s, mu, sweep, beta, seed, replica, margin);
}

void orc3_sweeps(const int32_t dims[4], double *U, int32_t nsweeps, uint32_t sweep0,
                 double beta, uint64_t seed, uint32_t replica, int32_t reunit_every,
                 int nthreads, double *plaq_hist, double *poly_hist)
{
    orc3_sweeps_or(dims, U, nsweeps, 0, sweep0, beta, seed, replica, reunit_every, nthreads,
                   plaq_hist, poly_hist);
}

void orc3_sweeps_or(const int32_t dims[4], double *U, int32_t nsweeps, int32_t n_or,
                    uint32_t sweep0, double beta, uint64_t seed, uint32_t replica,
                    int32_t reunit_every, int nthreads, double *plaq_hist, double *poly_hist)
{
    for (int32_t n = 0; n < nsweeps; ++n) {
        uint32_t sw = sweep0 + (uint32_t)n;
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                orc3_pass(dims, U, mu, p, sw, beta, seed, replica, nthreads, NULL);
        for (int32_t o = 0; o < n_or; ++o)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p) orc3_or_pass(dims, U, mu, p, nthreads);
        if (reunit_every > 0 && ((sw + 1u) % (uint32_t)reunit_every) == 0u)
            orc3_reunitarize(dims, U);
        if (plaq_hist) plaq_hist[n] = orc3_plaquette(dims, U);
        if (poly_hist) {
            double re, im, mag;
            orc3_polyakov(dims, U, &re, &im, &mag);
            poly_hist[n] = re;
        }
    }
}

/* ------------------------------------------------------------ init / misc */
void orc3_hot_link(int64_t s, int mu, uint64_t seed, uint32_t replica, double *out)
{
    haar3(seed, (uint32_t)s, word2((uint32_t)mu, ORC_TAG_SU3_HOT, replica), (cplx *)out);
}

void orc3_init(const int32_t dims[4], double *U, int start, uint64_t seed, uint32_t replica)
{
    int64_t V = orc_volume(dims);
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            cplx *m = mlink(U, s, mu);
            if (start == 0) {
                for (int e = 0; e < 9; ++e) m[e] = (e % 4 == 0) ? 1.0 : 0.0;
            } else {
                orc3_hot_link(s, mu, seed, replica, (double *)m);
            }
        }
}

struct hot_key3 {
    uint64_t seed;
    uint32_t replica;
};

static void hot_link3_of(const void *ctx, int64_t s, int mu, cplx out[9])
{
    const struct hot_key3 *k = (const struct hot_key3 *)ctx;
    orc3_hot_link(s, mu, k->seed, k->replica, (double *)out);
}

void orc3_hot_staple(const int32_t dims[4], int64_t s, int mu, uint64_t seed, uint32_t replica,
                     double *A)
{
    struct hot_key3 k = {seed, replica};
    staple_with(dims, hot_link3_of, &k, s, mu, (cplx *)A);
}

void orc3_reunitarize(const int32_t dims[4], double *U)
{
    int64_t n = orc_volume(dims) * 4;
    for (int64_t l = 0; l < n; ++l) gram_schmidt((cplx *)(U + 18 * l));
}

double orc3_plaquette(const int32_t dims[4], const double *U)
{
    int64_t V = orc_volume(dims);
    double sum = 0.0;
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 1; mu < 4; ++mu)
            for (int nu = 0; nu < mu; ++nu) {
                /* U_mu(s) U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+ */
                cplx t1[9], t2[9], d[9];
                m3_mul(clink(U, s, mu), clink(U, orc_shift(dims, s, mu, +1), nu), t1);
                m3_adj(clink(U, orc_shift(dims, s, nu, +1), mu), d);
                m3_mul(t1, d, t2);
                m3_adj(clink(U, s, nu), d);
                m3_mul(t2, d, t1);
                sum += m3_retr(t1) / 3.0;
            }
    return sum / (6.0 * (double)V);
}

void orc3_polyakov(const int32_t dims[4], const double *U, double *re, double *im, double *mag)
{
    int64_t VS = (int64_t)dims[0] * dims[1] * dims[2];
    double sr = 0.0, si = 0.0, sm = 0.0;
    for (int64_t x = 0; x < VS; ++x) {
        cplx L[9], t[9];
        memcpy(L, clink(U, x, 3), sizeof(L));
        for (int t_ = 1; t_ < dims[3]; ++t_) {
            m3_mul(L, clink(U, x + VS * t_, 3), t);
            memcpy(L, t, sizeof(L));
        }
        cplx tr = (L[0] + L[4] + L[8]) / 3.0;
        sr += creal(tr);
        si += cimag(tr);
        sm += cabs(tr);
    }
    *re = sr / (double)VS;
    *im = si / (double)VS;
    *mag = sm / (double)VS;
}

double orc3_staple_action(const int32_t dims[4], const double *U)
{
    int64_t V = orc_volume(dims);
    double sum = 0.0;
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            cplx A[9], t[9];
            orc3_staple(dims, U, s, mu, (double *)A);
            m3_mul(clink(U, s, mu), A, t);
            sum += m3_retr(t);
        }
    return sum;
}

void orc3_gauge_transform(const int32_t dims[4], double *U, uint64_t seed, uint32_t replica)
{
    int64_t V = orc_volume(dims);
    cplx *G = (cplx *)malloc(sizeof(cplx) * 9 * (size_t)V);
    for (int64_t s = 0; s < V; ++s)
        haar3(seed, (uint32_t)s, word2(0u, ORC_TAG_GAUGE, replica), G + 9 * s);
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            cplx t[9], d[9], r[9];
            m3_mul(G + 9 * s, clink(U, s, mu), t);
            m3_adj(G + 9 * orc_shift(dims, s, mu, +1), d);
            m3_mul(t, d, r);
            memcpy(mlink(U, s, mu), r, sizeof(r));
        }
    free(G);
}

void orc3_link_chain(const double *A, double beta, int64_t nsteps, uint64_t seed, double *U,
                     double *obs)
{
    for (int64_t t = 0; t < nsteps; ++t) {
        orc3_heatbath_link(U, A, beta, seed, 0u, (uint32_t)t, 0u, 0u, U, NULL);
        cplx W[9];
        m3_mul((const cplx *)U, (const cplx *)A, W);
        const cplx *u = (const cplx *)U;
        const cplx tw = W[0] + W[4] + W[8], tu = u[0] + u[4] + u[8];
        obs[4 * t] = creal(tw);
        obs[4 * t + 1] = cimag(tw);
        obs[4 * t + 2] = creal(tu);
        obs[4 * t + 3] = cimag(tu);
    }
}
