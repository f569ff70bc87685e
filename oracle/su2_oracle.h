/*
 * su2_oracle.h -- plain FP64 CPU reference for the pure-gauge SU(2) heat bath.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library; it is
 * compiled and called only by the test suite, the smoke check and the CPU
 * baseline of the benchmark.  The product path never links or calls it, and it
 * shares no source with the GPU library (its own Philox, its own quaternion
 * algebra, its own lattice indexing).
 *
 * Paper: N. Cardoso and P. Bicudo, "Lattice SU(2) on GPU's", LAT2010
 * (arXiv:1010.1486).  The update equations follow Sec. 2 of the paper; the
 * schedule (per direction, even sites then odd sites) follows Sec. 4 and the
 * caption of its Fig. 3.
 *
 * Conventions (identical to the GPU library, restated here independently):
 *   site    s = x + Nx*(y + Ny*(z + Nz*t)), directions mu = 0:x 1:y 2:z 3:t
 *   parity  (x+y+z+t) & 1; every extent must be even and >= 2
 *   links   U[(s*4 + mu)*4 + c], c = a0..a3 with U = a0*1 + i a.sigma
 *   randoms Philox4x32-10, key = seed, counter = (site, sweep,
 *           mu | tag<<2 | replica<<6, draw); tags: 0 a0 trials (the low 9 bits
 *           of the words of draw 0 give the direction), 1 reserved,
 *           2 hot start, 3 gauge transform, 4 learned proposal, 5 training data,
 *           6 replica beta, 7..9 SU(3) subgroup trials, 10 SU(3) hot start
 */
#ifndef SU2_ORACLE_H
#define SU2_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_TAG_TRIAL 0u
#define ORC_TAG_DIR 1u
#define ORC_TAG_HOT 2u
#define ORC_TAG_GAUGE 3u
#define ORC_TAG_LEARN 4u
#define ORC_TAG_TRAIN 5u
#define ORC_TAG_BETA 6u
#define ORC_TAG_SU3_SUB 7u /* SU(3) subgroups 0, 1, 2: tags 7, 8, 9 */
#define ORC_TAG_SU3_HOT 10u

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Batch form for tests: n counters (4 words each) -> n outputs. */
void orc_philox_batch(int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out);
/* 32-bit word -> uniform in (0,1): (2*(w>>9)+1) * 2^-24. */
double orc_uniform(uint32_t w);
/* 18-bit value m -> (2m+1) * 2^-19 (direction uniforms). */
double orc_uniform18(uint32_t m);

/* Quaternion algebra for U = a0 + i a.sigma. */
void orc_qmul(const double a[4], const double b[4], double c[4]);
void orc_qdag(const double a[4], double c[4]);
void orc_qmul_batch(int64_t n, const double *a, const double *b, double *c);

/* Lattice indexing. */
int orc_check_dims(const int32_t dims[4]);               /* 0 ok, -1 bad */
int64_t orc_volume(const int32_t dims[4]);
int orc_parity(const int32_t dims[4], int64_t s);
int64_t orc_shift(const int32_t dims[4], int64_t s, int mu, int step);

/* Sum of the six staples around U_mu(s) (Sec. 2). */
void orc_staple(const int32_t dims[4], const double *U, int64_t s, int mu, double V[4]);
/* U_mu(s) of the hot start (the orc_init recipe), computed on its own, and the
 * staple sum of the hot-start configuration at (s, mu) without building the
 * lattice: for lattices too large to hold in FP64 on the host. */
void orc_hot_link(int64_t s, int mu, uint64_t seed, uint32_t replica, double out[4]);
void orc_hot_staple(const int32_t dims[4], int64_t s, int mu, uint64_t seed, uint32_t replica,
                    double V[4]);

/* Exact a0 sampler for density ~ sqrt(1-a0^2) exp(alpha a0).  Returns
 * delta = 1 - a0; *ntrials = trials used; *margin = smallest |decision margin|
 * of every floating-point decision taken (branch choice and accept tests). */
double orc_sample_delta(double alpha, uint64_t seed, uint32_t site, uint32_t sweep,
                        uint32_t mu, uint32_t replica, int32_t *ntrials, double *margin);
double orc_sample_delta_w2(double alpha, uint64_t seed, uint32_t site, uint32_t sweep,
                           uint32_t w2, int32_t *ntrials, double *margin);
void orc_sample_delta_batch(int64_t n, const double *alpha, uint64_t seed,
                            const uint32_t *site, uint32_t sweep, uint32_t mu,
                            uint32_t replica, double *delta, int32_t *ntrials,
                            double *margin);

/* Heat-bath update of one link given its staple sum V (writes the new link). */
void orc_heatbath_link(const double V[4], double beta, uint64_t seed, uint32_t site,
                       uint32_t sweep, uint32_t mu, uint32_t replica, double out[4],
                       double *margin);
/* The same with the third Philox counter word given directly (the SU(3)
 * subgroup updates draw from their own tags). */
void orc_heatbath_link_w2(const double V[4], double beta, uint64_t seed, uint32_t site,
                          uint32_t sweep, uint32_t w2, double out[4], double *margin);

/* One checkerboard pass over every site of the given parity, direction mu.
 * order: 0 lexicographic, 1 reversed, 2 shuffled (order_seed), 3 OpenMP.
 * margin (length V, may be NULL) receives each updated site's smallest margin. */
void orc_pass(const int32_t dims[4], double *U, int mu, int parity, uint32_t sweep,
              double beta, uint64_t seed, uint32_t replica, int order, uint64_t order_seed,
              double *margin);
/* nsweeps full sweeps (mu 0..3, even then odd) starting at sweep index sweep0.
 * reunit_every > 0 reunitarises after every sweep whose 1-based count is a
 * multiple of it.  plaq_hist (may be NULL) receives the plaquette after every
 * sweep.  nthreads > 1 uses OpenMP inside each pass.  margin (length 4V,
 * [site][mu], may be NULL) receives each link's smallest accept-decision
 * margin over the call's updates of it (the caller fills it with +inf). */
void orc_sweeps(const int32_t dims[4], double *U, int32_t nsweeps, uint32_t sweep0,
                double beta, uint64_t seed, uint32_t replica, int32_t reunit_every,
                int nthreads, double *plaq_hist, double *poly_hist, double *margin);

/* Microcanonical over-relaxation of one link (not in the paper; Brown & Woch
 * 1987, Creutz 1987): with U~ = V/|V| and X = U U~, the reflection X -> X^+
 * keeps x0 = (1/2)Tr(U V)/|V|, hence the Sec. 2 weight exp[(beta/2) Tr(U V)],
 * and the Haar measure; U' = X^+ U~^+ = U~^+ U^+ U~^+.  V = 0 leaves U. */
void orc_overrelax_link(const double V[4], const double U[4], double out[4]);
/* One over-relaxation pass (direction mu, sites of the given parity). */
void orc_or_pass(const int32_t dims[4], double *U, int mu, int parity);
/* nsweeps compound sweeps: the heat-bath sweep of index sweep0 + i, then n_or
 * over-relaxation sweeps (mu 0..3, even then odd), then reunitarisation and
 * the measurements as orc_sweeps (reunit_every counts compound sweeps). */
void orc_sweeps_or(const int32_t dims[4], double *U, int32_t nsweeps, int32_t n_or,
                   uint32_t sweep0, double beta, uint64_t seed, uint32_t replica,
                   int32_t reunit_every, int nthreads, double *plaq_hist, double *poly_hist);

void orc_init(const int32_t dims[4], double *U, int start, uint64_t seed, uint32_t replica);
void orc_reunitarize(const int32_t dims[4], double *U);
double orc_plaquette(const int32_t dims[4], const double *U);
/* sum over all sites and mu of (1/2) Tr(U_mu(s) V(s,mu)). */
double orc_staple_action(const int32_t dims[4], const double *U);
void orc_polyakov(const int32_t dims[4], const double *U, double *mean_signed,
                  double *abs_mean);
void orc_gauge_transform(const int32_t dims[4], double *U, uint64_t seed, uint32_t replica);
/* Rectangular Wilson loops averaged over sites and the 12 ordered planes,
 * R = 1..rmax along mu, T = 1..tmax along nu: out[(R-1) tmax + (T-1)]. */
void orc_wilson_loops(const int32_t dims[4], const double *U, int rmax, int tmax, double *out);
/* Haar-random SU(2) element from one Philox block (Box-Muller + normalise). */
void orc_haar_from_block(const uint32_t w[4], double out[4]);

/* ===================================================== learned proposal ===
 * Conditioner: MLP 1 -> 32 -> 32 -> 47 (tanh, tanh, linear) on the feature
 * f(alpha) = 2 (ln alpha - ln 0.5) / (ln 30 - ln 0.5) - 1.  Parameters (FP32,
 * 2671): W1[32], b1[32], W2[32][32] (row = output unit), b2[32], W3[47][32],
 * b3[47].  Outputs: 16 width logits, 16 height logits, 15 derivative logits.
 * Spline: monotone rational-quadratic on [-1, 1] (Durkan et al. 2019), 16
 * bins, widths/heights 2 (m + (1 - 16 m) softmax), m = 1e-3, interior
 * derivatives 1e-3 + softplus, boundary derivatives 1.  The flow maps a0 to
 * u = g(a0), uniform on [-1, 1]; the proposal density is q(a0) = g'(a0) / 2.
 * Table: rows j = 0..255 at f_j = -1 + 2 j / 255 holding 48 floats
 * [x1..x15, 1, y1..y15, 1, d1..d15, 1]; an update uses the nearest row. */
#define ORC_NN_H 32
#define ORC_NN_OUT 47
#define ORC_NN_BINS 16
#define ORC_NN_NPARAM 2671
#define ORC_NN_TABLE_ROWS 64
#define ORC_NN_ROW 48
#define ORC_NN_ALPHA_LO 0.5
#define ORC_NN_ALPHA_HI 30.0

double orc_nn_feature(double alpha);
void orc_nn_forward(const float *params, double f, double out[ORC_NN_OUT]);
/* knots x[0..16], y[0..16], derivatives d[0..16] from the 47 raw outputs */
void orc_spline_from_raw(const double raw[ORC_NN_OUT], double x[17], double y[17], double d[17]);
/* g(x) and ln g'(x) */
double orc_spline_fwd(const double x[17], const double y[17], const double d[17], double xv,
                      double *logderiv);
/* g^{-1}(u) and ln g'(x) at that point */
double orc_spline_inv(const double x[17], const double y[17], const double d[17], double u,
                      double *logderiv);
void orc_nn_table(const float *params, double *table /* 64 x 48 */);
/* Row index used for alpha (nearest), with the margin of that choice. */
int orc_table_row(double alpha, double *margin);
void orc_table_knots(const double *table, int row, double x[17], double y[17], double d[17]);
/* Learned-proposal Metropolis update of one link (fallback: exact heat bath).
 * or_width < 0: independence proposal u = 2 r0 - 1 in the flow coordinate;
 * 0 <= or_width <= 1: over-relaxed proposal u = -g(x_old) + or_width (2 r0 - 1)
 * modulo 2 into [-1, 1) (a symmetric proposal in u; ordered over-relaxation,
 * Neal 1998, as or_width -> 0 for an exact flow).
 * accepted: 1 accepted, 0 rejected, -1 exact fallback.  margin[3]: the
 * Metropolis log-ratio margin (or the exact sampler's; with over-relaxation
 * also the distance of the unwrapped u to +-1), the table-row rounding margin
 * in rows, the distance of alpha to the table range ends. */
void orc_learned_link(const double V[4], const double Uold[4], const double *table, double beta,
                      uint64_t seed, uint32_t site, uint32_t sweep, uint32_t mu, uint32_t replica,
                      double or_width, double out[4], double margin[3], int *accepted);
/* margin: 3 per site (as above), may be NULL. */
void orc_learned_pass(const int32_t dims[4], double *U, const double *table, int mu, int parity,
                      uint32_t sweep, double beta, uint64_t seed, uint32_t replica,
                      double or_width, double *margin, int32_t *accepted);

void orc_nn_data(int64_t n, double lo, double hi, uint64_t seed, double *alpha, double *a0);

int orc_max_threads(void);

#ifdef __cplusplus
}
#endif

#endif

