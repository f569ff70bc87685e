/*
 * su3_oracle.h -- plain FP64 CPU reference for the SU(3) pure-gauge heat bath
 * built from SU(2) subgroups (Cabibbo & Marinari, Phys. Lett. B 119 (1982) 387).
 *
 * TEST INFRASTRUCTURE ONLY.  Compiled and called only by the test suite, the
 * smoke check and the CPU baseline of the benchmark; the product path never
 * links or calls it, and it shares no source with the GPU library.  It reuses
 * the SU(2) oracle's Philox, a0 sampler and quaternion heat-bath step
 * (su2_oracle.h), which is the point of the construction: the SU(2) heat bath of
 * Sec. 2 of Cardoso & Bicudo, "Lattice SU(2) on GPU's", applied to the three
 * SU(2) subgroups of SU(3).
 *
 * Conventions (identical to the GPU library, restated here independently):
 *   site    s = x + Nx*(y + Ny*(z + Nz*t)), directions mu = 0:x 1:y 2:z 3:t,
 *           parity (x+y+z+t) & 1, every extent even and >= 2
 *   links   U[((s*4 + mu)*9 + 3*a + b)*2 + {0: re, 1: im}], row a, column b
 *   action  S = beta sum_p (1 - Re Tr U_p / 3)
 *   randoms Philox4x32-10, key = seed, counter = (site, sweep,
 *           mu | tag<<2 | replica<<6, draw); subgroup g (rows (0,1), (1,2),
 *           (0,2) for g = 0, 1, 2) draws with tag 7 + g, the hot start with tag 10
 */
#ifndef SU3_ORACLE_H
#define SU3_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sum of the six staples around U_mu(s): A (9 complex) such that the action's
 * dependence on U_mu(s) is -(beta/3) Re Tr(U_mu(s) A). */
void orc3_staple(const int32_t dims[4], const double *U, int64_t s, int mu, double *A);

/* One Cabibbo-Marinari update of a link U (9 complex, in place allowed via
 * out == U) with staple sum A: subgroups 0, 1, 2 in that order, each an SU(2)
 * heat-bath draw.  margin (may be NULL): smallest |decision margin| of the three
 * a0 samplers. */
void orc3_heatbath_link(const double *U, const double *A, double beta, uint64_t seed,
                        uint32_t site, uint32_t sweep, uint32_t mu, uint32_t replica,
                        double *out, double *margin);

/* One checkerboard pass (direction mu, sites of the given parity); nthreads > 1
 * runs the sites in parallel (they are independent within a pass).  margin
 * (length V, may be NULL) receives each updated site's smallest margin. */
void orc3_pass(const int32_t dims[4], double *U, int mu, int parity, uint32_t sweep,
               double beta, uint64_t seed, uint32_t replica, int nthreads, double *margin);

/* nsweeps sweeps (mu 0..3, even then odd sites) from sweep index sweep0;
 * reunit_every > 0 reunitarises after every sweep whose 1-based index is a
 * multiple of it.  plaq_hist / poly_hist (may be NULL): after every sweep, the
 * plaquette and the real part of the Polyakov loop. */
void orc3_sweeps(const int32_t dims[4], double *U, int32_t nsweeps, uint32_t sweep0,
                 double beta, uint64_t seed, uint32_t replica, int32_t reunit_every,
                 int nthreads, double *plaq_hist, double *poly_hist);

/* Microcanonical over-relaxation of one link with staple sum A (the subgroups
 * and order of the heat bath; r = (v^+)^2 with v = a/|a|): Re Tr(U A) is
 * unchanged and the map is its own inverse.  No randoms. */
void orc3_overrelax_link(const double *U, const double *A, double *out);
/* One over-relaxation pass (direction mu, sites of the given parity). */
void orc3_or_pass(const int32_t dims[4], double *U, int mu, int parity, int nthreads);
/* As orc3_sweeps, each heat-bath sweep followed by n_or over-relaxation sweeps
 * (eight passes each, same schedule) before the reunitarisation and the
 * measurements; the sweep index counts heat-bath sweeps only. */
void orc3_sweeps_or(const int32_t dims[4], double *U, int32_t nsweeps, int32_t n_or,
                    uint32_t sweep0, double beta, uint64_t seed, uint32_t replica,
                    int32_t reunit_every, int nthreads, double *plaq_hist, double *poly_hist);

/* start 0: every link 1; start 1: Haar-random links (Gram-Schmidt of two
 * complex Gaussian rows, third row the conjugate cross product). */
void orc3_init(const int32_t dims[4], double *U, int start, uint64_t seed, uint32_t replica);

/* U_mu(s) of the hot start (the orc3_init recipe), computed on its own, and the
 * staple sum of the hot-start configuration at (s, mu) without building the
 * lattice: for lattices too large to hold in FP64 on the host. */
void orc3_hot_link(int64_t s, int mu, uint64_t seed, uint32_t replica, double *out);
void orc3_hot_staple(const int32_t dims[4], int64_t s, int mu, uint64_t seed, uint32_t replica,
                     double *A);

/* Gram-Schmidt of rows 0 and 1, row 2 = conj(row0 x row1), for every link. */
void orc3_reunitarize(const int32_t dims[4], double *U);

/* <Re Tr U_p / 3> over the 6V plaquettes. */
double orc3_plaquette(const int32_t dims[4], const double *U);

/* Mean over spatial sites of Tr L / 3, L the ordered product of U_3 along t:
 * real and imaginary parts, and the mean of |Tr L / 3|. */
void orc3_polyakov(const int32_t dims[4], const double *U, double *re, double *im, double *mag);

/* sum over s, mu of Re Tr(U_mu(s) A_mu(s)) (each plaquette counted 4 times). */
double orc3_staple_action(const int32_t dims[4], const double *U);

/* U_mu(s) -> G(s) U_mu(s) G(s+mu)^+ with Haar G (tag 3 of the SU(2) oracle, mu 0). */
void orc3_gauge_transform(const int32_t dims[4], double *U, uint64_t seed, uint32_t replica);

/* Markov chain of one link with a fixed staple A: nsteps updates, step t using
 * sweep index t (site 0, mu 0); obs[4 t .. 4 t + 3] = Re Tr(U A), Im Tr(U A),
 * Re Tr U, Im Tr U after step t.  U (9 complex) is the start and receives the end state. */
void orc3_link_chain(const double *A, double beta, int64_t nsteps, uint64_t seed, double *U,
                     double *obs);

#ifdef __cplusplus
}
#endif

#endif
