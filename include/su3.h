/*
 * su3.h -- C ABI of the SU(3) pure-gauge heat bath in libsu2 (gfx950).
 *
 * Method: the SU(2) heat bath of N. Cardoso and P. Bicudo, "Lattice SU(2) on
 * GPU's", LAT2010 (arXiv:1010.1486), Sec. 2, applied to SU(3) through its SU(2)
 * subgroups (N. Cabibbo and E. Marinari, Phys. Lett. B 119 (1982) 387).  The
 * action is S = beta sum_p (1 - Re Tr U_p / 3); the weight of one link is
 * exp[(beta/3) Re Tr(U A)] with A the sum of the six staples (the same staples
 * as Sec. 2).  A link update multiplies U from the left by SU(2) matrices
 * embedded in the row pairs (0,1), (1,2), (0,2), in that order; for pair (i,j),
 * with W = U A, the quaternion part a of the (i,j) block of W plays the role of
 * the SU(2) staple: k = |a|, a0 drawn from sqrt(1 - a0^2) exp((2 beta / 3) k a0)
 * by the same sampler as the SU(2) path, subgroup element X (a/k)^+.  The
 * schedule is Sec. 4's: per direction mu, even sites, then odd sites.  Before
 * a link is stored its rows 0 and 1 are re-orthonormalised in FP32 (a no-op in
 * exact arithmetic): the rotations of the (1,2) and (0,2) subgroups mix the
 * rebuilt row 2 into the stored rows, and without it deviations from
 * unitarity would grow from update to update.
 *
 * Conventions
 *   Lattice     as su2.h: periodic Nx x Ny x Nz x Nt, every extent even and
 *               >= 2, site s = x + Nx*(y + Ny*(z + Nz*t)), mu = 0:x .. 3:t,
 *               parity (x+y+z+t) & 1, V/2 < 2^28.
 *   Links       3x3 complex, FP32 on the device, rows 0 and 1 stored (12
 *               floats) and row 2 = conj(row0 x row1) rebuilt when read.
 *               Device layout: 24 arrays of V/2 float4, array
 *               ((mu*2 + parity)*3 + c) holding float4 c of U_mu at the
 *               half-site h = s >> 1: c = 0 (Re u00, Im u00, Re u01, Im u01),
 *               c = 1 (Re u02, Im u02, Re u10, Im u10), c = 2 (Re u11, Im u11,
 *               Re u12, Im u12); 192*V bytes.  Host exchange layout (get/set):
 *               double[V][4 mu][3 row][3 col][2 re/im] in canonical site order.
 *   Randoms     Philox4x32-10, key = seed, counter = (site, sweep index,
 *               mu | tag<<2, draw): tag 7 + g for subgroup g's a0 trials (the
 *               low 9 bits of draw 0's words give the direction), tag 10 for
 *               the hot start.  Results are bit-identical for identical
 *               (links, seed, sweep index, beta), whatever the launch
 *               configuration (su3_set_launch).
 *
 * Errors: the SU2_* codes of su2.h; su2_last_error() gives the message.  Calls
 * documented as "enqueue" return after launching work on the context's stream;
 * calls returning host values synchronise it.  One context must not be used
 * from two host threads at once, and every call on it must be made with the
 * device that was current at su3_init current again.
 */
#ifndef SU3_H
#define SU3_H

#include <stddef.h>
#include <stdint.h>

#include "su2.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct su3_ctx su3_ctx;
typedef struct su3_batch su3_batch;

/* Device bytes of the link arrays of a lattice (0 for invalid dims). */
size_t su3_links_bytes(const int32_t dims[4]);

/* Create an SU(3) lattice: library-owned device memory on the current device,
 * work enqueued on hip_stream (a hipStream_t; NULL is the null stream, which
 * the caller keeps valid for the context's lifetime).  start SU2_COLD: every
 * link 1; SU2_HOT: Haar-random links (rows 0 and 1 by Gram-Schmidt of complex
 * Gaussian rows from Box-Muller on three Philox blocks).  The sweep index
 * starts at 0.  SU2_EODD / SU2_ERANGE for bad extents, SU2_EINVAL for a NULL
 * pointer, a beta that is not finite or is negative, or a bad start. */
int su3_init(su3_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
             void *hip_stream);

/* Synchronise the stream and release the context. */
int su3_destroy(su3_ctx *ctx);

/* Enqueue nsweeps (>= 0) sweeps: for mu = 0..3, a pass over the even sites,
 * then one over the odd sites, each link taking one Cabibbo-Marinari update.
 * reunit_every > 0: after every sweep whose index j satisfies
 * (j + 1) % reunit_every == 0, rows 0 and 1 of every link are
 * re-orthonormalised.  plaq_hist (host double[nsweeps] or NULL): the mean
 * plaquette after every sweep, measured inside the odd passes of mu = 1, 2, 3
 * (before that sweep's reunitarisation); with it the call synchronises.  The
 * sweep index advances by nsweeps. */
int su3_heatbath_sweep(su3_ctx *ctx, int32_t nsweeps, int32_t reunit_every, double *plaq_hist);

/* Enqueue nsweeps (>= 0) microcanonical over-relaxation sweeps (Brown & Woch,
 * Phys. Rev. Lett. 58 (1987) 2394; Creutz, Phys. Rev. D 36 (1987) 515): the
 * same schedule and subgroups as the heat bath, each subgroup element replaced
 * by r = (v^+)^2, v = a/|a|, which reflects it about the element the staple
 * prefers.  Re Tr(U A) of every updated link, hence the action and the
 * plaquette, is unchanged; no randoms are drawn and the sweep index does not
 * advance.  Interleaved with heat-bath sweeps it shortens autocorrelations
 * without changing the equilibrium distribution. */
int su3_overrelax(su3_ctx *ctx, int32_t nsweeps);

/* Enqueue Gram-Schmidt of rows 0 and 1 of every link (row 2 stays implied). */
int su3_reunitarize(su3_ctx *ctx);

/* Mean plaquette (1/6V) sum_s sum_{mu<nu} Re Tr[U_mu(s) U_nu(s+mu) U_mu(s+nu)^+
 * U_nu(s)^+] / 3; per-site FP32 products, FP64 sums (64-bit fixed point,
 * 2^-28, across workgroups).  Synchronous; *out is a host pointer. */
int su3_plaquette(su3_ctx *ctx, double *out);

/* Polyakov loop: the mean over spatial sites of Tr[U_3(x,0) ... U_3(x,Nt-1)]/3
 * (real and imaginary parts) and the mean of its modulus.  Synchronous; out is
 * host double[3] = {re, im, mean modulus}. */
int su3_polyakov(su3_ctx *ctx, double *out);

/* Copy links to / from the host exchange layout (host double[V][4][3][3][2],
 * 576*V bytes).  get_links rebuilds row 2 in FP64 from the stored rows;
 * set_links stores rows 0 and 1 rounded to FP32 (row 2 of the input is not
 * read).  Synchronous. */
int su3_get_links(su3_ctx *ctx, double *host);
int su3_set_links(su3_ctx *ctx, const double *host);

/* Sweep index (Philox counter word 1) of the next sweep; beta.  Setters apply
 * to work enqueued later. */
int su3_get_sweep(su3_ctx *ctx, uint32_t *out);
int su3_set_sweep(su3_ctx *ctx, uint32_t sweep);
int su3_set_beta(su3_ctx *ctx, double beta);
/* Philox replica id (< 2^26, else SU2_EINVAL; default 0) of later sweeps: a
 * lattice with replica id r draws the randoms of replica r of a batch.  Drops
 * captured sweeps. */
int su3_set_replica(su3_ctx *ctx, uint32_t replica);

/* hipGraph capture of heat-bath sweeps, for loops over many short calls
 * (small lattices are bound by launch overhead): record nsweeps sweeps exactly
 * as su3_heatbath_sweep enqueues them (meas 1: with the fused plaquette, into
 * the caller's device buffer dev_history of history_rows doubles; meas 0:
 * none), then replay the recording `count` times with su3_replay_sweeps, one
 * graph launch each.  The sweep index lives on the device, so every replay
 * continues the chain: links and plaquettes are bit for bit those of the same
 * sweeps run by su3_heatbath_sweep, and the k-th replay since the capture
 * writes history rows k*nsweeps..(k+1)*nsweeps-1.  With reunit_every > 0,
 * nsweeps must be a multiple of it and the sweep index at capture a multiple
 * of it (else SU2_EINVAL), and a replay is refused (SU2_ESTATE) unless the
 * sweep index is again a multiple of it; a replay that would write past
 * history_rows is refused (SU2_EINVAL); nothing is enqueued then.  Needs a
 * non-null stream (SU2_ESTATE).  su3_set_beta and su3_set_launch drop the
 * recording (replay: SU2_ESTATE); su3_set_sweep does not (replays continue
 * from the new index). */
int su3_capture_sweeps(su3_ctx *ctx, int32_t nsweeps, int32_t reunit_every, int meas,
                       double *dev_history, int64_t history_rows);
int su3_replay_sweeps(su3_ctx *ctx, int32_t count);

/* Pass-kernel launch: block 64, 128, 192 or 256 threads; remap 1 maps
 * workgroups to contiguous lattice stretches per XCD; snake 1 runs odd-parity
 * passes backwards; tile_z, tile_t (powers of two <= 256, 0 = keep) set the
 * (z, t) plane tiling of the traversal.  Results do not depend on it. */
int su3_set_launch(su3_ctx *ctx, int block, int remap, int snake, int tile_z, int tile_t);

/* Device pointer of the link arrays and the context's hipStream_t. */
int su3_links_device(su3_ctx *ctx, void **links_dev, void **hip_stream);

/* Wait for all work enqueued on the context's stream. */
int su3_synchronize(su3_ctx *ctx);

/* Batches: n replicas (1 <= n <= 65535, else SU2_EINVAL) of one lattice
 * size, run by the same kernels with one launch per pass for all of them
 * (grid z = replica), for workloads of many small lattices (coupling scans,
 * ensembles) that would leave most of the GPU idle one lattice at a time.
 * Replica r has coupling betas[r] (host double[n], each finite and >= 0, else
 * SU2_EINVAL), Philox replica id r (its hot start and every draw are those of
 * a single lattice with su3_set_replica(r)), its own links, accumulators and
 * history, and follows that single lattice bit for bit.  Memory: n times a
 * single lattice's (su3_links_bytes plus about 140 KiB of scratch).  Calls
 * match the single-lattice ones (same arguments, errors and synchronisation)
 * with these differences: plaq_hist of su3_batch_heatbath_sweep is host
 * double[nsweeps][n]; su3_batch_plaquette writes double[n] and
 * su3_batch_polyakov double[n][3]; get/set_links take the replica r (0 <= r <
 * n, else SU2_EINVAL).  The sweep index is common to all replicas. */
int su3_batch_init(su3_batch **out, int32_t n, const int32_t dims[4], const double *betas,
                   uint64_t seed, int start, void *hip_stream);
int su3_batch_destroy(su3_batch *b);
int su3_batch_size(su3_batch *b, int32_t *n);
int su3_batch_heatbath_sweep(su3_batch *b, int32_t nsweeps, int32_t reunit_every,
                             double *plaq_hist);
int su3_batch_overrelax(su3_batch *b, int32_t nsweeps);
int su3_batch_reunitarize(su3_batch *b);
int su3_batch_plaquette(su3_batch *b, double *out);
int su3_batch_polyakov(su3_batch *b, double *out);
int su3_batch_get_links(su3_batch *b, int32_t r, double *host);
int su3_batch_set_links(su3_batch *b, int32_t r, const double *host);
int su3_batch_get_sweep(su3_batch *b, uint32_t *out);
int su3_batch_set_sweep(su3_batch *b, uint32_t sweep);
int su3_batch_set_launch(su3_batch *b, int block, int remap, int snake, int tile_z, int tile_t);
int su3_batch_synchronize(su3_batch *b);

/* Test hook: enqueue one pass (direction mu, parity) at the current sweep
 * index, which does not advance. */
int su3_test_pass(su3_ctx *ctx, int mu, int parity);
/* Test hook: read U_mu at n sites (canonical indices, host array) into host
 * double[n][3][3][2] (row 2 rebuilt in FP64) without copying the whole field;
 * synchronous.  SU2_EINVAL for a site outside the lattice. */
int su3_test_read_links(su3_ctx *ctx, int64_t n, const int64_t *sites, int mu, double *out);
/* Test hook: enqueue one over-relaxation pass (direction mu, parity). */
int su3_test_or_pass(su3_ctx *ctx, int mu, int parity);

#ifdef __cplusplus
}
#endif

#endif
