/*
 * su2.h -- C ABI of libsu2, the MI355X (gfx950) SU(2) pure-gauge heat bath.
 *
 * Method: N. Cardoso and P. Bicudo, "Lattice SU(2) on GPU's", LAT2010
 * (arXiv:1010.1486).  Sec. 2 defines the update: for each link, the staple
 * sum V of the six neighbouring products, k = sqrt(det V), U~ = V/k, a0 drawn
 * from sqrt(1 - a0^2) exp(beta k a0), a uniform direction for the rest of the
 * element X, and U' = X U~^{-1}.  Sec. 4 (and the caption of its Fig. 3) fixes
 * the schedule: per direction mu, first the even sites, then the odd sites,
 * eight passes per sweep; and the measurements: mean plaquette and Polyakov
 * loop summed over the lattice.
 *
 * Conventions
 *   Lattice     periodic Nx x Ny x Nz x Nt, every extent even and >= 2; site
 *               s = x + Nx*(y + Ny*(z + Nz*t)); mu = 0:x 1:y 2:z 3:t; parity
 *               (x+y+z+t) & 1.
 *   Links       U = a0 + i a.sigma stored as 4 FP32 reals (a float4).
 *               Device layout: 8 arrays of V/2 float4, array (mu*2 + parity)
 *               holding U_mu at the half-site h = s >> 1 of every site of
 *               that parity, i.e. float[8][V/2][4] (64*V bytes; float
 *               ((mu*2 + parity)*V/2 + h)*4 + c).  Host exchange layout
 *               (get/set): float[V][4 mu][4 c] in canonical site order.
 *   Randoms     Philox4x32-10, key = seed, counter = (site, sweep index,
 *               mu | tag<<2 | replica<<6, draw).  Results are bit-identical
 *               for identical (links, seed, sweep index, replica, beta).
 *   Sampler     alpha = beta k >= 1: Kennedy-Pendleton; alpha < 1: rejection
 *               from the Haar (semicircle) marginal; both exact.
 *
 * Errors: every function returns SU2_OK (0) or a negative code and never
 * aborts; su2_last_error() gives a thread-local message for the last failure.
 * Asynchrony: functions documented as "enqueue" return after launching work on
 * the context's stream; functions returning host values synchronise it.
 * Threading: contexts are independent; one context must not be used from two
 * host threads at once.
 * Device: a context (lattice, batch, network) lives on the HIP device that was
 * current when it was created; every later call on it must be made with that
 * device current again (hipSetDevice), as its stream and memory belong to it.
 */
#ifndef SU2_H
#define SU2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct su2_ctx su2_ctx;

enum {
    SU2_OK = 0,
    SU2_EINVAL = -1, /* null pointer, negative count, beta not finite or < 0, bad enum */
    SU2_EODD = -2,   /* an extent is odd or < 2 (the checkerboard needs even extents) */
    SU2_ENOMEM = -3, /* device allocation failed, or caller buffer too small */
    SU2_EHIP = -4,   /* a HIP runtime call failed (message has the HIP error string) */
    SU2_ESTATE = -5, /* call not valid in the context's state (e.g. no proposal loaded) */
    SU2_ERANGE = -6  /* a size exceeds the library's index range (V/2 >= 2^28) */
};

enum { SU2_COLD = 0, SU2_HOT = 1 };
enum { SU2_KP = 0, SU2_LEARNED = 1, SU2_KP_OR = 2 };
enum { SU2_MEAS_PLAQ = 1, SU2_MEAS_POLY = 2 };

/* Message for the last failing call on this host thread ("" if none). */
const char *su2_last_error(void);

/* Device bytes the caller must provide to su2_init_ext for these extents:
 * links 64*V; scratch about 131 KB (descriptor, sweep counter, history index,
 * the fixed-point accumulators of the global sums in 256 buckets, FP64 result
 * slots).  Return 0 when the extents are invalid or out of range. */
size_t su2_links_bytes(const int32_t dims[4]);
size_t su2_scratch_bytes(const int32_t dims[4]);

/* Create a context with library-owned device memory and stream, and write the
 * cold (all links 1) or hot (Haar-random, Philox tag 2) start (Sec. 4: the
 * initialisation kernels).  dims: host array of 4 extents.  beta: finite and
 * >= 0 (beta = 4/g^2 of Sec. 2; 0 makes every update Haar-random); the same
 * range holds for every beta argument of this header.  The sweep index starts
 * at 0.  Free with su2_destroy. */
int su2_init(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start);

/* As su2_init, but on caller-owned device memory and stream: links_dev
 * (>= su2_links_bytes) and scratch_dev (>= su2_scratch_bytes), both device
 * pointers that the caller keeps alive until su2_destroy; hip_stream is a
 * hipStream_t (NULL = the null stream).  The library allocates no device
 * memory for the context. */
int su2_init_ext(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
                 void *links_dev, size_t links_bytes, void *scratch_dev, size_t scratch_bytes,
                 void *hip_stream);

/* Rectangular Wilson loops for scale setting (the T/Tc axis of the Polyakov
 * loop needs a lattice spacing, which the paper does not give):
 * out[(R - 1) tmax + (T - 1)] = (1/(12 V)) sum_s sum_{mu != nu}
 * (1/2) Tr[L_mu(s,R) L_nu(s+R mu,T) L_mu(s+T nu,R)^+ L_nu(s,T)^+], with
 * L_mu(x, n) = U_mu(x) U_mu(x+mu) ... U_mu(x+(n-1)mu), R = 1..rmax,
 * T = 1..tmax; W(1,1) is the plaquette.  Per-site values FP32, sums FP64
 * (deterministic order).  Synchronous; allocates a temporary device buffer.
 * SU2_EINVAL unless 1 <= rmax, tmax <= 4 and both are below every extent;
 * SU2_ESTATE on an FP64 context.  out: host double[rmax * tmax]. */
int su2_wilson_loops(su2_ctx *ctx, int rmax, int tmax, double *out);

/* As su2_init with FP64 links and staples (library-owned memory, 128 V bytes;
 * work runs on hip_stream, NULL being the null stream):
 * the double-precision variant the paper names as its next step
 * (Conclusions).  Every step of the update is FP64 -- staple sum, k, the a0
 * sampler (same Philox trials as the FP32 path), direction, product, hot start
 * (Box-Muller in FP64) and reunitarisation -- so at equal seeds the two
 * precisions differ only by FP32 rounding and by the rare decisions that
 * rounding flips.  Supported on such a context: the heat-bath sweeps
 * (SU2_KP; SU2_LEARNED gives SU2_ESTATE), su2_sweep_measure, capture/replay,
 * su2_reunitarize, su2_plaquette, su2_polyakov, get/set links (float or
 * double host arrays), set_sweep/beta/replica, set_launch/autotune (block,
 * remap, pass order and tiles; the whole-sweep, work-queue and persistent
 * grid-cap launches are FP32 only, a grid cap is ignored), su2_test_pass.  Device layout: 8 classes (mu * 2 + parity),
 * each two arrays of V/2 double pairs, (a0, a1) then (a2, a3). */
int su2_init_f64(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
                 void *hip_stream);
/* *out = 1 for an FP64 context, else 0. */
int su2_is_f64(su2_ctx *ctx, int *out);
/* Links in the canonical host layout as FP64 (host double[V][4][4]); on an
 * FP32 context the values are widened / rounded to FP32. */
int su2_get_links_f64(su2_ctx *ctx, double *host);
int su2_set_links_f64(su2_ctx *ctx, const double *host);

/* Synchronise the stream and release the context (and library-owned memory). */
int su2_destroy(su2_ctx *ctx);

/* Enqueue nsweeps (>= 0) heat-bath sweeps (Sec. 2 update, Sec. 4 schedule: for
 * mu = 0..3, even sites then odd sites).  mode SU2_KP uses the exact sampler;
 * SU2_LEARNED the learned proposal with an exact Metropolis step (needs
 * su2_set_proposal); SU2_KP_OR makes each sweep a compound sweep: the SU2_KP
 * sweep, then n_or microcanonical over-relaxation sweeps (su2_set_hb_overrelax;
 * default 1) in the same order, each link U -> U~^+ U^+ U~^+ with U~ = V/|V|
 * (keeps (1/2)Tr(U V) and the Haar measure, draws no randoms; V = 0 leaves
 * U), always as per-pass launches.  The sweep index advances by nsweeps
 * (one per compound sweep).  FP64 contexts: SU2_KP only. */
int su2_heatbath_sweep(su2_ctx *ctx, int32_t nsweeps, int mode);

/* Enqueue nsweeps sweeps and measure after each one.  reunit_every > 0
 * reunitarises after every sweep whose index j satisfies (j+1) % reunit_every
 * == 0, before measuring.  meas: SU2_MEAS_PLAQ | SU2_MEAS_POLY.  dev_history:
 * device FP64 buffer of 3*nsweeps entries, receiving (plaquette, signed mean
 * Polyakov loop, its absolute value) per sweep (0 where not measured).  The
 * plaquette is fused into the odd passes of mu = 1, 2, 3 (no extra read of the
 * field) except on reunitarisation sweeps, where it is measured afterwards
 * (unless the reunitarisation is fused, su2_set_reunit_fused).
 * Global sums: FP64 within each workgroup, then 64-bit fixed point (2^-28)
 * across workgroups, so results are bit-reproducible. */
int su2_sweep_measure(su2_ctx *ctx, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                      double *dev_history);

/* For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): su2_sweep_measure
 * (SU2_KP) without a context.  Enqueues on hip_stream (NULL: the null stream)
 * nsweeps heat-bath sweeps of the lattice whose links the caller holds at
 * links_dev, starting at sweep index sweep0, with reunit_every and meas as in
 * su2_sweep_measure, and writes FP64[nsweeps][3] history rows to dev_history.
 * links_dev: su2_links_bytes(dims) bytes in the device layout of su2.h (the
 * buffer su2_init_ext takes; su2_links_device of a context of the same
 * extents points at one); both buffers stay the caller's.  The links and
 * history are bit for bit those of su2_sweep_measure on a context in its
 * default launch configuration with the same links, beta, seed and sweep
 * index.  The descriptor, counters and fixed-point accumulators (about
 * 131 KiB, whatever the lattice's size) live in a fixed 160 KiB device array
 * each GPU holds until the process ends; nothing is allocated.  Every call on a GPU shares that array: calls that overlap on one
 * GPU (other streams, other threads) race and give wrong results; each call
 * clears what must start at zero.  Errors: SU2_EINVAL (NULL buffer, negative
 * count, bad meas, beta not finite or < 0), SU2_EODD / SU2_ERANGE (extents as
 * su2_init; SU2_ERANGE also if the array could not hold the lattice's scratch),
 * SU2_EHIP (device lookup or launch failed).  Asynchronous. */
int su2_sweep_measure_static(float *links_dev, const int32_t dims[4], double beta, uint64_t seed,
                             uint32_t sweep0, int32_t nsweeps, int32_t reunit_every, int meas,
                             double *dev_history, void *hip_stream);

/* Enqueue U <- U/|U| for every link, |U|^2 in FP64. */
int su2_reunitarize(su2_ctx *ctx);

/* Mean plaquette (1/6V) sum_s sum_{mu<nu} (1/2)Tr U_mu(s) U_nu(s+mu) U_mu(s+nu)^+
 * U_nu(s)^+ (Sec. 4), per-site FP32 products, FP64 global sum.  Synchronous:
 * *out is a host pointer. */
int su2_plaquette(su2_ctx *ctx, double *out);

/* Mean Polyakov loop (1/Ns^3) sum_x (1/2)Tr prod_{t=0}^{Nt-1} U_3(x,t) (Sec. 4),
 * ordered product with t = 0 leftmost, FP64 sum; and its absolute value.
 * Synchronous; host pointers (either may be NULL). */
int su2_polyakov(su2_ctx *ctx, double *out_signed, double *out_abs);

/* Copy links to / from the host exchange layout float[V][4][4] (host pointer,
 * 64*V bytes).  Synchronous. */
int su2_get_links(su2_ctx *ctx, float *host);
int su2_set_links(su2_ctx *ctx, const float *host);

/* Sweep index (Philox counter word 1) of the next sweep; beta; replica id
 * (Philox counter word 2 bits 6..31).  Setters apply to work enqueued later. */
int su2_get_sweep(su2_ctx *ctx, uint32_t *out);
int su2_set_sweep(su2_ctx *ctx, uint32_t sweep);
int su2_set_beta(su2_ctx *ctx, double beta);
int su2_set_replica(su2_ctx *ctx, uint32_t replica);

/* Device pointer of the link arrays and the context's hipStream_t. */
int su2_links_device(su2_ctx *ctx, void **links_dev, void **hip_stream);

/* Wait for all work enqueued on the context's stream. */
int su2_synchronize(su2_ctx *ctx);

/* Launch configuration of the pass kernel: block size (64, 128, 192 or 256
 * threads); flags: bit 0 = XCD-contiguous workgroup remap, bit 1 = disable
 * the alternating (forward, backward) pass order, bit 2 = disable the
 * whole-sweep kernel for small lattices (by default, when every V/2 <= 2048,
 * one launch runs whole sweeps with one workgroup per lattice), bit 3 = run
 * sweeps as one persistent work-queue launch per call (every pass, the
 * reunitarisation and the measurements of all replicas, ordered per replica
 * by completion counters; each replica is served by one XCD, replicas spread
 * over the XCDs by size; grid_cap = its workgroups, at least one per XCD,
 * 0 = as many as the device holds at once), bits 4-5 = log2 of the items it
 * takes per ticket, bit 6 = batches: all pass workgroups of a replica on one
 * XCD (replicas spread over the XCDs by size, each replica's blocks in
 * order on its XCD's L2; bit 0 is then unused), bit 7 = single FP32 lattices:
 * the pass with its neighbour links staged in LDS (heat bath and
 * over-relaxation; SU2_LEARNED keeps the plain pass): workgroups of R =
 * tile_z full x-rows of an (x, y) plane walk T = tile_t planes along t
 * (R must divide Ny and T divide Nt, 2 <= R, R Nx/2 <= 256; SU2_EINVAL
 * otherwise, and with bit 3); it implies bit 2;
 * the traversal
 * tile of (z, t) planes, tile_z x tile_t (powers of two <= 256, clipped to
 * divisors of Nz and Nt; 0 keeps the current value); grid_cap > 0 runs the
 * pass as a persistent grid of at most grid_cap workgroups looping over the
 * work (0 = one workgroup per tile).  Links do not depend on it; the
 * whole-sweep kernel rounds each site's plaquette and Polyakov value to the
 * 2^-28 fixed point instead of each workgroup's sum (differences ~1e-9).
 * Drops captured sweeps. */
int su2_set_launch(su2_ctx *ctx, int block, int flags, int tile_z, int tile_t, int grid_cap);
/* Current launch configuration (tiles as applied to this lattice's extents). */
int su2_get_launch(su2_ctx *ctx, int *block, int *flags, int *tile_z, int *tile_t, int *grid_cap);

/* Autotuner: times candidate launch configurations (block size, order flags,
 * traversal tile, persistent grid) on this lattice with sweeps of `mode` that
 * measure the plaquette (every candidate on 2 sweeps, the three fastest again
 * on 8; the faster of two timings each), restores links and counters
 * afterwards, and applies the fastest.  With a
 * cache_path (JSON lines, one entry per device and set of extents), a cached
 * choice is applied without timing and new choices are appended.
 * *best_us_per_sweep (may be NULL) receives its time per sweep. */
int su2_autotune(su2_ctx *ctx, const char *cache_path, int mode, double *best_us_per_sweep);

/* hipGraph capture: record nsweeps sweeps exactly as su2_sweep_measure (meas
 * = 0: as su2_heatbath_sweep) would enqueue them, then replay the recording
 * `count` times with su2_replay_sweeps (one graph launch per replay).  The
 * sweep index and the graph's own history row index advance on the device:
 * the k-th replay since the capture (k = 0, 1, ...) writes rows
 * k*nsweeps..(k+1)*nsweeps-1 of dev_history, whatever direct calls run between
 * replays (they count their rows separately).  history_rows: rows (3 doubles
 * each) dev_history holds (>= nsweeps when meas != 0, else SU2_EINVAL); a
 * replay that would write past them is refused with SU2_EINVAL and enqueues
 * nothing.  With reunit_every > 0, nsweeps must be a multiple of it and the
 * current sweep index a multiple of it, and a replay is refused (SU2_ESTATE)
 * unless the sweep index is again a multiple of it.  Needs a non-null
 * stream.  Later changes of the launch configuration, the proposal, either
 * over-relaxation setting, beta or the replica id drop the recording
 * (su2_replay_sweeps then returns SU2_ESTATE); su2_set_sweep does not (the
 * replays read the sweep index on the device and continue from it). */
int su2_capture_sweeps(su2_ctx *ctx, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                       double *dev_history, int64_t history_rows);
int su2_replay_sweeps(su2_ctx *ctx, int32_t count);

/* ============================================================== batches
 * n replicas with their own extents, couplings and starts advance together:
 * every kernel launch covers all of them (the pass maps its workgroups onto
 * the replicas' tiles), so small lattices fill the GPU.  Replica r uses
 * Philox replica id r, i.e. it follows exactly the chain of a single context
 * with the same extents, beta, seed and su2_set_replica(r).  Library-owned
 * device memory; hip_stream as for su2_init_ext (capture and autotuning need
 * a non-null stream). */
typedef struct su2_batch su2_batch;

/* dims: host int32[n][4]; betas: host double[n]; starts: host int[n]. */
int su2_batch_init(su2_batch **out, int32_t n, const int32_t *dims, const double *betas,
                   const int *starts, uint64_t seed, void *hip_stream);
int su2_batch_destroy(su2_batch *b);
int su2_batch_size(su2_batch *b, int32_t *n);
int su2_batch_sweep(su2_batch *b, int32_t nsweeps, int mode);
/* As su2_sweep_measure; dev_history is FP64[nsweeps][n][3]. */
int su2_batch_sweep_measure(su2_batch *b, int32_t nsweeps, int mode, int32_t reunit_every,
                            int meas, double *dev_history);
/* As su2_capture_sweeps; dev_history is FP64[history_rows][n][3]. */
int su2_batch_capture(su2_batch *b, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                      double *dev_history, int64_t history_rows);
int su2_batch_replay(su2_batch *b, int32_t count);
/* Plaquette and Polyakov loop of every replica into host arrays of n (any may
 * be NULL).  Synchronous. */
int su2_batch_observables(su2_batch *b, double *plaq, double *poly_signed, double *poly_abs);
int su2_batch_get_links(su2_batch *b, int32_t replica, float *host);
int su2_batch_set_links(su2_batch *b, int32_t replica, const float *host);
int su2_batch_set_launch(su2_batch *b, int block, int flags, int tile_z, int tile_t,
                         int grid_cap);
/* The batch's launch configuration (as su2_get_launch; tiles of replica 0). */
int su2_batch_get_launch(su2_batch *b, int *block, int *flags, int *tile_z, int *tile_t,
                         int *grid_cap);
int su2_batch_autotune(su2_batch *b, const char *cache_path, int mode, double *best_us);
int su2_batch_synchronize(su2_batch *b);
/* Per-replica learned proposals made / accepted (host uint64[n] each). */
int su2_batch_get_accept_stats(su2_batch *b, uint64_t *proposed, uint64_t *accepted, int reset);

/* ======================================================= learned proposal
 * An independence-Metropolis update of a0 with a learned proposal replaces the
 * exact sampler inside the pass (SU2_LEARNED); the heat-bath distribution of
 * Sec. 2 stays exact because the Metropolis ratio uses the proposal density.
 * Proposal: a 16-bin monotone rational-quadratic spline flow g on [-1, 1]
 * (Durkan et al. 2019) with q(a0) = g'(a0)/2, its 47 parameters given by an
 * MLP 1 -> 32 -> 32 -> 47 (tanh) of f(alpha) = 2 ln(alpha/0.5)/ln 60 - 1,
 * alpha = beta k.  For alpha outside [0.5, 30] the exact sampler is used.
 * Parameters: 2671 FP32, order W1[32] b1[32] W2[32][32] b2[32] W3[47][32]
 * b3[47] (rows = output units).  Training minimises the NLL of exact-sampler
 * draws with Adam (b1 0.9, b2 0.999, eps 1e-8), all on the GPU.  The pass
 * uses a 64-row table of the spline at f = -1 + 2j/63 (nearest row), rows
 * of 48 floats [x1..x15, 1, y1..y15, 1, d1..d15, 1]. */
typedef struct su2_nn su2_nn;

int su2_nn_num_params(void);
/* params_host: 2671 floats, or NULL for the default initialisation from
 * `seed` (hidden layers uniform in +-1/sqrt(fan_in), output weights 0, output
 * biases giving the identity spline, i.e. a uniform proposal).  hip_stream:
 * stream for the object's work (NULL = null stream).  Library-owned memory. */
int su2_nn_create(su2_nn **out, const float *params_host, uint64_t seed, void *hip_stream);
/* SU2_ESTATE (nothing freed) while a context or batch has it attached. */
int su2_nn_destroy(su2_nn *nn);
int su2_nn_get_params(su2_nn *nn, float *params_host);
int su2_nn_set_params(su2_nn *nn, const float *params_host);
/* Generate n training pairs on the GPU: alpha log-uniform in [alpha_lo,
 * alpha_hi] (Philox tag 5, draw (i, 0, 0|5<<2, 0)), a0 from the exact sampler
 * (trial blocks (i, 0, 1|5<<2, t)).  Replaces any data held. */
int su2_nn_sample_data(su2_nn *nn, int64_t n, double alpha_lo, double alpha_hi, uint64_t seed);
/* Caller-provided training data (host arrays of n floats). */
int su2_nn_set_data(su2_nn *nn, int64_t n, const float *alpha_host, const float *a0_host);
/* Data held: *n, and (if non-NULL) copies into host arrays of *n floats. */
int su2_nn_get_data(su2_nn *nn, int64_t *n, float *alpha_host, float *a0_host);
/* Mean NLL and its gradient (host float[2671]) over samples [offset,
 * offset + batch) (indices mod n).  Synchronous. */
int su2_nn_loss_grad(su2_nn *nn, int64_t offset, int32_t batch, double *loss, float *grad_host);
/* `steps` Adam steps on consecutive minibatches of the data (wrapping);
 * loss_history_host (may be NULL) receives each step's mean NLL.  Synchronous. */
int su2_nn_train(su2_nn *nn, int32_t steps, int32_t batch, double lr, double *loss_history_host);
/* As su2_nn_train with a cosine learning-rate schedule: step t (0-based) uses
 * lr1 + (lr0 - lr1)(1 + cos(pi t / steps))/2, from lr0 down towards lr1. */
int su2_nn_train_cosine(su2_nn *nn, int32_t steps, int32_t batch, double lr0, double lr1,
                        double *loss_history_host);
/* Evaluate the 64-row spline table from the current parameters / copy it
 * (host float[64 * 48]). */
int su2_nn_build_table(su2_nn *nn);
int su2_nn_get_table(su2_nn *nn, float *table_host);
/* Use nn's table for SU2_LEARNED sweeps of ctx (NULL unsets); its table must
 * be built (SU2_ESTATE otherwise).  While attached, the context or batch holds
 * the su2_nn: su2_nn_destroy returns SU2_ESTATE until every context and batch
 * using it has detached (set_proposal with NULL or another su2_nn) or been
 * destroyed.  Rebuilding the table of an attached su2_nn changes later sweeps. */
int su2_set_proposal(su2_ctx *ctx, su2_nn *nn);
int su2_batch_set_proposal(su2_batch *b, su2_nn *nn);
/* Over-relaxation sweeps after each heat-bath sweep of an SU2_KP_OR sweep
 * (0 <= n_or <= 16, else SU2_EINVAL; 0 makes SU2_KP_OR the plain heat bath;
 * default 1).  Not in the paper: the standard companion of a heat bath that
 * the learned proposal is compared with.  Drops captured sweeps. */
int su2_set_hb_overrelax(su2_ctx *ctx, int32_t n_or);
int su2_batch_set_hb_overrelax(su2_batch *b, int32_t n_or);
/* Where the reunitarisation of su2_sweep_measure / su2_capture_sweeps (and
 * the batch forms) happens.  on = 0 (default): a separate pass over the field
 * after each reunitarisation sweep, then the plaquette measured afresh.
 * on = 1: the last pass stage of a reunitarisation sweep (the heat bath, or
 * the last over-relaxation sweep of SU2_KP_OR) reunitarises each link as it
 * stores it (the same U/|U| with |U|^2 in FP64), and the plaquette stays fused
 * into the odd passes, so the sweep costs no extra read or write of the field.
 * Every link of the configuration after the sweep is reunitarised in both
 * forms; they differ in rounding only, because the passes of that sweep after
 * the first read the reunitarised links of the passes before (in exact
 * arithmetic a heat-bath link is unit and the reunitarisation is the
 * identity).  Calls with reunit_every > 0 then run as per-pass launches (no
 * work queue, no whole-sweep kernel for small lattices).  on not 0 or 1:
 * SU2_EINVAL; on = 1 on an FP64 context: SU2_ESTATE.  Not in the paper.
 * Drops captured sweeps. */
int su2_set_reunit_fused(su2_ctx *ctx, int on);
int su2_batch_set_reunit_fused(su2_batch *b, int on);
/* Over-relaxed use of the learned flow in SU2_LEARNED sweeps.  width < 0
 * (default): the independence proposal u = 2z - 1 above.  0 <= width <= 1:
 * the proposal u' = -g(x_old) + width (2z - 1), wrapped onto [-1, 1) with
 * period 2 (the reflection of the old link's flow coordinate plus uniform
 * noise), a0' = g^{-1}(u').  Its density in u is symmetric in (u, u'), so the
 * same Metropolis ratio w(a0')/w(x_old) keeps the heat-bath distribution of
 * Sec. 2 exact; width > 0 makes the chain irreducible, width = 1 is the
 * independence proposal in distribution, and for an exact flow width -> 0 is
 * ordered over-relaxation of a0 (Neal 1998): a0 moves to its opposite quantile
 * and successive configurations anticorrelate.  The direction of X is drawn
 * afresh as in the independence form.  SU2_EINVAL for width > 1 or NaN.
 * Drops captured sweeps. */
int su2_set_overrelax(su2_ctx *ctx, double width);
int su2_batch_set_overrelax(su2_batch *b, double width);
/* Learned proposals made and accepted since the last reset (synchronous). */
int su2_get_accept_stats(su2_ctx *ctx, uint64_t *proposed, uint64_t *accepted, int reset);

/* ----------------------------------------------------------- test hooks */
/* Philox4x32-10 on the GPU: n counters (host, 4 words each) -> host out. */
int su2_test_philox(const uint32_t *ctr_host, int64_t n, uint64_t seed, uint32_t *out_host);
/* Heat-bath update of n independent links from given staple sums V (host,
 * float[n][4]); link i uses site index i.  out_host float[n][4]; ntrials_host
 * (may be NULL) receives the sampler's trial count per link. */
int su2_test_heatbath_links(const float *V_host, int64_t n, double beta, uint64_t seed,
                            uint32_t sweep, uint32_t mu, uint32_t replica, float *out_host,
                            int32_t *ntrials_host);
/* Enqueue one (mu, parity) pass at the current sweep index (index unchanged);
 * mode SU2_KP or SU2_LEARNED, or SU2_KP_OR for one over-relaxation pass. */
int su2_test_pass(su2_ctx *ctx, int mu, int parity, int mode);
/* Bandwidth floor of a (mu, parity) pass (measurement aid): enqueue a kernel
 * that moves the same bytes as the pass -- the seven plane groups it reads,
 * each at the thread's own half-site, no stencil -- and writes the
 * per-half-site sum of those seven quaternions to out_dev (caller-owned
 * device memory of V/2 quaternions, one 16-byte nontemporal store each:
 * out[4 h + c], c = a0..a3).  No link or counter of ctx changes. */
int su2_test_stream_pass(su2_ctx *ctx, int mu, int parity, void *out_dev);
/* Host-side evaluation (no GPU needed) of the pass kernel's index map for
 * extents dims and traversal tile tile_z x tile_t (0 = default): for each of
 * the V/2 thread indices g of a pass over `parity`, out[9g] = canonical site of
 * the thread, out[9g + 1 + 2d] / out[9g + 2 + 2d] = half-site index (s >> 1)
 * of its +1 / -1 neighbour in direction d.  out: host uint32[9 * V/2]. */
int su2_test_index_map(const int32_t dims[4], int tile_z, int tile_t, int parity, uint32_t *out);
/* Host-side run (no GPU needed) of the work-queue schedule of a batch of n
 * lattices (dims: n x 4 extents) with `block`-thread workgroups and `queues`
 * queues (one per XCD, 1..16): nsweeps sweeps starting at sweep index
 * first_sweep, reunitarisation every reunit_every sweeps (0: none),
 * measurements `meas` with history rows when rows != 0.  Checks that the
 * replicas' slots tile the queues exactly, then runs each queue's items one
 * at a time in ticket order, checking that every item's wait target counts
 * exactly the replica's earlier items (so the queue can neither deadlock nor
 * start an item early) and that every sweep of every replica ends.
 * items_out (may be NULL): items run.  SU2_ERANGE with a message on the first
 * violation. */
int su2_test_queue_plan(int32_t n, const int32_t *dims, int block, int32_t queues,
                        int32_t nsweeps, int32_t reunit_every, uint32_t first_sweep, int meas,
                        int rows, int64_t *items_out);
/* Polls allowed per bounded wait of the batch's work-queue launches (default
 * 2^22).  A small value makes the waits run out on purpose: the launch then
 * drains normally and the next synchronising call returns SU2_EHIP. */
int su2_test_batch_spin_limit(su2_batch *b, uint32_t polls);
/* Learned-proposal update of n independent links (host float[n][4] staples V
 * and old links Uold); link i uses site index i; or_width as
 * su2_set_overrelax (< 0: independence proposal).  accepted_host (may be
 * NULL): 1 accepted, 0 rejected, -1 exact fallback. */
int su2_test_learned_links(su2_nn *nn, const float *V_host, const float *Uold_host, int64_t n,
                           double beta, uint64_t seed, uint32_t sweep, uint32_t mu,
                           uint32_t replica, double or_width, float *out_host,
                           int32_t *accepted_host);
/* Enqueue U_mu(x) -> G(x) U_mu(x) G(x+mu)^+ with G Haar from Philox tag 3. */
int su2_test_gauge_transform(su2_ctx *ctx, uint64_t seed);

#ifdef __cplusplus
}
#endif

#endif /* SU2_H */
