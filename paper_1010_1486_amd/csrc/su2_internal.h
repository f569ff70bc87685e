// su2_internal.h -- host-side declarations shared by the runtime and the
// kernel launchers of libsu2 (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "su2_device.h"

namespace su2rt {

void set_error(const std::string &msg);

// Global sums: every workgroup reduces its values in FP64 (wave shuffles,
// then LDS) and adds the block sum, rounded to a multiple of 2^-kFixedShift,
// to a 64-bit integer accumulator.  Integer addition is associative, so the
// total does not depend on the order in which workgroups finish, and the adds
// can be spread over kBuckets counters (workgroup b uses bucket b mod
// kBuckets, each on its own 128-byte line) so that they do not serialise on
// one address.
constexpr int kFixedShift = 28;
constexpr int kBuckets = 256;
constexpr int kBucketStride = 16;  // 16 x 8 B = one 128-byte line per bucket
constexpr int kNumAcc = 4;  // plaquette, Polyakov (fixed point); proposals, accepts (counts)
constexpr size_t kAccBytes = (size_t)kNumAcc * kBuckets * kBucketStride * 8;

enum Result { R_PLAQ = 0, R_POLY_SIGNED = 1, R_POLY_ABS = 2, R_COUNTS = 4 };
enum Acc { ACC_PLAQ = 0, ACC_POLY = 1, ACC_PROPOSED = 2, ACC_ACCEPTED = 3 };

struct Counters {
    uint32_t sweep;     // sweep index used by the next pass (Philox counter word 1)
    uint32_t meas_idx;  // next history row written by a measured sweep
    uint32_t done;      // work-queue items of this replica finished in the current launch
    uint32_t graph_row; // next history row written by a replay of captured sweeps
    uint32_t pad[12];
};

// History-row counter of a measured sweep: direct calls count rows from the
// start of each call (meas_idx); the sweeps of a captured graph count on
// across replays (graph_row, reset at capture), untouched by direct calls.
__host__ __device__ inline uint32_t *row_counter(Counters *c, bool graph)
{
    return graph ? &c->graph_row : &c->meas_idx;
}

// Shared state of the persistent work-queue launch: one queue per XCD.
constexpr int kMaxQueues = 16;  // the XCC id is 4 bits
struct QueueState {
    uint32_t ticket[kMaxQueues][32];  // next item of queue q (own 128-byte line each)
    uint32_t error;                   // nonzero: a bounded wait ran out or work was left over
    uint32_t pad0[31];
    int32_t rank[kMaxQueues];         // XCC id -> queue (-1: the XCD takes no work)
    uint32_t slots[kMaxQueues];       // items per stage of queue q
    uint32_t off[kMaxQueues];         // first entry of queue q in the slot -> replica map
};

// Device-resident descriptor of one lattice (replica) of an ensemble.  A
// single lattice is an ensemble of one.
struct Rep {
    su2dev::Geom g;
    float *links;              // 32 planes of g.vh floats
    Counters *cnt;             // this replica's counters
    unsigned long long *acc;   // this replica's kNumAcc x kBuckets accumulators
    double *results;           // 8 FP64 result slots
    float beta;
    double beta_d;             // beta for the FP64 path
    uint32_t replica;          // Philox replica id
    uint32_t first_block;      // first pass workgroup of this replica (multiple of 8)
    uint32_t nblocks;          // pass workgroups of this replica
    uint32_t qfirst;           // first work-queue slot of this replica in its queue
    float orw;                 // learned proposal: < 0 independence, else over-relaxed
                               // with noise half-width orw (learned_link)
};

// Per-replica scratch: counters, accumulators, result slots.
constexpr size_t kRepScratch = sizeof(Counters) + kAccBytes + 8 * sizeof(double);

struct LaunchCfg {
    int pass_block = 256;
    bool xcd_remap = true;
    bool snake = true;        // odd-parity passes traverse backwards
    uint32_t grid_cap = 0;    // > 0: persistent pass grid of at most this many workgroups
    bool small = true;        // whole sweeps in one launch when every V/2 <= kSmallMaxVh
    bool queue = false;       // whole sweeps in one persistent work-queue launch
    bool affine = false;      // batches: each replica's pass workgroups on one XCD
    int grain = 1;            // work-queue items per ticket
    uint32_t march_R = 0;     // > 0: single lattices run the LDS-staged march pass
    uint32_t march_T = 0;     //      (tiles of march_R rows, march_T planes per workgroup)
};

// ------------------------------------------------------------- work queue
// A persistent launch runs ns sweeps of every replica.  Each replica belongs
// to one queue, and each queue is served by the workgroups of one XCD only,
// so a replica's links stay in that XCD's L2 and its items need ordering
// only within the XCD.  A queue is a list of items in the order (sweep,
// stage, slot).  Per sweep the stages are the 8 passes (mu = stage >> 1,
// parity = stage & 1), then the reunitarisation (sweeps j with
// (j + 1) mod reunit = 0), the plaquette after it (when measured) and the
// Polyakov loop (when measured).  Every stage has one item per slot of the
// queue, the slots of its replicas side by side, nblocks (pass workgroups of
// the replica) slots each.  The end-of-sweep bookkeeping of a replica (sums,
// history row) is done by the workgroup that finishes its last item of the
// sweep and counts as one more item.
struct QueuePlan {
    uint32_t ns;      // sweeps in the launch
    uint32_t reunit;  // reunitarisation period (0: none)
    uint32_t phase;   // index of the first sweep mod reunit (0 without)
    uint32_t want_p, want_l, rows;  // plaquette, Polyakov loop, history rows (0/1)
    uint32_t graph_rows;            // rows counted by the graph's counter (row_counter)
};

enum QueueKind { QK_PASS = 0, QK_REUNIT = 1, QK_PLAQ = 2, QK_POLY = 3 };

struct QueueItem {
    uint32_t sweep;  // sweep within the launch
    uint32_t stage;  // stage within the sweep
    uint32_t slot;   // pass workgroup slot
    int kind;
};

__host__ __device__ inline bool queue_reunit_sweep(const QueuePlan &p, uint32_t i)
{
    return p.reunit > 0u && (p.phase + i + 1u) % p.reunit == 0u;
}

// Stages of the sweeps before sweep i (i <= ns).
__host__ __device__ inline uint32_t queue_stages_before(const QueuePlan &p, uint32_t i)
{
    const uint32_t nre = p.reunit > 0u ? (p.phase + i) / p.reunit : 0u;
    return (8u + p.want_l) * i + (1u + p.want_p) * nre;
}

__host__ __device__ inline uint32_t queue_total_stages(const QueuePlan &p)
{
    return queue_stages_before(p, p.ns);
}

// Item t of a queue with `slots` items per stage.
__host__ __device__ inline QueueItem queue_decode(const QueuePlan &p, uint32_t t, uint32_t slots)
{
    QueueItem it;
    const uint32_t gs = t / slots;
    it.slot = t - gs * slots;
    uint32_t lo = 0u, hi = p.ns;  // stages_before(lo) <= gs < stages_before(hi)
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (queue_stages_before(p, mid) <= gs) lo = mid;
        else hi = mid;
    }
    it.sweep = lo;
    it.stage = gs - queue_stages_before(p, lo);
    if (it.stage < 8u) {
        it.kind = QK_PASS;
    } else {
        const uint32_t k = it.stage - 8u;
        if (queue_reunit_sweep(p, lo))
            it.kind = k == 0u ? QK_REUNIT : (k == 1u && p.want_p ? QK_PLAQ : QK_POLY);
        else
            it.kind = QK_POLY;
    }
    return it;
}

// Items of a replica with n slots that must be finished before its items of
// (sweep, stage) start: every item of the earlier stages plus one
// bookkeeping item per earlier sweep.
__host__ __device__ inline uint32_t queue_target(const QueuePlan &p, uint32_t n, uint32_t sweep,
                                                 uint32_t stage)
{
    return (queue_stages_before(p, sweep) + stage) * n + sweep;
}

// Done count reached when the last item of `sweep` finishes (before its
// bookkeeping item).
__host__ __device__ inline uint32_t queue_sweep_last(const QueuePlan &p, uint32_t n,
                                                     uint32_t sweep)
{
    return queue_stages_before(p, sweep + 1u) * n + sweep;
}

// Largest V/2 of the whole-sweep kernel (one workgroup per replica, up to
// 1024 threads, 2 sites per thread).
constexpr uint32_t kSmallMaxVh = 2048;

// Everything a launch needs to address an ensemble on the device.
struct Ens {
    const Rep *reps;          // device array of nrep descriptors
    const uint32_t *bmap;     // pass workgroup -> replica (nullptr when nrep == 1)
    // XCD-affine pass launch (nullptr: off): workgroup b -> (replica, block of
    // the replica), replica 0xFFFFFFFF for padding; amap_len workgroups
    const uint2 *amap;
    uint32_t amap_len;
    int nrep;
    uint32_t total_blocks;    // pass workgroups over all replicas (padded)
    uint32_t max_vh;          // largest V/2 over the replicas
    uint32_t max_ns3;         // largest spatial volume
    int poly_s;               // Polyakov segments (common divisor of every Nt)
    uint32_t plane_hs = 0;    // half-sites per (x, y) plane if every replica has the same, else 0
};

// Kernel launchers (all asynchronous on `stream`; return hipError_t).
hipError_t launch_init(const Ens &e, const int *starts_dev, uint64_t seed, hipStream_t stream);
// measure: accumulate (1/2)Tr(U' V_nu), nu < mu, into acc[ACC_PLAQ].
// table != nullptr: learned-proposal Metropolis update (counts into
// acc[ACC_PROPOSED] / acc[ACC_ACCEPTED]); else the exact heat bath.  norm:
// reunitarise each new link before it is stored (and measured).
hipError_t launch_pass(const Ens &e, int mu, int par, uint64_t seed, bool measure,
                       const float *table, const LaunchCfg &cfg, hipStream_t stream,
                       bool norm = false);
// The pass with LDS-staged neighbour planes (su2_march.hip), single lattice:
// workgroups of `block` threads own R full x-rows of an (x, y) plane at one z
// and walk T planes along t; nunits workgroups (ntile = Ny / R tiles per
// plane), per = nunits / 8 when that divides (XCD-contiguous ranges, else 0);
// an LDS slot holds (R + 2) Nx/2 links.  march_shape fills m and returns
// false when the lattice does not fit (Ny % R, Nt % T, Nx/2 R > 256 or
// < Nx, LDS over 64 KiB).
struct MarchShape {
    uint32_t R, T, block, ntile, nunits, per, slot_elems;
};
bool march_shape(const int32_t dims[4], uint32_t R, uint32_t T, MarchShape *m);
hipError_t launch_pass_march(const Ens &e, int mu, int par, uint64_t seed, bool measure, bool orx,
                             const MarchShape &m, int rev, hipStream_t stream);
// One microcanonical over-relaxation pass (U' = U~^+ U^+ U~^+, no randoms),
// in the workgroup layout of launch_pass; measure and norm as launch_pass.
hipError_t launch_or_pass(const Ens &e, int mu, int par, bool measure, const LaunchCfg &cfg,
                          hipStream_t stream, bool norm = false);
// Sum of all plaquettes into acc[ACC_PLAQ]; sum of L(x) into acc[ACC_POLY].
hipError_t launch_plaquette(const Ens &e, hipStream_t stream);
hipError_t launch_polyakov(const Ens &e, hipStream_t stream);
// results[R_PLAQ] = plaquette, results[R_POLY_*] = Polyakov loop from the
// accumulators (flags 1 / 2), which are reset.
hipError_t launch_take(const Ens &e, int flags, hipStream_t stream);
// End of a sweep.  flags: 1 plaquette in acc[ACC_PLAQ], 2 Polyakov in
// acc[ACC_POLY], 4 append a history row (P, L, |L|) per replica at
// hist[3 * (row * nrep + r)] with row from row_counter (8: the graph's
// counter).  Resets the accumulators, advances sweep.
hipError_t launch_sweep_end(const Ens &e, int flags, double *hist, hipStream_t stream);
hipError_t launch_reunitarize(const Ens &e, hipStream_t stream);
// ns whole sweeps of every replica (all V/2 <= kSmallMaxVh) in one launch:
// passes, reunitarisation every reunit_every sweeps (absolute sweep index),
// measurements (flags 1 plaquette, 2 Polyakov loop, 4 history rows at
// hist[3 * (row * nrep + r)], 8 rows from the graph's counter); advances the
// sweep and row counters.
// table != nullptr: learned-proposal Metropolis updates.
hipError_t launch_small_sweeps(const Ens &e, int ns, uint64_t seed, int reunit_every, int flags,
                               double *hist, const float *table, hipStream_t stream);
// ns sweeps of every replica in one persistent work-queue launch (see
// QueuePlan; qs holds the queues, qmap their slot -> replica maps, nullptr
// for a single replica), followed by a one-workgroup-per-replica launch that
// checks that every item ran, advances the sweep and row counters and clears
// the queue state.  grid workgroups of `block` threads (block = the pass
// block of the slot layout).  spin_limit bounds every wait (polls); when it
// runs out qs->error is raised and the launch drains without waiting.
hipError_t launch_queue_sweeps(const Ens &e, const QueuePlan &plan, const uint32_t *qmap,
                               uint64_t seed, int block, uint32_t grid, int grain, bool snake,
                               double *hist, const float *table, QueueState *qs,
                               uint32_t spin_limit, hipStream_t stream);
// Bit mask of the XCC ids that run workgroups of a large launch (one-time
// probe of the current device; synchronous).
hipError_t probe_xcc_mask(uint32_t *mask);
// FP64 links (single lattice; links point to 8 arrays of V/2 x 4 doubles):
// start (hot != 0: Haar from Philox tag 2), one heat-bath pass (measure as
// launch_pass), plaquette / Polyakov sums into the accumulators,
// reunitarisation.
hipError_t launch_init64(const Ens &e, int hot, uint64_t seed, hipStream_t stream);
hipError_t launch_pass64(const Ens &e, int mu, int par, uint64_t seed, bool measure,
                         const LaunchCfg &cfg, hipStream_t stream);
hipError_t launch_plaquette64(const Ens &e, hipStream_t stream);
hipError_t launch_polyakov64(const Ens &e, hipStream_t stream);
hipError_t launch_reunitarize64(const Ens &e, hipStream_t stream);
// Rectangular Wilson loops of a single FP32 lattice, R <= rmax, T <= tmax
// (<= kWilsonMax): part holds wilson_blocks(e) * kWilsonMax^2 doubles, sums
// receives kWilsonMax^2 sums over sites and the 12 ordered planes,
// sums[(R - 1) kWilsonMax + (T - 1)] (divide by 12 V).
constexpr int kWilsonMax = 4;
inline uint32_t wilson_blocks(const Ens &e) { return 12u * (uint32_t)((2ull * e.max_vh + 255) / 256); }
hipError_t launch_wilson(const Ens &e, int rmax, int tmax, double *part, double *sums,
                         hipStream_t stream);
// Workgroups of `block` threads of the queue kernel the device holds at once.
uint32_t queue_resident_grid(int block, bool learned);
// which: 1 set sweep, 2 set meas_idx, 4 zero all accumulators, 8 zero counts,
// 16 zero the work-queue state (done counters; qs ticket and error), 32 set
// graph_row.
hipError_t launch_set_counter(const Ens &e, uint32_t sweep, uint32_t meas, int which,
                              hipStream_t stream, QueueState *qs = nullptr);
// results[R_COUNTS..] = proposals, accepts (as uint64); reset if asked.
hipError_t launch_counts(const Ens &e, int reset, hipStream_t stream);
hipError_t launch_gauge(const Ens &e, float *G, uint64_t seed, hipStream_t stream);
// Streaming floor of a pass (single lattice): see stream_kernel.
hipError_t launch_test_stream(const Ens &e, int mu, int par, float *out, hipStream_t stream);
hipError_t launch_test_philox(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out,
                              hipStream_t stream);
hipError_t launch_test_links(const float *V, int64_t n, float beta, uint64_t seed,
                             uint32_t sweep, uint32_t mu, uint32_t replica, float *out,
                             int32_t *ntrials, hipStream_t stream);

// ------------------------------------------------------- learned proposal
constexpr int kNNParams = 2671;
constexpr int kNNActRows = 176;  // per-sample record rows of the backward pass

struct NNBuffers {
    float *params, *grad, *m, *v;  // kNNParams each
    float *alpha, *a0;             // training data
    float *act, *loss;             // kNNActRows x batch, batch
    float *table;                  // kNNRows x kNNRow, kNNTablePad floats into table_alloc
    float *table_alloc;
};

hipError_t launch_nn_data(float *alpha, float *a0, int64_t n, float lo, float hi, uint64_t seed,
                          hipStream_t stream);
// Forward/backward of samples [offset, offset + batch) (mod n) and the
// gradient of the mean NLL into nb.grad; mean loss into *loss_out if given.
hipError_t launch_nn_step(const NNBuffers &nb, int64_t offset, int batch, int64_t n,
                          double *loss_out, hipStream_t stream);
hipError_t launch_nn_adam(const NNBuffers &nb, float lr, int step, hipStream_t stream);
hipError_t launch_nn_table(const float *params, float *table, hipStream_t stream);
hipError_t launch_test_learned(const float *table, const float *V, const float *Uold, int64_t n,
                               float beta, uint64_t seed, uint32_t sweep, uint32_t mu,
                               uint32_t replica, float orw, float *out, int32_t *accepted,
                               hipStream_t stream);

}  // namespace su2rt
