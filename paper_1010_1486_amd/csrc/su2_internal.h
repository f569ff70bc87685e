// su2_internal.h -- host-side declarations shared by the runtime and the
// kernel launchers of libsu2 (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "su2_device.h"

namespace su2rt {

void set_error(const std::string &msg);

// Scratch layout (bytes): [0,64) device counters, [64,256) FP64 result
// slots, [256, 256 + kAccBytes) fixed-point accumulators.
constexpr size_t kCountersOff = 0;
constexpr size_t kResultsOff = 64;
constexpr size_t kAccOff = 256;

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
constexpr size_t kScratchBytes = kAccOff + kAccBytes;

struct Counters {
    uint32_t sweep;     // sweep index used by the next pass (Philox counter word 1)
    uint32_t meas_idx;  // next history row written by a measured sweep
};

enum Result { R_PLAQ = 0, R_POLY_SIGNED = 1, R_POLY_ABS = 2 };
enum Acc { ACC_PLAQ = 0, ACC_POLY = 1, ACC_PROPOSED = 2, ACC_ACCEPTED = 3 };

// Accumulator `which`, bucket b: acc + (which * kBuckets + b) * kBucketStride.
struct Sums {
    Counters *cnt;
    unsigned long long *acc;
};

struct LaunchCfg {
    int pass_block = 256;
    bool xcd_remap = true;
    bool snake = true;  // odd-parity passes traverse backwards
};

// Kernel launchers (all asynchronous on `stream`; return hipError_t).
hipError_t launch_init(float *links, const su2dev::Geom &g, int start, uint64_t seed,
                       uint32_t replica, hipStream_t stream);
// measure: accumulate (1/2)Tr(U' V_nu), nu < mu, into acc[ACC_PLAQ].
// table != nullptr: learned-proposal Metropolis update (counts into
// acc[ACC_PROPOSED] / acc[ACC_ACCEPTED]); else the exact heat bath.
hipError_t launch_pass(float *links, const su2dev::Geom &g, int mu, int par, Sums c,
                       float beta, uint64_t seed, uint32_t replica, bool measure,
                       const float *table, const LaunchCfg &cfg, hipStream_t stream);
// out[0] = proposals, out[1] = accepts summed over the buckets; reset if asked.
hipError_t launch_counts(Sums c, unsigned long long *out, int reset, hipStream_t stream);

// ------------------------------------------------------- learned proposal
constexpr int kNNParams = 2671;
constexpr int kNNActRows = 176;  // per-sample record rows of the backward pass

struct NNBuffers {
    float *params, *grad, *m, *v;  // kNNParams each
    float *alpha, *a0;             // training data
    float *act, *loss;             // kNNActRows x batch, batch
    float *table;                  // kNNRows x kNNRow
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
                               uint32_t replica, float *out, int32_t *accepted,
                               hipStream_t stream);
int pass_grid(const su2dev::Geom &g, const LaunchCfg &cfg);
// Sum of all plaquettes into acc[ACC_PLAQ]; sum of L(x) into acc[ACC_POLY].
hipError_t launch_plaquette(const float *links, const su2dev::Geom &g, Sums c,
                            hipStream_t stream);
hipError_t launch_polyakov(const float *links, const su2dev::Geom &g, Sums c,
                           hipStream_t stream);
// out[0] = acc[which] * scale, out[1] = |out[0]|; resets acc[which].
hipError_t launch_take(Sums c, int which, double scale, double *out, hipStream_t stream);
// End of a sweep.  flags: 1 plaquette in acc[ACC_PLAQ], 2 Polyakov in
// acc[ACC_POLY], 4 append a history row (P, L, |L|) at hist[3*meas_idx].
// Resets the accumulators and advances the sweep counter.
hipError_t launch_sweep_end(Sums c, int flags, double plaq_scale, double poly_scale,
                            double *hist, hipStream_t stream);
hipError_t launch_reunitarize(float *links, const su2dev::Geom &g, hipStream_t stream);
hipError_t launch_gauge(float *links, const su2dev::Geom &g, float *G, uint64_t seed,
                        uint32_t replica, hipStream_t stream);
hipError_t launch_test_philox(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out,
                              hipStream_t stream);
hipError_t launch_test_links(const float *V, int64_t n, float beta, uint64_t seed,
                             uint32_t sweep, uint32_t mu, uint32_t replica, float *out,
                             int32_t *ntrials, hipStream_t stream);
// which: 1 set sweep, 2 set meas_idx, 4 zero the accumulators.
hipError_t launch_set_counter(Sums c, uint32_t sweep, uint32_t meas, int which,
                              hipStream_t stream);

}  // namespace su2rt
