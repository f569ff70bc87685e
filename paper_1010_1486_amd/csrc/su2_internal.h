// su2_internal.h -- host-side declarations shared by the runtime and the
// kernel launchers of libsu2 (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "su2_device.h"

namespace su2rt {

void set_error(const std::string &msg);

// Scratch layout (bytes): [0,64) device counters, [64,256) FP64 result slots,
// [256, ...) FP64 block partials (kPartialArrays arrays of max_blocks each).
constexpr size_t kCountersOff = 0;
constexpr size_t kResultsOff = 64;
constexpr size_t kPartialsOff = 256;
constexpr int kPartialArrays = 4;
constexpr int kMinBlock = 64;

struct Counters {
    uint32_t sweep;     // sweep index used by the next pass (Philox counter word 1)
    uint32_t meas_idx;  // next history slot written by a measured sweep
};

enum Result { R_PLAQ = 0, R_POLY_SIGNED = 1, R_POLY_ABS = 2 };

size_t max_partial_blocks(int64_t volume);

struct LaunchCfg {
    int pass_block = 256;
    int pass_sites_per_thread = 1;
    bool xcd_remap = true;
};

// Kernel launchers (all asynchronous on `stream`; return hipError_t).
hipError_t launch_init(float *links, const su2dev::Geom &g, int start, uint64_t seed,
                       uint32_t replica, hipStream_t stream);
hipError_t launch_pass(float *links, const su2dev::Geom &g, int mu, int par,
                       const uint32_t *sweep_ptr, float beta, uint64_t seed, uint32_t replica,
                       double *partial, const LaunchCfg &cfg, hipStream_t stream);
int pass_grid(const su2dev::Geom &g, const LaunchCfg &cfg);
hipError_t launch_plaquette(const float *links, const su2dev::Geom &g, double *partial,
                            int *nblocks, hipStream_t stream);
hipError_t launch_polyakov(const float *links, const su2dev::Geom &g, double *partial,
                           int *nblocks, hipStream_t stream);
// Sum `narrays` partial arrays of `nblocks` entries (stride `stride`) in a fixed
// order, scale, and store into out[0] (and |.| into out[1] when abs_too).
hipError_t launch_finalize(const double *partial, int nblocks, int narrays, size_t stride,
                           double scale, double *out, int abs_too, hipStream_t stream);
// Plaquette of a fused sweep: sums the three measured passes' partials,
// appends to hist[3 * meas_idx] and advances the counters.
hipError_t launch_sweep_end(Counters *counters, const double *partial, int nblocks,
                            size_t stride, double scale, int measure, double *hist,
                            const double *extra_poly, hipStream_t stream);
hipError_t launch_reunitarize(float *links, const su2dev::Geom &g, hipStream_t stream);
hipError_t launch_gauge(float *links, const su2dev::Geom &g, float *G, uint64_t seed,
                        uint32_t replica, hipStream_t stream);
hipError_t launch_test_philox(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out,
                              hipStream_t stream);
hipError_t launch_test_links(const float *V, int64_t n, float beta, uint64_t seed,
                             uint32_t sweep, uint32_t mu, uint32_t replica, float *out,
                             int32_t *ntrials, hipStream_t stream);
hipError_t launch_set_counter(Counters *c, uint32_t sweep, uint32_t meas, int which,
                              hipStream_t stream);

}  // namespace su2rt
