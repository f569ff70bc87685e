// su2_static.hip -- heat-bath sweeps with measurements on caller-owned links
// that allocate no device memory (su2_sweep_measure_static in su2.h).
//
// The sweep kernels keep a descriptor of the lattice and its counters, fixed-
// point accumulators and result slots in a scratch buffer; a context keeps it
// in memory the library allocates (su2_init) or the caller brings
// (su2_init_ext).  This entry point keeps it in `scratch`, a file-scope
// device array of kStaticScratchBytes that every GPU holds for the life of
// the process, so that callers that cannot allocate (graph capture, serving
// loops) can run sweeps.  The launches are those su2_sweep_measure enqueues
// for a lattice in its default launch configuration, so links and history
// are bit for bit the same.
#include <mutex>
#include <string>

#include "../../include/su2.h"
#include "su2_internal.h"
#include "su3_internal.h"
#include "su2_api.h"

using namespace su2dev;

namespace su2rt {
namespace {

// Layout of the static scratch: the descriptor, then the lattice's counters,
// accumulators and result slots (as in a context's scratch for one lattice).
constexpr size_t kRepBytes = (sizeof(Rep) + 255) / 256 * 256;
constexpr size_t kStaticScratchNeed = kRepBytes + (kRepScratch + 255) / 256 * 256;
constexpr size_t kStaticScratchBytes = 160 * 1024;
static_assert(kStaticScratchNeed <= kStaticScratchBytes, "static scratch too small");

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Device address of `scratch` on each device, looked up on the first call
// with that device current (each GPU holds its own copy of the array).
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_of_current_device(unsigned char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SU2_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SU2_ERANGE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SU2_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return SU2_OK;
}

// The descriptor goes in as a kernel argument (no host buffer to keep alive).
__global__ void put_rep_kernel(Rep r, Rep *dst) { *dst = r; }

#define STATIC_TRY(expr)                                                                \
    do {                                                                                \
        const hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) return fail(SU2_EHIP, std::string(#expr) + ": " +         \
                                                        hipGetErrorString(e_));         \
    } while (0)

int sweep_measure_static(float *links, const int32_t dims[4], double beta, uint64_t seed,
                         uint32_t sweep0, int32_t ns, int32_t reunit_every, int meas,
                         double *hist, hipStream_t stream)
{
    if (!links || !hist) return fail(SU2_EINVAL, "links_dev or dev_history is NULL");
    if (int rc = check_dims(dims)) return rc;
    if (!beta_ok(beta)) return fail(SU2_EINVAL, "beta must be finite and >= 0");
    if (ns < 0 || reunit_every < 0) return fail(SU2_EINVAL, "negative count");
    if (meas & ~(SU2_MEAS_PLAQ | SU2_MEAS_POLY)) return fail(SU2_EINVAL, "bad meas flags");
    if (kStaticScratchNeed > kStaticScratchBytes)
        return fail(SU2_ERANGE, "the static scratch holds " + std::to_string(kStaticScratchBytes) +
                                    " B, the lattice needs " + std::to_string(kStaticScratchNeed));
    unsigned char *ptr = nullptr;
    if (int rc = scratch_of_current_device(&ptr)) return rc;
    if (ns == 0) return SU2_OK;

    // the descriptor a context of these extents holds in its default launch
    const LaunchCfg cfg;
    const Geom g = make_geom(dims, 3, 3);
    if (!geom_selfcheck(g))
        return fail(SU2_ERANGE, "index arithmetic self-check failed for these extents");
    Rep *reps = reinterpret_cast<Rep *>(ptr);
    unsigned char *rs = ptr + kRepBytes;
    Rep r{};
    r.g = g;
    r.links = links;
    r.cnt = reinterpret_cast<Counters *>(rs);
    r.acc = reinterpret_cast<unsigned long long *>(rs + sizeof(Counters));
    r.results = reinterpret_cast<double *>(rs + sizeof(Counters) + kAccBytes);
    r.beta = (float)beta;
    r.beta_d = beta;
    r.replica = 0u;
    r.first_block = 0u;
    r.nblocks = (g.vh + (uint32_t)cfg.pass_block - 1u) / (uint32_t)cfg.pass_block;
    r.qfirst = 0u;
    r.orw = -1.0f;
    int poly_s = 8;
    while (dims[3] % poly_s) poly_s /= 2;
    const Ens e{reps, nullptr, nullptr, 0u, 1, r.nblocks, g.vh,
                (uint32_t)(dims[0] * dims[1] * dims[2]), poly_s, g.P};

    hipLaunchKernelGGL(put_rep_kernel, dim3(1), dim3(1), 0, stream, r, reps);
    STATIC_TRY(hipGetLastError());
    // sweep index sweep0, history row 0, every accumulator cleared (the array
    // keeps whatever the previous call on this GPU left)
    STATIC_TRY(launch_set_counter(e, sweep0, 0u, 1 | 2 | 4, stream));
    const bool want_p = (meas & SU2_MEAS_PLAQ) != 0, want_l = (meas & SU2_MEAS_POLY) != 0;
    if (cfg.small && g.vh <= kSmallMaxVh) {
        const int flags = (want_p ? 1 : 0) | (want_l ? 2 : 0) | 4;
        STATIC_TRY(launch_small_sweeps(e, ns, seed, reunit_every, flags, hist, nullptr, stream));
        return SU2_OK;
    }
    for (int32_t i = 0; i < ns; ++i) {
        const uint32_t j = sweep0 + (uint32_t)i;
        const bool reunit = reunit_every > 0 && ((j + 1u) % (uint32_t)reunit_every) == 0u;
        const bool fused = want_p && !reunit;
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par)
                STATIC_TRY(launch_pass(e, mu, par, seed, fused && par == 1 && mu >= 1, nullptr,
                                       cfg, stream));
        if (reunit) STATIC_TRY(launch_reunitarize(e, stream));
        if (want_p && !fused) STATIC_TRY(launch_plaquette(e, stream));
        if (want_l) STATIC_TRY(launch_polyakov(e, stream));
        STATIC_TRY(launch_sweep_end(e, (want_p ? 1 : 0) | (want_l ? 2 : 0) | 4, hist, stream));
    }
    return SU2_OK;
}

}  // namespace
}  // namespace su2rt

extern "C" {

int su2_sweep_measure_static(float *links_dev, const int32_t dims[4], double beta, uint64_t seed,
                             uint32_t sweep0, int32_t nsweeps, int32_t reunit_every, int meas,
                             double *dev_history, void *hip_stream)
{
    SU2_API_BEGIN
    return su2rt::sweep_measure_static(links_dev, dims, beta, seed, sweep0, nsweeps, reunit_every,
                                       meas, dev_history, static_cast<hipStream_t>(hip_stream));
    SU2_API_END
}

}  // extern "C"
