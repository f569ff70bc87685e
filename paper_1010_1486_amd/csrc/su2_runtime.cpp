// su2_runtime.cpp -- C ABI of libsu2: contexts, argument checks, memory,
// the sweep schedule (Sec. 4: per direction, even then odd sites) and the
// measurement plumbing around the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/su2.h"
#include "su2_internal.h"

using su2dev::Geom;
using su2dev::kNNRow;
using su2dev::kNNRows;

namespace su2rt {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace su2rt

using namespace su2rt;

struct su2_ctx {
    int32_t dims[4];
    Geom g;
    int64_t volume;
    double beta;
    uint64_t seed;
    uint32_t replica;
    uint32_t sweep;  // host mirror of the device sweep counter
    float *links;
    size_t links_bytes;
    unsigned char *scratch;
    size_t scratch_bytes;
    bool own_mem;
    bool own_stream;
    hipStream_t stream;
    LaunchCfg cfg;
    const float *table = nullptr;  // learned-proposal table (device), owned by an su2_nn

    Counters *counters() { return reinterpret_cast<Counters *>(scratch + kCountersOff); }
    Sums sums()
    {
        return Sums{counters(), reinterpret_cast<unsigned long long *>(scratch + kAccOff)};
    }
    double *results() { return reinterpret_cast<double *>(scratch + kResultsOff); }
};

namespace {

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));              \
            return SU2_EHIP;                                                            \
        }                                                                               \
    } while (0)

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int check_dims(const int32_t *dims)
{
    if (!dims) return fail(SU2_EINVAL, "dims is NULL");
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || (dims[i] & 1))
            return fail(SU2_EODD, "every extent must be even and >= 2 (got " +
                                      std::to_string(dims[i]) + " in direction " +
                                      std::to_string(i) + ")");
    int64_t v = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    if (v / 2 >= (int64_t)1 << 30) return fail(SU2_ERANGE, "V/2 must be < 2^30");
    return SU2_OK;
}

// Multiplier and shift for exact division of 31-bit numerators by d
// (Granlund & Montgomery 1994, Thm. 4.2 with N = 31).
void magic(uint32_t d, uint32_t &m, uint32_t &s)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    m = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
    s = 31 + l;
}

uint32_t host_fdiv(uint32_t n, uint32_t m, uint32_t s)
{
    return (uint32_t)(((uint64_t)n * m) >> s);
}

uint32_t pow2_divisor_log(int32_t n, uint32_t cap)
{
    uint32_t l = 0;
    while (l < cap && (n % (2 << l)) == 0) ++l;
    return l;
}

Geom make_geom(const int32_t *d, uint32_t lg_tz, uint32_t lg_tt)
{
    Geom g;
    g.nx = d[0];
    g.ny = d[1];
    g.nz = d[2];
    g.nt = d[3];
    g.vh = (uint32_t)(((int64_t)d[0] * d[1] * d[2] * d[3]) / 2);
    g.hx = (uint32_t)(d[0] / 2);
    g.P = g.hx * (uint32_t)d[1];
    g.PZ = g.P * (uint32_t)d[2];
    g.wy = (uint32_t)(d[1] - 1) * g.hx;
    g.wz = (uint32_t)(d[2] - 1) * g.P;
    g.wt = (uint32_t)(d[3] - 1) * g.PZ;
    g.lg_tz = std::min(lg_tz, pow2_divisor_log(d[2], 8));
    g.lg_tt = std::min(lg_tt, pow2_divisor_log(d[3], 8));
    g.ntz = (uint32_t)d[2] >> g.lg_tz;
    magic(g.P, g.m_P, g.s_P);
    magic(g.hx, g.m_hx, g.s_hx);
    magic(g.ntz, g.m_ntz, g.s_ntz);
    return g;
}

// The divisions are exact by construction; check the extreme numerators.
bool geom_selfcheck(const Geom &g)
{
    const uint32_t ns[] = {0u, 1u, g.P - 1u, g.P, g.vh - 1u, g.vh / 2u + 7u};
    for (uint32_t n : ns) {
        if (host_fdiv(n, g.m_P, g.s_P) != n / g.P) return false;
        if (host_fdiv(n, g.m_hx, g.s_hx) != n / g.hx) return false;
        if (host_fdiv(n, g.m_ntz, g.s_ntz) != n / g.ntz) return false;
    }
    return true;
}

size_t scratch_bytes_for(int64_t) { return kScratchBytes; }

int check_ctx(su2_ctx *c)
{
    if (!c) return fail(SU2_EINVAL, "context is NULL");
    return SU2_OK;
}

// The sweep index the device uses is read from the device counter; keep the
// host mirror in step.
int enqueue_sweeps(su2_ctx *c, int32_t n, int mode, int32_t reunit_every, int meas,
                   double *hist)
{
    if (mode != SU2_KP && mode != SU2_LEARNED) return fail(SU2_EINVAL, "unknown mode");
    if (mode == SU2_LEARNED && !c->table)
        return fail(SU2_ESTATE, "no learned proposal loaded (su2_set_proposal)");
    const float *table = mode == SU2_LEARNED ? c->table : nullptr;
    const float beta = (float)c->beta;
    const double inv6v = 1.0 / (6.0 * (double)c->volume);
    const double inv_ns3 = 1.0 / ((double)c->dims[0] * c->dims[1] * c->dims[2]);
    // history rows restart at 0 for this call
    if (hist) HIP_TRY(launch_set_counter(c->sums(), 0, 0, 2, c->stream));
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t j = c->sweep + (uint32_t)i;
        const bool reunit = reunit_every > 0 && ((j + 1u) % (uint32_t)reunit_every) == 0u;
        const bool want_p = hist && (meas & SU2_MEAS_PLAQ);
        const bool fused = want_p && !reunit;
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par)
                HIP_TRY(launch_pass(c->links, c->g, mu, par, c->sums(), beta, c->seed,
                                    c->replica, fused && par == 1 && mu >= 1, table, c->cfg,
                                    c->stream));
        if (reunit) HIP_TRY(launch_reunitarize(c->links, c->g, c->stream));
        if (want_p && !fused) HIP_TRY(launch_plaquette(c->links, c->g, c->sums(), c->stream));
        const bool want_l = hist && (meas & SU2_MEAS_POLY);
        if (want_l) HIP_TRY(launch_polyakov(c->links, c->g, c->sums(), c->stream));
        const int flags = (want_p ? 1 : 0) | (want_l ? 2 : 0) | (hist ? 4 : 0);
        HIP_TRY(launch_sweep_end(c->sums(), flags, inv6v, inv_ns3, hist, c->stream));
    }
    c->sweep += (uint32_t)n;
    return SU2_OK;
}

}  // namespace

extern "C" {

const char *su2_last_error(void) { return g_last_error.c_str(); }

size_t su2_links_bytes(const int32_t dims[4])
{
    if (!dims) return 0;
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || (dims[i] & 1)) return 0;
    return (size_t)64 * (size_t)dims[0] * dims[1] * dims[2] * dims[3];
}

size_t su2_scratch_bytes(const int32_t dims[4])
{
    if (!su2_links_bytes(dims)) return 0;
    return scratch_bytes_for((int64_t)dims[0] * dims[1] * dims[2] * dims[3]);
}

static int init_common(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed,
                       int start, void *links_dev, size_t links_bytes, void *scratch_dev,
                       size_t scratch_bytes, void *stream, bool ext)
{
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!std::isfinite(beta)) return fail(SU2_EINVAL, "beta must be finite");
    if (start != SU2_COLD && start != SU2_HOT) return fail(SU2_EINVAL, "start must be COLD or HOT");
    const size_t need_l = su2_links_bytes(dims), need_s = su2_scratch_bytes(dims);
    if (ext) {
        if (!links_dev || !scratch_dev) return fail(SU2_EINVAL, "device buffer is NULL");
        if (links_bytes < need_l || scratch_bytes < need_s)
            return fail(SU2_ENOMEM, "caller buffers too small: need links " +
                                        std::to_string(need_l) + " B, scratch " +
                                        std::to_string(need_s) + " B");
    }
    su2_ctx *c = new (std::nothrow) su2_ctx();
    if (!c) return fail(SU2_ENOMEM, "host allocation failed");
    std::memcpy(c->dims, dims, sizeof(c->dims));
    c->g = make_geom(dims, 3, 3);
    if (!geom_selfcheck(c->g)) {
        delete c;
        return fail(SU2_ERANGE, "index arithmetic self-check failed for these extents");
    }
    c->volume = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    c->beta = beta;
    c->seed = seed;
    c->replica = 0;
    c->sweep = 0;
    c->links_bytes = need_l;
    c->scratch_bytes = need_s;
    c->own_mem = !ext;
    c->own_stream = false;
    if (ext) {
        c->links = static_cast<float *>(links_dev);
        c->scratch = static_cast<unsigned char *>(scratch_dev);
        c->stream = static_cast<hipStream_t>(stream);
    } else {
        void *l = nullptr, *s = nullptr;
        hipError_t e = hipMalloc(&l, need_l);
        if (e == hipSuccess) e = hipMalloc(&s, need_s);
        if (e != hipSuccess) {
            if (l) (void)hipFree(l);
            delete c;
            return fail(e == hipErrorOutOfMemory ? SU2_ENOMEM : SU2_EHIP,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        c->links = static_cast<float *>(l);
        c->scratch = static_cast<unsigned char *>(s);
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            (void)hipFree(l);
            (void)hipFree(s);
            delete c;
            return fail(SU2_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        c->stream = st;
        c->own_stream = true;
    }
    hipError_t e = launch_set_counter(c->sums(), 0, 0, 7, c->stream);
    if (e == hipSuccess) e = launch_init(c->links, c->g, start, seed, 0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        set_error(std::string("init: ") + hipGetErrorString(e));
        su2_destroy(c);
        return SU2_EHIP;
    }
    *out = c;
    return SU2_OK;
}

int su2_init(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start)
{
    return init_common(out, dims, beta, seed, start, nullptr, 0, nullptr, 0, nullptr, false);
}

int su2_init_ext(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
                 void *links_dev, size_t links_bytes, void *scratch_dev, size_t scratch_bytes,
                 void *hip_stream)
{
    return init_common(out, dims, beta, seed, start, links_dev, links_bytes, scratch_dev,
                       scratch_bytes, hip_stream, true);
}

int su2_destroy(su2_ctx *c)
{
    if (!c) return fail(SU2_EINVAL, "context is NULL");
    int rc = SU2_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(SU2_EHIP, "sync on destroy");
    if (c->own_mem) {
        (void)hipFree(c->links);
        (void)hipFree(c->scratch);
    }
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return rc;
}

int su2_heatbath_sweep(su2_ctx *c, int32_t nsweeps, int mode)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsweeps < 0) return fail(SU2_EINVAL, "nsweeps must be >= 0");
    return enqueue_sweeps(c, nsweeps, mode, 0, 0, nullptr);
}

int su2_sweep_measure(su2_ctx *c, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                      double *dev_history)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsweeps < 0 || reunit_every < 0) return fail(SU2_EINVAL, "negative count");
    if (!dev_history) return fail(SU2_EINVAL, "dev_history is NULL");
    if (meas & ~(SU2_MEAS_PLAQ | SU2_MEAS_POLY)) return fail(SU2_EINVAL, "bad meas flags");
    return enqueue_sweeps(c, nsweeps, mode, reunit_every, meas, dev_history);
}

int su2_reunitarize(su2_ctx *c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(launch_reunitarize(c->links, c->g, c->stream));
    return SU2_OK;
}

int su2_plaquette(su2_ctx *c, double *out)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    HIP_TRY(launch_plaquette(c->links, c->g, c->sums(), c->stream));
    HIP_TRY(launch_take(c->sums(), ACC_PLAQ, 1.0 / (6.0 * (double)c->volume),
                        c->results() + R_PLAQ, c->stream));
    double v[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(v, c->results() + R_PLAQ, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *out = v[0];
    return SU2_OK;
}

int su2_polyakov(su2_ctx *c, double *out_signed, double *out_abs)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(launch_polyakov(c->links, c->g, c->sums(), c->stream));
    HIP_TRY(launch_take(c->sums(), ACC_POLY,
                        1.0 / ((double)c->dims[0] * c->dims[1] * c->dims[2]),
                        c->results() + R_POLY_SIGNED, c->stream));
    double v[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(v, c->results() + R_POLY_SIGNED, 2 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (out_signed) *out_signed = v[0];
    if (out_abs) *out_abs = v[1];
    return SU2_OK;
}

int su2_get_links(su2_ctx *c, float *host)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    std::vector<float> planes(c->links_bytes / sizeof(float));
    HIP_TRY(hipMemcpyAsync(planes.data(), c->links, c->links_bytes, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int64_t vh = c->g.vh;
    const int32_t *d = c->dims;
    for (int64_t s = 0; s < c->volume; ++s) {
        int64_t r = s;
        const int x = (int)(r % d[0]);
        r /= d[0];
        const int y = (int)(r % d[1]);
        r /= d[1];
        const int z = (int)(r % d[2]);
        const int t = (int)(r / d[2]);
        const int par = (x + y + z + t) & 1;
        const int64_t h = s >> 1;
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 4; ++k)
                host[(s * 4 + mu) * 4 + k] = planes[((mu * 2 + par) * 4 + k) * vh + h];
    }
    return SU2_OK;
}

int su2_set_links(su2_ctx *c, const float *host)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    std::vector<float> planes(c->links_bytes / sizeof(float));
    const int64_t vh = c->g.vh;
    const int32_t *d = c->dims;
    for (int64_t s = 0; s < c->volume; ++s) {
        int64_t r = s;
        const int x = (int)(r % d[0]);
        r /= d[0];
        const int y = (int)(r % d[1]);
        r /= d[1];
        const int z = (int)(r % d[2]);
        const int t = (int)(r / d[2]);
        const int par = (x + y + z + t) & 1;
        const int64_t h = s >> 1;
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 4; ++k)
                planes[((mu * 2 + par) * 4 + k) * vh + h] = host[(s * 4 + mu) * 4 + k];
    }
    HIP_TRY(hipMemcpyAsync(c->links, planes.data(), c->links_bytes, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SU2_OK;
}

int su2_get_sweep(su2_ctx *c, uint32_t *out)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = c->sweep;
    return SU2_OK;
}

int su2_set_sweep(su2_ctx *c, uint32_t sweep)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(launch_set_counter(c->sums(), sweep, 0, 1, c->stream));
    c->sweep = sweep;
    return SU2_OK;
}

int su2_set_beta(su2_ctx *c, double beta)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!std::isfinite(beta)) return fail(SU2_EINVAL, "beta must be finite");
    c->beta = beta;
    return SU2_OK;
}

int su2_set_replica(su2_ctx *c, uint32_t replica)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (replica >= (1u << 26)) return fail(SU2_EINVAL, "replica id must be < 2^26");
    c->replica = replica;
    return SU2_OK;
}

int su2_links_device(su2_ctx *c, void **links_dev, void **hip_stream)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (links_dev) *links_dev = c->links;
    if (hip_stream) *hip_stream = c->stream;
    return SU2_OK;
}

int su2_synchronize(su2_ctx *c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SU2_OK;
}

static int lg_of_tile(int tile, int32_t extent, uint32_t cur, uint32_t *out)
{
    if (tile == 0) {
        *out = cur;
        return SU2_OK;
    }
    if (tile < 0 || (tile & (tile - 1)) || extent % tile)
        return fail(SU2_EINVAL, "tile sizes must be powers of two dividing the extent");
    uint32_t l = 0;
    while ((1 << l) < tile) ++l;
    *out = l;
    return SU2_OK;
}

int su2_set_launch(su2_ctx *c, int block, int xcd_remap, int tile_z, int tile_t)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (block < 64 || block > 256 || (block % 64) != 0)
        return fail(SU2_EINVAL, "block must be 64, 128, 192 or 256");
    uint32_t lz, lt;
    if ((rc = lg_of_tile(tile_z, c->dims[2], c->g.lg_tz, &lz))) return rc;
    if ((rc = lg_of_tile(tile_t, c->dims[3], c->g.lg_tt, &lt))) return rc;
    Geom g = make_geom(c->dims, lz, lt);
    if (!geom_selfcheck(g)) return fail(SU2_ERANGE, "index arithmetic self-check failed");
    c->g = g;
    c->cfg.pass_block = block;
    c->cfg.xcd_remap = (xcd_remap & 1) != 0;
    c->cfg.snake = (xcd_remap & 2) == 0;
    return SU2_OK;
}

int su2_test_philox(const uint32_t *ctr_host, int64_t n, uint64_t seed, uint32_t *out_host)
{
    if (n < 0 || (n > 0 && (!ctr_host || !out_host))) return fail(SU2_EINVAL, "bad arguments");
    if (n == 0) return SU2_OK;
    void *d_in = nullptr, *d_out = nullptr;
    const size_t bytes = (size_t)n * 16;
    HIP_TRY(hipMalloc(&d_in, bytes));
    hipError_t e = hipMalloc(&d_out, bytes);
    if (e == hipSuccess) e = hipMemcpy(d_in, ctr_host, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_test_philox((const uint32_t *)d_in, n, seed, (uint32_t *)d_out, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out_host, d_out, bytes, hipMemcpyDeviceToHost);
    (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    if (e != hipSuccess) return fail(SU2_EHIP, std::string("test_philox: ") + hipGetErrorString(e));
    return SU2_OK;
}

int su2_test_heatbath_links(const float *V_host, int64_t n, double beta, uint64_t seed,
                            uint32_t sweep, uint32_t mu, uint32_t replica, float *out_host,
                            int32_t *ntrials_host)
{
    if (n < 0 || (n > 0 && (!V_host || !out_host))) return fail(SU2_EINVAL, "bad arguments");
    if (!std::isfinite(beta) || mu > 3) return fail(SU2_EINVAL, "bad beta or mu");
    if (n >= ((int64_t)1 << 32)) return fail(SU2_ERANGE, "n must be < 2^32");
    if (n == 0) return SU2_OK;
    void *d_v = nullptr, *d_o = nullptr, *d_t = nullptr;
    const size_t bytes = (size_t)n * 16;
    HIP_TRY(hipMalloc(&d_v, bytes));
    hipError_t e = hipMalloc(&d_o, bytes);
    if (e == hipSuccess && ntrials_host) e = hipMalloc(&d_t, (size_t)n * 4);
    if (e == hipSuccess) e = hipMemcpy(d_v, V_host, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_test_links((const float *)d_v, n, (float)beta, seed, sweep, mu, replica,
                              (float *)d_o, (int32_t *)d_t, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out_host, d_o, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ntrials_host)
        e = hipMemcpy(ntrials_host, d_t, (size_t)n * 4, hipMemcpyDeviceToHost);
    (void)hipFree(d_v);
    if (d_o) (void)hipFree(d_o);
    if (d_t) (void)hipFree(d_t);
    if (e != hipSuccess)
        return fail(SU2_EHIP, std::string("test_heatbath_links: ") + hipGetErrorString(e));
    return SU2_OK;
}

int su2_test_pass(su2_ctx *c, int mu, int parity, int mode)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (mu < 0 || mu > 3 || parity < 0 || parity > 1) return fail(SU2_EINVAL, "bad mu/parity");
    if (mode != SU2_KP && mode != SU2_LEARNED) return fail(SU2_EINVAL, "unknown mode");
    if (mode == SU2_LEARNED && !c->table) return fail(SU2_ESTATE, "no learned proposal loaded");
    HIP_TRY(launch_pass(c->links, c->g, mu, parity, c->sums(), (float)c->beta, c->seed,
                        c->replica, false, mode == SU2_LEARNED ? c->table : nullptr, c->cfg,
                        c->stream));
    return SU2_OK;
}

int su2_test_index_map(const int32_t dims[4], int tile_z, int tile_t, int parity, uint32_t *out)
{
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!out || (parity != 0 && parity != 1)) return fail(SU2_EINVAL, "bad arguments");
    Geom g0 = make_geom(dims, 3, 3);
    uint32_t lz, lt;
    if ((rc = lg_of_tile(tile_z, dims[2], g0.lg_tz, &lz))) return rc;
    if ((rc = lg_of_tile(tile_t, dims[3], g0.lg_tt, &lt))) return rc;
    const Geom g = make_geom(dims, lz, lt);
    if (!geom_selfcheck(g)) return fail(SU2_ERANGE, "index arithmetic self-check failed");
    for (uint32_t gid = 0; gid < g.vh; ++gid) {
        const su2dev::PassSite ps = su2dev::pass_site(g, gid, parity);
        const su2dev::Deltas d = su2dev::neighbour_deltas(g, ps);
        uint32_t *o = out + 9 * (size_t)gid;
        o[0] = 2u * ps.h + (uint32_t)(ps.x & 1);
        for (int k = 0; k < 4; ++k) {
            o[1 + 2 * k] = ps.h + d.p[k];
            o[2 + 2 * k] = ps.h + d.m[k];
        }
    }
    return SU2_OK;
}

int su2_test_gauge_transform(su2_ctx *c, uint64_t seed)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    void *G = nullptr;
    HIP_TRY(hipMalloc(&G, (size_t)c->volume * 16));
    hipError_t e = launch_gauge(c->links, c->g, (float *)G, seed, c->replica, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(G);
    if (e != hipSuccess) return fail(SU2_EHIP, std::string("gauge: ") + hipGetErrorString(e));
    return SU2_OK;
}

/* ===================================================== learned proposal */
struct su2_nn {
    NNBuffers b;
    int64_t ndata = 0;     // training samples held
    int64_t act_cap = 0;   // batch capacity of the per-sample record
    int step = 0;          // Adam step counter
    bool table_ready = false;
    hipStream_t stream = nullptr;
    double *dev_loss = nullptr;  // per-step losses of the last train call
    int loss_cap = 0;
};

static void nn_free(su2_nn *n)
{
    // b.a0 lives inside the b.alpha allocation and b.loss inside b.act
    float *bufs[] = {n->b.params, n->b.grad, n->b.m, n->b.v, n->b.alpha, n->b.act, n->b.table};
    for (float *p : bufs)
        if (p) (void)hipFree(p);
    if (n->dev_loss) (void)hipFree(n->dev_loss);
}

// Default parameters: hidden layers uniform in +-1/sqrt(fan_in) from a
// splitmix64 stream of the seed, biases 0; output weights 0 and output biases
// that make the spline the identity (the untrained proposal is uniform).
static void nn_default_params(uint64_t seed, std::vector<float> &p)
{
    p.assign(kNNParams, 0.0f);
    uint64_t st = seed ^ 0x5DEECE66Dull;
    auto next = [&]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * 0x1.0p-53;
    };
    for (int i = 0; i < 32; ++i) p[i] = (float)(2.0 * next() - 1.0);  // fan_in 1
    for (int i = 0; i < 1024; ++i) p[64 + i] = (float)((2.0 * next() - 1.0) / std::sqrt(32.0));
    const float id = (float)std::log(std::expm1(1.0 - 1e-3));
    for (int i = 32; i < 47; ++i) p[2624 + i] = id;
}

int su2_nn_num_params(void) { return kNNParams; }

int su2_nn_create(su2_nn **out, const float *params_host, uint64_t seed, void *hip_stream)
{
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    su2_nn *n = new (std::nothrow) su2_nn();
    if (!n) return fail(SU2_ENOMEM, "host allocation failed");
    n->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
    float **bufs[] = {&n->b.params, &n->b.grad, &n->b.m, &n->b.v};
    for (float **pp : bufs)
        if (e == hipSuccess) e = hipMalloc(pp, kNNParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->b.table, (size_t)kNNRows * kNNRow * sizeof(float));
    std::vector<float> init;
    if (!params_host) nn_default_params(seed, init);
    const float *src = params_host ? params_host : init.data();
    if (e == hipSuccess)
        e = hipMemcpy(n->b.params, src, kNNParams * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->b.m, 0, kNNParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->b.v, 0, kNNParams * sizeof(float));
    if (e != hipSuccess) {
        nn_free(n);
        delete n;
        return fail(SU2_EHIP, std::string("nn_create: ") + hipGetErrorString(e));
    }
    *out = n;
    return SU2_OK;
}

int su2_nn_destroy(su2_nn *n)
{
    if (!n) return fail(SU2_EINVAL, "nn is NULL");
    (void)hipStreamSynchronize(n->stream);
    nn_free(n);
    delete n;
    return SU2_OK;
}

int su2_nn_get_params(su2_nn *n, float *host)
{
    if (!n || !host) return fail(SU2_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(n->stream));
    HIP_TRY(hipMemcpy(host, n->b.params, kNNParams * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
}

int su2_nn_set_params(su2_nn *n, const float *host)
{
    if (!n || !host) return fail(SU2_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(n->stream));
    HIP_TRY(hipMemcpy(n->b.params, host, kNNParams * sizeof(float), hipMemcpyHostToDevice));
    n->table_ready = false;
    return SU2_OK;
}

static int nn_reserve_data(su2_nn *n, int64_t count)
{
    if (n->b.alpha) (void)hipFree(n->b.alpha);
    n->b.alpha = n->b.a0 = nullptr;
    n->ndata = 0;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, (size_t)count * 2 * sizeof(float)));
    n->b.alpha = static_cast<float *>(p);
    n->b.a0 = n->b.alpha + count;
    n->ndata = count;
    return SU2_OK;
}

int su2_nn_sample_data(su2_nn *n, int64_t count, double alpha_lo, double alpha_hi, uint64_t seed)
{
    if (!n) return fail(SU2_EINVAL, "nn is NULL");
    if (count <= 0 || count >= ((int64_t)1 << 32)) return fail(SU2_EINVAL, "count out of range");
    if (!(alpha_lo > 0.0) || !(alpha_hi > alpha_lo) || !std::isfinite(alpha_hi))
        return fail(SU2_EINVAL, "need 0 < alpha_lo < alpha_hi");
    int rc = nn_reserve_data(n, count);
    if (rc) return rc;
    HIP_TRY(launch_nn_data(n->b.alpha, n->b.a0, count, (float)alpha_lo, (float)alpha_hi, seed,
                           n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SU2_OK;
}

int su2_nn_set_data(su2_nn *n, int64_t count, const float *alpha_host, const float *a0_host)
{
    if (!n || !alpha_host || !a0_host || count <= 0) return fail(SU2_EINVAL, "bad arguments");
    int rc = nn_reserve_data(n, count);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(n->b.alpha, alpha_host, count * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(n->b.a0, a0_host, count * sizeof(float), hipMemcpyHostToDevice));
    return SU2_OK;
}

int su2_nn_get_data(su2_nn *n, int64_t *count, float *alpha_host, float *a0_host)
{
    if (!n || !count) return fail(SU2_EINVAL, "bad arguments");
    *count = n->ndata;
    HIP_TRY(hipStreamSynchronize(n->stream));
    if (alpha_host && n->ndata)
        HIP_TRY(hipMemcpy(alpha_host, n->b.alpha, n->ndata * sizeof(float), hipMemcpyDeviceToHost));
    if (a0_host && n->ndata)
        HIP_TRY(hipMemcpy(a0_host, n->b.a0, n->ndata * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
}

static int nn_reserve_act(su2_nn *n, int batch)
{
    if (batch <= n->act_cap) return SU2_OK;
    if (n->b.act) (void)hipFree(n->b.act);
    n->b.act = n->b.loss = nullptr;
    n->act_cap = 0;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, (size_t)batch * (kNNActRows + 1) * sizeof(float)));
    n->b.act = static_cast<float *>(p);
    n->b.loss = n->b.act + (size_t)batch * kNNActRows;
    n->act_cap = batch;
    return SU2_OK;
}

int su2_nn_loss_grad(su2_nn *n, int64_t offset, int32_t batch, double *loss, float *grad_host)
{
    if (!n || batch <= 0 || offset < 0) return fail(SU2_EINVAL, "bad arguments");
    if (!n->ndata) return fail(SU2_ESTATE, "no training data");
    int rc = nn_reserve_act(n, batch);
    if (rc) return rc;
    if (n->loss_cap < 1) {
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, sizeof(double)));
        n->dev_loss = static_cast<double *>(p);
        n->loss_cap = 1;
    }
    HIP_TRY(launch_nn_step(n->b, offset % n->ndata, batch, n->ndata, n->dev_loss, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    if (loss) HIP_TRY(hipMemcpy(loss, n->dev_loss, sizeof(double), hipMemcpyDeviceToHost));
    if (grad_host)
        HIP_TRY(hipMemcpy(grad_host, n->b.grad, kNNParams * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
}

int su2_nn_train(su2_nn *n, int32_t steps, int32_t batch, double lr, double *loss_history_host)
{
    if (!n || steps < 0 || batch <= 0 || !(lr > 0.0)) return fail(SU2_EINVAL, "bad arguments");
    if (!n->ndata) return fail(SU2_ESTATE, "no training data");
    int rc = nn_reserve_act(n, batch);
    if (rc) return rc;
    if (n->loss_cap < steps) {
        if (n->dev_loss) (void)hipFree(n->dev_loss);
        n->dev_loss = nullptr;
        n->loss_cap = 0;
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, (size_t)std::max(steps, 1) * sizeof(double)));
        n->dev_loss = static_cast<double *>(p);
        n->loss_cap = std::max(steps, 1);
    }
    int64_t offset = 0;
    for (int32_t t = 0; t < steps; ++t) {
        HIP_TRY(launch_nn_step(n->b, offset, batch, n->ndata,
                               loss_history_host ? n->dev_loss + t : nullptr, n->stream));
        HIP_TRY(launch_nn_adam(n->b, (float)lr, ++n->step, n->stream));
        offset = (offset + batch) % n->ndata;
    }
    n->table_ready = false;
    if (loss_history_host && steps > 0) {
        HIP_TRY(hipStreamSynchronize(n->stream));
        HIP_TRY(hipMemcpy(loss_history_host, n->dev_loss, steps * sizeof(double),
                          hipMemcpyDeviceToHost));
    }
    HIP_TRY(hipStreamSynchronize(n->stream));
    return SU2_OK;
}

int su2_nn_build_table(su2_nn *n)
{
    if (!n) return fail(SU2_EINVAL, "nn is NULL");
    HIP_TRY(launch_nn_table(n->b.params, n->b.table, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    n->table_ready = true;
    return SU2_OK;
}

int su2_nn_get_table(su2_nn *n, float *host)
{
    if (!n || !host) return fail(SU2_EINVAL, "NULL argument");
    if (!n->table_ready) return fail(SU2_ESTATE, "table not built (su2_nn_build_table)");
    HIP_TRY(hipMemcpy(host, n->b.table, (size_t)kNNRows * kNNRow * sizeof(float),
                      hipMemcpyDeviceToHost));
    return SU2_OK;
}

int su2_set_proposal(su2_ctx *c, su2_nn *n)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (n && !n->table_ready) return fail(SU2_ESTATE, "table not built (su2_nn_build_table)");
    c->table = n ? n->b.table : nullptr;
    return SU2_OK;
}

int su2_get_accept_stats(su2_ctx *c, uint64_t *proposed, uint64_t *accepted, int reset)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    unsigned long long *slot = reinterpret_cast<unsigned long long *>(c->results() + 4);
    HIP_TRY(launch_counts(c->sums(), slot, reset, c->stream));
    unsigned long long v[2] = {0ull, 0ull};
    HIP_TRY(hipMemcpyAsync(v, slot, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (proposed) *proposed = v[0];
    if (accepted) *accepted = v[1];
    return SU2_OK;
}

int su2_test_learned_links(su2_nn *n, const float *V_host, const float *Uold_host, int64_t count,
                           double beta, uint64_t seed, uint32_t sweep, uint32_t mu,
                           uint32_t replica, float *out_host, int32_t *accepted_host)
{
    if (!n || count < 0 || (count > 0 && (!V_host || !Uold_host || !out_host)))
        return fail(SU2_EINVAL, "bad arguments");
    if (!n->table_ready) return fail(SU2_ESTATE, "table not built (su2_nn_build_table)");
    if (count >= ((int64_t)1 << 32) || mu > 3) return fail(SU2_EINVAL, "bad count or mu");
    if (count == 0) return SU2_OK;
    const size_t bytes = (size_t)count * 16;
    void *dv = nullptr, *du = nullptr, *dout = nullptr, *dacc = nullptr;
    hipError_t e = hipMalloc(&dv, bytes);
    if (e == hipSuccess) e = hipMalloc(&du, bytes);
    if (e == hipSuccess) e = hipMalloc(&dout, bytes);
    if (e == hipSuccess && accepted_host) e = hipMalloc(&dacc, (size_t)count * 4);
    if (e == hipSuccess) e = hipMemcpy(dv, V_host, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(du, Uold_host, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_test_learned(n->b.table, (const float *)dv, (const float *)du, count,
                                (float)beta, seed, sweep, mu, replica, (float *)dout,
                                (int32_t *)dacc, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out_host, dout, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && accepted_host)
        e = hipMemcpy(accepted_host, dacc, (size_t)count * 4, hipMemcpyDeviceToHost);
    void *bufs[] = {dv, du, dout, dacc};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    if (e != hipSuccess) return fail(SU2_EHIP, std::string("test_learned: ") + hipGetErrorString(e));
    return SU2_OK;
}

}  // extern "C"

