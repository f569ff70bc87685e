// su3_runtime.cpp -- C ABI of the SU(3) heat bath in libsu2: argument checks,
// device memory, the sweep schedule (Sec. 4: per direction, even sites then
// odd sites), the measurements and the host exchange of links.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <memory>
#include <new>
#include <string>

#include "../../include/su3.h"
#include "su3_internal.h"
#include "su2_api.h"

using namespace su2rt;
using namespace su3rt;

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));              \
            return SU2_EHIP;                                                            \
        }                                                                               \
    } while (0)

// HIP_TRY for one of several asynchronous copies into a host buffer: on failure
// the copies already enqueued are waited for before the buffer goes away.
#define HIP_TRY_DRAIN(expr, strm)                                                       \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));              \
            (void)hipStreamSynchronize(strm);                                           \
            return SU2_EHIP;                                                            \
        }                                                                               \
    } while (0)

struct su3_ctx {
    int32_t dims[4] = {0, 0, 0, 0};
    int32_t nrep = 1;  // replicas (a batch; 1 for a single lattice)
    Lat3 L{};
    Launch3 cfg;
    uint32_t lg_tz = 3, lg_tt = 3;
    hipStream_t stream = nullptr;
    uint64_t seed = 0;
    uint32_t sweep = 0;  // host copy of the device sweep index L.ctr[0]
    void *links_mem = nullptr;
    void *scratch_mem = nullptr;
    // captured sweeps (su3_capture_sweeps): the graph, its sweeps per replay,
    // reunitarisation period, and history rows written / available
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int32_t g_ns = 0, g_reunit = 0;
    bool g_meas = false;
    int64_t g_rows_cap = 0, g_rows_next = 0;
};

// A batch of replicas with common extents: the context with nrep > 1 (its own
// C type, so that single-lattice entry points refuse it at compile time).
struct su3_batch : su3_ctx {};

namespace {

constexpr size_t kScratch3 = kAccBytes + (size_t)kRes3 * 8 + (size_t)kHist3 * 8 + 256;
// scratch of one replica (accumulators, results, history, counters)
constexpr size_t kStride3 = (kScratch3 + 255) & ~(size_t)255;

int64_t volume3(const int32_t *d) { return (int64_t)d[0] * d[1] * d[2] * d[3]; }

int check3(su3_ctx *c)
{
    if (!c) return fail(SU2_EINVAL, "context is NULL");
    return SU2_OK;
}

void drop_graph(su3_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_ns = c->g_reunit = 0;
    c->g_meas = false;
    c->g_rows_cap = c->g_rows_next = 0;
}

// The eight passes of one heat-bath sweep, its end-of-sweep kernel (history
// row, sweep index) and the reunitarisation when the sweep completes a period.
// flags: as launch_su3_finish (8 is always added).
int enqueue_sweep(su3_ctx *c, const Lat3 &L, bool measure, int flags, int row,
                  int32_t reunit_every, uint32_t sweep)
{
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par)
            HIP_TRY(launch_su3_pass(L, mu, par, c->seed, measure && par == 1 && mu >= 1, c->cfg,
                                    c->stream));
    HIP_TRY(launch_su3_finish(L, flags | 8, row, c->stream));
    if (reunit_every > 0 && (sweep + 1u) % (uint32_t)reunit_every == 0u)
        HIP_TRY(launch_su3_reunit(L, c->stream));
    return SU2_OK;
}

int lg_tile(int tile, uint32_t cur, uint32_t *out)
{
    if (tile == 0) {
        *out = cur;
        return SU2_OK;
    }
    if (tile < 0 || (tile & (tile - 1)) || tile > 256)
        return fail(SU2_EINVAL, "tile sizes must be powers of two <= 256");
    uint32_t l = 0;
    while ((1 << l) < tile) ++l;
    *out = l;
    return SU2_OK;
}

// Totals of the accumulators (flags 1 plaquette, 2 Polyakov) into the result
// slots, then nres slots from `first` of every replica copied to the host
// (host[r * nres + i]).
int finish_to_host(su3_ctx *c, int flags, int first, int nres, double *host)
{
    HIP_TRY(launch_su3_finish(c->L, flags, 0, c->stream));
    HIP_TRY(hipMemcpy2DAsync(host, sizeof(double) * (size_t)nres, c->L.results + first, kStride3,
                             sizeof(double) * (size_t)nres, (size_t)c->nrep,
                             hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SU2_OK;
}

// Coordinates of canonical site s.
void coords(const int32_t *d, int64_t s, int c[4])
{
    for (int i = 0; i < 4; ++i) {
        c[i] = (int)(s % d[i]);
        s /= d[i];
    }
}

}  // namespace

extern "C" {

size_t su3_links_bytes(const int32_t dims[4])
{
    SU2_API_BEGIN
    if (!dims) return 0;
    const std::string keep = su2_last_error();  // a size query is not a failure
    const int rc = check_dims(dims);
    set_error(keep);
    if (rc) return 0;
    return (size_t)volume3(dims) * 192u;
    SU2_API_END_SIZE
}

}  // extern "C"

namespace {

void release3(su3_ctx *c)
{
    if (c->links_mem || c->scratch_mem) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->links_mem) (void)hipFree(c->links_mem);
    if (c->scratch_mem) (void)hipFree(c->scratch_mem);
    c->links_mem = c->scratch_mem = nullptr;
}

// Device memory and hot/cold start of n replicas of extents dims: couplings
// betas[r] (nullptr: beta for the single lattice), Philox replica ids 0..n-1.
// On failure the caller releases c.
int init3(su3_ctx *c, int32_t n, const int32_t dims[4], const double *betas, double beta,
          uint64_t seed, int start, void *hip_stream)
{
    int rc = check_dims(dims);
    if (rc) return rc;
    if (betas) {
        for (int32_t r = 0; r < n; ++r)
            if (!beta_ok(betas[r])) return fail(SU2_EINVAL, "every beta must be finite and >= 0");
    } else if (!beta_ok(beta)) {
        return fail(SU2_EINVAL, "beta must be finite and >= 0");
    }
    if (start != SU2_COLD && start != SU2_HOT) return fail(SU2_EINVAL, "start must be COLD or HOT");
    for (int i = 0; i < 4; ++i) c->dims[i] = dims[i];
    c->nrep = n;
    c->L.g = make_geom(dims, c->lg_tz, c->lg_tt);
    if (!geom_selfcheck(c->L.g)) return fail(SU2_ERANGE, "index arithmetic self-check failed");
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->seed = seed;
    c->L.beta = (float)(betas ? betas[0] : beta);
    c->L.replica = 0u;
    c->L.nrep = (uint32_t)n;
    c->L.link_stride = (size_t)volume3(dims) * 12u;
    c->L.scratch_stride = kStride3;
    const size_t beta_bytes = betas ? sizeof(float) * (size_t)n : 0;
    hipError_t e = hipMalloc(&c->links_mem, su3_links_bytes(dims) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&c->scratch_mem, kStride3 * (size_t)n + beta_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(c->scratch_mem, 0, kStride3 * (size_t)n, c->stream);
    std::unique_ptr<float[]> bf;
    if (e == hipSuccess && betas) {
        bf.reset(new (std::nothrow) float[(size_t)n]);
        if (!bf) return fail(SU2_ENOMEM, "host staging of the couplings");
        for (int32_t r = 0; r < n; ++r) bf[r] = (float)betas[r];
        float *bd = reinterpret_cast<float *>(static_cast<unsigned char *>(c->scratch_mem) +
                                              kStride3 * (size_t)n);
        e = hipMemcpyAsync(bd, bf.get(), beta_bytes, hipMemcpyHostToDevice, c->stream);
        c->L.betas = bd;
    }
    if (e == hipSuccess) {
        c->L.links = static_cast<float4 *>(c->links_mem);
        c->L.acc = static_cast<unsigned long long *>(c->scratch_mem);
        c->L.results = reinterpret_cast<double *>(static_cast<unsigned char *>(c->scratch_mem) +
                                                  kAccBytes);
        c->L.hist = c->L.results + kRes3;
        c->L.ctr = reinterpret_cast<uint32_t *>(c->L.hist + kHist3);  // zeroed above
        e = launch_su3_init(c->L, start, seed, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // bf outlives its copy
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? SU2_ENOMEM : SU2_EHIP,
                    std::string("su3 init: ") + hipGetErrorString(e));
    return SU2_OK;
}

}  // namespace

extern "C" {

int su3_init(su3_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
             void *hip_stream)
{
    SU2_API_BEGIN
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    su3_ctx *c = new (std::nothrow) su3_ctx();
    if (!c) return fail(SU2_ENOMEM, "host allocation failed");
    const int rc = init3(c, 1, dims, nullptr, beta, seed, start, hip_stream);
    if (rc) {
        release3(c);
        delete c;
        return rc;
    }
    *out = c;
    return SU2_OK;
    SU2_API_END
}

int su3_destroy(su3_ctx *c)
{
    SU2_API_BEGIN
    if (!c) return fail(SU2_EINVAL, "context is NULL");
    release3(c);
    delete c;
    return SU2_OK;
    SU2_API_END
}

int su3_batch_init(su3_batch **out, int32_t n, const int32_t dims[4], const double *betas,
                   uint64_t seed, int start, void *hip_stream)
{
    SU2_API_BEGIN
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 65535) return fail(SU2_EINVAL, "n must be in [1, 65535]");
    if (!betas) return fail(SU2_EINVAL, "betas is NULL");
    su3_batch *b = new (std::nothrow) su3_batch();
    if (!b) return fail(SU2_ENOMEM, "host allocation failed");
    const int rc = init3(b, n, dims, betas, 0.0, seed, start, hip_stream);
    if (rc) {
        release3(b);
        delete b;
        return rc;
    }
    *out = b;
    return SU2_OK;
    SU2_API_END
}

int su3_batch_destroy(su3_batch *b)
{
    SU2_API_BEGIN
    if (!b) return fail(SU2_EINVAL, "batch is NULL");
    release3(b);
    delete b;
    return SU2_OK;
    SU2_API_END
}

int su3_batch_size(su3_batch *b, int32_t *n)
{
    SU2_API_BEGIN
    if (!b || !n) return fail(SU2_EINVAL, "batch or n is NULL");
    *n = b->nrep;
    return SU2_OK;
    SU2_API_END
}

}  // extern "C"

namespace {

// Enqueue nsweeps sweeps of every replica; plaq_hist (host, may be NULL)
// receives the plaquette after each sweep, row j holding the nrep replicas.
int heatbath3(su3_ctx *c, int32_t nsweeps, int32_t reunit_every, double *plaq_hist)
{
    int rc;
    if (nsweeps < 0 || reunit_every < 0)
        return fail(SU2_EINVAL, "nsweeps and reunit_every must be >= 0");
    const size_t nr = (size_t)c->nrep;
    std::unique_ptr<double[]> stage;
    if (plaq_hist && nr > 1) {
        stage.reset(new (std::nothrow) double[nr * (size_t)std::min<int32_t>(nsweeps, kHist3)]);
        if (!stage) return fail(SU2_ENOMEM, "host staging of the plaquette history");
    }
    int32_t done = 0;
    while (done < nsweeps) {
        const int32_t chunk = plaq_hist ? std::min<int32_t>(nsweeps - done, kHist3)
                                        : nsweeps - done;
        for (int32_t j = 0; j < chunk; ++j) {
            if ((rc = enqueue_sweep(c, c->L, plaq_hist != nullptr, plaq_hist ? 1 | 4 : 0, j,
                                    reunit_every, c->sweep)))
                return rc;
            ++c->sweep;
        }
        if (plaq_hist && nr == 1) {
            HIP_TRY(hipMemcpyAsync(plaq_hist + done, c->L.hist, sizeof(double) * (size_t)chunk,
                                   hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        } else if (plaq_hist) {
            // replica r's rows sit in its own scratch: [r][j] staged, then [j][r]
            const size_t w = sizeof(double) * (size_t)chunk;
            HIP_TRY(hipMemcpy2DAsync(stage.get(), w, c->L.hist, kStride3, w, nr,
                                     hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            for (size_t r = 0; r < nr; ++r)
                for (int32_t j = 0; j < chunk; ++j)
                    plaq_hist[(size_t)(done + j) * nr + r] = stage[r * (size_t)chunk + (size_t)j];
        }
        done += chunk;
    }
    return SU2_OK;
}

int overrelax3(su3_ctx *c, int32_t nsweeps)
{
    if (nsweeps < 0) return fail(SU2_EINVAL, "nsweeps must be >= 0");
    for (int32_t j = 0; j < nsweeps; ++j)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par)
                HIP_TRY(launch_su3_pass(c->L, mu, par, c->seed, false, c->cfg, c->stream, true));
    return SU2_OK;
}

int plaquette3(su3_ctx *c, double *out)
{
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    HIP_TRY(launch_su3_plaquette(c->L, c->stream));
    return finish_to_host(c, 1, R3_PLAQ, 1, out);
}

int polyakov3(su3_ctx *c, double *out)
{
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    HIP_TRY(launch_su3_polyakov(c->L, c->stream));
    return finish_to_host(c, 2, R3_POLY_RE, 3, out);
}

}  // namespace

extern "C" {

int su3_heatbath_sweep(su3_ctx *c, int32_t nsweeps, int32_t reunit_every, double *plaq_hist)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return heatbath3(c, nsweeps, reunit_every, plaq_hist);
    SU2_API_END
}

int su3_overrelax(su3_ctx *c, int32_t nsweeps)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return overrelax3(c, nsweeps);
    SU2_API_END
}

int su3_reunitarize(su3_ctx *c)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    HIP_TRY(launch_su3_reunit(c->L, c->stream));
    return SU2_OK;
    SU2_API_END
}

int su3_plaquette(su3_ctx *c, double *out)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return plaquette3(c, out);
    SU2_API_END
}

int su3_polyakov(su3_ctx *c, double *out)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return polyakov3(c, out);
    SU2_API_END
}

}  // extern "C"

namespace {

// Links of replica r as full FP64 matrices (host layout of su3.h).
int get_links3(su3_ctx *c, int32_t r, double *host)
{
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    if (r < 0 || r >= c->nrep) return fail(SU2_EINVAL, "replica out of range");
    const int64_t V = volume3(c->dims), vh = V / 2;
    const size_t n = (size_t)V * 48u;
    std::unique_ptr<float[]> dev(new (std::nothrow) float[n]);
    if (!dev) return fail(SU2_ENOMEM, "host staging buffer of " + std::to_string(4 * n) + " B");
    HIP_TRY(hipMemcpyAsync(dev.get(), c->L.links + (size_t)r * c->L.link_stride,
                           n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    typedef std::complex<double> cd;
    for (int64_t s = 0; s < V; ++s) {
        int x[4];
        coords(c->dims, s, x);
        const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
        const int64_t h = s >> 1;
        for (int mu = 0; mu < 4; ++mu) {
            float f[12];
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 4; ++j)
                    f[4 * k + j] = dev[(((size_t)(mu * 2 + par) * 3 + (size_t)k) * (size_t)vh +
                                        (size_t)h) * 4u + (size_t)j];
            cd m[3][3];
            for (int e = 0; e < 6; ++e) m[e / 3][e % 3] = cd(f[2 * e], f[2 * e + 1]);
            m[2][0] = std::conj(m[0][1] * m[1][2] - m[0][2] * m[1][1]);
            m[2][1] = std::conj(m[0][2] * m[1][0] - m[0][0] * m[1][2]);
            m[2][2] = std::conj(m[0][0] * m[1][1] - m[0][1] * m[1][0]);
            double *o = host + ((size_t)s * 4 + (size_t)mu) * 18;
            for (int e = 0; e < 9; ++e) {
                o[2 * e] = m[e / 3][e % 3].real();
                o[2 * e + 1] = m[e / 3][e % 3].imag();
            }
        }
    }
    return SU2_OK;
}

// Replica r's links from full matrices (rows 0 and 1 are stored).
int set_links3(su3_ctx *c, int32_t r, const double *host)
{
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    if (r < 0 || r >= c->nrep) return fail(SU2_EINVAL, "replica out of range");
    const int64_t V = volume3(c->dims), vh = V / 2;
    const size_t n = (size_t)V * 48u;
    std::unique_ptr<float[]> dev(new (std::nothrow) float[n]);
    if (!dev) return fail(SU2_ENOMEM, "host staging buffer of " + std::to_string(4 * n) + " B");
    for (int64_t s = 0; s < V; ++s) {
        int x[4];
        coords(c->dims, s, x);
        const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
        const int64_t h = s >> 1;
        for (int mu = 0; mu < 4; ++mu) {
            const double *in = host + ((size_t)s * 4 + (size_t)mu) * 18;  // rows 0, 1 = 12 reals
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 4; ++j)
                    dev[(((size_t)(mu * 2 + par) * 3 + (size_t)k) * (size_t)vh + (size_t)h) * 4u +
                        (size_t)j] = (float)in[4 * k + j];
        }
    }
    HIP_TRY(hipMemcpyAsync(c->L.links + (size_t)r * c->L.link_stride, dev.get(),
                           n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SU2_OK;
}

}  // namespace

extern "C" {

int su3_get_links(su3_ctx *c, double *host)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return get_links3(c, 0, host);
    SU2_API_END
}

int su3_set_links(su3_ctx *c, const double *host)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return set_links3(c, 0, host);
    SU2_API_END
}

int su3_get_sweep(su3_ctx *c, uint32_t *out)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = c->sweep;
    return SU2_OK;
    SU2_API_END
}

int su3_set_sweep(su3_ctx *c, uint32_t sweep)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    HIP_TRY(launch_su3_set_counter(c->L, sweep, 0, c->stream));
    c->sweep = sweep;
    return SU2_OK;
    SU2_API_END
}

int su3_set_beta(su3_ctx *c, double beta)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (!beta_ok(beta)) return fail(SU2_EINVAL, "beta must be finite and >= 0");
    c->L.beta = (float)beta;
    drop_graph(c);  // the captured kernels hold the old coupling
    return SU2_OK;
    SU2_API_END
}

}  // extern "C"

namespace {

int set_launch3(su3_ctx *c, int block, int remap, int snake, int tile_z, int tile_t)
{
    int rc;
    if (block != 64 && block != 128 && block != 192 && block != 256)
        return fail(SU2_EINVAL, "block must be 64, 128, 192 or 256");
    uint32_t lz, lt;
    if ((rc = lg_tile(tile_z, c->lg_tz, &lz)) || (rc = lg_tile(tile_t, c->lg_tt, &lt))) return rc;
    const Geom g = make_geom(c->dims, lz, lt);
    if (!geom_selfcheck(g)) return fail(SU2_ERANGE, "index arithmetic self-check failed");
    HIP_TRY(hipStreamSynchronize(c->stream));  // passes already enqueued keep their launch
    c->cfg.block = block;
    c->cfg.remap = remap != 0;
    c->cfg.snake = snake != 0;
    c->lg_tz = lz;
    c->lg_tt = lt;
    c->L.g = g;
    drop_graph(c);
    return SU2_OK;
}

int check_batch3(su3_batch *b)
{
    if (!b) return fail(SU2_EINVAL, "batch is NULL");
    return SU2_OK;
}

}  // namespace

extern "C" {

int su3_set_launch(su3_ctx *c, int block, int remap, int snake, int tile_z, int tile_t)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    return set_launch3(c, block, remap, snake, tile_z, tile_t);
    SU2_API_END
}

int su3_set_replica(su3_ctx *c, uint32_t replica)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (replica >= (1u << 26)) return fail(SU2_EINVAL, "replica id must be < 2^26");
    c->L.replica = replica;
    drop_graph(c);  // the captured kernels hold the old replica id
    return SU2_OK;
    SU2_API_END
}

int su3_batch_heatbath_sweep(su3_batch *b, int32_t nsweeps, int32_t reunit_every,
                             double *plaq_hist)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return heatbath3(b, nsweeps, reunit_every, plaq_hist);
    SU2_API_END
}

int su3_batch_overrelax(su3_batch *b, int32_t nsweeps)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return overrelax3(b, nsweeps);
    SU2_API_END
}

int su3_batch_reunitarize(su3_batch *b)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    HIP_TRY(launch_su3_reunit(b->L, b->stream));
    return SU2_OK;
    SU2_API_END
}

int su3_batch_plaquette(su3_batch *b, double *out)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return plaquette3(b, out);
    SU2_API_END
}

int su3_batch_polyakov(su3_batch *b, double *out)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return polyakov3(b, out);
    SU2_API_END
}

int su3_batch_get_links(su3_batch *b, int32_t r, double *host)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return get_links3(b, r, host);
    SU2_API_END
}

int su3_batch_set_links(su3_batch *b, int32_t r, const double *host)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return set_links3(b, r, host);
    SU2_API_END
}

int su3_batch_get_sweep(su3_batch *b, uint32_t *out)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return su3_get_sweep(b, out);
    SU2_API_END
}

int su3_batch_set_sweep(su3_batch *b, uint32_t sweep)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return su3_set_sweep(b, sweep);
    SU2_API_END
}

int su3_batch_set_launch(su3_batch *b, int block, int remap, int snake, int tile_z, int tile_t)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    return set_launch3(b, block, remap, snake, tile_z, tile_t);
    SU2_API_END
}

int su3_batch_synchronize(su3_batch *b)
{
    SU2_API_BEGIN
    int rc = check_batch3(b);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SU2_OK;
    SU2_API_END
}

int su3_links_device(su3_ctx *c, void **links_dev, void **hip_stream)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (links_dev) *links_dev = c->L.links;
    if (hip_stream) *hip_stream = c->stream;
    return SU2_OK;
    SU2_API_END
}

int su3_synchronize(su3_ctx *c)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SU2_OK;
    SU2_API_END
}

int su3_test_pass(su3_ctx *c, int mu, int parity)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (mu < 0 || mu > 3 || parity < 0 || parity > 1)
        return fail(SU2_EINVAL, "mu must be 0..3 and parity 0..1");
    HIP_TRY(launch_su3_pass(c->L, mu, parity, c->seed, false, c->cfg, c->stream));
    return SU2_OK;
    SU2_API_END
}

int su3_test_read_links(su3_ctx *c, int64_t n, const int64_t *sites, int mu, double *out)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!sites || !out)) || mu < 0 || mu > 3)
        return fail(SU2_EINVAL, "n >= 0, non-NULL sites and out, mu 0..3");
    const int64_t V = volume3(c->dims), vh = V / 2;
    std::unique_ptr<float[]> buf(new (std::nothrow) float[(size_t)n * 12u + 1u]);
    if (!buf) return fail(SU2_ENOMEM, "host buffer for the sampled links");
    for (int64_t i = 0; i < n; ++i)
        if (sites[i] < 0 || sites[i] >= V) return fail(SU2_EINVAL, "site out of range");
    for (int64_t i = 0; i < n; ++i) {
        int x[4];
        coords(c->dims, sites[i], x);
        const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
        for (int k = 0; k < 3; ++k) {
            const float4 *src = c->L.links + ((size_t)(mu * 2 + par) * 3 + (size_t)k) * (size_t)vh +
                                (size_t)(sites[i] >> 1);
            HIP_TRY_DRAIN(hipMemcpyAsync(buf.get() + 12 * i + 4 * k, src, sizeof(float4),
                                         hipMemcpyDeviceToHost, c->stream), c->stream);
        }
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    typedef std::complex<double> cd;
    for (int64_t i = 0; i < n; ++i) {
        const float *f = buf.get() + 12 * i;
        cd m[3][3];
        for (int e = 0; e < 6; ++e) m[e / 3][e % 3] = cd(f[2 * e], f[2 * e + 1]);
        m[2][0] = std::conj(m[0][1] * m[1][2] - m[0][2] * m[1][1]);
        m[2][1] = std::conj(m[0][2] * m[1][0] - m[0][0] * m[1][2]);
        m[2][2] = std::conj(m[0][0] * m[1][1] - m[0][1] * m[1][0]);
        for (int e = 0; e < 9; ++e) {
            out[18 * i + 2 * e] = m[e / 3][e % 3].real();
            out[18 * i + 2 * e + 1] = m[e / 3][e % 3].imag();
        }
    }
    return SU2_OK;
    SU2_API_END
}

int su3_test_or_pass(su3_ctx *c, int mu, int parity)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (mu < 0 || mu > 3 || parity < 0 || parity > 1)
        return fail(SU2_EINVAL, "mu must be 0..3 and parity 0..1");
    HIP_TRY(launch_su3_pass(c->L, mu, parity, c->seed, false, c->cfg, c->stream, true));
    return SU2_OK;
    SU2_API_END
}

int su3_capture_sweeps(su3_ctx *c, int32_t nsweeps, int32_t reunit_every, int meas,
                       double *dev_history, int64_t history_rows)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (nsweeps <= 0 || reunit_every < 0)
        return fail(SU2_EINVAL, "nsweeps must be > 0 and reunit_every >= 0");
    if (meas != 0 && meas != 1) return fail(SU2_EINVAL, "meas must be 0 or 1 (plaquette)");
    if (meas && (!dev_history || history_rows < nsweeps))
        return fail(SU2_EINVAL, "a measured capture needs dev_history with >= nsweeps rows");
    if (reunit_every > 0 &&
        (nsweeps % reunit_every != 0 || c->sweep % (uint32_t)reunit_every != 0u))
        return fail(SU2_EINVAL, "with reunitarisation the captured sweeps must span whole "
                                "periods starting at a period boundary");
    if (!c->stream) return fail(SU2_ESTATE, "capture needs a non-null stream");
    drop_graph(c);
    HIP_TRY(launch_su3_set_counter(c->L, 0u, 1, c->stream));  // history row of the replays
    HIP_TRY(hipStreamSynchronize(c->stream));
    Lat3 Lg = c->L;
    if (meas) Lg.hist = dev_history;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int32_t j = 0; j < nsweeps && rc == SU2_OK; ++j)
        rc = enqueue_sweep(c, Lg, meas != 0, meas ? 1 | 4 | 16 : 0, 0, reunit_every,
                           c->sweep + (uint32_t)j);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ee != hipSuccess) return fail(SU2_EHIP, std::string("hipStreamEndCapture: ") +
                                                    hipGetErrorString(ee));
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SU2_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    c->graph = g;
    c->gexec = x;
    c->g_ns = nsweeps;
    c->g_reunit = reunit_every;
    c->g_meas = meas != 0;
    c->g_rows_cap = meas ? history_rows : 0;
    c->g_rows_next = 0;
    return SU2_OK;
    SU2_API_END
}

int su3_replay_sweeps(su3_ctx *c, int32_t count)
{
    SU2_API_BEGIN
    int rc = check3(c);
    if (rc) return rc;
    if (!c->gexec) return fail(SU2_ESTATE, "no captured sweeps");
    if (count < 0) return fail(SU2_EINVAL, "count must be >= 0");
    if (c->g_reunit > 0 && c->sweep % (uint32_t)c->g_reunit != 0u)
        return fail(SU2_ESTATE, "replay must start at a reunitarisation period boundary");
    if (c->g_meas && c->g_rows_next + (int64_t)count * c->g_ns > c->g_rows_cap)
        return fail(SU2_EINVAL, "the replays would write history rows past the " +
                                    std::to_string(c->g_rows_cap) + " captured rows");
    for (int32_t i = 0; i < count; ++i) HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
    c->sweep += (uint32_t)count * (uint32_t)c->g_ns;
    if (c->g_meas) c->g_rows_next += (int64_t)count * c->g_ns;
    return SU2_OK;
    SU2_API_END
}

}  // extern "C"
