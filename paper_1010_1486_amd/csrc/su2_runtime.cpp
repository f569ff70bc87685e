// su2_runtime.cpp -- C ABI of libsu2: ensembles of lattices (a single lattice
// is an ensemble of one), argument checks, memory, the sweep schedule (Sec. 4:
// per direction, even sites then odd sites), measurements, hipGraph capture of
// sweeps and the launch autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/su2.h"
#include "su2_internal.h"
#include "su3_internal.h"
#include "su2_api.h"

using su2dev::Geom;
using su2dev::kNNRow;
using su2dev::kNNRows;

namespace su2rt {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int api_nomem() noexcept
{
    try {
        g_last_error = "host allocation failed";
    } catch (...) {
    }
    return SU2_ENOMEM;
}

int api_unexpected() noexcept
{
    try {
        g_last_error = "unexpected host-side exception";
    } catch (...) {
    }
    return SU2_EINVAL;
}

}  // namespace su2rt

using namespace su2rt;

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

namespace {

// Device position of component k of U_mu at half-site h of parity par: FP32
// links are one array of V/2 float4 per class (mu * 2 + parity); FP64 links
// two arrays of V/2 double pairs per class, (a0, a1) then (a2, a3).
template <typename D>
inline size_t dev_index(int mu, int par, int k, int64_t h, int64_t vh)
{
    if (sizeof(D) == sizeof(double))
        return (((size_t)(mu * 2 + par) * 2u + (size_t)(k >> 1)) * (size_t)vh + (size_t)h) * 2u +
               (size_t)(k & 1);
    return ((size_t)(mu * 2 + par) * (size_t)vh + (size_t)h) * 4u + (size_t)k;
}

}  // namespace

// Argument checks and the lattice geometry, shared with the SU(3) runtime.
namespace su2rt {

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
    // multiply step by step so that huge extents cannot overflow
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        v *= dims[i];
        if (v / 2 >= (int64_t)1 << 28) return fail(SU2_ERANGE, "V/2 must be < 2^28");
    }
    return SU2_OK;
}

}  // namespace su2rt

namespace {

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

}  // namespace

namespace su2rt {

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

}  // namespace su2rt

namespace {

// tile 0 keeps `cur`; else a power of two (the geometry clips it to a divisor).
int lg_of_tile(int tile, uint32_t cur, uint32_t *out)
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

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t volume_of(const int32_t *d) { return (int64_t)d[0] * d[1] * d[2] * d[3]; }

// Pass workgroup slots: replica r owns nblocks[r] = ceil(V/2 / block) slots
// starting at first[r], a multiple of 8 (so that slot mod 8 is the XCD of a
// one-workgroup-per-slot launch); a single lattice has no padding.
uint32_t slot_layout(const std::vector<std::array<int32_t, 4>> &dims, int block,
                     std::vector<uint32_t> &first, std::vector<uint32_t> &nblocks)
{
    const size_t n = dims.size();
    first.resize(n);
    nblocks.resize(n);
    uint32_t fb = 0;
    for (size_t r = 0; r < n; ++r) {
        const uint32_t vh = (uint32_t)(volume_of(dims[r].data()) / 2);
        nblocks[r] = (vh + (uint32_t)block - 1u) / (uint32_t)block;
        first[r] = fb;
        fb += (nblocks[r] + 7u) & ~7u;
    }
    return n > 1 ? fb : nblocks[0];
}

// Work-queue layout over nq queues (one per XCD): replicas in decreasing
// order of slots (ties by index) go to the queue with the fewest slots so
// far (ties: lowest queue); within a queue the replicas' slots are
// contiguous in increasing replica order, qfirst[r] being r's first slot.
void queue_layout(const std::vector<uint32_t> &nblocks, int nq, std::vector<int> &qof,
                  std::vector<uint32_t> &qfirst, std::vector<uint32_t> &qslots)
{
    const size_t n = nblocks.size();
    std::vector<size_t> order(n);
    for (size_t r = 0; r < n; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return nblocks[a] > nblocks[b]; });
    qof.assign(n, 0);
    qslots.assign((size_t)nq, 0u);
    for (size_t r : order) {
        int best = 0;
        for (int q = 1; q < nq; ++q)
            if (qslots[q] < qslots[best]) best = q;
        qof[r] = best;
        qslots[best] += nblocks[r];
    }
    std::vector<uint32_t> fill((size_t)nq, 0u);
    qfirst.assign(n, 0u);
    for (size_t r = 0; r < n; ++r) {
        qfirst[r] = fill[qof[r]];
        fill[qof[r]] += nblocks[r];
    }
}

// XCC ids that run workgroups on the current device (probed once).
int xcc_ids(std::vector<int> &ids)
{
    // one probe per device; contexts on several host threads may race to fill
    // an entry, which is harmless (every probe finds the same mask)
    static std::atomic<uint32_t> masks[64];
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(SU2_ERANGE, "device index out of range");
    uint32_t mask = masks[dev].load(std::memory_order_acquire);
    if (!mask) {
        HIP_TRY(probe_xcc_mask(&mask));
        if (!mask) return fail(SU2_EHIP, "XCC probe found no XCD");
        masks[dev].store(mask, std::memory_order_release);
    }
    ids.clear();
    for (int k = 0; k < kMaxQueues; ++k)
        if (mask & (1u << k)) ids.push_back(k);
    return SU2_OK;
}

}  // namespace

// ================================================================ Ensemble
// n lattices (replicas) with their own extents and couplings, run by the same
// launches.  Device scratch layout: [descriptors][pass workgroup -> replica map
// (n > 1)][per replica: counters, accumulators, result slots].
class Ensemble {
public:
    int n = 0;
    std::vector<std::array<int32_t, 4>> dims;
    std::vector<double> beta;
    std::vector<uint32_t> replica;
    std::vector<float *> links;
    std::vector<Geom> geom;
    std::vector<uint32_t> first_block, nblocks;
    uint32_t total_blocks = 0, max_vh = 0, max_ns3 = 0;
    int poly_s = 1;
    uint32_t plane_hs = 0;  // common (x, y)-plane half-sites, 0 if they differ
    float *pool = nullptr;
    bool own_pool = false;
    unsigned char *scratch = nullptr;
    bool own_scratch = false;
    size_t bmap_off = 0, qmap_off = 0, rep_off = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t seed = 0;
    uint32_t sweep = 0;  // host mirror of the (common) sweep counter
    float orw = -1.0f;   // learned proposal: over-relaxation noise width (< 0: off)
    int n_or = 1;        // SU2_KP_OR: over-relaxation sweeps after each heat-bath sweep
    bool reunit_fused = false;  // reunitarise in the last pass stage of a reunitarisation sweep
    bool f64 = false;    // FP64 links (single lattice): the su2_f64.hip kernels
    uint2 *amap = nullptr;  // XCD-affine pass map (device, owned), see Ens
    uint32_t amap_len = 0;
    LaunchCfg cfg;
    uint32_t lg_tz = 3, lg_tt = 3;
    const float *table = nullptr;
    // captured sweeps
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int32_t g_nsweeps = 0;
    int32_t g_reunit = 0;  // reunitarisation period baked into the graph (0: none)
    bool rows_graph = false;  // enqueue() is being captured: rows on the graph's counter
    MarchShape march{};       // the LDS-staged pass's layout (cfg.march_R > 0)
    int64_t g_rows_cap = 0;   // history rows the capture's buffer holds (0: no history)
    int64_t g_rows_next = 0;  // first row the next replay writes
    // work queue
    bool queue_used = false;           // queue launches since the last error check
    uint32_t spin_limit = 1u << 22;    // polls per bounded wait
    uint32_t queue_grid_auto[2] = {0, 0};  // resident workgroups (heat bath, learned)
    int queue_nq = 1;                      // queues (XCDs)

    // descriptors, then the work-queue state
    static size_t qs_off(int n) { return align_up((size_t)n * sizeof(Rep), 256); }
    static size_t descr_bytes(int n) { return qs_off(n) + align_up(sizeof(QueueState), 256); }
    static size_t bmap_bytes(int n, const std::vector<std::array<int32_t, 4>> &d)
    {
        if (n <= 1) return 0;
        size_t blocks = 0;  // worst case: 64-thread workgroups
        for (auto &x : d) blocks += align_up((size_t)(volume_of(x.data()) / 2 + 63) / 64, 8);
        return align_up(blocks * 4, 256);
    }
    static size_t rep_bytes() { return align_up(kRepScratch, 256); }
    static size_t scratch_need(int n, const std::vector<std::array<int32_t, 4>> &d)
    {
        return descr_bytes(n) + 2 * bmap_bytes(n, d) + (size_t)n * rep_bytes();
    }

    Rep *d_reps() const { return reinterpret_cast<Rep *>(scratch); }
    QueueState *d_qs() const { return reinterpret_cast<QueueState *>(scratch + qs_off(n)); }
    uint32_t *d_qmap() const
    {
        return n > 1 ? reinterpret_cast<uint32_t *>(scratch + qmap_off) : nullptr;
    }
    uint32_t *d_bmap() const
    {
        return n > 1 ? reinterpret_cast<uint32_t *>(scratch + bmap_off) : nullptr;
    }
    unsigned char *rep_scratch(int r) const { return scratch + rep_off + (size_t)r * rep_bytes(); }
    Counters *cnt(int r) const { return reinterpret_cast<Counters *>(rep_scratch(r)); }
    unsigned long long *acc(int r) const
    {
        return reinterpret_cast<unsigned long long *>(rep_scratch(r) + sizeof(Counters));
    }
    double *results(int r) const
    {
        return reinterpret_cast<double *>(rep_scratch(r) + sizeof(Counters) + kAccBytes);
    }

    Ens ens() const
    {
        return Ens{d_reps(), d_bmap(), amap, amap_len, n,
                   total_blocks, max_vh, max_ns3, poly_s, plane_hs};
    }

    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        g_nsweeps = 0;
        g_reunit = 0;
        g_rows_cap = g_rows_next = 0;
    }

    // Geometry, workgroup ranges and descriptors (uploaded synchronously).
    int upload()
    {
        drop_graph();
        geom.resize(n);
        total_blocks = slot_layout(dims, cfg.pass_block, first_block, nblocks);
        max_vh = max_ns3 = 0;
        poly_s = 8;
        for (int r = 0; r < n; ++r) {
            geom[r] = make_geom(dims[r].data(), lg_tz, lg_tt);
            if (!geom_selfcheck(geom[r]))
                return fail(SU2_ERANGE, "index arithmetic self-check failed for these extents");
            max_vh = std::max(max_vh, geom[r].vh);
            max_ns3 = std::max(max_ns3, (uint32_t)(dims[r][0] * dims[r][1] * dims[r][2]));
            while (dims[r][3] % poly_s) poly_s /= 2;
            plane_hs = (r == 0 || plane_hs == geom[r].P) ? geom[r].P : 0u;
        }
        std::vector<Rep> h(n);
        for (int r = 0; r < n; ++r) {
            h[r].g = geom[r];
            h[r].links = links[r];
            h[r].cnt = cnt(r);
            h[r].acc = acc(r);
            h[r].results = results(r);
            h[r].beta = (float)beta[r];
            h[r].beta_d = beta[r];
            h[r].replica = replica[r];
            h[r].first_block = first_block[r];
            h[r].nblocks = nblocks[r];
            h[r].qfirst = 0u;
            h[r].orw = orw;
        }
        if (amap) {
            HIP_TRY(hipStreamSynchronize(stream));  // no pass may still read it
            (void)hipFree(amap);
        }
        amap = nullptr;
        amap_len = 0;
        if (cfg.affine && n > 1 && !f64) {
            // replicas spread over the XCDs by size (as the work queue); the
            // blocks of replica r go, in order, to workgroups b = slot * nq + x
            // of its XCD x (workgroups are dispatched to the XCDs in turn)
            std::vector<int> ids;
            if (int rc = xcc_ids(ids)) return rc;
            const int nq = (int)ids.size();
            std::vector<int> qof;
            std::vector<uint32_t> qfirst, qslots;
            queue_layout(nblocks, nq, qof, qfirst, qslots);
            const uint32_t maxlen = *std::max_element(qslots.begin(), qslots.end());
            std::vector<uint2> m((size_t)nq * maxlen, uint2{0xFFFFFFFFu, 0u});
            for (int r = 0; r < n; ++r)
                for (uint32_t k = 0; k < nblocks[r]; ++k)
                    m[(size_t)(qfirst[r] + k) * nq + qof[r]] = uint2{(uint32_t)r, k};
            HIP_TRY(hipMalloc(&amap, m.size() * sizeof(uint2)));
            HIP_TRY(hipMemcpy(amap, m.data(), m.size() * sizeof(uint2), hipMemcpyHostToDevice));
            amap_len = (uint32_t)m.size();
        }
        if (cfg.queue) {
            std::vector<int> ids;
            if (int rc = xcc_ids(ids)) return rc;
            const int nq = (int)ids.size();
            queue_nq = nq;
            std::vector<int> qof;
            std::vector<uint32_t> qfirst, qslots;
            queue_layout(nblocks, nq, qof, qfirst, qslots);
            QueueState hq;
            std::fill(std::begin(hq.rank), std::end(hq.rank), -1);
            std::fill(std::begin(hq.slots), std::end(hq.slots), 0u);
            std::fill(std::begin(hq.off), std::end(hq.off), 0u);
            uint32_t off = 0;
            for (int q = 0; q < nq; ++q) {
                hq.rank[ids[q]] = q;
                hq.slots[q] = qslots[q];
                hq.off[q] = off;
                off += qslots[q];
            }
            for (int r = 0; r < n; ++r) h[r].qfirst = qfirst[r];
            HIP_TRY(hipStreamSynchronize(stream));
            const size_t a = offsetof(QueueState, rank), z = sizeof(QueueState);
            HIP_TRY(hipMemcpy(reinterpret_cast<char *>(d_qs()) + a,
                              reinterpret_cast<const char *>(&hq) + a, z - a,
                              hipMemcpyHostToDevice));
            if (n > 1) {
                std::vector<uint32_t> qmap(off);
                for (int r = 0; r < n; ++r)
                    for (uint32_t k = 0; k < nblocks[r]; ++k)
                        qmap[hq.off[qof[r]] + qfirst[r] + k] = (uint32_t)r;
                HIP_TRY(hipMemcpy(d_qmap(), qmap.data(), qmap.size() * 4, hipMemcpyHostToDevice));
            }
        }
        HIP_TRY(hipStreamSynchronize(stream));
        HIP_TRY(hipMemcpy(d_reps(), h.data(), n * sizeof(Rep), hipMemcpyHostToDevice));
        if (n > 1) {
            std::vector<uint32_t> map(total_blocks);
            for (int r = 0; r < n; ++r) {
                const uint32_t end = r + 1 < n ? first_block[r + 1] : total_blocks;
                for (uint32_t b = first_block[r]; b < end; ++b) map[b] = (uint32_t)r;
            }
            HIP_TRY(hipMemcpy(d_bmap(), map.data(), map.size() * 4, hipMemcpyHostToDevice));
        }
        return SU2_OK;
    }

    int init(const std::vector<int> &starts)
    {
        int *d = nullptr;
        HIP_TRY(hipMalloc(&d, n * sizeof(int)));
        hipError_t e = hipMemcpy(d, starts.data(), n * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_set_counter(ens(), 0, 0, 7 | 16, stream, d_qs());
        if (e == hipSuccess)
            e = f64 ? launch_init64(ens(), starts[0], seed, stream) : launch_init(ens(), d, seed, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        (void)hipFree(d);
        if (e != hipSuccess) return fail(SU2_EHIP, std::string("init: ") + hipGetErrorString(e));
        sweep = 0;
        return SU2_OK;
    }

    // Whole sweeps in one launch (small lattices only).
    bool small_path() const
    {
        return !f64 && !cfg.queue && cfg.small && max_vh <= kSmallMaxVh;
    }

    // Workgroups of the persistent queue launch: the grid cap if set, else
    // as many as the device holds at once.
    // (at least one workgroup per queue: workgroups go to the XCDs in turn)
    uint32_t queue_grid(bool learned) const
    {
        const uint32_t g = cfg.grid_cap ? cfg.grid_cap : queue_grid_auto[learned ? 1 : 0];
        return std::max(g, (uint32_t)queue_nq);
    }

    // ns sweeps as persistent work-queue launches of < 2^31 items each.
    int enqueue_queue(int32_t ns, const float *tab, int32_t reunit_every, int meas, double *hist)
    {
        QueuePlan p{};
        p.reunit = reunit_every > 0 ? (uint32_t)reunit_every : 0u;
        p.want_p = hist && (meas & SU2_MEAS_PLAQ) ? 1u : 0u;
        p.want_l = hist && (meas & SU2_MEAS_POLY) ? 1u : 0u;
        p.rows = hist ? 1u : 0u;
        p.graph_rows = rows_graph ? 1u : 0u;
        const uint64_t per_sweep = (uint64_t)(8u + p.want_l + (p.reunit ? 1u + p.want_p : 0u)) *
                                   total_blocks;
        const int64_t max_ns = (int64_t)((((uint64_t)1 << 31) - 1u) / per_sweep);
        if (max_ns < 1) return fail(SU2_ERANGE, "work-queue launch too large");
        const uint32_t grid = queue_grid(tab != nullptr);
        int32_t done = 0;
        while (done < ns) {
            const int32_t c = (int32_t)std::min<int64_t>(ns - done, max_ns);
            p.ns = (uint32_t)c;
            p.phase = p.reunit ? (sweep + (uint32_t)done) % p.reunit : 0u;
            HIP_TRY(launch_queue_sweeps(ens(), p, d_qmap(), seed, cfg.pass_block, grid, cfg.grain,
                                        cfg.snake, hist, tab, d_qs(), spin_limit, stream));
            done += c;
        }
        sweep += (uint32_t)ns;
        queue_used = true;
        return SU2_OK;
    }

    // After queue launches: wait for the stream and report a wait that ran
    // out (the flag is cleared).
    int check_queue()
    {
        if (!queue_used) return SU2_OK;
        uint32_t err = 0;
        HIP_TRY(hipMemcpyAsync(&err, &d_qs()->error, sizeof(err), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        queue_used = false;
        if (err) {
            HIP_TRY(launch_set_counter(ens(), 0, 0, 16, stream, d_qs()));
            HIP_TRY(hipStreamSynchronize(stream));
            return fail(SU2_EHIP, err == 1u ? "work-queue launch: a bounded wait ran out of polls; "
                                              "the sweeps since the last check are invalid"
                                            : "work-queue launch: an XCD queue was not served "
                                              "(too few workgroups); the sweeps since the last "
                                              "check are invalid");
        }
        return SU2_OK;
    }

    const float *mode_table(int mode, int *rc)
    {
        *rc = SU2_OK;
        if (mode != SU2_KP && mode != SU2_LEARNED && mode != SU2_KP_OR)
            *rc = fail(SU2_EINVAL, "unknown mode");
        else if (mode == SU2_LEARNED && f64)
            *rc = fail(SU2_ESTATE, "the learned proposal runs on FP32 links only");
        else if (mode == SU2_KP_OR && f64)
            *rc = fail(SU2_ESTATE, "over-relaxation runs on FP32 links only");
        else if (mode == SU2_LEARNED && !table)
            *rc = fail(SU2_ESTATE, "no learned proposal loaded (su2_set_proposal)");
        return mode == SU2_LEARNED ? table : nullptr;
    }

    // One (mu, parity) pass in the configured kernel: the LDS-staged march
    // for single FP32 lattices when configured (heat bath and
    // over-relaxation), else the plain pass kernels.
    // norm: the plain pass kernel that reunitarises each link it stores.
    hipError_t pass_launch(int mu, int par, bool measure, const float *tab, bool orx,
                           bool norm = false)
    {
        if (f64) return launch_pass64(ens(), mu, par, seed, measure, cfg, stream);
        if (cfg.march_R && !tab && !norm)
            return launch_pass_march(ens(), mu, par, seed, measure, orx, march,
                                     cfg.snake ? par : 0, stream);
        return orx ? launch_or_pass(ens(), mu, par, measure, cfg, stream, norm)
                   : launch_pass(ens(), mu, par, seed, measure, tab, cfg, stream, norm);
    }

    // Enqueue n sweeps; the sweep index the device uses comes from the
    // device counters, and the host mirror decides the reunitarisation
    // schedule.  hist rows restart at 0 for this call.  With reunit_fused
    // the links of a reunitarisation sweep are reunitarised by the passes
    // that store them last, and the plaquette stays fused into the passes.
    int enqueue(int32_t ns, int mode, int32_t reunit_every, int meas, double *hist,
                bool reset_rows = true)
    {
        int rc;
        const float *tab = mode_table(mode, &rc);
        if (rc) return rc;
        if (hist && reset_rows) HIP_TRY(launch_set_counter(ens(), 0, 0, 2, stream));
        // heat bath + over-relaxation, and fused reunitarisation: per-pass
        // launches whatever the configuration
        const int nor = mode == SU2_KP_OR ? n_or : 0;
        const bool per_pass = mode == SU2_KP_OR || (reunit_fused && reunit_every > 0);
        if (cfg.queue && !f64 && !per_pass)
            return enqueue_queue(ns, tab, reunit_every, meas, hist);
        const int gflag = rows_graph ? 8 : 0;
        if (small_path() && !per_pass) {
            const int flags = (hist && (meas & SU2_MEAS_PLAQ) ? 1 : 0) |
                              (hist && (meas & SU2_MEAS_POLY) ? 2 : 0) | (hist ? 4 | gflag : 0);
            HIP_TRY(launch_small_sweeps(ens(), ns, seed, reunit_every, flags, hist, tab, stream));
            sweep += (uint32_t)ns;
            return SU2_OK;
        }
        for (int32_t i = 0; i < ns; ++i) {
            const uint32_t j = sweep + (uint32_t)i;
            const bool reunit = reunit_every > 0 && ((j + 1u) % (uint32_t)reunit_every) == 0u;
            const bool norm = reunit && reunit_fused;
            const bool want_p = hist && (meas & SU2_MEAS_PLAQ);
            const bool fused = want_p && (!reunit || norm);
            // the plaquette is fused into the odd passes of mu >= 1 of the last stage
            for (int mu = 0; mu < 4; ++mu)
                for (int par = 0; par < 2; ++par)
                    HIP_TRY(pass_launch(mu, par, fused && par == 1 && mu >= 1 && nor == 0, tab,
                                        false, norm && nor == 0));
            for (int k = 0; k < nor; ++k)
                for (int mu = 0; mu < 4; ++mu)
                    for (int par = 0; par < 2; ++par)
                        HIP_TRY(pass_launch(mu, par, fused && par == 1 && mu >= 1 && k == nor - 1,
                                            nullptr, true, norm && k == nor - 1));
            if (reunit && !norm) HIP_TRY(reunitarize_launch());
            if (want_p && !fused) HIP_TRY(plaquette_launch());
            const bool want_l = hist && (meas & SU2_MEAS_POLY);
            if (want_l) HIP_TRY(polyakov_launch());
            const int flags = (want_p ? 1 : 0) | (want_l ? 2 : 0) | (hist ? 4 | gflag : 0);
            HIP_TRY(launch_sweep_end(ens(), flags, hist, stream));
        }
        sweep += (uint32_t)ns;
        return SU2_OK;
    }

    // Capture `ns` sweeps (as enqueue) into a graph replayed by replay().  The
    // history rows continue across replays: the graph's sweeps count rows on
    // their own device counter (graph_row), reset here and advanced only by
    // replays, so direct measured sweeps between replays do not move them.
    int capture(int32_t ns, int mode, int32_t reunit_every, int meas, double *hist,
                int64_t hist_rows)
    {
        if (ns <= 0) return fail(SU2_EINVAL, "nsweeps must be > 0");
        if (hist && hist_rows < ns)
            return fail(SU2_EINVAL, "dev_history must hold at least nsweeps rows");
        if (reunit_every > 0 && (ns % reunit_every || sweep % (uint32_t)reunit_every))
            return fail(SU2_EINVAL, "with reunitarisation the captured sweeps must span whole "
                                    "periods starting at a period boundary");
        int rc;
        mode_table(mode, &rc);
        if (rc) return rc;
        if (!stream) return fail(SU2_ESTATE, "graph capture needs a non-null stream");
        drop_graph();
        if (hist) HIP_TRY(launch_set_counter(ens(), 0, 0, 32, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const uint32_t s0 = sweep;
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        rows_graph = true;
        rc = enqueue(ns, mode, reunit_every, meas, hist, false);
        rows_graph = false;
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &gr);
        sweep = s0;  // capturing ran nothing
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e != hipSuccess)
            return fail(SU2_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gr);
            return fail(SU2_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        graph = gr;
        g_nsweeps = ns;
        g_reunit = reunit_every > 0 ? reunit_every : 0;
        g_rows_cap = hist ? hist_rows : 0;
        g_rows_next = 0;
        return SU2_OK;
    }

    int replay(int32_t count)
    {
        if (!gexec) return fail(SU2_ESTATE, "no captured sweeps");
        if (count < 0) return fail(SU2_EINVAL, "count must be >= 0");
        // the graph's reunitarisation sweeps sit at fixed positions: replaying
        // off a period boundary would move them away from the schedule
        if (g_reunit > 0 && sweep % (uint32_t)g_reunit)
            return fail(SU2_ESTATE, "replay must start at a reunitarisation period boundary "
                                    "(sweeps were run since the capture)");
        if (g_rows_cap > 0 && g_rows_next + (int64_t)count * g_nsweeps > g_rows_cap)
            return fail(SU2_EINVAL, "the replays would write history rows " +
                                        std::to_string(g_rows_next) + ".." +
                                        std::to_string(g_rows_next + (int64_t)count * g_nsweeps - 1) +
                                        " but dev_history holds " + std::to_string(g_rows_cap));
        for (int32_t i = 0; i < count; ++i) HIP_TRY(hipGraphLaunch(gexec, stream));
        sweep += (uint32_t)(count * g_nsweeps);
        if (g_rows_cap > 0) g_rows_next += (int64_t)count * g_nsweeps;
        return SU2_OK;
    }

    // Measurement and reunitarisation kernels of the ensemble's precision.
    hipError_t plaquette_launch()
    {
        return f64 ? launch_plaquette64(ens(), stream) : launch_plaquette(ens(), stream);
    }
    hipError_t polyakov_launch()
    {
        return f64 ? launch_polyakov64(ens(), stream) : launch_polyakov(ens(), stream);
    }
    hipError_t reunitarize_launch()
    {
        return f64 ? launch_reunitarize64(ens(), stream) : launch_reunitarize(ens(), stream);
    }

    // flags 1 plaquette, 2 Polyakov; results into host arrays (n entries).
    int observe(int flags, double *plaq, double *poly_s, double *poly_a)
    {
        if (flags & 1) HIP_TRY(plaquette_launch());
        if (flags & 2) HIP_TRY(polyakov_launch());
        HIP_TRY(launch_take(ens(), flags, stream));
        std::vector<double> v(3 * (size_t)n);
        for (int r = 0; r < n; ++r)
            HIP_TRY_DRAIN(hipMemcpyAsync(&v[3 * r], results(r), 3 * sizeof(double),
                                         hipMemcpyDeviceToHost, stream), stream);
        HIP_TRY(hipStreamSynchronize(stream));
        if (int rc = check_queue()) return rc;
        for (int r = 0; r < n; ++r) {
            if (plaq) plaq[r] = v[3 * r + R_PLAQ];
            if (poly_s) poly_s[r] = v[3 * r + R_POLY_SIGNED];
            if (poly_a) poly_a[r] = v[3 * r + R_POLY_ABS];
        }
        return SU2_OK;
    }

    int counts(int reset, uint64_t *proposed, uint64_t *accepted)
    {
        HIP_TRY(launch_counts(ens(), reset, stream));
        std::vector<unsigned long long> v(2 * (size_t)n);
        for (int r = 0; r < n; ++r)
            HIP_TRY_DRAIN(hipMemcpyAsync(&v[2 * r], results(r) + R_COUNTS, 2 * sizeof(uint64_t),
                                         hipMemcpyDeviceToHost, stream), stream);
        HIP_TRY(hipStreamSynchronize(stream));
        for (int r = 0; r < n; ++r) {
            if (proposed) proposed[r] = v[2 * r];
            if (accepted) accepted[r] = v[2 * r + 1];
        }
        return SU2_OK;
    }

    // Host layout [t][z][y][x][mu][c] in H (float or double) <-> the device
    // planes in the ensemble's precision.
    template <typename D, typename H>
    void gather(int r, const D *planes, H *host) const
    {
        const int32_t *d = dims[r].data();
        const int64_t V = volume_of(d), vh = V / 2;
        for (int64_t s = 0; s < V; ++s) {
            int64_t q = s;
            const int x = (int)(q % d[0]);
            q /= d[0];
            const int y = (int)(q % d[1]);
            q /= d[1];
            const int z = (int)(q % d[2]);
            const int t = (int)(q / d[2]);
            const int par = (x + y + z + t) & 1;
            for (int mu = 0; mu < 4; ++mu)
                for (int k = 0; k < 4; ++k)
                    host[(s * 4 + mu) * 4 + k] = (H)planes[dev_index<D>(mu, par, k, s >> 1, vh)];
        }
    }

    template <typename D, typename H>
    void scatter(int r, const H *host, D *planes) const
    {
        const int32_t *d = dims[r].data();
        const int64_t V = volume_of(d), vh = V / 2;
        for (int64_t s = 0; s < V; ++s) {
            int64_t q = s;
            const int x = (int)(q % d[0]);
            q /= d[0];
            const int y = (int)(q % d[1]);
            q /= d[1];
            const int z = (int)(q % d[2]);
            const int t = (int)(q / d[2]);
            const int par = (x + y + z + t) & 1;
            for (int mu = 0; mu < 4; ++mu)
                for (int k = 0; k < 4; ++k)
                    planes[dev_index<D>(mu, par, k, s >> 1, vh)] = (D)host[(s * 4 + mu) * 4 + k];
        }
    }

    template <typename D, typename H>
    int get_links_as(int r, H *host)
    {
        const size_t n = (size_t)volume_of(dims[r].data()) * 16;
        std::unique_ptr<D[]> planes(new (std::nothrow) D[n]);
        if (!planes) return fail(SU2_ENOMEM, "host staging buffer of " + std::to_string(n * sizeof(D)) + " B");
        HIP_TRY(hipMemcpyAsync(planes.get(), links[r], n * sizeof(D), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (int rc = check_queue()) return rc;
        gather(r, planes.get(), host);
        return SU2_OK;
    }

    template <typename D, typename H>
    int set_links_as(int r, const H *host)
    {
        const size_t n = (size_t)volume_of(dims[r].data()) * 16;
        std::unique_ptr<D[]> planes(new (std::nothrow) D[n]);
        if (!planes) return fail(SU2_ENOMEM, "host staging buffer of " + std::to_string(n * sizeof(D)) + " B");
        scatter(r, host, planes.get());
        HIP_TRY(hipMemcpyAsync(links[r], planes.get(), n * sizeof(D), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return SU2_OK;
    }

    template <typename H>
    int get_links(int r, H *host)
    {
        return f64 ? get_links_as<double>(r, host) : get_links_as<float>(r, host);
    }

    template <typename H>
    int set_links(int r, const H *host)
    {
        return f64 ? set_links_as<double>(r, host) : set_links_as<float>(r, host);
    }

    int set_sweep(uint32_t s)
    {
        HIP_TRY(launch_set_counter(ens(), s, 0, 1, stream));
        sweep = s;
        return SU2_OK;
    }

    int set_launch(int block, int flags, int tile_z, int tile_t, int grid_cap)
    {
        if (block < 64 || block > 256 || (block % 64) != 0)
            return fail(SU2_EINVAL, "block must be 64, 128, 192 or 256");
        if (flags < 0 || flags > 255) return fail(SU2_EINVAL, "flags must be in [0, 255]");
        if (grid_cap < 0) return fail(SU2_EINVAL, "grid_cap must be >= 0");
        const bool march_on = (flags & 128) != 0;
        MarchShape ms{};
        if (march_on) {
            if (n != 1 || f64 || (flags & 8))
                return fail(SU2_EINVAL, "the LDS-staged pass (flag 128) runs single FP32 lattices "
                                        "without the work queue");
            if (tile_z <= 0 || tile_t <= 0 || !march_shape(dims[0].data(), (uint32_t)tile_z,
                                                            (uint32_t)tile_t, &ms))
                return fail(SU2_EINVAL, "the LDS-staged pass needs rows R = tile_z dividing Ny "
                                        "and T = tile_t dividing Nt, with 2 <= R, R Nx/2 <= 256");
        }
        uint32_t lz = lg_tz, lt = lg_tt;
        int rc;
        if (!march_on) {
            if ((rc = lg_of_tile(tile_z, lg_tz, &lz))) return rc;
            if ((rc = lg_of_tile(tile_t, lg_tt, &lt))) return rc;
        }
        cfg.pass_block = block;
        cfg.xcd_remap = (flags & 1) != 0;
        cfg.snake = (flags & 2) == 0;
        cfg.small = (flags & 4) == 0;
        cfg.queue = (flags & 8) != 0;
        cfg.affine = (flags & 64) != 0;
        cfg.grain = 1 << ((flags >> 4) & 3);
        cfg.grid_cap = (uint32_t)grid_cap;
        cfg.march_R = march_on ? (uint32_t)tile_z : 0u;
        cfg.march_T = march_on ? (uint32_t)tile_t : 0u;
        if (march_on) cfg.small = false;
        march = ms;
        if (cfg.queue) {  // device queries stay out of any stream capture
            queue_grid_auto[0] = queue_resident_grid(block, false);
            queue_grid_auto[1] = queue_resident_grid(block, true);
        }
        lg_tz = lz;
        lg_tt = lt;
        return upload();
    }

    // Time candidate launch configurations on the ensemble itself (state saved
    // and restored), keep the fastest; cache by device and extents.
    int autotune(const char *cache_path, int mode, double *best_us);

    void release()
    {
        drop_graph();
        if (stream) (void)hipStreamSynchronize(stream);
        if (own_pool && pool) (void)hipFree(pool);
        if (own_scratch && scratch) (void)hipFree(scratch);
        if (amap) (void)hipFree(amap);
        amap = nullptr;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        pool = nullptr;
        scratch = nullptr;
        stream = nullptr;
    }
};

namespace {

std::string tune_key(const Ensemble &E, int mode)
{
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::string k = "dev=";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) k += prop.gcnArchName;
    std::vector<std::array<int32_t, 4>> d = E.dims;
    std::sort(d.begin(), d.end());
    k += ";mode=" + std::to_string(mode) + ";n=" + std::to_string(E.n);
    if (E.f64) k += ";f64";  // another kernel: its own choice
    if (mode == SU2_KP_OR) k += ";n_or=" + std::to_string(E.n_or);
    k += ";dims=";
    for (auto &x : d)
        k += std::to_string(x[0]) + "x" + std::to_string(x[1]) + "x" + std::to_string(x[2]) +
             "x" + std::to_string(x[3]) + ",";
    return k;
}

struct TuneEntry {
    int block, flags, tz, tt, grid;
    double us;
};

bool cache_lookup(const char *path, const std::string &key, TuneEntry *e)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    std::vector<char> line(1 << 16);
    std::vector<char> k(1 << 16);
    bool found = false;
    while (std::fgets(line.data(), (int)line.size(), f)) {
        TuneEntry t;
        if (std::sscanf(line.data(),
                        "{\"key\": \"%65000[^\"]\", \"block\": %d, \"flags\": %d, \"tile_z\": %d, "
                        "\"tile_t\": %d, \"grid_cap\": %d, \"us_per_sweep\": %lf}",
                        k.data(), &t.block, &t.flags, &t.tz, &t.tt, &t.grid, &t.us) == 7 &&
            key == k.data()) {
            *e = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const TuneEntry &t)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"block\": %d, \"flags\": %d, \"tile_z\": %d, \"tile_t\": %d, "
                 "\"grid_cap\": %d, \"us_per_sweep\": %.3f}\n",
                 key.c_str(), t.block, t.flags, t.tz, t.tt, t.grid, t.us);
    std::fclose(f);
}

}  // namespace

int Ensemble::autotune(const char *cache_path, int mode, double *best_us)
{
    int rc;
    mode_table(mode, &rc);
    if (rc) return rc;
    const std::string key = tune_key(*this, mode);
    TuneEntry best{};
    if (cache_lookup(cache_path, key, &best)) {
        if (best_us) *best_us = best.us;
        return set_launch(best.block, best.flags, best.tz, best.tt, best.grid);
    }
    // Snapshot of everything the trial sweeps change: the links and each
    // replica's counters, accumulators (accept statistics included) and
    // result slots.  Every failure below still restores it.
    const size_t rb = rep_bytes();
    std::vector<void *> saved(n, nullptr);
    void *rep_saved = nullptr;
    hipError_t e = hipMalloc(&rep_saved, (size_t)n * rb);
    for (int r = 0; r < n && e == hipSuccess; ++r) {
        const size_t b = (size_t)volume_of(dims[r].data()) * (f64 ? 128 : 64);  // 16 reals per site
        e = hipMalloc(&saved[r], b);
        if (e == hipSuccess)
            e = hipMemcpyAsync(saved[r], links[r], b, hipMemcpyDeviceToDevice, stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(rep_saved, rep_scratch(0), (size_t)n * rb, hipMemcpyDeviceToDevice,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        for (void *p : saved)
            if (p) (void)hipFree(p);
        if (rep_saved) (void)hipFree(rep_saved);
        return fail(SU2_EHIP, std::string("autotune snapshot: ") + hipGetErrorString(e));
    }
    const uint32_t sweep0 = sweep;
    const LaunchCfg cfg0 = cfg;
    const uint32_t lz0 = lg_tz, lt0 = lg_tt;
    // candidates: the whole-sweep kernel when the lattices are small enough,
    // then the pass kernels over block sizes, traversal flags, tiles and
    // persistent grid sizes
    struct Cand {
        int block, flags, tz, tt, grid;
    };
    std::vector<Cand> cands;
    const bool small_ok = !f64 && max_vh <= kSmallMaxVh && mode != SU2_KP_OR;
    if (small_ok) cands.push_back({256, 1, 8, 8, 0});
    const int no_small = small_ok ? 4 : 0;
    for (int b : {256, 128})
        for (int fl : {1, 3})  // remap + alternating order, remap only
            for (auto t : {std::array<int, 2>{8, 8}, {4, 8}, {2, 16}, {1, 1}, {16, 16}})
                for (int gc : {0, 2048, 4096}) {
                    if (f64 && gc) continue;  // the FP64 pass always launches its full grid
                    cands.push_back({b, fl | no_small, t[0], t[1], gc});
                }
    // the persistent work queue (one item per ticket is always slower: the
    // per-run synchronisation dominates)
    if (!f64 && mode != SU2_KP_OR)
        for (int b : {256, 128})
            for (int gr : {1, 2}) cands.push_back({b, 1 | 8 | (gr << 4), 8, 8, 0});
    // single lattices: the LDS-staged march pass (heat bath and over-relaxation)
    if (n == 1 && !f64 && mode != SU2_LEARNED)
        for (int R : {4, 8, 16})
            for (int T : {4, 8, 16}) {
                MarchShape ms;
                if (march_shape(dims[0].data(), (uint32_t)R, (uint32_t)T, &ms))
                    cands.push_back({256, 1 | 4 | 128, R, T, 0});
            }
    // batches: every replica's pass workgroups on one XCD
    if (n > 1 && !f64) {
        for (int b : {256, 128})
            for (int fl : {64, 66})
                for (auto t : {std::array<int, 2>{8, 8}, {4, 8}, {1, 1}})
                    cands.push_back({b, fl | no_small, t[0], t[1], 0});
        // persistent grids (a learned pass then loads its LDS table once per workgroup)
        for (auto t : {std::array<int, 2>{8, 8}, {1, 1}})
            for (int gc : {1024, 4096}) cands.push_back({256, 64 | no_small, t[0], t[1], gc});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    best.us = 1e30;
    const int trial_sweeps = 2;
    // Trial sweeps measure the plaquette, as the benchmarked and most other
    // sweeps do (the fused measurement changes which launch is fastest); their
    // history rows go to a buffer of the autotuner's own.  Every candidate is
    // timed on `trial_sweeps` sweeps, then the three fastest again on
    // `final_sweeps`; each timing is the faster of two runs.
    const int final_sweeps = 8;
    double *thist = nullptr;
    if (e == hipSuccess) e = hipMalloc(&thist, (size_t)final_sweeps * (size_t)n * 3 * sizeof(double));
    rc = SU2_OK;
    auto time_cand = [&](const Cand &c, int ns, double *us) -> bool {
        *us = 1e30;
        if ((rc = set_launch(c.block, c.flags, c.tz, c.tt, c.grid))) return false;
        if ((rc = enqueue(1, mode, 0, SU2_MEAS_PLAQ, thist))) return false;  // warm-up
        for (int rep = 0; rep < 2; ++rep) {
            if ((e = hipEventRecord(e0, stream)) != hipSuccess) return false;
            if ((rc = enqueue(ns, mode, 0, SU2_MEAS_PLAQ, thist))) return false;
            if ((e = hipEventRecord(e1, stream)) != hipSuccess) return false;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return false;
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return false;
            *us = std::min(*us, 1e3 * ms / ns);
        }
        return (rc = check_queue()) == SU2_OK;
    };
    std::vector<std::pair<double, size_t>> first;
    for (size_t i = 0; i < cands.size() && e == hipSuccess && !rc; ++i) {
        double us;
        if (!time_cand(cands[i], trial_sweeps, &us)) break;
        first.push_back({us, i});
    }
    std::sort(first.begin(), first.end());
    for (size_t k = 0; k < first.size() && k < 3 && e == hipSuccess && !rc; ++k) {
        const Cand &c = cands[first[k].second];
        double us;
        if (!time_cand(c, final_sweeps, &us)) break;
        if (us < best.us) best = TuneEntry{c.block, c.flags, c.tz, c.tt, c.grid, us};
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // restore the state whatever happened (the trial history buffer goes once
    // the stream has drained)
    const hipError_t es = hipStreamSynchronize(stream);
    if (thist) (void)hipFree(thist);
    if (e == hipSuccess) e = es;
    hipError_t er = hipStreamSynchronize(stream);
    for (int r = 0; r < n; ++r) {
        const size_t b = (size_t)volume_of(dims[r].data()) * (f64 ? 128 : 64);
        if (er == hipSuccess)
            er = hipMemcpyAsync(links[r], saved[r], b, hipMemcpyDeviceToDevice, stream);
    }
    if (er == hipSuccess)
        er = hipMemcpyAsync(rep_scratch(0), rep_saved, (size_t)n * rb, hipMemcpyDeviceToDevice,
                            stream);
    if (er == hipSuccess) er = hipStreamSynchronize(stream);
    for (void *p : saved) (void)hipFree(p);
    (void)hipFree(rep_saved);
    sweep = sweep0;
    if (er != hipSuccess)
        return fail(SU2_EHIP, std::string("autotune restore: ") + hipGetErrorString(er));
    if (e != hipSuccess) rc = fail(SU2_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    if (rc) {
        // keep the launch configuration the ensemble had before
        cfg = cfg0;
        lg_tz = lz0;
        lg_tt = lt0;
        const int rc2 = upload();
        return rc2 ? rc2 : rc;
    }
    cache_store(cache_path, key, best);
    if (best_us) *best_us = best.us;
    return set_launch(best.block, best.flags, best.tz, best.tt, best.grid);
}

// ===================================================== single lattice (C ABI)
struct su2_nn {
    NNBuffers b;
    int64_t ndata = 0;     // training samples held
    int64_t act_cap = 0;   // batch capacity of the per-sample record
    int step = 0;          // Adam step counter
    bool table_ready = false;
    hipStream_t stream = nullptr;
    double *dev_loss = nullptr;  // per-step losses of the last train call
    int loss_cap = 0;
    std::atomic<int> users{0};   // contexts and batches whose sweeps read the table
};

struct su2_ctx {
    Ensemble E;
    su2_nn *proposal = nullptr;  // attached learned proposal (its table is E.table)
};

struct su2_batch {
    Ensemble E;
    su2_nn *proposal = nullptr;
};

namespace {

// Point `slot` at n: the previous proposal loses a user, n gains one, so
// su2_nn_destroy can refuse while any lattice still reads its table.
void attach_proposal(su2_nn *&slot, su2_nn *n)
{
    if (slot) slot->users.fetch_sub(1);
    slot = n;
    if (n) n->users.fetch_add(1);
}

}  // namespace

namespace {

int check_ctx(su2_ctx *c)
{
    if (!c) return fail(SU2_EINVAL, "context is NULL");
    return SU2_OK;
}

int check_batch(su2_batch *b)
{
    if (!b) return fail(SU2_EINVAL, "batch is NULL");
    return SU2_OK;
}

}  // namespace

extern "C" {

const char *su2_last_error(void) { return g_last_error.c_str(); }

size_t su2_links_bytes(const int32_t dims[4])
{
    SU2_API_BEGIN
    if (!dims) return 0;
    const std::string keep = g_last_error;  // a size query is not a failure
    const int rc = check_dims(dims);
    g_last_error = keep;
    if (rc) return 0;
    return (size_t)64 * (size_t)volume_of(dims);
    SU2_API_END_SIZE
}

size_t su2_scratch_bytes(const int32_t dims[4])
{
    SU2_API_BEGIN
    if (!su2_links_bytes(dims)) return 0;
    std::vector<std::array<int32_t, 4>> d{{dims[0], dims[1], dims[2], dims[3]}};
    return Ensemble::scratch_need(1, d);
    SU2_API_END_SIZE
}

static int init_common(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed,
                       int start, void *links_dev, size_t links_bytes, void *scratch_dev,
                       size_t scratch_bytes, void *stream, bool ext, bool f64 = false)
{
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!beta_ok(beta)) return fail(SU2_EINVAL, "beta must be finite and >= 0");
    if (start != SU2_COLD && start != SU2_HOT) return fail(SU2_EINVAL, "start must be COLD or HOT");
    const size_t need_l = su2_links_bytes(dims) * (f64 ? 2 : 1), need_s = su2_scratch_bytes(dims);
    if (ext) {
        if (!links_dev || !scratch_dev) return fail(SU2_EINVAL, "device buffer is NULL");
        if (links_bytes < need_l || scratch_bytes < need_s)
            return fail(SU2_ENOMEM, "caller buffers too small: need links " +
                                        std::to_string(need_l) + " B, scratch " +
                                        std::to_string(need_s) + " B");
    }
    su2_ctx *c = new (std::nothrow) su2_ctx();
    if (!c) return fail(SU2_ENOMEM, "host allocation failed");
    Ensemble &E = c->E;
    E.n = 1;
    E.f64 = f64;
    E.dims = {{dims[0], dims[1], dims[2], dims[3]}};
    E.beta = {beta};
    E.replica = {0u};
    E.seed = seed;
    if (ext) {
        E.pool = static_cast<float *>(links_dev);
        E.scratch = static_cast<unsigned char *>(scratch_dev);
        E.stream = static_cast<hipStream_t>(stream);
    } else {
        void *l = nullptr, *s = nullptr;
        hipError_t e = hipMalloc(&l, need_l);
        if (e == hipSuccess) e = hipMalloc(&s, need_s);
        if (e == hipSuccess && f64) E.stream = static_cast<hipStream_t>(stream);
        else if (e == hipSuccess) e = hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            if (l) (void)hipFree(l);
            if (s) (void)hipFree(s);
            delete c;
            return fail(e == hipErrorOutOfMemory ? SU2_ENOMEM : SU2_EHIP,
                        std::string("allocation: ") + hipGetErrorString(e));
        }
        E.pool = static_cast<float *>(l);
        E.scratch = static_cast<unsigned char *>(s);
        E.own_pool = E.own_scratch = true;
        E.own_stream = !f64;
    }
    E.links = {E.pool};
    E.bmap_off = E.qmap_off = E.rep_off = Ensemble::descr_bytes(1);
    if ((rc = E.upload()) || (rc = E.init({start}))) {
        E.release();
        delete c;
        return rc;
    }
    *out = c;
    return SU2_OK;
}

int su2_init(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start)
{
    SU2_API_BEGIN
    return init_common(out, dims, beta, seed, start, nullptr, 0, nullptr, 0, nullptr, false);
    SU2_API_END
}

int su2_init_f64(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
                 void *hip_stream)
{
    SU2_API_BEGIN
    return init_common(out, dims, beta, seed, start, nullptr, 0, nullptr, 0, hip_stream, false,
                       true);
    SU2_API_END
}

int su2_is_f64(su2_ctx *c, int *out)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = c->E.f64 ? 1 : 0;
    return SU2_OK;
    SU2_API_END
}

int su2_get_links_f64(su2_ctx *c, double *host)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    return c->E.get_links(0, host);
    SU2_API_END
}

int su2_set_links_f64(su2_ctx *c, const double *host)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    return c->E.set_links(0, host);
    SU2_API_END
}

int su2_init_ext(su2_ctx **out, const int32_t dims[4], double beta, uint64_t seed, int start,
                 void *links_dev, size_t links_bytes, void *scratch_dev, size_t scratch_bytes,
                 void *hip_stream)
{
    SU2_API_BEGIN
    return init_common(out, dims, beta, seed, start, links_dev, links_bytes, scratch_dev,
                       scratch_bytes, hip_stream, true);
    SU2_API_END
}

int su2_destroy(su2_ctx *c)
{
    SU2_API_BEGIN
    if (!c) return fail(SU2_EINVAL, "context is NULL");
    c->E.release();
    attach_proposal(c->proposal, nullptr);
    delete c;
    return SU2_OK;
    SU2_API_END
}

int su2_heatbath_sweep(su2_ctx *c, int32_t nsweeps, int mode)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsweeps < 0) return fail(SU2_EINVAL, "nsweeps must be >= 0");
    return c->E.enqueue(nsweeps, mode, 0, 0, nullptr);
    SU2_API_END
}

int su2_sweep_measure(su2_ctx *c, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                      double *dev_history)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsweeps < 0 || reunit_every < 0) return fail(SU2_EINVAL, "negative count");
    if (!dev_history) return fail(SU2_EINVAL, "dev_history is NULL");
    if (meas & ~(SU2_MEAS_PLAQ | SU2_MEAS_POLY)) return fail(SU2_EINVAL, "bad meas flags");
    return c->E.enqueue(nsweeps, mode, reunit_every, meas, dev_history);
    SU2_API_END
}

int su2_capture_sweeps(su2_ctx *c, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                       double *dev_history, int64_t history_rows)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (reunit_every < 0 || (meas & ~(SU2_MEAS_PLAQ | SU2_MEAS_POLY)))
        return fail(SU2_EINVAL, "bad arguments");
    if (meas && !dev_history) return fail(SU2_EINVAL, "dev_history is NULL");
    return c->E.capture(nsweeps, mode, reunit_every, meas, meas ? dev_history : nullptr,
                        history_rows);
    SU2_API_END
}

int su2_replay_sweeps(su2_ctx *c, int32_t count)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->E.replay(count);
    SU2_API_END
}

int su2_reunitarize(su2_ctx *c)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(c->E.reunitarize_launch());
    return SU2_OK;
    SU2_API_END
}

int su2_plaquette(su2_ctx *c, double *out)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    return c->E.observe(1, out, nullptr, nullptr);
    SU2_API_END
}

int su2_polyakov(su2_ctx *c, double *out_signed, double *out_abs)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->E.observe(2, nullptr, out_signed, out_abs);
    SU2_API_END
}

int su2_wilson_loops(su2_ctx *c, int rmax, int tmax, double *out)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    Ensemble &E = c->E;
    const int32_t *d = E.dims[0].data();
    const int lmin = std::min(std::min(d[0], d[1]), std::min(d[2], d[3]));
    if (rmax < 1 || tmax < 1 || rmax > kWilsonMax || tmax > kWilsonMax || rmax >= lmin ||
        tmax >= lmin)
        return fail(SU2_EINVAL, "rmax and tmax must be in [1, 4] and below every extent");
    if (E.f64) return fail(SU2_ESTATE, "Wilson loops are measured on FP32 links");
    const Ens e = E.ens();
    void *part = nullptr, *sums = nullptr;
    HIP_TRY(hipMalloc(&part, (size_t)wilson_blocks(e) * kWilsonMax * kWilsonMax * 8));
    hipError_t er = hipMalloc(&sums, kWilsonMax * kWilsonMax * 8);
    double hs[kWilsonMax * kWilsonMax];
    if (er == hipSuccess)
        er = launch_wilson(e, rmax, tmax, (double *)part, (double *)sums, E.stream);
    if (er == hipSuccess)
        er = hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, E.stream);
    if (er == hipSuccess) er = hipStreamSynchronize(E.stream);
    (void)hipFree(part);
    if (sums) (void)hipFree(sums);
    if (er != hipSuccess) return fail(SU2_EHIP, std::string("wilson: ") + hipGetErrorString(er));
    if (int q = E.check_queue()) return q;
    const double norm = 12.0 * (double)volume_of(d);
    for (int r = 0; r < rmax; ++r)
        for (int t = 0; t < tmax; ++t) out[r * tmax + t] = hs[r * kWilsonMax + t] / norm;
    return SU2_OK;
    SU2_API_END
}

int su2_get_links(su2_ctx *c, float *host)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    return c->E.get_links(0, host);
    SU2_API_END
}

int su2_set_links(su2_ctx *c, const float *host)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!host) return fail(SU2_EINVAL, "host is NULL");
    return c->E.set_links(0, host);
    SU2_API_END
}

int su2_get_sweep(su2_ctx *c, uint32_t *out)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = c->E.sweep;
    return SU2_OK;
    SU2_API_END
}

int su2_set_sweep(su2_ctx *c, uint32_t sweep)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->E.set_sweep(sweep);
    SU2_API_END
}

static int set_overrelax(Ensemble &E, double width)
{
    if (!(width <= 1.0)) return fail(SU2_EINVAL, "width must be <= 1 (< 0: off)");
    E.orw = width < 0.0 ? -1.0f : (float)width;
    return E.upload();
}

int su2_set_overrelax(su2_ctx *c, double width)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return set_overrelax(c->E, width);
    SU2_API_END
}

int su2_batch_set_overrelax(su2_batch *b, double width)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    return set_overrelax(b->E, width);
    SU2_API_END
}

int su2_set_hb_overrelax(su2_ctx *c, int32_t n_or)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (n_or < 0 || n_or > 16) return fail(SU2_EINVAL, "n_or must be in [0, 16]");
    c->E.drop_graph();
    c->E.n_or = n_or;
    return SU2_OK;
    SU2_API_END
}

static int set_reunit_fused(Ensemble &E, int on)
{
    if (on != 0 && on != 1) return fail(SU2_EINVAL, "on must be 0 or 1");
    if (on && E.f64) return fail(SU2_ESTATE, "the fused reunitarisation runs on FP32 links only");
    E.drop_graph();
    E.reunit_fused = on != 0;
    return SU2_OK;
}

int su2_set_reunit_fused(su2_ctx *c, int on)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return set_reunit_fused(c->E, on);
    SU2_API_END
}

int su2_batch_set_reunit_fused(su2_batch *b, int on)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    return set_reunit_fused(b->E, on);
    SU2_API_END
}

int su2_batch_set_hb_overrelax(su2_batch *b, int32_t n_or)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (n_or < 0 || n_or > 16) return fail(SU2_EINVAL, "n_or must be in [0, 16]");
    b->E.drop_graph();
    b->E.n_or = n_or;
    return SU2_OK;
    SU2_API_END
}

int su2_set_beta(su2_ctx *c, double beta)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!beta_ok(beta)) return fail(SU2_EINVAL, "beta must be finite and >= 0");
    c->E.beta[0] = beta;
    return c->E.upload();
    SU2_API_END
}

int su2_set_replica(su2_ctx *c, uint32_t replica)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (replica >= (1u << 26)) return fail(SU2_EINVAL, "replica id must be < 2^26");
    c->E.replica[0] = replica;
    return c->E.upload();
    SU2_API_END
}

int su2_links_device(su2_ctx *c, void **links_dev, void **hip_stream)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (links_dev) *links_dev = c->E.links[0];
    if (hip_stream) *hip_stream = c->E.stream;
    return SU2_OK;
    SU2_API_END
}

int su2_synchronize(su2_ctx *c)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->E.stream));
    return c->E.check_queue();
    SU2_API_END
}

int su2_set_launch(su2_ctx *c, int block, int flags, int tile_z, int tile_t, int grid_cap)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->E.set_launch(block, flags, tile_z, tile_t, grid_cap);
    SU2_API_END
}

static void get_launch(const Ensemble &E, int *block, int *flags, int *tile_z, int *tile_t,
                       int *grid_cap)
{
    if (block) *block = E.cfg.pass_block;
    if (flags) {
        int lg = 0;
        while ((1 << lg) < E.cfg.grain) ++lg;
        *flags = (E.cfg.xcd_remap ? 1 : 0) | (E.cfg.snake ? 0 : 2) | (E.cfg.small ? 0 : 4) |
                 (E.cfg.queue ? 8 : 0) | (lg << 4) | (E.cfg.affine ? 64 : 0) |
                 (E.cfg.march_R ? 128 : 0);
    }
    if (tile_z) *tile_z = E.cfg.march_R ? (int)E.cfg.march_R : 1 << E.geom[0].lg_tz;
    if (tile_t) *tile_t = E.cfg.march_R ? (int)E.cfg.march_T : 1 << E.geom[0].lg_tt;
    if (grid_cap) *grid_cap = (int)E.cfg.grid_cap;
}

int su2_get_launch(su2_ctx *c, int *block, int *flags, int *tile_z, int *tile_t, int *grid_cap)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    get_launch(c->E, block, flags, tile_z, tile_t, grid_cap);
    return SU2_OK;
    SU2_API_END
}

int su2_autotune(su2_ctx *c, const char *cache_path, int mode, double *best_us_per_sweep)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->E.autotune(cache_path, mode, best_us_per_sweep);
    SU2_API_END
}

/* ============================================================== batches */
int su2_batch_init(su2_batch **out, int32_t n, const int32_t *dims, const double *betas,
                   const int *starts, uint64_t seed, void *hip_stream)
{
    SU2_API_BEGIN
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    if (n <= 0 || n > 65535 || !dims || !betas || !starts)
        return fail(SU2_EINVAL, "need 1 <= n <= 65535 and non-NULL arrays");
    int rc;
    for (int r = 0; r < n; ++r) {
        if ((rc = check_dims(dims + 4 * r))) return rc;
        if (!beta_ok(betas[r])) return fail(SU2_EINVAL, "betas must be finite and >= 0");
        if (starts[r] != SU2_COLD && starts[r] != SU2_HOT)
            return fail(SU2_EINVAL, "start must be COLD or HOT");
    }
    su2_batch *b = new (std::nothrow) su2_batch();
    if (!b) return fail(SU2_ENOMEM, "host allocation failed");
    Ensemble &E = b->E;
    E.n = n;
    E.seed = seed;
    E.stream = static_cast<hipStream_t>(hip_stream);
    size_t pool_bytes = 0;
    std::vector<size_t> off(n);
    for (int r = 0; r < n; ++r) {
        E.dims.push_back({dims[4 * r], dims[4 * r + 1], dims[4 * r + 2], dims[4 * r + 3]});
        E.beta.push_back(betas[r]);
        E.replica.push_back((uint32_t)r);
        off[r] = pool_bytes;
        pool_bytes = align_up(pool_bytes + (size_t)volume_of(dims + 4 * r) * 64, 256);
    }
    const size_t scratch = Ensemble::scratch_need(n, E.dims);
    void *p = nullptr, *s = nullptr;
    hipError_t e = hipMalloc(&p, pool_bytes);
    if (e == hipSuccess) e = hipMalloc(&s, scratch);
    if (e != hipSuccess) {
        if (p) (void)hipFree(p);
        delete b;
        return fail(e == hipErrorOutOfMemory ? SU2_ENOMEM : SU2_EHIP,
                    std::string("allocation: ") + hipGetErrorString(e));
    }
    E.pool = static_cast<float *>(p);
    E.scratch = static_cast<unsigned char *>(s);
    E.own_pool = E.own_scratch = true;
    for (int r = 0; r < n; ++r)
        E.links.push_back(reinterpret_cast<float *>(reinterpret_cast<char *>(p) + off[r]));
    E.bmap_off = Ensemble::descr_bytes(n);
    E.qmap_off = E.bmap_off + Ensemble::bmap_bytes(n, E.dims);
    E.rep_off = E.qmap_off + Ensemble::bmap_bytes(n, E.dims);
    if ((rc = E.upload()) || (rc = E.init(std::vector<int>(starts, starts + n)))) {
        E.release();
        delete b;
        return rc;
    }
    *out = b;
    return SU2_OK;
    SU2_API_END
}

int su2_batch_destroy(su2_batch *b)
{
    SU2_API_BEGIN
    if (!b) return fail(SU2_EINVAL, "batch is NULL");
    b->E.release();
    attach_proposal(b->proposal, nullptr);
    delete b;
    return SU2_OK;
    SU2_API_END
}

int su2_batch_size(su2_batch *b, int32_t *n)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (!n) return fail(SU2_EINVAL, "n is NULL");
    *n = b->E.n;
    return SU2_OK;
    SU2_API_END
}

int su2_batch_sweep(su2_batch *b, int32_t nsweeps, int mode)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (nsweeps < 0) return fail(SU2_EINVAL, "nsweeps must be >= 0");
    return b->E.enqueue(nsweeps, mode, 0, 0, nullptr);
    SU2_API_END
}

int su2_batch_sweep_measure(su2_batch *b, int32_t nsweeps, int mode, int32_t reunit_every,
                            int meas, double *dev_history)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (nsweeps < 0 || reunit_every < 0) return fail(SU2_EINVAL, "negative count");
    if (!dev_history) return fail(SU2_EINVAL, "dev_history is NULL");
    if (meas & ~(SU2_MEAS_PLAQ | SU2_MEAS_POLY)) return fail(SU2_EINVAL, "bad meas flags");
    return b->E.enqueue(nsweeps, mode, reunit_every, meas, dev_history);
    SU2_API_END
}

int su2_batch_capture(su2_batch *b, int32_t nsweeps, int mode, int32_t reunit_every, int meas,
                      double *dev_history, int64_t history_rows)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (reunit_every < 0 || (meas & ~(SU2_MEAS_PLAQ | SU2_MEAS_POLY)))
        return fail(SU2_EINVAL, "bad arguments");
    if (meas && !dev_history) return fail(SU2_EINVAL, "dev_history is NULL");
    return b->E.capture(nsweeps, mode, reunit_every, meas, meas ? dev_history : nullptr,
                        history_rows);
    SU2_API_END
}

int su2_batch_replay(su2_batch *b, int32_t count)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    return b->E.replay(count);
    SU2_API_END
}

int su2_batch_observables(su2_batch *b, double *plaq, double *poly_signed, double *poly_abs)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    const int flags = (plaq ? 1 : 0) | ((poly_signed || poly_abs) ? 2 : 0);
    if (!flags) return SU2_OK;
    return b->E.observe(flags, plaq, poly_signed, poly_abs);
    SU2_API_END
}

int su2_batch_get_links(su2_batch *b, int32_t r, float *host)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (r < 0 || r >= b->E.n || !host) return fail(SU2_EINVAL, "bad replica or NULL");
    return b->E.get_links(r, host);
    SU2_API_END
}

int su2_batch_set_links(su2_batch *b, int32_t r, const float *host)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (r < 0 || r >= b->E.n || !host) return fail(SU2_EINVAL, "bad replica or NULL");
    return b->E.set_links(r, host);
    SU2_API_END
}

int su2_batch_set_launch(su2_batch *b, int block, int flags, int tile_z, int tile_t,
                         int grid_cap)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    return b->E.set_launch(block, flags, tile_z, tile_t, grid_cap);
    SU2_API_END
}

int su2_batch_get_launch(su2_batch *b, int *block, int *flags, int *tile_z, int *tile_t,
                         int *grid_cap)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    get_launch(b->E, block, flags, tile_z, tile_t, grid_cap);
    return SU2_OK;
    SU2_API_END
}

int su2_batch_autotune(su2_batch *b, const char *cache_path, int mode, double *best_us)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    return b->E.autotune(cache_path, mode, best_us);
    SU2_API_END
}

int su2_batch_synchronize(su2_batch *b)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(b->E.stream));
    return b->E.check_queue();
    SU2_API_END
}

int su2_batch_get_accept_stats(su2_batch *b, uint64_t *proposed, uint64_t *accepted, int reset)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    return b->E.counts(reset, proposed, accepted);
    SU2_API_END
}

/* ================================================================ tests */
int su2_test_queue_plan(int32_t n, const int32_t *dims, int block, int32_t queues,
                        int32_t nsweeps, int32_t reunit_every, uint32_t first_sweep, int meas,
                        int rows, int64_t *items_out)
{
    SU2_API_BEGIN
    if (n < 1 || !dims || nsweeps < 1 || reunit_every < 0 || (block % 64) || block < 64 ||
        block > 256 || queues < 1 || queues > kMaxQueues)
        return fail(SU2_EINVAL, "bad arguments");
    std::vector<std::array<int32_t, 4>> d(n);
    for (int r = 0; r < n; ++r) {
        if (int rc = check_dims(dims + 4 * r)) return rc;
        for (int k = 0; k < 4; ++k) d[r][k] = dims[4 * r + k];
    }
    std::vector<uint32_t> first, nb, qfirst, qslots;
    std::vector<int> qof;
    const uint32_t total_blocks = slot_layout(d, block, first, nb);
    queue_layout(nb, queues, qof, qfirst, qslots);
    QueuePlan p{};
    p.ns = (uint32_t)nsweeps;
    p.reunit = (uint32_t)reunit_every;
    p.phase = reunit_every ? first_sweep % (uint32_t)reunit_every : 0u;
    p.want_p = rows && (meas & SU2_MEAS_PLAQ) ? 1u : 0u;
    p.want_l = rows && (meas & SU2_MEAS_POLY) ? 1u : 0u;
    p.rows = rows ? 1u : 0u;
    if ((uint64_t)queue_total_stages(p) * total_blocks >= ((uint64_t)1 << 31))
        return fail(SU2_ERANGE, "too many items");
    // every slot of every replica belongs to exactly one queue position
    for (int q = 0; q < queues; ++q) {
        std::vector<int> owner(qslots[q], -1);
        for (int r = 0; r < n; ++r)
            if (qof[r] == q)
                for (uint32_t k = 0; k < nb[r]; ++k) {
                    if (qfirst[r] + k >= qslots[q] || owner[qfirst[r] + k] >= 0)
                        return fail(SU2_ERANGE, "queue layout overlaps");
                    owner[qfirst[r] + k] = r;
                }
        for (int o : owner)
            if (o < 0) return fail(SU2_ERANGE, "queue layout has a hole");
    }
    // Run each queue's items one at a time in ticket order, in runs of
    // `grain` = 1.  Deadlock freedom and completeness: when an item starts,
    // its replica's done count must equal its target plus the items of the
    // same stage already run (the target covers every earlier item of the
    // replica and nothing later).
    std::vector<uint32_t> done(n, 0u), in_stage(n, 0u), last_gs(n, 0xFFFFFFFFu), ends(n, 0u);
    int64_t items = 0;
    for (int q = 0; q < queues; ++q) {
        std::vector<int> owner(qslots[q]);
        for (int r = 0; r < n; ++r)
            if (qof[r] == q)
                for (uint32_t k = 0; k < nb[r]; ++k) owner[qfirst[r] + k] = r;
        const uint64_t total = (uint64_t)queue_total_stages(p) * qslots[q];
        for (uint64_t t = 0; t < total; ++t) {
            const QueueItem it = queue_decode(p, (uint32_t)t, qslots[q]);
            const uint32_t gs = queue_stages_before(p, it.sweep) + it.stage;
            if (gs != t / qslots[q] || it.slot != t % qslots[q] || it.sweep >= p.ns)
                return fail(SU2_ERANGE, "decode mismatch at item " + std::to_string(t));
            const int r = owner[it.slot];
            const bool reunit = queue_reunit_sweep(p, it.sweep);
            const int want_kind = it.stage < 8u ? QK_PASS
                                  : (reunit && it.stage == 8u) ? QK_REUNIT
                                  : (reunit && p.want_p && it.stage == 9u) ? QK_PLAQ : QK_POLY;
            if (it.kind != want_kind || (it.kind == QK_POLY && !p.want_l))
                return fail(SU2_ERANGE, "stage kind mismatch at item " + std::to_string(t));
            if (gs != last_gs[r]) {
                last_gs[r] = gs;
                in_stage[r] = 0u;
            }
            const uint32_t target = queue_target(p, nb[r], it.sweep, it.stage);
            if (done[r] != target + in_stage[r])
                return fail(SU2_ERANGE, "item " + std::to_string(t) + " of replica " +
                                            std::to_string(r) + ": done " +
                                            std::to_string(done[r]) + ", target " +
                                            std::to_string(target));
            ++in_stage[r];
            ++items;
            if (++done[r] == queue_sweep_last(p, nb[r], it.sweep)) {
                if (ends[r] != it.sweep) return fail(SU2_ERANGE, "sweep ends out of order");
                ++ends[r];
                ++done[r];  // the bookkeeping item
            }
        }
    }
    for (int r = 0; r < n; ++r)
        if (ends[r] != p.ns || done[r] != queue_target(p, nb[r], p.ns, 0u))
            return fail(SU2_ERANGE, "replica " + std::to_string(r) + " did not finish");
    if (items_out) *items_out = items;
    return SU2_OK;
    SU2_API_END
}

int su2_test_batch_spin_limit(su2_batch *b, uint32_t polls)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    b->E.spin_limit = polls;
    return SU2_OK;
    SU2_API_END
}

int su2_test_philox(const uint32_t *ctr_host, int64_t n, uint64_t seed, uint32_t *out_host)
{
    SU2_API_BEGIN
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
    SU2_API_END
}

int su2_test_heatbath_links(const float *V_host, int64_t n, double beta, uint64_t seed,
                            uint32_t sweep, uint32_t mu, uint32_t replica, float *out_host,
                            int32_t *ntrials_host)
{
    SU2_API_BEGIN
    if (n < 0 || (n > 0 && (!V_host || !out_host))) return fail(SU2_EINVAL, "bad arguments");
    if (!beta_ok(beta) || mu > 3 || replica >= (1u << 26))
        return fail(SU2_EINVAL, "bad beta, mu or replica");
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
    SU2_API_END
}

int su2_test_pass(su2_ctx *c, int mu, int parity, int mode)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (mu < 0 || mu > 3 || parity < 0 || parity > 1) return fail(SU2_EINVAL, "bad mu/parity");
    const float *tab = c->E.mode_table(mode, &rc);
    if (rc) return rc;
    HIP_TRY(c->E.pass_launch(mu, parity, false, tab, mode == SU2_KP_OR));
    return SU2_OK;
    SU2_API_END
}

int su2_test_stream_pass(su2_ctx *c, int mu, int parity, void *out_dev)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (mu < 0 || mu > 3 || parity < 0 || parity > 1 || !out_dev)
        return fail(SU2_EINVAL, "bad mu/parity or NULL output");
    if (c->E.f64) return fail(SU2_ESTATE, "the streaming floor kernel covers FP32 links");
    HIP_TRY(launch_test_stream(c->E.ens(), mu, parity, static_cast<float *>(out_dev), c->E.stream));
    return SU2_OK;
    SU2_API_END
}

int su2_test_index_map(const int32_t dims[4], int tile_z, int tile_t, int parity, uint32_t *out)
{
    SU2_API_BEGIN
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!out || (parity != 0 && parity != 1)) return fail(SU2_EINVAL, "bad arguments");
    uint32_t lz, lt;
    if ((rc = lg_of_tile(tile_z, 3, &lz))) return rc;
    if ((rc = lg_of_tile(tile_t, 3, &lt))) return rc;
    if ((tile_z && dims[2] % tile_z) || (tile_t && dims[3] % tile_t))
        return fail(SU2_EINVAL, "tile sizes must divide the extents");
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
    SU2_API_END
}

int su2_test_gauge_transform(su2_ctx *c, uint64_t seed)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->E.f64) return fail(SU2_ESTATE, "the gauge transformation covers FP32 links");
    void *G = nullptr;
    HIP_TRY(hipMalloc(&G, (size_t)volume_of(c->E.dims[0].data()) * 16));
    hipError_t e = launch_gauge(c->E.ens(), (float *)G, seed, c->E.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->E.stream);
    (void)hipFree(G);
    if (e != hipSuccess) return fail(SU2_EHIP, std::string("gauge: ") + hipGetErrorString(e));
    return SU2_OK;
    SU2_API_END
}

/* ===================================================== learned proposal */

static void nn_free(su2_nn *n)
{
    // b.a0 lives inside the b.alpha allocation and b.loss inside b.act
    // (b.table points kNNTablePad floats into b.table_alloc)
    float *bufs[] = {n->b.params, n->b.grad, n->b.m, n->b.v, n->b.alpha, n->b.act,
                     n->b.table_alloc};
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
    SU2_API_BEGIN
    if (!out) return fail(SU2_EINVAL, "out is NULL");
    *out = nullptr;
    su2_nn *n = new (std::nothrow) su2_nn();
    if (!n) return fail(SU2_ENOMEM, "host allocation failed");
    n->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
    float **bufs[] = {&n->b.params, &n->b.grad, &n->b.m, &n->b.v};
    for (float **pp : bufs)
        if (e == hipSuccess) e = hipMalloc(pp, kNNParams * sizeof(float));
    const size_t tab_bytes = ((size_t)su2dev::kNNTablePad + (size_t)kNNRows * kNNRow) * sizeof(float);
    if (e == hipSuccess) e = hipMalloc(&n->b.table_alloc, tab_bytes);
    if (e == hipSuccess) e = hipMemset(n->b.table_alloc, 0, tab_bytes);
    if (e == hipSuccess) n->b.table = n->b.table_alloc + su2dev::kNNTablePad;
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
    SU2_API_END
}

int su2_nn_destroy(su2_nn *n)
{
    SU2_API_BEGIN
    if (!n) return fail(SU2_EINVAL, "nn is NULL");
    if (const int u = n->users.load())
        return fail(SU2_ESTATE, "the proposal is still attached to " + std::to_string(u) +
                                    " lattice(s) or batch(es); detach it with "
                                    "su2_set_proposal(..., NULL) or destroy them first");
    (void)hipStreamSynchronize(n->stream);
    nn_free(n);
    delete n;
    return SU2_OK;
    SU2_API_END
}

int su2_nn_get_params(su2_nn *n, float *host)
{
    SU2_API_BEGIN
    if (!n || !host) return fail(SU2_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(n->stream));
    HIP_TRY(hipMemcpy(host, n->b.params, kNNParams * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
    SU2_API_END
}

int su2_nn_set_params(su2_nn *n, const float *host)
{
    SU2_API_BEGIN
    if (!n || !host) return fail(SU2_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(n->stream));
    HIP_TRY(hipMemcpy(n->b.params, host, kNNParams * sizeof(float), hipMemcpyHostToDevice));
    n->table_ready = false;
    return SU2_OK;
    SU2_API_END
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
    SU2_API_BEGIN
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
    SU2_API_END
}

int su2_nn_set_data(su2_nn *n, int64_t count, const float *alpha_host, const float *a0_host)
{
    SU2_API_BEGIN
    if (!n || !alpha_host || !a0_host || count <= 0) return fail(SU2_EINVAL, "bad arguments");
    int rc = nn_reserve_data(n, count);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(n->b.alpha, alpha_host, count * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(n->b.a0, a0_host, count * sizeof(float), hipMemcpyHostToDevice));
    return SU2_OK;
    SU2_API_END
}

int su2_nn_get_data(su2_nn *n, int64_t *count, float *alpha_host, float *a0_host)
{
    SU2_API_BEGIN
    if (!n || !count) return fail(SU2_EINVAL, "bad arguments");
    *count = n->ndata;
    HIP_TRY(hipStreamSynchronize(n->stream));
    if (alpha_host && n->ndata)
        HIP_TRY(hipMemcpy(alpha_host, n->b.alpha, n->ndata * sizeof(float), hipMemcpyDeviceToHost));
    if (a0_host && n->ndata)
        HIP_TRY(hipMemcpy(a0_host, n->b.a0, n->ndata * sizeof(float), hipMemcpyDeviceToHost));
    return SU2_OK;
    SU2_API_END
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
    SU2_API_BEGIN
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
    SU2_API_END
}

// Learning rate of Adam step t of `steps`: constant lr0, or a cosine from
// lr0 down towards lr1.
struct LRSchedule {
    double lr0, lr1;
    int32_t steps;
    bool cosine;
    double at(int32_t t) const
    {
        if (!cosine) return lr0;
        const double pi = 3.14159265358979323846;
        return lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(pi * (double)t / (double)steps));
    }
};

static int nn_train_steps(su2_nn *n, int32_t steps, int32_t batch, const LRSchedule &sched,
                          double *loss_history_host)
{
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
        HIP_TRY(launch_nn_adam(n->b, (float)sched.at(t), ++n->step, n->stream));
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

int su2_nn_train(su2_nn *n, int32_t steps, int32_t batch, double lr, double *loss_history_host)
{
    SU2_API_BEGIN
    if (!n || steps < 0 || batch <= 0 || !(lr > 0.0)) return fail(SU2_EINVAL, "bad arguments");
    return nn_train_steps(n, steps, batch, LRSchedule{lr, lr, steps, false}, loss_history_host);
    SU2_API_END
}

int su2_nn_train_cosine(su2_nn *n, int32_t steps, int32_t batch, double lr0, double lr1,
                        double *loss_history_host)
{
    SU2_API_BEGIN
    if (!n || steps < 0 || batch <= 0 || !(lr0 > 0.0) || !(lr1 > 0.0))
        return fail(SU2_EINVAL, "bad arguments");
    return nn_train_steps(n, steps, batch, LRSchedule{lr0, lr1, steps, true}, loss_history_host);
    SU2_API_END
}

int su2_nn_build_table(su2_nn *n)
{
    SU2_API_BEGIN
    if (!n) return fail(SU2_EINVAL, "nn is NULL");
    HIP_TRY(launch_nn_table(n->b.params, n->b.table, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    n->table_ready = true;
    return SU2_OK;
    SU2_API_END
}

int su2_nn_get_table(su2_nn *n, float *host)
{
    SU2_API_BEGIN
    if (!n || !host) return fail(SU2_EINVAL, "NULL argument");
    if (!n->table_ready) return fail(SU2_ESTATE, "table not built (su2_nn_build_table)");
    HIP_TRY(hipMemcpy(host, n->b.table, (size_t)kNNRows * kNNRow * sizeof(float),
                      hipMemcpyDeviceToHost));
    return SU2_OK;
    SU2_API_END
}

int su2_set_proposal(su2_ctx *c, su2_nn *n)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    if (n && !n->table_ready) return fail(SU2_ESTATE, "table not built (su2_nn_build_table)");
    c->E.drop_graph();
    c->E.table = n ? n->b.table : nullptr;
    attach_proposal(c->proposal, n);
    return SU2_OK;
    SU2_API_END
}

int su2_batch_set_proposal(su2_batch *b, su2_nn *n)
{
    SU2_API_BEGIN
    int rc = check_batch(b);
    if (rc) return rc;
    if (n && !n->table_ready) return fail(SU2_ESTATE, "table not built (su2_nn_build_table)");
    b->E.drop_graph();
    b->E.table = n ? n->b.table : nullptr;
    attach_proposal(b->proposal, n);
    return SU2_OK;
    SU2_API_END
}

int su2_get_accept_stats(su2_ctx *c, uint64_t *proposed, uint64_t *accepted, int reset)
{
    SU2_API_BEGIN
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->E.counts(reset, proposed, accepted);
    SU2_API_END
}

int su2_test_learned_links(su2_nn *n, const float *V_host, const float *Uold_host, int64_t count,
                           double beta, uint64_t seed, uint32_t sweep, uint32_t mu,
                           uint32_t replica, double or_width, float *out_host,
                           int32_t *accepted_host)
{
    SU2_API_BEGIN
    if (!n || count < 0 || (count > 0 && (!V_host || !Uold_host || !out_host)))
        return fail(SU2_EINVAL, "bad arguments");
    if (!(or_width <= 1.0)) return fail(SU2_EINVAL, "or_width must be <= 1 (< 0: off)");
    if (!beta_ok(beta)) return fail(SU2_EINVAL, "beta must be finite and >= 0");
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
                                (float)beta, seed, sweep, mu, replica,
                                or_width < 0.0 ? -1.0f : (float)or_width, (float *)dout,
                                (int32_t *)dacc, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out_host, dout, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && accepted_host)
        e = hipMemcpy(accepted_host, dacc, (size_t)count * 4, hipMemcpyDeviceToHost);
    void *bufs[] = {dv, du, dout, dacc};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    if (e != hipSuccess) return fail(SU2_EHIP, std::string("test_learned: ") + hipGetErrorString(e));
    return SU2_OK;
    SU2_API_END
}

}  // extern "C"

