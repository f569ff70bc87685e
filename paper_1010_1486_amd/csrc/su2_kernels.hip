// su2_kernels.hip -- gfx950 kernels of the SU(2) checkerboard heat bath.
//
// Cardoso & Bicudo, "Lattice SU(2) on GPU's" (LAT2010):
//   Sec. 2   six-staple sum V, k = sqrt(det V), a0 ~ sqrt(1-a0^2) exp(beta k a0),
//            U' = X U~^{-1}
//   Sec. 4   kernels: cold/hot start, heat bath per (direction, parity),
//            plaquette, Polyakov loop, sum over the lattice
// The pass kernel streams the structure-of-arrays planes of one (mu, parity)
// class; plaquette and Polyakov sums are FP64 wave/LDS trees with block
// partials summed by a one-block kernel in a fixed order (deterministic).
#include "su2_internal.h"

using namespace su2dev;

namespace su2rt {

namespace {

__device__ __forceinline__ void decode(const Geom &g, uint32_t h, int par, int &x, int &y,
                                       int &z, int &t)
{
    uint32_t xh = h % g.hx;
    uint32_t r = h / g.hx;
    y = (int)(r % (uint32_t)g.ny);
    r /= (uint32_t)g.ny;
    z = (int)(r % (uint32_t)g.nz);
    t = (int)(r / (uint32_t)g.nz);
    x = 2 * (int)xh + ((par + y + z + t) & 1);
}

__device__ __forceinline__ uint32_t hidx(const Geom &g, int x, int y, int z, int t)
{
    return (uint32_t)(x >> 1) + g.hx * ((uint32_t)y + (uint32_t)g.ny * ((uint32_t)z +
                                        (uint32_t)g.nz * (uint32_t)t));
}

__device__ __forceinline__ int wrap_up(int c, int n) { return c + 1 == n ? 0 : c + 1; }
__device__ __forceinline__ int wrap_dn(int c, int n) { return c == 0 ? n - 1 : c - 1; }

struct Site {
    int c[4];
};

__device__ __forceinline__ uint32_t hidx(const Geom &g, const Site &s)
{
    return hidx(g, s.c[0], s.c[1], s.c[2], s.c[3]);
}

__device__ __forceinline__ Site shifted(const Geom &g, Site s, int mu, int step)
{
    const int n = mu == 0 ? g.nx : mu == 1 ? g.ny : mu == 2 ? g.nz : g.nt;
    s.c[mu] = step > 0 ? wrap_up(s.c[mu], n) : wrap_dn(s.c[mu], n);
    return s;
}

// FP64 sum over the block; the result is valid in thread 0.  Fixed order.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double wsum[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) wsum[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r += wsum[i];
    }
    return r;
}

// Map the hardware workgroup id to a logical tile so that the workgroups one
// XCD runs (dispatched round-robin over the 8 XCDs) cover one contiguous
// stretch of the lattice and share that XCD's L2.
__device__ __forceinline__ uint32_t logical_block(uint32_t b, uint32_t nb, bool remap)
{
    if (!remap) return b;
    const uint32_t per = nb >> 3;          // full rounds
    const uint32_t full = per << 3;
    if (b >= full) return b;               // ragged tail keeps its id
    return (b & 7u) * per + (b >> 3);
}

// ------------------------------------------------------------------- init
__global__ void init_kernel(float *__restrict__ links, Geom g, int start, uint32_t k0,
                            uint32_t k1, uint32_t replica)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    const int mp = blockIdx.y;  // mu * 2 + parity
    if (h >= g.vh) return;
    const int mu = mp >> 1, par = mp & 1;
    Q q{1.0f, 0.0f, 0.0f, 0.0f};
    if (start) {
        int x, y, z, t;
        decode(g, h, par, x, y, z, t);
        const uint32_t s = 2u * h + (uint32_t)(x & 1);
        q = haar_from_block(philox(s, 0u, word2((uint32_t)mu, TAG_HOT, replica), 0u, k0, k1));
    }
    store_q(links, g.vh, mu, par, h, q);
}

// ------------------------------------------------------------------- pass
// One heat-bath pass over the sites of parity `par`, direction `mu`.  With
// MEASURE, (1/2)Tr(U'_mu(s) V_nu(s)) summed over nu < mu is accumulated: over
// the odd passes of mu = 1, 2, 3 this is every plaquette of the end-of-sweep
// configuration exactly once.
template <bool MEASURE>
__global__ __launch_bounds__(256) void pass_kernel(float *__restrict__ links, Geom g, int mu,
                                                   int par, const uint32_t *__restrict__ sweep_ptr,
                                                   float beta, uint32_t k0, uint32_t k1,
                                                   uint32_t replica, double *__restrict__ partial,
                                                   int remap)
{
    const uint32_t blk = logical_block(blockIdx.x, gridDim.x, remap);
    const uint32_t h = blk * blockDim.x + threadIdx.x;
    float meas = 0.0f;
    if (h < g.vh) {
        const uint32_t sweep = *sweep_ptr;
        const int opp = par ^ 1;
        Site s;
        decode(g, h, par, s.c[0], s.c[1], s.c[2], s.c[3]);
        const Site s_pmu = shifted(g, s, mu, +1);
        Q V{0.0f, 0.0f, 0.0f, 0.0f};
        Q Vlow{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            const Site s_pnu = shifted(g, s, nu, +1);
            const Site s_mnu = shifted(g, s, nu, -1);
            const Site s_pmu_mnu = shifted(g, s_pmu, nu, -1);
            // forward: U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+
            const Q A = load_q(links, g.vh, nu, opp, hidx(g, s_pmu));
            const Q B = load_q(links, g.vh, mu, opp, hidx(g, s_pnu));
            const Q C = load_q(links, g.vh, nu, par, h);
            const Q fwd = qmul(qmul(A, qdag(B)), qdag(C));
            // backward: U_nu(s+mu-nu)^+ U_mu(s-nu)^+ U_nu(s-nu)
            const Q D = load_q(links, g.vh, nu, par, hidx(g, s_pmu_mnu));
            const Q E = load_q(links, g.vh, mu, opp, hidx(g, s_mnu));
            const Q F = load_q(links, g.vh, nu, opp, hidx(g, s_mnu));
            const Q bwd = qmul(qmul(qdag(D), qdag(E)), F);
            const Q st = qadd(fwd, bwd);
            V = qadd(V, st);
            if (MEASURE && nu < mu) Vlow = qadd(Vlow, st);
        }
        const uint32_t site = 2u * h + (uint32_t)(s.c[0] & 1);
        const Q Un = heatbath_link(V, beta, site, sweep, (uint32_t)mu, replica, k0, k1);
        store_q(links, g.vh, mu, par, h, Un);
        if (MEASURE) meas = retr(Un, Vlow);
    }
    if (MEASURE) {
        const double b = block_sum((double)meas);
        if (threadIdx.x == 0) partial[blk] = b;
    }
}

// -------------------------------------------------------------- plaquette
// One thread per site (both parities): the six plaquettes
// (1/2)Tr U_mu(s) U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+ = (1/2)Tr(P Q^+) with
// P = U_mu(s) U_nu(s+mu), Q = U_nu(s) U_mu(s+nu).
__global__ __launch_bounds__(256) void plaquette_kernel(const float *__restrict__ links, Geom g,
                                                        double *__restrict__ partial)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < 2u * g.vh) {
        const int par = i >= g.vh ? 1 : 0;
        const uint32_t h = par ? i - g.vh : i;
        const int opp = par ^ 1;
        Site s;
        decode(g, h, par, s.c[0], s.c[1], s.c[2], s.c[3]);
        Q U[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) U[mu] = load_q(links, g.vh, mu, par, h);
        float sum = 0.0f;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const uint32_t hm = hidx(g, shifted(g, s, mu, +1));
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                const uint32_t hn = hidx(g, shifted(g, s, nu, +1));
                const Q P = qmul(U[mu], load_q(links, g.vh, nu, opp, hm));
                const Q Qq = qmul(U[nu], load_q(links, g.vh, mu, opp, hn));
                sum += retr_adj(P, Qq);
            }
        }
        acc = (double)sum;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// --------------------------------------------------------------- Polyakov
// One thread per spatial site: L(x) = (1/2)Tr prod_{t=0}^{Nt-1} U_3(x, t).
__global__ __launch_bounds__(256) void polyakov_kernel(const float *__restrict__ links, Geom g,
                                                       double *__restrict__ partial)
{
    const uint32_t ns3 = (uint32_t)g.nx * g.ny * g.nz;
    const uint32_t xs = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (xs < ns3) {
        const int x = (int)(xs % (uint32_t)g.nx);
        const uint32_t r = xs / (uint32_t)g.nx;
        const int y = (int)(r % (uint32_t)g.ny), z = (int)(r / (uint32_t)g.ny);
        Q P{1.0f, 0.0f, 0.0f, 0.0f};
        for (int t = 0; t < g.nt; ++t) {
            const int par = (x + y + z + t) & 1;
            P = qmul(P, load_q(links, g.vh, 3, par, hidx(g, x, y, z, t)));
        }
        acc = (double)P.w;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ partial,
                                                       int nblocks, int narrays, size_t stride,
                                                       double scale, double *__restrict__ out,
                                                       int abs_too)
{
    double acc = 0.0;
    for (int a = 0; a < narrays; ++a)
        for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partial[a * stride + i];
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) {
        out[0] = tot * scale;
        if (abs_too) out[1] = fabs(tot * scale);
    }
}

// End of a sweep: optional fused-plaquette sum, history append, counters.
// measure: bit 0 plaquette from the fused partials, bit 1 plaquette from
// extra[R_PLAQ], bit 2 Polyakov from extra[R_POLY_*].
__global__ __launch_bounds__(256) void sweep_end_kernel(Counters *__restrict__ c,
                                                        const double *__restrict__ partial,
                                                        int nblocks, size_t stride, double scale,
                                                        int measure, double *__restrict__ hist,
                                                        const double *__restrict__ extra)
{
    double acc = 0.0;
    if (measure & 1)
        for (int a = 0; a < 3; ++a)
            for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partial[a * stride + i];
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) {
        if (measure && hist) {
            const uint32_t m = c->meas_idx;
            double p = 0.0, ls = 0.0, la = 0.0;
            if (measure & 1) p = tot * scale;
            if (measure & 2) p = extra[R_PLAQ];
            if (measure & 4) {
                ls = extra[R_POLY_SIGNED];
                la = extra[R_POLY_ABS];
            }
            hist[3 * (size_t)m + 0] = p;
            hist[3 * (size_t)m + 1] = ls;
            hist[3 * (size_t)m + 2] = la;
            c->meas_idx = m + 1;
        }
        c->sweep = c->sweep + 1;
    }
}

__global__ void set_counter_kernel(Counters *c, uint32_t sweep, uint32_t meas, int which)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (which & 1) c->sweep = sweep;
        if (which & 2) c->meas_idx = meas;
    }
}

// --------------------------------------------------------------- reunit
// U <- U / |U| with |U|^2 accumulated in FP64.
__global__ __launch_bounds__(256) void reunit_kernel(float *__restrict__ links, Geom g)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    const int mp = blockIdx.y;
    if (h >= g.vh) return;
    const int mu = mp >> 1, par = mp & 1;
    const Q q = load_q(links, g.vh, mu, par, h);
    const double n2 = (double)q.w * q.w + (double)q.x * q.x + (double)q.y * q.y +
                      (double)q.z * q.z;
    const double inv = 1.0 / sqrt(n2);
    store_q(links, g.vh, mu, par, h,
            Q{(float)(q.w * inv), (float)(q.x * inv), (float)(q.y * inv), (float)(q.z * inv)});
}

// ---------------------------------------------------------- gauge (tests)
__global__ void gauge_gen_kernel(float4 *__restrict__ G, Geom g, uint32_t k0, uint32_t k1,
                                 uint32_t replica)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 2u * g.vh) return;
    const Q q = haar_from_block(philox(s, 0u, word2(0u, TAG_GAUGE, replica), 0u, k0, k1));
    G[s] = make_float4(q.w, q.x, q.y, q.z);
}

__global__ void gauge_apply_kernel(float *__restrict__ links, Geom g,
                                   const float4 *__restrict__ G)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    const int mp = blockIdx.y;
    if (h >= g.vh) return;
    const int mu = mp >> 1, par = mp & 1;
    Site s;
    decode(g, h, par, s.c[0], s.c[1], s.c[2], s.c[3]);
    const uint32_t site = 2u * h + (uint32_t)(s.c[0] & 1);
    const Site f = shifted(g, s, mu, +1);
    const uint32_t fsite = 2u * hidx(g, f) + (uint32_t)(f.c[0] & 1);
    const float4 a = G[site], b = G[fsite];
    const Q U = load_q(links, g.vh, mu, par, h);
    const Q r = qmul(qmul(Q{a.x, a.y, a.z, a.w}, U), qdag(Q{b.x, b.y, b.z, b.w}));
    store_q(links, g.vh, mu, par, h, r);
}

// ---------------------------------------------------------- test hooks
__global__ void test_philox_kernel(const uint32_t *__restrict__ ctr, int64_t n, uint32_t k0,
                                   uint32_t k1, uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 w = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = w.a;
    out[4 * i + 1] = w.b;
    out[4 * i + 2] = w.c;
    out[4 * i + 3] = w.d;
}

__global__ void test_links_kernel(const float4 *__restrict__ V, int64_t n, float beta,
                                  uint32_t k0, uint32_t k1, uint32_t sweep, uint32_t mu,
                                  uint32_t replica, float4 *__restrict__ out,
                                  int32_t *__restrict__ ntrials)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 v = V[i];
    const Q Vq{v.x, v.y, v.z, v.w};
    const Q U = heatbath_link(Vq, beta, (uint32_t)i, sweep, mu, replica, k0, k1);
    out[i] = make_float4(U.w, U.x, U.y, U.z);
    if (ntrials) {
        int nt = 0;
        sample_delta(beta * sqrtf(qdot(Vq, Vq)), (uint32_t)i, sweep, word2(mu, TAG_TRIAL, replica),
                     k0, k1, &nt);
        ntrials[i] = nt;
    }
}

inline uint32_t lo32(uint64_t v) { return (uint32_t)v; }
inline uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
inline unsigned nblk(uint64_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t max_partial_blocks(int64_t volume)
{
    return (size_t)((volume + kMinBlock - 1) / kMinBlock) + 8;
}

hipError_t launch_init(float *links, const Geom &g, int start, uint64_t seed, uint32_t replica,
                       hipStream_t stream)
{
    dim3 grid(nblk(g.vh, 256), 8);
    hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, stream, links, g, start, lo32(seed),
                       hi32(seed), replica);
    return hipGetLastError();
}

int pass_grid(const Geom &g, const LaunchCfg &cfg) { return (int)nblk(g.vh, cfg.pass_block); }

hipError_t launch_pass(float *links, const Geom &g, int mu, int par, const uint32_t *sweep_ptr,
                       float beta, uint64_t seed, uint32_t replica, double *partial,
                       const LaunchCfg &cfg, hipStream_t stream)
{
    const unsigned nb = (unsigned)pass_grid(g, cfg);
    if (partial)
        hipLaunchKernelGGL(pass_kernel<true>, dim3(nb), dim3(cfg.pass_block), 0, stream, links, g,
                           mu, par, sweep_ptr, beta, lo32(seed), hi32(seed), replica, partial,
                           (int)cfg.xcd_remap);
    else
        hipLaunchKernelGGL(pass_kernel<false>, dim3(nb), dim3(cfg.pass_block), 0, stream, links,
                           g, mu, par, sweep_ptr, beta, lo32(seed), hi32(seed), replica, partial,
                           (int)cfg.xcd_remap);
    return hipGetLastError();
}

hipError_t launch_plaquette(const float *links, const Geom &g, double *partial, int *nblocks,
                            hipStream_t stream)
{
    const unsigned nb = nblk(2ull * g.vh, 256);
    *nblocks = (int)nb;
    hipLaunchKernelGGL(plaquette_kernel, dim3(nb), dim3(256), 0, stream, links, g, partial);
    return hipGetLastError();
}

hipError_t launch_polyakov(const float *links, const Geom &g, double *partial, int *nblocks,
                           hipStream_t stream)
{
    const unsigned nb = nblk((uint64_t)g.nx * g.ny * g.nz, 256);
    *nblocks = (int)nb;
    hipLaunchKernelGGL(polyakov_kernel, dim3(nb), dim3(256), 0, stream, links, g, partial);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, int nblocks, int narrays, size_t stride,
                           double scale, double *out, int abs_too, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, stream, partial, nblocks, narrays,
                       stride, scale, out, abs_too);
    return hipGetLastError();
}

hipError_t launch_sweep_end(Counters *counters, const double *partial, int nblocks,
                            size_t stride, double scale, int measure, double *hist,
                            const double *extra, hipStream_t stream)
{
    hipLaunchKernelGGL(sweep_end_kernel, dim3(1), dim3(256), 0, stream, counters, partial,
                       nblocks, stride, scale, measure, hist, extra);
    return hipGetLastError();
}

hipError_t launch_set_counter(Counters *c, uint32_t sweep, uint32_t meas, int which,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, stream, c, sweep, meas, which);
    return hipGetLastError();
}

hipError_t launch_reunitarize(float *links, const Geom &g, hipStream_t stream)
{
    hipLaunchKernelGGL(reunit_kernel, dim3(nblk(g.vh, 256), 8), dim3(256), 0, stream, links, g);
    return hipGetLastError();
}

hipError_t launch_gauge(float *links, const Geom &g, float *G, uint64_t seed, uint32_t replica,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(gauge_gen_kernel, dim3(nblk(2ull * g.vh, 256)), dim3(256), 0, stream,
                       (float4 *)G, g, lo32(seed), hi32(seed), replica);
    hipLaunchKernelGGL(gauge_apply_kernel, dim3(nblk(g.vh, 256), 8), dim3(256), 0, stream, links,
                       g, (const float4 *)G);
    return hipGetLastError();
}

hipError_t launch_test_philox(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out,
                              hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(test_philox_kernel, dim3(nblk((uint64_t)n, 256)), dim3(256), 0, stream,
                       ctr, n, lo32(seed), hi32(seed), out);
    return hipGetLastError();
}

hipError_t launch_test_links(const float *V, int64_t n, float beta, uint64_t seed,
                             uint32_t sweep, uint32_t mu, uint32_t replica, float *out,
                             int32_t *ntrials, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(test_links_kernel, dim3(nblk((uint64_t)n, 256)), dim3(256), 0, stream,
                       (const float4 *)V, n, beta, lo32(seed), hi32(seed), sweep, mu, replica,
                       (float4 *)out, ntrials);
    return hipGetLastError();
}

}  // namespace su2rt
