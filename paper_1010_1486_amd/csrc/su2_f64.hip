// su2_f64.hip -- the heat bath with FP64 links and staples (single lattice).
//
// The paper ran in single precision and names double precision as the next
// step (Conclusions).  This path keeps every link, staple, normalisation,
// sampler step and product of the update in FP64: the Sec. 2 update
// (six-staple sum V, k = sqrt(det V), a0 ~ sqrt(1 - a0^2) exp(beta k a0),
// U' = X U~^+), the Sec. 4 kernels (cold/hot start, one launch per
// (direction, parity), plaquette, Polyakov loop) and the reunitarisation.  The
// Philox streams, the traversal of the lattice and the fixed-point global sums
// are those of the FP32 path, so the two precisions differ at equal seeds only
// by the FP32 rounding.  Layout: 8 classes (mu * 2 + parity), each two arrays
// of V/2 double pairs -- (a0, a1), then (a2, a3) -- indexed by the half-site
// h = s >> 1, so that every wave-wide 16-byte load reads one contiguous
// kilobyte (a 32-byte link per lane would spread each load over twice the
// cache lines).
#include "su2_internal.h"
#include "su2_kcommon.h"

using namespace su2dev;

namespace su2rt {

namespace {

struct QD {
    double w, x, y, z;
};

// (a0 + i a.s)(b0 + i b.s) = (a0 b0 - a.b) + i (a0 b + b0 a - a x b).s
__device__ __forceinline__ QD dmul(const QD &a, const QD &b)
{
    QD c;
    c.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    c.x = a.w * b.x + b.w * a.x - (a.y * b.z - a.z * b.y);
    c.y = a.w * b.y + b.w * a.y - (a.z * b.x - a.x * b.z);
    c.z = a.w * b.z + b.w * a.z - (a.x * b.y - a.y * b.x);
    return c;
}
__device__ __forceinline__ QD ddag(const QD &a) { return QD{a.w, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ QD dadd(const QD &a, const QD &b)
{
    return QD{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z};
}
__device__ __forceinline__ double ddot(const QD &a, const QD &b)
{
    return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}
// (1/2) Tr(a b) = a0 b0 - a.b
__device__ __forceinline__ double dretr(const QD &a, const QD &b)
{
    return a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
}

// Class (mu, par) starts at byte 32 vh (mu * 2 + par); its (a2, a3) half
// 16 vh bytes further.  Uniform bases and one 32-bit offset h * 16 per link
// (V/2 < 2^28).
typedef __attribute__((address_space(1))) const char gcd;
typedef __attribute__((address_space(1))) char gcd_w;
typedef double v2d __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const v2d gv2d;
typedef __attribute__((address_space(1))) v2d gv2d_w;

__device__ __forceinline__ QD ldd(const double *links, uint32_t vh, int mu, int par, uint32_t h)
{
    gcd *lo = (gcd *)links + (size_t)(mu * 2 + par) * vh * 32u;
    gcd *hi = lo + (size_t)vh * 16u;
    const v2d a = *(gv2d *)(lo + h * 16u), b = *(gv2d *)(hi + h * 16u);
    return QD{a.x, a.y, b.x, b.y};
}

__device__ __forceinline__ void std4(double *links, uint32_t vh, int mu, int par, uint32_t h,
                                     const QD &q)
{
    gcd_w *lo = (gcd_w *)links + (size_t)(mu * 2 + par) * vh * 32u;
    gcd_w *hi = lo + (size_t)vh * 16u;
    *(gv2d_w *)(lo + h * 16u) = v2d{q.w, q.x};
    *(gv2d_w *)(hi + h * 16u) = v2d{q.y, q.z};
}

// Store with the nontemporal hint (the pass writes a class no other site of
// the pass reads).
__device__ __forceinline__ void std4_nt(double *links, uint32_t vh, int mu, int par, uint32_t h,
                                        const QD &q)
{
    v2d *lo = reinterpret_cast<v2d *>(links) + (size_t)(mu * 2 + par) * 2u * vh;
    v2d *hi = lo + vh;
    __builtin_nontemporal_store(v2d{q.w, q.x}, lo + h);
    __builtin_nontemporal_store(v2d{q.y, q.z}, hi + h);
}

// The uniform of a Philox word, (2 (w >> 9) + 1) 2^-24 (exact in FP64).
__device__ __forceinline__ double ud(uint32_t w) { return (double)(2u * (w >> 9) + 1u) * 0x1p-24; }

// Exact draw of delta = 1 - a0 from sqrt(1 - a0^2) exp(alpha a0), in FP64
// with the trials of the FP32 sampler: Kennedy-Pendleton for alpha >= 1
// (delta = -(ln r1 + cos^2(2 pi r2) ln r3) / alpha, accepted when
// r4^2 <= 1 - delta/2), else a0 = sqrt(r1) cos(2 pi r2) accepted when
// r3 <= exp(alpha (a0 - 1)).  Trial t uses block (site, sweep, w2, t).
__device__ __forceinline__ double sample_delta_d(double alpha, U4 w, uint32_t site,
                                                 uint32_t sweep, uint32_t w2, uint32_t k0,
                                                 uint32_t k1)
{
    const bool kp = alpha >= (double)kKPMinAlpha;
    double delta = 0.0;
    int t = 0;
    for (;;) {
        const double r1 = ud(w.a), r2 = ud(w.b), r3 = ud(w.c), r4 = ud(w.d);
        double d;
        bool acc;
        if (kp) {
            const double c = cospi(2.0 * r2);
            d = -(log(r1) + c * c * log(r3)) / alpha;
            acc = r4 * r4 <= 1.0 - 0.5 * d;
        } else {
            const double a0 = sqrt(r1) * cospi(2.0 * r2);
            d = 1.0 - a0;
            acc = r3 <= exp(alpha * (a0 - 1.0));
        }
        if (acc) {
            delta = d;
            break;
        }
        if (++t >= kTrialCap) break;
        w = philox(site, sweep, w2, (uint32_t)t, k0, k1);
    }
    return delta;
}

// U' = X U~^+ with U~ = V / |V|; X = (1 - delta, |a| n), |a| = sqrt(delta (2 -
// delta)), n from the direction uniforms of trial 0 (cos theta = 1 - 2 r5,
// phi = 2 pi r6).  k = 0 gives U~ = 1 and a Haar X.
__device__ __forceinline__ QD heatbath_link_d(const QD &V, double beta, uint32_t site,
                                              uint32_t sweep, uint32_t w2, uint32_t k0,
                                              uint32_t k1)
{
    const double k2 = ddot(V, V);
    const bool zero = !(k2 > 0.0);
    const double k = sqrt(k2);
    const double alpha = beta * k;
    const U4 w0 = philox(site, sweep, w2, 0u, k0, k1);
    float r5f, r6f;
    dir_uniforms(w0, r5f, r6f);  // 18-bit uniforms, exact in FP32 and FP64
    const double r5 = r5f, r6 = r6f;
    const double delta = sample_delta_d(alpha, w0, site, sweep, w2, k0, k1);
    const double amag = sqrt(delta * (2.0 - delta));
    const double sth = 2.0 * sqrt(r5 * (1.0 - r5));
    const double as = amag * sth;
    const QD X{1.0 - delta, as * cospi(2.0 * r6), as * sinpi(2.0 * r6), amag * (1.0 - 2.0 * r5)};
    const double inv = zero ? 0.0 : 1.0 / k;
    const QD Ut = zero ? QD{1.0, 0.0, 0.0, 0.0} : QD{V.w * inv, V.x * inv, V.y * inv, V.z * inv};
    return dmul(X, ddag(Ut));
}

// Haar element from one Philox block: two Box-Muller pairs, normalised.
__device__ __forceinline__ QD haar_d(const U4 &w)
{
    const double u0 = ud(w.a), u1 = ud(w.b), u2 = ud(w.c), u3 = ud(w.d);
    const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
    const QD g{r01 * cospi(2.0 * u1), r01 * sinpi(2.0 * u1), r23 * cospi(2.0 * u3),
               r23 * sinpi(2.0 * u3)};
    const double inv = 1.0 / sqrt(ddot(g, g));
    return QD{g.w * inv, g.x * inv, g.y * inv, g.z * inv};
}

// grid (blocks over V/2, 8 = mu * 2 + parity)
__global__ void init64_kernel(const Rep *__restrict__ reps, int hot, uint32_t k0, uint32_t k1)
{
    const Rep &R = reps[0];
    const Geom &g = R.g;
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= g.vh) return;
    const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
    QD q{1.0, 0.0, 0.0, 0.0};
    if (hot) {
        // site of half-site h with parity par (x fastest, then y, z, t)
        const uint32_t xh = h % g.hx;
        uint32_t r = h / g.hx;
        const uint32_t y = r % (uint32_t)g.ny;
        r /= (uint32_t)g.ny;
        const uint32_t z = r % (uint32_t)g.nz, t = r / (uint32_t)g.nz;
        const uint32_t x = 2u * xh + (((uint32_t)par + y + z + t) & 1u);
        const uint32_t s = 2u * h + (x & 1u);
        q = haar_d(philox(s, 0u, word2((uint32_t)mu, TAG_HOT, R.replica), 0u, k0, k1));
    }
    std4(reinterpret_cast<double *>(R.links), g.vh, mu, par, h, q);
}

// One heat-bath pass (direction MU, parity par) over the lattice, one thread
// per link, in the traversal and workgroup order of the FP32 pass.  MEASURE:
// (1/2)Tr(U'_MU V_nu) summed over nu < MU into the plaquette accumulator.
template <int MU, bool MEASURE>
__global__ __launch_bounds__(256) void pass64_kernel(const Rep *__restrict__ reps, int par,
                                                     uint32_t k0, uint32_t k1, int remap,
                                                     int reverse)
{
    const Rep &R = reps[0];
    const Geom &g = R.g;
    const uint32_t blk = logical_block(blockIdx.x, R.nblocks, remap, reverse);
    const uint32_t gid = blk * blockDim.x + threadIdx.x;
    double meas = 0.0;
    if (gid < g.vh) {
        const uint32_t sweep = *(const __attribute__((address_space(4))) uint32_t *)&R.cnt->sweep;
        double *links = reinterpret_cast<double *>(R.links);
        const int opp = par ^ 1;
        const PassSite s = pass_site(g, gid, par);
        const Deltas d = neighbour_deltas(g, s);
        const uint32_t h = s.h;
        // All 36 loads of the 18 neighbour links are issued before any staple
        // product (the scheduling barrier keeps them together): 156 instead
        // of 104 VGPRs (3 instead of 4 waves per SIMD), every gather of a wave
        // in flight at once instead of about ten; 137-138 instead of
        // 141-142 us per pass at 48^4, the same links.
        QD Ld[3][6];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int nu = j + (j >= MU ? 1 : 0);  // the three nu != MU, in increasing order
            // forward: U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+
            Ld[j][0] = ldd(links, g.vh, nu, opp, h + d.p[MU]);
            Ld[j][1] = ldd(links, g.vh, MU, opp, h + d.p[nu]);
            Ld[j][2] = ldd(links, g.vh, nu, par, h);
            // backward: U_nu(s+mu-nu)^+ U_mu(s-nu)^+ U_nu(s-nu) = (E D)^+ F
            Ld[j][3] = ldd(links, g.vh, nu, par, h + d.p[MU] + d.m[nu]);
            Ld[j][4] = ldd(links, g.vh, MU, opp, h + d.m[nu]);
            Ld[j][5] = ldd(links, g.vh, nu, opp, h + d.m[nu]);
        }
        __builtin_amdgcn_sched_barrier(0);
        QD V{0.0, 0.0, 0.0, 0.0}, Vlow{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int nu = j + (j >= MU ? 1 : 0);
            const QD &A = Ld[j][0], &B = Ld[j][1], &C = Ld[j][2];
            const QD &D = Ld[j][3], &E = Ld[j][4], &F = Ld[j][5];
            const QD st = dadd(dmul(dmul(A, ddag(B)), ddag(C)), dmul(ddag(dmul(E, D)), F));
            V = dadd(V, st);
            if (MEASURE && nu < MU) Vlow = dadd(Vlow, st);
        }
        const uint32_t site = 2u * h + (uint32_t)(s.x & 1);
        const QD Un = heatbath_link_d(V, R.beta_d, site, sweep,
                                      word2((uint32_t)MU, TAG_TRIAL, R.replica), k0, k1);
        std4_nt(links, g.vh, MU, par, h, Un);
        if (MEASURE) meas = dretr(Un, Vlow);
    }
    if (MEASURE) block_accumulate(meas, R.acc, ACC_PLAQ, blockIdx.x);
}

// The six plaquettes rooted at the site of parity par at traversal position
// gid: (1/2)Tr(P Q^+) with P = U_mu(s) U_nu(s+mu), Q = U_nu(s) U_mu(s+nu).
__device__ __forceinline__ double site_plaquettes64(const Geom &g, const double *links,
                                                    uint32_t gid, int par)
{
    const int opp = par ^ 1;
    const PassSite s = pass_site(g, gid, par);
    const Deltas d = neighbour_deltas(g, s);
    QD U[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) U[mu] = ldd(links, g.vh, mu, par, s.h);
    double acc = 0.0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int nu = mu + 1; nu < 4; ++nu) {
            const QD P = dmul(U[mu], ldd(links, g.vh, nu, opp, s.h + d.p[mu]));
            const QD Qq = dmul(U[nu], ldd(links, g.vh, mu, opp, s.h + d.p[nu]));
            acc += ddot(P, Qq);  // (1/2) Tr(P Q^+)
        }
    return acc;
}

// One thread per half-site: the plaquettes rooted at both of its sites (the
// two parities), so that each link class is read as own and as neighbour
// links by the same workgroup.
__global__ __launch_bounds__(256) void plaquette64_kernel(const Rep *__restrict__ reps)
{
    const Rep &R = reps[0];
    const Geom &g = R.g;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < g.vh) {
        const double *links = reinterpret_cast<const double *>(R.links);
        acc = site_plaquettes64(g, links, i, 0) + site_plaquettes64(g, links, i, 1);
    }
    block_accumulate(acc, R.acc, ACC_PLAQ, blockIdx.x);
}

// One thread per spatial site: L(x) = (1/2)Tr prod_t U_3(x, t), t = 0 leftmost.
__global__ __launch_bounds__(256) void polyakov64_kernel(const Rep *__restrict__ reps)
{
    const Rep &R = reps[0];
    const Geom &g = R.g;
    const uint32_t ns3 = (uint32_t)g.nx * g.ny * g.nz;
    const uint32_t xs = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (xs < ns3) {
        const double *links = reinterpret_cast<const double *>(R.links);
        const uint32_t x = xs % (uint32_t)g.nx, q = xs / (uint32_t)g.nx;
        const uint32_t y = q % (uint32_t)g.ny, z = q / (uint32_t)g.ny;
        const uint32_t pbase = (x + y + z) & 1u;
        QD P{1.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < g.nt; ++t)
            P = dmul(P, ldd(links, g.vh, 3, (int)((pbase + (uint32_t)t) & 1u),
                            (xs >> 1) + (uint32_t)t * (ns3 >> 1)));
        acc = P.w;
    }
    block_accumulate(acc, R.acc, ACC_POLY, blockIdx.x);
}

// grid (blocks over V/2, 8): U <- U / |U|.
__global__ void reunit64_kernel(const Rep *__restrict__ reps)
{
    const Rep &R = reps[0];
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= R.g.vh) return;
    const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
    double *links = reinterpret_cast<double *>(R.links);
    const QD q = ldd(links, R.g.vh, mu, par, h);
    const double inv = 1.0 / sqrt(ddot(q, q));
    std4(links, R.g.vh, mu, par, h, QD{q.w * inv, q.x * inv, q.y * inv, q.z * inv});
}

inline uint32_t lo32(uint64_t v) { return (uint32_t)v; }
inline uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
inline unsigned nblk(uint64_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <int MU>
void pass64_mu(const Ens &e, int par, uint64_t seed, bool measure, const LaunchCfg &cfg,
               hipStream_t stream)
{
    const unsigned grid = e.total_blocks;
    const int rev = cfg.snake ? par : 0;
    if (measure)
        hipLaunchKernelGGL((pass64_kernel<MU, true>), dim3(grid), dim3(cfg.pass_block), 0, stream,
                           e.reps, par, lo32(seed), hi32(seed), (int)cfg.xcd_remap, rev);
    else
        hipLaunchKernelGGL((pass64_kernel<MU, false>), dim3(grid), dim3(cfg.pass_block), 0, stream,
                           e.reps, par, lo32(seed), hi32(seed), (int)cfg.xcd_remap, rev);
}

}  // namespace

hipError_t launch_init64(const Ens &e, int hot, uint64_t seed, hipStream_t stream)
{
    hipLaunchKernelGGL(init64_kernel, dim3(nblk(e.max_vh, 256), 8), dim3(256), 0, stream, e.reps,
                       hot, lo32(seed), hi32(seed));
    return hipGetLastError();
}

hipError_t launch_pass64(const Ens &e, int mu, int par, uint64_t seed, bool measure,
                         const LaunchCfg &cfg, hipStream_t stream)
{
    switch (mu) {
    case 0: pass64_mu<0>(e, par, seed, measure, cfg, stream); break;
    case 1: pass64_mu<1>(e, par, seed, measure, cfg, stream); break;
    case 2: pass64_mu<2>(e, par, seed, measure, cfg, stream); break;
    default: pass64_mu<3>(e, par, seed, measure, cfg, stream); break;
    }
    return hipGetLastError();
}

hipError_t launch_plaquette64(const Ens &e, hipStream_t stream)
{
    hipLaunchKernelGGL(plaquette64_kernel, dim3(nblk(e.max_vh, 256)), dim3(256), 0, stream,
                       e.reps);
    return hipGetLastError();
}

hipError_t launch_polyakov64(const Ens &e, hipStream_t stream)
{
    hipLaunchKernelGGL(polyakov64_kernel, dim3(nblk(e.max_ns3, 256)), dim3(256), 0, stream,
                       e.reps);
    return hipGetLastError();
}

hipError_t launch_reunitarize64(const Ens &e, hipStream_t stream)
{
    hipLaunchKernelGGL(reunit64_kernel, dim3(nblk(e.max_vh, 256), 8), dim3(256), 0, stream,
                       e.reps);
    return hipGetLastError();
}

}  // namespace su2rt
