// su2_device.h -- device-side building blocks of the SU(2) heat bath (gfx950).
//
// Quaternion algebra for U = a0 + i a.sigma (Sec. 2 of Cardoso & Bicudo,
// "Lattice SU(2) on GPU's"), the Philox4x32-10 counter-based generator
// (Salmon et al., SC'11), the exact a0 sampler, and the even/odd lattice
// indexing of the structure-of-arrays link layout.
#pragma once

#include <hip/hip_runtime.h>

// Products and sums are fused into FMAs only within one source expression
// (never across statements after inlining), so every kernel built on these
// functions rounds the update identically whatever surrounds it: the plain and
// the LDS-staged pass give bit-identical links.
#pragma clang fp contract(on)
#include <stdint.h>

namespace su2dev {

// ------------------------------------------------------------------ layout
// Links live in 8 classes (mu, parity), each an array of V/2 quaternions
// (float4, components a0..a3) indexed by the half-site h = s >> 1 of the
// canonical site s = x + Nx*(y + Ny*(z + Nz*t)).
struct Geom {
    int32_t nx, ny, nz, nt;
    uint32_t vh;  // V/2
    uint32_t hx;  // Nx/2: half-sites per x row
    uint32_t P;   // Nx*Ny/2: half-sites per (x, y) plane = half-site stride of z
    uint32_t PZ;  // Nx*Ny*Nz/2: half-site stride of t
    // wrap-around jumps in half-sites: (Ny-1)*hx, (Nz-1)*P, (Nt-1)*PZ
    uint32_t wy, wz, wt;
    // Traversal of the pass kernel: (x, y) planes are visited in tiles of
    // 2^lg_tz x 2^lg_tt (z, t) planes, ntz tiles along z.
    uint32_t lg_tz, lg_tt, ntz;
    // Exact division of 31-bit numerators by P, hx and ntz: q = (n * m) >> s.
    uint32_t m_P, s_P, m_hx, s_hx, m_ntz, s_ntz;
};

// n / d for n < 2^31 with m = ceil(2^(31+l)/d), s = 31 + l, l = ceil(log2 d)
// (Granlund & Montgomery 1994, Thm. 4.2 with N = 31).
__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m, uint32_t s)
{
    return (uint32_t)(((uint64_t)n * m) >> s);
}

// ---------------------------------------------------- pass traversal
// Coordinates of the thread's site in the pass traversal: (x, y) planes are
// contiguous in memory; the order of the (z, t) planes is tiled so that the
// t-neighbours a workgroup needs were fetched by recent workgroups of the same
// XCD (the logical block id already groups each XCD's workgroups).
struct PassSite {
    uint32_t h;  // half-site index
    int x, y, z, t;
};

__host__ __device__ __forceinline__ PassSite pass_site(const Geom &g, uint32_t gid, int par)
{
    PassSite ps;
    const uint32_t q = fdiv(gid, g.m_P, g.s_P);  // plane in traversal order
    const uint32_t r = gid - q * g.P;             // half-site within the (x, y) plane
    const uint32_t lg = g.lg_tz + g.lg_tt;
    const uint32_t tile = q >> lg, w = q & ((1u << lg) - 1u);
    const uint32_t tt = fdiv(tile, g.m_ntz, g.s_ntz), tzi = tile - tt * g.ntz;
    ps.z = (int)((tzi << g.lg_tz) + (w & ((1u << g.lg_tz) - 1u)));
    ps.t = (int)((tt << g.lg_tt) + (w >> g.lg_tz));
    const uint32_t y = fdiv(r, g.m_hx, g.s_hx);
    const uint32_t xh = r - y * g.hx;
    ps.y = (int)y;
    ps.x = (int)(2u * xh) + ((par + ps.y + ps.z + ps.t) & 1);
    ps.h = r + g.P * (uint32_t)ps.z + g.PZ * (uint32_t)ps.t;
    return ps;
}

// Half-site offsets (mod 2^32) of the +/-1 neighbours in each direction; they
// add up for diagonal neighbours because each depends on its own coordinate.
struct Deltas {
    uint32_t p[4], m[4];
};

__host__ __device__ __forceinline__ Deltas neighbour_deltas(const Geom &g, const PassSite &s)
{
    Deltas d;
    const bool xodd = s.x & 1;
    d.p[0] = xodd ? (s.x == g.nx - 1 ? 1u - g.hx : 1u) : 0u;
    d.m[0] = xodd ? 0u : (s.x == 0 ? g.hx - 1u : 0xFFFFFFFFu);
    d.p[1] = s.y == g.ny - 1 ? 0u - g.wy : g.hx;
    d.m[1] = s.y == 0 ? g.wy : 0u - g.hx;
    d.p[2] = s.z == g.nz - 1 ? 0u - g.wz : g.P;
    d.m[2] = s.z == 0 ? g.wz : 0u - g.P;
    d.p[3] = s.t == g.nt - 1 ? 0u - g.wt : g.PZ;
    d.m[3] = s.t == 0 ? g.wt : 0u - g.PZ;
    return d;
}

// ------------------------------------------------------------- quaternions
struct Q {
    float w, x, y, z;
};

__device__ __forceinline__ Q qmul(const Q &a, const Q &b)
{
    // (a0 + i a.s)(b0 + i b.s) = (a0 b0 - a.b) + i (a0 b + b0 a - a x b).s, each
    // component as one multiply and three FMAs (a chain with no separate
    // subtraction: 16 VALU operations per product)
    Q c;
    c.w = fmaf(a.w, b.w, -fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)));
    c.x = fmaf(a.w, b.x, fmaf(b.w, a.x, fmaf(-a.y, b.z, a.z * b.y)));
    c.y = fmaf(a.w, b.y, fmaf(b.w, a.y, fmaf(-a.z, b.x, a.x * b.z)));
    c.z = fmaf(a.w, b.z, fmaf(b.w, a.z, fmaf(-a.x, b.y, a.y * b.x)));
    return c;
}
__device__ __forceinline__ Q qdag(const Q &a) { return Q{a.w, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ Q qadd(const Q &a, const Q &b)
{
    return Q{a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z};
}
__device__ __forceinline__ float qdot(const Q &a, const Q &b)
{
    return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}
// (1/2) Tr(a b^+) = a0 b0 + a.b
__device__ __forceinline__ float retr_adj(const Q &a, const Q &b) { return qdot(a, b); }
// (1/2) Tr(a b) = a0 b0 - a.b
__device__ __forceinline__ float retr(const Q &a, const Q &b)
{
    return a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
}

__device__ __forceinline__ Q load_q(const float *__restrict__ base, uint32_t vh, int mu, int par,
                                    uint32_t h)
{
    const float *p = base + (size_t)((mu * 2 + par) * 4) * vh + h;
    return Q{p[0], p[vh], p[2 * (size_t)vh], p[3 * (size_t)vh]};
}

__device__ __forceinline__ void store_q(float *__restrict__ base, uint32_t vh, int mu, int par,
                                        uint32_t h, const Q &q)
{
    float *p = base + (size_t)((mu * 2 + par) * 4) * vh + h;
    p[0] = q.w;
    p[vh] = q.x;
    p[2 * (size_t)vh] = q.y;
    p[3 * (size_t)vh] = q.z;
}

// ------------------------------------------------------------------ Philox
// Philox4x32-10: multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
// 0x9E3779B9 / 0xBB67AE85, ten rounds with the key bumped between rounds.
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// 32-bit word -> (2*(w>>9)+1) * 2^-24: exact in FP32, never 0 or 1.  The 23
// high bits become the mantissa of a float in [1, 2); subtracting 1 - 2^-24
// is exact (Sterbenz) and yields (2m+1) 2^-24.
__device__ __forceinline__ float u01(uint32_t w)
{
    return __uint_as_float((w >> 9) | 0x3f800000u) - 0.99999994039535522f;
}

// 18-bit value m -> (2m+1) * 2^-19.
__device__ __forceinline__ float u18(uint32_t m)
{
    return (float)(2u * m + 1u) * 1.9073486328125e-06f;
}

enum : uint32_t {
    TAG_TRIAL = 0,  // a0 trials; the low 9 bits of draw 0's words give the direction
    TAG_RESERVED = 1,
    TAG_HOT = 2,
    TAG_GAUGE = 3,
    TAG_LEARN = 4,
    TAG_TRAIN = 5,
    TAG_BETA = 6
};

__device__ __forceinline__ uint32_t word2(uint32_t mu, uint32_t tag, uint32_t replica)
{
    return mu | (tag << 2) | (replica << 6);
}

// Hardware transcendentals (single instructions on gfx950).
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// cos(2 pi x), sin(2 pi x): the hardware sine/cosine take revolutions.
__device__ __forceinline__ float hw_cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float hw_sin_rev(float x) { return __builtin_amdgcn_sinf(x); }

constexpr float kLn2 = 0.69314718055994531f;
constexpr float kLog2e = 1.4426950408889634f;

// ----------------------------------------------------------------- sampler
// Exact draw of a0 from sqrt(1 - a0^2) exp(alpha a0) on [-1, 1] (Sec. 2),
// returned as delta = 1 - a0.  alpha >= 1: Kennedy-Pendleton (delta is
// Gamma(3/2, alpha) from two logs and a cos^2, accepted with probability
// sqrt(1 - delta/2)).  alpha < 1: a0 = sqrt(r1) cos(2 pi r2) is Haar
// (semicircle) distributed, accepted with probability exp(alpha (a0 - 1)),
// tested as log2 r3 <= alpha (a0 - 1) log2 e.  Trial t uses the Philox block
// (site, sweep, w2trial, t); the caller passes trial 0's block in `w0`.
// The trial cap is unreachable in practice (acceptance >= 0.41 everywhere);
// on reaching it delta = 0.
constexpr int kTrialCap = 1000;
constexpr float kKPMinAlpha = 1.0f;

__device__ __forceinline__ float sample_delta(float alpha, U4 w, uint32_t site, uint32_t sweep,
                                              uint32_t w2trial, uint32_t k0, uint32_t k1,
                                              int *ntrials = nullptr)
{
    const bool kp = alpha >= kKPMinAlpha;
    const float neg_ln2_over_alpha = -kLn2 * hw_rcp(alpha);
    float delta = 0.0f;
    int t = 0;
    for (;;) {
        const float r1 = u01(w.a), r2 = u01(w.b), r3 = u01(w.c), r4 = u01(w.d);
        float d;
        bool acc;
        if (kp) {
            const float c = hw_cos_rev(r2);
            d = neg_ln2_over_alpha * (hw_log2(r1) + c * c * hw_log2(r3));
            acc = r4 * r4 <= 1.0f - 0.5f * d;
        } else {
            const float a0 = hw_sqrt(r1) * hw_cos_rev(r2);
            d = 1.0f - a0;
            acc = hw_log2(r3) <= alpha * (a0 - 1.0f) * kLog2e;
        }
        if (acc) {
            delta = d;
            break;
        }
        if (++t >= kTrialCap) break;
        w = philox(site, sweep, w2trial, (uint32_t)t, k0, k1);
    }
    if (ntrials) *ntrials = t + 1;
    return delta;
}

// Direction uniforms from the low 9 bits of trial 0's words.
__device__ __forceinline__ void dir_uniforms(const U4 &w, float &r5, float &r6)
{
    r5 = u18((w.a & 511u) | ((w.b & 511u) << 9));
    r6 = u18((w.c & 511u) | ((w.d & 511u) << 9));
}

// X = (1 - delta, |a| n), n uniform on the sphere from (r5, r6):
// cos(theta) = 1 - 2 r5, sin(theta) = 2 sqrt(r5 (1 - r5)), phi = 2 pi r6;
// |a| = sqrt(delta (2 - delta)) avoids cancellation near a0 = 1.
__device__ __forceinline__ Q element_from_delta(float delta, float r5, float r6)
{
    const float amag = hw_sqrt(delta * (2.0f - delta));
    const float cth = 1.0f - 2.0f * r5;
    const float sth = 2.0f * hw_sqrt(r5 * (1.0f - r5));
    const float as = amag * sth;
    return Q{1.0f - delta, as * hw_cos_rev(r6), as * hw_sin_rev(r6), amag * cth};
}

// Heat-bath update of one link from its staple sum V: U' = X U~^+ with
// U~ = V/k, k = |V| (det V = |V|^2 for a sum of quaternions).  k = 0 (only in
// constructed inputs) gives U~ = 1 and a Haar X.
__device__ __forceinline__ Q heatbath_link(const Q &V, float beta, uint32_t site, uint32_t sweep,
                                           uint32_t w2trial, uint32_t k0, uint32_t k1,
                                           int *ntrials = nullptr)
{
    const float k2 = qdot(V, V);
    const bool zero = !(k2 > 0.0f);
    const float inv_k = zero ? 0.0f : hw_rsq(k2);
    const float alpha = beta * k2 * inv_k;
    const U4 w0 = philox(site, sweep, w2trial, 0u, k0, k1);
    float r5, r6;
    dir_uniforms(w0, r5, r6);
    const float delta = sample_delta(alpha, w0, site, sweep, w2trial, k0, k1, ntrials);
    const Q X = element_from_delta(delta, r5, r6);
    const Q Ut = zero ? Q{1.0f, 0.0f, 0.0f, 0.0f}
                      : Q{V.w * inv_k, V.x * inv_k, V.y * inv_k, V.z * inv_k};
    return qmul(X, qdag(Ut));
}


// Microcanonical over-relaxation of one link (not in the paper; Brown & Woch
// 1987, Creutz 1987): with U~ = V/k and X = U U~, the reflection X -> X^+
// keeps x0 = (1/2)Tr(U V)/k and so the weight exp(beta k x0) of Sec. 2, and it
// keeps the Haar measure: U' = X^+ U~^+ = U~^+ U^+ U~^+.  k = 0 leaves U.
__device__ __forceinline__ Q overrelax_link(const Q &V, const Q &U)
{
    const float k2 = qdot(V, V);
    if (!(k2 > 0.0f)) return U;
    const float inv_k = hw_rsq(k2);
    const Q Utd{V.w * inv_k, -V.x * inv_k, -V.y * inv_k, -V.z * inv_k};
    return qmul(qmul(Utd, qdag(U)), Utd);
}

// Reunitarisation of one link: U / |U| with |U|^2 summed in FP64 and each
// component rounded once to FP32.  The reunitarisation kernels and the passes
// that normalise the links they store share it, so both give the same bits.
__device__ __forceinline__ Q unit_q(const Q &q)
{
    const double n2 = (double)q.w * q.w + (double)q.x * q.x + (double)q.y * q.y +
                      (double)q.z * q.z;
    const double inv = 1.0 / sqrt(n2);
    return Q{(float)(q.w * inv), (float)(q.x * inv), (float)(q.y * inv), (float)(q.z * inv)};
}

// ---------------------------------------------------------- learned proposal
// A monotone rational-quadratic spline flow g on [-1, 1] (Durkan et al. 2019)
// maps a0 to u = g(a0), uniform on [-1, 1]; its density q(a0) = g'(a0)/2 is
// the proposal of an independence Metropolis step whose weight
// w(x) = exp(alpha x) sqrt(1 - x^2) / q(x) keeps the heat-bath distribution of
// Sec. 2 exact.  The spline of each alpha comes from the nearest row of a
// 64-row table (rows at f = -1 + 2 j / 63, f = log-scaled alpha in [0.5, 30];
// neighbouring rows are 6.7% apart in alpha) holding [x1..x15, 1, y1..y15, 1,
// d1..d15, 1]; x0 = y0 = -1 and d0 = 1 are implicit.  The table is 12 KB, so
// the pass keeps it in LDS.  Outside [0.5, 30] the exact sampler is used.
constexpr int kNNRows = 64;
constexpr int kNNRow = 48;
constexpr float kNNAlphaLo = 0.5f;
constexpr float kNNAlphaHi = 30.0f;
constexpr float kNNLog2Range = 5.9068905956085187f;  // log2(30 / 0.5)

__device__ __forceinline__ int nn_table_row(float alpha)
{
    // p = (f + 1) (rows - 1) / 2 = log2(alpha / 0.5) (rows - 1) / log2(60)
    const float p = hw_log2(alpha * 2.0f) * ((float)(kNNRows - 1) / kNNLog2Range);
    const int j = (int)(p + 0.5f);
    return j < 0 ? 0 : (j > kNNRows - 1 ? kNNRows - 1 : j);
}

// The device table is preceded by kNNTablePad floats of padding (the LDS copy
// in the pass by 4), so that the update may read the float before a row
// unconditionally (bin 0 has no stored left knot) and then select the
// implicit value.
constexpr int kNNTablePad = 16;

// Index k of the bin holding v among the knots t1..t15 of one row (held in
// registers, loaded as four float4: t[i] = knots[i - 1]): k = #{i : v >= t_i}
// for increasing knots, found by a four-step binary search with selects.
__device__ __forceinline__ int rq_bin_index(const float4 &a, const float4 &b, const float4 &c,
                                            const float4 &d, float v)
{
    // t1..t4 = a, t5..t8 = b, t9..t12 = c, t13..t15 = d.xyz
    const bool c1 = v >= b.w;                       // t8
    const bool c2 = v >= (c1 ? c.w : a.w);          // t12 | t4
    const float s2lo = c1 ? c.y : a.y;              // t10 | t2
    const float s2hi = c1 ? d.y : b.y;              // t14 | t6
    const bool c3 = v >= (c2 ? s2hi : s2lo);
    const float q0 = c1 ? c.x : a.x, q1 = c1 ? c.z : a.z;  // t9 | t1, t11 | t3
    const float q2 = c1 ? d.x : b.x, q3 = c1 ? d.z : b.z;  // t13 | t5, t15 | t7
    const float r0 = c2 ? q2 : q0, r1 = c2 ? q3 : q1;
    const bool c4 = v >= (c3 ? r1 : r0);
    return (c1 ? 8 : 0) | (c2 ? 4 : 0) | (c3 ? 2 : 0) | (c4 ? 1 : 0);
}

struct RQBin {
    float xl, W, yl, H, dl, dh;
};

// Bin k of a row: x_k, x_{k+1} - x_k, y_k, y_{k+1} - y_k, d_k, d_{k+1}.  One
// vector offset serves all six loads (the k - 1 entries may read the padding
// or the previous row; bin 0 then takes the implicit -1, -1, 1).
__device__ __forceinline__ RQBin rq_bin_at(const float *__restrict__ row, int k)
{
    const float *p = row + k;
    const float x0 = p[-1], x1 = p[0], y0 = p[15], y1 = p[16], d0 = p[31], d1 = p[32];
    const bool first = k == 0;
    RQBin b;
    b.xl = first ? -1.0f : x0;
    b.yl = first ? -1.0f : y0;
    b.dl = first ? 1.0f : d0;
    b.W = x1 - b.xl;
    b.H = y1 - b.yl;
    b.dh = d1;
    return b;
}

// g'(x) = s^2 num / den^2 at relative position xi in the bin (s = H / W),
// returned as (s^2 num, den^2) so that quotients can share one reciprocal.
__device__ __forceinline__ void rq_deriv_parts(const RQBin &b, float s, float xi, float &num,
                                               float &den2)
{
    const float om = xi * (1.0f - xi);
    const float den = s + (b.dh + b.dl - 2.0f * s) * om;
    const float omx = 1.0f - xi;
    num = s * s * (b.dh * xi * xi + 2.0f * s * om + b.dl * omx * omx);
    den2 = den * den;
}

// Learned-proposal Metropolis update of one link.  acc: 1 accepted, 0
// rejected (U' = Uold), -1 exact fallback (alpha outside the table range).
//
// orw < 0: independence proposal u = 2 z - 1.  orw >= 0: over-relaxed
// proposal u = wrap(-g(x_old) + orw (2 z - 1)) with wrap onto [-1, 1) of
// period 2 -- the reflection of the old link's flow coordinate plus uniform
// noise of half-width orw.  Its density in u is symmetric, f(u + u_old), so
// the Metropolis ratio is the same weight ratio w(a0') / w(x_old); any orw > 0
// makes two steps a random walk on the circle (irreducible), and orw = 1 is
// the independence proposal again.  With an exact flow the reflection maps
// a0 to its opposite quantile (ordered over-relaxation, Neal 1998).
__device__ __forceinline__ Q learned_link(const Q &V, const Q &Uold, const float *__restrict__ table,
                                          float beta, uint32_t site, uint32_t sweep, uint32_t mu,
                                          uint32_t replica, uint32_t k0, uint32_t k1, int &acc,
                                          float orw = -1.0f)
{
    const float k2 = qdot(V, V);
    const float inv_k = k2 > 0.0f ? hw_rsq(k2) : 0.0f;
    const float alpha = beta * k2 * inv_k;
    if (!(alpha >= kNNAlphaLo && alpha <= kNNAlphaHi)) {
        acc = -1;
        return heatbath_link(V, beta, site, sweep, word2(mu, TAG_TRIAL, replica), k0, k1);
    }
    const Q Ut{V.w * inv_k, V.x * inv_k, V.y * inv_k, V.z * inv_k};
    const float *row = table + (size_t)nn_table_row(alpha) * kNNRow;
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
    const float4 xa = r4[0], xb = r4[1], xc = r4[2], xd = r4[3];
    const float4 ya = r4[4], yb = r4[5], yc = r4[6], yd = r4[7];
    const U4 w = philox(site, sweep, word2(mu, TAG_LEARN, replica), 0u, k0, k1);
    // current link in the frame of the staple: x_old = (U_old U~)_0
    const float xo = fminf(fmaxf(retr(Uold, Ut), -1.0f), 1.0f);
    const RQBin bo = rq_bin_at(row, rq_bin_index(xa, xb, xc, xd, xo));
    float u = 2.0f * u01(w.a) - 1.0f;
    if (orw >= 0.0f) {  // uniform over the launch
        // g(x_old) in its bin: y_l + H (s xi^2 + d_l xi (1 - xi)) / (s + (d_h + d_l - 2 s) xi (1 - xi))
        const float rw = hw_rcp(bo.W);
        const float s = bo.H * rw, xi = (xo - bo.xl) * rw, om = xi * (1.0f - xi);
        const float yo = bo.yl + bo.H * (s * xi * xi + bo.dl * om) *
                                     hw_rcp(s + (bo.dh + bo.dl - 2.0f * s) * om);
        float v = orw * u - yo;
        v = v >= 1.0f ? v - 2.0f : (v < -1.0f ? v + 2.0f : v);
        u = v;
    }
    const RQBin bn = rq_bin_at(row, rq_bin_index(ya, yb, yc, yd, u));
    // proposal a0' = g^{-1}(u): root xi of qa xi^2 + qb xi + qc = 0 in the bin
    const float sn = bn.H * hw_rcp(bn.W);
    const float dy = u - bn.yl, tt = bn.dh + bn.dl - 2.0f * sn;
    const float qa = bn.H * (sn - bn.dl) + dy * tt;
    const float qb = bn.H * bn.dl - dy * tt;
    const float qc = -sn * dy;
    const float disc = fmaxf(qb * qb - 4.0f * qa * qc, 0.0f);
    const float xin = 2.0f * qc * hw_rcp(-qb - hw_sqrt(disc));
    const float a0n = bn.xl + xin * bn.W;
    const float rwo = hw_rcp(bo.W);
    const float so = bo.H * rwo;
    float nn_, dn2, no_, do2;
    rq_deriv_parts(bn, sn, xin, nn_, dn2);
    rq_deriv_parts(bo, so, (xo - bo.xl) * rwo, no_, do2);
    // ln w(a0') - ln w(x_old) = alpha (a0' - x_old)
    //   + (1/2) ln[(1 - a0'^2) / (1 - x_old^2)] + ln[g'(x_old) / g'(a0')],
    // g'(x_old) / g'(a0') = (no_ dn2) / (nn_ do2).  Both quotients stay well
    // inside the FP32 range; 1 - x_old^2 = 0 gives +inf (accept), 1 - a0'^2
    // = 0 gives -inf (reject), both NaN (reject).
    const float qg = (no_ * dn2) * hw_rcp(nn_ * do2);
    const float qs = (1.0f - a0n) * (1.0f + a0n) * hw_rcp((1.0f - xo) * (1.0f + xo));
    const float dlog2 = alpha * (a0n - xo) * kLog2e + 0.5f * hw_log2(qs) + hw_log2(qg);
    if (hw_log2(u01(w.b)) < dlog2) {
        acc = 1;
        const float r5 = u01(w.c), r6 = u01(w.d);
        const float amag = hw_sqrt((1.0f - a0n) * (1.0f + a0n));
        const float as = amag * 2.0f * hw_sqrt(r5 * (1.0f - r5));
        const Q X{a0n, as * hw_cos_rev(r6), as * hw_sin_rev(r6), amag * (1.0f - 2.0f * r5)};
        return qmul(X, qdag(Ut));
    }
    acc = 0;
    return Uold;
}

// Haar-random element from one Philox block: two Box-Muller pairs, normalised.
__device__ __forceinline__ Q haar_from_block(const U4 &w)
{
    const float u0 = u01(w.a), u1 = u01(w.b), u2 = u01(w.c), u3 = u01(w.d);
    const float r01 = sqrtf(-2.0f * logf(u0)), r23 = sqrtf(-2.0f * logf(u2));
    Q g{r01 * cospif(2.0f * u1), r01 * sinpif(2.0f * u1), r23 * cospif(2.0f * u3),
        r23 * sinpif(2.0f * u3)};
    const float inv = 1.0f / sqrtf(qdot(g, g));
    return Q{g.w * inv, g.x * inv, g.y * inv, g.z * inv};
}

}  // namespace su2dev
