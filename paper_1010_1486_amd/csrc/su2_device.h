// su2_device.h -- device-side building blocks of the SU(2) heat bath (gfx950).
//
// Quaternion algebra for U = a0 + i a.sigma (Sec. 2 of Cardoso & Bicudo,
// "Lattice SU(2) on GPU's"), the Philox4x32-10 counter-based generator
// (Salmon et al., SC'11), the exact a0 sampler, and the even/odd lattice
// indexing of the structure-of-arrays link layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace su2dev {

// ------------------------------------------------------------------ layout
// Links live in 32 planes of V/2 floats: plane (mu, parity, c) holds
// component c of U_mu at every site of that parity, indexed by the half-site
// h = s >> 1 of the canonical site s = x + Nx*(y + Ny*(z + Nz*t)).
struct Geom {
    int32_t nx, ny, nz, nt;
    uint32_t vh;   // V/2
    uint32_t hx;   // Nx/2 (half-sites per x row)
    uint32_t sy;   // half-site stride of y (= Nx/2)
    uint32_t sz;   // half-site stride of z (= Nx*Ny/2)
    uint32_t st;   // half-site stride of t (= Nx*Ny*Nz/2)
};

__device__ __forceinline__ const float *plane(const float *base, uint32_t vh, int mu, int par,
                                              int c)
{
    return base + (size_t)(((mu * 2 + par) * 4 + c)) * vh;
}
__device__ __forceinline__ float *plane(float *base, uint32_t vh, int mu, int par, int c)
{
    return base + (size_t)(((mu * 2 + par) * 4 + c)) * vh;
}

// ------------------------------------------------------------- quaternions
struct Q {
    float w, x, y, z;
};

__device__ __forceinline__ Q qmul(const Q &a, const Q &b)
{
    // (a0 + i a.s)(b0 + i b.s) = (a0 b0 - a.b) + i (a0 b + b0 a - a x b).s
    Q c;
    c.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    c.x = a.w * b.x + b.w * a.x - (a.y * b.z - a.z * b.y);
    c.y = a.w * b.y + b.w * a.y - (a.z * b.x - a.x * b.z);
    c.z = a.w * b.z + b.w * a.z - (a.x * b.y - a.y * b.x);
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

// 32-bit word -> (2*(w>>9)+1) * 2^-24: exact in FP32, never 0 or 1.
__device__ __forceinline__ float u01(uint32_t w)
{
    return (float)(((w >> 9) << 1) | 1u) * 5.9604644775390625e-08f;
}

enum : uint32_t {
    TAG_TRIAL = 0,
    TAG_DIR = 1,
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

// ----------------------------------------------------------------- sampler
// Exact draw of a0 from sqrt(1 - a0^2) exp(alpha a0) on [-1, 1] (Sec. 2),
// returned as delta = 1 - a0.  alpha >= 1: Kennedy-Pendleton (delta is
// Gamma(3/2, alpha) from two logs and a cos^2, accepted with probability
// sqrt(1 - delta/2)).  alpha < 1: a0 = sqrt(r1) cos(2 pi r2) is Haar
// (semicircle) distributed, accepted with probability exp(alpha (a0 - 1)).
// The trial cap is unreachable in practice (acceptance >= 0.41 everywhere);
// on reaching it delta = 0.
constexpr int kTrialCap = 1000;
constexpr float kKPMinAlpha = 1.0f;

__device__ __forceinline__ float sample_delta(float alpha, uint32_t site, uint32_t sweep,
                                              uint32_t w2trial, uint32_t k0, uint32_t k1,
                                              int *ntrials = nullptr)
{
    float delta = 0.0f;
    int t = 0;
    if (alpha >= kKPMinAlpha) {
        const float inv_alpha = 1.0f / alpha;
        for (; t < kTrialCap; ++t) {
            U4 w = philox(site, sweep, w2trial, (uint32_t)t, k0, k1);
            const float r1 = u01(w.a), r2 = u01(w.b), r3 = u01(w.c), r4 = u01(w.d);
            const float c = cospif(2.0f * r2);
            const float d = -(logf(r1) + c * c * logf(r3)) * inv_alpha;
            if (r4 * r4 <= 1.0f - 0.5f * d) {
                delta = d;
                break;
            }
        }
    } else {
        for (; t < kTrialCap; ++t) {
            U4 w = philox(site, sweep, w2trial, (uint32_t)t, k0, k1);
            const float r1 = u01(w.a), r2 = u01(w.b), r3 = u01(w.c);
            const float a0 = sqrtf(r1) * cospif(2.0f * r2);
            if (r3 <= expf(alpha * (a0 - 1.0f))) {
                delta = 1.0f - a0;
                break;
            }
        }
    }
    if (ntrials) *ntrials = t + 1;
    return delta;
}

// X = (1 - delta, |a| n), n uniform on the sphere from (r5, r6) of the
// direction block; |a| = sqrt(delta (2 - delta)) avoids cancellation near a0 = 1.
__device__ __forceinline__ Q element_from_delta(float delta, float r5, float r6)
{
    const float amag = sqrtf(delta * (2.0f - delta));
    const float cth = 1.0f - 2.0f * r5;
    const float sth = 2.0f * sqrtf(r5 * (1.0f - r5));
    const float cph = cospif(2.0f * r6), sph = sinpif(2.0f * r6);
    return Q{1.0f - delta, amag * sth * cph, amag * sth * sph, amag * cth};
}

// Heat-bath update of one link from its staple sum V: U' = X U~^+, U~ = V/k.
__device__ __forceinline__ Q heatbath_link(const Q &V, float beta, uint32_t site, uint32_t sweep,
                                           uint32_t mu, uint32_t replica, uint32_t k0,
                                           uint32_t k1)
{
    const float k2 = qdot(V, V);
    const float k = sqrtf(k2);
    const float alpha = beta * k;
    const float delta = sample_delta(alpha, site, sweep, word2(mu, TAG_TRIAL, replica), k0, k1);
    const U4 wd = philox(site, sweep, word2(mu, TAG_DIR, replica), 0u, k0, k1);
    const Q X = element_from_delta(delta, u01(wd.a), u01(wd.b));
    Q Ut = (k2 > 0.0f) ? Q{V.w / k, V.x / k, V.y / k, V.z / k} : Q{1.0f, 0.0f, 0.0f, 0.0f};
    return qmul(X, qdag(Ut));
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
