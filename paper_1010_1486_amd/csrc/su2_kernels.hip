// su2_kernels.hip -- gfx950 kernels of the SU(2) checkerboard heat bath.
//
// Cardoso & Bicudo, "Lattice SU(2) on GPU's" (LAT2010):
//   Sec. 2   six-staple sum V, k = sqrt(det V), a0 ~ sqrt(1-a0^2) exp(beta k a0),
//            U' = X U~^{-1}
//   Sec. 4   kernels: cold/hot start, heat bath per (direction, parity),
//            plaquette, Polyakov loop, sum over the lattice
// The pass kernel streams the structure-of-arrays planes of one (mu, parity)
// class.  Plaquette and Polyakov sums are FP64 within a workgroup (wave
// shuffles, then LDS) and 64-bit fixed point across workgroups, so every sum
// is independent of scheduling order.
#include "su2_internal.h"
#include "su2_kcommon.h"

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

// One (mu, parity) class of the link field: an array of V/2 quaternions
// (16-byte float4, components a0..a3) at a uniform byte address in the global
// address space, so that a load is one 16-byte access with a scalar base and
// a 32-bit vector offset (V/2 < 2^28 keeps h * 16 in 32 bits).
typedef __attribute__((address_space(1))) const char gchar;
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) float gfloat_w;
struct __attribute__((aligned(16))) F4 {
    float x, y, z, w;
};
typedef __attribute__((address_space(1))) const F4 gf4;
typedef __attribute__((address_space(1))) F4 gf4_w;

struct Arr {
    gchar *base;
};

__device__ __forceinline__ Arr arr(const float *links, uint32_t vh, int mu, int par)
{
    return Arr{(gchar *)links + (size_t)(mu * 2 + par) * vh * 16u};
}

__device__ __forceinline__ Q ld(const Arr &a, uint32_t h)
{
    gf4 *p = (gf4 *)(a.base + h * 16u);
    return Q{p->x, p->y, p->z, p->w};
}

__device__ __forceinline__ void st(float *links, uint32_t vh, int mu, int par, uint32_t h,
                                   const Q &q)
{
    gf4_w *p = (gf4_w *)links + (size_t)(mu * 2 + par) * vh + h;
    p->x = q.w;
    p->y = q.x;
    p->z = q.y;
    p->w = q.z;
}

// Store with the nontemporal hint: the class a pass writes is read by no
// other site of that pass, so its lines need not displace the neighbour
// classes the pass re-reads from L2.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4f gv4f;
__device__ __forceinline__ void st_nt(float *links, uint32_t vh, int mu, int par, uint32_t h,
                                      const Q &q)
{
    gv4f *p = (gv4f *)links + (size_t)(mu * 2 + par) * vh + h;
    const v4f v = {q.w, q.x, q.y, q.z};
    __builtin_nontemporal_store(v, p);
}

__device__ __forceinline__ Q ldq(const float *links, uint32_t vh, int mu, int par, uint32_t h)
{
    gf4 *p = (gf4 *)links + (size_t)(mu * 2 + par) * vh + h;
    return Q{p->x, p->y, p->z, p->w};
}

// ------------------------------------------------------------------- init
// grid (blocks over V/2, 8 = mu * 2 + parity, replica)
__global__ void init_kernel(const Rep *__restrict__ reps, const int *__restrict__ starts,
                            uint32_t k0, uint32_t k1)
{
    const Rep &R = reps[blockIdx.z];
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= R.g.vh) return;
    const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
    Q q{1.0f, 0.0f, 0.0f, 0.0f};
    if (starts[blockIdx.z]) {
        int x, y, z, t;
        decode(R.g, h, par, x, y, z, t);
        const uint32_t s = 2u * h + (uint32_t)(x & 1);
        q = haar_from_block(philox(s, 0u, word2((uint32_t)mu, TAG_HOT, R.replica), 0u, k0, k1));
    }
    st(R.links, R.g.vh, mu, par, h, q);
}

// ------------------------------------------------------------------- pass
// The two staples of the (mu, nu) plane at s from the six links they use:
// forward U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+ = A B^+ C^+, backward
// U_nu(s+mu-nu)^+ U_mu(s-nu)^+ U_nu(s-nu) = (E D)^+ F.
__device__ __forceinline__ Q staple_pair(const Q &A, const Q &B, const Q &C, const Q &D,
                                         const Q &E, const Q &F)
{
    return qadd(qmul(qmul(A, qdag(B)), qdag(C)), qmul(qdag(qmul(E, D)), F));
}

// Update of the link U_MU at half-site index gid (pass order) of parity par:
// the six-staple sum V (Sec. 2), then the exact heat bath or, with LEARNED,
// the learned-proposal Metropolis step; the new link is stored.  With
// MEASURE, meas = (1/2)Tr(U'_MU V_nu) summed over nu < MU.  acc: as
// learned_link (-1 for the heat bath).  With NORM the new link is
// reunitarised (unit_q) before it is stored and measured.  GROUP: issue the
// 18 neighbour loads together (below); the update is the same either way.
// The learned update keeps the default schedule: its spline evaluation needs
// the registers (grouped, the 64-replica learned sweep took 368 instead of
// 354 us, the plain one 320 either way).
template <int MU, bool MEASURE, bool LEARNED, bool OR = false, bool NORM = false,
          bool GROUP = !LEARNED>
__device__ __forceinline__ void update_at(const Rep &R, const PassSite &s, int par,
                                          uint32_t sweep, uint32_t k0, uint32_t k1,
                                          const float *ltab, float &meas, int &acc)
{
    const Geom &g = R.g;
    const int opp = par ^ 1;
    const float *links = R.links;
    const Deltas d = neighbour_deltas(g, s);
    const uint32_t h = s.h;
    const Arr Umu_o = arr(links, g.vh, MU, opp);
    Q V{0.0f, 0.0f, 0.0f, 0.0f};
    Q Vlow{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (GROUP) {
        // All 18 neighbour loads are issued before any staple product (the
        // scheduling barrier keeps them together): each wave has all its
        // gathers in flight at once instead of the six or seven of the
        // register-frugal schedule below.  The pass kernel then needs 82
        // instead of 58 VGPRs (5 instead of 8 waves per SIMD) and is 3-4 %
        // faster at 48^4; the work-queue kernel, whose other stages already
        // need 107-117 VGPRs, and the learned update keep the schedule below.
        Q Ld[3][6];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int nu = j + (j >= MU ? 1 : 0);  // the three nu != MU, in increasing order
            const Arr Unu_p = arr(links, g.vh, nu, par);
            const Arr Unu_o = arr(links, g.vh, nu, opp);
            Ld[j][0] = ld(Unu_o, h + d.p[MU]);
            Ld[j][1] = ld(Umu_o, h + d.p[nu]);
            Ld[j][2] = ld(Unu_p, h);
            Ld[j][3] = ld(Unu_p, h + d.p[MU] + d.m[nu]);
            Ld[j][4] = ld(Umu_o, h + d.m[nu]);
            Ld[j][5] = ld(Unu_o, h + d.m[nu]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int nu = j + (j >= MU ? 1 : 0);
            const Q st = staple_pair(Ld[j][0], Ld[j][1], Ld[j][2], Ld[j][3], Ld[j][4], Ld[j][5]);
            V = qadd(V, st);
            if (MEASURE && nu < MU) Vlow = qadd(Vlow, st);
        }
    } else {
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == MU) continue;
            const Arr Unu_p = arr(links, g.vh, nu, par);
            const Arr Unu_o = arr(links, g.vh, nu, opp);
            const Q st = staple_pair(ld(Unu_o, h + d.p[MU]), ld(Umu_o, h + d.p[nu]), ld(Unu_p, h),
                                     ld(Unu_p, h + d.p[MU] + d.m[nu]), ld(Umu_o, h + d.m[nu]),
                                     ld(Unu_o, h + d.m[nu]));
            V = qadd(V, st);
            if (MEASURE && nu < MU) Vlow = qadd(Vlow, st);
        }
    }
    const uint32_t site = 2u * h + (uint32_t)(s.x & 1);
    Q Un;
    if (OR) {
        Un = overrelax_link(V, ld(arr(links, g.vh, MU, par), h));
    } else if (LEARNED) {
        const Q Uold = ld(arr(links, g.vh, MU, par), h);
        Un = learned_link(V, Uold, ltab, R.beta, site, sweep, (uint32_t)MU, R.replica, k0, k1,
                          acc, R.orw);
    } else {
        Un = heatbath_link(V, R.beta, site, sweep, word2((uint32_t)MU, TAG_TRIAL, R.replica), k0,
                           k1);
    }
    if (NORM) Un = unit_q(Un);
    st_nt(R.links, g.vh, MU, par, h, Un);
    if (MEASURE) meas = retr(Un, Vlow);
}

template <int MU, bool MEASURE, bool LEARNED, bool OR = false, bool NORM = false,
          bool GROUP = !LEARNED>
__device__ __forceinline__ void update_site(const Rep &R, uint32_t gid, int par, uint32_t sweep,
                                            uint32_t k0, uint32_t k1, const float *ltab,
                                            float &meas, int &acc)
{
    update_at<MU, MEASURE, LEARNED, OR, NORM, GROUP>(R, pass_site(R.g, gid, par), par, sweep, k0,
                                                     k1, ltab, meas, acc);
}

// Fill the LDS copy of the spline table (4 floats of padding first, like the
// device copy); every thread of the workgroup takes part.
__device__ __forceinline__ const float *load_table_lds(float4 *stab4, const float *table)
{
    const float4 *t4 = reinterpret_cast<const float4 *>(table);
    for (int i = threadIdx.x; i < kNNRows * kNNRow / 4; i += blockDim.x) stab4[1 + i] = t4[i];
    if (threadIdx.x == 0) stab4[0] = float4{0.0f, 0.0f, 0.0f, 0.0f};
    __syncthreads();
    return reinterpret_cast<const float *>(stab4) + 4;
}

// One heat-bath pass over the sites of parity `par` in direction MU, for
// every replica of the ensemble.  Workgroup ids b in [0, total) are mapped
// to replicas by bmap (each replica's range starts at a multiple of 8, so
// b mod 8 is still the XCD), or, XCD-affine, to (replica, block) by amap so
// that all blocks of a replica run on one XCD; with a capped grid (a multiple
// of 8) the workgroups loop over b (persistent).  With MEASURE, (1/2)Tr(U'_mu(s) V_nu(s)) summed over nu < mu
// is accumulated: over the odd passes of mu = 1, 2, 3 this is every
// plaquette of the end-of-sweep configuration exactly once.  With NORM every
// stored link is reunitarised first (the last pass stage of a
// reunitarisation sweep when the reunitarisation is fused into the passes).
template <int MU, bool MEASURE, bool LEARNED, bool OR = false, bool NORM = false>
__global__ __launch_bounds__(256) void pass_kernel(const Rep *__restrict__ reps,
                                                   const uint32_t *__restrict__ bmap,
                                                   const uint2 *__restrict__ amap,
                                                   uint32_t total, int par, uint32_t k0,
                                                   uint32_t k1, int remap, int reverse,
                                                   const float *__restrict__ table)
{
    // LEARNED: the spline table in LDS (filled once per workgroup)
    __shared__ float4 stab4[LEARNED ? 1 + kNNRows * kNNRow / 4 : 1];
    const float *ltab = LEARNED ? load_table_lds(stab4, table) : nullptr;
    for (uint32_t b = blockIdx.x; b < total; b += gridDim.x) {
        uint32_t r, local;
        if (amap) {
            const uint2 a = amap[b];
            if (a.x == 0xFFFFFFFFu) continue;  // padding workgroup (uniform)
            r = a.x;
            local = a.y;
        } else {
            r = bmap ? bmap[b] : 0u;
            local = b - reps[r].first_block;
        }
        const Rep &R = reps[r];
        if (local >= R.nblocks) continue;  // padding workgroup (uniform)
        const Geom &g = R.g;
        // the blocks of an XCD-affine replica run in order on one XCD
        const uint32_t blk = amap ? (reverse ? R.nblocks - 1u - local : local)
                                  : logical_block(local, R.nblocks, remap, reverse);
        const uint32_t gid = blk * blockDim.x + threadIdx.x;
        float meas = 0.0f;
        int acc = -1;
        if (gid < g.vh) {
            // uniform: a scalar load through the constant address space
            const uint32_t sweep =
                *(const __attribute__((address_space(4))) uint32_t *)&R.cnt->sweep;
            update_site<MU, MEASURE, LEARNED, OR, NORM>(R, gid, par, sweep, k0, k1, ltab, meas,
                                                        acc);
        }
        if (MEASURE) block_accumulate((double)meas, R.acc, ACC_PLAQ, b);
        if (LEARNED) {
            // per-wave counts (ballot) added by lane 0 of each wave
            const unsigned long long mp = __ballot(acc >= 0);
            const unsigned long long ma = __ballot(acc == 1);
            if ((threadIdx.x & 63) == 0) {
                const uint32_t wb = b * (blockDim.x >> 6) + (threadIdx.x >> 6);
                if (mp) atomicAdd(bucket(R.acc, ACC_PROPOSED, wb), (unsigned long long)__popcll(mp));
                if (ma) atomicAdd(bucket(R.acc, ACC_ACCEPTED, wb), (unsigned long long)__popcll(ma));
            }
        }
    }
}

// ------------------------------------------------------- streaming floor
// The byte pattern of a (mu, parity) pass without its stencil: the seven
// plane groups a pass reads (U_nu at both parities for nu != mu, U_mu at the
// opposite parity), each at the thread's own half-site, and one quaternion
// per half-site written to `out` (V/2 float4).  Its duration is the
// bandwidth floor of the pass's traffic; no link is touched.
__global__ __launch_bounds__(256) void stream_kernel(const Rep *__restrict__ reps, int mu,
                                                     int par, float *__restrict__ out)
{
    const Rep &R = reps[0];
    const uint32_t vh = R.g.vh;
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    const int opp = par ^ 1;
    Q a = ld(arr(R.links, vh, mu, opp), h);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        a = qadd(a, ld(arr(R.links, vh, nu, par), h));
        a = qadd(a, ld(arr(R.links, vh, nu, opp), h));
    }
    // one 16-byte nontemporal store, as the pass stores its updated link
    st_nt(out, vh, 0, 0, h, a);
}

// -------------------------------------------------------------- plaquette
// Sum of (1/2)Tr U_mu(s) U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+ over mu < nu at
// site i of [0, V) in pass order (parity 0 first), as (1/2)Tr(P Q^+) with
// P = U_mu(s) U_nu(s+mu), Q = U_nu(s) U_mu(s+nu).
__device__ __forceinline__ float site_plaquettes(const Rep &R, uint32_t i)
{
    const Geom &g = R.g;
    const int par = i >= g.vh ? 1 : 0;
    const int opp = par ^ 1;
    const float *links = R.links;
    const PassSite s = pass_site(g, par ? i - g.vh : i, par);
    const Deltas d = neighbour_deltas(g, s);
    Q U[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) U[mu] = ld(arr(links, g.vh, mu, par), s.h);
    float sum = 0.0f;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int nu = mu + 1; nu < 4; ++nu) {
            const Q P = qmul(U[mu], ld(arr(links, g.vh, nu, opp), s.h + d.p[mu]));
            const Q Qq = qmul(U[nu], ld(arr(links, g.vh, mu, opp), s.h + d.p[nu]));
            sum += retr_adj(P, Qq);
        }
    return sum;
}

// Sum of the six plaquettes rooted at a site with own links S and +a
// neighbours F[a][b] = U_b(s + a) (F[a][a] unused), in the order of
// site_plaquettes.
__device__ __forceinline__ float plaquettes_from(const Q S[4], const Q F[4][4])
{
    float sum = 0.0f;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int nu = mu + 1; nu < 4; ++nu)
            sum += retr_adj(qmul(S[mu], F[mu][nu]), qmul(S[nu], F[nu][mu]));
    return sum;
}

// grid (multiple of 8 workgroups, 1, replica), blockDim.x threads; T divides
// every replica's Nt.  A unit is a tile of blockDim.x consecutive half-sites
// of an (x, y) plane at one z over T consecutive t; units are numbered z
// fastest, then t-chunk, then tile (the +z unit is the next one and the +t
// chunk nz units on), each XCD walks one contiguous stretch of them, and
// workgroups loop while units remain.  A thread takes both sites of
// its half-site (x even and x odd) on every plane of its chunk: the links of
// plane t + 1, loaded once, serve as the +t neighbours at t and as the own
// links at t + 1, the odd site is the even site's +x neighbour, and only the
// odd site's +x and both sites' +y and +z neighbours are further loads (the
// z + 1 unit is the next unit of the same XCD, so those come from its L2).
// Per half-site and plane: 23 loads, plus the 8 own links of a chunk's first
// plane (reading the 4 own and 12 neighbour links of both sites
// independently takes 28, 6 of them from plane t + 1).
__global__ __launch_bounds__(256) void plaquette_march_kernel(const Rep *__restrict__ reps,
                                                              uint32_t T)
{
    const Rep &R = reps[blockIdx.z];
    const Geom &g = R.g;
    const float *links = R.links;
    const uint32_t B = blockDim.x;
    const uint32_t ntile = (g.P + B - 1u) / B;
    const uint32_t nchunk = (uint32_t)g.nt / T;
    const uint32_t nunits = ntile * (uint32_t)g.nz * nchunk;
    double acc = 0.0;
    for (uint32_t b = blockIdx.x; b < nunits; b += gridDim.x) {
        const uint32_t u = logical_block(b, nunits, 1, 0);
        const uint32_t z = u % (uint32_t)g.nz, rest = u / (uint32_t)g.nz;
        const uint32_t tc = rest % nchunk, tile = rest / nchunk;
        const uint32_t r = tile * B + threadIdx.x;
        if (r >= g.P) continue;
        const uint32_t y = fdiv(r, g.m_hx, g.s_hx), xh = r - y * g.hx;
        const uint32_t dx = xh == g.hx - 1u ? 1u - g.hx : 1u;
        const uint32_t dy = y == (uint32_t)g.ny - 1u ? 0u - g.wy : g.hx;
        const uint32_t dz = z == (uint32_t)g.nz - 1u ? 0u - g.wz : g.P;
        uint32_t t = tc * T;
        uint32_t h = r + g.P * z + g.PZ * t;
        int pe = (int)((y + z + t) & 1u);  // parity of the even-x site
        Q S0[4], S1[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            S0[mu] = ld(arr(links, g.vh, mu, pe), h);
            S1[mu] = ld(arr(links, g.vh, mu, pe ^ 1), h);
        }
        for (uint32_t j = 0; j < T; ++j, ++t) {
            const uint32_t dt = t == (uint32_t)g.nt - 1u ? 0u - g.wt : g.PZ;
            Q F0[4][4], F1[4][4];
#pragma unroll
            for (int nu = 0; nu < 4; ++nu) {
                // +t: the sites of plane t + 1 (x even there has parity pe ^ 1)
                F0[3][nu] = ld(arr(links, g.vh, nu, pe ^ 1), h + dt);
                F1[3][nu] = ld(arr(links, g.vh, nu, pe), h + dt);
                // +x: the odd site for the even one, the next half-site's even site
                F0[0][nu] = S1[nu];
                if (nu != 0) F1[0][nu] = ld(arr(links, g.vh, nu, pe), h + dx);
                if (nu != 1) {
                    F0[1][nu] = ld(arr(links, g.vh, nu, pe ^ 1), h + dy);
                    F1[1][nu] = ld(arr(links, g.vh, nu, pe), h + dy);
                }
                if (nu != 2) {
                    F0[2][nu] = ld(arr(links, g.vh, nu, pe ^ 1), h + dz);
                    F1[2][nu] = ld(arr(links, g.vh, nu, pe), h + dz);
                }
            }
            // the plane's 23 loads issued as one group ahead of the products
            // (as in the pass): 93 -> 82 us per 48^4 plaquette, 140 VGPRs
            __builtin_amdgcn_sched_barrier(0);
            acc += (double)plaquettes_from(S0, F0) + (double)plaquettes_from(S1, F1);
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                S0[mu] = F0[3][mu];
                S1[mu] = F1[3][mu];
            }
            h += dt;
            pe ^= 1;
        }
    }
    block_accumulate(acc, R.acc, ACC_PLAQ, blockIdx.x);
}

// --------------------------------------------------------------- Polyakov
// grid (spatial sites / 64, 1, replica).  L(x) = (1/2)Tr prod_t U_3(x, t),
// t = 0 leftmost.  A workgroup holds 64 spatial sites and S waves; wave w
// multiplies the w-th of S contiguous t-segments for its 64 sites
// (consecutive lanes read consecutive sites), and wave 0 multiplies the S
// segment products in t order from LDS.
template <int S>
__global__ __launch_bounds__(512) void polyakov_kernel(const Rep *__restrict__ reps)
{
    __shared__ Q seg_prod[S][64];
    const Rep &R = reps[blockIdx.z];
    const Geom &g = R.g;
    const uint32_t ns3 = (uint32_t)g.nx * g.ny * g.nz;
    if (blockIdx.x * 64u >= ns3) return;  // uniform: whole workgroup
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t xs = blockIdx.x * 64u + (uint32_t)lane;
    Q P{1.0f, 0.0f, 0.0f, 0.0f};
    if (xs < ns3) {
        const int x = (int)(xs % (uint32_t)g.nx);
        const uint32_t r = xs / (uint32_t)g.nx;
        const int y = (int)(r % (uint32_t)g.ny), z = (int)(r / (uint32_t)g.ny);
        const int len = g.nt / S;
        const int t0 = w * len;
        const int pbase = (x + y + z) & 1;
        const uint32_t h0 = xs >> 1;
        for (int t = t0; t < t0 + len; ++t) {
            // site xs + ns3 t has half-site (xs >> 1) + t ns3/2 because ns3 is even
            const Q U = ldq(R.links, g.vh, 3, (pbase + t) & 1, h0 + (uint32_t)t * (ns3 >> 1));
            P = qmul(P, U);
        }
    }
    seg_prod[w][lane] = P;
    __syncthreads();
    double acc = 0.0;
    if (w == 0 && xs < ns3) {
        Q T = seg_prod[0][lane];
#pragma unroll
        for (int k = 1; k < S; ++k) T = qmul(T, seg_prod[k][lane]);
        acc = (double)T.w;
    }
    block_accumulate(acc, R.acc, ACC_POLY, blockIdx.x);
}

// ---------------------------------------------------------- bookkeeping
// All launched with grid (1, 1, replica) and kBuckets threads.
__global__ __launch_bounds__(kBuckets) void take_kernel(const Rep *__restrict__ reps, int flags)
{
    const Rep &R = reps[blockIdx.z];
    const unsigned long long tp = (flags & 1) ? take_total(R.acc, ACC_PLAQ) : 0ull;
    const unsigned long long tl = (flags & 2) ? take_total(R.acc, ACC_POLY) : 0ull;
    if (threadIdx.x == 0) {
        const Geom &g = R.g;
        if (flags & 1) R.results[R_PLAQ] = from_fixed(tp) / (12.0 * (double)g.vh);
        if (flags & 2) {
            const double l = from_fixed(tl) / ((double)g.nx * g.ny * g.nz);
            R.results[R_POLY_SIGNED] = l;
            R.results[R_POLY_ABS] = fabs(l);
        }
    }
}

__global__ __launch_bounds__(kBuckets) void sweep_end_kernel(const Rep *__restrict__ reps,
                                                             int nrep, int flags,
                                                             double *__restrict__ hist)
{
    const Rep &R = reps[blockIdx.z];
    const unsigned long long tp = take_total(R.acc, ACC_PLAQ);
    const unsigned long long tl = take_total(R.acc, ACC_POLY);
    if (threadIdx.x == 0) {
        Counters *c = R.cnt;
        const Geom &g = R.g;
        if ((flags & 4) && hist) {
            uint32_t *rc = row_counter(c, (flags & 8) != 0);
            const uint32_t m = *rc;
            const double p = (flags & 1) ? from_fixed(tp) / (12.0 * (double)g.vh) : 0.0;
            const double l = (flags & 2) ? from_fixed(tl) / ((double)g.nx * g.ny * g.nz) : 0.0;
            double *row = hist + 3 * ((size_t)m * nrep + blockIdx.z);
            row[0] = p;
            row[1] = l;
            row[2] = fabs(l);
            *rc = m + 1;
        }
        c->sweep = c->sweep + 1;
    }
}

__global__ __launch_bounds__(kBuckets) void counts_kernel(const Rep *__restrict__ reps,
                                                          int reset)
{
    __shared__ unsigned long long part[2][kBuckets / 64];
    const Rep &R = reps[blockIdx.z];
    for (int a = 0; a < 2; ++a) {
        unsigned long long *p = bucket(R.acc, ACC_PROPOSED + a, threadIdx.x);
        unsigned long long v = *p;
        if (reset) *p = 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) part[a][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *out = reinterpret_cast<unsigned long long *>(R.results + R_COUNTS);
        for (int a = 0; a < 2; ++a) {
            unsigned long long t = 0ull;
            for (int i = 0; i < kBuckets / 64; ++i) t += part[a][i];
            out[a] = t;
        }
    }
}

__global__ __launch_bounds__(kBuckets) void set_counter_kernel(const Rep *__restrict__ reps,
                                                               uint32_t sweep, uint32_t meas,
                                                               int which, QueueState *qs)
{
    const Rep &R = reps[blockIdx.z];
    if ((which & 16) && threadIdx.x == 0) {
        R.cnt->done = 0u;
        if (qs && blockIdx.z == 0) {
            for (int k = 0; k < kMaxQueues; ++k) qs->ticket[k][0] = 0u;
            qs->error = 0u;
        }
    }
    if (which & 4)
        for (int a = 0; a < kNumAcc; ++a) *bucket(R.acc, a, threadIdx.x) = 0ull;
    else if (which & 8)
        for (int a = ACC_PROPOSED; a < kNumAcc; ++a) *bucket(R.acc, a, threadIdx.x) = 0ull;
    if (threadIdx.x == 0) {
        if (which & 1) R.cnt->sweep = sweep;
        if (which & 2) R.cnt->meas_idx = meas;
        if (which & 32) R.cnt->graph_row = meas;
    }
}

// --------------------------------------------------------------- reunit
// U <- U / |U| with the norm in FP64 (unit_q).
__device__ __forceinline__ void reunit_link(const Rep &R, int mu, int par, uint32_t h)
{
    st(R.links, R.g.vh, mu, par, h, unit_q(ldq(R.links, R.g.vh, mu, par, h)));
}

// grid (blocks over V/2, 8, replica)

__global__ __launch_bounds__(256) void reunit_kernel(const Rep *__restrict__ reps)
{
    const Rep &R = reps[blockIdx.z];
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= R.g.vh) return;
    reunit_link(R, blockIdx.y >> 1, blockIdx.y & 1, h);
}

// ----------------------------------------------------------- small lattices
// Whole sweeps of small lattices in one launch: workgroup r runs replica r
// alone -- the 8 passes of a sweep separated by workgroup barriers, the
// plaquette (fused into the odd passes of mu = 1, 2, 3, or recomputed after
// a reunitarisation), the Polyakov loop, the reunitarisation and the history
// row -- for ns sweeps.  Link updates are the pass kernel's, bit for bit.
// Each site's plaquette and Polyakov value is added in 64-bit fixed point,
// so the sums do not depend on the workgroup size.
template <int MU, bool LEARNED>
__device__ __forceinline__ void small_pass(const Rep &R, int par, bool measure, uint32_t sweep,
                                           uint32_t k0, uint32_t k1, const float *ltab,
                                           unsigned long long &psum, unsigned long long &np,
                                           unsigned long long &na)
{
    for (uint32_t gid = threadIdx.x; gid < R.g.vh; gid += blockDim.x) {
        float m = 0.0f;
        int a = -1;
        if (measure) {
            update_site<MU, true, LEARNED>(R, gid, par, sweep, k0, k1, ltab, m, a);
            psum += to_fixed((double)m);
        } else {
            update_site<MU, false, LEARNED>(R, gid, par, sweep, k0, k1, ltab, m, a);
        }
        np += a >= 0 ? 1ull : 0ull;
        na += a == 1 ? 1ull : 0ull;
    }
    __syncthreads();
}

// Exact sum over the workgroup of 64-bit integers (valid in thread 0).
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v)
{
    __shared__ unsigned long long wpart[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) wpart[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0ull;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) t += wpart[i];
    __syncthreads();
    return t;
}

// flags: 1 plaquette, 2 Polyakov loop, 4 history rows, 8 rows from the
// graph's row counter.
template <bool LEARNED>
__global__ __launch_bounds__(1024) void small_sweeps_kernel(const Rep *__restrict__ reps, int nrep,
                                                            int ns, uint32_t k0, uint32_t k1,
                                                            int reunit_every, int flags,
                                                            double *__restrict__ hist,
                                                            const float *__restrict__ table)
{
    __shared__ float4 stab4[LEARNED ? 1 + kNNRows * kNNRow / 4 : 1];
    const float *ltab = LEARNED ? load_table_lds(stab4, table) : nullptr;
    const Rep &R = reps[blockIdx.x];
    const Geom &g = R.g;
    const uint32_t ns3 = (uint32_t)g.nx * g.ny * g.nz;
    uint32_t sweep = R.cnt->sweep;  // written back by thread 0 at the end
    uint32_t *const row_ctr = row_counter(R.cnt, (flags & 8) != 0);
    uint32_t midx = *row_ctr;
    unsigned long long np = 0ull, na = 0ull;
    const bool want_p = (flags & 1) != 0, want_l = (flags & 2) != 0;
    const bool rows = (flags & 4) != 0 && hist != nullptr;
    for (int i = 0; i < ns; ++i, ++sweep) {
        const bool reunit = reunit_every > 0 && ((sweep + 1u) % (uint32_t)reunit_every) == 0u;
        const bool fused = want_p && !reunit;
        unsigned long long psum = 0ull, lsum = 0ull;
        small_pass<0, LEARNED>(R, 0, false, sweep, k0, k1, ltab, psum, np, na);
        small_pass<0, LEARNED>(R, 1, false, sweep, k0, k1, ltab, psum, np, na);
        small_pass<1, LEARNED>(R, 0, false, sweep, k0, k1, ltab, psum, np, na);
        small_pass<1, LEARNED>(R, 1, fused, sweep, k0, k1, ltab, psum, np, na);
        small_pass<2, LEARNED>(R, 0, false, sweep, k0, k1, ltab, psum, np, na);
        small_pass<2, LEARNED>(R, 1, fused, sweep, k0, k1, ltab, psum, np, na);
        small_pass<3, LEARNED>(R, 0, false, sweep, k0, k1, ltab, psum, np, na);
        small_pass<3, LEARNED>(R, 1, fused, sweep, k0, k1, ltab, psum, np, na);
        if (reunit) {
            for (uint32_t j = threadIdx.x; j < 8u * g.vh; j += blockDim.x) {
                const uint32_t grp = j / g.vh;
                reunit_link(R, (int)(grp >> 1), (int)(grp & 1u), j - grp * g.vh);
            }
            __syncthreads();
            if (want_p)
                for (uint32_t j = threadIdx.x; j < 2u * g.vh; j += blockDim.x)
                    psum += to_fixed((double)site_plaquettes(R, j));
        }
        if (want_l) {
            // L(x) = (1/2)Tr prod_t U_3(x, t), t = 0 leftmost
            for (uint32_t xs = threadIdx.x; xs < ns3; xs += blockDim.x) {
                const uint32_t x = xs % (uint32_t)g.nx, r = xs / (uint32_t)g.nx;
                const uint32_t y = r % (uint32_t)g.ny, z = r / (uint32_t)g.ny;
                const uint32_t pbase = (x + y + z) & 1u;
                Q P{1.0f, 0.0f, 0.0f, 0.0f};
                for (int t = 0; t < g.nt; ++t)
                    P = qmul(P, ldq(R.links, g.vh, 3, (int)((pbase + (uint32_t)t) & 1u),
                                    (xs >> 1) + (uint32_t)t * (ns3 >> 1)));
                lsum += to_fixed((double)P.w);
            }
        }
        const unsigned long long tp = block_sum_u64(psum);
        const unsigned long long tl = block_sum_u64(lsum);
        if (rows) {
            if (threadIdx.x == 0) {
                const double p = want_p ? from_fixed(tp) / (12.0 * (double)g.vh) : 0.0;
                const double l = want_l ? from_fixed(tl) / (double)ns3 : 0.0;
                double *row = hist + 3 * ((size_t)midx * nrep + blockIdx.x);
                row[0] = p;
                row[1] = l;
                row[2] = fabs(l);
            }
            ++midx;
        }
    }
    if (LEARNED) {
        // per-wave totals added by lane 0 of each wave
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            np += __shfl_down(np, off, 64);
            na += __shfl_down(na, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            const uint32_t wb = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
            if (np) atomicAdd(bucket(R.acc, ACC_PROPOSED, wb), np);
            if (na) atomicAdd(bucket(R.acc, ACC_ACCEPTED, wb), na);
        }
    }
    __syncthreads();  // every thread has read the counters before they change
    if (threadIdx.x == 0) {
        R.cnt->sweep = sweep;
        *row_ctr = midx;
    }
}

// ---------------------------------------------------------- Wilson loops
// W(R, T) of the rectangle R along mu, T along nu at site s, for the 12
// ordered planes: (1/2)Tr[A_R C_T (B_T D_T)^+] = qdot(A_R C_T, B_T D_T) with
// A_R = L_mu(s, R), C_T = L_nu(s + R mu, T), B_T = L_nu(s, T),
// D_T = L_mu(s + T nu, R), L_mu(x, n) = U_mu(x) ... U_mu(x + (n - 1) mu).
// The lines are extended one link at a time (R outer, T inner), so a plane
// costs R + T + 2RT link loads for all R, T <= N.  One thread per site (both
// parities) and plane; per-site values FP32, the sum over a workgroup FP64
// into part[slot * N * N + (R - 1) N + (T - 1)], slot = plane * blocks + block.

// Site-index offset of k steps along a direction from coordinate c (extent n,
// canonical stride st), periodic for any k >= 0.
__device__ __forceinline__ int32_t step_off(int c, int k, int n, int32_t st)
{
    return ((c + k) % n - c) * st;
}

__device__ __forceinline__ int pick4(int a, int v0, int v1, int v2, int v3)
{
    return a == 0 ? v0 : a == 1 ? v1 : a == 2 ? v2 : v3;
}

// grid (blocks over the V sites, 12 ordered planes): one thread per site and
// plane, partial sums per (plane, workgroup).
template <int N>
__global__ __launch_bounds__(256) void wilson_kernel(const Rep *__restrict__ reps, int rmax,
                                                     int tmax, double *__restrict__ part)
{
    const Rep &R = reps[0];
    const Geom &g = R.g;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int o = (int)blockIdx.y, mu = o / 3, nu = o % 3 < mu ? o % 3 : o % 3 + 1;
    float w[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int t = 0; t < N; ++t) w[r][t] = 0.0f;
    if (i < 2u * g.vh) {
        const int par = i >= g.vh ? 1 : 0;
        int c0[4];
        decode(g, par ? i - g.vh : i, par, c0[0], c0[1], c0[2], c0[3]);
        const int32_t sy = g.nx, sz = g.nx * g.ny, stt = g.nx * g.ny * g.nz;
        // canonical index of the site; the link k steps along mu and l along nu
        // from it lies at s0 + oa[k] + ob[l] and has parity par + k + l
        const uint32_t s0 = (uint32_t)c0[0] + (uint32_t)sy * (uint32_t)c0[1] +
                            (uint32_t)sz * (uint32_t)c0[2] + (uint32_t)stt * (uint32_t)c0[3];
        const int ca = pick4(mu, c0[0], c0[1], c0[2], c0[3]);
        const int na = pick4(mu, g.nx, g.ny, g.nz, g.nt);
        const int32_t sa = pick4(mu, 1, sy, sz, stt);
        const int cb = pick4(nu, c0[0], c0[1], c0[2], c0[3]);
        const int nb = pick4(nu, g.nx, g.ny, g.nz, g.nt);
        const int32_t sb = pick4(nu, 1, sy, sz, stt);
        int32_t oa[N + 1], ob[N + 1];
#pragma unroll
        for (int k = 0; k <= N; ++k) {
            oa[k] = step_off(ca, k, na, sa);
            ob[k] = step_off(cb, k, nb, sb);
        }
        // the two parities of each direction's class
        const Arr Amu[2] = {arr(R.links, g.vh, mu, par), arr(R.links, g.vh, mu, par ^ 1)};
        const Arr Anu[2] = {arr(R.links, g.vh, nu, par), arr(R.links, g.vh, nu, par ^ 1)};
#define SU2_WL(A, k, l) ld(A[((k) + (l)) & 1], (s0 + (uint32_t)(oa[k] + ob[l])) >> 1)
        // every size up to N x N is computed without branches, so that the loads
        // can be issued ahead of the products; sizes beyond (rmax, tmax) are not
        // reported (the offsets wrap periodically, so every load stays inside)
        // the links of each stage are loaded together (the scheduling barrier
        // keeps them ahead of the products that use them)
        const Q one{1.0f, 0.0f, 0.0f, 0.0f};
        Q B[N], D[N], L[2 * N + 1];
#pragma unroll
        for (int t = 0; t < N; ++t) L[t] = SU2_WL(Anu, 0, t);
        __builtin_amdgcn_sched_barrier(0);
        Q P = one;
#pragma unroll
        for (int t = 0; t < N; ++t) {
            P = qmul(P, L[t]);
            B[t] = P;
            D[t] = one;
        }
        Q A = one;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            L[2 * N] = SU2_WL(Amu, r, 0);
#pragma unroll
            for (int t = 0; t < N; ++t) {
                L[2 * t] = SU2_WL(Amu, r, t + 1);
                L[2 * t + 1] = SU2_WL(Anu, r + 1, t);
            }
            __builtin_amdgcn_sched_barrier(0);
            A = qmul(A, L[2 * N]);
            Q C = one;
#pragma unroll
            for (int t = 0; t < N; ++t) {
                D[t] = qmul(D[t], L[2 * t]);
                C = qmul(C, L[2 * t + 1]);
                w[r][t] = qdot(qmul(A, C), qmul(B[t], D[t]));
            }
        }
        (void)rmax;
        (void)tmax;
#undef SU2_WL
    }
    const uint32_t slot = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int t = 0; t < N; ++t) {
            const double bs = block_sum((double)w[r][t]);
            if (threadIdx.x == 0) part[(size_t)slot * N * N + r * N + t] = bs;
        }
}

// Workgroup k: the sum of partial k over all slots in a fixed order (thread j
// takes slots j, j + 256, ... in turn, then the fixed-order block sum).
__global__ __launch_bounds__(256) void wilson_sum_kernel(const double *__restrict__ part,
                                                         uint32_t nslots, int nn,
                                                         double *__restrict__ out)
{
    const int k = (int)blockIdx.x;
    double s = 0.0;
    for (uint32_t b = threadIdx.x; b < nslots; b += blockDim.x) s += part[(size_t)b * nn + k];
    s = block_sum(s);
    if (threadIdx.x == 0) out[k] = s;
}

// ------------------------------------------------------------- work queue
// Whole sweeps of every replica in one persistent launch (QueuePlan).  A
// workgroup serves the queue of its XCD (hardware XCC id -> qs->rank) and
// takes `grain` consecutive items per ticket; consecutive items of one
// replica and stage form a run that waits once and signals once.  A run of
// replica r waits until r's done counter reaches queue_target: every item of
// r's earlier stages and the bookkeeping of r's earlier sweeps are finished.
// Items wait only on items of their own queue with smaller tickets, which
// running workgroups of the same XCD have already taken, so a queue cannot
// deadlock; every wait is still bounded by spin_limit polls, after which
// qs->error is raised and all workgroups drain without waiting.
//
// Ordering within one XCD: the L1 caches are write-through and the L2 is
// shared by the XCD's compute units, so a producer only waits until its
// stores have reached the L2 (vmcnt 0) before the done counter is
// incremented; an agent-scope release, which also writes the L2 back to
// memory, is not needed and costs about a microsecond per run.  The waiting
// thread performs an agent-scope acquire after seeing the count (it
// invalidates the compute unit's L1; a workgroup-scope L1 invalidation alone
// left stale lines on gfx950 when producer and consumer ran on different
// compute units).  The counters, the tickets and the measurement
// accumulators are device-scope atomics.
__device__ __forceinline__ uint32_t xcc_id()
{
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;  // hwreg(HW_REG_XCC_ID, 0, 4)
}

// Invalidate this compute unit's L1 (vector data cache).
__device__ __forceinline__ void l1_invalidate() { asm volatile("buffer_inv sc0" ::: "memory"); }

__device__ __forceinline__ void queue_wait(const Rep &R, uint32_t target, QueueState *qs,
                                           uint32_t spin_limit)
{
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load(&R.cnt->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
            if (__hip_atomic_load(&qs->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (++spins > spin_limit) {
                __hip_atomic_store(&qs->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    l1_invalidate();  // every wave (workgroup scope)
}

// Every wave's stores reach the L2, then thread 0 adds k to the done
// counter; returns the counter's previous value in thread 0.
__device__ __forceinline__ uint32_t queue_signal(const Rep &R, uint32_t k)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    uint32_t old = 0u;
    if (threadIdx.x == 0)
        old = __hip_atomic_fetch_add(&R.cnt->done, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return old;
}

template <bool LEARNED>
__device__ __forceinline__ void queue_pass(const Rep &R, int mu, int par, bool measure,
                                           uint32_t gid, uint32_t sweep, uint32_t k0, uint32_t k1,
                                           const float *ltab, float &m, int &a)
{
#define SU2_QPASS(MU)                                                                      \
    if (measure)                                                                           \
        update_site<MU, true, LEARNED, false, false, false>(R, gid, par, sweep, k0, k1, ltab, \
                                                            m, a);                         \
    else                                                                                   \
        update_site<MU, false, LEARNED, false, false, false>(R, gid, par, sweep, k0, k1,     \
                                                             ltab, m, a);
    switch (mu) {
    case 0: SU2_QPASS(0) break;
    case 1: SU2_QPASS(1) break;
    case 2: SU2_QPASS(2) break;
    default: SU2_QPASS(3) break;
    }
#undef SU2_QPASS
}

// End of sweep i of replica r: totals of the plaquette and Polyakov
// accumulators (taken and reset atomically), history row (row counter) + i.
__device__ __forceinline__ void queue_sweep_end(const Rep &R, const QueuePlan &plan, uint32_t i,
                                                double *hist, int nrep, uint32_t r)
{
    unsigned long long tp = 0ull, tl = 0ull;
    for (uint32_t j = threadIdx.x; j < (uint32_t)kBuckets; j += blockDim.x) {
        tp += __hip_atomic_exchange(bucket(R.acc, ACC_PLAQ, j), 0ull, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
        tl += __hip_atomic_exchange(bucket(R.acc, ACC_POLY, j), 0ull, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    }
    tp = block_sum_u64(tp);
    tl = block_sum_u64(tl);
    if (plan.rows && hist && threadIdx.x == 0) {
        const Geom &g = R.g;
        const double p = plan.want_p ? from_fixed(tp) / (12.0 * (double)g.vh) : 0.0;
        const double l = plan.want_l ? from_fixed(tl) / ((double)g.nx * g.ny * g.nz) : 0.0;
        double *row = hist + 3 * ((size_t)(*row_counter(R.cnt, plan.graph_rows != 0u) + i) *
                                      nrep + r);
        row[0] = p;
        row[1] = l;
        row[2] = fabs(l);
    }
}

// One item: slot `local` of replica R in stage `it` of the sweep.
template <bool LEARNED>
__device__ __forceinline__ void queue_item(const Rep &R, const QueuePlan &plan, const QueueItem &it,
                                           uint32_t local, uint32_t k0, uint32_t k1, int snake,
                                           const float *ltab)
{
    const Geom &g = R.g;
    const uint32_t B = blockDim.x, n = R.nblocks;
    if (it.kind == QK_PASS) {
        const int mu = (int)(it.stage >> 1), par = (int)(it.stage & 1u);
        const bool measure =
            plan.want_p && par == 1 && mu >= 1 && !queue_reunit_sweep(plan, it.sweep);
        const uint32_t blk = (snake && par) ? n - 1u - local : local;
        const uint32_t gid = blk * B + threadIdx.x;
        float m = 0.0f;
        int a = -1;
        if (gid < g.vh) {
            const uint32_t sweep =
                *(const __attribute__((address_space(4))) uint32_t *)&R.cnt->sweep + it.sweep;
            queue_pass<LEARNED>(R, mu, par, measure, gid, sweep, k0, k1, ltab, m, a);
        }
        if (measure) block_accumulate((double)m, R.acc, ACC_PLAQ, local);
        if (LEARNED) {
            const unsigned long long mp = __ballot(a >= 0);
            const unsigned long long ma = __ballot(a == 1);
            if ((threadIdx.x & 63) == 0) {
                const uint32_t wb = local * (B >> 6) + (threadIdx.x >> 6);
                if (mp) atomicAdd(bucket(R.acc, ACC_PROPOSED, wb), (unsigned long long)__popcll(mp));
                if (ma) atomicAdd(bucket(R.acc, ACC_ACCEPTED, wb), (unsigned long long)__popcll(ma));
            }
        }
    } else if (it.kind == QK_REUNIT) {
        const uint32_t h = local * B + threadIdx.x;
        if (h < g.vh)
            for (int k = 0; k < 8; ++k) reunit_link(R, k >> 1, k & 1, h);
    } else if (it.kind == QK_PLAQ) {
        const uint32_t i = local * B + threadIdx.x;
        double v = 0.0;
        if (i < g.vh) v = (double)site_plaquettes(R, i) + (double)site_plaquettes(R, i + g.vh);
        block_accumulate(v, R.acc, ACC_PLAQ, local);
    } else {
        // L(x) = (1/2)Tr prod_t U_3(x, t), t = 0 leftmost
        const uint32_t ns3 = (uint32_t)g.nx * g.ny * g.nz;
        if (local * B < ns3) {
            const uint32_t xs = local * B + threadIdx.x;
            double v = 0.0;
            if (xs < ns3) {
                const uint32_t x = xs % (uint32_t)g.nx, q = xs / (uint32_t)g.nx;
                const uint32_t y = q % (uint32_t)g.ny, z = q / (uint32_t)g.ny;
                const uint32_t pbase = (x + y + z) & 1u;
                Q P{1.0f, 0.0f, 0.0f, 0.0f};
                for (int tt = 0; tt < g.nt; ++tt)
                    P = qmul(P, ldq(R.links, g.vh, 3, (int)((pbase + (uint32_t)tt) & 1u),
                                    (xs >> 1) + (uint32_t)tt * (ns3 >> 1)));
                v = (double)P.w;
            }
            block_accumulate(v, R.acc, ACC_POLY, local);
        }
    }
}

template <bool LEARNED>
__global__ __launch_bounds__(256) void queue_sweeps_kernel(
    const Rep *__restrict__ reps, const uint32_t *__restrict__ qmap, QueuePlan plan, int grain,
    uint32_t k0, uint32_t k1, int snake, double *__restrict__ hist, int nrep, QueueState *qs,
    uint32_t spin_limit, const float *__restrict__ table)
{
    __shared__ float4 stab4[LEARNED ? 1 + kNNRows * kNNRow / 4 : 1];
    __shared__ uint32_t s_ticket, s_last;
    const int q = qs->rank[xcc_id()];  // uniform over the workgroup
    if (q < 0) return;
    const uint32_t slots = qs->slots[q];
    if (slots == 0u) return;
    const uint32_t total = queue_total_stages(plan) * slots;
    const uint32_t *map = qmap ? qmap + qs->off[q] : nullptr;
    const float *ltab = LEARNED ? load_table_lds(stab4, table) : nullptr;
    for (;;) {
        if (threadIdx.x == 0)
            s_ticket = __hip_atomic_fetch_add(&qs->ticket[q][0], (uint32_t)grain,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t t0 = s_ticket;
        __syncthreads();  // every thread has read s_ticket
        if (t0 >= total) break;
        const uint32_t t1 = min(t0 + (uint32_t)grain, total);
        for (uint32_t t = t0; t < t1;) {
            const QueueItem it = queue_decode(plan, t, slots);
            const uint32_t r = map ? map[it.slot] : 0u;
            const Rep &R = reps[r];
            const uint32_t local = it.slot - R.qfirst, n = R.nblocks;
            // run: the following items of the same replica and stage
            const uint32_t len = min(t1 - t, n - local);
            queue_wait(R, queue_target(plan, n, it.sweep, it.stage), qs, spin_limit);
            for (uint32_t k = 0; k < len; ++k)
                queue_item<LEARNED>(R, plan, it, local + k, k0, k1, snake, ltab);
            const uint32_t old = queue_signal(R, len);
            if (threadIdx.x == 0) s_last = old + len == queue_sweep_last(plan, n, it.sweep);
            __syncthreads();
            if (s_last) {  // uniform: this workgroup finished the sweep of replica r
                if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __syncthreads();
                queue_sweep_end(R, plan, it.sweep, hist, nrep, r);
                (void)queue_signal(R, 1u);
            }
            __syncthreads();  // s_last is rewritten by the next run
            t += len;
        }
    }
}

// grid (1, 1, replica): check that every item of the replica ran (else raise
// the error flag), advance the counters past the launch's sweeps and clear
// the queue state for the next launch.
__global__ void queue_epilogue_kernel(const Rep *__restrict__ reps, QueuePlan plan,
                                      QueueState *qs)
{
    const Rep &R = reps[blockIdx.z];
    if (R.cnt->done != queue_target(plan, R.nblocks, plan.ns, 0u)) qs->error = 2u;
    R.cnt->sweep += plan.ns;
    if (plan.rows) *row_counter(R.cnt, plan.graph_rows != 0u) += plan.ns;
    R.cnt->done = 0u;
    if (blockIdx.z == 0)
        for (int k = 0; k < kMaxQueues; ++k) qs->ticket[k][0] = 0u;
}

__global__ void xcc_probe_kernel(uint32_t *mask)
{
    if (threadIdx.x == 0) atomicOr(mask, 1u << xcc_id());
}

// ---------------------------------------------------------- gauge (tests)
// Replica 0 only (G holds one field of gauge rotations).
__global__ void gauge_gen_kernel(const Rep *__restrict__ reps, float4 *__restrict__ G,
                                 uint32_t k0, uint32_t k1)
{
    const Rep &R = reps[0];
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 2u * R.g.vh) return;
    const Q q = haar_from_block(philox(s, 0u, word2(0u, TAG_GAUGE, R.replica), 0u, k0, k1));
    G[s] = make_float4(q.w, q.x, q.y, q.z);
}

__global__ void gauge_apply_kernel(const Rep *__restrict__ reps, const float4 *__restrict__ G)
{
    const Rep &R = reps[0];
    const Geom &g = R.g;
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= g.vh) return;
    const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
    int c[4];
    decode(g, h, par, c[0], c[1], c[2], c[3]);
    const uint32_t site = 2u * h + (uint32_t)(c[0] & 1);
    const int n[4] = {g.nx, g.ny, g.nz, g.nt};
    c[mu] = c[mu] + 1 == n[mu] ? 0 : c[mu] + 1;
    const uint32_t fsite = 2u * hidx(g, c[0], c[1], c[2], c[3]) + (uint32_t)(c[0] & 1);
    const float4 a = G[site], b = G[fsite];
    const Q U = ldq(R.links, g.vh, mu, par, h);
    const Q r = qmul(qmul(Q{a.x, a.y, a.z, a.w}, U), qdag(Q{b.x, b.y, b.z, b.w}));
    st(R.links, g.vh, mu, par, h, r);
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
    int nt = 0;
    const Q U = heatbath_link(Q{v.x, v.y, v.z, v.w}, beta, (uint32_t)i, sweep,
                              word2(mu, TAG_TRIAL, replica), k0, k1, &nt);
    out[i] = make_float4(U.w, U.x, U.y, U.z);
    if (ntrials) ntrials[i] = nt;
}

inline uint32_t lo32(uint64_t v) { return (uint32_t)v; }
inline uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
inline unsigned nblk(uint64_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }
inline unsigned round8(unsigned n) { return (n + 7u) & ~7u; }

template <int MU, bool LEARNED, bool OR, bool NORM>
void launch_pass_mn(const Ens &e, int par, uint64_t seed, bool measure, const float *table,
                    const LaunchCfg &cfg, hipStream_t stream)
{
    const unsigned total = e.amap ? e.amap_len : e.total_blocks;
    unsigned grid = total;
    if (cfg.grid_cap && cfg.grid_cap < grid) grid = cfg.grid_cap & ~7u;
    if (grid == 0) grid = 8;
    const int rev = cfg.snake ? par : 0;
    if (measure)
        hipLaunchKernelGGL((pass_kernel<MU, true, LEARNED, OR, NORM>), dim3(grid),
                           dim3(cfg.pass_block), 0, stream, e.reps, e.bmap, e.amap, total, par,
                           lo32(seed), hi32(seed), (int)cfg.xcd_remap, rev, table);
    else
        hipLaunchKernelGGL((pass_kernel<MU, false, LEARNED, OR, NORM>), dim3(grid),
                           dim3(cfg.pass_block), 0, stream, e.reps, e.bmap, e.amap, total, par,
                           lo32(seed), hi32(seed), (int)cfg.xcd_remap, rev, table);
}

template <int MU, bool LEARNED, bool OR = false>
void launch_pass_mu(const Ens &e, int par, uint64_t seed, bool measure, const float *table,
                    const LaunchCfg &cfg, bool norm, hipStream_t stream)
{
    if (norm)
        launch_pass_mn<MU, LEARNED, OR, true>(e, par, seed, measure, table, cfg, stream);
    else
        launch_pass_mn<MU, LEARNED, OR, false>(e, par, seed, measure, table, cfg, stream);
}

template <bool LEARNED>
void launch_pass_l(const Ens &e, int mu, int par, uint64_t seed, bool measure,
                   const float *table, const LaunchCfg &cfg, bool norm, hipStream_t stream)
{
    switch (mu) {
    case 0: launch_pass_mu<0, LEARNED>(e, par, seed, measure, table, cfg, norm, stream); break;
    case 1: launch_pass_mu<1, LEARNED>(e, par, seed, measure, table, cfg, norm, stream); break;
    case 2: launch_pass_mu<2, LEARNED>(e, par, seed, measure, table, cfg, norm, stream); break;
    default: launch_pass_mu<3, LEARNED>(e, par, seed, measure, table, cfg, norm, stream); break;
    }
}

}  // namespace

hipError_t launch_init(const Ens &e, const int *starts_dev, uint64_t seed, hipStream_t stream)
{
    hipLaunchKernelGGL(init_kernel, dim3(nblk(e.max_vh, 256), 8, e.nrep), dim3(256), 0, stream,
                       e.reps, starts_dev, lo32(seed), hi32(seed));
    return hipGetLastError();
}

hipError_t launch_pass(const Ens &e, int mu, int par, uint64_t seed, bool measure,
                       const float *table, const LaunchCfg &cfg, hipStream_t stream, bool norm)
{
    if (table)
        launch_pass_l<true>(e, mu, par, seed, measure, table, cfg, norm, stream);
    else
        launch_pass_l<false>(e, mu, par, seed, measure, nullptr, cfg, norm, stream);
    return hipGetLastError();
}

hipError_t launch_or_pass(const Ens &e, int mu, int par, bool measure, const LaunchCfg &cfg,
                          hipStream_t stream, bool norm)
{
    switch (mu) {
    case 0: launch_pass_mu<0, false, true>(e, par, 0, measure, nullptr, cfg, norm, stream); break;
    case 1: launch_pass_mu<1, false, true>(e, par, 0, measure, nullptr, cfg, norm, stream); break;
    case 2: launch_pass_mu<2, false, true>(e, par, 0, measure, nullptr, cfg, norm, stream); break;
    default: launch_pass_mu<3, false, true>(e, par, 0, measure, nullptr, cfg, norm, stream); break;
    }
    return hipGetLastError();
}

// Standalone plaquette launch: t-chunks of 2 planes; workgroups of
// 256 threads, or of 192 or 128 where that size divides the (x, y) plane of
// every replica and 256 does not (no idle lanes in the last tile).
hipError_t launch_plaquette(const Ens &e, hipStream_t stream)
{
    const uint32_t T = (uint32_t)std::min(e.poly_s, 2);  // poly_s divides every Nt
    uint32_t B = 256;
    if (e.plane_hs && e.plane_hs % 256u) {
        if (e.plane_hs % 192u == 0) B = 192;
        else if (e.plane_hs % 128u == 0) B = 128;
    }
    hipLaunchKernelGGL(plaquette_march_kernel, dim3(round8(nblk(e.max_vh, B * T)), 1, e.nrep),
                       dim3(B), 0, stream, e.reps, T);
    return hipGetLastError();
}

hipError_t launch_polyakov(const Ens &e, hipStream_t stream)
{
    const dim3 grid(nblk(e.max_ns3, 64), 1, e.nrep), block(64 * e.poly_s);
    switch (e.poly_s) {
    case 8: hipLaunchKernelGGL(polyakov_kernel<8>, grid, block, 0, stream, e.reps); break;
    case 4: hipLaunchKernelGGL(polyakov_kernel<4>, grid, block, 0, stream, e.reps); break;
    case 2: hipLaunchKernelGGL(polyakov_kernel<2>, grid, block, 0, stream, e.reps); break;
    default: hipLaunchKernelGGL(polyakov_kernel<1>, grid, block, 0, stream, e.reps); break;
    }
    return hipGetLastError();
}

hipError_t launch_take(const Ens &e, int flags, hipStream_t stream)
{
    hipLaunchKernelGGL(take_kernel, dim3(1, 1, e.nrep), dim3(kBuckets), 0, stream, e.reps, flags);
    return hipGetLastError();
}

hipError_t launch_sweep_end(const Ens &e, int flags, double *hist, hipStream_t stream)
{
    hipLaunchKernelGGL(sweep_end_kernel, dim3(1, 1, e.nrep), dim3(kBuckets), 0, stream, e.reps,
                       e.nrep, flags, hist);
    return hipGetLastError();
}

hipError_t launch_counts(const Ens &e, int reset, hipStream_t stream)
{
    hipLaunchKernelGGL(counts_kernel, dim3(1, 1, e.nrep), dim3(kBuckets), 0, stream, e.reps,
                       reset);
    return hipGetLastError();
}

hipError_t launch_set_counter(const Ens &e, uint32_t sweep, uint32_t meas, int which,
                              hipStream_t stream, QueueState *qs)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1, 1, e.nrep), dim3(kBuckets), 0, stream, e.reps,
                       sweep, meas, which, qs);
    return hipGetLastError();
}

hipError_t launch_reunitarize(const Ens &e, hipStream_t stream)
{
    hipLaunchKernelGGL(reunit_kernel, dim3(nblk(e.max_vh, 256), 8, e.nrep), dim3(256), 0, stream,
                       e.reps);
    return hipGetLastError();
}

hipError_t launch_gauge(const Ens &e, float *G, uint64_t seed, hipStream_t stream)
{
    hipLaunchKernelGGL(gauge_gen_kernel, dim3(nblk(2ull * e.max_vh, 256)), dim3(256), 0, stream,
                       e.reps, (float4 *)G, lo32(seed), hi32(seed));
    hipLaunchKernelGGL(gauge_apply_kernel, dim3(nblk(e.max_vh, 256), 8), dim3(256), 0, stream,
                       e.reps, (const float4 *)G);
    return hipGetLastError();
}

hipError_t launch_small_sweeps(const Ens &e, int ns, uint64_t seed, int reunit_every, int flags,
                               double *hist, const float *table, hipStream_t stream)
{
    if (ns <= 0) return hipSuccess;
    const uint32_t block = std::min<uint32_t>(1024u, (e.max_vh + 63u) & ~63u);
    if (table)
        hipLaunchKernelGGL(small_sweeps_kernel<true>, dim3(e.nrep), dim3(block), 0, stream, e.reps,
                           e.nrep, ns, lo32(seed), hi32(seed), reunit_every, flags, hist, table);
    else
        hipLaunchKernelGGL(small_sweeps_kernel<false>, dim3(e.nrep), dim3(block), 0, stream, e.reps,
                           e.nrep, ns, lo32(seed), hi32(seed), reunit_every, flags, hist, table);
    return hipGetLastError();
}

hipError_t launch_queue_sweeps(const Ens &e, const QueuePlan &plan, const uint32_t *qmap,
                               uint64_t seed, int block, uint32_t grid, int grain, bool snake,
                               double *hist, const float *table, QueueState *qs,
                               uint32_t spin_limit, hipStream_t stream)
{
    if (plan.ns == 0u) return hipSuccess;
    if (grid == 0u) grid = 1u;
    if (table)
        hipLaunchKernelGGL(queue_sweeps_kernel<true>, dim3(grid), dim3(block), 0, stream, e.reps,
                           qmap, plan, grain, lo32(seed), hi32(seed), (int)snake, hist, e.nrep, qs,
                           spin_limit, table);
    else
        hipLaunchKernelGGL(queue_sweeps_kernel<false>, dim3(grid), dim3(block), 0, stream, e.reps,
                           qmap, plan, grain, lo32(seed), hi32(seed), (int)snake, hist, e.nrep, qs,
                           spin_limit, table);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(queue_epilogue_kernel, dim3(1, 1, e.nrep), dim3(1), 0, stream, e.reps, plan,
                       qs);
    return hipGetLastError();
}

hipError_t probe_xcc_mask(uint32_t *mask)
{
    uint32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(uint32_t));
    if (e != hipSuccess) return e;
    e = hipMemset(d, 0, sizeof(uint32_t));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(xcc_probe_kernel, dim3(4096), dim3(64), 0, nullptr, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(mask, d, sizeof(uint32_t), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e;
}

uint32_t queue_resident_grid(int block, bool learned)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = learned ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                 &per_cu, queue_sweeps_kernel<true>, block, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                 &per_cu, queue_sweeps_kernel<false>, block, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || per_cu <= 0 || cus <= 0) return 1024u;
    return (uint32_t)(per_cu * cus);
}

hipError_t launch_wilson(const Ens &e, int rmax, int tmax, double *part, double *sums,
                         hipStream_t stream)
{
    const uint32_t nb = nblk(2ull * e.max_vh, 256);
    hipLaunchKernelGGL(wilson_kernel<kWilsonMax>, dim3(nb, 12), dim3(256), 0, stream, e.reps,
                       rmax, tmax, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(wilson_sum_kernel, dim3(kWilsonMax * kWilsonMax), dim3(256), 0, stream,
                       part, 12u * nb, kWilsonMax * kWilsonMax, sums);
    return hipGetLastError();
}

hipError_t launch_test_stream(const Ens &e, int mu, int par, float *out, hipStream_t stream)
{
    hipLaunchKernelGGL(stream_kernel, dim3(nblk(e.max_vh, 256)), dim3(256), 0, stream, e.reps, mu,
                       par, out);
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
