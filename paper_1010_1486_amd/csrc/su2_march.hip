// su2_march.hip -- the heat-bath (and over-relaxation) pass with its
// neighbour links staged in LDS, marching along t.
//
// The update of U_mu(s) (Sec. 2: six-staple sum V, k = sqrt(det V), a0 from
// sqrt(1 - a0^2) exp(beta k a0), U' = X U~^+) reads 18 neighbouring links
// from 7 of the 8 link classes.  In the plain pass kernel each thread loads
// them itself and the caches have to catch the re-reads; the z and t
// neighbours lie one or many (x, y) planes away and are mostly fetched again
// from memory.  Here a workgroup owns a tile of R full x-rows of one (x, y)
// plane at fixed z and walks T planes along t.  Every class the update reads
// in the tile's own plane is staged in LDS (with one halo row above and
// below), together with the neighbouring t-plane where the update needs it,
// so each link is loaded once per workgroup; the loads of the next plane are
// issued before the current plane is computed.  Only the z neighbours are
// read from global memory: the workgroups of z - 1 and z + 1 are launched
// next to it on the same XCD and stage those planes at the same time, so the
// reads are served by that XCD's L2.  The arithmetic is the plain pass's (the
// same inline functions in the same order), so the links are bit for bit
// those of the plain pass kernel.
#include "su2_internal.h"
#include "su2_kcommon.h"

using namespace su2dev;

namespace su2rt {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4f gv4f;
typedef __attribute__((address_space(1))) const v4f gv4fc;

// Residency of link class (nu, q) -- q = 0 the pass's parity, 1 the opposite
// one -- during the step that updates plane t: planes t + lo .. t + hi live
// in LDS (hi < lo: the class is not read).  The planes a pass needs follow
// from the staple's offsets: for mu != t the t-links one plane back (the
// backward t staple) and U_mu one plane ahead (the forward one); for mu = t
// the x and y links one plane ahead.
__host__ __device__ constexpr int res_lo(int MU, int nu, int q)
{
    return MU != 3 ? (nu == 3 && q == 0 && MU != 2 ? -1 : 0)
                   : (nu == 2 && q == 1 ? 1 : 0);
}
__host__ __device__ constexpr int res_hi(int MU, int nu, int q)
{
    return (nu == MU && q == 0) ? -1  // the class the pass writes is never read
           : MU != 3 ? (nu == MU ? 1 : 0)
                     : (nu == 3 ? 0 : (nu == 2 ? (q == 1 ? 1 : 0) : 1));
}
__host__ __device__ constexpr int res_n(int MU, int nu, int q)
{
    return res_hi(MU, nu, q) >= res_lo(MU, nu, q) ? res_hi(MU, nu, q) - res_lo(MU, nu, q) + 1 : 0;
}
// first LDS slot of class k = nu * 2 + q
__host__ __device__ constexpr int res_base(int MU, int k)
{
    int b = 0;
    for (int i = 0; i < k; ++i) b += res_n(MU, i >> 1, i & 1);
    return b;
}
__host__ __device__ constexpr int res_slots(int MU) { return res_base(MU, 8); }
// classes whose own link one plane back is kept in a register (it is needed
// only at the thread's own (x, y) position)
__host__ __device__ constexpr bool carried(int MU, int nu, int q)
{
    return MU != 3 && q == 1 && (nu == MU || nu == 3);
}

struct Tile {
    const Geom *g;
    const char *links;  // base of the 8 class arrays
    int par;
    uint32_t hx, R, z, y0;
    uint32_t xh, yl;    // the thread's position in the tile (yl < R when active)
    bool active;
    int bit;            // x & 1 of the updated site on the current plane
    uint32_t t;         // current plane (wrapped)
    int tl;             // current plane (logical, for the ring slots)
};

__device__ __forceinline__ uint32_t wrap(int v, int n) { return (uint32_t)(v < 0 ? v + n : (v >= n ? v - n : v)); }

__device__ __forceinline__ gv4fc *cls_ptr(const char *links, uint32_t vh, int nu, int parity)
{
    return (gv4fc *)(links + (size_t)(nu * 2 + parity) * vh * 16u);
}

// Half-site index of the (x, y)-position (xh, y) on plane (z, t).
__device__ __forceinline__ uint32_t hidx(const Geom &g, uint32_t xh, uint32_t y, uint32_t z,
                                         uint32_t t)
{
    return xh + g.hx * y + g.P * z + g.PZ * t;
}

// x-half-index of the neighbour dx in {-1, 0, 1} of a site with x & 1 = bit.
__device__ __forceinline__ uint32_t nbx(uint32_t xh, int bit, int dx, uint32_t hx)
{
    if (dx == 0) return xh;
    const int v = (int)xh + bit + (dx > 0 ? 0 : -1);
    return wrap(v, (int)hx);
}

__device__ __forceinline__ Q toq(v4f v) { return Q{v.x, v.y, v.z, v.w}; }

// The link of class (NU, Q_) at offset (DX, DY, DZ, DT) from the updated site.
template <int MU, int NU, int Q_, int DX, int DY, int DZ, int DT>
__device__ __forceinline__ Q fetch(const Tile &T, const v4f *lds, uint32_t slot_sz,
                                   const Q *carry)
{
    const Geom &g = *T.g;
    const uint32_t xn = nbx(T.xh, T.bit, DX, T.hx);
    if constexpr (DZ != 0) {  // another workgroup's plane: global memory (that XCD's L2)
        const uint32_t y = wrap((int)(T.y0 + T.yl) + DY, g.ny);
        const uint32_t z = wrap((int)T.z + DZ, g.nz);
        const uint32_t t = wrap((int)T.t + DT, g.nt);
        const v4f v = cls_ptr(T.links, g.vh, NU, T.par ^ Q_)[hidx(g, xn, y, z, t)];
        return toq(v);
    } else if constexpr (DT < res_lo(MU, NU, Q_)) {  // own link one plane back
        static_assert(DX == 0 && DY == 0 && DT == -1 && carried(MU, NU, Q_),
                      "link neither staged nor carried");
        return carry[NU == 3 ? 1 : 0];
    } else {
        static_assert(DT <= res_hi(MU, NU, Q_), "link not staged");
        constexpr int n = res_n(MU, NU, Q_);
        const int slot = res_base(MU, NU * 2 + Q_) + (n == 2 ? ((T.tl + DT) & 1) : 0);
        return toq(lds[slot * slot_sz + (T.yl + 1 + DY) * T.hx + xn]);
    }
}

// Staple sum of U_MU at the tile site, in the order and arithmetic of the
// plain pass (update_at): for nu != MU, forward U_nu(s+mu) U_mu(s+nu)^+
// U_nu(s)^+ and backward (U_mu(s-nu) U_nu(s+mu-nu))^+ U_nu(s-nu).
template <int MU, int NU, bool MEASURE>
__device__ __forceinline__ void staple_term(const Tile &T, const v4f *lds, uint32_t ssz,
                                            const Q *carry, Q &V, Q &Vlow)
{
    constexpr int mx = MU == 0, my = MU == 1, mz = MU == 2, mt = MU == 3;
    constexpr int nx = NU == 0, ny = NU == 1, nz = NU == 2, nt = NU == 3;
    const Q A = fetch<MU, NU, 1, mx, my, mz, mt>(T, lds, ssz, carry);
    const Q B = fetch<MU, MU, 1, nx, ny, nz, nt>(T, lds, ssz, carry);
    const Q C = fetch<MU, NU, 0, 0, 0, 0, 0>(T, lds, ssz, carry);
    const Q D = fetch<MU, NU, 0, mx - nx, my - ny, mz - nz, mt - nt>(T, lds, ssz, carry);
    const Q E = fetch<MU, MU, 1, -nx, -ny, -nz, -nt>(T, lds, ssz, carry);
    const Q F = fetch<MU, NU, 1, -nx, -ny, -nz, -nt>(T, lds, ssz, carry);
    const Q st = qadd(qmul(qmul(A, qdag(B)), qdag(C)), qmul(qdag(qmul(E, D)), F));
    V = qadd(V, st);
    if (MEASURE && NU < MU) Vlow = qadd(Vlow, st);
}

template <int MU, bool MEASURE>
__device__ __forceinline__ Q staple_tile(const Tile &T, const v4f *lds, uint32_t ssz,
                                         const Q *carry, Q &Vlow)
{
    Q V{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (MU != 0) staple_term<MU, 0, MEASURE>(T, lds, ssz, carry, V, Vlow);
    if constexpr (MU != 1) staple_term<MU, 1, MEASURE>(T, lds, ssz, carry, V, Vlow);
    if constexpr (MU != 2) staple_term<MU, 2, MEASURE>(T, lds, ssz, carry, V, Vlow);
    if constexpr (MU != 3) staple_term<MU, 3, MEASURE>(T, lds, ssz, carry, V, Vlow);
    return V;
}

// Loads of plane tl (logical) of class (nu, q) for this thread: its own
// element and, for the first 2 hx threads, one halo-row element.
struct Pre {
    v4f own, halo;
};

__device__ __forceinline__ Pre load_plane(const Tile &T, int nu, int q, int tl)
{
    const Geom &g = *T.g;
    const uint32_t t = wrap(tl, g.nt);
    gv4fc *p = cls_ptr(T.links, g.vh, nu, T.par ^ q);
    Pre r;
    r.own = T.active ? p[hidx(g, T.xh, T.y0 + T.yl, T.z, t)] : v4f{0.0f, 0.0f, 0.0f, 0.0f};
    r.halo = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    if (threadIdx.x < 2u * T.hx) {
        const uint32_t x = threadIdx.x % T.hx;
        const uint32_t y = threadIdx.x < T.hx ? wrap((int)T.y0 - 1, g.ny) : wrap((int)(T.y0 + T.R), g.ny);
        r.halo = p[hidx(g, x, y, T.z, t)];
    }
    return r;
}

__device__ __forceinline__ void store_plane(const Tile &T, v4f *lds, uint32_t ssz, int slot,
                                            const Pre &r)
{
    v4f *s = lds + slot * ssz;
    if (T.active) s[(T.yl + 1) * T.hx + T.xh] = r.own;
    if (threadIdx.x < 2u * T.hx) {
        const uint32_t x = threadIdx.x % T.hx;
        s[(threadIdx.x < T.hx ? 0u : T.R + 1u) * T.hx + x] = r.halo;
    }
}

template <int MU>
__device__ __forceinline__ int slot_of(int nu, int q, int tl)
{
    return res_base(MU, nu * 2 + q) + (res_n(MU, nu, q) == 2 ? (tl & 1) : 0);
}

}  // namespace

// One (MU, parity) pass of a single lattice.  Workgroup b runs unit u: plane
// rows [y0, y0 + R) at z, planes t0 .. t0 + T - 1, with z fastest among the
// units of one XCD's contiguous range (units u = xcd * per + j when the unit
// count is a multiple of 8; per = 0: u = b), walked backwards when `rev`.
template <int MU, bool MEASURE, bool OR>
__global__ __launch_bounds__(256) void march_kernel(const Rep *__restrict__ reps, int par,
                                                     uint32_t k0, uint32_t k1, uint32_t R,
                                                     uint32_t TT, uint32_t ntile, uint32_t nunits,
                                                     uint32_t per, int rev)
{
    extern __shared__ v4f lds[];
    const Rep &Rp = reps[0];
    const Geom &g = Rp.g;
    const uint32_t b = blockIdx.x;
    uint32_t u;
    if (per) {
        const uint32_t j = b >> 3;
        u = (b & 7u) * per + (rev ? per - 1u - j : j);
    } else {
        u = rev ? nunits - 1u - b : b;
    }
    Tile T;
    T.g = &g;
    T.links = reinterpret_cast<const char *>(Rp.links);
    T.par = par;
    T.hx = g.hx;
    T.R = R;
    T.z = u % (uint32_t)g.nz;
    const uint32_t rest = u / (uint32_t)g.nz;
    T.y0 = (rest % ntile) * R;
    const uint32_t t0 = (rest / ntile) * TT;
    T.xh = threadIdx.x % g.hx;
    T.yl = threadIdx.x / g.hx;
    T.active = T.yl < R;
    const uint32_t ssz = (R + 2u) * g.hx;
    const uint32_t sweep = *(const __attribute__((address_space(4))) uint32_t *)&Rp.cnt->sweep;

    // stage the planes the first step needs, and the carried links one plane back
    Q carry[2] = {Q{0.0f, 0.0f, 0.0f, 0.0f}, Q{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int nu = k >> 1, q = k & 1;
        if (res_n(MU, nu, q) == 0) continue;
        for (int d = res_lo(MU, nu, q); d <= res_hi(MU, nu, q); ++d)
            store_plane(T, lds, ssz, slot_of<MU>(nu, q, (int)t0 + d), load_plane(T, nu, q, (int)t0 + d));
        if (carried(MU, nu, q) && T.active)
            carry[nu == 3 ? 1 : 0] = toq(load_plane(T, nu, q, (int)t0 - 1).own);
    }
    __syncthreads();

    double macc = 0.0;
    for (uint32_t i = 0; i < TT; ++i) {
        const int tl = (int)(t0 + i);
        T.tl = tl;
        T.t = (uint32_t)tl;
        const bool more = i + 1 < TT;
        // loads of the planes the next step adds (issued before the arithmetic)
        Pre pre[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int nu = k >> 1, q = k & 1;
            if (res_n(MU, nu, q) == 0 || !more) continue;
            pre[k] = load_plane(T, nu, q, tl + res_hi(MU, nu, q) + 1);
        }
        if (T.active) {
            const uint32_t y = T.y0 + T.yl;
            T.bit = (par + (int)y + (int)T.z + tl) & 1;
            Q Vlow{0.0f, 0.0f, 0.0f, 0.0f};
            const Q V = staple_tile<MU, MEASURE>(T, lds, ssz, carry, Vlow);
            const uint32_t h = hidx(g, T.xh, y, T.z, T.t);
            Q Un;
            if (OR) {
                const v4f u = cls_ptr(T.links, g.vh, MU, par)[h];
                const Q Uold = toq(u);
                Un = overrelax_link(V, Uold);
            } else {
                const uint32_t site = 2u * h + (uint32_t)T.bit;
                Un = heatbath_link(V, Rp.beta, site, sweep, word2((uint32_t)MU, TAG_TRIAL, Rp.replica),
                                   k0, k1);
            }
            gv4f *dst = (gv4f *)(reinterpret_cast<char *>(Rp.links) +
                                 (size_t)(MU * 2 + par) * g.vh * 16u) + h;
            const v4f w = {Un.w, Un.x, Un.y, Un.z};
            __builtin_nontemporal_store(w, dst);
            if (MEASURE) macc += (double)retr(Un, Vlow);
        }
        if (!more) break;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int nu = k >> 1, q = k & 1;
            if (carried(MU, nu, q) && T.active)  // own link of plane tl, needed one step on
                carry[nu == 3 ? 1 : 0] =
                    toq(lds[slot_of<MU>(nu, q, tl) * ssz + (T.yl + 1) * T.hx + T.xh]);
        }
        __syncthreads();  // every read of the planes about to be replaced is done
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int nu = k >> 1, q = k & 1;
            if (res_n(MU, nu, q) == 0) continue;
            store_plane(T, lds, ssz, slot_of<MU>(nu, q, tl + res_hi(MU, nu, q) + 1), pre[k]);
        }
        __syncthreads();
    }
    if (MEASURE) block_accumulate(macc, Rp.acc, ACC_PLAQ, b);
}

namespace {

template <int MU, bool OR>
void launch_march_mu(const Ens &e, int par, uint64_t seed, bool measure, const MarchShape &m,
                     int rev, hipStream_t stream)
{
    const size_t lds = (size_t)res_slots(MU) * m.slot_elems * sizeof(v4f);
    const dim3 grid(m.nunits), block(m.block);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (measure)
        hipLaunchKernelGGL((march_kernel<MU, true, OR>), grid, block, lds, stream, e.reps, par, k0,
                           k1, m.R, m.T, m.ntile, m.nunits, m.per, rev);
    else
        hipLaunchKernelGGL((march_kernel<MU, false, OR>), grid, block, lds, stream, e.reps, par, k0,
                           k1, m.R, m.T, m.ntile, m.nunits, m.per, rev);
}

}  // namespace

bool march_shape(const int32_t dims[4], uint32_t R, uint32_t T, MarchShape *m)
{
    const uint32_t hx = (uint32_t)dims[0] / 2u, ny = (uint32_t)dims[1];
    if (R == 0 || T == 0 || ny % R || (uint32_t)dims[3] % T) return false;
    const uint32_t threads = hx * R;
    if (threads > 256u || 2u * hx > threads) return false;
    const uint32_t slot_elems = (R + 2u) * hx;
    if ((size_t)11 * slot_elems * 16u > 64u * 1024u) return false;  // LDS of the largest plan
    m->R = R;
    m->T = T;
    m->block = (threads + 63u) / 64u * 64u;
    m->ntile = ny / R;
    m->nunits = m->ntile * (uint32_t)dims[2] * ((uint32_t)dims[3] / T);
    m->per = m->nunits % 8u == 0u ? m->nunits / 8u : 0u;
    m->slot_elems = slot_elems;
    return true;
}

hipError_t launch_pass_march(const Ens &e, int mu, int par, uint64_t seed, bool measure, bool orx,
                             const MarchShape &m, int rev, hipStream_t stream)
{
    switch (mu * 2 + (orx ? 1 : 0)) {
    case 0: launch_march_mu<0, false>(e, par, seed, measure, m, rev, stream); break;
    case 1: launch_march_mu<0, true>(e, par, seed, measure, m, rev, stream); break;
    case 2: launch_march_mu<1, false>(e, par, seed, measure, m, rev, stream); break;
    case 3: launch_march_mu<1, true>(e, par, seed, measure, m, rev, stream); break;
    case 4: launch_march_mu<2, false>(e, par, seed, measure, m, rev, stream); break;
    case 5: launch_march_mu<2, true>(e, par, seed, measure, m, rev, stream); break;
    case 6: launch_march_mu<3, false>(e, par, seed, measure, m, rev, stream); break;
    default: launch_march_mu<3, true>(e, par, seed, measure, m, rev, stream); break;
    }
    return hipGetLastError();
}

}  // namespace su2rt
