// su3_kernels.hip -- gfx950 kernels of the SU(3) pure-gauge heat bath.
//
// Each link update is a Cabibbo-Marinari step (Phys. Lett. B 119 (1982) 387):
// U_mu(s) is multiplied from the left by SU(2) matrices embedded in the row
// pairs (0,1), (1,2), (0,2).  For pair (i,j), with W = U A (A the six-staple
// sum of Sec. 2 of Cardoso & Bicudo, "Lattice SU(2) on GPU's") the weight
// exp[(beta/3) Re Tr(R W)] depends on the 2x2 block of W only through its
// quaternion part a, so the SU(2) heat bath of Sec. 2 (k = |a|,
// a0 ~ sqrt(1-a0^2) exp(alpha a0), X (a/k)^+) draws the subgroup element with
// alpha = (2 beta / 3) k.  The sampler, the Philox generator and the even/odd
// traversal are those of the SU(2) pass.
//
// Links keep rows 0 and 1 (12 floats in three float4 planes per (mu, parity)
// class); row 2 = conj(row0 x row1) is rebuilt in registers on every load, and
// products of SU(3) matrices compute two rows and complete the third the same
// way.  Sums are FP64 per workgroup and 64-bit fixed point across workgroups.
#include "su2_kcommon.h"
#include "su3_internal.h"

using namespace su2dev;
using su2rt::block_accumulate;
using su2rt::kBuckets;
using su2rt::from_fixed;
using su2rt::logical_block;
using su2rt::take_total;

namespace su3rt {

namespace {

constexpr uint32_t TAG_SU3_SUB = 7;  // subgroup g draws with Philox tag 7 + g
constexpr uint32_t TAG_SU3_HOT = 10;

// The lattice of replica blockIdx.z of a batch (uniform: scalar arithmetic).
__device__ __forceinline__ Lat3 rep3(const Lat3 &L0)
{
    Lat3 L = L0;
    const uint32_t r = blockIdx.z;
    const size_t off = (size_t)r * L0.scratch_stride;
    L.links = L0.links + (size_t)r * L0.link_stride;
    L.acc = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(L0.acc) + off);
    L.results = reinterpret_cast<double *>(reinterpret_cast<char *>(L0.results) + off);
    L.hist = reinterpret_cast<double *>(reinterpret_cast<char *>(L0.hist) + off);
    L.ctr = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(L0.ctr) + off);
    if (L0.betas) L.beta = L0.betas[r];
    L.replica = L0.replica + r;
    return L;
}

// ----------------------------------------------------------- complex algebra
struct Cx {
    float r, i;
};

// acc + a b
__device__ __forceinline__ Cx madd(Cx acc, Cx a, Cx b)
{
    return Cx{fmaf(a.r, b.r, fmaf(-a.i, b.i, acc.r)), fmaf(a.r, b.i, fmaf(a.i, b.r, acc.i))};
}
// acc + a conj(b)
__device__ __forceinline__ Cx madd_cb(Cx acc, Cx a, Cx b)
{
    return Cx{fmaf(a.r, b.r, fmaf(a.i, b.i, acc.r)), fmaf(a.i, b.r, fmaf(-a.r, b.i, acc.i))};
}
// acc + conj(a) b
__device__ __forceinline__ Cx madd_ca(Cx acc, Cx a, Cx b)
{
    return Cx{fmaf(a.r, b.r, fmaf(a.i, b.i, acc.r)), fmaf(a.r, b.i, fmaf(-a.i, b.r, acc.i))};
}
// conj(x1 y2 - x2 y1)
__device__ __forceinline__ Cx cross_conj(Cx x1, Cx y2, Cx x2, Cx y1)
{
    return Cx{fmaf(x1.r, y2.r, fmaf(-x1.i, y2.i, fmaf(-x2.r, y1.r, x2.i * y1.i))),
              fmaf(-x1.r, y2.i, fmaf(-x1.i, y2.r, fmaf(x2.r, y1.i, x2.i * y1.r)))};
}

struct M3 {
    Cx e[3][3];
};

// row 2 = conj(row0 x row1): the third row of an SU(3) matrix
__device__ __forceinline__ void complete(M3 &u)
{
    const Cx *a = u.e[0], *b = u.e[1];
    u.e[2][0] = cross_conj(a[1], b[2], a[2], b[1]);
    u.e[2][1] = cross_conj(a[2], b[0], a[0], b[2]);
    u.e[2][2] = cross_conj(a[0], b[1], a[1], b[0]);
}

// rows 0, 1 of a b^+
__device__ __forceinline__ void rows_nd(const M3 &a, const M3 &b, M3 &c)
{
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Cx t{0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < 3; ++k) t = madd_cb(t, a.e[r][k], b.e[q][k]);
            c.e[r][q] = t;
        }
}
// rows 0, 1 of a b
__device__ __forceinline__ void rows_nn(const M3 &a, const M3 &b, M3 &c)
{
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Cx t{0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < 3; ++k) t = madd(t, a.e[r][k], b.e[k][q]);
            c.e[r][q] = t;
        }
}
// rows 0, 1 of a^+ b
__device__ __forceinline__ void rows_dn(const M3 &a, const M3 &b, M3 &c)
{
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Cx t{0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < 3; ++k) t = madd_ca(t, a.e[k][r], b.e[k][q]);
            c.e[r][q] = t;
        }
}
// all rows of a b (b need not be unitary)
__device__ __forceinline__ M3 mul_full(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Cx t{0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < 3; ++k) t = madd(t, a.e[r][k], b.e[k][q]);
            c.e[r][q] = t;
        }
    return c;
}
__device__ __forceinline__ void add_to(M3 &a, const M3 &b)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) a.e[r][q] = Cx{a.e[r][q].r + b.e[r][q].r, a.e[r][q].i + b.e[r][q].i};
}
__device__ __forceinline__ M3 zero3()
{
    M3 z;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) z.e[r][q] = Cx{0.0f, 0.0f};
    return z;
}
// Re Tr(a b)
__device__ __forceinline__ float retr_mul(const M3 &a, const M3 &b)
{
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            s = fmaf(a.e[r][k].r, b.e[k][r].r, fmaf(-a.e[r][k].i, b.e[k][r].i, s));
    return s;
}

// ----------------------------------------------------------------- storage
// One (mu, parity) class: three planes of V/2 float4 at uniform addresses in
// the global address space; a load is a 16-byte access with a scalar base and
// a 32-bit vector offset (V/2 < 2^28 keeps h * 16 in 32 bits).
typedef __attribute__((address_space(1))) const char gchar;
typedef __attribute__((address_space(1))) char gchar_w;
struct __attribute__((aligned(16))) F4 {
    float x, y, z, w;
};
typedef __attribute__((address_space(1))) const F4 gf4;
typedef __attribute__((address_space(1))) F4 gf4_w;

struct Cls {
    gchar *p0, *p1, *p2;
};

__device__ __forceinline__ Cls cls(const float4 *links, uint32_t vh, int mu, int par)
{
    gchar *b = (gchar *)links + (size_t)((mu * 2 + par) * 3) * vh * 16u;
    return Cls{b, b + (size_t)vh * 16u, b + (size_t)vh * 32u};
}

// rows 0, 1 from the planes, row 2 completed (dropped by the compiler when unused)
__device__ __forceinline__ M3 ld3(const Cls &c, uint32_t h)
{
    const uint32_t off = h * 16u;
    gf4 *a = (gf4 *)(c.p0 + off), *b = (gf4 *)(c.p1 + off), *d = (gf4 *)(c.p2 + off);
    M3 u;
    u.e[0][0] = Cx{a->x, a->y};
    u.e[0][1] = Cx{a->z, a->w};
    u.e[0][2] = Cx{b->x, b->y};
    u.e[1][0] = Cx{b->z, b->w};
    u.e[1][1] = Cx{d->x, d->y};
    u.e[1][2] = Cx{d->z, d->w};
    complete(u);
    return u;
}

// The two stored rows of a link as loaded (three 16-byte loads), and the
// matrix they give (row 2 completed): ld3 split in two, so that a group of
// loads can be issued before any of their arithmetic.
struct Raw3 {
    F4 a, b, d;
};
__device__ __forceinline__ Raw3 raw3(const Cls &c, uint32_t h)
{
    const uint32_t off = h * 16u;
    gf4 *pa = (gf4 *)(c.p0 + off), *pb = (gf4 *)(c.p1 + off), *pd = (gf4 *)(c.p2 + off);
    Raw3 r;
    r.a.x = pa->x; r.a.y = pa->y; r.a.z = pa->z; r.a.w = pa->w;
    r.b.x = pb->x; r.b.y = pb->y; r.b.z = pb->z; r.b.w = pb->w;
    r.d.x = pd->x; r.d.y = pd->y; r.d.z = pd->z; r.d.w = pd->w;
    return r;
}
__device__ __forceinline__ M3 m3_of(const Raw3 &r)
{
    M3 u;
    u.e[0][0] = Cx{r.a.x, r.a.y};
    u.e[0][1] = Cx{r.a.z, r.a.w};
    u.e[0][2] = Cx{r.b.x, r.b.y};
    u.e[1][0] = Cx{r.b.z, r.b.w};
    u.e[1][1] = Cx{r.d.x, r.d.y};
    u.e[1][2] = Cx{r.d.z, r.d.w};
    complete(u);
    return u;
}

__device__ __forceinline__ void st3(float4 *links, uint32_t vh, int mu, int par, uint32_t h,
                                    const M3 &u)
{
    gchar_w *b = (gchar_w *)links + (size_t)((mu * 2 + par) * 3) * vh * 16u + h * 16u;
    gf4_w *p0 = (gf4_w *)b, *p1 = (gf4_w *)(b + (size_t)vh * 16u), *p2 = (gf4_w *)(b + (size_t)vh * 32u);
    p0->x = u.e[0][0].r;
    p0->y = u.e[0][0].i;
    p0->z = u.e[0][1].r;
    p0->w = u.e[0][1].i;
    p1->x = u.e[0][2].r;
    p1->y = u.e[0][2].i;
    p1->z = u.e[1][0].r;
    p1->w = u.e[1][0].i;
    p2->x = u.e[1][1].r;
    p2->y = u.e[1][1].i;
    p2->z = u.e[1][2].r;
    p2->w = u.e[1][2].i;
}

// The updated class is read once and written once per pass and by no other
// site of it: its loads and stores carry the nontemporal hint, which keeps the
// neighbour classes (read by up to six sites each) resident in the L2.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4f gv4;
typedef __attribute__((address_space(1))) const v4f gv4c;

__device__ __forceinline__ M3 ld3_stream(const Cls &c, uint32_t h)
{
    const uint32_t off = h * 16u;
    const v4f a = __builtin_nontemporal_load((gv4c *)(c.p0 + off));
    const v4f b = __builtin_nontemporal_load((gv4c *)(c.p1 + off));
    const v4f d = __builtin_nontemporal_load((gv4c *)(c.p2 + off));
    M3 u;
    u.e[0][0] = Cx{a.x, a.y};
    u.e[0][1] = Cx{a.z, a.w};
    u.e[0][2] = Cx{b.x, b.y};
    u.e[1][0] = Cx{b.z, b.w};
    u.e[1][1] = Cx{d.x, d.y};
    u.e[1][2] = Cx{d.z, d.w};
    complete(u);
    return u;
}

__device__ __forceinline__ void st3_stream(float4 *links, uint32_t vh, int mu, int par, uint32_t h,
                                           const M3 &u)
{
    gchar_w *b = (gchar_w *)links + (size_t)((mu * 2 + par) * 3) * vh * 16u + h * 16u;
    const v4f x0 = {u.e[0][0].r, u.e[0][0].i, u.e[0][1].r, u.e[0][1].i};
    const v4f x1 = {u.e[0][2].r, u.e[0][2].i, u.e[1][0].r, u.e[1][0].i};
    const v4f x2 = {u.e[1][1].r, u.e[1][1].i, u.e[1][2].r, u.e[1][2].i};
    __builtin_nontemporal_store(x0, (gv4 *)b);
    __builtin_nontemporal_store(x1, (gv4 *)(b + (size_t)vh * 16u));
    __builtin_nontemporal_store(x2, (gv4 *)(b + (size_t)vh * 32u));
}

// Rows 0, 1 orthonormalised (Gram-Schmidt in FP32); row 2 stays implied.
__device__ __forceinline__ void gram_schmidt(M3 &u)
{
    float n0 = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) n0 = fmaf(u.e[0][c].r, u.e[0][c].r, fmaf(u.e[0][c].i, u.e[0][c].i, n0));
    const float i0 = hw_rsq(n0);
#pragma unroll
    for (int c = 0; c < 3; ++c) u.e[0][c] = Cx{u.e[0][c].r * i0, u.e[0][c].i * i0};
    Cx p{0.0f, 0.0f};  // <row0, row1>
#pragma unroll
    for (int c = 0; c < 3; ++c) p = madd_ca(p, u.e[0][c], u.e[1][c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Cx q = madd(Cx{0.0f, 0.0f}, p, u.e[0][c]);
        u.e[1][c] = Cx{u.e[1][c].r - q.r, u.e[1][c].i - q.i};
    }
    float n1 = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) n1 = fmaf(u.e[1][c].r, u.e[1][c].r, fmaf(u.e[1][c].i, u.e[1][c].i, n1));
    const float i1 = hw_rsq(n1);
#pragma unroll
    for (int c = 0; c < 3; ++c) u.e[1][c] = Cx{u.e[1][c].r * i1, u.e[1][c].i * i1};
}

// ------------------------------------------------------------ subgroup step
// Quaternion part a of the (I, J) block of W: the block is M(a) + i M(c) with
// M(a) = a0 + i a.sigma, and Re Tr(r w) for r in SU(2) only sees M(a).
template <int I, int J>
__device__ __forceinline__ Q block_quaternion(const M3 &W)
{
    return Q{0.5f * (W.e[I][I].r + W.e[J][J].r), 0.5f * (W.e[I][J].i + W.e[J][I].i),
             0.5f * (W.e[I][J].r - W.e[J][I].r), 0.5f * (W.e[I][I].i - W.e[J][J].i)};
}

// Rows I, J of U (and of W, when it is used again) multiplied from the left by
// M(r) = [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]].
template <int I, int J, bool UPDATE_W>
__device__ __forceinline__ void rotate(M3 &U, M3 &W, const Q &r)
{
    const Cx r00{r.w, r.z}, r01{r.y, r.x}, r10{-r.y, r.x}, r11{r.w, -r.z};
    const Cx zero{0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Cx ui = U.e[I][c], uj = U.e[J][c];
        U.e[I][c] = madd(madd(zero, r00, ui), r01, uj);
        U.e[J][c] = madd(madd(zero, r10, ui), r11, uj);
        if (UPDATE_W) {
            const Cx wi = W.e[I][c], wj = W.e[J][c];
            W.e[I][c] = madd(madd(zero, r00, wi), r01, wj);
            W.e[J][c] = madd(madd(zero, r10, wi), r11, wj);
        }
    }
}

// Heat-bath draw in the SU(2) subgroup of rows (I, J): r = X (a/|a|)^+ from the
// SU(2) sampler with beta -> 2 beta / 3.
template <int I, int J, bool UPDATE_W>
__device__ __forceinline__ void subgroup(M3 &U, M3 &W, float beta23, uint32_t site,
                                         uint32_t sweep, uint32_t w2, uint32_t k0, uint32_t k1)
{
    const Q r = heatbath_link(block_quaternion<I, J>(W), beta23, site, sweep, w2, k0, k1);
    rotate<I, J, UPDATE_W>(U, W, r);
}

// Microcanonical over-relaxation in the subgroup of rows (I, J) (Brown & Woch
// 1987; Creutz 1987): r = (v^+)^2 with v = a/|a| reflects the subgroup
// element about the one the staple prefers (v^+), so Re Tr(R W) is unchanged;
// |a| = 0 leaves the link alone.  No randoms.
template <int I, int J, bool UPDATE_W>
__device__ __forceinline__ void or_subgroup(M3 &U, M3 &W)
{
    const Q a = block_quaternion<I, J>(W);
    const float k2 = qdot(a, a);
    if (!(k2 > 0.0f)) return;
    const float ik = hw_rsq(k2);
    const Q vd{a.w * ik, -a.x * ik, -a.y * ik, -a.z * ik};
    rotate<I, J, UPDATE_W>(U, W, qmul(vd, vd));
}

// ------------------------------------------------------------------ pass
// Update of U_MU at half-site gid (pass order) of parity par.  With MEASURE
// returns Re Tr(U'_MU A_low) / 3, A_low the staples with nu < MU.
template <int MU, bool MEASURE, bool OR>
__device__ __forceinline__ float update_site3(const Lat3 &L, uint32_t gid, int par,
                                              uint32_t sweep, uint32_t k0, uint32_t k1)
{
    const Geom &g = L.g;
    const int opp = par ^ 1;
    const PassSite s = pass_site(g, gid, par);
    const Deltas d = neighbour_deltas(g, s);
    const uint32_t h = s.h;
    const Cls Umu_o = cls(L.links, g.vh, MU, opp);
    M3 A = zero3(), Alow = zero3();
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU) continue;
        const Cls Unu_p = cls(L.links, g.vh, nu, par);
        const Cls Unu_o = cls(L.links, g.vh, nu, opp);
        M3 T, S;
        // The 18 loads of the plane's six links are issued before any of its
        // products (the scheduling barrier keeps them together) instead of
        // trickling out between them: 167 instead of 156 VGPRs, the same 3
        // waves per SIMD, 243-245 instead of 252-255 us per pass at 48^4.
        Raw3 r[6];
        r[0] = raw3(Unu_o, h + d.p[MU]);
        r[1] = raw3(Umu_o, h + d.p[nu]);
        r[2] = raw3(Unu_p, h);
        r[3] = raw3(Umu_o, h + d.m[nu]);
        r[4] = raw3(Unu_p, h + d.p[MU] + d.m[nu]);
        r[5] = raw3(Unu_o, h + d.m[nu]);
        __builtin_amdgcn_sched_barrier(0);
        // forward: U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+
        {
            const M3 a = m3_of(r[0]);
            const M3 b = m3_of(r[1]);
            rows_nd(a, b, T);
            const M3 c = m3_of(r[2]);
            rows_nd(T, c, S);
            complete(S);
            add_to(A, S);
            if (MEASURE && nu < MU) add_to(Alow, S);
        }
        // backward: U_nu(s+mu-nu)^+ U_mu(s-nu)^+ U_nu(s-nu) = (E D)^+ F
        {
            const M3 e = m3_of(r[3]);
            const M3 dd = m3_of(r[4]);
            rows_nn(e, dd, T);
            complete(T);
            const M3 f = m3_of(r[5]);
            rows_dn(T, f, S);
            complete(S);
            add_to(A, S);
            if (MEASURE && nu < MU) add_to(Alow, S);
        }
    }
    M3 U = ld3_stream(cls(L.links, g.vh, MU, par), h);
    M3 W = mul_full(U, A);
    if (OR) {
        or_subgroup<0, 1, true>(U, W);
        or_subgroup<1, 2, true>(U, W);
        or_subgroup<0, 2, false>(U, W);
    } else {
        const uint32_t site = 2u * h + (uint32_t)(s.x & 1);
        const float beta23 = L.beta * (2.0f / 3.0f);
        const uint32_t w2 = word2((uint32_t)MU, TAG_SU3_SUB, L.replica);
        subgroup<0, 1, true>(U, W, beta23, site, sweep, w2, k0, k1);
        subgroup<1, 2, true>(U, W, beta23, site, sweep, w2 + (1u << 2), k0, k1);
        subgroup<0, 2, false>(U, W, beta23, site, sweep, w2 + (2u << 2), k0, k1);
    }
    // The rotations of the (1,2) and (0,2) subgroups mix the rebuilt row 2 into
    // the stored rows, so an FP32 deviation from unitarity would be fed back
    // and grow from update to update; re-orthonormalising the stored rows (a
    // no-op in exact arithmetic) keeps every link unitary to FP32 rounding.
    gram_schmidt(U);
    complete(U);
    st3_stream(L.links, g.vh, MU, par, h, U);
    return MEASURE ? retr_mul(U, Alow) * (1.0f / 3.0f) : 0.0f;
}

template <int MU, bool MEASURE, bool OR>
__global__ __launch_bounds__(256) void su3_pass_kernel(Lat3 L0, int par, uint32_t k0,
                                                       uint32_t k1, uint32_t nblocks, int remap,
                                                       int reverse)
{
    const Lat3 L = rep3(L0);
    const uint32_t blk = logical_block(blockIdx.x, nblocks, remap, reverse);
    const uint32_t gid = blk * blockDim.x + threadIdx.x;
    float meas = 0.0f;
    if (gid < L.g.vh) {
        // the sweep index lives on the device (uniform: a scalar load through
        // the constant address space), so captured sweeps replay correctly
        const uint32_t sweep = *(const __attribute__((address_space(4))) uint32_t *)L.ctr;
        meas = update_site3<MU, MEASURE, OR>(L, gid, par, sweep, k0, k1);
    }
    if (MEASURE) block_accumulate((double)meas, L.acc, A3_PLAQ, blockIdx.x);
}

// ------------------------------------------------------------ observables
// Re Tr(U_mu(s) U_nu(s+mu) U_mu(s+nu)^+ U_nu(s)^+) / 3 over the six planes of
// every site, as Re sum_ab P_ab conj(Q_ab) with P = U_mu(s) U_nu(s+mu) and
// Q = U_nu(s) U_mu(s+nu).  grid (blocks over V/2, parity, replica)
__global__ __launch_bounds__(256) void su3_plaquette_kernel(Lat3 L0)
{
    const Lat3 L = rep3(L0);
    const Geom &g = L.g;
    const int par = blockIdx.y, opp = par ^ 1;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (gid < g.vh) {
        const PassSite s = pass_site(g, gid, par);
        const Deltas d = neighbour_deltas(g, s);
#pragma unroll
        for (int mu = 1; mu < 4; ++mu)
#pragma unroll
            for (int nu = 0; nu < mu; ++nu) {
                M3 P, Qm;
                rows_nn(ld3(cls(L.links, g.vh, mu, par), s.h),
                        ld3(cls(L.links, g.vh, nu, opp), s.h + d.p[mu]), P);
                complete(P);
                rows_nn(ld3(cls(L.links, g.vh, nu, par), s.h),
                        ld3(cls(L.links, g.vh, mu, opp), s.h + d.p[nu]), Qm);
                complete(Qm);
                float t = 0.0f;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        t = fmaf(P.e[r][q].r, Qm.e[r][q].r, fmaf(P.e[r][q].i, Qm.e[r][q].i, t));
                v += (double)t * (1.0 / 3.0);
            }
    }
    block_accumulate(v, L.acc, A3_PLAQ, blockIdx.x + blockIdx.y * gridDim.x);
}

// Tr L / 3, L = U_3(x, 0) U_3(x, 1) ... U_3(x, Nt-1), one thread per spatial site.
__global__ __launch_bounds__(256) void su3_polyakov_kernel(Lat3 L0)
{
    const Lat3 L = rep3(L0);
    const Geom &g = L.g;
    const uint32_t vs = (uint32_t)g.nx * (uint32_t)g.ny * (uint32_t)g.nz;
    const uint32_t xs = blockIdx.x * blockDim.x + threadIdx.x;
    double re = 0.0, im = 0.0, ab = 0.0;
    if (xs < vs) {
        const int x = (int)(xs % (uint32_t)g.nx), y = (int)((xs / (uint32_t)g.nx) % (uint32_t)g.ny);
        const int z = (int)(xs / ((uint32_t)g.nx * (uint32_t)g.ny));
        const int p0 = (x + y + z) & 1;
        M3 P = ld3(cls(L.links, g.vh, 3, p0), xs >> 1);
        for (int t = 1; t < g.nt; ++t) {
            const uint32_t sidx = xs + vs * (uint32_t)t;
            M3 N;
            rows_nn(P, ld3(cls(L.links, g.vh, 3, (p0 + t) & 1), sidx >> 1), N);
            complete(N);
            P = N;
        }
        const float tr_r = (P.e[0][0].r + P.e[1][1].r + P.e[2][2].r) * (1.0f / 3.0f);
        const float tr_i = (P.e[0][0].i + P.e[1][1].i + P.e[2][2].i) * (1.0f / 3.0f);
        re = tr_r;
        im = tr_i;
        ab = sqrt((double)tr_r * tr_r + (double)tr_i * tr_i);
    }
    block_accumulate(re, L.acc, A3_POLY_RE, blockIdx.x);
    block_accumulate(im, L.acc, A3_POLY_IM, blockIdx.x);
    block_accumulate(ab, L.acc, A3_POLY_ABS, blockIdx.x);
}

__global__ __launch_bounds__(kBuckets) void su3_finish_kernel(Lat3 L0, int flags, int row)
{
    const Lat3 L = rep3(L0);
    const Geom &g = L.g;
    if (flags & 1) {
        const unsigned long long t = take_total(L.acc, A3_PLAQ);
        if (threadIdx.x == 0) {
            const double p = from_fixed(t) / (12.0 * (double)g.vh);
            L.results[R3_PLAQ] = p;
            if (flags & 4) {
                // flags 16: the row comes from the device row counter (captured sweeps)
                const uint32_t r = (flags & 16) ? L.ctr[1]++ : (uint32_t)row;
                L.hist[r] = p;
            }
        }
    }
    if ((flags & 8) && threadIdx.x == 0) L.ctr[0] += 1u;  // the sweep is complete
    if (flags & 2) {
        const unsigned long long tr = take_total(L.acc, A3_POLY_RE);
        const unsigned long long ti = take_total(L.acc, A3_POLY_IM);
        const unsigned long long ta = take_total(L.acc, A3_POLY_ABS);
        if (threadIdx.x == 0) {
            const double vs = (double)g.nx * g.ny * g.nz;
            L.results[R3_POLY_RE] = from_fixed(tr) / vs;
            L.results[R3_POLY_IM] = from_fixed(ti) / vs;
            L.results[R3_POLY_ABS] = from_fixed(ta) / vs;
        }
    }
}

// ------------------------------------------------------- init / reunitarise
// grid (blocks over V/2, 8 = mu * 2 + parity, replica)
__global__ __launch_bounds__(256) void su3_reunit_kernel(Lat3 L0)
{
    const Lat3 L = rep3(L0);
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= L.g.vh) return;
    const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
    M3 u = ld3(cls(L.links, L.g.vh, mu, par), h);
    gram_schmidt(u);
    st3(L.links, L.g.vh, mu, par, h, u);
}

// Haar SU(3): rows 0, 1 of complex Gaussians (Box-Muller on the Philox blocks
// (site, 0, mu | 10<<2 | replica<<6, d), d = 0, 1, 2) by Gram-Schmidt; row 2
// is implied.  grid (blocks over V/2, 8 = mu * 2 + parity, replica)
__global__ __launch_bounds__(256) void su3_init_kernel(Lat3 L0, int start, uint32_t k0, uint32_t k1)
{
    const Lat3 L = rep3(L0);
    const Geom &g = L.g;
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= g.vh) return;
    const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
    M3 u = zero3();
    u.e[0][0] = Cx{1.0f, 0.0f};
    u.e[1][1] = Cx{1.0f, 0.0f};
    if (start) {
        const uint32_t xh = h % g.hx, r = h / g.hx;
        const int y = (int)(r % (uint32_t)g.ny), z = (int)((r / (uint32_t)g.ny) % (uint32_t)g.nz);
        const int t = (int)(r / ((uint32_t)g.ny * (uint32_t)g.nz));
        const int x = 2 * (int)xh + ((par + y + z + t) & 1);
        const uint32_t site = 2u * h + (uint32_t)(x & 1);
        const uint32_t w2 = word2((uint32_t)mu, TAG_SU3_HOT, L.replica);
        float gs[12];
#pragma unroll
        for (uint32_t dr = 0; dr < 3; ++dr) {
            const U4 w = philox(site, 0u, w2, dr, k0, k1);
            const float ra = hw_sqrt(-2.0f * kLn2 * hw_log2(u01(w.a)));
            const float rb = hw_sqrt(-2.0f * kLn2 * hw_log2(u01(w.c)));
            const float pa = u01(w.b), pb = u01(w.d);
            gs[4 * dr + 0] = ra * hw_cos_rev(pa);
            gs[4 * dr + 1] = ra * hw_sin_rev(pa);
            gs[4 * dr + 2] = rb * hw_cos_rev(pb);
            gs[4 * dr + 3] = rb * hw_sin_rev(pb);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u.e[0][c] = Cx{gs[2 * c], gs[2 * c + 1]};
            u.e[1][c] = Cx{gs[6 + 2 * c], gs[6 + 2 * c + 1]};
        }
        gram_schmidt(u);
    }
    st3(L.links, g.vh, mu, par, h, u);
}

uint32_t nblk(uint64_t n, int b) { return (uint32_t)((n + (uint64_t)b - 1) / (uint64_t)b); }

template <int MU, bool OR>
void launch_pass_mu(const Lat3 &L, int par, uint32_t k0, uint32_t k1,
                    bool measure, const Launch3 &cfg, hipStream_t s)
{
    const uint32_t nb = nblk(L.g.vh, cfg.block);
    const int reverse = (cfg.snake && par == 1) ? 1 : 0;
    const int remap = cfg.remap ? 1 : 0;
    if (measure)
        hipLaunchKernelGGL((su3_pass_kernel<MU, true, OR>), dim3(nb, 1, L.nrep), dim3(cfg.block), 0, s, L,
                           par, k0, k1, nb, remap, reverse);
    else
        hipLaunchKernelGGL((su3_pass_kernel<MU, false, OR>), dim3(nb, 1, L.nrep), dim3(cfg.block), 0, s, L,
                           par, k0, k1, nb, remap, reverse);
}

template <bool OR>
void launch_pass_or(const Lat3 &L, int mu, int par, uint32_t k0, uint32_t k1,
                    bool measure, const Launch3 &cfg, hipStream_t s)
{
    switch (mu) {
    case 0: launch_pass_mu<0, OR>(L, par, k0, k1, measure, cfg, s); break;
    case 1: launch_pass_mu<1, OR>(L, par, k0, k1, measure, cfg, s); break;
    case 2: launch_pass_mu<2, OR>(L, par, k0, k1, measure, cfg, s); break;
    default: launch_pass_mu<3, OR>(L, par, k0, k1, measure, cfg, s); break;
    }
}

}  // namespace

hipError_t launch_su3_init(const Lat3 &L, int start, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(su3_init_kernel, dim3(nblk(L.g.vh, 256), 8, L.nrep), dim3(256), 0, s, L, start,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_su3_pass(const Lat3 &L, int mu, int par, uint64_t seed, bool measure,
                           const Launch3 &cfg, hipStream_t s, bool overrelax)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (overrelax)
        launch_pass_or<true>(L, mu, par, k0, k1, measure, cfg, s);
    else
        launch_pass_or<false>(L, mu, par, k0, k1, measure, cfg, s);
    return hipGetLastError();
}

hipError_t launch_su3_reunit(const Lat3 &L, hipStream_t s)
{
    hipLaunchKernelGGL(su3_reunit_kernel, dim3(nblk(L.g.vh, 256), 8, L.nrep), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_su3_plaquette(const Lat3 &L, hipStream_t s)
{
    hipLaunchKernelGGL(su3_plaquette_kernel, dim3(nblk(L.g.vh, 256), 2, L.nrep), dim3(256), 0, s,
                       L);
    return hipGetLastError();
}

hipError_t launch_su3_polyakov(const Lat3 &L, hipStream_t s)
{
    const uint64_t vs = (uint64_t)L.g.nx * L.g.ny * L.g.nz;
    hipLaunchKernelGGL(su3_polyakov_kernel, dim3(nblk(vs, 256), 1, L.nrep), dim3(256), 0, s, L);
    return hipGetLastError();
}

// grid (1, 1, replica)
__global__ void su3_set_counter_kernel(Lat3 L0, uint32_t value, int which)
{
    rep3(L0).ctr[which] = value;
}

hipError_t launch_su3_set_counter(const Lat3 &L, uint32_t value, int which, hipStream_t s)
{
    hipLaunchKernelGGL(su3_set_counter_kernel, dim3(1, 1, L.nrep), dim3(1), 0, s, L, value, which);
    return hipGetLastError();
}

hipError_t launch_su3_finish(const Lat3 &L, int flags, int row, hipStream_t s)
{
    hipLaunchKernelGGL(su3_finish_kernel, dim3(1, 1, L.nrep), dim3(kBuckets), 0, s, L, flags, row);
    return hipGetLastError();
}

}  // namespace su3rt
