// su3_internal.h -- host/device declarations of the SU(3) heat bath of libsu2
// (not part of the public C ABI).
#pragma once

#include "su2_internal.h"

namespace su3rt {

using su2dev::Geom;

// Links of an SU(3) lattice: 24 planes of V/2 float4, plane
// ((mu * 2 + parity) * 3 + c) holding float4 c of U_mu at every half-site of
// that parity.  Only rows 0 and 1 are stored (12 floats):
//   c = 0: (Re u00, Im u00, Re u01, Im u01)
//   c = 1: (Re u02, Im u02, Re u10, Im u10)
//   c = 2: (Re u11, Im u11, Re u12, Im u12)
// and row 2 = conj(row0 x row1) is rebuilt on every load.
constexpr int kPlanes3 = 24;
constexpr int kHist3 = 1024;  // device history rows per measured call chunk

struct Lat3 {
    Geom g;
    float4 *links;
    unsigned long long *acc;  // kNumAcc x kBuckets fixed-point accumulators
    double *results;          // kRes3 result slots
    double *hist;             // kHist3 plaquette history rows
    uint32_t *ctr;            // device counters: [0] sweep index, [1] history row of captured sweeps
    float beta;
    uint32_t replica;
    // Batches of replicas with the extents of g: every launch has grid z =
    // nrep, and replica r = blockIdx.z uses links + r * link_stride (float4),
    // the acc, results, hist and ctr of its own scratch (r * scratch_stride
    // bytes on), coupling betas[r] (device array; nullptr: beta) and Philox
    // replica id replica + r.  A single lattice is a batch of one.
    const float *betas;
    size_t link_stride;
    size_t scratch_stride;
    uint32_t nrep;
};

enum Acc3 { A3_PLAQ = 0, A3_POLY_RE = 1, A3_POLY_IM = 2, A3_POLY_ABS = 3 };
enum Res3 { R3_PLAQ = 0, R3_POLY_RE = 1, R3_POLY_IM = 2, R3_POLY_ABS = 3, kRes3 = 8 };

struct Launch3 {
    int block = 128;       // 128 beats 256 by 3-4 % with the grouped loads of the pass
    bool remap = true;     // XCD-aware workgroup -> tile mapping
    bool snake = true;     // odd-parity passes traverse backwards
};

hipError_t launch_su3_init(const Lat3 &L, int start, uint64_t seed, hipStream_t s);
// One heat-bath pass (direction mu, parity par), or with overrelax one
// microcanonical over-relaxation pass (no randoms); with measure, the plaquette
// terms of the passes' nu < mu staples are accumulated (odd passes of mu >= 1
// cover every plaquette of the end-of-sweep configuration once).
// The sweep index is read from L.ctr[0] on the device.
hipError_t launch_su3_pass(const Lat3 &L, int mu, int par, uint64_t seed, bool measure,
                           const Launch3 &cfg, hipStream_t s, bool overrelax = false);
hipError_t launch_su3_reunit(const Lat3 &L, hipStream_t s);
hipError_t launch_su3_plaquette(const Lat3 &L, hipStream_t s);
hipError_t launch_su3_polyakov(const Lat3 &L, hipStream_t s);
// Totals of the accumulators named by flags (1 plaquette, 2 Polyakov) into the
// result slots (the accumulators are reset); flags & 4: the plaquette also
// goes to hist[row] (flags & 16: to hist[ctr[1]++] instead); flags & 8: the
// sweep index ctr[0] advances by one.
hipError_t launch_su3_finish(const Lat3 &L, int flags, int row, hipStream_t s);
// ctr[which] = value (a kernel, so that it can sit in a captured graph).
hipError_t launch_su3_set_counter(const Lat3 &L, uint32_t value, int which, hipStream_t s);

}  // namespace su3rt

namespace su2rt {
// Host helpers of the SU(2) runtime reused by the SU(3) one.
int check_dims(const int32_t *dims);
su2dev::Geom make_geom(const int32_t *d, uint32_t lg_tz, uint32_t lg_tt);
bool geom_selfcheck(const su2dev::Geom &g);
int fail(int code, const std::string &msg);
}  // namespace su2rt
