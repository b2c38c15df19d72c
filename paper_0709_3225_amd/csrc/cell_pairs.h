// Shared machinery of the cell-pair kernels (forces, adjoint, virial
// gradient): the 27-cell neighbourhood table, LDS staging in the home cell's
// frame, the dot-product screen into accept words and the walk over the
// accepted bits. See forces.hip for the design.
#pragma once

#include "md_device.h"

namespace mdlj {
namespace {

constexpr int kTile = 1024;  // staged atoms per LDS pass of the neighbour export (16 KiB)

// The 27-cell neighbourhood of a home cell as runs of memory-contiguous cells
// that share one image shift ("segments"): the three cells of an x-row are
// consecutive in the sorted arrays unless the row wraps around the box in x,
// so an interior home cell has 9 segments and a cell on an x face 27 (one per
// cell). Segments list the cells in the order dx, dy, dz (dx fastest) and
// tile the neighbourhood index range [0, total) in that order.
struct Neighbourhood {
    int total;       // atoms in the 27 cells
    int home_pos;    // neighbourhood index of the home cell's first atom
    int home_first;  // its sorted slot
    int n_home;
    int nseg;
    int seg_pos[27];    // neighbourhood index of the segment's first atom
    int seg_first[27];  // its sorted slot
    int seg_len[27];
    float sx[27], sy[27], sz[27];  // frame offset o - sh of the segment's cells
};

// Fill the neighbourhood table of home cell c (lanes 0..26 one cell each).
__device__ __forceinline__ void load_neighbourhood(const SimArgs& a, int c, Neighbourhood& nb,
                                                   float& ox, float& oy, float& oz) {
    const int lane = threadIdx.x;
    const int nc = a.nc;
    const int ix = c % nc, iy = (c / nc) % nc, iz = c / (nc * nc);
    ox = ix * a.s;
    oy = iy * a.s;
    oz = iz * a.s;
    int cnt = 0, first = 0;
    float bx = ox, by = oy, bz = oz;
    if (lane < 27) {
        int jx = ix + lane % 3 - 1, jy = iy + (lane / 3) % 3 - 1, jz = iz + lane / 9 - 1;
        if (jx < 0) { jx += nc; bx = ox + a.box; } else if (jx >= nc) { jx -= nc; bx = ox - a.box; }
        if (jy < 0) { jy += nc; by = oy + a.box; } else if (jy >= nc) { jy -= nc; by = oy - a.box; }
        if (jz < 0) { jz += nc; bz = oz + a.box; } else if (jz >= nc) { jz -= nc; bz = oz - a.box; }
        const int cj = a.cbase + jx + nc * (jy + nc * jz);
        first = a.start[cj];
        cnt = a.start[cj + 1] - first;
    }
    const int incl = wave_incl_scan(cnt);
    const int pos = incl - cnt;
    const bool rows = ix >= 1 && ix <= nc - 2;  // uniform: x-rows are contiguous, unshifted in x
    const int row_end = __shfl(incl, lane + 2 < kWave ? lane + 2 : lane);
    if (rows) {
        if (lane < 27 && lane % 3 == 0) {
            const int r = lane / 3;
            nb.seg_pos[r] = pos;
            nb.seg_first[r] = first;
            nb.seg_len[r] = row_end - pos;
            nb.sx[r] = bx;
            nb.sy[r] = by;
            nb.sz[r] = bz;
        }
    } else if (lane < 27) {
        nb.seg_pos[lane] = pos;
        nb.seg_first[lane] = first;
        nb.seg_len[lane] = cnt;
        nb.sx[lane] = bx;
        nb.sy[lane] = by;
        nb.sz[lane] = bz;
    }
    if (lane == 13) {
        nb.home_pos = pos;
        nb.home_first = first;
        nb.n_home = cnt;
    }
    if (lane == 26) nb.total = incl;
    if (lane == 0) nb.nseg = rows ? 9 : 27;
    __syncthreads();
}

__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Stage neighbourhood atoms [t0, t0 + tn) into the tile, frame-translated.
// w carries the user index (ID_IN_W) or |x|^2 in the frame (for the screen).
// With WITH_VEC the matching entries of a per-atom vector (sorted order) are
// copied into vtile as well. A uniform cursor walks the segments in chunks of
// at most one wavefront; the segment table sits in lanes 0..nseg-1 and is read
// with readlane, and kBatch chunks have their loads in flight before the LDS
// stores, so an interior cell's neighbourhood costs one global round trip.
template <bool ID_IN_W, bool WITH_VEC = false>
__device__ __forceinline__ void stage_tile(const SimArgs& a, const Neighbourhood& nb, float4* tile,
                                           int t0, int tn, const float4* vec = nullptr,
                                           float4* vtile = nullptr) {
    constexpr int kBatch = WITH_VEC ? 5 : 9;  // chunks in flight (register budget)
    const int lane = threadIdx.x;
    const int nseg = nb.nseg;
    int s_pos = 0, s_first = 0, s_len = 0;
    float s_x = 0.f, s_y = 0.f, s_z = 0.f;
    if (lane < nseg) {
        s_pos = nb.seg_pos[lane];
        s_first = nb.seg_first[lane];
        s_len = nb.seg_len[lane];
        s_x = nb.sx[lane];
        s_y = nb.sy[lane];
        s_z = nb.sz[lane];
    }
    const int t1 = t0 + tn;
    int sg = 0;  // uniform cursor: segment sg, neighbourhood index g
    while (sg < nseg && lane_value(s_pos, sg) + lane_value(s_len, sg) <= t0) ++sg;
    int g = t0;
    while (g < t1 && sg < nseg) {
        float4 q[kBatch], vq[kBatch];
        int dst[kBatch], seg[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            dst[u] = -1;
            seg[u] = 0;
            int slot = 0;  // lanes without an atom load slot 0 (always valid) and store nothing
            if (g < t1 && sg < nseg) {
                const int p = lane_value(s_pos, sg), end = p + lane_value(s_len, sg);
                const int ce = min(min(g + kWave, end), t1);
                const int my = g + lane;
                if (my < ce) {
                    slot = lane_value(s_first, sg) + (my - p);
                    dst[u] = my - t0;
                }
                seg[u] = sg;
                g = ce;
                if (g >= end) ++sg;
            }
            q[u] = a.pos0[slot];
            if (WITH_VEC) vq[u] = vec[slot];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (dst[u] >= 0) {
                const float x = q[u].x - lane_value(s_x, seg[u]);
                const float y = q[u].y - lane_value(s_y, seg[u]);
                const float z = q[u].z - lane_value(s_z, seg[u]);
                tile[dst[u]] = make_float4(x, y, z, ID_IN_W ? q[u].w : x * x + y * y + z * z);
                if (WITH_VEC) vtile[dst[u]] = vq[u];
            }
        }
    }
}

// Cell-pair kernels. One wavefront per home cell; lane = (home atom h, slice s)
// with ns = floor(64 / home atoms) slices, so a cell of 15 atoms keeps 60
// lanes busy. The staged candidates are screened in spans of up to 128 per
// lane:
//  screen : lane (h, s) tests candidates s, s + ns, s + 2 ns, ... (slices
//           interleave, so every slice samples the whole neighbourhood and
//           the slices of one atom find similar numbers of partners) with
//           r^2 - |x_i|^2 = |x_j|^2 - 2 x_i.x_j (three FMAs) against a bound a
//           little above r_c^2, and shifts each verdict's sign bit into a
//           32-bit accept word (one v_alignbit). Lanes of one slice read the
//           same candidate, so every LDS read of the screen is a broadcast.
//  pairs  : the home atom's own bit is cleared; every lane walks the set bits
//           of its words, recomputes the exact displacement, keeps
//           r^2 < r_c^2 and applies the kernel's pair operation (for the force
//           kernel: the truncated, shifted LJ force of section 2).
// Slice partials are summed in slice order, so the result does not depend on
// timing.
constexpr int kWords = 4;              // accept words per lane per span
constexpr int kGroups = 32 * kWords;   // candidates per lane per span
constexpr int kMaxSlices = 16;
constexpr int kScreenUnroll = 4;
constexpr int kTilePad = kMaxSlices * (kScreenUnroll + 1);  // far-away entries after the staged atoms

// Screen of one span: word w, bit 31 - k holds the verdict on the lane's
// candidate 32 w + k, i.e. tile entry first + (32 w + k) * ns. groups is the
// largest candidate count of any slice (uniform); entries past the staged
// atoms are padding that never passes. NS > 0 fixes the stride at compile
// time (immediate LDS offsets); NS = 0 takes it from ns.
template <int NS>
__device__ __forceinline__ void screen_span(const float4* tile, int first, int ns_rt, int groups, float mx,
                                            float my, float mz, float thr_i, uint32_t (&wd)[kWords]) {
    const int ns = NS > 0 ? NS : ns_rt;
    const float4* cand = tile + first;
#pragma unroll
    for (int w = 0; w < kWords; ++w) {
        uint32_t bits = 0;
        const int n = min(32, groups - 32 * w);  // uniform
        if (n > 0) {
            for (int k0 = 0; k0 < n; k0 += kScreenUnroll) {
#pragma unroll
                for (int u = 0; u < kScreenUnroll; ++u) {
                    const float4 q = cand[(32 * w + k0 + u) * ns];
                    // negative iff accepted; its sign bit is shifted into the word
                    const float d = fmaf(mx, q.x, fmaf(my, q.y, fmaf(mz, q.z, q.w - thr_i)));
                    bits = __builtin_amdgcn_alignbit(bits, __float_as_uint(d), 31);
                }
            }
            const int done = (n + kScreenUnroll - 1) / kScreenUnroll * kScreenUnroll;
            if (done < 32) bits <<= (32 - done);
        }
        wd[w] = bits;
    }
}

// Walk the accepted bits of one span, calling op(byte_offset, live) once per
// iteration: byte_offset locates the accepted candidate relative to
// tile + first (and the same offset in any parallel tile); live is false for
// lanes that have spent their bits. The words rotate through four registers
// (never indexed, which would put them in scratch memory); an exhausted word
// is replaced by the next one without a branch.
template <class Op>
__device__ __forceinline__ void walk_bits(int ns, uint32_t m, uint32_t n1, uint32_t n2, uint32_t n3, Op& op) {
    const uint32_t cstep = static_cast<uint32_t>(ns) * sizeof(float4);  // bytes between candidates
    const uint32_t wstep = 32u * cstep;                                  // bytes between words
    uint32_t wb = 0;                                                     // byte offset of the word's candidate 0
    uint32_t left = __builtin_popcount(m) + __builtin_popcount(n1) + __builtin_popcount(n2) +
                    __builtin_popcount(n3);
    if (!__any(left != 0u)) return;
    do {
        const bool next = (m == 0u);
        m = next ? n1 : m;
        n1 = next ? n2 : n1;
        n2 = next ? n3 : n2;
        n3 = next ? 0u : n3;
        wb = next ? wb + wstep : wb;
        const bool live = m != 0u;
        const uint32_t k = live ? __builtin_clz(m) : 0u;
        m &= ~(0x80000000u >> k);
        left -= live ? 1u : 0u;
        // a spent lane keeps rotating (wb grows past its span): it reads its
        // span's first candidate instead, which is always staged
        op(live ? wb + k * cstep : 0u, live);
    } while (__any(left != 0u));
}

// Clear the screen bit of the home atom itself (tile index self_t) if it lies
// in this lane's span: span candidates are first + g * ns for g < groups.
__device__ __forceinline__ void clear_self(int self_t, int first, int ns, int groups, uint32_t (&wd)[kWords]) {
    const int off = self_t - first;
    if (off < 0 || off % ns != 0) return;
    const int g = off / ns;
    if (g >= groups) return;
    const uint32_t bit = 0x80000000u >> (g & 31);
    const int w = g >> 5;
    wd[0] &= (w == 0) ? ~bit : ~0u;
    wd[1] &= (w == 1) ? ~bit : ~0u;
    wd[2] &= (w == 2) ? ~bit : ~0u;
    wd[3] &= (w == 3) ? ~bit : ~0u;
}

}  // namespace
}  // namespace mdlj
