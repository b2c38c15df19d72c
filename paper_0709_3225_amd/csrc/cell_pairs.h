// Shared machinery of the cell-pair kernels (forces, adjoint, virial
// gradient): the 27-cell neighbourhood table, LDS staging in the home cell's
// frame, the dot-product screen into accept words and the walk over the
// accepted bits. See forces.hip for the design.
#pragma once

#include "md_device.h"

namespace mdlj {
namespace {

constexpr int kTile = 1024;  // staged atoms per LDS pass of the neighbour export (16 KiB)

struct Neighbourhood {
    int pref[28];   // exclusive prefix of the 27 cell counts; pref[27] = total
    int first[27];  // first sorted slot of each neighbour cell
    float bx[27], by[27], bz[27];  // frame offset o - sh of each neighbour cell
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
    if (lane < 27) {
        nb.pref[lane] = incl - cnt;
        nb.first[lane] = first;
        nb.bx[lane] = bx;
        nb.by[lane] = by;
        nb.bz[lane] = bz;
    }
    if (lane == 26) nb.pref[27] = incl;
    __syncthreads();
}

// Stage neighbourhood atoms [t0, t0 + tn) into the tile, frame-translated.
// w carries the user index (ID_IN_W) or |x|^2 in the frame (for the screen).
// With WITH_VEC the matching entries of a per-atom vector (sorted
// order) are copied into vtile as well. Loads are issued four per lane before
// their LDS stores, so a wavefront waits on global memory about tn / 256
// times instead of tn / 64.
template <bool ID_IN_W, bool WITH_VEC = false>
__device__ __forceinline__ void stage_tile(const SimArgs& a, const Neighbourhood& nb, float4* tile,
                                           int t0, int tn, const float4* vec = nullptr,
                                           float4* vtile = nullptr) {
    constexpr int kBatch = 4;
    for (int t = threadIdx.x; t < tn; t += kWave * kBatch) {
        float4 q[kBatch], vq[kBatch];
        int kk[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int tt = t + u * kWave;
            const int g = t0 + (tt < tn ? tt : 0);
            int k = 0;  // largest k with pref[k] <= g
#pragma unroll
            for (int step = 16; step > 0; step >>= 1)
                if (k + step < 27 && nb.pref[k + step] <= g) k += step;
            kk[u] = k;
            const int slot = nb.first[k] + (g - nb.pref[k]);
            q[u] = a.pos0[slot];
            if (WITH_VEC) vq[u] = vec[slot];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int tt = t + u * kWave;
            if (tt < tn) {
                const int k = kk[u];
                const float x = q[u].x - nb.bx[k], y = q[u].y - nb.by[k], z = q[u].z - nb.bz[k];
                tile[tt] = make_float4(x, y, z, ID_IN_W ? q[u].w : x * x + y * y + z * z);
                if (WITH_VEC) vtile[tt] = vq[u];
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
        op(wb + k * cstep, live);
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
