// Shared machinery of the cell-pair kernels (forces, adjoint, virial
// gradient): the 27-cell neighbourhood table, LDS staging in the home cell's
// frame, the dot-product screen into accept words and the walk over the
// accepted bits. See forces.hip for the design.
#pragma once

#include "md_device.h"

namespace mdlj {
namespace {


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
    float origin[3];    // home-cell origin
    int seg_pos[27];    // neighbourhood index of the segment's first atom
    int seg_first[27];  // its sorted slot
    int seg_len[27];
    float sx[27], sy[27], sz[27];  // frame offset o - sh of the segment's cells
};

// The same table while it is built, in registers: lane l < 27 first holds
// neighbour cell l (HoodLoads: its CSR range, still in flight), then segment l
// (HoodSegs). The uniform fields are the same in every lane.
struct HoodLoads {
    int first = 0, next = 0;  // start[cj], start[cj + 1]
    float bx = 0.f, by = 0.f, bz = 0.f;
    int cell = 0;  // the home cell
    bool rows = false;
};

// Origin of cell c (local index) in the box. The frame offsets o +- L are
// formed from this rounded product; contraction is off wherever they are
// computed, since fma(i, s, -L) is not the exact o - L the frame relies on.
__device__ __forceinline__ void cell_origin(const SimArgs& a, int c, float& ox, float& oy, float& oz) {
#pragma clang fp contract(off)
    const int nc = a.nc;
    ox = static_cast<float>(c % nc) * a.s;
    oy = static_cast<float>((c / nc) % nc) * a.s;
    oz = static_cast<float>(c / (nc * nc)) * a.s;
}

// Uniform facts are spread over lanes (meta: lane 0 total, 1 home_pos,
// 2 home_first, 3 n_home, 4 nseg; org: lanes 0..2 the home-cell origin) so
// that a table held across the pair loops costs vector registers, not scalar
// ones.
struct HoodSegs {
    int pos = 0, first = 0, len = 0;
    float x = 0.f, y = 0.f, z = 0.f;
    int meta = 0;
    float org = 0.f;
    __device__ __forceinline__ int total() const { return __builtin_amdgcn_readlane(meta, 0); }
    __device__ __forceinline__ int home_pos() const { return __builtin_amdgcn_readlane(meta, 1); }
    __device__ __forceinline__ int home_first() const { return __builtin_amdgcn_readlane(meta, 2); }
    __device__ __forceinline__ int n_home() const { return __builtin_amdgcn_readlane(meta, 3); }
    __device__ __forceinline__ int nseg() const { return __builtin_amdgcn_readlane(meta, 4); }
    __device__ __forceinline__ float origin(int d) const {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(org), d));
    }
};

// Issue the CSR loads of home cell c's 27 neighbours (lanes 0..26); nothing
// waits for them here.
__device__ __forceinline__ void hood_issue(const SimArgs& a, int c, HoodLoads& h) {
#pragma clang fp contract(off)
    const int lane = __lane_id();
    const int nc = a.nc;
    const int ix = c % nc, iy = (c / nc) % nc, iz = c / (nc * nc);
    float ox, oy, oz;
    cell_origin(a, c, ox, oy, oz);
    h.cell = c;
    h.rows = ix >= 1 && ix <= nc - 2;  // x-rows are contiguous and unshifted in x
    h.bx = ox;
    h.by = oy;
    h.bz = oz;
    if (lane < 27) {
        int jx = ix + lane % 3 - 1, jy = iy + (lane / 3) % 3 - 1, jz = iz + lane / 9 - 1;
        if (jx < 0) { jx += nc; h.bx = ox + a.box; } else if (jx >= nc) { jx -= nc; h.bx = ox - a.box; }
        if (jy < 0) { jy += nc; h.by = oy + a.box; } else if (jy >= nc) { jy -= nc; h.by = oy - a.box; }
        if (jz < 0) { jz += nc; h.bz = oz + a.box; } else if (jz >= nc) { jz -= nc; h.bz = oz - a.box; }
        const int cj = a.cbase + jx + nc * (jy + nc * jz);
        h.first = a.start[cj];
        h.next = a.start[cj + 1];
    }
}

__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Segments of a neighbourhood from its CSR ranges (waits for hood_issue's loads).
__device__ __forceinline__ void hood_segments(const SimArgs& a, const HoodLoads& h, HoodSegs& g) {
    const int lane = __lane_id();
    const int cnt = lane < 27 ? h.next - h.first : 0;
    const int incl = wave_incl_scan(cnt);
    const int pos = incl - cnt;
    int nseg;
    if (h.rows) {
        // segment r = cells 3r .. 3r + 2, gathered from lanes 3r and 3r + 2
        const int src = lane < 9 ? 3 * lane : 0;
        const int end = __shfl(incl, lane < 9 ? 3 * lane + 2 : 0);
        g.pos = __shfl(pos, src);
        g.first = __shfl(h.first, src);
        g.len = end - g.pos;
        g.x = __shfl(h.bx, src);
        g.y = __shfl(h.by, src);
        g.z = __shfl(h.bz, src);
        nseg = 9;
    } else {
        g.pos = pos;
        g.first = h.first;
        g.len = cnt;
        g.x = h.bx;
        g.y = h.by;
        g.z = h.bz;
        nseg = 27;
    }
    const int total = __shfl(incl, 26), home_pos = __shfl(pos, 13), home_first = __shfl(h.first, 13),
              n_home = __shfl(cnt, 13);
    g.meta = lane == 0 ? total : lane == 1 ? home_pos : lane == 2 ? home_first : lane == 3 ? n_home : nseg;
    float ox, oy, oz;
    cell_origin(a, h.cell, ox, oy, oz);
    g.org = lane == 0 ? ox : lane == 1 ? oy : oz;
}

// Write the table to LDS (the caller synchronises before it is read).
__device__ __forceinline__ void hood_store(const HoodSegs& g, Neighbourhood& nb) {
    const int lane = __lane_id();
    if (lane < g.nseg()) {
        nb.seg_pos[lane] = g.pos;
        nb.seg_first[lane] = g.first;
        nb.seg_len[lane] = g.len;
        nb.sx[lane] = g.x;
        nb.sy[lane] = g.y;
        nb.sz[lane] = g.z;
    }
    if (lane == 0) nb.total = g.meta;
    if (lane == 1) nb.home_pos = g.meta;
    if (lane == 2) nb.home_first = g.meta;
    if (lane == 3) nb.n_home = g.meta;
    if (lane == 4) nb.nseg = g.meta;
    if (lane < 3) nb.origin[lane] = g.org;
}

// The segment table of nb back in registers (lane l holds segment l).
__device__ __forceinline__ HoodSegs hood_from_lds(const Neighbourhood& nb) {
    const int lane = __lane_id();
    HoodSegs g;
    const int nseg = nb.nseg;
    g.meta = lane == 0 ? nb.total : lane == 1 ? nb.home_pos : lane == 2 ? nb.home_first : lane == 3 ? nb.n_home : nseg;
    g.org = nb.origin[lane < 3 ? lane : 0];
    if (lane < nseg) {
        g.pos = nb.seg_pos[lane];
        g.first = nb.seg_first[lane];
        g.len = nb.seg_len[lane];
        g.x = nb.sx[lane];
        g.y = nb.sy[lane];
        g.z = nb.sz[lane];
    }
    return g;
}

// Fill the neighbourhood table of home cell c and synchronise.
__device__ __forceinline__ void load_neighbourhood(const SimArgs& a, int c, Neighbourhood& nb,
                                                   float& ox, float& oy, float& oz) {
    HoodLoads h;
    hood_issue(a, c, h);
    HoodSegs g;
    hood_segments(a, h, g);
    if (threadIdx.x < kWave) hood_store(g, nb);  // every wavefront holds the same table
    cell_origin(a, c, ox, oy, oz);
    __syncthreads();
}

// Staging of neighbourhood atoms [t0, t1) into the tile, frame-translated: a
// uniform cursor (segment sg, neighbourhood index g) walks the segments in
// chunks of at most one wavefront; a batch of B chunks has its loads in flight
// before its LDS stores. w carries the user index (ID_IN_W) or |x|^2 in the
// frame (for the screen); with WITH_VEC the matching entries of a per-atom
// vector (sorted order) go to vtile as well.
struct StageCursor {
    int sg, g;
};

__device__ __forceinline__ StageCursor stage_begin(const HoodSegs& h, int t0) {
    StageCursor cur{0, t0};
    const int nseg = h.nseg();
    while (cur.sg < nseg && lane_value(h.pos, cur.sg) + lane_value(h.len, cur.sg) <= t0) ++cur.sg;
    return cur;
}

__device__ __forceinline__ bool stage_more(const HoodSegs& h, const StageCursor& cur, int t1) {
    return cur.g < t1 && cur.sg < h.nseg();
}

// One batch of chunks: per chunk the loaded atoms (one per lane). The chunk
// boundaries are not stored: the commit replays the cursor from the position
// the issue started at (a few scalar operations per chunk, and no scalar
// registers held between issue and commit).
template <int B, bool WITH_VEC>
struct StageBatch {
    float4 q[B], vq[B];
};

// Bounds of the chunk at the cursor: atoms [cur.g, ce) of segment cur.sg,
// whose first atom has neighbourhood index p and sorted slot first; advances
// the cursor past it.
__device__ __forceinline__ void stage_chunk(const HoodSegs& h, StageCursor& cur, int t1, int& p, int& first,
                                            int& base, int& cnt, int& seg) {
    p = lane_value(h.pos, cur.sg);
    const int end = p + lane_value(h.len, cur.sg);
    const int ce = min(min(cur.g + kWave, end), t1);
    first = lane_value(h.first, cur.sg);
    base = cur.g;
    cnt = ce - cur.g;
    seg = cur.sg;
    cur.g = ce;
    if (cur.g >= end) ++cur.sg;
}

template <int B, bool WITH_VEC>
__device__ __forceinline__ void stage_issue(const SimArgs& a, const HoodSegs& h, StageCursor& cur, int t1,
                                            StageBatch<B, WITH_VEC>& b, const float4* vec) {
    const int lane = __lane_id();
#pragma unroll
    for (int u = 0; u < B; ++u) {
        int slot = 0;  // lanes without an atom load slot 0 (always valid) and store nothing
        if (stage_more(h, cur, t1)) {
            int p, first, base, cnt, seg;
            stage_chunk(h, cur, t1, p, first, base, cnt, seg);
            if (lane < cnt) slot = first + (base - p) + lane;
        }
        b.q[u] = a.pos0[slot];
        if (WITH_VEC) b.vq[u] = vec[slot];
    }
}

// cur: the cursor stage_issue started from; on return, past the batch.
template <int B, bool ID_IN_W, bool WITH_VEC>
__device__ __forceinline__ void stage_commit(const HoodSegs& h, const StageBatch<B, WITH_VEC>& b, StageCursor& cur,
                                             int t0, int t1, float4* tile, float4* vtile) {
    const int lane = __lane_id();
#pragma unroll
    for (int u = 0; u < B; ++u) {
        if (stage_more(h, cur, t1)) {
            int p, first, base, cnt, seg;
            stage_chunk(h, cur, t1, p, first, base, cnt, seg);
            if (lane < cnt) {
                const int dst = base - t0 + lane;
                const float x = b.q[u].x - lane_value(h.x, seg);
                const float y = b.q[u].y - lane_value(h.y, seg);
                const float z = b.q[u].z - lane_value(h.z, seg);
                tile[dst] = make_float4(x, y, z, ID_IN_W ? b.q[u].w : x * x + y * y + z * z);
                if (WITH_VEC) vtile[dst] = b.vq[u];
            }
        }
    }
}

// Staging of a whole neighbourhood in one pass (total <= tile capacity), with
// few instructions per segment: every lane of a wavefront loads and stores
// entry pos + lane of each segment whether or not the segment has that many
// atoms. Segments are written in order and tile [0, total) without gaps, so
// the surplus entries of segment k (indices pos_k + len_k .. pos_k + 63) are
// overwritten by a later segment, or fall into the padding after total,
// which the caller fills afterwards; loads past the arrays' end are clamped.
// Atoms 64 and up of a longer segment follow, masked, after every segment's
// first 64: no surplus store reaches that far (pos_j + 63 < pos_k + 64 for
// j < k). The tile needs room for total + 63 entries.
template <bool ID_IN_W>
__device__ __forceinline__ void stage_whole(const SimArgs& a, const HoodSegs& h, float4* tile) {
    const int lane = __lane_id();
    const int nseg = h.nseg();  // 9 or 27
    const int last = a.natoms - 1;
    // 32-bit byte offsets from the array base (scalar base + vector offset loads)
    const char* pbase = reinterpret_cast<const char*>(a.pos0);
    for (int k0 = 0; k0 < nseg; k0 += 9) {
        float4 q[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            const uint32_t off = static_cast<uint32_t>(min(lane_value(h.first, k0 + u) + lane, last)) << 4;
            q[u] = *reinterpret_cast<const float4*>(pbase + off);
        }
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            const int k = k0 + u;
            const float x = q[u].x - lane_value(h.x, k);
            const float y = q[u].y - lane_value(h.y, k);
            const float z = q[u].z - lane_value(h.z, k);
            tile[lane_value(h.pos, k) + lane] = make_float4(x, y, z, ID_IN_W ? q[u].w : x * x + y * y + z * z);
            // store as each load arrives: nine results held for one burst of
            // stores would cost 36 more registers
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    uint64_t longs = __ballot(lane < nseg && h.len > kWave);
    while (longs) {
        const int k = __ffsll(static_cast<unsigned long long>(longs)) - 1;
        longs &= longs - 1;
        const int len = lane_value(h.len, k), first = lane_value(h.first, k), pos = lane_value(h.pos, k);
        const float sx = lane_value(h.x, k), sy = lane_value(h.y, k), sz = lane_value(h.z, k);
        for (int off = kWave + lane; off - lane < len; off += kWave) {
            if (off < len) {
                const float4 q = a.pos0[first + off];
                const float x = q.x - sx, y = q.y - sy, z = q.z - sz;
                tile[pos + off] = make_float4(x, y, z, ID_IN_W ? q.w : x * x + y * y + z * z);
            }
        }
    }
}

// Neighbourhood of a home cell away from the x faces (1 <= ix <= nc - 2), held
// in scalar registers: its nine x-rows (dy, dz) of three cells each are
// contiguous in the sorted arrays and need no image shift in x, so the row
// bounds come from nine uniform loads of four CSR offsets each and the
// staging below needs no per-segment table lookups.
struct RowHood {
    int first[9];  // sorted slot of each row's first atom
    int pos[10];   // neighbourhood index of each row's first atom; pos[9] = total
    int home_first, n_home, home_pos;
    float ox, oy, oz;  // home-cell origin
    float fy[3], fz[3];  // frame offsets o - sh of the rows with dy, dz = -1, 0, 1
};

// Fill r for home cell c (local index, uniform); false for a cell on an x
// face. Lane k < 9 loads the CSR offsets of row k's cells ix - 1 .. ix + 2
// (one 16-byte load, one round trip for the table); the values then move to
// scalar registers.
typedef int Int4u __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ bool row_hood(const SimArgs& a, int c, RowHood& r) {
#pragma clang fp contract(off)
    const int lane = __lane_id();
    const int nc = a.nc;
    const int ix = __builtin_amdgcn_readfirstlane(c % nc);
    const int iy = __builtin_amdgcn_readfirstlane((c / nc) % nc);
    const int iz = __builtin_amdgcn_readfirstlane(c / (nc * nc));
    if (ix < 1 || ix > nc - 2) return false;
    r.ox = static_cast<float>(ix) * a.s;
    r.oy = static_cast<float>(iy) * a.s;
    r.oz = static_cast<float>(iz) * a.s;
    r.fy[0] = iy == 0 ? r.oy + a.box : r.oy;
    r.fy[1] = r.oy;
    r.fy[2] = iy == nc - 1 ? r.oy - a.box : r.oy;
    r.fz[0] = iz == 0 ? r.oz + a.box : r.oz;
    r.fz[1] = r.oz;
    r.fz[2] = iz == nc - 1 ? r.oz - a.box : r.oz;
    Int4u row = {0, 0, 0, 0};
    if (lane < 9) {
        int jy = iy + lane % 3 - 1, jz = iz + lane / 3 - 1;
        jy = jy < 0 ? jy + nc : (jy >= nc ? jy - nc : jy);
        jz = jz < 0 ? jz + nc : (jz >= nc ? jz - nc : jz);
        row = *reinterpret_cast<const Int4u*>(a.start + a.cbase + (ix - 1) + nc * (jy + nc * jz));
    }
    int s0[9], s3[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        s0[k] = __builtin_amdgcn_readlane(row.x, k);
        s3[k] = __builtin_amdgcn_readlane(row.w, k);
    }
    const int s1 = __builtin_amdgcn_readlane(row.y, 4), s2 = __builtin_amdgcn_readlane(row.z, 4);
    int p = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        r.first[k] = s0[k];
        r.pos[k] = p;
        if (k == 4) r.home_pos = p + (s1 - s0[k]);
        p += s3[k] - s0[k];
    }
    r.home_first = s1;
    r.n_home = s2 - s1;
    r.pos[9] = p;
    return true;
}

// Second tile of the staging functions below (SECOND): none; the untranslated
// positions (w = user index); the entries of vsrc, a per-atom vector in
// sorted order; or (SECOND_CODE, 32-bit entries) each atom's neighbour-list
// entry: its sorted slot with the code of the periodic image the frame
// translation applied. Any of them goes to raw at the same indices as the
// positions.
enum { SECOND_NONE = 0, SECOND_RAW = 1, SECOND_VEC = 2, SECOND_CODE = 3 };

// Image shift along one axis of a neighbour whose atoms are staged at
// x - f in the frame of origin o: the partner of the home atom is x + s L
// with s L = o - f, i.e. s = -1, 0 or +1.
__device__ __forceinline__ int image_shift(float o, float f, float box) {
    const float d = o - f;
    return d > 0.5f * box ? 1 : (d < -0.5f * box ? -1 : 0);
}

__device__ __forceinline__ uint32_t list_entry(int slot, int sx, int sy, int sz) {
    return static_cast<uint32_t>(slot) | (static_cast<uint32_t>((sx + 1) + 3 * (sy + 1) + 9 * (sz + 1)) << kSlotBits);
}

// Staging of a RowHood neighbourhood in one pass (total <= tile capacity), by
// the same unmasked scheme as stage_whole (rows tile [0, total) in order).
template <int SECOND = SECOND_NONE>
__device__ __forceinline__ void stage_rows(const SimArgs& a, const RowHood& r, float4* tile, float4* raw = nullptr,
                                           const float4* vsrc = nullptr) {
    const int lane = __lane_id();
    const int last = a.natoms - 1;
    const char* pbase = reinterpret_cast<const char*>(a.pos0);
    const char* vbase = reinterpret_cast<const char*>(vsrc);
    float4 q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint32_t off = static_cast<uint32_t>(min(r.first[k] + lane, last)) << 4;
        q[k] = *reinterpret_cast<const float4*>(pbase + off);
    }
    uint32_t* codes = reinterpret_cast<uint32_t*>(raw);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float x = q[k].x - r.ox;
        const float y = q[k].y - r.fy[k % 3];
        const float z = q[k].z - r.fz[k / 3];
        tile[r.pos[k] + lane] = make_float4(x, y, z, x * x + y * y + z * z);
        if (SECOND == SECOND_RAW) raw[r.pos[k] + lane] = q[k];
        if (SECOND == SECOND_CODE)
            codes[r.pos[k] + lane] = list_entry(r.first[k] + lane, 0, image_shift(r.oy, r.fy[k % 3], a.box),
                                                image_shift(r.oz, r.fz[k / 3], a.box));
        __builtin_amdgcn_sched_barrier(0);
    }
    if (SECOND == SECOND_VEC) {  // a second round (the positions' registers are free again)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const uint32_t off = static_cast<uint32_t>(min(r.first[k] + lane, last)) << 4;
            q[k] = *reinterpret_cast<const float4*>(vbase + off);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            raw[r.pos[k] + lane] = q[k];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int len = r.pos[k + 1] - r.pos[k];
        if (len > kWave) {  // uniform; rare
            for (int off = kWave + lane; off - lane < len; off += kWave) {
                if (off < len) {
                    const float4 u = a.pos0[r.first[k] + off];
                    const float x = u.x - r.ox, y = u.y - r.fy[k % 3], z = u.z - r.fz[k / 3];
                    tile[r.pos[k] + off] = make_float4(x, y, z, x * x + y * y + z * z);
                    if (SECOND == SECOND_RAW) raw[r.pos[k] + off] = u;
                    if (SECOND == SECOND_VEC) raw[r.pos[k] + off] = vsrc[r.first[k] + off];
                    if (SECOND == SECOND_CODE)
                        codes[r.pos[k] + off] = list_entry(r.first[k] + off, 0, image_shift(r.oy, r.fy[k % 3], a.box),
                                                           image_shift(r.oz, r.fz[k / 3], a.box));
                }
            }
        }
    }
}

// Stage neighbourhood atoms [t0, t0 + tn) of the table in nb (an interior
// cell's neighbourhood costs one global round trip).
// B chunks in flight per batch (default: 9, or 5 with a vector).
template <bool ID_IN_W, bool WITH_VEC = false, int B = (WITH_VEC ? 5 : 9)>
__device__ __forceinline__ void stage_tile(const SimArgs& a, const Neighbourhood& nb, float4* tile,
                                           int t0, int tn, const float4* vec = nullptr,
                                           float4* vtile = nullptr) {
    const HoodSegs h = hood_from_lds(nb);
    if (!WITH_VEC && t0 == 0 && tn == h.total()) {
        stage_whole<ID_IN_W>(a, h, tile);
        return;
    }
    const int t1 = t0 + tn;
    StageCursor cur = stage_begin(h, t0);
    while (stage_more(h, cur, t1)) {
        StageBatch<B, WITH_VEC> b;
        StageCursor issue = cur;
        stage_issue(a, h, issue, t1, b, vec);
        stage_commit<B, ID_IN_W, WITH_VEC>(h, b, cur, t0, t1, tile, vtile);
    }
}

// Neighbour-list entries (list_entry) of neighbourhood atoms [t0, t0 + tn) of
// the table in nb, into codes[0, tn): the companion of stage_tile for the
// pass that writes the neighbour lists.
__device__ __forceinline__ void stage_codes(const SimArgs& a, const Neighbourhood& nb, uint32_t* codes, int t0,
                                            int tn) {
    const int lane = __lane_id();
    const int t1 = t0 + tn;
    const int nseg = nb.nseg;
    for (int k = 0; k < nseg; ++k) {  // uniform
        const int p = nb.seg_pos[k], len = nb.seg_len[k], first = nb.seg_first[k];
        const int lo = max(p, t0), hi = min(p + len, t1);
        const int sx = image_shift(nb.origin[0], nb.sx[k], a.box);
        const int sy = image_shift(nb.origin[1], nb.sy[k], a.box);
        const int sz = image_shift(nb.origin[2], nb.sz[k], a.box);
        for (int t = lo + lane; t < hi; t += kWave) codes[t - t0] = list_entry(first + (t - p), sx, sy, sz);
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
constexpr int kMaxCellWaves = 4;                            // wavefronts per force workgroup

// LDS entries (float4) of a force workgroup: the tile and its padding, which
// the reduction reuses (five floats per lane and wavefront)
__host__ __device__ constexpr size_t cell_lds_entries(int tile_cap, int waves) {
    return static_cast<size_t>(tile_cap + kTilePad > 80 * waves ? tile_cap + kTilePad : 80 * waves);
}

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

// The LDS byte address of a pointer into shared memory (the low half of its
// generic address), and a 16-byte load from such an address: walks that
// carry absolute LDS addresses read their candidates with no add.
__device__ __forceinline__ uint32_t lds_address(const void* p) {
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p));
}
typedef float lds_float4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 lds_load(uint32_t addr) {
    const lds_float4 v = *(const __attribute__((address_space(3))) lds_float4*)(static_cast<uintptr_t>(addr));
    return make_float4(v.x, v.y, v.z, v.w);
}

// Walk the accepted bits of one span in order, calling op(address, live) for
// each: address is the LDS byte address of the accepted candidate, the span's
// candidate 0 lying at wb0; live is false for lanes that have spent their
// bits. The words rotate through four registers (never indexed, which would
// put them in scratch memory); an exhausted word is replaced by the next one
// without a branch. Each iteration takes two candidates (the second may come from the
// next word), so the wave-wide loop test and branch run once per pair; the
// calls keep the one-at-a-time order, so sums do not depend on the
// unrolling.
template <class Op>
__device__ __forceinline__ void walk_bits(int ns, uint32_t wb0, uint32_t m, uint32_t n1, uint32_t n2, uint32_t n3,
                                          Op& op) {
    const uint32_t cstep = static_cast<uint32_t>(ns) * sizeof(float4);   // bytes between candidates
    const uint32_t wstep = 32u * cstep;                                  // bytes between words
    uint32_t wb = wb0;                                                   // LDS address of the word's candidate 0
    uint32_t left = __builtin_popcount(m) + __builtin_popcount(n1) + __builtin_popcount(n2) +
                    __builtin_popcount(n3);
    if (!__any(left != 0u)) return;
    do {
        uint32_t off[2];
        bool live[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const bool next = (m == 0u);
            m = next ? n1 : m;
            n1 = next ? n2 : n1;
            n2 = next ? n3 : n2;
            n3 = next ? 0u : n3;
            wb = next ? wb + wstep : wb;
            live[u] = m != 0u;
            // all ones for a spent lane (m = 0): its shift clears no bit of
            // m, and its offset is replaced below
            const uint32_t k = __builtin_clzg(m, -1);
            m &= ~(0x80000000u >> (k & 31u));
            left -= live[u] ? 1u : 0u;
            // a spent lane keeps rotating (wb grows past its span): it reads
            // its span's first candidate instead, which is always staged
            // (a constant stride, as the matrix-core screen's four slices
            // give, makes the product one shift-and-add; otherwise the 24-bit
            // multiply-add; either is garbage for a spent lane, replaced here)
            const uint32_t step = __builtin_constant_p(cstep) ? k * cstep : __umul24(k, cstep);
            off[u] = live[u] ? wb + step : wb0;
        }
        op(off[0], live[0]);
        op(off[1], live[1]);
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

// ---- screen on the matrix cores ------------------------------------------
// For a home cell of 11..16 atoms the screen runs as 16 x 16 x 4 FP32
// matrix products: D = A B + C with A the 16 candidates of a block (rows:
// x, y, z, |x|^2 in the home frame), B the 16 home atoms (columns:
// -2 x_i, -2 y_i, -2 z_i, 1) and C = -(bound - |x_i|^2) per column, so that
// D[j][i] = |x_j|^2 - 2 x_i.x_j - (bound - |x_i|^2) = r^2 - bound, negative
// iff accepted. Lane l supplies B[l / 16][l % 16] and A[l % 16][l / 16],
// where row m of A is candidate 4 (m % 4) + m / 4 of the block, and receives
// D[4 (l / 16) + q][l % 16], q = 0..3: lane (home atom l % 16, slice
// s = l / 16) gets the verdicts on candidates 16 b + 4 q + s of every block
// b, four sign bits per block, one v_alignbit each (about one VALU
// instruction per candidate instead of five). A lane's bits thus follow its
// candidates s, s + 4, s + 8, ... in order: the words are those of the VALU
// screen with ns = 4 slices, and the same walk takes them. Unused home
// columns carry C = +inf and B = (0, 0, 0, 1): their D is +inf. Padding
// entries (w = +inf) are never accepted either.
constexpr int kMfmaMinHome = 11;  // below this the VALU screen's extra slices win
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// Screen one span of nblk <= 32 blocks starting at candidate first (a
// multiple of 16): word w, bit 31 - k holds the verdict on the lane's
// candidate first + 4 (32 w + k) + s. bval: this lane's B element; cneg: C.
__device__ __forceinline__ void screen_mfma(const float4* tile, int first, int nblk, float bval, float cneg,
                                            uint32_t (&wd)[kWords]) {
    const int lane = __lane_id();
    const int row = lane & 15;  // A row: candidate 4 (row % 4) + row / 4 of each block
    const float* base = reinterpret_cast<const float*>(tile + first) + (4 * (row & 3) + (row >> 2)) * 4 + (lane >> 4);
    const mfma_f4 c = {cneg, cneg, cneg, cneg};
#pragma unroll
    for (int w = 0; w < kWords; ++w) {
        uint32_t bits = 0;
        const int nb = min(8, nblk - 8 * w);  // uniform
        if (nb > 0) {
            for (int b0 = 0; b0 < nb; b0 += 4) {
                float av[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) av[u] = base[(8 * w + b0 + u) * 64];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const mfma_f4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bval, c, 0, 0, 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) bits = __builtin_amdgcn_alignbit(bits, __float_as_uint(d[q]), 31);
                }
            }
            const int done = (nb + 3) / 4 * 4;  // blocks shifted in (the last group may run past nb)
            if (done < 8) bits <<= (32 - 4 * done);
        }
        wd[w] = bits;
    }
}

// ---- neighbourhood of a cell on an x face as x-row pieces -------------------
// The 27-cell neighbourhood is nine x-rows (dy, dz). In each row the cells
// that need no image shift in x are consecutive in the sorted arrays (piece A:
// three cells, or two for a home cell on an x face); on an x face the row's
// third cell wraps around the box (piece B, one cell, shifted by -+L in x).
// Interior cells take the scalar row table RowHood; this one, for the cells on
// the x faces, stages them in one pass too instead of through the LDS segment
// table of 27 single cells.
// Pieces are staged in the order A0..A8, B0..B8, so the tile holds the
// neighbourhood without gaps. The piece table is held one piece per lane
// (lane k < 9: Ak, lane 9 + k: Bk); the rest is uniform.
struct RowPieces {
    int first = 0, pos = 0, len = 0;  // this lane's piece: sorted slot and tile index of its first atom, length
    int total, home_first, n_home, home_pos;
    float ox, oy, oz;   // home-cell origin
    float fxb;          // frame offset in x of the B pieces
    float fy[3], fz[3];  // frame offsets o - sh of rows with dy, dz = -1, 0, 1
    bool face;
};

// Fill r for home cell c (local index, uniform). Lane k < 9 reads the CSR
// offsets of row k's piece A (four consecutive entries: the start array has
// four entries of padding after its end) and, on a face, of its piece B.
__device__ __forceinline__ void row_pieces(const SimArgs& a, int c, RowPieces& r) {
#pragma clang fp contract(off)
    const int lane = __lane_id();
    const int nc = a.nc;
    const int nn = nc * nc;
    const int iz = c / nn;
    const int rem = c - iz * nn;
    const int iy = rem / nc;
    const int ix = rem - iy * nc;
    r.face = ix == 0 || ix == nc - 1;
    r.ox = static_cast<float>(ix) * a.s;
    r.oy = static_cast<float>(iy) * a.s;
    r.oz = static_cast<float>(iz) * a.s;
    r.fy[0] = iy == 0 ? r.oy + a.box : r.oy;
    r.fy[1] = r.oy;
    r.fy[2] = iy == nc - 1 ? r.oy - a.box : r.oy;
    r.fz[0] = iz == 0 ? r.oz + a.box : r.oz;
    r.fz[1] = r.oz;
    r.fz[2] = iz == nc - 1 ? r.oz - a.box : r.oz;
    r.fxb = ix == 0 ? r.ox + a.box : r.ox - a.box;
    // first cell of piece A; the home cell is cell hoff of it (0 or 1)
    const int a0 = ix == 0 ? 0 : (ix == nc - 1 ? nc - 2 : ix - 1);
    const int hoff = ix - a0;
    const int bcell = ix == 0 ? nc - 1 : 0;
    Int4u row = {0, 0, 0, 0};
    int b0 = 0, b1 = 0;
    if (lane < 9) {
        int jy = iy + lane % 3 - 1, jz = iz + lane / 3 - 1;
        jy = jy < 0 ? jy + nc : (jy >= nc ? jy - nc : jy);
        jz = jz < 0 ? jz + nc : (jz >= nc ? jz - nc : jz);
        const int* rs = a.start + a.cbase + nc * (jy + nc * jz);
        row = *reinterpret_cast<const Int4u*>(rs + a0);
        if (r.face) {
            b0 = rs[bcell];
            b1 = rs[bcell + 1];
        }
    }
    const int aend = r.face ? row.z : row.w;
    if (lane < 9) {
        r.first = row.x;
        r.len = aend - row.x;
    }
    if (r.face) {  // B pieces to lanes 9..17
        const int src = lane >= 9 && lane < 18 ? lane - 9 : 0;
        const int bf = __shfl(b0, src), bl = __shfl(b1 - b0, src);
        if (lane >= 9 && lane < 18) {
            r.first = bf;
            r.len = bl;
        }
    }
    const int incl = wave_incl_scan(r.len);
    r.pos = incl - r.len;
    r.total = __builtin_amdgcn_readlane(incl, 17);
    const int hb = hoff == 0 ? row.x : row.y, he = hoff == 0 ? row.y : row.z;
    r.home_first = __builtin_amdgcn_readlane(hb, 4);
    r.n_home = __builtin_amdgcn_readlane(he, 4) - r.home_first;
    r.home_pos = __builtin_amdgcn_readlane(r.pos, 4) + (r.home_first - __builtin_amdgcn_readlane(r.first, 4));
}

// Staging of nine pieces (table lanes k0 .. k0 + 8) in one pass by the
// unmasked scheme of stage_whole: every lane loads and stores entry
// pos + lane of each piece; pieces are written in order, so a piece's surplus
// entries are overwritten by a later piece or fall into the padding after the
// total. Atoms 64 and up of a longer piece follow, masked. SECOND as for
// stage_rows.
template <int K0, int SECOND>
__device__ __forceinline__ void stage_nine(const SimArgs& a, const RowPieces& r, float fx, float4* tile,
                                           float4* raw, const float4* vsrc) {
    const int lane = __lane_id();
    const int last = a.natoms - 1;
    const char* pbase = reinterpret_cast<const char*>(a.pos0);
    const char* vbase = reinterpret_cast<const char*>(vsrc);
    float4 q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint32_t off = static_cast<uint32_t>(min(__builtin_amdgcn_readlane(r.first, K0 + k) + lane, last)) << 4;
        q[k] = *reinterpret_cast<const float4*>(pbase + off);
    }
    uint32_t* codes = reinterpret_cast<uint32_t*>(raw);
    const int sx = SECOND == SECOND_CODE ? image_shift(r.ox, fx, a.box) : 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float x = q[k].x - fx;
        const float y = q[k].y - r.fy[k % 3];
        const float z = q[k].z - r.fz[k / 3];
        const int p = __builtin_amdgcn_readlane(r.pos, K0 + k);
        tile[p + lane] = make_float4(x, y, z, x * x + y * y + z * z);
        if (SECOND == SECOND_RAW) raw[p + lane] = q[k];
        if (SECOND == SECOND_CODE)
            codes[p + lane] = list_entry(__builtin_amdgcn_readlane(r.first, K0 + k) + lane, sx,
                                         image_shift(r.oy, r.fy[k % 3], a.box), image_shift(r.oz, r.fz[k / 3], a.box));
        __builtin_amdgcn_sched_barrier(0);
    }
    if (SECOND == SECOND_VEC) {  // a second round (the positions' registers are free again)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const uint32_t off = static_cast<uint32_t>(min(__builtin_amdgcn_readlane(r.first, K0 + k) + lane, last))
                                 << 4;
            q[k] = *reinterpret_cast<const float4*>(vbase + off);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            raw[__builtin_amdgcn_readlane(r.pos, K0 + k) + lane] = q[k];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (__any(lane >= K0 && lane < K0 + 9 && r.len > kWave)) {  // rare
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int len = __builtin_amdgcn_readlane(r.len, K0 + k);
            if (len > kWave) {
                const int f = __builtin_amdgcn_readlane(r.first, K0 + k), p = __builtin_amdgcn_readlane(r.pos, K0 + k);
                for (int off = kWave + lane; off - lane < len; off += kWave) {
                    if (off < len) {
                        const float4 u = a.pos0[f + off];
                        const float x = u.x - fx, y = u.y - r.fy[k % 3], z = u.z - r.fz[k / 3];
                        tile[p + off] = make_float4(x, y, z, x * x + y * y + z * z);
                        if (SECOND == SECOND_RAW) raw[p + off] = u;
                        if (SECOND == SECOND_VEC) raw[p + off] = vsrc[f + off];
                        if (SECOND == SECOND_CODE)
                            codes[p + off] = list_entry(f + off, sx, image_shift(r.oy, r.fy[k % 3], a.box),
                                                        image_shift(r.oz, r.fz[k / 3], a.box));
                    }
                }
            }
        }
    }
}

// The whole neighbourhood of r in one pass (total <= tile capacity; the tile
// needs room for total + 63 entries).
template <int SECOND = SECOND_NONE>
__device__ __forceinline__ void stage_pieces(const SimArgs& a, const RowPieces& r, float4* tile, float4* raw = nullptr,
                                             const float4* vsrc = nullptr) {
    stage_nine<0, SECOND>(a, r, r.ox, tile, raw, vsrc);
    if (r.face) stage_nine<9, SECOND>(a, r, r.fxb, tile, raw, vsrc);
}

}  // namespace
}  // namespace mdlj
