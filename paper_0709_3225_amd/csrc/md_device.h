// Device helpers shared by the kernels: periodic wrap, cell index,
// wavefront-aggregated histogram ranks, wave reductions, XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "md_internal.h"

namespace mdlj {

constexpr int kWave = 64;

// Bring one FP32 coordinate into [0, L). x - L*floor(x/L) can round to L
// exactly; then subtract L once more, and fall back to 0 for the last ulp.
__device__ __forceinline__ float wrap_coord(float x, float L, float invL) {
    x = x - L * floorf(x * invL);
    if (x >= L) x -= L;
    if (x < 0.0f || x >= L) x = 0.0f;
    return x;
}

__device__ __forceinline__ int cell_coord(float x, float inv_s, int nc) {
    int i = static_cast<int>(x * inv_s);
    return i < 0 ? 0 : (i >= nc ? nc - 1 : i);
}

__device__ __forceinline__ int cell_index(float x, float y, float z, const SimArgs& a) {
    return cell_coord(x, a.inv_s, a.nc) + a.nc * (cell_coord(y, a.inv_s, a.nc) + a.nc * cell_coord(z, a.inv_s, a.nc));
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
    return isfinite(x) && isfinite(y) && isfinite(z);
}

// First half of a velocity-Verlet step for one atom (section 2): v += dt/(2m) f,
// r += dt v (the unwrapped form stops here), wrap into the box. A non-finite position raises DEV_NONFINITE and
// is parked at the origin. Returns the atom's new cell (global index). The
// drift kernel and the fused force epilogue both use this, so the two paths
// round identically.
__device__ __forceinline__ void half_kick_drift_unwrapped(const SimArgs& a, float4& p, float4& v, float fx,
                                                          float fy, float fz) {
    v.x += a.hdt_m * fx;
    v.y += a.hdt_m * fy;
    v.z += a.hdt_m * fz;
    p.x += a.dt * v.x;
    p.y += a.dt * v.y;
    p.z += a.dt * v.z;
    if (!finite3(p.x, p.y, p.z)) {
        atomicOr(&a.hdr[HDR_ERROR], DEV_NONFINITE);
        p.x = p.y = p.z = 0.f;
    }
}

__device__ __forceinline__ int half_kick_drift(const SimArgs& a, float4& p, float4& v, float fx, float fy,
                                               float fz) {
    const float invL = 1.0f / a.box;
    half_kick_drift_unwrapped(a, p, v, fx, fy, fz);
    p.x = wrap_coord(p.x, a.box, invL);
    p.y = wrap_coord(p.y, a.box, invL);
    p.z = wrap_coord(p.z, a.box, invL);
    return a.cbase + cell_index(p.x, p.y, p.z, a);
}

// Arrival rank of each lane's atom in cell c (c < 0: no atom). Lanes holding
// the same cell in a contiguous run share one atomicAdd of the run length on
// the histogram; input that is already cell-sorted (every step after the
// first) turns most per-atom atomics into one per run. bcount (nullable)
// receives the count per block of 16 cells too, one atomic per run of lanes
// in the same block. Atomics on one address
// serialise (about 0.15 us each here), so nothing coarser than 16 cells is
// counted atomically. Must be called by all 64 lanes of the wave.
__device__ __forceinline__ int histogram_rank(int* count, int* bcount, int c) {
    const int lane = __lane_id();
    const int prev = __shfl_up(c, 1);
    const bool head = (lane == 0) || (prev != c);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t above = heads & ~upto;
    const int next_head = above ? (__ffsll(static_cast<unsigned long long>(above)) - 1) : kWave;
    const int my_head = 63 - __clzll(static_cast<long long>(heads & upto));
    int base = 0;
    if (head && c >= 0) base = atomicAdd(&count[c], next_head - lane);
    if (bcount) {
        // the block counts, one atomic per run of lanes in the same block of
        // cells (several cells of a run share a block counter)
        const int bk = c >= 0 ? (c >> kBlockShift) : -1;
        const int prevb = __shfl_up(bk, 1);
        const bool bhead = (lane == 0) || (prevb != bk);
        const uint64_t bheads = __ballot(bhead);
        const uint64_t babove = bheads & ~upto;
        const int next_bhead = babove ? (__ffsll(static_cast<unsigned long long>(babove)) - 1) : kWave;
        if (bhead && bk >= 0) atomicAdd(&bcount[bk], next_bhead - lane);
    }
    base = __shfl(base, my_head);
    return base + (lane - my_head);
}

// Bin an atom (position p with its user index in w, velocity v) into cell c
// (global index; c < 0: this lane has no atom): rank in the cell, then the
// atom goes to the cell's bucket, or to the overflow list once the bucket is
// full. Must be called by all 64 lanes of the wave.
__device__ __forceinline__ void bin_atom(const SimArgs& a, float4 p, float4 v, int c) {
    const int r = histogram_rank(a.counts, a.direct ? a.bcounts + a.par * a.nbstride : nullptr, c);
    if (c < 0) return;
    if (r < a.cap) {
        const size_t e = static_cast<size_t>(c) * a.cap + r;
        a.bpos[e] = p;
        a.bvel[e] = v;
    } else {
        const int j = atomicAdd(&a.hdr[HDR_OVF + a.par], 1);
        if (j < a.natoms) {
            a.ovf_cell[j] = c;
            a.ovf_rank[j] = r - a.cap;
            a.pos1[j] = p;
            a.vel1[j] = v;
        } else {
            atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);  // histogram not cleared: a call sequence was cut short
        }
    }
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with
// its own L2. Renumber blocks so that every XCD receives one contiguous range
// of work items (here: cells in z-major order, i.e. a slab of the box), which
// keeps the 27-cell neighbourhoods a block stages in the L2 its neighbours use.
__device__ __forceinline__ int xcd_block_order(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, k = b >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Arguments of one replica of a batch: the batch's arrays and shared
// constants with the replica's geometry and cell offset.
__device__ __forceinline__ SimArgs replica_view(const SimArgs& base, const Replica& r) {
    SimArgs a = base;
    a.n = r.n;
    a.nc = r.nc;
    a.ncells = r.ncells;
    a.cbase = r.cbase;
    a.tile_cap = r.tile_cap;
    a.box = r.box;
    a.s = r.s;
    a.inv_s = r.inv_s;
    a.screen2 = r.screen2;
    return a;
}

// True if the workspace holds a built state for exactly these arguments
// (cells built, or forces too when need_forces).
__device__ __forceinline__ bool state_ok(const SimArgs& a, bool need_forces) {
    const int st = a.hdr[HDR_STATE];
    const bool built = need_forces ? (st == STATE_FORCES) : (st == STATE_CELLS || st == STATE_FORCES);
    return built && a.hdr[HDR_N] == a.n && a.hdr[HDR_NC] == a.nc;
}

}  // namespace mdlj
