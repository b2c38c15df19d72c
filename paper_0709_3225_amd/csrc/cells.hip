// Cell-list build by counting sort into per-cell buckets (section 3 cells of
// side >= r_c; section 3.1 membership kept current as particles move), and the
// velocity-Verlet drift that feeds it (section 2).
//
// A build is three launches:
//   bin        : wrap + cell index + histogram rank (one atomic per run of
//                equal cells in a wavefront); the atom's position and
//                velocity go to its cell's bucket (or the overflow list
//                beyond the bucket capacity).
//                Inside a multi-step run the force kernel's epilogue bins the
//                drifted atoms, so this launch only starts a build or a run.
//   block scan : one workgroup sums the histogram over blocks of 16 cells
//                and scans the sums into the atoms before each block.
//   cell order : the workgroup of a 16-cell block adds its cells' counts to
//                the block's offset, writes the cell offsets, clears its
//                cells' counts, orders each cell's members by user index and
//                moves them into the sorted arrays.
// The cell order clears its own cells' counts after the block scan has read
// them, so the histogram is zero between builds. The paper updated each cell with one
// serial thread per cell (section 3.1); here nothing runs serially per cell and
// there is no capacity per cell (the overflow list takes the excess).
#include "md_device.h"

namespace mdlj {

namespace {

constexpr int kBlock = 256;

// Header and histograms cleared (the whole workspace of a batch).
__global__ void __launch_bounds__(kBlock) k_build_init(SimArgs a) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int stride = gridDim.x * kBlock;
    if (t == 0) {
        a.hdr[HDR_ERROR] = 0;
        a.hdr[HDR_STATE] = STATE_BUILDING;
        a.hdr[HDR_N] = a.n;
        a.hdr[HDR_NC] = a.nc;
        a.hdr[HDR_OVF] = 0;
        a.hdr[HDR_OVF + 1] = 0;
        a.hdr[HDR_OVFA] = 0;
        a.hdr[HDR_OVFA + 1] = 0;
    }
    for (int c = t; c < (a.nblocks << kBlockShift); c += stride) a.counts[c] = 0;
    for (int b = t; b < 2 * a.nbstride; b += stride) a.bcounts[b] = 0;
}

__global__ void k_set_state(SimArgs a, int state) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.hdr[HDR_STATE] = state;
}

// Clear the counters of parity par (overflow count, block histogram).
__global__ void __launch_bounds__(kBlock) k_zero_blocks(SimArgs a, int par) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t == 0) {
        a.hdr[HDR_OVF + par] = 0;
        a.hdr[HDR_OVFA + par] = 0;
    }
    for (int b = t; b < a.nbstride; b += gridDim.x * kBlock) a.bcounts[par * a.nbstride + b] = 0;
}

// Load one user-order atom i: wrap, cell index, binning.
// Called by every lane of the wave (valid = false for
// lanes past the end); cells are numbered globally (a.cbase + local index).
__device__ __forceinline__ void load_atom(const SimArgs& a, int i, bool valid, const float4* __restrict__ pos_in,
                                          const float4* __restrict__ vel_in) {
    const float invL = 1.0f / a.box;
    int c = -1;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
        p = pos_in[i];
        if (vel_in) v = vel_in[i];
        if (!finite3(p.x, p.y, p.z) || !finite3(v.x, v.y, v.z)) {
            atomicOr(&a.hdr[HDR_ERROR], DEV_NONFINITE);
            p.x = p.y = p.z = 0.f;
        }
        p.x = wrap_coord(p.x, a.box, invL);
        p.y = wrap_coord(p.y, a.box, invL);
        p.z = wrap_coord(p.z, a.box, invL);
        p.w = __int_as_float(i);
        v.w = 0.f;
        c = a.cbase + cell_index(p.x, p.y, p.z, a);
    }
    bin_atom(a, p, v, c);
}

// Velocity-Verlet first half for sorted slot i (half kick, drift, wrap), then
// the binning for the rebuild. Called by every lane of the wave.
__device__ __forceinline__ void integrate_atom(const SimArgs& a, int i, bool valid) {
    int c = -1;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), v = p;
    if (valid) {
        p = a.pos0[i];
        v = a.vel0[i];
        const float4 f = a.force[i];
        c = half_kick_drift(a, p, v, f.x, f.y, f.z);
    }
    bin_atom(a, p, v, c);
}

__global__ void __launch_bounds__(kBlock) k_load(SimArgs a, const float4* __restrict__ pos_in,
                                                 const float4* __restrict__ vel_in) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    load_atom(a, i, i < a.n, pos_in, vel_in);
}

__global__ void __launch_bounds__(kBlock) k_integrate(SimArgs a) {
    // A step needs forces of the current state; while a call-order error is
    // pending (until md_check clears it) every step kernel does nothing.
    if (!state_ok(a, true) || (a.hdr[HDR_ERROR] & DEV_ORDER)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    const int i = blockIdx.x * kBlock + threadIdx.x;
    integrate_atom(a, i, i < a.n);
}

// Batched load and drift: one lane per atom of the whole batch (global
// index; replica from the per-atom table). a.n of the base is the batch total.
__global__ void __launch_bounds__(kBlock) k_batch_load(SimArgs base, const Replica* __restrict__ reps,
                                                       const int* __restrict__ atom_rep,
                                                       const float4* __restrict__ pos_in,
                                                       const float4* __restrict__ vel_in) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < base.n;
    const SimArgs a = replica_view(base, reps[valid ? atom_rep[i] : 0]);
    load_atom(a, i, valid, pos_in, vel_in);
}

__global__ void __launch_bounds__(kBlock) k_batch_integrate(SimArgs base, const Replica* __restrict__ reps,
                                                            const int* __restrict__ atom_rep) {
    if (base.hdr[HDR_STATE] != STATE_FORCES || (base.hdr[HDR_ERROR] & DEV_ORDER)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&base.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < base.n;
    const SimArgs a = replica_view(base, reps[valid ? atom_rep[i] : 0]);
    integrate_atom(a, i, valid);
}

// Batch set-up: per-atom and per-cell replica tables and the batch marker in
// the header (k_build_init has cleared the rest). One workgroup per replica.
__global__ void __launch_bounds__(kBlock) k_batch_setup(SimArgs base, const Replica* __restrict__ reps,
                                                        int* __restrict__ atom_rep, int* __restrict__ cell_rep,
                                                        int* __restrict__ class_cells, int count) {
    const int b = blockIdx.x;
    const Replica r = reps[b];
    if (b == 0 && threadIdx.x == 0) base.hdr[HDR_NC] = -count;  // marks a batch workspace
    for (int i = threadIdx.x; i < r.n; i += kBlock) atom_rep[r.abase + i] = b;
    for (int c = threadIdx.x; c < r.ncells; c += kBlock) {
        cell_rep[r.cbase + c] = b;
        if (class_cells) class_cells[r.lbase + c] = r.cbase + c;
    }
}

// Block scan: bstart[b] = atoms in the cells of blocks 0 .. b - 1 (16 cells
// a block), for grids of more than kDirectBlocks blocks. Workgroup g of 1024
// lanes owns tile g of kScanTile blocks; a lane reads kScanBlocks whole
// blocks as consecutive int4 (adjacent lanes read adjacent 128-byte runs),
// all loads issued before any arithmetic, and a wavefront scan plus a scan of
// the 16 wave totals give each block's offset within the tile. Two launches:
// PHASE 0 stores each tile's total, PHASE 1 adds the totals of the tiles
// before its own (read by every workgroup; there are at most a few thousand)
// and writes bstart. The tile totals live in the block-count array, which
// the binning only fills on grids of at most kDirectBlocks blocks.
constexpr int kScanBlock = 1024;
constexpr int kScanBlocks = 2;                          // blocks per lane per tile
constexpr int kScanTile = kScanBlock * kScanBlocks;      // 2048 blocks = 32768 cells
constexpr int kBlockInts = 1 << kBlockShift;
template <int PHASE>
__global__ void __launch_bounds__(kScanBlock) k_block_scan(SimArgs a, bool from_step) {
    __shared__ int wave_tot[kScanBlock / kWave];
    __shared__ int wave_carry[kScanBlock / kWave];
    const int err = a.hdr[HDR_ERROR];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nb = a.nblocks;
    const int g = blockIdx.x;
    int* tile_tot_arr = a.bcounts;
    const int b0 = g * kScanTile + tid * kScanBlocks;
    int4 v[kScanBlocks * kBlockInts / 4];
#pragma unroll
    for (int q = 0; q < kScanBlocks * kBlockInts / 4; ++q) {
        // counts holds whole blocks (zero past the last cell)
        v[q] = (b0 + q / (kBlockInts / 4) < nb) ? reinterpret_cast<const int4*>(a.counts)[b0 * (kBlockInts / 4) + q]
                                                : make_int4(0, 0, 0, 0);
    }
    int carry = 0;
    if (PHASE == 1) {
        for (int k = tid; k < g; k += kScanBlock) carry += tile_tot_arr[k];
    }
    if (from_step && (err & DEV_ORDER)) return;  // uniform over the grid
    int bsum[kScanBlocks];
    int tsum = 0;
#pragma unroll
    for (int j = 0; j < kScanBlocks; ++j) {
        int t = 0;
#pragma unroll
        for (int q = 0; q < kBlockInts / 4; ++q) {
            const int4 x = v[j * (kBlockInts / 4) + q];
            t += x.x + x.y + x.z + x.w;
        }
        bsum[j] = t;
        tsum += t;
    }
    const int incl = wave_incl_scan(tsum);
    if (lane == kWave - 1) wave_tot[wave] = incl;
    if (PHASE == 1) {
        carry = wave_sum_int(carry);
        if (lane == 0) wave_carry[wave] = carry;
    }
    __syncthreads();
    int wave_off = 0, tile_tot = 0, before = 0;
#pragma unroll
    for (int k = 0; k < kScanBlock / kWave; ++k) {
        const int t = wave_tot[k];
        if (k < wave) wave_off += t;
        tile_tot += t;
        if (PHASE == 1) before += wave_carry[k];
    }
    if (PHASE == 0) {
        if (tid == 0) tile_tot_arr[g] = tile_tot;
        return;
    }
    int run = before + wave_off + incl - tsum;
#pragma unroll
    for (int j = 0; j < kScanBlocks; ++j) {
        if (b0 + j < nb) a.bstart[b0 + j] = run;
        run += bsum[j];
    }
}

// Cell order. Workgroup b owns cells c0 = 16 b .. c0 + 15 (one block of the
// block histogram): the offset of cell c is bstart[b] plus the owned cells
// before c. For a batch the cells of all replicas are one sequence, so the
// offset of a replica's first cell is its first atom. The workgroup writes
// its cells' offsets and clears their counts.
// Members of a cell are bucket entries 0 .. min(n, cap) - 1 and the cell's
// entries of the overflow list beyond that. They are ranked by user index and
// moved to pos0/vel0[start + rank], which makes the sorted layout independent
// of the arrival order of the binning atomics. One 16-lane group per cell; a
// lane holds two members (sub and sub + 16) of each 32-member window, and a
// member's rank counts the smaller indices of its cell, read four at a time
// from the window's indices in LDS. Loop bounds are the workgroup's largest
// cell, so the barriers are uniform.
constexpr int kOrderBlock = 256;
constexpr int kOrderGroup = 16;
constexpr int kOrderWin = 2 * kOrderGroup;
constexpr int kOrderCells = kOrderBlock / kOrderGroup;
constexpr int kNoId = 0x7fffffff;  // larger than any user index

// Member m of cell c: bucket entry m, or past the capacity the cell's
// (m - cap)-th overflow entry, found through the per-cell overflow index the
// workgroup built (ovf0: the cell's first slot there). Both indices are
// clamped to the arrays: a histogram and list that disagree (a call sequence
// cut short, reported as DEV_ORDER) give a wrong but in-bounds member.
__device__ __forceinline__ int overflow_slot(const SimArgs& a, int m, int ovf0) {
    const int k = min(ovf0 + m - a.cap, a.natoms - 1);
    return min(max(a.ovf_idx[k], 0), a.natoms - 1);
}

__device__ __forceinline__ void load_member(const SimArgs& a, int c, int m, int ovf0, float4& p, float4& v) {
    if (m < a.cap) {
        const size_t e = static_cast<size_t>(c) * a.cap + m;
        p = a.bpos[e];
        v = a.bvel[e];
    } else {
        const int j = overflow_slot(a, m, ovf0);
        p = a.pos1[j];
        v = a.vel1[j];
    }
}

__device__ __forceinline__ int member_id(const SimArgs& a, int c, int m, int n, int ovf0) {
    if (m >= n) return kNoId;
    const float4 p = m < a.cap ? a.bpos[static_cast<size_t>(c) * a.cap + m] : a.pos1[overflow_slot(a, m, ovf0)];
    return __float_as_int(p.w);
}

__device__ __forceinline__ int count_below(int4 k, int id) {
    return (k.x < id ? 1 : 0) + (k.y < id ? 1 : 0) + (k.z < id ? 1 : 0) + (k.w < id ? 1 : 0);
}

__global__ void __launch_bounds__(kOrderBlock) k_cell_order(SimArgs a, bool from_step) {
    static_assert(kOrderCells == (1 << kBlockShift), "a cell-order workgroup owns one histogram block");
    __shared__ int4 win[kOrderCells][kOrderWin / 4];
    __shared__ int cnt_s[kOrderCells];
    __shared__ int part_s[kOrderBlock / kWave];
    __shared__ int ovf_base_s;
    const int err = a.hdr[HDR_ERROR];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int cl = tid / kOrderGroup, sub = tid & (kOrderGroup - 1);
    // blocks in the force kernel's XCD order: the cells a workgroup orders are
    // those whose bins the same XCD's force waves filled, and whose sorted
    // arrays its next force waves stage
    const int blk = xcd_block_order(blockIdx.x, gridDim.x);
    const int c0 = blk * kOrderCells, c = c0 + cl;
    const int nct = a.ncells;
    // What the first window needs is requested before anything waits: the
    // cell's count, its first 16 bucket entries (a cell of the headline
    // density holds about 15 atoms; entries past the count are never used),
    // and the block offset (or the block counts before this block). Entries
    // 16..31 are loaded once the count shows that they exist, while the block
    // counts are still in flight: loading them unconditionally read twice the
    // bucket bytes the cells hold.
    const int n = c < nct ? a.counts[c] : 0;
    float4 pa0 = make_float4(0.f, 0.f, 0.f, 0.f), va0 = pa0, pb0 = pa0, vb0 = pa0;
    const size_t e0 = static_cast<size_t>(c) * a.cap + sub;
    if (c < nct) {
        pa0 = a.bpos[e0];
        va0 = a.bvel[e0];
    }
    int part = 0;
    if (a.direct) {
        // all loads in flight at once (a loop bounded by blockIdx.x waited for
        // each before the next)
        static_assert(kDirectBlocks % kOrderBlock == 0, "direct block sums take whole rounds");
        const int* bc = a.bcounts + a.par * a.nbstride;
        int v[kDirectBlocks / kOrderBlock];
#pragma unroll
        for (int u = 0; u < kDirectBlocks / kOrderBlock; ++u) {
            const int j = tid + u * kOrderBlock;
            v[u] = j < blk ? bc[j] : 0;
        }
        if (sub + kOrderGroup < n) {  // c < nct whenever n > 0
            pb0 = a.bpos[e0 + kOrderGroup];
            vb0 = a.bvel[e0 + kOrderGroup];
        }
#pragma unroll
        for (int u = 0; u < kDirectBlocks / kOrderBlock; ++u) part += v[u];
    } else if (sub + kOrderGroup < n) {
        pb0 = a.bpos[e0 + kOrderGroup];
        vb0 = a.bvel[e0 + kOrderGroup];
    }
    const int bs = a.direct ? 0 : a.bstart[blk];
    const int novf = min(a.hdr[HDR_OVF + a.par], a.natoms);
    if (from_step && (err & DEV_ORDER)) return;  // uniform over the workgroup
    part = wave_sum_int(part);
    if (lane == 0) part_s[wave] = part;
    if (sub == 0) cnt_s[cl] = n;
    __syncthreads();
    int first = a.direct ? part_s[0] + part_s[1] + part_s[2] + part_s[3] : bs;
    for (int j = 0; j < cl; ++j) first += cnt_s[j];
    int nmax = 0;
#pragma unroll
    for (int j = 0; j < kOrderCells; ++j) nmax = max(nmax, cnt_s[j]);
    if (c < nct && sub == 0) {
        a.start[c] = first;
        if (c == nct - 1) a.start[nct] = first + n;
        a.counts[c] = 0;  // the next build's histogram
    }
    // the other parity's counters, for the next build
    if (a.direct && tid == 0) a.bcounts[(1 - a.par) * a.nbstride + blk] = 0;
    if (blockIdx.x == 0 && tid == 0) {
        a.hdr[HDR_OVF + 1 - a.par] = 0;
        a.hdr[HDR_OVFA + 1 - a.par] = 0;
    }
    // Cells past the bucket capacity (rare): the workgroup takes a range of
    // the overflow index, scans the overflow list once and files each entry of
    // its cells under (cell, overflow rank), so that a member past the
    // capacity is one indexed load away, at any cell size.
    int ovf0 = 0;
    if (nmax > a.cap) {  // uniform over the workgroup
        int before = 0, ovf_tot = 0;
#pragma unroll
        for (int j = 0; j < kOrderCells; ++j) {
            const int e = max(0, cnt_s[j] - a.cap);
            if (j < cl) before += e;
            ovf_tot += e;
        }
        if (tid == 0) ovf_base_s = atomicAdd(&a.hdr[HDR_OVFA + a.par], ovf_tot);
        __syncthreads();
        const int base = ovf_base_s;
        ovf0 = base + before;
        for (int j = tid; j < novf; j += kOrderBlock) {
            const int cj = a.ovf_cell[j];
            if (cj < c0 || cj >= c0 + kOrderCells) continue;
            int off = base;
            for (int q = 0; q < cj - c0; ++q) off += max(0, cnt_s[q] - a.cap);
            const int slot = off + a.ovf_rank[j];
            if (slot >= 0 && slot < a.natoms) a.ovf_idx[slot] = j;
        }
        __threadfence_block();
        __syncthreads();
    }
    int* wids = reinterpret_cast<int*>(win[cl]);
    for (int m0 = 0; m0 < nmax; m0 += kOrderWin) {
        const int ma = m0 + sub, mb = ma + kOrderGroup;
        float4 pa = pa0, va = va0, pb = pb0, vb = vb0;
        if (m0 > 0) {
            if (ma < n) load_member(a, c, ma, ovf0, pa, va);
            if (mb < n) load_member(a, c, mb, ovf0, pb, vb);
        }
        const int ida = ma < n ? __float_as_int(pa.w) : kNoId;
        const int idb = mb < n ? __float_as_int(pb.w) : kNoId;
        int ra = 0, rb = 0;
        for (int k0 = 0; k0 < nmax; k0 += kOrderWin) {
            int ka = ida, kb = idb;
            if (k0 != m0) {
                ka = member_id(a, c, k0 + sub, n, ovf0);
                kb = member_id(a, c, k0 + kOrderGroup + sub, n, ovf0);
            }
            __syncthreads();  // the previous window has been read
            wids[sub] = ka;
            wids[kOrderGroup + sub] = kb;
            __syncthreads();
            const int kn = min(kOrderWin, nmax - k0);
            for (int l = 0; l < kn; l += 4) {
                const int4 k4 = win[cl][l / 4];
                ra += count_below(k4, ida);
                rb += count_below(k4, idb);
            }
        }
        // (a consistent histogram keeps first + n within the atoms; the guard
        // keeps an inconsistent one from writing past them)
        if (ma < n && first + ra < a.natoms) {
            a.pos0[first + ra] = pa;
            a.vel0[first + ra] = va;
        }
        if (mb < n && first + rb < a.natoms) {
            a.pos0[first + rb] = pb;
            a.vel0[first + rb] = vb;
        }
    }
    if (blockIdx.x == 0 && tid == 0 && !from_step) a.hdr[HDR_STATE] = STATE_CELLS;
}

__global__ void __launch_bounds__(kBlock) k_gather_user(SimArgs a, float4* pos_out, float4* vel_out,
                                                        float4* force_out) {
    if (!state_ok(a, force_out != nullptr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.n) return;
    const float4 p = a.pos0[k];
    const int id = __float_as_int(p.w);
    if (id < 0 || id >= a.n) return;
    if (pos_out) pos_out[id] = make_float4(p.x, p.y, p.z, 0.f);
    if (vel_out) {
        const float4 v = a.vel0[k];
        vel_out[id] = make_float4(v.x, v.y, v.z, 0.f);
    }
    if (force_out) {
        const float4 f = a.force[k];
        force_out[id] = make_float4(f.x, f.y, f.z, 0.f);
    }
}

__global__ void __launch_bounds__(kBlock) k_cell_lists(SimArgs a, int* cell_start, int* order) {
    if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (cell_start && k <= a.ncells) cell_start[k] = a.start[k];
    if (order && k < a.n) order[k] = __float_as_int(a.pos0[k].w);
}

inline int blocks_for(int n, int b) { return (n + b - 1) / b; }

inline int clamp_blocks(int b) { return b < 1 ? 1 : (b > 4096 ? 4096 : b); }

inline SimArgs with_par(const SimArgs& a, int par) {
    SimArgs b = a;
    b.par = par;
    return b;
}

}  // namespace

hipError_t launch_build_init(const SimArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_build_init, dim3(clamp_blocks(blocks_for(a.ncells, kBlock))), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_load(const SimArgs& a, const float4* pos_in, const float4* vel_in, hipStream_t st) {
    hipLaunchKernelGGL(k_load, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, with_par(a, 0), pos_in, vel_in);
    return hipGetLastError();
}

hipError_t launch_integrate(const SimArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_integrate, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, with_par(a, 0));
    return hipGetLastError();
}

hipError_t launch_block_scan(const SimArgs& a, bool from_step, hipStream_t st) {
    const int tiles = (a.nblocks + kScanTile - 1) / kScanTile;  // <= 2 nbstride: the tile totals fit
    hipLaunchKernelGGL(k_block_scan<0>, dim3(tiles), dim3(kScanBlock), 0, st, a, from_step);
    hipLaunchKernelGGL(k_block_scan<1>, dim3(tiles), dim3(kScanBlock), 0, st, a, from_step);
    return hipGetLastError();
}

hipError_t launch_cell_order(const SimArgs& a, int par, bool from_step, hipStream_t st) {
    hipLaunchKernelGGL(k_cell_order, dim3(a.nblocks), dim3(kOrderBlock), 0, st, with_par(a, par), from_step);
    return hipGetLastError();
}

hipError_t launch_set_state(const SimArgs& a, int state, hipStream_t st) {
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(kWave), 0, st, a, state);
    return hipGetLastError();
}

hipError_t launch_zero_blocks(const SimArgs& a, int par, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_blocks, dim3(clamp_blocks(blocks_for(a.nbstride, kBlock))), dim3(kBlock), 0, st, a,
                       par);
    return hipGetLastError();
}

hipError_t launch_gather_user(const SimArgs& a, float4* pos_out, float4* vel_out, float4* force_out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_gather_user, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, a, pos_out,
                       vel_out, force_out);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const SimArgs& base, const Replica* reps, int* atom_rep, int* cell_rep,
                              int* class_cells, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_setup, dim3(count), dim3(kBlock), 0, st, base, reps, atom_rep, cell_rep, class_cells,
                       count);
    return hipGetLastError();
}

hipError_t launch_batch_load(const SimArgs& base, const Replica* reps, const int* atom_rep, const float4* pos_in,
                             const float4* vel_in, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_load, dim3(blocks_for(base.n, kBlock)), dim3(kBlock), 0, st, with_par(base, 0), reps,
                       atom_rep, pos_in, vel_in);
    return hipGetLastError();
}

hipError_t launch_batch_integrate(const SimArgs& base, const Replica* reps, const int* atom_rep, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_integrate, dim3(blocks_for(base.n, kBlock)), dim3(kBlock), 0, st, with_par(base, 0),
                       reps, atom_rep);
    return hipGetLastError();
}

hipError_t launch_cell_lists(const SimArgs& a, int* cell_start, int* order, hipStream_t st) {
    const int m = (a.n > a.ncells + 1) ? a.n : a.ncells + 1;
    hipLaunchKernelGGL(k_cell_lists, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, st, a, cell_start, order);
    return hipGetLastError();
}

}  // namespace mdlj
