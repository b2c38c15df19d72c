// Cell-list build by counting sort (section 3 cells of side >= r_c; section
// 3.1 membership kept current as particles move), and the velocity-Verlet
// drift that feeds it (section 2).
//
// One build is four launches, all HBM/L2-bound streaming passes:
//   load or drift : wrap + cell index + histogram rank (one atomic per run of
//                   equal cells in a wavefront); inside a multi-step run the
//                   force kernel's epilogue does this for every step after
//                   the first, and the drift kernel only starts a run
//   scan          : exclusive prefix of the histogram -> cell offsets;
//                   clears the histogram for the next build
//   scatter       : key[offset + rank] = staging slot
//   cell order    : a 16-lane group per cell orders its members by user
//                   index and moves them into the sorted arrays
// The paper updated each cell with one serial thread per cell (section 3.1);
// a counting sort has no serial part and no capacity per cell.
#include "md_device.h"

namespace mdlj {

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_build_init(SimArgs a) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t == 0) {
        a.hdr[HDR_ERROR] = 0;
        a.hdr[HDR_STATE] = STATE_BUILDING;
        a.hdr[HDR_N] = a.n;
        a.hdr[HDR_NC] = a.nc;
    }
    for (int c = t; c < a.ncells; c += gridDim.x * kBlock) a.count[c] = 0;
}

// Load one user-order atom i into the staging arrays: wrap, cell index,
// rank. Called by every lane of the wave (valid = false for lanes past the
// end); cells are numbered globally (a.cbase + local index).
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
    const int r = histogram_rank(a.count, c);
    if (valid) {
        a.pos1[i] = p;
        a.vel1[i] = v;
        a.cell[i] = c;
        a.rank[i] = r;
    }
}

// Velocity-Verlet first half for sorted slot i (half kick, drift, wrap),
// then the histogram rank for the rebuild. Reads the sorted state, writes
// staging. Called by every lane of the wave.
__device__ __forceinline__ void integrate_atom(const SimArgs& a, int i, bool valid) {
    int c = -1;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), v = p;
    if (valid) {
        p = a.pos0[i];
        v = a.vel0[i];
        const float4 f = a.force[i];
        c = half_kick_drift(a, p, v, f.x, f.y, f.z);
    }
    const int r = histogram_rank(a.count, c);
    if (valid) {
        a.pos1[i] = p;
        a.vel1[i] = v;
        a.cell[i] = c;
        a.rank[i] = r;
    }
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

// Batch set-up: per-atom and per-cell replica tables, zero histogram, header.
// One workgroup per replica.
__global__ void __launch_bounds__(kBlock) k_batch_setup(SimArgs base, const Replica* __restrict__ reps,
                                                        int* __restrict__ atom_rep, int* __restrict__ cell_rep,
                                                        int count) {
    const int b = blockIdx.x;
    const Replica r = reps[b];
    if (b == 0 && threadIdx.x == 0) {
        base.hdr[HDR_ERROR] = 0;
        base.hdr[HDR_STATE] = STATE_BUILDING;
        base.hdr[HDR_N] = base.n;
        base.hdr[HDR_NC] = -count;  // marks a batch workspace
    }
    for (int i = threadIdx.x; i < r.n; i += kBlock) atom_rep[r.abase + i] = b;
    for (int c = threadIdx.x; c < r.ncells; c += kBlock) {
        cell_rep[r.cbase + c] = b;
        base.count[r.cbase + c] = 0;
    }
}

// Batched scan: one workgroup per replica scans its own histogram into
// start[cbase .. cbase + ncells) (global slots: abase + prefix) and clears it;
// the last replica also writes the terminal entry.
__global__ void __launch_bounds__(kBlock) k_batch_scan(SimArgs base, const Replica* __restrict__ reps, int count) {
    if (base.hdr[HDR_ERROR] & DEV_ORDER) return;
    __shared__ int wave_tot[kBlock / kWave];
    const Replica r = reps[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    int carry = r.abase;
    for (int base_c = 0; base_c < r.ncells; base_c += kBlock) {
        const int c = base_c + tid;
        const int v = (c < r.ncells) ? base.count[r.cbase + c] : 0;
        const int incl = wave_incl_scan(v);
        if (lane == kWave - 1) wave_tot[wave] = incl;
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            const int t = wave_tot[w];
            if (w < wave) off += t;
            tot += t;
        }
        if (c < r.ncells) {
            base.start[r.cbase + c] = carry + off + incl - v;
            base.count[r.cbase + c] = 0;
        }
        carry += tot;
        __syncthreads();
    }
    if (blockIdx.x == count - 1 && tid == 0) base.start[r.cbase + r.ncells] = carry;
}

// Exclusive prefix scan of the histogram into start[0..ncells], by one
// workgroup of 1024 lanes. One workgroup runs on one CU, whose memory pipeline
// serves a few cache lines per clock, so every global access here is a
// coalesced int4 (consecutive lanes, consecutive 16 bytes) and the transpose
// to "each lane owns 4 kScanVec consecutive cells" goes through LDS. Per tile of
// 4096 kScanVec cells: coalesced loads into LDS, per-lane sums, a wavefront
// scan and a scan of the 16 wave totals, exclusive offsets back into LDS,
// coalesced stores of the offsets and of zeros into the histogram (cleared
// for the next build). A carry links the tiles.
constexpr int kScanBlock = 1024;
constexpr int kScanVec = 3;                       // int4 per lane per tile
constexpr int kScanTile = kScanBlock * 4 * kScanVec;  // 12288 cells, 48 KiB of LDS
__global__ void __launch_bounds__(kScanBlock) k_scan(SimArgs a, bool from_step) {
    __shared__ int4 buf[kScanTile / 4];
    __shared__ int wave_tot[kScanBlock / kWave];
    const int err = a.hdr[HDR_ERROR];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nc = a.ncells;
    int carry = 0;
    for (int base = 0; base < nc; base += kScanTile) {
        int4 v[kScanVec];
#pragma unroll
        for (int q = 0; q < kScanVec; ++q) {
            const int c = base + 4 * (q * kScanBlock + tid);
            if (c + 3 < nc) {
                v[q] = *reinterpret_cast<const int4*>(a.count + c);
            } else {
                v[q].x = c < nc ? a.count[c] : 0;
                v[q].y = c + 1 < nc ? a.count[c + 1] : 0;
                v[q].z = c + 2 < nc ? a.count[c + 2] : 0;
                v[q].w = 0;
            }
        }
        if (from_step && (err & DEV_ORDER)) return;  // uniform over the workgroup
#pragma unroll
        for (int q = 0; q < kScanVec; ++q) buf[q * kScanBlock + tid] = v[q];
        __syncthreads();
        // this lane's cells: tile entries kScanVec * tid .. + kScanVec - 1
        int4 w[kScanVec];
        int tsum = 0;
#pragma unroll
        for (int q = 0; q < kScanVec; ++q) {
            w[q] = buf[kScanVec * tid + q];
            tsum += w[q].x + w[q].y + w[q].z + w[q].w;
        }
        const int incl = wave_incl_scan(tsum);
        if (lane == kWave - 1) wave_tot[wave] = incl;
        __syncthreads();
        int wave_off = 0, tile_tot = 0;
#pragma unroll
        for (int k = 0; k < kScanBlock / kWave; ++k) {
            const int t = wave_tot[k];
            if (k < wave) wave_off += t;
            tile_tot += t;
        }
        int run = carry + wave_off + incl - tsum;
#pragma unroll
        for (int q = 0; q < kScanVec; ++q) {
            const int s0 = run, s1 = s0 + w[q].x, s2 = s1 + w[q].y, s3 = s2 + w[q].z;
            run = s3 + w[q].w;
            buf[kScanVec * tid + q] = make_int4(s0, s1, s2, s3);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kScanVec; ++q) {
            const int c = base + 4 * (q * kScanBlock + tid);
            const int4 o = buf[q * kScanBlock + tid];
            if (c + 3 < nc) {
                *reinterpret_cast<int4*>(a.start + c) = o;
                *reinterpret_cast<int4*>(a.count + c) = make_int4(0, 0, 0, 0);
            } else {
                if (c < nc) { a.start[c] = o.x; a.count[c] = 0; }
                if (c + 1 < nc) { a.start[c + 1] = o.y; a.count[c + 1] = 0; }
                if (c + 2 < nc) { a.start[c + 2] = o.z; a.count[c + 2] = 0; }
            }
        }
        carry += tile_tot;
        __syncthreads();
    }
    if (tid == 0) a.start[nc] = carry;
}

// The error word is read alongside the kernels' first loads (not before them),
// so a pending order error costs no extra memory round trip; nothing is
// written, and nothing is read through a loaded index, once it is seen.
__global__ void __launch_bounds__(kBlock) k_scatter(SimArgs a, bool from_step) {
    const int err = a.hdr[HDR_ERROR];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    int c = 0, r = 0;
    if (i < a.n) {
        c = a.cell[i];
        r = a.rank[i];
    }
    if (from_step && (err & DEV_ORDER)) return;
    if (i < a.n) a.key[a.start[c] + r] = i;
}

// In-cell order: the members of cell c (staging slots key[start .. start + n))
// are ranked by user index and moved to pos0/vel0[start + rank], which makes
// the sorted layout independent of the arrival order of the histogram
// atomics. One 16-lane group per cell, 16 cells per workgroup; a lane holds
// two members (sub and sub + 16) of each 32-member window. A member's rank
// counts the smaller indices of its cell: each window's indices are put in
// LDS and every lane reads them back four at a time (a broadcast within the
// group). Loop bounds are the workgroup's largest cell, so the barriers are
// uniform.
constexpr int kOrderBlock = 256;
constexpr int kOrderGroup = 16;
constexpr int kOrderWin = 2 * kOrderGroup;
constexpr int kOrderCells = kOrderBlock / kOrderGroup;
constexpr int kNoId = 0x7fffffff;  // larger than any user index

__device__ __forceinline__ int staged_id(const SimArgs& a, int first, int m, int n) {
    return m < n ? __float_as_int(a.pos1[a.key[first + m]].w) : kNoId;
}

__device__ __forceinline__ int count_below(int4 k, int id) {
    return (k.x < id ? 1 : 0) + (k.y < id ? 1 : 0) + (k.z < id ? 1 : 0) + (k.w < id ? 1 : 0);
}

__global__ void __launch_bounds__(kOrderBlock) k_cell_order(SimArgs a, bool from_step) {
    __shared__ int4 win[kOrderCells][kOrderWin / 4];
    __shared__ int wave_max[kOrderBlock / kWave];
    const int err = a.hdr[HDR_ERROR];
    const int cl = threadIdx.x / kOrderGroup;
    const int c = blockIdx.x * kOrderCells + cl;
    const int sub = threadIdx.x & (kOrderGroup - 1);
    int first = 0, n = 0;
    if (c < a.ncells) {
        first = a.start[c];
        n = a.start[c + 1] - first;
    }
    if (from_step && (err & DEV_ORDER)) return;  // uniform over the workgroup
    int nmax = max(n, __shfl_xor(n, 16));
    nmax = max(nmax, __shfl_xor(nmax, 32));
    if ((threadIdx.x & (kWave - 1)) == 0) wave_max[threadIdx.x / kWave] = nmax;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kOrderBlock / kWave; ++w) nmax = max(nmax, wave_max[w]);
    int* wids = reinterpret_cast<int*>(win[cl]);
    for (int m0 = 0; m0 < nmax; m0 += kOrderWin) {
        const int ma = m0 + sub, mb = ma + kOrderGroup;
        float4 pa = make_float4(0.f, 0.f, 0.f, 0.f), va = pa, pb = pa, vb = pa;
        int ida = kNoId, idb = kNoId;
        if (ma < n) {
            const int src = a.key[first + ma];
            pa = a.pos1[src];
            va = a.vel1[src];
            ida = __float_as_int(pa.w);
        }
        if (mb < n) {
            const int src = a.key[first + mb];
            pb = a.pos1[src];
            vb = a.vel1[src];
            idb = __float_as_int(pb.w);
        }
        int ra = 0, rb = 0;
        for (int k0 = 0; k0 < nmax; k0 += kOrderWin) {
            int ka = ida, kb = idb;
            if (k0 != m0) {
                ka = staged_id(a, first, k0 + sub, n);
                kb = staged_id(a, first, k0 + kOrderGroup + sub, n);
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
        if (ma < n) {
            a.pos0[first + ra] = pa;
            a.vel0[first + ra] = va;
        }
        if (mb < n) {
            a.pos0[first + rb] = pb;
            a.vel0[first + rb] = vb;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && !from_step) a.hdr[HDR_STATE] = STATE_CELLS;
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

}  // namespace

hipError_t launch_build_init(const SimArgs& a, hipStream_t st) {
    int g = blocks_for(a.ncells, kBlock);
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_build_init, dim3(g), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_load(const SimArgs& a, const float4* pos_in, const float4* vel_in, hipStream_t st) {
    hipLaunchKernelGGL(k_load, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, a, pos_in, vel_in);
    return hipGetLastError();
}

hipError_t launch_integrate(const SimArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_integrate, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_scan(const SimArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanBlock), 0, st, a, true);
    return hipGetLastError();
}

hipError_t launch_scatter(const SimArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, a, true);
    return hipGetLastError();
}

hipError_t launch_cell_order(const SimArgs& a, bool from_step, hipStream_t st) {
    hipLaunchKernelGGL(k_cell_order, dim3(blocks_for(a.ncells, kOrderCells)), dim3(kOrderBlock), 0, st, a,
                       from_step);
    return hipGetLastError();
}

hipError_t launch_gather_user(const SimArgs& a, float4* pos_out, float4* vel_out, float4* force_out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_gather_user, dim3(blocks_for(a.n, kBlock)), dim3(kBlock), 0, st, a, pos_out,
                       vel_out, force_out);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const SimArgs& base, const Replica* reps, int* atom_rep, int* cell_rep, int count,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_batch_setup, dim3(count), dim3(kBlock), 0, st, base, reps, atom_rep, cell_rep, count);
    return hipGetLastError();
}

hipError_t launch_batch_load(const SimArgs& base, const Replica* reps, const int* atom_rep, const float4* pos_in,
                             const float4* vel_in, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_load, dim3(blocks_for(base.n, kBlock)), dim3(kBlock), 0, st, base, reps, atom_rep,
                       pos_in, vel_in);
    return hipGetLastError();
}

hipError_t launch_batch_integrate(const SimArgs& base, const Replica* reps, const int* atom_rep, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_integrate, dim3(blocks_for(base.n, kBlock)), dim3(kBlock), 0, st, base, reps,
                       atom_rep);
    return hipGetLastError();
}

hipError_t launch_batch_scan(const SimArgs& base, const Replica* reps, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_scan, dim3(count), dim3(kBlock), 0, st, base, reps, count);
    return hipGetLastError();
}

hipError_t launch_cell_lists(const SimArgs& a, int* cell_start, int* order, hipStream_t st) {
    const int m = (a.n > a.ncells + 1) ? a.n : a.ncells + 1;
    hipLaunchKernelGGL(k_cell_lists, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, st, a, cell_start, order);
    return hipGetLastError();
}

}  // namespace mdlj
