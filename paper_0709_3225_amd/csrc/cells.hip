// Cell-list build by counting sort (section 3 cells of side >= r_c; section
// 3.1 membership kept current as particles move), and the velocity-Verlet
// drift that feeds it (section 2).
//
// One build is four launches, all HBM/L2-bound streaming passes:
//   load or integrate : wrap + cell index + histogram rank (one atomic per
//                       run of equal cells in a wavefront)
//   scan              : exclusive prefix of the histogram -> cell offsets;
//                       clears the histogram for the next build
//   scatter           : key[offset + rank] = staging slot
//   cell order        : one wavefront per cell orders its members by user
//                       index and moves them into the sorted arrays
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

// Velocity-Verlet first half for sorted slot i: v += dt/(2m) F, r += dt v,
// wrap, then the histogram rank for the rebuild. Reads the sorted state,
// writes staging. Called by every lane of the wave.
__device__ __forceinline__ void integrate_atom(const SimArgs& a, int i, bool valid) {
    const float invL = 1.0f / a.box;
    int c = -1;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), v = p;
    if (valid) {
        p = a.pos0[i];
        v = a.vel0[i];
        const float4 f = a.force[i];
        v.x += a.hdt_m * f.x;
        v.y += a.hdt_m * f.y;
        v.z += a.hdt_m * f.z;
        p.x += a.dt * v.x;
        p.y += a.dt * v.y;
        p.z += a.dt * v.z;
        if (!finite3(p.x, p.y, p.z)) {
            atomicOr(&a.hdr[HDR_ERROR], DEV_NONFINITE);
            p.x = p.y = p.z = 0.f;
        }
        p.x = wrap_coord(p.x, a.box, invL);
        p.y = wrap_coord(p.y, a.box, invL);
        p.z = wrap_coord(p.z, a.box, invL);
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
// workgroup of 1024 lanes walking the histogram in tiles of 4096 cells:
// per-lane sums of four cells, a wavefront scan, a scan of the 16 wave totals,
// and a running carry. Clears the histogram behind it.
constexpr int kScanBlock = 1024;
__global__ void __launch_bounds__(kScanBlock) k_scan(SimArgs a, bool from_step) {
    if (from_step && (a.hdr[HDR_ERROR] & DEV_ORDER)) return;
    __shared__ int wave_tot[kScanBlock / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    int carry = 0;
    for (int base = 0; base < a.ncells; base += kScanBlock * 4) {
        const int c0 = base + tid * 4;
        int v0 = 0, v1 = 0, v2 = 0, v3 = 0;
        if (c0 + 3 < a.ncells) {
            const int4 v = *reinterpret_cast<const int4*>(a.count + c0);
            v0 = v.x; v1 = v.y; v2 = v.z; v3 = v.w;
        } else {
            if (c0 < a.ncells) v0 = a.count[c0];
            if (c0 + 1 < a.ncells) v1 = a.count[c0 + 1];
            if (c0 + 2 < a.ncells) v2 = a.count[c0 + 2];
        }
        const int tsum = v0 + v1 + v2 + v3;
        const int incl = wave_incl_scan(tsum);
        if (lane == kWave - 1) wave_tot[wave] = incl;
        __syncthreads();
        int wave_off = 0, tile_tot = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) {
            const int t = wave_tot[w];
            if (w < wave) wave_off += t;
            tile_tot += t;
        }
        const int excl = carry + wave_off + incl - tsum;
        if (c0 + 3 < a.ncells) {
            *reinterpret_cast<int4*>(a.start + c0) = make_int4(excl, excl + v0, excl + v0 + v1, excl + v0 + v1 + v2);
            *reinterpret_cast<int4*>(a.count + c0) = make_int4(0, 0, 0, 0);
        } else {
            if (c0 < a.ncells) { a.start[c0] = excl; a.count[c0] = 0; }
            if (c0 + 1 < a.ncells) { a.start[c0 + 1] = excl + v0; a.count[c0 + 1] = 0; }
            if (c0 + 2 < a.ncells) { a.start[c0 + 2] = excl + v0 + v1; a.count[c0 + 2] = 0; }
        }
        carry += tile_tot;
        __syncthreads();
    }
    if (tid == 0) a.start[a.ncells] = carry;
}

__global__ void __launch_bounds__(kBlock) k_scatter(SimArgs a, bool from_step) {
    if (from_step && (a.hdr[HDR_ERROR] & DEV_ORDER)) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < a.n) a.key[a.start[a.cell[i]] + a.rank[i]] = i;
}

// One wavefront per cell: rank every member by user index among the cell's
// members (ids are unique), then move position and velocity to
// start + rank. Chunks of 64 members; ids of other chunks are fetched and
// broadcast lane by lane.
__global__ void __launch_bounds__(kWave) k_cell_order(SimArgs a, bool from_step) {
    if (from_step && (a.hdr[HDR_ERROR] & DEV_ORDER)) return;
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const int first = a.start[c];
    const int n = a.start[c + 1] - first;
    for (int m0 = 0; m0 < n; m0 += kWave) {
        const int m = m0 + lane;
        const bool act = m < n;
        float4 p = make_float4(0.f, 0.f, 0.f, 0.f), v = p;
        if (act) {
            const int src = a.key[first + m];
            p = a.pos1[src];
            v = a.vel1[src];
        }
        const int myid = act ? __float_as_int(p.w) : 0x7fffffff;
        int r = 0;
        for (int k0 = 0; k0 < n; k0 += kWave) {
            int kid;
            if (k0 == m0) {
                kid = myid;
            } else {
                kid = (k0 + lane < n) ? __float_as_int(a.pos1[a.key[first + k0 + lane]].w) : 0x7fffffff;
            }
            const int kn = min(kWave, n - k0);
            for (int l = 0; l < kn; ++l) r += (__shfl(kid, l) < myid) ? 1 : 0;
        }
        if (act) {
            a.pos0[first + r] = p;
            a.vel0[first + r] = v;
        }
    }
    if (c == 0 && lane == 0 && !from_step) a.hdr[HDR_STATE] = STATE_CELLS;
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
    hipLaunchKernelGGL(k_cell_order, dim3(a.ncells), dim3(kWave), 0, st, a, from_step);
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
