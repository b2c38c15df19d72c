// Truncated, force-shifted Lennard-Jones forces over the cell list
// (section 2: force sum, f_LJ and the shifted f(r); section 3: partners in
// the home cell and its 26 neighbours).
//
// One wavefront per home cell. The wavefront stages the 27-cell neighbourhood
// into LDS once, translated into the home cell's frame so that the periodic
// image shift costs nothing per pair, and every lane then runs its home atom
// against the staged atoms. This replaces the paper's fixed array of 32
// placeholders per cell (section 3.1) by exact CSR ranges: no capacity limit
// and no virtual particles.
//
// Frame arithmetic: with home-cell origin o and image shift sh of a
// neighbour cell, the displacement is d = (x_i - o) - (x_j - (o - sh)).
// o - sh is exact in FP32 (o = 0 with sh = -L gives L; o >= L/2 with sh = +L
// is a Sterbenz subtraction), and both differences are of numbers within a
// few cells of each other, so d carries only the rounding of small numbers
// instead of ulp(L).
#include "md_device.h"

namespace mdlj {

namespace {

constexpr int kTile = 1024;  // staged atoms per LDS pass (16 KiB)

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
        const int cj = jx + nc * (jy + nc * jz);
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
__device__ __forceinline__ void stage_tile(const SimArgs& a, const Neighbourhood& nb, float4* tile,
                                           int t0, int tn) {
    for (int t = threadIdx.x; t < tn; t += kWave) {
        const int g = t0 + t;
        int k = 0;  // largest k with pref[k] <= g
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
            if (k + step < 27 && nb.pref[k + step] <= g) k += step;
        const float4 q = a.pos0[nb.first[k] + (g - nb.pref[k])];
        tile[t] = make_float4(q.x - nb.bx[k], q.y - nb.by[k], q.z - nb.bz[k], q.w);
    }
}

template <bool KICK, bool ENERGY, bool WRITE>
__global__ void __launch_bounds__(kWave) k_forces(SimArgs a, bool from_step) {
    if (from_step) {
        if (a.hdr[HDR_ERROR] & DEV_ORDER) return;
    } else if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    __shared__ float4 tile[kTile];
    __shared__ Neighbourhood nb;
    const int lane = threadIdx.x;
    const int c = xcd_block_order(blockIdx.x, a.ncells);
    float ox, oy, oz;
    load_neighbourhood(a, c, nb, ox, oy, oz);
    const int total = nb.pref[27];
    const int home_first = nb.first[13];
    const int n_home = nb.pref[14] - nb.pref[13];

    double u_acc = 0.0, w_acc = 0.0, k_acc = 0.0;
    bool bad = false;
    for (int h0 = 0; h0 < n_home; h0 += kWave) {
        const int h = h0 + lane;
        const bool act = h < n_home;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
        if (act) pi = a.pos0[home_first + h];
        const float xi = pi.x - ox, yi = pi.y - oy, zi = pi.z - oz;
        const int idi = __float_as_int(pi.w);
        float fx = 0.f, fy = 0.f, fz = 0.f;
        float u_loc = 0.f, w_loc = 0.f;
        for (int t0 = 0; t0 < total; t0 += kTile) {
            const int tn = min(kTile, total - t0);
            __syncthreads();
            stage_tile(a, nb, tile, t0, tn);
            __syncthreads();
            if (act) {
                for (int j = 0; j < tn; ++j) {
                    const float4 q = tile[j];
                    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < a.rc2 && __float_as_int(q.w) != idi) {
                        const float rinv = rsqrtf(r2);
                        const float ir2 = rinv * rinv;
                        const float s2 = a.sig2 * ir2;
                        const float s6 = s2 * s2 * s2;
                        const float fr = a.eps24 * ir2 * s6 * (2.0f * s6 - 1.0f) - a.fc * rinv;
                        fx += fr * dx;
                        fy += fr * dy;
                        fz += fr * dz;
                        if (ENERGY) {
                            const float r = r2 * rinv;
                            u_loc += a.eps4 * s6 * (s6 - 1.0f) - a.uc + (r - a.rc) * a.fc;
                            w_loc += fr * r2;
                        }
                    }
                }
            }
        }
        if (act) {
            const int k = home_first + h;
            if (!finite3(fx, fy, fz)) bad = true;
            if (WRITE) a.force[k] = make_float4(fx, fy, fz, 0.f);
            if (KICK || ENERGY) {
                float4 v = a.vel0[k];
                if (KICK) {
                    v.x += a.hdt_m * fx;
                    v.y += a.hdt_m * fy;
                    v.z += a.hdt_m * fz;
                    a.vel0[k] = v;
                }
                if (ENERGY) {
                    u_acc += static_cast<double>(u_loc);
                    w_acc += static_cast<double>(w_loc);
                    k_acc += static_cast<double>(a.half_m) * (static_cast<double>(v.x) * v.x +
                                                              static_cast<double>(v.y) * v.y +
                                                              static_cast<double>(v.z) * v.z);
                }
            }
        }
    }
    if (bad) atomicOr(&a.hdr[HDR_ERROR], DEV_NONFINITE);
    if (ENERGY) {
        u_acc = wave_sum(u_acc);
        w_acc = wave_sum(w_acc);
        k_acc = wave_sum(k_acc);
        if (lane == 0) {
            a.epart[3 * blockIdx.x + 0] = u_acc;
            a.epart[3 * blockIdx.x + 1] = w_acc;
            a.epart[3 * blockIdx.x + 2] = k_acc;
        }
    }
    if (WRITE && blockIdx.x == 0 && lane == 0) a.hdr[HDR_STATE] = STATE_FORCES;
}

// Fixed-order final sum of the per-block partials: U = 1/2 sum, W = 1/2 sum
// (every pair is visited from both sides), K as is.
constexpr int kRedBlock = 256;
__global__ void __launch_bounds__(kRedBlock) k_energy_final(SimArgs a, double* out3, bool from_step) {
    if (from_step && (a.hdr[HDR_ERROR] & DEV_ORDER)) return;
    __shared__ double su[kRedBlock], sw[kRedBlock], sk[kRedBlock];
    const int t = threadIdx.x;
    double u = 0.0, w = 0.0, k = 0.0;
    for (int b = t; b < a.ncells; b += kRedBlock) {
        u += a.epart[3 * b + 0];
        w += a.epart[3 * b + 1];
        k += a.epart[3 * b + 2];
    }
    su[t] = u;
    sw[t] = w;
    sk[t] = k;
    __syncthreads();
    for (int off = kRedBlock / 2; off > 0; off >>= 1) {
        if (t < off) {
            su[t] += su[t + off];
            sw[t] += sw[t + off];
            sk[t] += sk[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        out3[0] = 0.5 * su[0];
        out3[1] = sk[0];
        out3[2] = 0.5 * sw[0];
    }
}

// Neighbour export: same staging and cutoff test as the force kernel.
__global__ void __launch_bounds__(kWave) k_neighbors(SimArgs a, int* counts, int* idx, int max_nb) {
    if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    __shared__ float4 tile[kTile];
    __shared__ Neighbourhood nb;
    const int lane = threadIdx.x;
    const int c = blockIdx.x;
    float ox, oy, oz;
    load_neighbourhood(a, c, nb, ox, oy, oz);
    const int total = nb.pref[27];
    const int home_first = nb.first[13];
    const int n_home = nb.pref[14] - nb.pref[13];
    bool overflow = false;
    for (int h0 = 0; h0 < n_home; h0 += kWave) {
        const int h = h0 + lane;
        const bool act = h < n_home;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
        if (act) pi = a.pos0[home_first + h];
        const float xi = pi.x - ox, yi = pi.y - oy, zi = pi.z - oz;
        const int idi = __float_as_int(pi.w);
        int cnt = 0;
        for (int t0 = 0; t0 < total; t0 += kTile) {
            const int tn = min(kTile, total - t0);
            __syncthreads();
            stage_tile(a, nb, tile, t0, tn);
            __syncthreads();
            if (act) {
                for (int j = 0; j < tn; ++j) {
                    const float4 q = tile[j];
                    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < a.rc2 && __float_as_int(q.w) != idi) {
                        if (cnt < max_nb) idx[static_cast<size_t>(idi) * max_nb + cnt] = __float_as_int(q.w);
                        else overflow = true;
                        ++cnt;
                    }
                }
            }
        }
        if (act) counts[idi] = cnt;
    }
    if (overflow) atomicOr(&a.hdr[HDR_ERROR], DEV_NB_OVERFLOW);
}

}  // namespace

hipError_t launch_forces(const SimArgs& a, bool kick, bool energy, bool write_force, bool from_step,
                         hipStream_t st) {
    const dim3 g(a.ncells), b(kWave);
    if (kick && energy && write_force) {
        hipLaunchKernelGGL((k_forces<true, true, true>), g, b, 0, st, a, from_step);
    } else if (kick && !energy && write_force) {
        hipLaunchKernelGGL((k_forces<true, false, true>), g, b, 0, st, a, from_step);
    } else if (!kick && energy && !write_force) {
        hipLaunchKernelGGL((k_forces<false, true, false>), g, b, 0, st, a, from_step);
    } else if (!kick && !energy && write_force) {
        hipLaunchKernelGGL((k_forces<false, false, true>), g, b, 0, st, a, from_step);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_energy_final(const SimArgs& a, double* out3, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedBlock), 0, st, a, out3, true);
    return hipGetLastError();
}

hipError_t launch_neighbors(const SimArgs& a, int* counts, int* idx, int max_per_atom, hipStream_t st) {
    hipLaunchKernelGGL(k_neighbors, dim3(a.ncells), dim3(kWave), 0, st, a, counts, idx, max_per_atom);
    return hipGetLastError();
}

}  // namespace mdlj
