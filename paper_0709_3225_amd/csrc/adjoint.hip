// Adjoint of the velocity-Verlet LJ trajectory: Hessian-vector products of
// the force sum, parameter derivatives and the virial gradient.
//
// The force on particle i (section 2, force-sum equation with the truncated,
// force-shifted f(r)) is F_i = sum_j g(r) d, g = phi/r, d = r_i - r_j. Its
// Jacobian applied to a vector w is
//   (J w)_i = sum_j [ g (w_i - w_j) + B d (d . (w_i - w_j)) ],
//   B = (phi' - g) / r^2,  phi' = (24 eps / r^2) (7 (sigma/r)^6 - 26 (sigma/r)^12);
// the shift constant drops out of phi' but not out of g. With r_c = 2.5 sigma,
//   d phi / d eps = phi / eps,
//   d phi / d sigma = (24 eps / (r sigma)) (24 (sigma/r)^12 - 6 (sigma/r)^6) + f_LJ(r_c) / sigma,
// and no boundary term appears because phi(r_c) = 0. The energy-shift mode has
// a force jump at r_c and is not differentiable; the entry points refuse it.
//
// The kernels reuse the force kernel's cell-pair machinery (neighbourhood
// staging in the home cell's frame, screen, bit walk); the adjoint vector is
// staged in a second LDS tile next to the positions.
#include "cell_pairs.h"

namespace mdlj {

namespace {

enum { OP_ADJ = 0, OP_VGRAD = 1 };

// Pair constants of the passes below. With ir2 = 1/r^2, ir6 = ir2^3,
// ir8 = ir2 ir6, c12 = 48 eps sigma^12 and c6 = 24 eps sigma^6 (so that
// f_LJ(r)/r = ir8 (c12 ir6 - c6)) and fc = f_LJ(r_c):
//   g = phi / r                    = ir8 (c12 ir6 - c6) - fc / r
//   B = (phi' - g) / r^2           = ir2 [ir8 (8 c6 - 14 c12 ir6) + fc / r]
//   phi / r + phi'                 = ir8 (6 c6 - 12 c12 ir6) - fc / r
//   sigma (d phi / d sigma) / r    = ir8 (12 c12 ir6 - 6 c6) + fc / r
// (phi' = ir8 (7 c6 - 13 c12 ir6); the sigma derivative is taken at fixed
// r_c / sigma, so the shift contributes fc / r). Sums of the last line are
// divided by sigma once per atom.
struct PairConsts {
    float rc2, fc, c12, c6;
    float b12, b6;  // -14 c12, 8 c6
    float v12, v6;  // -12 c12, 6 c6
    float s12, s6;  // 12 c12, -6 c6
};

__device__ __forceinline__ PairConsts pair_consts(const SimArgs& a) {
    return PairConsts{a.rc2,          a.fc,          a.c12,         a.c6,          -14.0f * a.c12,
                      8.0f * a.c6,    -12.0f * a.c12, 6.0f * a.c6,  12.0f * a.c12, -6.0f * a.c6};
}

// One pair of the Hessian-vector product, plus the force (for d/d eps) and
// sigma times the sigma derivative projected on w_i.
struct AdjOp {
    const PairConsts& k;
    uint32_t wdelta;    // LDS distance from the position tile to the adjoint-vector tile
    float xi, yi, zi, wx, wy, wz;
    float jx = 0.f, jy = 0.f, jz = 0.f, fx = 0.f, fy = 0.f, fz = 0.f, sg = 0.f;
    __device__ __forceinline__ void operator()(uint32_t addr, bool live) {
        const float4 q = lds_load(addr);
        const float4 wj = lds_load(addr + wdelta);
        const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const bool ok = live && (r2 < k.rc2);
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float ir2 = rinv * rinv;
        const float ir6 = ir2 * ir2 * ir2;
        const float ir8 = ir2 * ir6;
        const float fcr = k.fc * rinv;
        float g = fmaf(ir8, fmaf(k.c12, ir6, -k.c6), -fcr);         // phi / r
        float bb = ir2 * fmaf(ir8, fmaf(k.b12, ir6, k.b6), fcr);    // (phi' - g) / r^2
        float dps = fmaf(ir8, fmaf(k.s12, ir6, k.s6), fcr);          // sigma (dphi/dsigma) / r
        g = ok ? g : 0.f;
        bb = ok ? bb : 0.f;
        dps = ok ? dps : 0.f;
        const float ux = wx - wj.x, uy = wy - wj.y, uz = wz - wj.z;
        const float dd = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
        const float t = bb * dd;
        jx = fmaf(g, ux, fmaf(t, dx, jx));
        jy = fmaf(g, uy, fmaf(t, dy, jy));
        jz = fmaf(g, uz, fmaf(t, dz, jz));
        fx = fmaf(g, dx, fx);
        fy = fmaf(g, dy, fy);
        fz = fmaf(g, dz, fz);
        sg = fmaf(dps, fmaf(dz, wz, fmaf(dy, wy, dx * wx)), sg);
    }
};

// One pair of the virial gradient: grad_i W = sum_j (phi + r phi') d / r,
// plus W and sigma r dphi/dsigma for the parameter derivatives.
struct VGradOp {
    const PairConsts& k;
    float xi, yi, zi;
    float gx = 0.f, gy = 0.f, gz = 0.f, wsum = 0.f, wsig = 0.f;
    __device__ __forceinline__ void operator()(uint32_t addr, bool live) {
        const float4 q = lds_load(addr);
        const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const bool ok = live && (r2 < k.rc2);
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float ir2 = rinv * rinv;
        const float ir6 = ir2 * ir2 * ir2;
        const float ir8 = ir2 * ir6;
        const float fcr = k.fc * rinv;
        const float g = fmaf(ir8, fmaf(k.c12, ir6, -k.c6), -fcr);    // phi / r
        const float sc = fmaf(ir8, fmaf(k.v12, ir6, k.v6), -fcr);    // phi / r + phi'
        const float dps = fmaf(ir8, fmaf(k.s12, ir6, k.s6), fcr);    // sigma (dphi/dsigma) / r
        const float scm = ok ? sc : 0.f;
        gx = fmaf(scm, dx, gx);
        gy = fmaf(scm, dy, gy);
        gz = fmaf(scm, dz, gz);
        wsum += ok ? g * r2 : 0.f;     // r phi
        wsig += ok ? dps * r2 : 0.f;   // sigma r dphi/dsigma
    }
};

// One pass over the pairs of every home cell: the Hessian-vector product
// (ADJ) or the virial gradient (VGRAD). Staging as in the force kernel: a
// neighbourhood that fits one tile is staged in one pass from the row table
// (cells away from the x faces) or the row-piece table (cells on an x face),
// with the adjoint vector (ADJ) in a second tile at the same indices; other
// cells take the LDS segment table and stage in the pass loop. The slice
// reduction reuses the tiles. With nw = blockDim / 64 <= MW wavefronts per
// cell, wavefront 0 stages, each screens and walks its own contiguous range
// of every pass's candidates, and wavefront 0 adds the partials (wavefronts
// in order, then slices) and finishes the atoms.
template <int OP, int MW>
__global__ void __launch_bounds__(MW * kWave)
    k_pair_pass(SimArgs a, const float4* __restrict__ wvec, float4* __restrict__ out_r, float4* __restrict__ out_v,
                float coef, float kcoef, double pcoef, bool accumulate) {
    if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    constexpr bool ADJ = (OP == OP_ADJ);
    constexpr int NRED = ADJ ? 7 : 5;  // partials per lane
    extern __shared__ float4 tile[];  // positions, then (ADJ) the adjoint vector: 2 x (tile_cap + kTilePad)
    __shared__ Neighbourhood nb;
    float4* wtile = tile + (a.tile_cap + kTilePad);
    float* red = reinterpret_cast<float*>(tile);  // NRED x 64 floats per wavefront, after the walk
    const int lane = __lane_id();
    const int wv = MW == 1 ? 0 : static_cast<int>(threadIdx.x) >> 6;  // uniform per wavefront
    const int nw = MW == 1 ? 1 : static_cast<int>(blockDim.x) >> 6;
    const int c = xcd_block_order(blockIdx.x, a.ncells);
    const PairConsts kc = pair_consts(a);
    float ox, oy, oz;
    RowHood rh;
    const bool interior = row_hood(a, c, rh);  // uniform
    bool rows = interior && rh.pos[9] <= a.tile_cap && rh.n_home <= kWave;
    int total, home_first, n_home, home_pos;
    if (rows) {
        ox = rh.ox;
        oy = rh.oy;
        oz = rh.oz;
        total = rh.pos[9];
        home_first = rh.home_first;
        n_home = rh.n_home;
        home_pos = rh.home_pos;
        if (wv == 0) stage_rows<ADJ ? SECOND_VEC : SECOND_NONE>(a, rh, tile, wtile, wvec);
    }
    RowPieces rp;
    if (!interior) row_pieces(a, c, rp);
    if (!interior && rp.total <= a.tile_cap && rp.n_home <= kWave) {
        rows = true;
        ox = rp.ox;
        oy = rp.oy;
        oz = rp.oz;
        total = rp.total;
        home_first = rp.home_first;
        n_home = rp.n_home;
        home_pos = rp.home_pos;
        if (wv == 0) stage_pieces<ADJ ? SECOND_VEC : SECOND_NONE>(a, rp, tile, wtile, wvec);
    }
    if (!rows) {
        load_neighbourhood(a, c, nb, ox, oy, oz);
        total = nb.total;
        home_first = nb.home_first;
        n_home = nb.n_home;
        home_pos = nb.home_pos;
    }
    const float inv_sig = 1.0f / sqrtf(a.sig2);
    const float inv_eps = 24.0f / a.eps24;

    double acc0 = 0.0, acc1 = 0.0;
    for (int h0 = 0; h0 < n_home; h0 += kWave) {
        const int nh = min(kWave, n_home - h0);
        // 11..16 home atoms: matrix-core screen with four slices, lane =
        // (atom lane % 16, slice lane / 16), as in the force kernel
        const bool mf = nh >= kMfmaMinHome && nh <= 16;  // uniform
        const int ns = mf ? 4 : min(kMaxSlices, kWave / nh);
        const int hstride = mf ? 16 : nh;
        const int h = lane % hstride, s = lane / hstride;
        const bool act = mf ? h < nh : s < ns;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f), wi = pi;
        if (act) {
            pi = a.pos0[home_first + h0 + h];
            if (ADJ) wi = wvec[home_first + h0 + h];
        }
        const float xi = pi.x - ox, yi = pi.y - oy, zi = pi.z - oz;
        const float ai = fmaf(zi, zi, fmaf(yi, yi, xi * xi));
        const float thr_i = act ? a.screen2 - ai : -__builtin_huge_valf();
        const float mx = -2.0f * xi, my = -2.0f * yi, mz = -2.0f * zi;
        const float bval = s == 3 ? 1.0f : (act ? (s == 0 ? mx : (s == 1 ? my : mz)) : 0.0f);
        const float cneg = -thr_i;
        float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f, v6 = 0.f;
        for (int t0 = 0; t0 < total; t0 += a.tile_cap) {
            const int tn = min(a.tile_cap, total - t0);
            if (!rows) {
                __syncthreads();
                if (wv == 0) stage_tile<false, ADJ>(a, nb, tile, t0, tn, wvec, wtile);
            }
            if (wv == 0) {
                for (int t = lane; t < kTilePad; t += kWave) {
                    tile[tn + t] = make_float4(0.f, 0.f, 0.f, __builtin_huge_valf());
                    if (ADJ) wtile[tn + t] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
            __syncthreads();
            const int self_t = home_pos + h0 + h - t0;
            // spans: 128 candidates per lane (32 blocks of 16 with the matrix cores);
            // this wavefront's groups [g_lo, g_hi), split at multiples of the
            // screen's step (four blocks, or four VALU groups)
            const int groups_all = mf ? 4 * ((tn + 15) / 16) : (tn + ns - 1) / ns;
            const int unit = mf ? 16 : kScreenUnroll;
            const int nu = (groups_all + unit - 1) / unit;
            const int g_lo = unit * ((nu * wv) / nw), g_hi = min(groups_all, unit * ((nu * (wv + 1)) / nw));
            for (int g0 = g_lo; g0 < g_hi; g0 += kGroups) {
                const int groups = min(kGroups, g_hi - g0);
                const int first = mf ? 4 * g0 + s : g0 * ns + (act ? s : 0);
                uint32_t wd[kWords];
                if (mf) {
                    screen_mfma(tile, 4 * g0, groups / 4, bval, cneg, wd);
                } else {
                    switch (ns) {
                        case 2: screen_span<2>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 3: screen_span<3>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 5: screen_span<5>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 6: screen_span<6>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        default: screen_span<0>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                    }
                }
                if (act) clear_self(self_t, first, ns, groups, wd);
                if (ADJ) {
                    AdjOp op{kc, lds_address(wtile) - lds_address(tile), xi, yi, zi, wi.x, wi.y, wi.z};
                    op.jx = v0; op.jy = v1; op.jz = v2; op.fx = v3; op.fy = v4; op.fz = v5; op.sg = v6;
                    walk_bits(ns, lds_address(tile + first), wd[0], wd[1], wd[2], wd[3], op);
                    v0 = op.jx; v1 = op.jy; v2 = op.jz; v3 = op.fx; v4 = op.fy; v5 = op.fz; v6 = op.sg;
                } else {
                    VGradOp op{kc, xi, yi, zi};
                    op.gx = v0; op.gy = v1; op.gz = v2; op.wsum = v3; op.wsig = v4;
                    walk_bits(ns, lds_address(tile + first), wd[0], wd[1], wd[2], wd[3], op);
                    v0 = op.gx; v1 = op.gy; v2 = op.gz; v3 = op.wsum; v4 = op.wsig;
                }
            }
        }
        // partials of each home atom, summed over wavefronts in order and
        // slices in order (red aliases the tiles: every lane has finished its
        // walk at this barrier; a cell of several home chunks restages in the
        // next chunk's pass)
        __syncthreads();
        float* mine = red + NRED * kWave * wv;
        mine[0 * kWave + lane] = v0;
        mine[1 * kWave + lane] = v1;
        mine[2 * kWave + lane] = v2;
        mine[3 * kWave + lane] = v3;
        mine[4 * kWave + lane] = v4;
        if (ADJ) {
            mine[5 * kWave + lane] = v5;
            mine[6 * kWave + lane] = v6;
        }
        __syncthreads();
        if (act && s == 0 && wv == 0) {
            float r[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int w = 0; w < nw; ++w) {
                const float* part = red + NRED * kWave * w;
                for (int q = 0; q < ns; ++q) {
                    const int l = h + q * hstride;
#pragma unroll
                    for (int k = 0; k < NRED; ++k) r[k] += part[k * kWave + l];
                }
            }
            const int slot = home_first + h0 + h;
            const int id = __float_as_int(pi.w);
            if (ADJ) {
                float4 o = out_r[id];
                o.x = fmaf(coef, r[0], o.x);
                o.y = fmaf(coef, r[1], o.y);
                o.z = fmaf(coef, r[2], o.z);
                o.w = 0.f;
                out_r[id] = o;
                // w_i . dF_i/d eps = w_i . F_i / eps ; w_i . dF_i/d sigma
                acc0 += static_cast<double>(inv_eps) *
                        (static_cast<double>(wi.x) * r[3] + static_cast<double>(wi.y) * r[4] +
                         static_cast<double>(wi.z) * r[5]);
                acc1 += static_cast<double>(inv_sig) * static_cast<double>(r[6]);
            } else {
                out_r[id] = make_float4(coef * r[0], coef * r[1], coef * r[2], 0.f);
                const float4 v = a.vel0[slot];
                const float km = kcoef * 2.0f * a.half_m;
                out_v[id] = make_float4(km * v.x, km * v.y, km * v.z, 0.f);
                // W = 1/2 sum over ordered pairs of r phi, dW/d eps = W / eps
                acc0 += 0.5 * static_cast<double>(inv_eps) * static_cast<double>(r[3]);
                acc1 += 0.5 * static_cast<double>(inv_sig) * static_cast<double>(r[4]);
            }
        }
    }
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    // the cell's parameter partials, scaled by pcoef; accumulate adds them to
    // the cell's running sums (the passes of one segment), else replaces them
    if (threadIdx.x == 0) {
        double* e = a.epart + 3 * static_cast<size_t>(blockIdx.x);
        e[0] = (accumulate ? e[0] : 0.0) + pcoef * acc0;
        e[1] = (accumulate ? e[1] : 0.0) + pcoef * acc1;
    }
}

// theta[0..1] += coef * (fixed-order sums of the per-block partials): lane t
// sums blocks t, t + kThetaBlock, ... in that order (the loads of kThetaUnroll
// blocks issued before their sums), then a fixed tree over the lanes.
constexpr int kThetaBlock = 1024;
constexpr int kThetaUnroll = 8;
__global__ void __launch_bounds__(kThetaBlock) k_theta_final(SimArgs a, double* theta, double coef) {
    if (!state_ok(a, false)) return;
    __shared__ double s0[kThetaBlock], s1[kThetaBlock];
    const int t = threadIdx.x;
    double x0 = 0.0, x1 = 0.0;
    for (int b0 = t; b0 < a.ncells; b0 += kThetaBlock * kThetaUnroll) {
        double p0[kThetaUnroll], p1[kThetaUnroll];
#pragma unroll
        for (int q = 0; q < kThetaUnroll; ++q) {
            const int b = b0 + q * kThetaBlock;
            p0[q] = b < a.ncells ? a.epart[3 * b + 0] : 0.0;
            p1[q] = b < a.ncells ? a.epart[3 * b + 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kThetaUnroll; ++q) {
            if (b0 + q * kThetaBlock < a.ncells) {
                x0 += p0[q];
                x1 += p1[q];
            }
        }
    }
    s0[t] = x0;
    s1[t] = x1;
    __syncthreads();
    for (int off = kThetaBlock / 2; off > 0; off >>= 1) {
        if (t < off) {
            s0[t] += s0[t + off];
            s1[t] += s1[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        theta[0] += coef * s0[0];
        theta[1] += coef * s1[0];
    }
}

// w (user order) -> sorted order, into the staging velocity array.
__global__ void __launch_bounds__(256) k_gather_vec(SimArgs a, const float4* __restrict__ w_user) {
    if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= a.n) return;
    const int id = __float_as_int(a.pos0[k].w);
    a.vel1[k] = (id >= 0 && id < a.n) ? w_user[id] : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Drift adjoint fused with the gather of the kick adjoint that follows it:
// for sorted slot k (atom id = the slot's user index) lam_v[id] += dt
// lam_r[id], as k_adjoint_drift computes it, and the new lam_v[id] goes to
// the staging velocity array. Each id is one slot's, so no two lanes touch
// the same atom.
__global__ void __launch_bounds__(256) k_drift_gather(SimArgs a, float dt, const float4* __restrict__ lam_r,
                                                      float4* __restrict__ lam_v) {
    if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= a.n) return;
    const int id = __float_as_int(a.pos0[k].w);
    if (id < 0 || id >= a.n) {
        a.vel1[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const float4 r = lam_r[id];
    float4 v = lam_v[id];
    v.x = fmaf(dt, r.x, v.x);
    v.y = fmaf(dt, r.y, v.y);
    v.z = fmaf(dt, r.z, v.z);
    lam_v[id] = v;
    a.vel1[k] = v;
}

// Adjoint of the drift r += dt v: lam_v += dt lam_r (user order).
__global__ void __launch_bounds__(256) k_adjoint_drift(int n, float dt, const float4* __restrict__ lam_r,
                                                       float4* __restrict__ lam_v) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 r = lam_r[i];
    float4 v = lam_v[i];
    v.x = fmaf(dt, r.x, v.x);
    v.y = fmaf(dt, r.y, v.y);
    v.z = fmaf(dt, r.z, v.z);
    lam_v[i] = v;
}

// One pair pass over all cells with a.waves wavefronts per cell: LDS for the
// position tile (and the vector tile with ADJ), at least the reduction's
// partials of every wavefront.
template <int OP, class... Args>
void launch_pair(const SimArgs& a, hipStream_t st, Args... args) {
    constexpr size_t nred = OP == OP_ADJ ? 7 : 5;
    const size_t tiles = (OP == OP_ADJ ? 2 : 1) * static_cast<size_t>(a.tile_cap + kTilePad);
    const size_t lds = sizeof(float4) * std::max(tiles, nred * 16 * static_cast<size_t>(a.waves));
    if (a.waves == 1)
        hipLaunchKernelGGL((k_pair_pass<OP, 1>), dim3(a.ncells), dim3(kWave), lds, st, a, args...);
    else
        hipLaunchKernelGGL((k_pair_pass<OP, kMaxCellWaves>), dim3(a.ncells), dim3(kWave * a.waves), lds, st, a,
                           args...);
}

}  // namespace

hipError_t launch_adjoint_kick(const SimArgs& a, const float4* w_user, float4* lam_r, double* theta, float coef,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_gather_vec, dim3((a.n + 255) / 256), dim3(256), 0, st, a, w_user);
    launch_pair<OP_ADJ>(a, st, static_cast<const float4*>(a.vel1), lam_r, static_cast<float4*>(nullptr), coef, 0.f, 1.0,
                        false);
    if (theta) hipLaunchKernelGGL(k_theta_final, dim3(1), dim3(kThetaBlock), 0, st, a, theta, static_cast<double>(coef));
    return hipGetLastError();
}

hipError_t launch_adjoint_drift_kick(const SimArgs& a, float dt, float4* lam_r, float4* lam_v, float coef,
                                     bool accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_drift_gather, dim3((a.n + 255) / 256), dim3(256), 0, st, a, dt,
                       static_cast<const float4*>(lam_r), lam_v);
    launch_pair<OP_ADJ>(a, st, static_cast<const float4*>(a.vel1), lam_r, static_cast<float4*>(nullptr), coef, 0.f,
                        static_cast<double>(coef), accumulate);
    return hipGetLastError();
}

hipError_t launch_theta_final(const SimArgs& a, double* theta, double coef, hipStream_t st) {
    hipLaunchKernelGGL(k_theta_final, dim3(1), dim3(kThetaBlock), 0, st, a, theta, coef);
    return hipGetLastError();
}

hipError_t launch_loss_grad(const SimArgs& a, float kcoef, float wcoef, float4* g_r, float4* g_v, double* theta,
                            hipStream_t st) {
    launch_pair<OP_VGRAD>(a, st, static_cast<const float4*>(nullptr), g_r, g_v, wcoef, kcoef, 1.0, false);
    if (theta) hipLaunchKernelGGL(k_theta_final, dim3(1), dim3(kThetaBlock), 0, st, a, theta, static_cast<double>(wcoef));
    return hipGetLastError();
}

hipError_t launch_adjoint_drift(int n, float dt, const float4* lam_r, float4* lam_v, hipStream_t st) {
    hipLaunchKernelGGL(k_adjoint_drift, dim3((n + 255) / 256), dim3(256), 0, st, n, dt, lam_r, lam_v);
    return hipGetLastError();
}

}  // namespace mdlj
