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
#include "cell_pairs.h"

namespace mdlj {

namespace {

template <bool ENERGY>
__device__ __forceinline__ float pair_force(const SimArgs& a, const float4 q, float xi, float yi, float zi,
                                            bool live, float& fx, float& fy, float& fz, float& u_loc,
                                            float& w_loc) {
    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    // the atom itself never reaches this point (its screen bit is cleared)
    const bool ok = live && (r2 < a.rc2);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float ir2 = rinv * rinv;
    const float ir6 = ir2 * ir2 * ir2;
    // f(r) / r = 24 eps (2 sigma^12 r^-14 - sigma^6 r^-8) - f_LJ(r_c) / r
    float fr = fmaf(ir2 * ir6, fmaf(a.c12, ir6, -a.c6), -a.fc * rinv);
    fr = ok ? fr : 0.0f;
    fx = fmaf(fr, dx, fx);
    fy = fmaf(fr, dy, fy);
    fz = fmaf(fr, dz, fz);
    if (ENERGY) {
        const float r = r2 * rinv;
        const float u = ir6 * fmaf(a.e12, ir6, -a.e6) - a.uc + (r - a.rc) * a.fc;
        u_loc += ok ? u : 0.0f;
        w_loc += fr * r2;
    }
    return r2;
}

// Pair operation of the force walk: the accepted candidate at an LDS address.
template <bool ENERGY>
struct ForceOp {
    const SimArgs& a;
    float xi, yi, zi;
    float fx = 0.f, fy = 0.f, fz = 0.f, u_loc = 0.f, w_loc = 0.f;
    __device__ __forceinline__ void operator()(uint32_t addr, bool live) {
        const float4 q = lds_load(addr);
        pair_force<ENERGY>(a, q, xi, yi, zi, live, fx, fy, fz, u_loc, w_loc);
    }
};

// Pair operation of the pass that writes the neighbour lists: the force as
// ForceOp, and every candidate the walk visits (all within the list radius)
// appended to the home atom's list at this lane's next free entry.
template <bool ENERGY>
struct RecordOp {
    const SimArgs& a;
    uint32_t tile0;     // LDS address of the tile
    const char* cbase;  // list entries of the staged atoms (4 bytes each, at a quarter of the tile's offsets)
    float xi, yi, zi;
    uint32_t* row;      // the home atom's list: entry k at row[4 n (k / 4) + k % 4]
    int next;
    float fx = 0.f, fy = 0.f, fz = 0.f, u_loc = 0.f, w_loc = 0.f;
    __device__ __forceinline__ void operator()(uint32_t addr, bool live) {
        const float4 q = lds_load(addr);
        pair_force<ENERGY>(a, q, xi, yi, zi, live, fx, fy, fz, u_loc, w_loc);
        if (live) {
            if (next < a.nlist_cap)
                row[4 * static_cast<size_t>(a.n) * (next >> 2) + (next & 3)] =
                    *reinterpret_cast<const uint32_t*>(cbase + ((addr - tile0) >> 2));
            ++next;
        }
    }
};

// Neighbour export from the force kernel's own staging, screen and walk: every
// pair the walk visits and the exact FP32 cutoff test of pair_force accepts
// appends the partner's user index to the home atom's row (row order follows
// the atomics, so it is unspecified).
struct ExportArgs {
    int* counts;
    int* idx;
    int max_nb;
};

struct ExportOp {
    const SimArgs& a;
    uint32_t tile0;     // LDS address of the tile
    const char* rbase;  // untranslated positions (user index in w) at the same offsets
    float xi, yi, zi;
    int idi;
    const ExportArgs& ex;
    bool over = false;
    __device__ __forceinline__ void operator()(uint32_t addr, bool live) {
        const uint32_t off = addr - tile0;
        const float4 q = lds_load(addr);
        const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (live && r2 < a.rc2) {
            const int idj = __float_as_int(reinterpret_cast<const float4*>(rbase + off)->w);
            const int slot = atomicAdd(&ex.counts[idi], 1);
            if (slot < ex.max_nb) ex.idx[static_cast<size_t>(idi) * ex.max_nb + slot] = idj;
            else over = true;
        }
    }
};

// Kept accept words (pair lists as bitmasks): span j of a lane is one 16-byte
// record; spans past kListSpans are only counted (the cell then screens).
__device__ __forceinline__ void keep_words(uint4* rows, int& n, const uint32_t (&wd)[kWords]) {
    if (n < kListSpans) rows[n] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
    ++n;
}

// Span j's kept words; span 0 was requested before the staging (w0). Bits
// past the span's groups candidates per lane are dropped, so a walk never
// leaves the staged span, whatever the words hold.
__device__ __forceinline__ void kept_words(const uint4* rows, const uint4& w0, int j, int groups,
                                           uint32_t (&wd)[kWords]) {
    const uint4 v = j == 0 ? w0 : (j < kListSpans ? rows[j] : make_uint4(0u, 0u, 0u, 0u));
    wd[0] = v.x;
    wd[1] = v.y;
    wd[2] = v.z;
    wd[3] = v.w;
#pragma unroll
    for (int w = 0; w < kWords; ++w) {
        const int valid = groups - 32 * w;  // uniform
        wd[w] &= valid >= 32 ? ~0u : (valid <= 0 ? 0u : ~0u << (32 - valid));
    }
}

// Forces on the atoms of home cell c (local index of the system described by
// a); one wavefront. Energy partials go to a.epart[3 (a.cbase + c) + 0..2].
// KICK completes the step's velocity (v += dt/(2m) F). DRIFT (with KICK) goes
// on into the next step's first half with the same force, as the drift kernel
// would (half kick, drift, wrap, cell, binning into the next rebuild's
// buckets) instead of writing vel0; force and vel0 are then left stale, since
// the rebuild replaces the sorted state.
// SKIN (with DRIFT): a step between rebuilds. The drift writes the unwrapped
// next position and velocity to pos2/vel2 (same sorted slot) instead of
// binning, and raises DEV_SKIN if the atom has left its cell's box by more
// than skin_half (cells of side r_c + skin then still hold every partner
// within r_c in the 27-cell neighbourhood, section 3.1) or, with pair lists,
// has moved more than disp_half since they were recorded (section 3).
// LIST 1: the screen takes the list radius (the cell side) as its bound and
// each lane's accept words are kept (one 16-byte record per span), and the
// home positions go to posref. LIST 2: a lane walks its kept words instead of
// screening: the same candidates in the same order plus some beyond r_c,
// which add exact zeros, so the sums are bitwise those of the screen. A cell
// with more than kListSpans spans per lane, or more than one pass, screens as
// usual (and with the plain bound).
// LIST 3: the screen takes the list radius and every candidate it accepts
// goes to the home atom's neighbour list (raw: the staged atoms' list
// entries, 4 bytes each); the slices of an atom append in slice order per
// span, so an atom's list is written without atomics.
// EXPORT: no forces; the pairs the walk accepts go to the neighbour rows of
// ex (raw: a second tile of untranslated positions).
template <bool KICK, bool ENERGY, bool WRITE, bool DRIFT, bool SKIN = false, int LIST = 0, bool EXPORT = false,
          int MW = 1>
__device__ __forceinline__ void force_cell(const SimArgs& a, int c, float4* tile, Neighbourhood& nb, float* red,
                                           float4* raw = nullptr, const ExportArgs& ex = ExportArgs{}) {
    // The workgroup holds nw <= MW wavefronts (1, 2 or 4). All of them compute
    // the neighbourhood table; wavefront 0 stages the tile they share, each
    // screens and walks its own contiguous range of every pass's candidates,
    // and wavefront 0 adds their partials (waves in order, then slices) and
    // runs the epilogue. MW = 1 compiles the one-wavefront kernel.
    const int lane = __lane_id();
    const int wv = MW == 1 ? 0 : static_cast<int>(threadIdx.x) >> 6;  // uniform per wavefront
    const int nw = MW == 1 ? 1 : static_cast<int>(blockDim.x) >> 6;
    float ox, oy, oz;
    // a cell away from the x faces whose neighbourhood and home atoms fit one
    // pass is staged here, from a table in scalar registers; others take the
    // LDS table and stage in the pass loop below
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
        if (wv == 0) stage_rows<EXPORT ? SECOND_RAW : (LIST == 3 ? SECOND_CODE : SECOND_NONE)>(a, rh, tile, raw);
    }
    // a cell on an x face: the same one-pass staging from a table of row pieces
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
        if (wv == 0) stage_pieces<EXPORT ? SECOND_RAW : (LIST == 3 ? SECOND_CODE : SECOND_NONE)>(a, rp, tile, raw);
    }
    if (!rows) {
        load_neighbourhood(a, c, nb, ox, oy, oz);
        total = nb.total;
        home_first = nb.home_first;
        n_home = nb.n_home;
        home_pos = nb.home_pos;
    }

    double u_acc = 0.0, w_acc = 0.0, k_acc = 0.0;
    bool bad = false, skin_out = false, over = false;
    const size_t lrow = (static_cast<size_t>(a.cbase + c) * kWave + lane);  // this lane's kept words
    uint4* lwords = reinterpret_cast<uint4*>(a.plist) + lrow * kListSpans;
    const bool list_fits = total <= a.tile_cap && n_home <= kWave;          // uniform
    int n_rec = 0;  // LIST 1: spans kept
    int list_n = 0;
    uint4 lw0 = make_uint4(0u, 0u, 0u, 0u);  // LIST 2: the first span's words, requested before staging
    if (LIST == 2) {
        list_n = a.plist_n[lrow];
        lw0 = lwords[0];
    }
    const bool use_list = LIST == 2 && list_fits && __all(list_n <= kListSpans);
    for (int h0 = 0; h0 < n_home; h0 += kWave) {
        const int nh = min(kWave, n_home - h0);
        // 11..16 home atoms: matrix-core screen, lane = (atom lane % 16, slice
        // lane / 16); otherwise the VALU screen with ns interleaved slices
        const bool mf = nh >= kMfmaMinHome && nh <= 16;  // uniform
        const int ns = mf ? 4 : min(kMaxSlices, kWave / nh);
        const int hstride = mf ? 16 : nh;  // lanes of one home atom: h, h + hstride, ...
        const int h = lane % hstride, s = lane / hstride;
        const bool act = mf ? h < nh : s < ns;
        // the lane that finishes home atom h (in wavefront 0); in the
        // matrix-core layout lanes nh..15 have s == 0 but no atom
        const bool lead = act && s == 0 && wv == 0;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
        if (act) pi = a.pos0[home_first + h0 + h];
        float4 vel = make_float4(0.f, 0.f, 0.f, 0.f);  // fetched now, used by the epilogue
        if ((KICK || ENERGY) && lead) vel = a.vel0[home_first + h0 + h];
        float4 pref = pi;  // LIST: position when the lists were recorded
        if (LIST == 2 && SKIN && lead) pref = a.posref[home_first + h0 + h];
        if ((LIST == 1 || LIST == 3) && lead) a.posref[home_first + h0 + h] = pi;
        const float xi = pi.x - ox, yi = pi.y - oy, zi = pi.z - oz;
        const float ai = fmaf(zi, zi, fmaf(yi, yi, xi * xi));
        // idle lanes get a bound no candidate can meet (q.w - thr_i = +inf)
        // (the list radius only where the words are kept: other cells sum as the plain screen does)
        const float thr_i = act ? (((LIST == 1 && list_fits) || LIST == 3) ? a.list_screen2 : a.screen2) - ai
                                : -__builtin_huge_valf();
        const float mx = -2.0f * xi, my = -2.0f * yi, mz = -2.0f * zi;
        // matrix-core operands: this lane's element of B (component s of
        // (-2 x_i, -2 y_i, -2 z_i, 1)) and of C (-bound + |x_i|^2; +inf idle)
        const float bval = s == 3 ? 1.0f : (act ? (s == 0 ? mx : (s == 1 ? my : mz)) : 0.0f);
        const float cneg = -thr_i;
        float fx = 0.f, fy = 0.f, fz = 0.f, u_loc = 0.f, w_loc = 0.f;
        int lcount = 0, rec_next = 0;  // LIST 3: the atom's entries so far; this lane's next one
        uint32_t* lrow_list = LIST == 3 ? a.nlist + 4 * static_cast<size_t>(home_first + h0 + h) : nullptr;
        for (int t0 = 0; t0 < total; t0 += a.tile_cap) {
            const int tn = min(a.tile_cap, total - t0);
            if (!rows) {
                __syncthreads();
                if (wv == 0) {
                    if (EXPORT) stage_tile<false, true>(a, nb, tile, t0, tn, a.pos0, raw);
                    else stage_tile<false>(a, nb, tile, t0, tn);
                    if (LIST == 3) stage_codes(a, nb, reinterpret_cast<uint32_t*>(raw), t0, tn);
                }
            }
            if (wv == 0)
                for (int t = lane; t < kTilePad; t += kWave) tile[tn + t] = make_float4(0.f, 0.f, 0.f, __builtin_huge_valf());
            __syncthreads();
            const int self_t = home_pos + h0 + h - t0;  // the home atom's own tile index (may be outside)
            // the walk over one span's words; the lane's candidates are cand0,
            // cand0 + ns_, cand0 + 2 ns_, ...
            // LIST 3: this lane's first entry for the span's accepted
            // candidates (after those of the atom's lower slices)
            auto list_base = [&](const uint32_t (&wd)[kWords]) {
                if (LIST != 3) return;
                const int cnt = __popc(wd[0]) + __popc(wd[1]) + __popc(wd[2]) + __popc(wd[3]);
                int pre = 0, tot = 0;
                for (int q = 0; q < ns; ++q) {
                    const int v = __shfl(cnt, h + q * hstride);
                    pre += q < s ? v : 0;
                    tot += v;
                }
                rec_next = lcount + pre;
                lcount += tot;
            };
            auto walk = [&](int ns_, int cand0, uint32_t (&wd)[kWords]) {
                const uint32_t tile0 = lds_address(tile);
                const uint32_t wb0 = tile0 + static_cast<uint32_t>(cand0) * sizeof(float4);
                if (LIST == 3) {
                    RecordOp<ENERGY> op{a,  tile0, reinterpret_cast<const char*>(raw), xi, yi, zi, lrow_list, rec_next,
                                        fx, fy, fz, u_loc, w_loc};
                    walk_bits(ns_, wb0, wd[0], wd[1], wd[2], wd[3], op);
                    fx = op.fx;
                    fy = op.fy;
                    fz = op.fz;
                    u_loc = op.u_loc;
                    w_loc = op.w_loc;
                } else if (EXPORT) {
                    ExportOp op{a, tile0, reinterpret_cast<const char*>(raw), xi, yi, zi, __float_as_int(pi.w), ex};
                    walk_bits(ns_, wb0, wd[0], wd[1], wd[2], wd[3], op);
                    over = over || op.over;
                } else {
                    ForceOp<ENERGY> op{a, xi, yi, zi, fx, fy, fz, u_loc, w_loc};
                    walk_bits(ns_, wb0, wd[0], wd[1], wd[2], wd[3], op);
                    fx = op.fx;
                    fy = op.fy;
                    fz = op.fz;
                    u_loc = op.u_loc;
                    w_loc = op.w_loc;
                }
            };
            if (mf) {
                // this wavefront's blocks [b_lo, b_hi), split at multiples of four
                // blocks (the screen's step), so no verdict is taken twice
                const int nblk_all = (tn + 15) / 16;
                const int q4 = (nblk_all + 3) >> 2;
                const int b_lo = 4 * ((q4 * wv) / nw), b_hi = min(nblk_all, 4 * ((q4 * (wv + 1)) / nw));
                for (int b0 = b_lo; b0 < b_hi; b0 += 8 * kWords) {
                    const int nblk = min(8 * kWords, b_hi - b0);
                    uint32_t wd[kWords];
                    if (LIST == 2 && use_list) {
                        kept_words(lwords, lw0, b0 / (8 * kWords), 4 * nblk, wd);
                    } else {
                        screen_mfma(tile, 16 * b0, nblk, bval, cneg, wd);
                        if (act) clear_self(self_t - 16 * b0, s, 4, 4 * nblk, wd);
                        if (LIST == 1 && list_fits) keep_words(lwords, n_rec, wd);
                        list_base(wd);
                    }
                    // the lane's candidates are tile + 16 b0 + s + 4 g, as for four VALU slices
                    walk(4, 16 * b0 + s, wd);
                }
                continue;
            }
            const int groups_all = (tn + ns - 1) / ns;  // candidates of the largest slice
            // this wavefront's groups [g_lo, g_hi), split at multiples of the screen's step
            const int q4 = (groups_all + kScreenUnroll - 1) / kScreenUnroll;
            const int g_lo = kScreenUnroll * ((q4 * wv) / nw);
            const int g_hi = min(groups_all, kScreenUnroll * ((q4 * (wv + 1)) / nw));
            for (int g0 = g_lo; g0 < g_hi; g0 += kGroups) {
                const int groups = min(kGroups, g_hi - g0);
                const int first = g0 * ns + (act ? s : 0);
                uint32_t wd[kWords];
                if (LIST == 2 && use_list) {
                    kept_words(lwords, lw0, g0 / kGroups, groups, wd);
                } else {
                    switch (ns) {
                        case 2: screen_span<2>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 3: screen_span<3>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 4: screen_span<4>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 5: screen_span<5>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        case 6: screen_span<6>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                        default: screen_span<0>(tile, first, ns, groups, mx, my, mz, thr_i, wd); break;
                    }
                    if (act) clear_self(self_t, first, ns, groups, wd);
                    if (LIST == 1 && list_fits) keep_words(lwords, n_rec, wd);
                    list_base(wd);
                }
                walk(ns, first, wd);
            }
        }
        if (EXPORT) continue;
        // sum the slice partials of each home atom in slice order (red aliases the
        // tile: every lane has finished its walk at this barrier)
        __syncthreads();
        float* mine = red + 5 * kWave * wv;  // this wavefront's partials
        mine[0 * kWave + lane] = fx;
        mine[1 * kWave + lane] = fy;
        mine[2 * kWave + lane] = fz;
        if (ENERGY) {
            mine[3 * kWave + lane] = u_loc;
            mine[4 * kWave + lane] = w_loc;
        }
        __syncthreads();
        const int k = home_first + h0 + h;
        int c_next = -1;  // DRIFT: the home atom's next cell, -1 on lanes without one
        float4 p_next = pi, v_next = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lead) {
            if (LIST == 3) {  // the atom's list length (the entries past the capacity were not kept)
                a.ncount[k] = min(lcount, a.nlist_cap);
                if (lcount > a.nlist_cap) over = true;
            }
            float gx = 0.f, gy = 0.f, gz = 0.f, gu = 0.f, gw = 0.f;
            for (int w = 0; w < nw; ++w) {
                const float* part = red + 5 * kWave * w;
                for (int q = 0; q < ns; ++q) {
                    const int l = h + q * hstride;
                    gx += part[0 * kWave + l];
                    gy += part[1 * kWave + l];
                    gz += part[2 * kWave + l];
                    if (ENERGY) {
                        gu += part[3 * kWave + l];
                        gw += part[4 * kWave + l];
                    }
                }
            }
            if (!finite3(gx, gy, gz)) bad = true;
            if (WRITE) a.force[k] = make_float4(gx, gy, gz, 0.f);
            if (KICK || ENERGY) {
                float4 v = vel;
                if (KICK) {
                    v.x += a.hdt_m * gx;
                    v.y += a.hdt_m * gy;
                    v.z += a.hdt_m * gz;
                    if (!DRIFT) a.vel0[k] = v;
                }
                if (ENERGY) {
                    u_acc += static_cast<double>(gu);
                    w_acc += static_cast<double>(gw);
                    k_acc += static_cast<double>(a.half_m) * (static_cast<double>(v.x) * v.x +
                                                              static_cast<double>(v.y) * v.y +
                                                              static_cast<double>(v.z) * v.z);
                }
                if (DRIFT) {
                    v_next = v;
                    if (SKIN) {
                        half_kick_drift_unwrapped(a, p_next, v_next, gx, gy, gz);
                        a.pos2[k] = p_next;
                        a.vel2[k] = v_next;
                        if (LIST != 0) {
                            const float ex = p_next.x - pref.x, ey = p_next.y - pref.y, ez = p_next.z - pref.z;
                            if (ex * ex + ey * ey + ez * ez > a.disp_half * a.disp_half) skin_out = true;
                        } else {
                            const float ex = fmaxf(fmaxf(ox - p_next.x, p_next.x - (ox + a.s)), 0.f);
                            const float ey = fmaxf(fmaxf(oy - p_next.y, p_next.y - (oy + a.s)), 0.f);
                            const float ez = fmaxf(fmaxf(oz - p_next.z, p_next.z - (oz + a.s)), 0.f);
                            if (ex * ex + ey * ey + ez * ez > a.skin_half * a.skin_half) skin_out = true;
                        }
                    } else {
                        c_next = half_kick_drift(a, p_next, v_next, gx, gy, gz);
                    }
                }
            }
        }
        if (DRIFT && !SKIN && wv == 0) bin_atom(a, p_next, v_next, c_next);  // all lanes of wavefront 0
    }
    if (LIST == 1) a.plist_n[lrow] = list_fits ? n_rec : kListSpans + 1;  // kept words of several passes are not used
    if ((EXPORT || LIST == 3) && over) atomicOr(&a.hdr[HDR_ERROR], DEV_NB_OVERFLOW);
    if (bad) atomicOr(&a.hdr[HDR_ERROR], DEV_NONFINITE);
    if (SKIN && skin_out) atomicOr(&a.hdr[HDR_ERROR], DEV_SKIN);
    if (ENERGY) {
        u_acc = wave_sum(u_acc);
        w_acc = wave_sum(w_acc);
        k_acc = wave_sum(k_acc);
        if (threadIdx.x == 0) {
            double* e = a.epart + 3 * static_cast<size_t>(a.cbase + c);
            e[0] = u_acc;
            e[1] = w_acc;
            e[2] = k_acc;
        }
    }
}

template <bool KICK, bool ENERGY, bool WRITE, bool DRIFT, int MW>
__global__ void __launch_bounds__(MW * kWave) k_forces(SimArgs a, bool from_step) {
    if (from_step) {
        if (a.hdr[HDR_ERROR] & DEV_ORDER) return;
    } else if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    extern __shared__ float4 tile[];  // cell_lds_entries(a.tile_cap, a.waves) entries
    __shared__ Neighbourhood nb;
    // the slice reduction reuses the tile (320 floats per wavefront)
    force_cell<KICK, ENERGY, WRITE, DRIFT, false, 0, false, MW>(a, xcd_block_order(blockIdx.x, a.ncells), tile, nb,
                                                                reinterpret_cast<float*>(tile));
    if (WRITE && blockIdx.x == 0 && threadIdx.x == 0) a.hdr[HDR_STATE] = STATE_FORCES;
}

// A step between rebuilds (md_step_every): forces, kick, and the next step's
// half kick and drift into pos2/vel2.
template <bool ENERGY, int MW>
__global__ void __launch_bounds__(MW * kWave) k_forces_skin(SimArgs a) {
    if (a.hdr[HDR_ERROR] & DEV_ORDER) return;
    extern __shared__ float4 tile[];
    __shared__ Neighbourhood nb;
    force_cell<true, ENERGY, false, true, true, 0, false, MW>(a, xcd_block_order(blockIdx.x, a.ncells), tile, nb,
                                                              reinterpret_cast<float*>(tile));
}

// Pair-list steps: RECORD right after a rebuild, else walk the recorded lists;
// BIN: the drift bins for the next rebuild, else it goes to pos2/vel2.
template <bool ENERGY, bool RECORD, bool BIN>
__global__ void __launch_bounds__(kWave) k_forces_list(SimArgs a) {
    if (a.hdr[HDR_ERROR] & DEV_ORDER) return;
    extern __shared__ float4 tile[];
    __shared__ Neighbourhood nb;
    force_cell<true, ENERGY, false, true, !BIN, RECORD ? 1 : 2>(a, xcd_block_order(blockIdx.x, a.ncells), tile, nb,
                                                                reinterpret_cast<float*>(tile));
}

// md_step_nlist, right after a rebuild: forces, kick and the next drift as
// k_forces_list, and every atom's neighbour list within the list radius.
template <bool ENERGY, bool BIN>
__global__ void __launch_bounds__(kWave) k_forces_record(SimArgs a) {
    if (a.hdr[HDR_ERROR] & DEV_ORDER) return;
    extern __shared__ float4 tile[];  // a.tile_cap + kTilePad positions, then as many 4-byte list entries
    __shared__ Neighbourhood nb;
    force_cell<true, ENERGY, false, true, !BIN, 3>(a, xcd_block_order(blockIdx.x, a.ncells), tile, nb,
                                                   reinterpret_cast<float*>(tile), tile + (a.tile_cap + kTilePad));
}

// md_step_nlist between rebuilds: kListLanes lanes per atom (sorted slots,
// in the XCD order of the cell kernels) walk the atom's neighbour list, lane
// s taking entry groups s, s + kListLanes, ...: partner j at x_j + s L (s
// from the entry's image code), the truncated, shifted force of section 2
// for r < r_c; the lanes' partials are added in a fixed order, then the
// first lane of each atom applies the kick and the next half kick and drift
// as the cell passes do (BIN: wrap and bin for the next rebuild; else
// unwrapped into pos2/vel2 with the displacement check against the
// positions the lists were written at). The displacement is formed as
// (x_i - max(sL, 0)) - (x_j + min(sL, 0)): an image shift is taken off the
// coordinate that lies within a cell of the far box face, where the
// subtraction is exact, so d carries only the rounding of small numbers (as
// the frame translation of the cell passes does).
constexpr int kListBlock = 256;
constexpr int kListLanes = 4;
constexpr int kListAtoms = kListBlock / kListLanes;

template <bool BIN>
__global__ void __launch_bounds__(kListBlock) k_nlist_forces(SimArgs a) {
    if (a.hdr[HDR_ERROR] & DEV_ORDER) return;
    // max(s L, 0) and min(s L, 0) of each image code (the five code bits
    // index 32 entries; codes past 26 never occur and shift by nothing)
    constexpr int kCenter = 13;  // (0, 0, 0)
    __shared__ float4 shp[32], shm[32];
    if (threadIdx.x < 32) {
        const int code = threadIdx.x < 27 ? threadIdx.x : kCenter;
        const float sx = static_cast<float>(code % 3 - 1) * a.box, sy = static_cast<float>((code / 3) % 3 - 1) * a.box,
                    sz = static_cast<float>(code / 9 - 1) * a.box;
        shp[threadIdx.x] = make_float4(fmaxf(sx, 0.f), fmaxf(sy, 0.f), fmaxf(sz, 0.f), 0.f);
        shm[threadIdx.x] = make_float4(fminf(sx, 0.f), fminf(sy, 0.f), fminf(sz, 0.f), 0.f);
    }
    __syncthreads();
    const int lane = __lane_id();
    const char* pbase = reinterpret_cast<const char*>(a.pos0);
    const int last = a.n - 1;
    const int sl = threadIdx.x % kListLanes;
    const int i = xcd_block_order(blockIdx.x, gridDim.x) * kListAtoms + static_cast<int>(threadIdx.x) / kListLanes;
    const bool valid = i < a.n;
    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
    int cnt = 0;
    if (valid) {
        pi = a.pos0[i];
        cnt = min(max(a.ncount[i], 0), a.nlist_cap);
    }
    // entries 4 g .. 4 g + 3 of every atom are one uint4, and the atoms' uint4
    // of one group are consecutive
    const uint4* col = reinterpret_cast<const uint4*>(a.nlist) + (valid ? i : 0);
    float fx = 0.f, fy = 0.f, fz = 0.f, u_loc = 0.f, w_loc = 0.f;
    // the capacity is a multiple of 4: whole uint4 loads. Each group's four
    // partners are requested together and the next group's entries are in
    // flight during this group's arithmetic; image shifts (pairs across a box
    // face, rare) are applied once all four partners have arrived.
    int g = sl;
    uint4 e4 = 4 * g < cnt ? col[static_cast<size_t>(a.n) * g] : make_uint4(0u, 0u, 0u, 0u);
    for (; 4 * g < cnt; g += kListLanes) {
        const uint32_t e[4] = {e4.x, e4.y, e4.z, e4.w};
        float4 q[4];
        int code[4];
        bool in[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            in[u] = 4 * g + u < cnt;
            // entries past the count are not this atom's: read the atom itself, masked
            const uint32_t ej = in[u] ? e[u] : (static_cast<uint32_t>(i) | (kCenter << kSlotBits));
            const uint32_t off = static_cast<uint32_t>(min(static_cast<int>(ej & kSlotMask), last)) << 4;
            q[u] = *reinterpret_cast<const float4*>(pbase + off);
            code[u] = static_cast<int>(ej >> kSlotBits);
        }
        const int gn = g + kListLanes;
        if (4 * gn < cnt) e4 = col[static_cast<size_t>(a.n) * gn];
        float xs[4], ys[4], zs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xs[u] = pi.x;
            ys[u] = pi.y;
            zs[u] = pi.z;
        }
        const bool shifted = (code[0] != kCenter) | (code[1] != kCenter) | (code[2] != kCenter) | (code[3] != kCenter);
        if (__any(shifted)) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 hp = shp[code[u]], hm = shm[code[u]];
                q[u].x += hm.x;
                q[u].y += hm.y;
                q[u].z += hm.z;
                xs[u] -= hp.x;
                ys[u] -= hp.y;
                zs[u] -= hp.z;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pair_force<false>(a, q[u], xs[u], ys[u], zs[u], in[u], fx, fy, fz, u_loc, w_loc);
    }
    // the atom's lanes are consecutive: sum (s0 + s1) + (s2 + s3)
#pragma unroll
    for (int off = 1; off < kListLanes; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
    }
    // the epilogue on one lane per atom: atom lane l of the wave's 16 from lane
    // kListLanes * l, so that consecutive atoms sit in consecutive lanes (the
    // binning's runs)
    const int src = (lane * kListLanes) & (kWave - 1);
    const float gx = __shfl(fx, src), gy = __shfl(fy, src), gz = __shfl(fz, src);
    const int ia = (i - static_cast<int>(threadIdx.x % kWave) / kListLanes) + lane;  // the wave's first atom + lane
    const bool own = lane < kWave / kListLanes && ia < a.n;
    bool bad = false;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f), p_next = v;
    if (own) {
        p_next = a.pos0[ia];
        v = a.vel0[ia];
        bad = !finite3(gx, gy, gz);
        v.x += a.hdt_m * gx;
        v.y += a.hdt_m * gy;
        v.z += a.hdt_m * gz;
    }
    if (BIN) {
        int c_next = -1;
        if (own) c_next = half_kick_drift(a, p_next, v, gx, gy, gz);
        bin_atom(a, p_next, v, c_next);  // all lanes
    } else if (own) {
        const float4 pref = a.posref[ia];
        half_kick_drift_unwrapped(a, p_next, v, gx, gy, gz);
        a.pos2[ia] = p_next;
        a.vel2[ia] = v;
        const float ex = p_next.x - pref.x, ey = p_next.y - pref.y, ez = p_next.z - pref.z;
        if (ex * ex + ey * ey + ez * ez > a.disp_half * a.disp_half) atomicOr(&a.hdr[HDR_ERROR], DEV_SKIN);
    }
    if (bad) atomicOr(&a.hdr[HDR_ERROR], DEV_NONFINITE);
}

// Batched forces: one workgroup per listed cell (global cell indices of the
// replicas of one tile class, XCD-ordered); the replica's own geometry comes
// from its descriptor.
template <bool KICK, bool ENERGY, bool WRITE, bool DRIFT, int MW>
__global__ void __launch_bounds__(MW * kWave)
    k_batch_forces(SimArgs base, const Replica* __restrict__ reps, const int* __restrict__ cell_rep,
                   const int* __restrict__ cells, int ncl) {
    if (base.hdr[HDR_ERROR] & DEV_ORDER) return;
    extern __shared__ float4 tile[];  // cell_lds_entries of the class's largest tile_cap
    __shared__ Neighbourhood nb;
    float* red = reinterpret_cast<float*>(tile);  // slice reduction, as in k_forces
    const int gc = cells[xcd_block_order(blockIdx.x, ncl)];
    const SimArgs a = replica_view(base, reps[cell_rep[gc]]);
    force_cell<KICK, ENERGY, WRITE, DRIFT, false, 0, false, MW>(a, gc - a.cbase, tile, nb, red);
    if (WRITE && blockIdx.x == 0 && threadIdx.x == 0) base.hdr[HDR_STATE] = STATE_FORCES;
}

// Fixed-order final sum of the per-block partials: U = 1/2 sum, W = 1/2 sum
// (every pair is visited from both sides), K as is.
constexpr int kRedBlock = 256;    // batched finals: one workgroup per replica
constexpr int kFinalBlock = 1024; // the single system's final sum
constexpr int kRedUnroll = 8;

// Lane t's running sums of the (U, W, K) partials of blocks t, t + BLOCK,
// t + 2 BLOCK, ... in that order; the loads of kRedUnroll blocks are issued
// before their sums, so the sequential order costs one round trip per
// BLOCK * kRedUnroll blocks.
template <int BLOCK>
__device__ __forceinline__ void sum_partials(const double* __restrict__ e, int n, int t, double& u, double& w,
                                             double& k) {
    for (int b0 = t; b0 < n; b0 += BLOCK * kRedUnroll) {
        double pu[kRedUnroll], pw[kRedUnroll], pk[kRedUnroll];
#pragma unroll
        for (int q = 0; q < kRedUnroll; ++q) {
            const int b = b0 + q * BLOCK;
            const bool ok = b < n;
            pu[q] = ok ? e[3 * b + 0] : 0.0;
            pw[q] = ok ? e[3 * b + 1] : 0.0;
            pk[q] = ok ? e[3 * b + 2] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kRedUnroll; ++q) {
            if (b0 + q * BLOCK < n) {
                u += pu[q];
                w += pw[q];
                k += pk[q];
            }
        }
    }
}
// LOSS: out3[0] = kcoef K + wcoef W instead of (U, K, W). With kcoef and
// wcoef nonzero otherwise, also out3[3] = kcoef K and out3[4] = wcoef (2 K + W)
// (the temperature and the pressure, with kcoef = 2 / (3 N - 3) and
// wcoef = 1 / (3 V)).
template <bool LOSS>
__global__ void __launch_bounds__(kFinalBlock) k_energy_final(SimArgs a, double* out3, bool from_step, double kcoef,
                                                              double wcoef) {
    if (from_step && (a.hdr[HDR_ERROR] & DEV_ORDER)) return;
    __shared__ double su[kFinalBlock], sw[kFinalBlock], sk[kFinalBlock];
    const int t = threadIdx.x;
    double u = 0.0, w = 0.0, k = 0.0;
    sum_partials<kFinalBlock>(a.epart, a.ncells, t, u, w, k);
    su[t] = u;
    sw[t] = w;
    sk[t] = k;
    __syncthreads();
    for (int off = kFinalBlock / 2; off > 0; off >>= 1) {
        if (t < off) {
            su[t] += su[t + off];
            sw[t] += sw[t + off];
            sk[t] += sk[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (LOSS) {
            out3[0] = kcoef * sk[0] + wcoef * (0.5 * sw[0]);
        } else {
            out3[0] = 0.5 * su[0];
            out3[1] = sk[0];
            out3[2] = 0.5 * sw[0];
            if (wcoef != 0.0) {
                out3[3] = kcoef * sk[0];
                out3[4] = wcoef * (2.0 * sk[0] + 0.5 * sw[0]);
            }
        }
    }
}

// Batched final sums: one workgroup per replica, fixed order over its cells;
// out[3 b + 0..2] = U, K, W of replica b.
__global__ void __launch_bounds__(kRedBlock)
    k_batch_energy_final(SimArgs base, const Replica* __restrict__ reps, double* out) {
    if (base.hdr[HDR_ERROR] & DEV_ORDER) return;
    __shared__ double su[kRedBlock], sw[kRedBlock], sk[kRedBlock];
    const Replica r = reps[blockIdx.x];
    const int t = threadIdx.x;
    double u = 0.0, w = 0.0, k = 0.0;
    sum_partials<kRedBlock>(base.epart + 3 * static_cast<size_t>(r.cbase), r.ncells, t, u, w, k);
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
        out[3 * blockIdx.x + 0] = 0.5 * su[0];
        out[3 * blockIdx.x + 1] = sk[0];
        out[3 * blockIdx.x + 2] = 0.5 * sw[0];
    }
}

// Neighbour export through the force kernel's own staging, screen and walk.
// LIST 1 screens against the list radius and keeps the accept words, as the
// force pass right after a rebuild of md_step_list does; LIST 2 walks the
// words kept last, as its passes between rebuilds do.
template <int LIST>
__global__ void __launch_bounds__(kWave) k_neighbors(SimArgs a, ExportArgs ex) {
    if (!state_ok(a, false)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.hdr[HDR_ERROR], DEV_ORDER);
        return;
    }
    extern __shared__ float4 tile[];  // 2 x (tile_cap + kTilePad): frame positions, then untranslated ones
    __shared__ Neighbourhood nb;
    force_cell<false, false, false, false, false, LIST, true>(a, xcd_block_order(blockIdx.x, a.ncells), tile, nb,
                                                              reinterpret_cast<float*>(tile),
                                                              tile + (a.tile_cap + kTilePad), ex);
}

}  // namespace

hipError_t launch_forces(const SimArgs& a_in, bool kick, bool energy, bool write_force, bool from_step, bool drift,
                         int par, hipStream_t st) {
    SimArgs a = a_in;
    a.par = par;
    const dim3 g(a.ncells), b(kWave * a.waves);
    const size_t lds = sizeof(float4) * cell_lds_entries(a.tile_cap, a.waves);
#define MD_FORCES(K, E, W, D)                                                                          \
    do {                                                                                               \
        if (a.waves == 1) hipLaunchKernelGGL((k_forces<K, E, W, D, 1>), g, b, lds, st, a, from_step);  \
        else hipLaunchKernelGGL((k_forces<K, E, W, D, kMaxCellWaves>), g, b, lds, st, a, from_step);   \
    } while (0)
    if (kick && drift && !write_force) {
        if (energy) MD_FORCES(true, true, false, true);
        else MD_FORCES(true, false, false, true);
    } else if (kick && !drift && write_force) {
        if (energy) MD_FORCES(true, true, true, false);
        else MD_FORCES(true, false, true, false);
    } else if (!kick && !drift && energy && !write_force) {
        MD_FORCES(false, true, false, false);
    } else if (!kick && !drift && !energy && write_force) {
        MD_FORCES(false, false, true, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef MD_FORCES
    return hipGetLastError();
}

hipError_t launch_forces_skin(const SimArgs& a, bool energy, hipStream_t st) {
    const dim3 g(a.ncells), b(kWave * a.waves);
    const size_t lds = sizeof(float4) * cell_lds_entries(a.tile_cap, a.waves);
    if (a.waves == 1) {
        if (energy) hipLaunchKernelGGL((k_forces_skin<true, 1>), g, b, lds, st, a);
        else hipLaunchKernelGGL((k_forces_skin<false, 1>), g, b, lds, st, a);
    } else {
        if (energy) hipLaunchKernelGGL((k_forces_skin<true, kMaxCellWaves>), g, b, lds, st, a);
        else hipLaunchKernelGGL((k_forces_skin<false, kMaxCellWaves>), g, b, lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_forces_list(const SimArgs& a_in, bool energy, bool record, bool bin, int par, hipStream_t st) {
    SimArgs a = a_in;
    a.par = par;
    a.waves = 1;  // the kept words are per lane of one wavefront
    const dim3 g(a.ncells), b(kWave);
    const size_t lds = sizeof(float4) * static_cast<size_t>(a.tile_cap + kTilePad);
#define MD_LIST(E, R, B) hipLaunchKernelGGL((k_forces_list<E, R, B>), g, b, lds, st, a)
    if (energy) {
        if (record) {
            if (bin) MD_LIST(true, true, true);
            else MD_LIST(true, true, false);
        } else {
            if (bin) MD_LIST(true, false, true);
            else MD_LIST(true, false, false);
        }
    } else {
        if (record) {
            if (bin) MD_LIST(false, true, true);
            else MD_LIST(false, true, false);
        } else {
            if (bin) MD_LIST(false, false, true);
            else MD_LIST(false, false, false);
        }
    }
#undef MD_LIST
    return hipGetLastError();
}

hipError_t launch_forces_record(const SimArgs& a_in, bool energy, bool bin, int par, hipStream_t st) {
    SimArgs a = a_in;
    a.par = par;
    const dim3 g(a.ncells), b(kWave);
    const size_t entries = static_cast<size_t>(a.tile_cap + kTilePad);
    const size_t lds = sizeof(float4) * entries + sizeof(uint32_t) * entries;
    if (energy) {
        if (bin) hipLaunchKernelGGL((k_forces_record<true, true>), g, b, lds, st, a);
        else hipLaunchKernelGGL((k_forces_record<true, false>), g, b, lds, st, a);
    } else {
        if (bin) hipLaunchKernelGGL((k_forces_record<false, true>), g, b, lds, st, a);
        else hipLaunchKernelGGL((k_forces_record<false, false>), g, b, lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_nlist_forces(const SimArgs& a_in, bool bin, int par, hipStream_t st) {
    SimArgs a = a_in;
    a.par = par;
    const dim3 g((a.n + kListAtoms - 1) / kListAtoms), b(kListBlock);
    if (bin) hipLaunchKernelGGL(k_nlist_forces<true>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_nlist_forces<false>, g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_energy_final(const SimArgs& a, double* out3, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_final<false>, dim3(1), dim3(kFinalBlock), 0, st, a, out3, true, 0.0, 0.0);
    return hipGetLastError();
}

hipError_t launch_thermo_final(const SimArgs& a, double t_coef, double p_coef, double* out5, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_final<false>, dim3(1), dim3(kFinalBlock), 0, st, a, out5, true, t_coef, p_coef);
    return hipGetLastError();
}

hipError_t launch_loss_final(const SimArgs& a, double kcoef, double wcoef, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_final<true>, dim3(1), dim3(kFinalBlock), 0, st, a, out, true, kcoef, wcoef);
    return hipGetLastError();
}

hipError_t launch_batch_forces(const SimArgs& base_in, const Replica* reps, const int* cell_rep, const int* cells,
                               int ncl, int tile_cap, int waves, bool kick, bool energy, bool write_force, bool drift,
                               int par, hipStream_t st) {
    SimArgs base = base_in;
    base.par = par;
    base.waves = waves;
    const dim3 g(ncl), b(kWave * base.waves);
    const size_t lds = sizeof(float4) * cell_lds_entries(tile_cap, base.waves);
#define MD_FORCES(K, E, W, D)                                                                                      \
    do {                                                                                                           \
        if (base.waves == 1)                                                                                       \
            hipLaunchKernelGGL((k_batch_forces<K, E, W, D, 1>), g, b, lds, st, base, reps, cell_rep, cells, ncl);  \
        else                                                                                                       \
            hipLaunchKernelGGL((k_batch_forces<K, E, W, D, kMaxCellWaves>), g, b, lds, st, base, reps, cell_rep,   \
                               cells, ncl);                                                                        \
    } while (0)
    if (kick && drift && !write_force) {
        if (energy) MD_FORCES(true, true, false, true);
        else MD_FORCES(true, false, false, true);
    } else if (kick && !drift && write_force) {
        if (energy) MD_FORCES(true, true, true, false);
        else MD_FORCES(true, false, true, false);
    } else if (!kick && !drift && energy && !write_force) {
        MD_FORCES(false, true, false, false);
    } else if (!kick && !drift && !energy && write_force) {
        MD_FORCES(false, false, true, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef MD_FORCES
    return hipGetLastError();
}

hipError_t launch_batch_energy_final(const SimArgs& base, const Replica* reps, int count, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_energy_final, dim3(count), dim3(kRedBlock), 0, st, base, reps, out);
    return hipGetLastError();
}

hipError_t launch_neighbors(const SimArgs& a, int* counts, int* idx, int max_per_atom, int list, hipStream_t st) {
    hipError_t e = hipMemsetAsync(counts, 0, sizeof(int) * static_cast<size_t>(a.n), st);
    if (e != hipSuccess) return e;
    const ExportArgs ex{counts, idx, max_per_atom};
    const size_t lds = 2 * sizeof(float4) * static_cast<size_t>(a.tile_cap + kTilePad);
    if (list == 1) hipLaunchKernelGGL(k_neighbors<1>, dim3(a.ncells), dim3(kWave), lds, st, a, ex);
    else if (list == 2) hipLaunchKernelGGL(k_neighbors<2>, dim3(a.ncells), dim3(kWave), lds, st, a, ex);
    else hipLaunchKernelGGL(k_neighbors<0>, dim3(a.ncells), dim3(kWave), lds, st, a, ex);
    return hipGetLastError();
}

}  // namespace mdlj
