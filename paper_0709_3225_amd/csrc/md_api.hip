// C-ABI layer: host-side validation, workspace layout and launch sequencing.
// Every entry point validates on the host before touching the device and
// returns an md_status; nothing here throws across the C boundary.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "md.h"
#include "md_internal.h"

namespace mdlj {
namespace {

thread_local char g_err[512] = "no error";

md_status fail(md_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
md_status fail(md_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

md_status hip_fail(hipError_t e, const char* where) {
    return fail(MD_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int32_t kMaxAtoms = 1 << 27;
constexpr int kMaxCellsPerDim = 1024;

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

float cutoff(const md_params* p) {
    const float k = p->rc_over_sigma > 0.f ? p->rc_over_sigma : 2.5f;
    return k * p->sigma;
}

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

md_status validate(const md_params* p) {
    if (!p) return fail(MD_ERR_ARG, "params is NULL");
    if (p->n < 1 || p->n > kMaxAtoms) return fail(MD_ERR_ARG, "n = %d outside [1, 2^27]", p->n);
    if (!finite_pos(p->box)) return fail(MD_ERR_ARG, "box must be finite and > 0");
    if (!finite_pos(p->epsilon) || !finite_pos(p->sigma) || !finite_pos(p->mass))
        return fail(MD_ERR_ARG, "epsilon, sigma and mass must be finite and > 0");
    if (!(std::isfinite(p->rc_over_sigma) && p->rc_over_sigma >= 0.f))
        return fail(MD_ERR_ARG, "rc_over_sigma must be finite and >= 0");
    if (!(std::isfinite(p->dt) && p->dt >= 0.f)) return fail(MD_ERR_ARG, "dt must be finite and >= 0");
    if (!(std::isfinite(p->cell_min) && p->cell_min >= 0.f))
        return fail(MD_ERR_ARG, "cell_min must be finite and >= 0");
    if (!(std::isfinite(p->list_radius) && p->list_radius >= 0.f))
        return fail(MD_ERR_ARG, "list_radius must be finite and >= 0");
    if (p->shift_mode != 0 && p->shift_mode != 1) return fail(MD_ERR_ARG, "shift_mode must be 0 or 1");
    if ((p->flags & ~(MD_FLAG_PAIR_LISTS | MD_FLAG_ATOM_LISTS)) != 0)
        return fail(MD_ERR_ARG, "flags hold unknown bits 0x%x", p->flags);
    if (p->waves_per_cell != 0 && p->waves_per_cell != 1 && p->waves_per_cell != 2 && p->waves_per_cell != 4)
        return fail(MD_ERR_ARG, "waves_per_cell must be 0, 1, 2 or 4 (got %d)", p->waves_per_cell);
    if (p->tile_cap != 0 && (p->tile_cap < 128 || p->tile_cap > 2048 || p->tile_cap % 64 != 0))
        return fail(MD_ERR_ARG, "tile_cap must be 0 or a multiple of 64 in [128, 2048] (got %d)", p->tile_cap);
    const float rc = cutoff(p);
    if (!(rc > 0.f) || !std::isfinite(rc)) return fail(MD_ERR_ARG, "cutoff must be finite and > 0");
    if (!(p->box >= 2.0f * rc)) return fail(MD_ERR_BOX, "box %g is shorter than two cutoffs (2 * %g)", p->box, rc);
    return MD_OK;
}

// Cells per dimension: int(L / side_min) (section 3.2), lowered while the
// side exceeds the minimum by less than 2^-18 L.
int cells_per_dim(const md_params* p) {
    const double L = p->box;
    const double smin = std::max(static_cast<double>(cutoff(p)), static_cast<double>(p->cell_min));
    int nc = static_cast<int>(std::floor(L / smin));
    while (nc > 1 && L / nc - smin < std::ldexp(L, -18)) --nc;
    if (nc > kMaxCellsPerDim) nc = kMaxCellsPerDim;
    return nc;
}

// Bucket entries per cell: twice the mean occupancy plus 16, in multiples of
// 16. A liquid's cells rarely hold more than 1.5 times the mean; atoms beyond
// the capacity go to the overflow list, which is correct at any occupancy and
// slow only for cells that use it.
int bucket_capacity(double mean_occupancy) {
    const int cap = static_cast<int>(std::ceil((2.0 * mean_occupancy + 16.0) / 16.0)) * 16;
    return std::min(1024, std::max(32, cap));
}

size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

constexpr int kWaveLanes = 64;  // lanes of the one-wavefront-per-cell kernels (pair-list rows)

// Histograms, buckets, overflow list and CSR offsets of a build over n atoms
// in ncells cells.
template <class Take>
void take_build_arrays(Layout& L, size_t n, size_t ncells, int cap, Take& take) {
    L.nblocks = static_cast<int>((ncells + (size_t{1} << kBlockShift) - 1) >> kBlockShift);
    L.cap = cap;
    L.counts = take(4 * (static_cast<size_t>(L.nblocks) << kBlockShift));  // whole blocks, padding stays zero
    L.bstart = take(4 * static_cast<size_t>(L.nblocks) + 16);
    L.nbstride = static_cast<int>(round_up(static_cast<size_t>(L.nblocks), 64));
    L.bcounts = take(4 * 2 * static_cast<size_t>(L.nbstride));
    L.bpos = take(16 * ncells * static_cast<size_t>(cap));
    L.bvel = take(16 * ncells * static_cast<size_t>(cap));
    L.ovf_cell = take(4 * n);
    L.ovf_rank = take(4 * n);
    L.ovf_idx = take(4 * n);
    L.start = take(4 * (ncells + 1) + 16);
}

// Entries per atom of the neighbour lists: 1.5 x the mean number of atoms
// within the list radius (the cell side) plus 32, in multiples of 32.
int atom_list_capacity(int n, float box, float side) {
    const double rho = static_cast<double>(n) / (static_cast<double>(box) * box * box);
    const double mean = rho * (4.0 / 3.0) * 3.14159265358979 * static_cast<double>(side) * side * side;
    const int cap = static_cast<int>(std::ceil((1.5 * mean + 32.0) / 32.0)) * 32;
    return std::min(std::max(cap, 64), 4096);
}

md_status make_layout(const md_params* p, Layout& L) {
    md_status s = validate(p);
    if (s != MD_OK) return s;
    const int nc = cells_per_dim(p);
    if (nc < 2) return fail(MD_ERR_BOX, "box %g holds fewer than 2 cells of side >= %g", p->box, cutoff(p));
    L.n = p->n;
    L.nc = nc;
    L.ncells = nc * nc * nc;
    L.nforce_blocks = L.ncells;
    L.s = p->box / nc;
    L.inv_s = nc / p->box;
    if (p->list_radius != 0.f && !(p->list_radius > cutoff(p) && p->list_radius <= L.s))
        return fail(MD_ERR_ARG, "list_radius %g outside (r_c, cell side] = (%g, %g]", p->list_radius, cutoff(p), L.s);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t n = static_cast<size_t>(p->n);
    L.hdr = take(sizeof(int) * HDR_WORDS);
    L.pos0 = take(16 * n);
    L.vel0 = take(16 * n);
    L.pos1 = take(16 * n);
    L.vel1 = take(16 * n);
    L.force = take(16 * n);
    L.pos2 = take(16 * n);
    L.vel2 = take(16 * n);
    if (p->flags & (MD_FLAG_PAIR_LISTS | MD_FLAG_ATOM_LISTS)) L.posref = take(16 * n);
    if (p->flags & MD_FLAG_PAIR_LISTS) {  // md_step_list's arrays, only where asked for
        L.plist = take(16 * static_cast<size_t>(L.ncells) * kWaveLanes * kListSpans);
        L.plist_n = take(4 * static_cast<size_t>(L.ncells) * kWaveLanes);
    }
    if (p->flags & MD_FLAG_ATOM_LISTS) {  // md_step_nlist's arrays
        L.nlist_cap = atom_list_capacity(p->n, p->box, p->list_radius > 0.f ? p->list_radius : L.s);
        L.nlist = take(4 * n * static_cast<size_t>(L.nlist_cap));
        L.ncount = take(4 * n);
    }
    take_build_arrays(L, n, static_cast<size_t>(L.ncells), bucket_capacity(static_cast<double>(p->n) / L.ncells),
                      take);
    L.epart = take(sizeof(double) * 3 * static_cast<size_t>(L.nforce_blocks));
    L.total = off;
    return MD_OK;
}

md_status check_ws(const Layout& L, const void* ws, size_t ws_bytes) {
    if (!ws) return fail(MD_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(MD_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(MD_ERR_WORKSPACE, "workspace holds %zu bytes, needs %zu", ws_bytes, L.total);
    return MD_OK;
}

bool aligned16(const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; }

// Screen bound: frame coordinates lie within [-s, 2s) per axis, so |x|^2 <= 12 s^2;
// the FP32 dot-product form of r^2 errs by a few ulp of that. 2^-17 * 12 s^2 leaves a
// wide margin, so the screen never drops a pair that the exact test accepts.
float screen_bound(double rc, double s) { return static_cast<float>(rc * rc + std::ldexp(12.0 * s * s, -17)); }

// One LDS pass of the cell-pair kernels holds the mean 27-cell neighbourhood
// plus 10% and half a wavefront (a liquid's neighbourhood counts vary by a few
// percent; a larger one takes a second pass). A small tile leaves room for
// more wavefronts per CU, which hide the latency of staging.
int tile_capacity(int n, int ncells) {
    const double hood = 27.0 * static_cast<double>(n) / ncells;
    const int cap = static_cast<int>(std::ceil((1.1 * hood + 32.0) / 64.0)) * 64;
    return std::min(2048, std::max(128, cap));
}

// Wavefronts per force workgroup: the caller's choice, else one (which is
// as fast or faster from about 2,000 cells up).
int waves_per_cell(const md_params* p) { return p->waves_per_cell != 0 ? p->waves_per_cell : 1; }

SimArgs make_args(const md_params* p, const Layout& L, void* ws) {
    char* b = static_cast<char*>(ws);
    SimArgs a{};
    a.hdr = reinterpret_cast<int*>(b + L.hdr);
    a.pos0 = reinterpret_cast<float4*>(b + L.pos0);
    a.vel0 = reinterpret_cast<float4*>(b + L.vel0);
    a.pos1 = reinterpret_cast<float4*>(b + L.pos1);
    a.vel1 = reinterpret_cast<float4*>(b + L.vel1);
    a.force = reinterpret_cast<float4*>(b + L.force);
    a.pos2 = L.pos2 ? reinterpret_cast<float4*>(b + L.pos2) : nullptr;
    a.vel2 = L.vel2 ? reinterpret_cast<float4*>(b + L.vel2) : nullptr;
    a.posref = L.posref ? reinterpret_cast<float4*>(b + L.posref) : nullptr;
    a.plist = L.plist ? reinterpret_cast<uint32_t*>(b + L.plist) : nullptr;
    a.plist_n = L.plist_n ? reinterpret_cast<int*>(b + L.plist_n) : nullptr;
    a.nlist = L.nlist ? reinterpret_cast<uint32_t*>(b + L.nlist) : nullptr;
    a.ncount = L.ncount ? reinterpret_cast<int*>(b + L.ncount) : nullptr;
    a.nlist_cap = L.nlist_cap;
    a.counts = reinterpret_cast<int*>(b + L.counts);
    a.bstart = reinterpret_cast<int*>(b + L.bstart);
    a.bpos = reinterpret_cast<float4*>(b + L.bpos);
    a.bvel = reinterpret_cast<float4*>(b + L.bvel);
    a.ovf_cell = reinterpret_cast<int*>(b + L.ovf_cell);
    a.ovf_rank = reinterpret_cast<int*>(b + L.ovf_rank);
    a.ovf_idx = reinterpret_cast<int*>(b + L.ovf_idx);
    a.start = reinterpret_cast<int*>(b + L.start);
    a.nblocks = L.nblocks;
    a.cap = L.cap;
    a.natoms = L.n;
    a.bcounts = reinterpret_cast<int*>(b + L.bcounts);
    a.nbstride = L.nbstride;
    a.par = 0;
    a.direct = L.nblocks <= kDirectBlocks ? 1 : 0;
    a.epart = reinterpret_cast<double*>(b + L.epart);
    a.n = L.n;
    a.nc = L.nc;
    a.ncells = L.ncells;
    a.box = p->box;
    a.s = L.s;
    a.inv_s = L.inv_s;
    // Pair constants: computed in double, rounded once.
    const double eps = p->epsilon, sig = p->sigma;
    const double rc = static_cast<double>(cutoff(p));
    const double sr6 = std::pow(sig / rc, 6.0);
    const double flj_rc = 24.0 * eps / rc * (2.0 * sr6 * sr6 - sr6);  // f_LJ(r_c) = -du_LJ/dr at r_c
    const double ulj_rc = 4.0 * eps * (sr6 * sr6 - sr6);
    a.rc = static_cast<float>(rc);
    a.rc2 = static_cast<float>(rc * rc);
    a.sig2 = static_cast<float>(sig * sig);
    a.eps24 = static_cast<float>(24.0 * eps);
    a.eps4 = static_cast<float>(4.0 * eps);
    const double sig6 = std::pow(sig, 6.0);
    a.c12 = static_cast<float>(48.0 * eps * sig6 * sig6);
    a.c6 = static_cast<float>(24.0 * eps * sig6);
    a.e12 = static_cast<float>(4.0 * eps * sig6 * sig6);
    a.e6 = static_cast<float>(4.0 * eps * sig6);
    a.fc = p->shift_mode == 0 ? static_cast<float>(flj_rc) : 0.f;
    a.uc = static_cast<float>(ulj_rc);
    a.screen2 = screen_bound(rc, L.s);
    // half the margin of the cell side over r_c, less a relative 2^-20 for the
    // FP32 comparison
    a.skin_half = static_cast<float>(std::max(0.0, 0.5 * (static_cast<double>(L.s) - rc) * (1.0 - std::ldexp(1.0, -20))));
    // pair lists: candidates within the cell side when the words are kept;
    // valid while no atom has moved by half the side's margin over r_c
    // pair and neighbour lists: candidates within r_V when recorded; valid
    // while no atom has moved by half of r_V - r_c (less a relative 2^-20)
    const double rv = p->list_radius > 0.f ? static_cast<double>(p->list_radius) : static_cast<double>(L.s);
    a.list_screen2 = screen_bound(rv, L.s);
    a.disp_half = static_cast<float>(std::max(0.0, 0.5 * (rv - rc) * (1.0 - std::ldexp(1.0, -20))));
    a.tile_cap = p->tile_cap != 0 ? p->tile_cap : tile_capacity(p->n, L.ncells);
    a.waves = waves_per_cell(p);
    a.dt = p->dt;
    a.hdt_m = static_cast<float>(0.5 * p->dt / p->mass);
    a.half_m = static_cast<float>(0.5 * p->mass);
    return a;
}

// The trajectory loss of the adjoint: L = K / N + W / (3 V), the mean kinetic
// energy per particle plus the virial part of the pressure; scale * L has
// coefficients kc on K and wc on W.
void loss_coefficients(const md_params* p, double scale, double& kc, double& wc) {
    const double box = p->box;
    kc = scale / static_cast<double>(p->n);
    wc = scale / (3.0 * box * box * box);
}

#define MD_TRY_HIP(expr, where)                  \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)



// Cell offsets and sorted arrays from the binned atoms (block histogram par).
md_status rebuild(const SimArgs& a, int par, bool from_step, hipStream_t st) {
    if (!a.direct) MD_TRY_HIP(launch_block_scan(a, from_step, st), "block scan");
    MD_TRY_HIP(launch_cell_order(a, par, from_step, st), "cell order");
    return MD_OK;
}

// Load a state and build its cell list (md_build_cells after validation).
md_status build_cells_impl(const SimArgs& a, const float4* pos4, const float4* vel4, hipStream_t stream) {
    MD_TRY_HIP(launch_build_init(a, stream), "build init");
    MD_TRY_HIP(launch_load(a, pos4, vel4, stream), "load");
    md_status s = rebuild(a, 0, false, stream);
    if (s != MD_OK) return s;
    MD_TRY_HIP(launch_zero_blocks(a, 0, stream), "counter clear");
    return MD_OK;
}

// ---- a workspace that needs no allocation (md_forces_noalloc) ----------------
// A file-scope device array holds the workspace for callers that cannot
// allocate device memory. Every GPU the library runs on holds its own copy
// until the process ends. In host code the array's name stands for a
// host-side symbol, not a device address: the device address of the current
// GPU's copy comes from hipGetSymbolAddress on the first call on that device
// and is kept per device; only that address is ever handed to a kernel.
constexpr size_t kScratchBytes = size_t{16} << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

md_status scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kScratchDevices)
        return fail(MD_ERR_ARG, "device %d is beyond the %d devices the static workspace serves", dev, kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(MD_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MD_OK;
}

// nsteps fused velocity-Verlet steps (md_step after validation).
md_status steps_impl(const SimArgs& a, int32_t nsteps, int32_t thermo_every, double* thermo, hipStream_t stream) {
    // The force pass of every step but the last also performs the next step's
    // half kick, drift and binning, so the drift kernel runs only on the first
    // step; a rebuild is then the block scan (large grids) and the cell order.
    // Step k's atoms are binned with parity (k - 1) mod 2; the counters of
    // both parities are zero again on return.
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool energy = thermo && thermo_every > 0 && (k % thermo_every) == 0;
        const bool last = k == nsteps;
        if (k == 1) MD_TRY_HIP(launch_integrate(a, stream), "integrate");
        md_status s = rebuild(a, (k - 1) & 1, true, stream);
        if (s != MD_OK) return s;
        MD_TRY_HIP(launch_forces(a, true, energy, last, true, !last, k & 1, stream), "forces");
        if (energy)
            MD_TRY_HIP(launch_energy_final(a, thermo + 3 * static_cast<size_t>(k / thermo_every - 1), stream),
                       "energy");
    }
    if (nsteps > 0) MD_TRY_HIP(launch_zero_blocks(a, (nsteps - 1) & 1, stream), "counter clear");
    return MD_OK;
}

// ---- kept paths of the adjoint --------------------------------------------

// Arguments whose sorted positions and cell offsets are path slice j: a
// path holds nsteps states, slice j being n float4 and n_c^3 + 1 offsets.
SimArgs path_slice(const SimArgs& a, float* path4, int32_t* path_start, int32_t j) {
    SimArgs x = a;
    x.pos0 = reinterpret_cast<float4*>(path4) + static_cast<size_t>(j) * static_cast<size_t>(a.n);
    x.start = path_start + static_cast<size_t>(j) * (static_cast<size_t>(a.ncells) + 1);
    return x;
}

md_status check_path_args(const md_params* p, int32_t first_step, int32_t nsteps, const float* path4,
                          const int32_t* path_start, bool adjoint) {
    if (adjoint && p->shift_mode != 0) return fail(MD_ERR_ARG, "the adjoint needs shift_mode 0 (force shift)");
    if (nsteps < 1 || first_step < 0) return fail(MD_ERR_ARG, "need nsteps >= 1 and first_step >= 0");
    if (!path4 || !path_start) return fail(MD_ERR_ARG, "path arrays are NULL");
    if (!aligned16(path4)) return fail(MD_ERR_ARG, "path4 must be 16-byte aligned");
    return MD_OK;
}

md_status check_ckpt(const float* pos4, const float* vel4) {
    if (!pos4 || !vel4) return fail(MD_ERR_ARG, "checkpoint arrays are NULL");
    if (!aligned16(pos4) || !aligned16(vel4)) return fail(MD_ERR_ARG, "checkpoint arrays must be 16-byte aligned");
    return MD_OK;
}

md_status check_adjoint_vecs(const float* lam_r4, const float* lam_v4) {
    if (!lam_r4 || !lam_v4) return fail(MD_ERR_ARG, "adjoint vectors are NULL");
    if (!aligned16(lam_r4) || !aligned16(lam_v4)) return fail(MD_ERR_ARG, "adjoint vectors must be 16-byte aligned");
    if (lam_r4 == lam_v4) return fail(MD_ERR_ARG, "lam_r and lam_v must not alias");
    return MD_OK;
}

// From a checkpoint, the states of a segment into the path: the checkpoint's
// cells (as md_build_cells), then the steps in md_step's fused order
// (bitwise the states md_step produces). The last state needs no forces:
// only its positions are used on the way back. The workspace's own sorted
// arrays are not written.
md_status recompute_impl(const SimArgs& a, const float* ckpt_pos4, const float* ckpt_vel4, int32_t nsteps,
                         float* path4, int32_t* path_start, hipStream_t stream) {
    const SimArgs a0 = path_slice(a, path4, path_start, 0);
    MD_TRY_HIP(launch_build_init(a0, stream), "build init");
    MD_TRY_HIP(launch_load(a0, reinterpret_cast<const float4*>(ckpt_pos4), reinterpret_cast<const float4*>(ckpt_vel4),
                           stream),
               "load");
    md_status s = rebuild(a0, 0, false, stream);
    if (s != MD_OK) return s;
    MD_TRY_HIP(launch_zero_blocks(a0, 0, stream), "counter clear");
    if (nsteps > 1) {
        MD_TRY_HIP(launch_forces(a0, false, false, true, false, false, 0, stream), "forces");
        MD_TRY_HIP(launch_integrate(a0, stream), "integrate");
        for (int32_t k = 1; k < nsteps; ++k) {
            const SimArgs ak = path_slice(a, path4, path_start, k);
            if ((s = rebuild(ak, (k - 1) & 1, true, stream)) != MD_OK) return s;
            if (k + 1 < nsteps) MD_TRY_HIP(launch_forces(ak, true, false, false, true, true, k & 1, stream), "forces");
        }
        MD_TRY_HIP(launch_zero_blocks(a, (nsteps - 2) & 1, stream), "counter clear");
    }
    return MD_OK;
}

// From the last state of a kept path back to its first: drift adjoint, then
// the kick adjoint on state j's cell list, with coefficient 2h, or h for the
// trajectory's step 0 (h = dt / 2m); the parameter terms are summed per cell
// over the path and added to theta once. Uses the workspace as scratch only.
md_status sweep_impl(const SimArgs& a, const md_params* p, int32_t first_step, int32_t nsteps, float* path4,
                     int32_t* path_start, float* lam_r4, float* lam_v4, double* theta, hipStream_t stream) {
    const float h = static_cast<float>(0.5 * p->dt / p->mass);
    for (int32_t j = nsteps - 1; j >= 0; --j) {
        const float coef = first_step + j >= 1 ? 2.0f * h : h;
        MD_TRY_HIP(launch_adjoint_drift_kick(path_slice(a, path4, path_start, j), p->dt,
                                             reinterpret_cast<float4*>(lam_r4), reinterpret_cast<float4*>(lam_v4), coef,
                                             j < nsteps - 1, stream),
                   "adjoint drift and kick");
    }
    if (theta) MD_TRY_HIP(launch_theta_final(a, theta, 1.0, stream), "parameter sums");
    return MD_OK;
}

// ---- batches of independent replicas -------------------------------------

// The batched force pass runs one launch per tile class: replicas whose
// neighbourhood tile falls into the same band, and that take the same
// number of wavefronts per cell, share a launch whose LDS fits the band's
// largest tile, so a few replicas with crowded cells do not cut the number
// of resident waves for all the others (about 16 per CU with tiles of up to
// 512 atoms, 9 with 1,024). Band upper bounds:
constexpr int kTileBands[] = {512, 640, 768, 1024, 2048};
constexpr int kNumTileBands = sizeof(kTileBands) / sizeof(kTileBands[0]);
constexpr int kWaveChoices[] = {1, 2, 4};  // wavefronts per cell, one class each
constexpr int kNumWaveChoices = 3;
constexpr int kNumClasses = kNumTileBands * kNumWaveChoices;

struct TileClass {
    int first = 0, ncells = 0, tile_cap = 0;  // range in the class cell list; largest tile_cap
    int waves = 1;
};

struct BatchPlan {
    Layout L{};                  // shared arrays; n = total atoms, ncells = total cells (unused offsets 0)
    int count = 0;
    double max_mean = 0.0;  // largest mean cell occupancy of any replica
    size_t reps = 0, atom_rep = 0, cell_rep = 0, class_cells = 0;
    std::vector<Replica> table;  // host copy of the replica table
    std::vector<int> waves;      // wavefronts per cell of each replica
    TileClass classes[kNumClasses];
};

int tile_band(int tile_cap) {
    for (int k = 0; k < kNumTileBands; ++k)
        if (tile_cap <= kTileBands[k]) return k;
    return kNumTileBands - 1;  // no tile exceeds the last band
}

// Class of a replica: its tile band and its wavefront count.
int tile_class(int tile_cap, int waves) {
    const int w = waves == 4 ? 2 : waves - 1;
    return tile_band(tile_cap) * kNumWaveChoices + w;
}

constexpr int32_t kMaxReplicas = 1 << 16;

// Validate every replica (shared parameters from p, n and box per replica)
// and lay out the batch workspace.
md_status batch_plan(const md_params* p, const md_replica* reps, int32_t count, BatchPlan& B) {
    if (!p) return fail(MD_ERR_ARG, "params is NULL");
    if (!reps) return fail(MD_ERR_ARG, "replica table is NULL");
    if (count < 1 || count > kMaxReplicas) return fail(MD_ERR_ARG, "replica count %d outside [1, 65536]", count);
    B.count = count;
    B.table.resize(count);
    B.waves.resize(count);
    int64_t ntot = 0, ctot = 0;
    for (int32_t b = 0; b < count; ++b) {
        md_params q = *p;
        q.n = reps[b].n;
        q.box = reps[b].box;
        q.tile_cap = 0;
        if (reps[b].cell_min != 0.f) q.cell_min = reps[b].cell_min;  // validated by make_layout
        const int32_t rw = reps[b].waves_per_cell, rt = reps[b].tile_cap;
        if (rw != 0 && rw != 1 && rw != 2 && rw != 4)
            return fail(MD_ERR_ARG, "replica %d: waves_per_cell must be 0, 1, 2 or 4 (got %d)", b, rw);
        if (rt != 0 && (rt < 128 || rt > 2048 || rt % 64 != 0))
            return fail(MD_ERR_ARG, "replica %d: tile_cap must be 0 or a multiple of 64 in [128, 2048] (got %d)", b,
                        rt);
        if (rw != 0) q.waves_per_cell = rw;
        Layout Lb{};
        const md_status s = make_layout(&q, Lb);
        if (s != MD_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "%s", g_err);
            return fail(s, "replica %d: %s", b, msg);
        }
        Replica& r = B.table[b];
        r.n = q.n;
        r.abase = static_cast<int>(ntot);
        r.nc = Lb.nc;
        r.ncells = Lb.ncells;
        r.cbase = static_cast<int>(ctot);
        r.tile_cap = rt != 0 ? rt : tile_capacity(q.n, Lb.ncells);
        B.waves[b] = waves_per_cell(&q);
        r.box = q.box;
        r.s = Lb.s;
        r.inv_s = Lb.inv_s;
        r.screen2 = screen_bound(static_cast<double>(cutoff(&q)), Lb.s);
        B.max_mean = std::max(B.max_mean, static_cast<double>(q.n) / Lb.ncells);
        ntot += q.n;
        ctot += Lb.ncells;
        if (ntot > kMaxAtoms) return fail(MD_ERR_ARG, "batch holds more than 2^27 atoms");
        if (ctot > (int64_t{1} << 30)) return fail(MD_ERR_ARG, "batch holds more than 2^30 cells");
    }
    // tile classes: each class's replicas in table order, classes one after another
    for (int k = 0; k < kNumClasses; ++k) B.classes[k].waves = kWaveChoices[k % kNumWaveChoices];
    for (int32_t b = 0; b < count; ++b) {
        const Replica& r = B.table[b];
        TileClass& t = B.classes[tile_class(r.tile_cap, B.waves[b])];
        t.ncells += r.ncells;
        t.tile_cap = std::max(t.tile_cap, r.tile_cap);
    }
    int first = 0;
    for (TileClass& t : B.classes) {
        t.first = first;
        first += t.ncells;
    }
    int fill[kNumClasses] = {};
    for (int32_t b = 0; b < count; ++b) {
        Replica& r = B.table[b];
        const int k = tile_class(r.tile_cap, B.waves[b]);
        r.lbase = B.classes[k].first + fill[k];
        fill[k] += r.ncells;
    }
    Layout& L = B.L;
    L.n = static_cast<int>(ntot);
    L.nc = -count;  // marks a batch workspace in the device header
    L.ncells = static_cast<int>(ctot);
    L.nforce_blocks = L.ncells;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t n = static_cast<size_t>(L.n), c = static_cast<size_t>(L.ncells);
    L.hdr = take(sizeof(int) * HDR_WORDS);
    B.reps = take(sizeof(Replica) * static_cast<size_t>(count));
    B.atom_rep = take(4 * n);
    B.cell_rep = take(4 * c);
    B.class_cells = take(4 * c);
    L.pos0 = take(16 * n);
    L.vel0 = take(16 * n);
    L.pos1 = take(16 * n);
    L.vel1 = take(16 * n);
    L.force = take(16 * n);
    take_build_arrays(L, n, c, bucket_capacity(B.max_mean), take);
    L.epart = take(sizeof(double) * 3 * c);
    L.total = off;
    return MD_OK;
}

struct BatchArgs {
    SimArgs base;
    const Replica* reps;
    int* atom_rep;
    int* cell_rep;
    int* class_cells;
};

BatchArgs batch_args(const md_params* p, const BatchPlan& B, void* ws) {
    md_params q = *p;  // shared constants; per-replica geometry lives in the table
    q.n = B.table[0].n;
    q.box = B.table[0].box;
    BatchArgs ba{};
    ba.base = make_args(&q, B.L, ws);
    char* b = static_cast<char*>(ws);
    ba.reps = reinterpret_cast<const Replica*>(b + B.reps);
    ba.atom_rep = reinterpret_cast<int*>(b + B.atom_rep);
    ba.cell_rep = reinterpret_cast<int*>(b + B.cell_rep);
    ba.class_cells = reinterpret_cast<int*>(b + B.class_cells);
    return ba;
}

// The batched force pass: one launch per non-empty tile class.
hipError_t batch_forces(const BatchPlan& B, const BatchArgs& ba, bool kick, bool energy, bool write_force,
                        bool drift, int par, hipStream_t st) {
    for (const TileClass& t : B.classes) {
        if (t.ncells == 0) continue;
        const hipError_t e = launch_batch_forces(ba.base, ba.reps, ba.cell_rep, ba.class_cells + t.first, t.ncells,
                                                 t.tile_cap, t.waves, kick, energy, write_force, drift, par, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

md_status batch_prepare(const md_params* p, const md_replica* reps, int32_t count, const void* ws, size_t ws_bytes,
                        BatchPlan& B) {
    md_status s = batch_plan(p, reps, count, B);
    if (s != MD_OK) return s;
    return check_ws(B.L, ws, ws_bytes);
}

// nsteps batched velocity-Verlet steps (kernels only, so the sequence can be
// captured into a graph).
md_status batch_steps(const BatchPlan& B, const BatchArgs& ba, int32_t nsteps, int32_t thermo_every, double* thermo,
                      hipStream_t st) {
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool energy = thermo && thermo_every > 0 && (k % thermo_every) == 0;
        const bool last = k == nsteps;
        if (k == 1) MD_TRY_HIP(launch_batch_integrate(ba.base, ba.reps, ba.atom_rep, st), "batch integrate");
        md_status s = rebuild(ba.base, (k - 1) & 1, true, st);
        if (s != MD_OK) return s;
        MD_TRY_HIP(batch_forces(B, ba, true, energy, last, !last, k & 1, st), "batch forces");
        if (energy)
            MD_TRY_HIP(launch_batch_energy_final(ba.base, ba.reps, B.count,
                                                 thermo + 3 * static_cast<size_t>(B.count) * (k / thermo_every - 1), st),
                       "batch energy");
    }
    if (nsteps > 0) MD_TRY_HIP(launch_zero_blocks(ba.base, (nsteps - 1) & 1, st), "batch counter clear");
    return MD_OK;
}

}  // namespace
}  // namespace mdlj

using namespace mdlj;

extern "C" {

size_t md_workspace_bytes(const md_params* p) {
    Layout L{};
    if (make_layout(p, L) != MD_OK) return 0;
    return L.total;
}

md_status md_cell_grid(const md_params* p, int32_t* cells_per_dim_out, float* cell_side) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if (cells_per_dim_out) *cells_per_dim_out = L.nc;
    if (cell_side) *cell_side = L.s;
    return MD_OK;
}

int32_t md_tile_capacity(const md_params* p) {
    Layout L{};
    if (make_layout(p, L) != MD_OK) return 0;
    return p->tile_cap != 0 ? p->tile_cap : tile_capacity(p->n, L.ncells);
}

md_status md_build_cells(const md_params* p, void* ws, size_t ws_bytes, const float* pos4, const float* vel4,
                         hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!pos4) return fail(MD_ERR_ARG, "positions are NULL");
    if (!aligned16(pos4) || (vel4 && !aligned16(vel4))) return fail(MD_ERR_ARG, "particle arrays must be 16-byte aligned");
    const SimArgs a = make_args(p, L, ws);
    return build_cells_impl(a, reinterpret_cast<const float4*>(pos4), reinterpret_cast<const float4*>(vel4), stream);
}

md_status md_forces(const md_params* p, void* ws, size_t ws_bytes, float* force4, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (force4 && !aligned16(force4)) return fail(MD_ERR_ARG, "force array must be 16-byte aligned");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_forces(a, false, false, true, false, false, 0, stream), "forces");
    if (force4) MD_TRY_HIP(launch_gather_user(a, nullptr, nullptr, reinterpret_cast<float4*>(force4), stream), "gather");
    return MD_OK;
}

md_status md_forces_noalloc(const md_params* p, const float* pos4, float* force4, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if (L.total > kScratchBytes)
        return fail(MD_ERR_WORKSPACE, "these parameters need a %zu-byte workspace; the static one holds %zu bytes",
                    L.total, kScratchBytes);
    if (!pos4 || !force4) return fail(MD_ERR_ARG, "positions and forces must not be NULL");
    if (!aligned16(pos4) || !aligned16(force4)) return fail(MD_ERR_ARG, "particle arrays must be 16-byte aligned");
    void* ws = nullptr;
    if ((s = scratch_address(&ws)) != MD_OK) return s;
    const SimArgs a = make_args(p, L, ws);
    if ((s = build_cells_impl(a, reinterpret_cast<const float4*>(pos4), nullptr, stream)) != MD_OK) return s;
    MD_TRY_HIP(launch_forces(a, false, false, true, false, false, 0, stream), "forces");
    MD_TRY_HIP(launch_gather_user(a, nullptr, nullptr, reinterpret_cast<float4*>(force4), stream), "gather");
    return MD_OK;
}

md_status md_step(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps, int32_t thermo_every,
                  double* thermo, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (nsteps < 0) return fail(MD_ERR_ARG, "nsteps must be >= 0");
    if (thermo_every < 0) return fail(MD_ERR_ARG, "thermo_every must be >= 0");
    if (thermo_every > 0 && !thermo) return fail(MD_ERR_ARG, "thermo_every > 0 needs a thermo buffer");
    return steps_impl(make_args(p, L, ws), nsteps, thermo_every, thermo, stream);
}

md_status md_step_every(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps, int32_t rebuild_every,
                        int32_t thermo_every, double* thermo, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (nsteps < 0) return fail(MD_ERR_ARG, "nsteps must be >= 0");
    if (rebuild_every < 1) return fail(MD_ERR_ARG, "rebuild_every must be >= 1");
    if (thermo_every < 0) return fail(MD_ERR_ARG, "thermo_every must be >= 0");
    if (thermo_every > 0 && !thermo) return fail(MD_ERR_ARG, "thermo_every > 0 needs a thermo buffer");
    const SimArgs a = make_args(p, L, ws);
    SimArgs alt = a;  // reads the alternate sorted buffers, drifts into the canonical ones
    std::swap(alt.pos0, alt.pos2);
    std::swap(alt.vel0, alt.vel2);
    // Cells are rebuilt before the forces of steps 1, 1 + e, 1 + 2e, ... and of
    // the last step (so the call ends on a rebuilt, wrapped state with forces
    // in the canonical order, as md_step does). The step before a rebuild bins
    // in its force epilogue exactly as md_step; the other steps drift into the
    // alternate buffers (unwrapped) and the live pair flips. Build b bins with
    // parity b mod 2, as consecutive steps do in md_step.
    int b = 0;
    bool live_alt = false;
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool energy = thermo && thermo_every > 0 && (k % thermo_every) == 0;
        const bool last = k == nsteps;
        const bool rebuild_now = k == 1 || last || (k - 1) % rebuild_every == 0;
        const bool rebuild_next = !last && (k + 1 == nsteps || k % rebuild_every == 0);
        if (k == 1) MD_TRY_HIP(launch_integrate(a, stream), "integrate");
        if (rebuild_now) {
            if (k > 1) ++b;
            if ((s = rebuild(a, b & 1, true, stream)) != MD_OK) return s;
            live_alt = false;
        }
        const SimArgs& cur = live_alt ? alt : a;
        if (last || rebuild_next) {
            MD_TRY_HIP(launch_forces(cur, true, energy, last, true, !last, (b + 1) & 1, stream), "forces");
        } else {
            MD_TRY_HIP(launch_forces_skin(cur, energy, stream), "forces");
            live_alt = !live_alt;
        }
        if (energy)
            MD_TRY_HIP(launch_energy_final(a, thermo + 3 * static_cast<size_t>(k / thermo_every - 1), stream),
                       "energy");
    }
    if (nsteps > 0) MD_TRY_HIP(launch_zero_blocks(a, b & 1, stream), "counter clear");
    return MD_OK;
}

md_status md_step_list(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps, int32_t rebuild_every,
                       int32_t thermo_every, double* thermo, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (nsteps < 0) return fail(MD_ERR_ARG, "nsteps must be >= 0");
    if (rebuild_every < 1) return fail(MD_ERR_ARG, "rebuild_every must be >= 1");
    if (thermo_every < 0) return fail(MD_ERR_ARG, "thermo_every must be >= 0");
    if (thermo_every > 0 && !thermo) return fail(MD_ERR_ARG, "thermo_every > 0 needs a thermo buffer");
    if (!(p->flags & MD_FLAG_PAIR_LISTS))
        return fail(MD_ERR_ARG, "md_step_list needs a workspace laid out with MD_FLAG_PAIR_LISTS");
    const SimArgs a = make_args(p, L, ws);
    SimArgs alt = a;
    std::swap(alt.pos0, alt.pos2);
    std::swap(alt.vel0, alt.vel2);
    // The schedule of md_step_every; the force pass right after a rebuild
    // keeps every lane's accept words (screened against the cell side), the
    // others walk the kept words instead of screening.
    int b = 0;
    bool live_alt = false;
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool energy = thermo && thermo_every > 0 && (k % thermo_every) == 0;
        const bool last = k == nsteps;
        const bool rebuild_now = k == 1 || last || (k - 1) % rebuild_every == 0;
        const bool rebuild_next = !last && (k + 1 == nsteps || k % rebuild_every == 0);
        if (k == 1) MD_TRY_HIP(launch_integrate(a, stream), "integrate");
        if (rebuild_now) {
            if (k > 1) ++b;
            if ((s = rebuild(a, b & 1, true, stream)) != MD_OK) return s;
            live_alt = false;
        }
        const SimArgs& cur = live_alt ? alt : a;
        if (last) {
            MD_TRY_HIP(launch_forces(cur, true, energy, true, true, false, (b + 1) & 1, stream), "forces");
        } else {
            MD_TRY_HIP(launch_forces_list(cur, energy, rebuild_now, rebuild_next, (b + 1) & 1, stream), "forces");
            if (!rebuild_next) live_alt = !live_alt;
        }
        if (energy)
            MD_TRY_HIP(launch_energy_final(a, thermo + 3 * static_cast<size_t>(k / thermo_every - 1), stream),
                       "energy");
    }
    if (nsteps > 0) MD_TRY_HIP(launch_zero_blocks(a, b & 1, stream), "counter clear");
    return MD_OK;
}

md_status md_step_nlist(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps, int32_t rebuild_every,
                        int32_t thermo_every, double* thermo, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (nsteps < 0) return fail(MD_ERR_ARG, "nsteps must be >= 0");
    if (rebuild_every < 1) return fail(MD_ERR_ARG, "rebuild_every must be >= 1");
    if (thermo_every < 0) return fail(MD_ERR_ARG, "thermo_every must be >= 0");
    if (thermo_every > 0 && !thermo) return fail(MD_ERR_ARG, "thermo_every > 0 needs a thermo buffer");
    if (!(p->flags & MD_FLAG_ATOM_LISTS))
        return fail(MD_ERR_ARG, "md_step_nlist needs a workspace laid out with MD_FLAG_ATOM_LISTS");
    const SimArgs a = make_args(p, L, ws);
    SimArgs alt = a;
    std::swap(alt.pos0, alt.pos2);
    std::swap(alt.vel0, alt.vel2);
    // The schedule of md_step_every; the force pass right after a rebuild
    // writes the neighbour lists, the others walk them (thermo steps screen).
    int b = 0;
    bool live_alt = false;
    bool lists = false;  // lists written since the last rebuild
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool energy = thermo && thermo_every > 0 && (k % thermo_every) == 0;
        const bool last = k == nsteps;
        const bool rebuild_now = k == 1 || last || (k - 1) % rebuild_every == 0;
        const bool rebuild_next = !last && (k + 1 == nsteps || k % rebuild_every == 0);
        if (k == 1) MD_TRY_HIP(launch_integrate(a, stream), "integrate");
        if (rebuild_now) {
            if (k > 1) ++b;
            if ((s = rebuild(a, b & 1, true, stream)) != MD_OK) return s;
            live_alt = false;
            lists = false;
        }
        const SimArgs& cur = live_alt ? alt : a;
        const int par = (b + 1) & 1;
        if (last) {
            MD_TRY_HIP(launch_forces(cur, true, energy, true, true, false, par, stream), "forces");
        } else if (rebuild_now) {
            MD_TRY_HIP(launch_forces_record(cur, energy, rebuild_next, par, stream), "forces");
            lists = true;
            if (!rebuild_next) live_alt = !live_alt;
        } else if (energy || !lists) {
            if (rebuild_next) {
                MD_TRY_HIP(launch_forces(cur, true, energy, false, true, true, par, stream), "forces");
            } else {
                MD_TRY_HIP(launch_forces_skin(cur, energy, stream), "forces");
                live_alt = !live_alt;
            }
        } else {
            MD_TRY_HIP(launch_nlist_forces(cur, rebuild_next, par, stream), "forces");
            if (!rebuild_next) live_alt = !live_alt;
        }
        if (energy)
            MD_TRY_HIP(launch_energy_final(a, thermo + 3 * static_cast<size_t>(k / thermo_every - 1), stream),
                       "energy");
    }
    if (nsteps > 0) MD_TRY_HIP(launch_zero_blocks(a, b & 1, stream), "counter clear");
    return MD_OK;
}

md_status md_energy_virial(const md_params* p, void* ws, size_t ws_bytes, double* out3, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!out3) return fail(MD_ERR_ARG, "output is NULL");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_forces(a, false, true, false, false, false, 0, stream), "energy pass");
    MD_TRY_HIP(launch_energy_final(a, out3, stream), "energy");
    return MD_OK;
}

md_status md_thermo(const md_params* p, void* ws, size_t ws_bytes, double* out5, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!out5) return fail(MD_ERR_ARG, "output is NULL");
    const SimArgs a = make_args(p, L, ws);
    const double box = static_cast<double>(p->box);
    const double t_coef = p->n > 1 ? 2.0 / (3.0 * static_cast<double>(p->n) - 3.0) : 0.0;
    const double p_coef = 1.0 / (3.0 * box * box * box);
    MD_TRY_HIP(launch_forces(a, false, true, false, false, false, 0, stream), "energy pass");
    MD_TRY_HIP(launch_thermo_final(a, t_coef, p_coef, out5, stream), "thermo");
    return MD_OK;
}

md_status md_get_state(const md_params* p, const void* ws, size_t ws_bytes, float* pos4, float* vel4,
                       hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if ((pos4 && !aligned16(pos4)) || (vel4 && !aligned16(vel4)))
        return fail(MD_ERR_ARG, "particle arrays must be 16-byte aligned");
    if (!pos4 && !vel4) return MD_OK;
    const SimArgs a = make_args(p, L, const_cast<void*>(ws));
    MD_TRY_HIP(launch_gather_user(a, reinterpret_cast<float4*>(pos4), reinterpret_cast<float4*>(vel4), nullptr, stream),
               "gather");
    return MD_OK;
}

md_status md_neighbors(const md_params* p, const void* ws, size_t ws_bytes, int32_t* counts, int32_t* idx,
                       int32_t max_per_atom, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!counts || !idx) return fail(MD_ERR_ARG, "neighbour outputs are NULL");
    if (max_per_atom < 1) return fail(MD_ERR_ARG, "max_per_atom must be >= 1");
    const SimArgs a = make_args(p, L, const_cast<void*>(ws));
    MD_TRY_HIP(launch_neighbors(a, counts, idx, max_per_atom, 0, stream), "neighbors");
    return MD_OK;
}

md_status md_neighbors_lists(const md_params* p, void* ws, size_t ws_bytes, int32_t* counts, int32_t* idx,
                             int32_t max_per_atom, int32_t record, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!(p->flags & MD_FLAG_PAIR_LISTS))
        return fail(MD_ERR_ARG, "md_neighbors_lists needs a workspace laid out with MD_FLAG_PAIR_LISTS");
    if (!counts || !idx) return fail(MD_ERR_ARG, "neighbour outputs are NULL");
    if (max_per_atom < 1) return fail(MD_ERR_ARG, "max_per_atom must be >= 1");
    if (record != 0 && record != 1) return fail(MD_ERR_ARG, "record must be 0 or 1");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_neighbors(a, counts, idx, max_per_atom, record ? 1 : 2, stream), "neighbors");
    return MD_OK;
}

md_status md_cell_lists(const md_params* p, const void* ws, size_t ws_bytes, int32_t* cell_start, int32_t* order,
                        hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!cell_start && !order) return MD_OK;
    const SimArgs a = make_args(p, L, const_cast<void*>(ws));
    MD_TRY_HIP(launch_cell_lists(a, cell_start, order, stream), "cell lists");
    return MD_OK;
}

md_status md_adjoint_kick(const md_params* p, void* ws, size_t ws_bytes, const float* w4, float* lam_r4, double* theta,
                          float coef, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (p->shift_mode != 0) return fail(MD_ERR_ARG, "the adjoint needs shift_mode 0 (force shift)");
    if (!w4 || !lam_r4) return fail(MD_ERR_ARG, "adjoint vectors are NULL");
    if (!aligned16(w4) || !aligned16(lam_r4)) return fail(MD_ERR_ARG, "adjoint vectors must be 16-byte aligned");
    if (w4 == lam_r4) return fail(MD_ERR_ARG, "w and lam_r must not alias");
    if (!std::isfinite(coef)) return fail(MD_ERR_ARG, "coef must be finite");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_adjoint_kick(a, reinterpret_cast<const float4*>(w4), reinterpret_cast<float4*>(lam_r4), theta,
                                   coef, stream),
               "adjoint kick");
    return MD_OK;
}

md_status md_adjoint_drift(const md_params* p, const float* lam_r4, float* lam_v4, hipStream_t stream) {
    md_status s = validate(p);
    if (s != MD_OK) return s;
    if (!lam_r4 || !lam_v4) return fail(MD_ERR_ARG, "adjoint vectors are NULL");
    if (!aligned16(lam_r4) || !aligned16(lam_v4)) return fail(MD_ERR_ARG, "adjoint vectors must be 16-byte aligned");
    MD_TRY_HIP(launch_adjoint_drift(p->n, p->dt, reinterpret_cast<const float4*>(lam_r4),
                                    reinterpret_cast<float4*>(lam_v4), stream),
               "adjoint drift");
    return MD_OK;
}

md_status md_adjoint_segment(const md_params* p, void* ws, size_t ws_bytes, const float* ckpt_pos4,
                             const float* ckpt_vel4, int32_t first_step, int32_t nsteps, float* path4,
                             int32_t* path_start, float* lam_r4, float* lam_v4, double* theta, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if ((s = check_path_args(p, first_step, nsteps, path4, path_start, true)) != MD_OK) return s;
    if ((s = check_ckpt(ckpt_pos4, ckpt_vel4)) != MD_OK) return s;
    if ((s = check_adjoint_vecs(lam_r4, lam_v4)) != MD_OK) return s;
    const SimArgs a = make_args(p, L, ws);
    if ((s = recompute_impl(a, ckpt_pos4, ckpt_vel4, nsteps, path4, path_start, stream)) != MD_OK) return s;
    if ((s = sweep_impl(a, p, first_step, nsteps, path4, path_start, lam_r4, lam_v4, theta, stream)) != MD_OK) return s;
    // the workspace's own sorted arrays were not written: it holds no state now
    MD_TRY_HIP(launch_set_state(a, STATE_BUILDING, stream), "state reset");
    return MD_OK;
}

md_status md_adjoint_recompute(const md_params* p, void* ws, size_t ws_bytes, const float* ckpt_pos4,
                               const float* ckpt_vel4, int32_t nsteps, float* path4, int32_t* path_start,
                               hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if ((s = check_path_args(p, 0, nsteps, path4, path_start, true)) != MD_OK) return s;
    if ((s = check_ckpt(ckpt_pos4, ckpt_vel4)) != MD_OK) return s;
    const SimArgs a = make_args(p, L, ws);
    if ((s = recompute_impl(a, ckpt_pos4, ckpt_vel4, nsteps, path4, path_start, stream)) != MD_OK) return s;
    MD_TRY_HIP(launch_set_state(a, STATE_BUILDING, stream), "state reset");
    return MD_OK;
}

md_status md_adjoint_path(const md_params* p, void* ws, size_t ws_bytes, int32_t first_step, int32_t nsteps,
                          const float* path4, const int32_t* path_start, float* lam_r4, float* lam_v4,
                          double* theta, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if ((s = check_path_args(p, first_step, nsteps, path4, path_start, true)) != MD_OK) return s;
    if ((s = check_adjoint_vecs(lam_r4, lam_v4)) != MD_OK) return s;
    const SimArgs a = make_args(p, L, ws);
    return sweep_impl(a, p, first_step, nsteps, const_cast<float*>(path4), const_cast<int32_t*>(path_start), lam_r4,
                      lam_v4, theta, stream);
}

md_status md_step_path(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps, float* path4,
                       int32_t* path_start, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if ((s = check_path_args(p, 0, nsteps, path4, path_start, false)) != MD_OK) return s;
    const SimArgs a = make_args(p, L, ws);
    // state 0 is the workspace's own (cells built, forces computed): its
    // sorted positions and offsets are copied once; every later state is
    // sorted straight into its slice, as in the recompute
    MD_TRY_HIP(hipMemcpyAsync(path4, a.pos0, static_cast<size_t>(p->n) * sizeof(float4), hipMemcpyDeviceToDevice,
                              stream),
               "path copy");
    MD_TRY_HIP(hipMemcpyAsync(path_start, a.start, (static_cast<size_t>(L.ncells) + 1) * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, stream),
               "path copy");
    // md_step's sequence; the rebuild before step k + 1 writes state k into
    // slice k, the last one into the workspace, which ends as after md_step
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool last = k == nsteps;
        const SimArgs ak = last ? a : path_slice(a, path4, path_start, k);
        if (k == 1) MD_TRY_HIP(launch_integrate(a, stream), "integrate");
        if ((s = rebuild(ak, (k - 1) & 1, true, stream)) != MD_OK) return s;
        MD_TRY_HIP(launch_forces(ak, true, false, last, true, !last, k & 1, stream), "forces");
    }
    MD_TRY_HIP(launch_zero_blocks(a, (nsteps - 1) & 1, stream), "counter clear");
    return MD_OK;
}

md_status md_loss_grad(const md_params* p, void* ws, size_t ws_bytes, float k_coef, float w_coef, float* g_r4,
                       float* g_v4, double* theta, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (p->shift_mode != 0) return fail(MD_ERR_ARG, "the adjoint needs shift_mode 0 (force shift)");
    if (!g_r4 || !g_v4) return fail(MD_ERR_ARG, "gradient outputs are NULL");
    if (!aligned16(g_r4) || !aligned16(g_v4)) return fail(MD_ERR_ARG, "gradient outputs must be 16-byte aligned");
    if (!std::isfinite(k_coef) || !std::isfinite(w_coef)) return fail(MD_ERR_ARG, "coefficients must be finite");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_loss_grad(a, k_coef, w_coef, reinterpret_cast<float4*>(g_r4), reinterpret_cast<float4*>(g_v4),
                                theta, stream),
               "loss gradient");
    return MD_OK;
}

md_status md_loss(const md_params* p, void* ws, size_t ws_bytes, double* loss, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!loss) return fail(MD_ERR_ARG, "loss output is NULL");
    const SimArgs a = make_args(p, L, ws);
    double kc, wc;
    loss_coefficients(p, 1.0, kc, wc);
    MD_TRY_HIP(launch_forces(a, false, true, false, false, false, 0, stream), "energy pass");
    MD_TRY_HIP(launch_loss_final(a, kc, wc, loss, stream), "loss");
    return MD_OK;
}

md_status md_adjoint_seed(const md_params* p, void* ws, size_t ws_bytes, float scale, float* lam_r4, float* lam_v4,
                          double* theta, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (p->shift_mode != 0) return fail(MD_ERR_ARG, "the adjoint needs shift_mode 0 (force shift)");
    if (!lam_r4 || !lam_v4) return fail(MD_ERR_ARG, "adjoint vectors are NULL");
    if (!aligned16(lam_r4) || !aligned16(lam_v4)) return fail(MD_ERR_ARG, "adjoint vectors must be 16-byte aligned");
    if (lam_r4 == lam_v4) return fail(MD_ERR_ARG, "lam_r and lam_v must not alias");
    if (!std::isfinite(scale)) return fail(MD_ERR_ARG, "scale must be finite");
    const SimArgs a = make_args(p, L, ws);
    double kc, wc;
    loss_coefficients(p, scale, kc, wc);
    // lam = scale dL/d(r, v) at the final state, then the kick adjoint that
    // ends the last step (coefficient dt / 2m)
    MD_TRY_HIP(launch_loss_grad(a, static_cast<float>(kc), static_cast<float>(wc), reinterpret_cast<float4*>(lam_r4),
                                reinterpret_cast<float4*>(lam_v4), theta, stream),
               "loss gradient");
    MD_TRY_HIP(launch_adjoint_kick(a, reinterpret_cast<const float4*>(lam_v4), reinterpret_cast<float4*>(lam_r4), theta,
                                   a.hdt_m, stream),
               "adjoint kick");
    return MD_OK;
}

size_t md_batch_workspace_bytes(const md_params* p, const md_replica* reps, int32_t count) {
    BatchPlan B;
    if (batch_plan(p, reps, count, B) != MD_OK) return 0;
    return B.L.total;
}

md_status md_batch_build(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                         const float* pos4, const float* vel4, hipStream_t stream) {
    BatchPlan B;
    md_status s = batch_prepare(p, reps, count, ws, ws_bytes, B);
    if (s != MD_OK) return s;
    if (!pos4) return fail(MD_ERR_ARG, "positions are NULL");
    if (!aligned16(pos4) || (vel4 && !aligned16(vel4))) return fail(MD_ERR_ARG, "particle arrays must be 16-byte aligned");
    const BatchArgs ba = batch_args(p, B, ws);
    // the replica table lives in the workspace; wait for the copy so the host table can go
    MD_TRY_HIP(hipMemcpyAsync(const_cast<Replica*>(ba.reps), B.table.data(), sizeof(Replica) * B.table.size(),
                              hipMemcpyHostToDevice, stream),
               "replica table upload");
    MD_TRY_HIP(hipStreamSynchronize(stream), "replica table upload");
    MD_TRY_HIP(launch_build_init(ba.base, stream), "batch init");
    MD_TRY_HIP(launch_batch_setup(ba.base, ba.reps, ba.atom_rep, ba.cell_rep, ba.class_cells, B.count, stream),
               "batch setup");
    MD_TRY_HIP(launch_batch_load(ba.base, ba.reps, ba.atom_rep, reinterpret_cast<const float4*>(pos4),
                                 reinterpret_cast<const float4*>(vel4), stream),
               "batch load");
    if ((s = rebuild(ba.base, 0, false, stream)) != MD_OK) return s;
    MD_TRY_HIP(launch_zero_blocks(ba.base, 0, stream), "batch counter clear");
    return MD_OK;
}

md_status md_batch_forces(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                          float* force4, hipStream_t stream) {
    BatchPlan B;
    md_status s = batch_prepare(p, reps, count, ws, ws_bytes, B);
    if (s != MD_OK) return s;
    if (force4 && !aligned16(force4)) return fail(MD_ERR_ARG, "force array must be 16-byte aligned");
    const BatchArgs ba = batch_args(p, B, ws);
    MD_TRY_HIP(batch_forces(B, ba, false, false, true, false, 0, stream),
               "batch forces");
    if (force4) MD_TRY_HIP(launch_gather_user(ba.base, nullptr, nullptr, reinterpret_cast<float4*>(force4), stream), "gather");
    return MD_OK;
}

md_status md_batch_step(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                        int32_t nsteps, int32_t thermo_every, double* thermo, hipStream_t stream) {
    BatchPlan B;
    md_status s = batch_prepare(p, reps, count, ws, ws_bytes, B);
    if (s != MD_OK) return s;
    if (nsteps < 0) return fail(MD_ERR_ARG, "nsteps must be >= 0");
    if (thermo_every < 0) return fail(MD_ERR_ARG, "thermo_every must be >= 0");
    if (thermo_every > 0 && !thermo) return fail(MD_ERR_ARG, "thermo_every > 0 needs a thermo buffer");
    return batch_steps(B, batch_args(p, B, ws), nsteps, thermo_every, thermo, stream);
}

md_status md_batch_energy_virial(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                                 double* out, hipStream_t stream) {
    BatchPlan B;
    md_status s = batch_prepare(p, reps, count, ws, ws_bytes, B);
    if (s != MD_OK) return s;
    if (!out) return fail(MD_ERR_ARG, "output is NULL");
    const BatchArgs ba = batch_args(p, B, ws);
    MD_TRY_HIP(batch_forces(B, ba, false, true, false, false, 0, stream),
               "batch energy pass");
    MD_TRY_HIP(launch_batch_energy_final(ba.base, ba.reps, B.count, out, stream), "batch energy");
    return MD_OK;
}

md_status md_batch_get_state(const md_params* p, const md_replica* reps, int32_t count, const void* ws,
                             size_t ws_bytes, float* pos4, float* vel4, hipStream_t stream) {
    BatchPlan B;
    md_status s = batch_prepare(p, reps, count, ws, ws_bytes, B);
    if (s != MD_OK) return s;
    if ((pos4 && !aligned16(pos4)) || (vel4 && !aligned16(vel4)))
        return fail(MD_ERR_ARG, "particle arrays must be 16-byte aligned");
    if (!pos4 && !vel4) return MD_OK;
    const BatchArgs ba = batch_args(p, B, const_cast<void*>(ws));
    MD_TRY_HIP(launch_gather_user(ba.base, reinterpret_cast<float4*>(pos4), reinterpret_cast<float4*>(vel4), nullptr,
                                  stream),
               "gather");
    return MD_OK;
}

struct md_graph_s {
    hipGraphExec_t exec;
};

md_status md_batch_graph_create(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                                int32_t nsteps, int32_t thermo_every, double* thermo, hipStream_t stream,
                                md_graph* graph_out) {
    BatchPlan B;
    md_status s = batch_prepare(p, reps, count, ws, ws_bytes, B);
    if (s != MD_OK) return s;
    if (!graph_out) return fail(MD_ERR_ARG, "graph output is NULL");
    if (!stream) return fail(MD_ERR_ARG, "graph capture needs a non-null stream");
    if (nsteps < 1) return fail(MD_ERR_ARG, "nsteps must be >= 1");
    if (thermo_every < 0) return fail(MD_ERR_ARG, "thermo_every must be >= 0");
    if (thermo_every > 0 && !thermo) return fail(MD_ERR_ARG, "thermo_every > 0 needs a thermo buffer");
    const BatchArgs ba = batch_args(p, B, ws);
    MD_TRY_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture");
    s = batch_steps(B, ba, nsteps, thermo_every, thermo, stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &graph);
    if (s != MD_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return s != MD_OK ? s : hip_fail(e, "end capture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei, "graph instantiate");
    md_graph g = new (std::nothrow) md_graph_s{exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return fail(MD_ERR_ARG, "out of host memory for the graph handle");
    }
    *graph_out = g;
    return MD_OK;
}

md_status md_graph_launch(md_graph g, hipStream_t stream) {
    if (!g) return fail(MD_ERR_ARG, "graph is NULL");
    MD_TRY_HIP(hipGraphLaunch(g->exec, stream), "graph launch");
    return MD_OK;
}

md_status md_graph_destroy(md_graph g) {
    if (!g) return MD_OK;
    const hipError_t e = hipGraphExecDestroy(g->exec);
    delete g;
    if (e != hipSuccess) return hip_fail(e, "graph destroy");
    return MD_OK;
}

md_status md_check(void* ws, size_t ws_bytes, hipStream_t stream, int32_t* flags_out) {
    if (!ws) return fail(MD_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(MD_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < sizeof(int) * HDR_WORDS) return fail(MD_ERR_WORKSPACE, "workspace too small");
    int word = 0;
    int* hdr = static_cast<int*>(ws);
    MD_TRY_HIP(hipMemcpyAsync(&word, hdr + HDR_ERROR, sizeof(int), hipMemcpyDeviceToHost, stream), "read error word");
    MD_TRY_HIP(hipStreamSynchronize(stream), "synchronize");
    if (flags_out) *flags_out = word;
    if (word != 0) {
        static const int zero = 0;
        MD_TRY_HIP(hipMemcpyAsync(hdr + HDR_ERROR, &zero, sizeof(int), hipMemcpyHostToDevice, stream), "clear error word");
        MD_TRY_HIP(hipStreamSynchronize(stream), "synchronize");
        return fail(MD_ERR_DEVICE, "device error bits 0x%x", word);
    }
    return MD_OK;
}

const char* md_last_error(void) { return g_err; }

const char* md_status_name(md_status s) {
    switch (s) {
        case MD_OK: return "MD_OK";
        case MD_ERR_ARG: return "MD_ERR_ARG";
        case MD_ERR_BOX: return "MD_ERR_BOX";
        case MD_ERR_WORKSPACE: return "MD_ERR_WORKSPACE";
        case MD_ERR_HIP: return "MD_ERR_HIP";
        case MD_ERR_DEVICE: return "MD_ERR_DEVICE";
    }
    return "MD_UNKNOWN";
}

}  // extern "C"
