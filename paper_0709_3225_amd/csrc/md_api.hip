// C-ABI layer: host-side validation, workspace layout and launch sequencing.
// Every entry point validates on the host before touching the device and
// returns an md_status; nothing here throws across the C boundary.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

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
    if (p->shift_mode != 0 && p->shift_mode != 1) return fail(MD_ERR_ARG, "shift_mode must be 0 or 1");
    if (p->flags != 0) return fail(MD_ERR_ARG, "flags must be 0");
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
    L.cell = take(4 * n);
    L.rank = take(4 * n);
    L.key = take(4 * n);
    L.count = take(4 * static_cast<size_t>(L.ncells) + 16);
    L.start = take(4 * (static_cast<size_t>(L.ncells) + 1) + 16);
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

SimArgs make_args(const md_params* p, const Layout& L, void* ws) {
    char* b = static_cast<char*>(ws);
    SimArgs a{};
    a.hdr = reinterpret_cast<int*>(b + L.hdr);
    a.pos0 = reinterpret_cast<float4*>(b + L.pos0);
    a.vel0 = reinterpret_cast<float4*>(b + L.vel0);
    a.pos1 = reinterpret_cast<float4*>(b + L.pos1);
    a.vel1 = reinterpret_cast<float4*>(b + L.vel1);
    a.force = reinterpret_cast<float4*>(b + L.force);
    a.cell = reinterpret_cast<int*>(b + L.cell);
    a.rank = reinterpret_cast<int*>(b + L.rank);
    a.key = reinterpret_cast<int*>(b + L.key);
    a.count = reinterpret_cast<int*>(b + L.count);
    a.start = reinterpret_cast<int*>(b + L.start);
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
    a.fc = p->shift_mode == 0 ? static_cast<float>(flj_rc) : 0.f;
    a.uc = static_cast<float>(ulj_rc);
    // Screen bound: frame coordinates lie within [-s, 2s) per axis, so |x|^2 <= 12 s^2;
    // the FP32 dot-product form of r^2 errs by a few ulp of that. 2^-17 * 12 s^2 leaves a
    // wide margin, so the screen never drops a pair that the exact test accepts.
    a.screen2 = static_cast<float>(rc * rc + std::ldexp(12.0 * L.s * L.s, -17));
    // One LDS pass holds the mean 27-cell neighbourhood plus 30% and a wavefront.
    const double hood = 27.0 * static_cast<double>(p->n) / L.ncells;
    int cap = static_cast<int>(std::ceil((1.3 * hood + 64.0) / 64.0)) * 64;
    a.tile_cap = std::min(2048, std::max(128, cap));
    a.dt = p->dt;
    a.hdt_m = static_cast<float>(0.5 * p->dt / p->mass);
    a.half_m = static_cast<float>(0.5 * p->mass);
    return a;
}

#define MD_TRY_HIP(expr, where)                  \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

md_status rebuild_from_staging(const SimArgs& a, bool from_step, hipStream_t st) {
    MD_TRY_HIP(launch_scan(a, st), "scan");
    MD_TRY_HIP(launch_scatter(a, st), "scatter");
    MD_TRY_HIP(launch_cell_order(a, from_step, st), "cell order");
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

md_status md_build_cells(const md_params* p, void* ws, size_t ws_bytes, const float* pos4, const float* vel4,
                         hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!pos4) return fail(MD_ERR_ARG, "positions are NULL");
    if (!aligned16(pos4) || (vel4 && !aligned16(vel4))) return fail(MD_ERR_ARG, "particle arrays must be 16-byte aligned");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_build_init(a, stream), "build init");
    MD_TRY_HIP(launch_load(a, reinterpret_cast<const float4*>(pos4), reinterpret_cast<const float4*>(vel4), stream),
               "load");
    return rebuild_from_staging(a, false, stream);
}

md_status md_forces(const md_params* p, void* ws, size_t ws_bytes, float* force4, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (force4 && !aligned16(force4)) return fail(MD_ERR_ARG, "force array must be 16-byte aligned");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_forces(a, false, false, true, false, stream), "forces");
    if (force4) MD_TRY_HIP(launch_gather_user(a, nullptr, nullptr, reinterpret_cast<float4*>(force4), stream), "gather");
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
    const SimArgs a = make_args(p, L, ws);
    for (int32_t k = 1; k <= nsteps; ++k) {
        const bool energy = thermo && thermo_every > 0 && (k % thermo_every) == 0;
        MD_TRY_HIP(launch_integrate(a, stream), "integrate");
        if ((s = rebuild_from_staging(a, true, stream)) != MD_OK) return s;
        MD_TRY_HIP(launch_forces(a, true, energy, true, true, stream), "forces");
        if (energy)
            MD_TRY_HIP(launch_energy_final(a, thermo + 3 * static_cast<size_t>(k / thermo_every - 1), stream),
                       "energy");
    }
    return MD_OK;
}

md_status md_energy_virial(const md_params* p, void* ws, size_t ws_bytes, double* out3, hipStream_t stream) {
    Layout L{};
    md_status s = make_layout(p, L);
    if (s != MD_OK) return s;
    if ((s = check_ws(L, ws, ws_bytes)) != MD_OK) return s;
    if (!out3) return fail(MD_ERR_ARG, "output is NULL");
    const SimArgs a = make_args(p, L, ws);
    MD_TRY_HIP(launch_forces(a, false, true, false, false, stream), "energy pass");
    MD_TRY_HIP(launch_energy_final(a, out3, stream), "energy");
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
    MD_TRY_HIP(launch_neighbors(a, counts, idx, max_per_atom, stream), "neighbors");
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
