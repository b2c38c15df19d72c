// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mdlj {

// Header words at the start of the workspace.
// HDR_N and HDR_NC record the particle count and cell grid the workspace was
// built for; kernels refuse a workspace whose record differs from their
// arguments (its array offsets would not match).
// HDR_OVF + p counts the overflow-list entries of a build binned with parity
// p (p = 0, 1; the same alternation as the block histograms); HDR_OVFA + p
// hands out index ranges of that list's per-cell index to the cell order.
enum : int { HDR_ERROR = 0, HDR_STATE = 1, HDR_N = 2, HDR_NC = 3, HDR_OVF = 4, HDR_OVFA = 6, HDR_WORDS = 64 };

// Workspace states. Distinctive values so that an uninitialised workspace is
// never mistaken for a built one.
enum : int { STATE_BUILDING = 0x4D440000, STATE_CELLS = 0x4D440001, STATE_FORCES = 0x4D440002 };

// The cell order runs one workgroup per block of 2^kBlockShift consecutive
// cells; the block scan gives each block its first atom, or on grids of up to
// kDirectBlocks blocks each workgroup sums the block counts before its own.
constexpr int kBlockShift = 4;
constexpr int kDirectBlocks = 2048;
// Pair lists: a cell's lanes keep the accept words of its screen (one span
// covers 128 candidates of a lane; a liquid-density neighbourhood of about
// 400 atoms needs one span with four slices, two with two or three).
constexpr int kListSpans = 4;  // kept accept-word spans (16 bytes each) per lane of a cell
constexpr int kSlotBits = 27;  // neighbour-list entry: sorted slot, then the image shift code
constexpr uint32_t kSlotMask = (1u << kSlotBits) - 1u;

// Device error bits (same values as the public MD_DEV_* macros).
enum : int { DEV_NONFINITE = 1, DEV_ORDER = 2, DEV_NB_OVERFLOW = 4, DEV_SKIN = 8 };

// Everything a kernel needs, passed by value.
struct SimArgs {
    int* hdr;
    float4* pos0;    // cell-sorted positions, w = user index bits
    float4* vel0;    // cell-sorted velocities
    float4* pos1;    // overflow storage of the cell build (entry j of the list), and
    float4* vel1;    // scratch for the adjoint between builds
    float4* force;   // cell-sorted forces
    // Steps between rebuilds (md_step_every): the drift of the force epilogue
    // writes the next positions and velocities here, in the same sorted slots;
    // the host swaps this pair with pos0/vel0 from step to step.
    float4* pos2;
    float4* vel2;
    float skin_half;  // an atom may leave its cell's box by this much before a rebuild is due
    // Pair lists (md_step_list): per cell and lane, the accept words of the
    // screen against the list radius (the cell side), kListSpans spans of
    // four words at most (plist_n: the count; more marks a cell that screens
    // instead); posref: positions when the words were kept.
    uint32_t* plist;
    int* plist_n;
    float4* posref;
    // Per-atom neighbour lists (md_step_nlist): atom slot i's partners within
    // the list radius are its first ncount[i] entries; entry k of atom i is
    // nlist[4 (n (k / 4) + i) + k % 4] (groups of four entries, atoms
    // consecutive within a group), each the partner's sorted slot (low
    // kSlotBits bits) and its periodic image (shift code (sx + 1) +
    // 3 (sy + 1) + 9 (sz + 1) in the high bits; the partner is taken at
    // x_j + s L).
    uint32_t* nlist;
    int* ncount;
    int nlist_cap;
    float list_screen2;  // screen bound when the words are kept (cell side^2 plus the screen margin)
    float disp_half;     // largest displacement since recording: (side - r_c) / 2
    // Cell build: per-cell histogram, zero between builds; a binned atom's
    // position and velocity go to its cell's bucket of cap entries, or to the
    // overflow list (pos1, vel1 and the cell) past the capacity.
    int* counts;     // ncells (+ 16 zero padding)
    int* bstart;     // nblocks = ceil(ncells / 16): atoms before each block of 16 cells
    // Builds alternate between two parities (par: the one being filled or
    // read; the other's counters are zero): the overflow count, and on grids
    // of at most kDirectBlocks blocks (direct != 0) a per-block atom count,
    // two histograms nbstride entries apart, which lets the cell order sum the
    // blocks before its own instead of reading bstart.
    int* bcounts;
    int nbstride, par, direct;
    float4* bpos;    // ncells x cap bucket entries (w = user index bits)
    float4* bvel;
    int* ovf_cell;   // cell of overflow entry j, one entry per atom at most
    int* ovf_rank;   // its rank among its cell's overflow entries (histogram rank - cap)
    int* ovf_idx;    // the cell order's per-cell index of the overflow entries
    int* start;      // per-cell CSR offsets, ncells + 1 entries
    double* epart;   // per-block energy partials, 3 doubles per force block
    int nblocks, cap, natoms;  // natoms: all atoms of the workspace

    int n;
    int nc;          // cells per dimension
    int ncells;      // nc^3
    int cbase;       // first cell of this system in the cell arrays (0 unless batched)
    float box;
    float s;         // cell side box / nc
    float inv_s;     // nc / box

    float rc2;       // r_c^2 (FP32)
    float rc;
    float sig2;      // sigma^2
    float eps24;     // 24 epsilon
    float eps4;      // 4 epsilon
    float c12, c6;   // 48 eps sigma^12, 24 eps sigma^6: f_LJ(r) / r = r^-8 (c12 r^-6 - c6)
    float e12, e6;   // 4 eps sigma^12, 4 eps sigma^6: u_LJ(r) = r^-6 (e12 r^-6 - e6)
    float fc;        // f_LJ(r_c) for the force shift, 0 for energy shift
    float uc;        // u_LJ(r_c)
    float screen2;   // conservative bound on r^2 for the dot-product screen
    int tile_cap;    // staged atoms per LDS pass of the force kernel
    int waves;       // wavefronts per force workgroup (1, 2 or 4), sharing one staged tile

    float dt;
    float hdt_m;     // dt / (2 m)
    float half_m;    // m / 2
};

// One replica of a batch: its atoms occupy [abase, abase + n) and its cells
// [cbase, cbase + ncells) of the batch's arrays; geometry as in SimArgs.
struct Replica {
    int n, abase, nc, ncells, cbase, tile_cap;
    float box, s, inv_s, screen2;
    int lbase;  // first entry of the replica's cells in the tile-class cell list
};

// Workspace layout (byte offsets, each 256-byte aligned).
struct Layout {
    int n, nc, ncells, nforce_blocks;
    float s, inv_s;
    int nblocks, cap;
    int nbstride;
    int nlist_cap;
    size_t hdr, pos0, vel0, pos1, vel1, force, pos2, vel2, posref, plist, plist_n, nlist, ncount, counts, bstart, bcounts,
        bpos, bvel,
        ovf_cell, ovf_rank, ovf_idx, start, epart, total;
};

// Kernel launchers (each returns hipGetLastError() after its launch).
hipError_t launch_build_init(const SimArgs& a, hipStream_t st);
hipError_t launch_load(const SimArgs& a, const float4* pos_in, const float4* vel_in, hipStream_t st);
// par: the block histogram a cell order reads (ignored unless a.direct); the
// binning launches (load, drift) fill histogram 0, the force pass's drift the
// one given to launch_forces.
hipError_t launch_block_scan(const SimArgs& a, bool from_step, hipStream_t st);
hipError_t launch_cell_order(const SimArgs& a, int par, bool from_step, hipStream_t st);
hipError_t launch_zero_blocks(const SimArgs& a, int par, hipStream_t st);
hipError_t launch_integrate(const SimArgs& a, hipStream_t st);
hipError_t launch_forces(const SimArgs& a, bool kick, bool energy, bool write_force, bool from_step, bool drift,
                         int par, hipStream_t st);
// A step between rebuilds: forces, kick, next drift into pos2/vel2 (md_step_every).
hipError_t launch_forces_skin(const SimArgs& a, bool energy, hipStream_t st);
// Pair-list steps (md_step_list): record (right after a rebuild) or use the
// lists; the drift bins for a rebuild (bin) or goes to pos2/vel2.
// md_step_nlist: the force pass right after a rebuild, writing the per-atom
// neighbour lists (one wavefront per cell, as the other cell passes), and the
// pass that walks them (one lane per atom); BIN as for launch_forces_list.
hipError_t launch_forces_record(const SimArgs& a, bool energy, bool bin, int par, hipStream_t st);
hipError_t launch_nlist_forces(const SimArgs& a, bool bin, int par, hipStream_t st);
hipError_t launch_forces_list(const SimArgs& a, bool energy, bool record, bool bin, int par, hipStream_t st);
hipError_t launch_energy_final(const SimArgs& a, double* out3, hipStream_t st);
// U, K, W as launch_energy_final, then out5[3] = t_coef K, out5[4] = p_coef (2 K + W).
hipError_t launch_thermo_final(const SimArgs& a, double t_coef, double p_coef, double* out5, hipStream_t st);
// out[0] = kcoef K + wcoef W from the partials of an energy pass.
hipError_t launch_loss_final(const SimArgs& a, double kcoef, double wcoef, double* out, hipStream_t st);
hipError_t launch_gather_user(const SimArgs& a, float4* pos_out, float4* vel_out, float4* force_out,
                              hipStream_t st);
// Neighbour export through the force kernel (list: 0 screen against r_c,
// 1 screen against the list radius and keep the words, 2 walk the kept words).
hipError_t launch_neighbors(const SimArgs& a, int* counts, int* idx, int max_per_atom, int list,
                            hipStream_t st);
hipError_t launch_cell_lists(const SimArgs& a, int* cell_start, int* order, hipStream_t st);
hipError_t launch_adjoint_kick(const SimArgs& a, const float4* w_user, float4* lam_r, double* theta, float coef,
                               hipStream_t st);
hipError_t launch_loss_grad(const SimArgs& a, float kcoef, float wcoef, float4* g_r, float4* g_v, double* theta,
                            hipStream_t st);
hipError_t launch_adjoint_drift(int n, float dt, const float4* lam_r, float4* lam_v, hipStream_t st);
// launch_adjoint_drift followed by the gather and pair pass of
// launch_adjoint_kick with w = lam_v, the drift folded into the gather (same
// arithmetic, one launch fewer). The parameter terms times coef go to the
// per-cell sums in epart (added to them with accumulate, else replacing
// them); launch_theta_final adds coef times their fixed-order total to theta.
hipError_t launch_adjoint_drift_kick(const SimArgs& a, float dt, float4* lam_r, float4* lam_v, float coef,
                                     bool accumulate, hipStream_t st);
hipError_t launch_theta_final(const SimArgs& a, double* theta, double coef, hipStream_t st);
// Mark the workspace as holding no built state (the header's state word only).
hipError_t launch_set_state(const SimArgs& a, int state, hipStream_t st);

// Batched replicas: base = the batch's arrays and shared constants (n and
// ncells are the batch totals), reps = device replica table.
// class_cells (nullable) receives the global cell indices grouped by tile
// class: replica b's cells at [lbase_b, lbase_b + ncells_b).
hipError_t launch_batch_setup(const SimArgs& base, const Replica* reps, int* atom_rep, int* cell_rep,
                              int* class_cells, int count, hipStream_t st);
hipError_t launch_batch_load(const SimArgs& base, const Replica* reps, const int* atom_rep, const float4* pos_in,
                             const float4* vel_in, hipStream_t st);
hipError_t launch_batch_integrate(const SimArgs& base, const Replica* reps, const int* atom_rep, hipStream_t st);
// One launch over the ncl global cells listed at cells (a tile class), with
// LDS for tile_cap staged atoms (at least every listed replica's tile_cap)
// and waves wavefronts per cell.
hipError_t launch_batch_forces(const SimArgs& base, const Replica* reps, const int* cell_rep, const int* cells,
                               int ncl, int tile_cap, int waves, bool kick, bool energy, bool write_force, bool drift,
                               int par, hipStream_t st);
hipError_t launch_batch_energy_final(const SimArgs& base, const Replica* reps, int count, double* out, hipStream_t st);

}  // namespace mdlj
