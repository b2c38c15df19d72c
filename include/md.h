/*
 * mdlj: short-range Lennard-Jones molecular dynamics over a cell list on one
 * AMD Instinct MI355X (gfx950) GPU.
 *
 * The method (van Meel, Arnold, Frenkel, Portegies Zwart, Belleman,
 * "Harvesting graphics power for MD simulations"):
 *   - pair force: LJ force truncated at r_c = 2.5 sigma and shifted so that it
 *     vanishes at the cutoff (section 2, equations for f_LJ and f(r));
 *   - force on particle i: sum over the other particles of f(r_ij) along the
 *     unit vector from j to i (section 2, force-sum equation);
 *   - partners found through cells whose side is at least the interaction
 *     range, so they lie in the home cell or its 26 neighbours, with
 *     n_x = int(L / r_c) cells per dimension (section 3 and section 3.2);
 *   - cell lists kept up to date as particles move (section 3.1);
 *   - velocity-Verlet time integration (section 2).
 *
 * Conventions for every entry point:
 *   - All functions are C ABI and never throw; all return an md_status
 *     except the queries md_workspace_bytes and md_tile_capacity (0 for
 *     invalid parameters), md_last_error and md_status_name.
 *   - Pointers named *_dev, ws and every particle array are DEVICE pointers
 *     owned by the caller; the library never allocates or frees memory.
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream);
 *     only md_check synchronises.
 *   - Particle arrays are float4 [n] (16-byte aligned); the w component of
 *     inputs is ignored. "User order" means the order of md_build_cells' input.
 *   - Argument and box validation happens on the host before any HIP call;
 *     a non-OK return enqueues nothing. md_last_error() then describes it.
 *   - Problems only the device can see (non-finite coordinates or forces,
 *     calls out of order) set bits in a device error word inside the
 *     workspace; md_check reads and clears it.
 *   - Calls that share one workspace must be ordered on one stream.
 */
#ifndef MDLJ_MD_H
#define MDLJ_MD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum md_status {
    MD_OK = 0,
    MD_ERR_ARG = 1,       /* invalid argument (null, non-finite, out of range) */
    MD_ERR_BOX = 2,       /* box shorter than two cutoffs: L < 2 r_c */
    MD_ERR_WORKSPACE = 3, /* workspace null, misaligned (256 B) or too small */
    MD_ERR_HIP = 5,       /* a HIP launch or runtime call failed */
    MD_ERR_DEVICE = 6     /* md_check found device error bits (see below) */
} md_status;

/* Device error bits reported through md_check's flags_out. */
#define MD_DEV_NONFINITE 1 /* a coordinate, velocity or force was not finite */
#define MD_DEV_ORDER 2     /* md_forces before md_build_cells, or md_step
                              before md_forces: the call did nothing */
#define MD_DEV_NB_OVERFLOW 4 /* md_neighbors: a row exceeded max_per_atom;
                              md_step_nlist: an atom had more partners
                              within the list radius than its list holds */
#define MD_DEV_SKIN 8      /* md_step_every: between rebuilds an atom left its
                              cell by more than half the skin; that run may
                              have missed pairs near r_c */

/* Physical and numerical parameters, reduced LJ units. */
typedef struct md_params {
    int32_t n;             /* particle count, 1 <= n <= 2^27 */
    float box;             /* cubic periodic box side L; this FP32 value is
                              authoritative for images and the cell grid */
    float epsilon;         /* LJ well depth, > 0 */
    float sigma;           /* LJ length, > 0 */
    float mass;            /* particle mass, > 0 */
    float rc_over_sigma;   /* cutoff r_c / sigma; 0 selects 2.5 (section 2) */
    float dt;              /* time step, finite, >= 0 */
    float cell_min;        /* minimum cell side; 0 selects r_c */
    int32_t shift_mode;    /* 0: force shifted to zero at r_c (section 2);
                              1: plain truncated force, energy shifted */
    int32_t flags;         /* MD_FLAG_* bits; 0 for a plain workspace */
    int32_t waves_per_cell; /* wavefronts per home cell in the force pass:
                              1, 2 or 4, sharing one staged neighbourhood and
                              splitting its candidates (0 selects 1). More
                              than one pays only on grids with too few cells
                              to fill the GPU. The pairs are the same for
                              every choice; only the order of the FP32 force
                              sums differs (bitwise reproducible for a fixed
                              choice). The pair-list and neighbour-export
                              passes always take one. */
    float list_radius;     /* md_step_list / md_step_nlist: radius r_V of the
                              pair and neighbour lists (section 3: r_c plus a
                              skin), r_c < r_V <= cell side; 0 selects the cell
                              side. The lists stay valid while no atom has
                              moved by more than (r_V - r_c) / 2. */
    int32_t tile_cap;      /* atoms staged per LDS pass of the force and pair
                              passes: 0 selects 1.1 x the mean 27-cell
                              neighbourhood + 32, rounded up to a multiple of
                              64 within [128, 2048]; else a multiple of 64 in
                              [128, 2048]. A neighbourhood larger than the tile
                              takes several passes; a smaller tile leaves LDS
                              for more wavefronts per CU. Results do not depend
                              on it except through the order of passes (bitwise
                              reproducible for a fixed value). The batch calls
                              ignore it (each replica takes the formula). */
} md_params;

/* md_params.flags: lay the workspace out with md_step_list's pair-list
 * arrays (about 4.3 KB per cell and 16 B per atom more); md_step_list
 * refuses a workspace without them. */
#define MD_FLAG_PAIR_LISTS 1
/* md_params.flags: lay the workspace out with md_step_nlist's per-atom
 * neighbour lists (about 4 B x the list capacity + 20 B per atom; the
 * capacity is 1.5 x the mean number of atoms within the cell side of an atom
 * plus 32, rounded up to a multiple of 32); md_step_nlist refuses a
 * workspace without them. */
#define MD_FLAG_ATOM_LISTS 2

/*
 * Bytes of device workspace for these parameters (0 if they are invalid).
 * Host only; needs no device. The workspace holds the cell-sorted state
 * (positions, velocities, forces), the cell lists, scratch and a small
 * header; its contents are private.
 */
size_t md_workspace_bytes(const md_params* p);

/*
 * Cell grid the library uses (host only). Cells per dimension is
 * n_c = int(L / max(r_c, cell_min)) as in section 3.2, lowered by one when
 * the resulting side L/n_c exceeds the minimum by less than 2^-18 L (so that
 * FP32 rounding of a cell index can never hide a partner); side = L / n_c.
 * Returns MD_ERR_BOX if L < 2 r_c.
 */
md_status md_cell_grid(const md_params* p, int32_t* cells_per_dim, float* cell_side);

/* The LDS tile (atoms per pass) the force pass takes for these parameters:
 * p->tile_cap, or the formula's value when it is 0. Returns 0 for invalid
 * parameters (md_last_error says why). */
int32_t md_tile_capacity(const md_params* p);

/*
 * Load a state and build the cell list (section 3: cells of side >= r_c;
 * section 3.1: membership rebuilt from current positions).
 *   pos4_dev: float4 [n] positions; wrapped into [0, L) on load.
 *   vel4_dev: float4 [n] velocities, or NULL for zero velocities.
 * Steps on the device: wrap + cell index + atomic histogram, prefix scan of
 * the histogram into cell offsets, scatter into cell-sorted order, and a
 * stable order inside every cell by user index (so the layout, and every
 * later floating-point sum, is independent of atomic timing).
 * (Re)initialises the workspace and clears its device error bits.
 * Forces are not computed: call md_forces before md_step.
 */
md_status md_build_cells(const md_params* p, void* ws, size_t ws_bytes, const float* pos4_dev,
                         const float* vel4_dev, hipStream_t stream);

/*
 * Forces on the current workspace state (section 2 force sum with the
 * truncated, shifted LJ force; partners from the 27 cells around each home
 * cell, minimum image). Stores them inside the workspace, which makes
 * md_step valid, and, if force4_dev is not NULL, writes float4 [n] forces in
 * user order (w = 0).
 */
md_status md_forces(const md_params* p, void* ws, size_t ws_bytes, float* force4_dev,
                    hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): md_build_cells on
 * pos4_dev (zero velocities) followed by md_forces with output force4_dev,
 * in a workspace the library keeps in a static device array of 16 MiB per
 * GPU (held until the process ends) instead of a caller's. It allocates
 * nothing. Parameters whose workspace (md_workspace_bytes) exceeds 16 MiB
 * (about 60,000 atoms at liquid density) are refused with MD_ERR_WORKSPACE
 * before any device call. The forces are those of md_forces on the same
 * positions (same kernels, same layout). Calls on one GPU share its array,
 * which keeps the last call's contents (every call rebuilds it from scratch):
 * calls that overlap on one GPU, on any streams, race. Device-side error
 * bits of the workspace are not reported (non-finite positions give
 * non-finite forces).
 */
md_status md_forces_noalloc(const md_params* p, const float* pos4_dev, float* force4_dev, hipStream_t stream);

/*
 * Advance nsteps velocity-Verlet steps (section 2). Each step: half kick
 * with the stored forces, drift, wrap into [0, L), cell-list rebuild
 * (histogram, scan, scatter, in-cell order), new forces, half kick.
 * Velocities are synchronous with positions after every call.
 * thermo_every > 0 with thermo_dev != NULL records (U, K, W) as doubles
 * after every thermo_every-th step: row r (0-based) holds step
 * (r + 1) * thermo_every, so thermo_dev needs 3 * (nsteps / thermo_every)
 * doubles. Needs md_forces since the last md_build_cells; otherwise sets
 * MD_DEV_ORDER and leaves the state unchanged.
 */
md_status md_step(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps,
                  int32_t thermo_every, double* thermo_dev, hipStream_t stream);

/*
 * md_step with the cell lists rebuilt only every rebuild_every steps
 * (section 3.1: cells larger than r_c by a skin, updated every few steps;
 * the Verlet displacement rule of section 3 bounds how far an atom may move
 * before the update). The skin is the grid's own margin, cell side - r_c:
 * choose it with md_params.cell_min = r_c + skin. Cells are rebuilt before
 * the forces of steps 1, 1 + e, 1 + 2e, ... (e = rebuild_every) and of the
 * last step; in between, positions are not wrapped and each atom keeps its
 * cell. If an atom leaves its cell's box by more than skin / 2 the device
 * sets MD_DEV_SKIN (the run may then have missed pairs; use a larger skin or
 * a smaller rebuild_every). rebuild_every = 1 is md_step exactly (bitwise).
 * On return the state is rebuilt and wrapped as after md_step; thermo_every
 * and thermo_dev as for md_step. rebuild_every < 1 gives MD_ERR_ARG.
 */
md_status md_step_every(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps,
                        int32_t rebuild_every, int32_t thermo_every, double* thermo_dev,
                        hipStream_t stream);

/*
 * md_step_every with pair lists (section 3: a Verlet list of partners within
 * a radius larger than r_c, rebuilt when a particle has moved more than half
 * the difference). Right after each cell rebuild the force pass screens the
 * 27-cell neighbourhood against the cell side instead of r_c and keeps, for
 * every lane of every home cell, its accept words (a bitmask over the staged
 * candidates); until the next rebuild the force pass walks the kept words
 * instead of screening. They hold the same candidates in the same order as
 * the screen plus some beyond r_c that add exact zeros, so the trajectory is
 * bitwise that of md_step_every with the same arguments and one wavefront
 * per cell (these passes always take one). MD_DEV_SKIN is set
 * if an atom moves more than (cell side - r_c) / 2 from where it was when the
 * words were kept. Cells that need more than one LDS pass, or more than four
 * 128-candidate spans per lane, screen as usual. Arguments and return values
 * as for md_step_every; the workspace must have been sized with
 * MD_FLAG_PAIR_LISTS in p->flags (MD_ERR_ARG otherwise).
 */
md_status md_step_list(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps,
                       int32_t rebuild_every, int32_t thermo_every, double* thermo_dev,
                       hipStream_t stream);

/*
 * md_step_every with per-atom Verlet neighbour lists (section 3: partners
 * within a radius larger than r_c, valid until a particle has moved by more
 * than half the difference). The force pass right after each cell rebuild
 * screens the 27-cell neighbourhood against the cell side and writes, for
 * every atom, the sorted slot and periodic image of every partner it finds;
 * until the next rebuild, one lane per atom walks its own list: no cell
 * staging and no screen. Thermo steps between rebuilds screen the cells
 * instead, and the last step of a call is an ordinary md_step force pass. An
 * atom with more partners than the list holds sets MD_DEV_NB_OVERFLOW (the
 * ones past the capacity are missed until the next rebuild); MD_DEV_SKIN is
 * set if an atom moves more than (cell side - r_c) / 2 from where it was when
 * the lists were written. The forces are those of md_step_every summed in
 * another order, so trajectories agree to FP32 rounding, not bitwise.
 * Arguments and return values as for md_step_every; the workspace must have
 * been sized with MD_FLAG_ATOM_LISTS in p->flags (MD_ERR_ARG otherwise).
 */
md_status md_step_nlist(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps,
                        int32_t rebuild_every, int32_t thermo_every, double* thermo_dev,
                        hipStream_t stream);

/*
 * Potential energy U, kinetic energy K = m/2 sum v^2 and virial
 * W = sum over pairs r phi(r) (positive = repulsive) of the current state,
 * written as out3_dev[0..2] (device doubles). Pair and per-atom terms are
 * FP32; all sums are FP64 in a fixed order, so the result is reproducible.
 * The paper prints no energy; U uses the energy that matches the shifted
 * force: u(r) = u_LJ(r) - u_LJ(r_c) + (r - r_c) f_LJ(r_c) (shift_mode 0), or
 * u_LJ(r) - u_LJ(r_c) (shift_mode 1).
 */
md_status md_energy_virial(const md_params* p, void* ws, size_t ws_bytes, double* out3_dev,
                           hipStream_t stream);

/*
 * md_energy_virial plus the temperature and the pressure of the state:
 * out5_dev[0..2] = U, K, W as there, out5_dev[3] = T = 2 K / (3 N - 3)
 * (k_B = 1, momentum conserved; 0 for N = 1) and out5_dev[4] =
 * P = (2 K + W) / (3 V), V = L^3 (the virial pressure). Device doubles, FP64
 * from the same fixed-order sums.
 */
md_status md_thermo(const md_params* p, void* ws, size_t ws_bytes, double* out5_dev, hipStream_t stream);

/* Copy the current positions (wrapped) and velocities out in user order;
 * either pointer may be NULL. float4 [n], w = 0. */
md_status md_get_state(const md_params* p, const void* ws, size_t ws_bytes, float* pos4_dev,
                       float* vel4_dev, hipStream_t stream);

/*
 * Test export of the neighbour sets the force kernel uses: for every atom i
 * (user order) the user indices j != i with r_ij^2 < r_c^2 (FP32 test on the
 * minimum-image displacement). counts_dev: int32 [n]. idx_dev: int32
 * [n * max_per_atom], row i at i * max_per_atom, order within a row
 * unspecified. A row longer than max_per_atom is truncated and sets
 * MD_DEV_NB_OVERFLOW (its count is still the full count).
 */
md_status md_neighbors(const md_params* p, const void* ws, size_t ws_bytes, int32_t* counts_dev,
                       int32_t* idx_dev, int32_t max_per_atom, hipStream_t stream);

/*
 * The same export through md_step_list's pair-list path (section 3: a list of
 * partners within a radius beyond r_c, here the cell side). record = 1:
 * screen the 27-cell neighbourhood against the list radius and keep every
 * lane's accept words, as the force pass right after a rebuild of
 * md_step_list does (this replaces the words md_step_list kept); record = 0:
 * walk the words kept last instead of screening, as its passes between
 * rebuilds do. Both export the pairs with r_ij^2 < r_c^2 that the walk
 * accepts, so for the current positions both must equal md_neighbors. Needs
 * a workspace laid out with MD_FLAG_PAIR_LISTS (MD_ERR_ARG otherwise);
 * record = 0 is meaningful only while the kept words belong to the current
 * cell lists (no rebuild since they were kept). Outputs and errors as for
 * md_neighbors.
 */
md_status md_neighbors_lists(const md_params* p, void* ws, size_t ws_bytes, int32_t* counts_dev,
                             int32_t* idx_dev, int32_t max_per_atom, int32_t record, hipStream_t stream);

/*
 * Test export of the cell list: cell_start_dev int32 [n_c^3 + 1] (CSR offsets
 * of every cell into the sorted order) and order_dev int32 [n] (user index of
 * the atom at each sorted slot). Either pointer may be NULL.
 */
md_status md_cell_lists(const md_params* p, const void* ws, size_t ws_bytes,
                        int32_t* cell_start_dev, int32_t* order_dev, hipStream_t stream);

/*
 * ---- Adjoint (differentiation through velocity Verlet) ----
 * These entry points build the discrete adjoint of md_step: with
 * h = dt / (2 m), one Verlet step is v' = v + h F(r), r' = r + dt v',
 * v'' = v' + h F(r'), so its transpose is a kick adjoint at r' (lam_r += h J
 * lam_v), a drift adjoint (lam_v += dt lam_r) and a kick adjoint at r. J is
 * the Jacobian of the force sum (section 2, force-sum equation with the
 * truncated, force-shifted f(r)); it is symmetric. Force-shift mode only
 * (shift_mode 0): the energy-shift variant has a force jump at r_c and no
 * derivative there (MD_ERR_ARG). Vectors are float4 [n] in user order.
 */

/*
 * Kick adjoint at the current workspace positions (md_build_cells first):
 *   lam_r4_dev += coef * J w,
 *   theta_dev[0] += coef * sum_i w_i . dF_i/d(epsilon),
 *   theta_dev[1] += coef * sum_i w_i . dF_i/d(sigma)   (r_c = rc_over_sigma * sigma
 *   moves with sigma). theta_dev: 2 device doubles, nullable; FP64 sums in a
 * fixed order. w4_dev and lam_r4_dev must not alias.
 */
md_status md_adjoint_kick(const md_params* p, void* ws, size_t ws_bytes, const float* w4_dev,
                          float* lam_r4_dev, double* theta_dev, float coef, hipStream_t stream);

/* Drift adjoint: lam_v4_dev += dt * lam_r4_dev (n float4 each; no workspace). */
md_status md_adjoint_drift(const md_params* p, const float* lam_r4_dev, float* lam_v4_dev,
                           hipStream_t stream);

/*
 * One checkpoint segment of the backward pass, composed of the calls above
 * with no host round trips: from the checkpoint (ckpt_pos4_dev,
 * ckpt_vel4_dev: the state after step first_step) recompute the segment's
 * nsteps states, keeping each one's cell-sorted positions in path4_dev
 * (nsteps * n float4) and its cell offsets in path_start_dev
 * (nsteps * (n_c^3 + 1) int32), both caller-owned scratch; then from the last
 * step back to the first apply the drift adjoint and the kick adjoint on the
 * kept cell list, with coefficient 2h, or h for step 0 (h = dt / 2m).
 * lam_r4_dev, lam_v4_dev and theta_dev accumulate as for md_adjoint_drift and
 * md_adjoint_kick (theta's terms are summed per cell over the segment, then
 * over cells in a fixed order). The workspace is overwritten and left without a built
 * state: calls that read one raise MD_DEV_ORDER until md_build_cells.
 */
md_status md_adjoint_segment(const md_params* p, void* ws, size_t ws_bytes, const float* ckpt_pos4_dev,
                             const float* ckpt_vel4_dev, int32_t first_step, int32_t nsteps,
                             float* path4_dev, int32_t* path_start_dev, float* lam_r4_dev,
                             float* lam_v4_dev, double* theta_dev, hipStream_t stream);

/*
 * The two halves of md_adjoint_segment, for callers that overlap them or
 * keep the whole trajectory. A path of nsteps states is path4_dev
 * (nsteps * n float4: state j's cell-sorted positions, w = user index bits)
 * and path_start_dev (nsteps * (n_c^3 + 1) int32: its cell offsets), both
 * caller-owned.
 *
 * md_adjoint_recompute: from the checkpoint (ckpt_pos4_dev, ckpt_vel4_dev),
 * the checkpoint and the states after its first nsteps - 1 steps into the
 * path, bitwise those md_step produces. The workspace serves as scratch and
 * is left without a built state (as md_adjoint_segment leaves it).
 *
 * md_adjoint_path: the backward sweep of md_adjoint_segment over a kept path
 * whose state 0 is the state after step first_step: from state nsteps - 1 back
 * to state 0, the drift adjoint and the kick adjoint on the state's cell list
 * (coefficient 2h, or h for the trajectory's step 0); lam_r4_dev, lam_v4_dev
 * and theta_dev accumulate as for md_adjoint_segment. The workspace must hold
 * a built state of these parameters (md_build_cells, md_step, ...); it serves
 * as scratch (its sorted arrays and forces are not touched) and keeps that
 * state. Calls on different workspaces and paths may run concurrently on
 * different streams. Force-shift mode only.
 *
 * md_step_path: nsteps steps of md_step (no thermo output, nsteps >= 1) that
 * also keep the states before each step as a path: state 0 is the workspace's
 * state at the call (copied), state j the state after j steps (sorted
 * straight into its slice); the workspace ends as after md_step. Needs a
 * state with forces, as md_step does. md_adjoint_path over this path and a
 * range of it gives bitwise the results of md_adjoint_segment over the same
 * range recomputed from a checkpoint (the recomputation is skipped at the
 * cost of nsteps * (16 n + 4 (n_c^3 + 1)) bytes of device memory).
 */
md_status md_adjoint_recompute(const md_params* p, void* ws, size_t ws_bytes, const float* ckpt_pos4_dev,
                               const float* ckpt_vel4_dev, int32_t nsteps, float* path4_dev,
                               int32_t* path_start_dev, hipStream_t stream);
md_status md_adjoint_path(const md_params* p, void* ws, size_t ws_bytes, int32_t first_step, int32_t nsteps,
                          const float* path4_dev, const int32_t* path_start_dev, float* lam_r4_dev,
                          float* lam_v4_dev, double* theta_dev, hipStream_t stream);
md_status md_step_path(const md_params* p, void* ws, size_t ws_bytes, int32_t nsteps, float* path4_dev,
                       int32_t* path_start_dev, hipStream_t stream);

/*
 * Gradient of the loss k_coef * K + w_coef * W at the current workspace
 * state (K = m/2 sum v^2, W = sum over pairs r phi(r)):
 *   g_r4_dev = w_coef * dW/dr, g_v4_dev = k_coef * m * v (both written),
 *   theta_dev[0] += w_coef * dW/d(epsilon), theta_dev[1] += w_coef * dW/d(sigma)
 * (theta_dev nullable). The mean kinetic energy plus the virial pressure,
 * K/N + W/(3V), is k_coef = 1/N, w_coef = 1/(3 L^3).
 */
md_status md_loss_grad(const md_params* p, void* ws, size_t ws_bytes, float k_coef, float w_coef,
                       float* g_r4_dev, float* g_v4_dev, double* theta_dev, hipStream_t stream);

/*
 * The loss of the adjoint workload at the current workspace state (cells
 * built): L = K / N + W / (3 V), V = L_box^3, the mean kinetic energy per
 * particle plus the virial part of the pressure (K and W as for
 * md_energy_virial; FP64 fixed-order sums). loss_dev: one device double.
 */
md_status md_loss(const md_params* p, void* ws, size_t ws_bytes, double* loss_dev, hipStream_t stream);

/*
 * Seed of the backward pass through md_step from md_loss at the current
 * (final) state r_T, v_T: with h = dt / (2 m),
 *   lam_v4_dev = scale dL/dv_T, lam_r4_dev = scale dL/dr_T + h J(r_T) lam_v4_dev
 * (written, not accumulated; the second term is the kick adjoint of the
 * step's closing half kick), theta_dev[0..1] += the matching scale
 * dL/d(epsilon, sigma) terms (nullable). Then md_adjoint_segment runs the
 * segments from the last back to the first. Force-shift mode only.
 */
md_status md_adjoint_seed(const md_params* p, void* ws, size_t ws_bytes, float scale, float* lam_r4_dev,
                          float* lam_v4_dev, double* theta_dev, hipStream_t stream);

/*
 * ---- Batches of independent replicas ----
 * Many LJ systems of different size and density advance together: every
 * phase (drift, histogram, scan, scatter, in-cell order, forces, kick) runs as
 * one launch over the atoms or cells of all replicas, and md_batch_graph_create
 * captures a whole multi-step run into one graph that md_graph_launch starts
 * with a single call. Each replica follows exactly the arithmetic of md_step
 * on that system alone (same cell grid, LDS pass length and summation order),
 * so its results are bitwise those of a solo run with the same cell side,
 * wavefronts per cell and LDS tile. The force pass runs one launch per class
 * of replicas sharing a tile band and a wavefront count.
 *
 * Shared parameters (epsilon, sigma, mass, rc_over_sigma, dt, shift_mode)
 * come from p; p->n, p->box and p->tile_cap are ignored. Per replica: the
 * minimum cell side is its own cell_min when that is nonzero, else
 * p->cell_min (the grid rule is that of md_cell_grid); the wavefronts per
 * cell its own waves_per_cell when nonzero, else p->waves_per_cell; the LDS
 * tile its own tile_cap when nonzero, else the formula of md_params.tile_cap. Replica b owns atoms
 * [A_b, A_b + n_b) of the concatenated float4 arrays, A_b = n_0 + ... +
 * n_(b-1); every replica needs box >= 2 r_c. The table is re-validated on
 * every call and must not change between calls on one workspace.
 */
typedef struct md_replica {
    int32_t n;              /* atoms of this replica, >= 1 */
    float box;              /* its cubic periodic box side */
    float cell_min;         /* its minimum cell side (finite, >= 0); 0 takes p->cell_min */
    int32_t waves_per_cell; /* 0 (p->waves_per_cell), 1, 2 or 4 */
    int32_t tile_cap;       /* 0 (the formula) or a multiple of 64 in [128, 2048] */
} md_replica;

/* Workspace bytes for this batch (0 if invalid). Host only. */
size_t md_batch_workspace_bytes(const md_params* p, const md_replica* reps, int32_t count);

/* Load all replicas (concatenated float4 arrays, vel4 nullable) and build
 * their cell lists. Uploads the replica table into the workspace and waits
 * for that copy (this call synchronises `stream` once). */
md_status md_batch_build(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                         const float* pos4_dev, const float* vel4_dev, hipStream_t stream);

/* Forces of every replica (needed once before md_batch_step); optional
 * float4 output in concatenated user order. */
md_status md_batch_forces(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                          float* force4_dev, hipStream_t stream);

/* nsteps velocity-Verlet steps of every replica. With thermo_every > 0,
 * thermo_dev receives (U, K, W) of replica b after step (r + 1) thermo_every at
 * thermo_dev[3 (r count + b) + 0..2]. */
md_status md_batch_step(const md_params* p, const md_replica* reps, int32_t count, void* ws, size_t ws_bytes,
                        int32_t nsteps, int32_t thermo_every, double* thermo_dev, hipStream_t stream);

/* U, K, W of every replica: out_dev[3 b + 0..2] (FP64, fixed-order sums). */
md_status md_batch_energy_virial(const md_params* p, const md_replica* reps, int32_t count, void* ws,
                                 size_t ws_bytes, double* out_dev, hipStream_t stream);

/* Positions and velocities in concatenated user order (either nullable). */
md_status md_batch_get_state(const md_params* p, const md_replica* reps, int32_t count, const void* ws,
                             size_t ws_bytes, float* pos4_dev, float* vel4_dev, hipStream_t stream);

/* An instantiated graph of a batched run, owned by the caller. */
typedef struct md_graph_s* md_graph;

/*
 * Capture nsteps batched steps (with optional thermo output, as in
 * md_batch_step) on `stream` into a graph and instantiate it; nothing runs
 * until md_graph_launch. stream must not be the null stream (graph capture
 * needs a real stream). The graph holds the workspace and thermo pointers:
 * both must outlive it. Creating a graph allocates host-side runtime objects
 * only; the library allocates no device memory of its own.
 */
md_status md_batch_graph_create(const md_params* p, const md_replica* reps, int32_t count, void* ws,
                                size_t ws_bytes, int32_t nsteps, int32_t thermo_every, double* thermo_dev,
                                hipStream_t stream, md_graph* graph_out);

/* Enqueue one run of the graph on `stream`. */
md_status md_graph_launch(md_graph graph, hipStream_t stream);

/* Release the graph (NULL is ignored). Synchronise any stream that launched it first. */
md_status md_graph_destroy(md_graph graph);

/*
 * Synchronise `stream`, then read and clear the device error word.
 * flags_out (host pointer, nullable) receives the MD_DEV_* bits.
 * Returns MD_ERR_DEVICE if any bit was set, MD_ERR_HIP on a runtime error.
 */
md_status md_check(void* ws, size_t ws_bytes, hipStream_t stream, int32_t* flags_out);

/* Text for the last non-OK status on this thread (never NULL). */
const char* md_last_error(void);

/* Stable name of a status code (never NULL). */
const char* md_status_name(md_status s);

#ifdef __cplusplus
}
#endif

#endif /* MDLJ_MD_H */
