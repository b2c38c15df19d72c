"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/md.h declares, and validates arguments on the host before any HIP
call. Also pins the cell-grid rule to the paper's worked example."""
import json
import os
import re

import pytest

import paper_0709_3225_amd as md
from paper_0709_3225_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "md.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(md_[a-z_]+)\s*\(", text, flags=re.M)


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 10
    lib = _lib.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(_lib.SYMBOLS)


def test_paper_worked_example_cell_grid():
    """Section 3.2: L = 11 sigma, r_c = 2.5 sigma -> 4 cells of side 2.75."""
    g = json.load(open(os.path.join(GOLDEN, "paper_cell_example.json")))
    p = md.make_params(100, g["box"])
    nc, side = md.md_cell_grid(p)
    assert nc == g["cells_per_dim"]
    assert side == pytest.approx(g["cell_side"], rel=1e-7)


@pytest.mark.parametrize("n,rho,nc_expect", [(4000, 0.8442, 6), (256000, 0.8442, 26), (2048000, 0.8442, 53),
                                             (32000, 0.8442, 13), (256, 0.8442, 2)])
def test_cell_grid_of_workloads(n, rho, nc_expect):
    import ljsynth

    L = ljsynth.box_length(n, rho)
    nc, side = md.md_cell_grid(md.make_params(n, L))
    assert nc == nc_expect
    assert side >= 2.5
    assert md.md_workspace_bytes(md.make_params(n, L)) > 80 * n


def test_cell_side_margin_rule():
    """A side that exceeds r_c by less than 2^-18 L drops one cell, so that an
    FP32 cell index can never be off by enough to hide a partner."""
    nc, side = md.md_cell_grid(md.make_params(10, 10.0))  # 10 / 4 = 2.5 exactly
    assert nc == 3
    nc, side = md.md_cell_grid(md.make_params(10, 10.1))
    assert nc == 4 and side > 2.5


def test_cell_min_parameter():
    nc, side = md.md_cell_grid(md.make_params(10, 30.0, cell_min=4.9))
    assert nc == 6 and side == pytest.approx(5.0)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), _lib.MD_ERR_ARG),
    (dict(n=-5), _lib.MD_ERR_ARG),
    (dict(box=float("nan")), _lib.MD_ERR_ARG),
    (dict(box=4.99), _lib.MD_ERR_BOX),
    (dict(epsilon=0.0), _lib.MD_ERR_ARG),
    (dict(sigma=-1.0), _lib.MD_ERR_ARG),
    (dict(mass=float("inf")), _lib.MD_ERR_ARG),
    (dict(dt=-0.1), _lib.MD_ERR_ARG),
    (dict(shift_mode=2), _lib.MD_ERR_ARG),
    (dict(flags=4), _lib.MD_ERR_ARG),
    (dict(waves_per_cell=3), _lib.MD_ERR_ARG),
    (dict(waves_per_cell=-1), _lib.MD_ERR_ARG),
    (dict(waves_per_cell=8), _lib.MD_ERR_ARG),
    (dict(list_radius=-1.0), _lib.MD_ERR_ARG),
    (dict(list_radius=float("nan")), _lib.MD_ERR_ARG),
    (dict(list_radius=2.4), _lib.MD_ERR_ARG),  # not above r_c = 2.5
    (dict(list_radius=3.5), _lib.MD_ERR_ARG),  # beyond the cell side 10 / 3
    (dict(rc_over_sigma=float("nan")), _lib.MD_ERR_ARG),
])
def test_invalid_params_rejected_on_host(kw, code):
    base = dict(n=100, box=10.0)
    base.update(kw)
    p = md.make_params(**base)
    assert md.md_workspace_bytes(p) == 0
    with pytest.raises(md.MDError) as e:
        md.md_cell_grid(p)
    assert e.value.code == code
    # entry points that take device pointers fail the same way before any HIP call
    lib = _lib.lib()
    import ctypes

    assert lib.md_build_cells(ctypes.byref(p), None, 0, None, None, None) == code
    assert lib.md_forces(ctypes.byref(p), None, 0, None, None) == code
    assert lib.md_forces_noalloc(ctypes.byref(p), None, None, None) == code
    assert lib.md_step(ctypes.byref(p), None, 0, 1, 0, None, None) == code
    assert lib.md_energy_virial(ctypes.byref(p), None, 0, None, None) == code


def test_workspace_and_pointer_checks_on_host():
    import ctypes

    lib = _lib.lib()
    p = md.make_params(100, 10.0)
    need = md.md_workspace_bytes(p)
    fake = ctypes.c_void_p(1 << 40)  # never dereferenced: validation fails first
    assert lib.md_build_cells(ctypes.byref(p), None, need, fake, None, None) == _lib.MD_ERR_WORKSPACE
    assert lib.md_build_cells(ctypes.byref(p), ctypes.c_void_p((1 << 40) + 64), need, fake, None, None) \
        == _lib.MD_ERR_WORKSPACE
    assert lib.md_build_cells(ctypes.byref(p), fake, need - 1, fake, None, None) == _lib.MD_ERR_WORKSPACE
    assert lib.md_build_cells(ctypes.byref(p), fake, need, None, None, None) == _lib.MD_ERR_ARG
    assert lib.md_build_cells(ctypes.byref(p), fake, need, ctypes.c_void_p((1 << 40) + 4), None, None) \
        == _lib.MD_ERR_ARG
    assert lib.md_step(ctypes.byref(p), fake, need, -1, 0, None, None) == _lib.MD_ERR_ARG
    assert lib.md_step(ctypes.byref(p), fake, need, 4, 2, None, None) == _lib.MD_ERR_ARG
    assert lib.md_neighbors(ctypes.byref(p), fake, need, fake, fake, 0, None) == _lib.MD_ERR_ARG
    # the static-workspace entry point: NULL or misaligned arrays, and a system
    # whose workspace exceeds the 16 MiB static array, refused before any HIP call
    assert lib.md_forces_noalloc(ctypes.byref(p), None, fake, None) == _lib.MD_ERR_ARG
    assert lib.md_forces_noalloc(ctypes.byref(p), fake, ctypes.c_void_p((1 << 40) + 8), None) == _lib.MD_ERR_ARG
    big = md.make_params(256000, 67.18385)
    assert md.md_workspace_bytes(big) > (16 << 20)
    assert lib.md_forces_noalloc(ctypes.byref(big), fake, fake, None) == _lib.MD_ERR_WORKSPACE
    small = md.make_params(32000, 33.59192)
    assert md.md_workspace_bytes(small) <= (16 << 20)
    assert lib.md_check(None, 0, None, None) == _lib.MD_ERR_WORKSPACE
    assert b"workspace" in lib.md_last_error()
    assert lib.md_loss(ctypes.byref(p), fake, need, None, None) == _lib.MD_ERR_ARG
    assert lib.md_thermo(ctypes.byref(p), fake, need, None, None) == _lib.MD_ERR_ARG
    assert lib.md_adjoint_seed(ctypes.byref(p), fake, need, ctypes.c_float(1.0), fake, fake, None, None) \
        == _lib.MD_ERR_ARG  # the two adjoint vectors alias


def test_tile_cap_parameter():
    """md_params.tile_cap: 0 takes the formula (1.1 x the mean 27-cell
    neighbourhood + 32, rounded up to a multiple of 64 in [128, 2048]), other
    values must be multiples of 64 in [128, 2048]; md_tile_capacity reports
    the tile and 0 for invalid parameters; the tile leaves the workspace
    layout alone."""
    import ctypes
    import math

    for n, box in ((256000, 67.18385), (4000, 16.79596), (32000, 33.59192), (2048000, 134.3677)):
        p = md.make_params(n, box)
        nc, _ = md.md_cell_grid(p)
        hood = 27.0 * n / nc ** 3
        want = min(2048, max(128, math.ceil((1.1 * hood + 32.0) / 64.0) * 64))
        assert md.md_tile_capacity(p) == want
        q = md.make_params(n, box, tile_cap=768)
        assert md.md_tile_capacity(q) == 768
        assert md.md_workspace_bytes(q) == md.md_workspace_bytes(p)
    assert md.md_tile_capacity(md.make_params(256000, 67.18385)) == 512
    lib = _lib.lib()
    for bad in (64, 100, 200, 2112, 4096, -64):
        p = md.make_params(4000, 16.79596, tile_cap=bad)
        assert md.md_workspace_bytes(p) == 0
        assert lib.md_tile_capacity(ctypes.byref(p)) == 0
        assert b"tile_cap" in lib.md_last_error()
    assert md.tile_options(md.make_params(256000, 67.18385)) == [0, 640, 448]
    # the formula's floor: 128 atoms for a sparse system, so -64 is dropped
    sparse = md.make_params(50, 10.0)
    assert md.md_tile_capacity(sparse) == 128
    assert md.tile_options(sparse, offsets=(0, -64, 128)) == [0, 256]


def test_path_entry_points_validate_on_host():
    """md_step_path, md_adjoint_recompute and md_adjoint_path refuse empty
    paths, NULL or misaligned arrays, aliased adjoint vectors and the
    energy-shift mode before any HIP call."""
    import ctypes

    lib = _lib.lib()
    p = md.make_params(100, 10.0)
    need = md.md_workspace_bytes(p)
    fake = ctypes.c_void_p(1 << 40)  # never dereferenced: validation fails first
    other = ctypes.c_void_p((1 << 40) + 4096)
    odd = ctypes.c_void_p((1 << 40) + 8)
    ERR = _lib.MD_ERR_ARG
    assert lib.md_step_path(ctypes.byref(p), fake, need, 0, fake, fake, None) == ERR
    assert lib.md_step_path(ctypes.byref(p), fake, need, 3, None, fake, None) == ERR
    assert lib.md_step_path(ctypes.byref(p), fake, need, 3, fake, None, None) == ERR
    assert lib.md_step_path(ctypes.byref(p), fake, need, 3, odd, fake, None) == ERR
    assert lib.md_step_path(ctypes.byref(p), None, need, 3, fake, fake, None) == _lib.MD_ERR_WORKSPACE
    assert lib.md_adjoint_recompute(ctypes.byref(p), fake, need, fake, fake, 0, fake, fake, None) == ERR
    assert lib.md_adjoint_recompute(ctypes.byref(p), fake, need, None, fake, 2, fake, fake, None) == ERR
    assert lib.md_adjoint_recompute(ctypes.byref(p), fake, need, fake, odd, 2, fake, fake, None) == ERR
    assert lib.md_adjoint_path(ctypes.byref(p), fake, need, -1, 2, fake, fake, fake, other, None, None) == ERR
    assert lib.md_adjoint_path(ctypes.byref(p), fake, need, 0, 0, fake, fake, fake, other, None, None) == ERR
    assert lib.md_adjoint_path(ctypes.byref(p), fake, need, 0, 2, fake, fake, fake, fake, None, None) == ERR
    assert lib.md_adjoint_path(ctypes.byref(p), fake, need, 0, 2, fake, fake, None, other, None, None) == ERR
    assert lib.md_adjoint_path(ctypes.byref(p), fake, need, 0, 2, fake, fake, odd, other, None, None) == ERR
    e = md.make_params(100, 10.0, shift_mode=1)
    assert lib.md_adjoint_path(ctypes.byref(e), fake, md.md_workspace_bytes(e), 0, 2, fake, fake, fake, other,
                               None, None) == ERR
    assert b"shift_mode 0" in lib.md_last_error()


def test_pair_list_arrays_only_on_request():
    """md_step_list's arrays are laid out only with MD_FLAG_PAIR_LISTS, and
    md_step_list refuses a workspace without them (host check)."""
    import ctypes

    lib = _lib.lib()
    plain = md.make_params(256000, 67.18385)
    lists = md.make_params(256000, 67.18385, flags=_lib.MD_FLAG_PAIR_LISTS)
    b0, b1 = md.md_workspace_bytes(plain), md.md_workspace_bytes(lists)
    assert b1 - b0 > 4096 * 26 ** 3  # about 4.3 KB per cell of accept words
    fake = ctypes.c_void_p(1 << 40)
    assert lib.md_step_list(ctypes.byref(plain), fake, b0, 4, 2, 0, None, None) == _lib.MD_ERR_ARG
    assert b"MD_FLAG_PAIR_LISTS" in lib.md_last_error()


def test_atom_list_arrays_only_on_request():
    """md_step_nlist's per-atom lists are laid out only with
    MD_FLAG_ATOM_LISTS (4 B per entry: 1.5 x the mean number of atoms within
    the cell side, plus 32, in multiples of 32; 128 entries at rho = 0.8442
    on the 26^3 grid), and md_step_nlist refuses a workspace without them."""
    import ctypes

    lib = _lib.lib()
    plain = md.make_params(256000, 67.18385)
    lists = md.make_params(256000, 67.18385, flags=_lib.MD_FLAG_ATOM_LISTS)
    both = md.make_params(256000, 67.18385, flags=_lib.MD_FLAG_ATOM_LISTS | _lib.MD_FLAG_PAIR_LISTS)
    b0, b1, b2 = md.md_workspace_bytes(plain), md.md_workspace_bytes(lists), md.md_workspace_bytes(both)
    extra = b1 - b0
    # lists (128 entries) + counts + reference positions, each array 256-byte aligned
    assert 256000 * (128 * 4 + 4 + 16) <= extra <= 256000 * (128 * 4 + 4 + 16) + 1024
    assert b2 > b1 > b0
    fake = ctypes.c_void_p(1 << 40)
    assert lib.md_step_nlist(ctypes.byref(plain), fake, b0, 4, 2, 0, None, None) == _lib.MD_ERR_ARG
    assert b"MD_FLAG_ATOM_LISTS" in lib.md_last_error()
    assert lib.md_step_nlist(ctypes.byref(lists), fake, b1, 4, 0, 0, None, None) == _lib.MD_ERR_ARG  # rebuild_every


def test_status_names():
    lib = _lib.lib()
    assert lib.md_status_name(0) == b"MD_OK"
    assert lib.md_status_name(2) == b"MD_ERR_BOX"
    assert lib.md_status_name(99) == b"MD_UNKNOWN"


def test_batch_validation_on_host():
    import ctypes

    lib = _lib.lib()
    p = md.make_params(1, 1.0)
    ok = _lib.replica_table([(100, 10.0), (4000, 16.8)])
    bad = _lib.replica_table([(100, 10.0), (50, 4.0)])
    assert lib.md_batch_workspace_bytes(ctypes.byref(p), ok, 2) > 0
    assert lib.md_batch_workspace_bytes(ctypes.byref(p), bad, 2) == 0
    assert lib.md_batch_build(ctypes.byref(p), bad, 2, None, 0, None, None, None) == _lib.MD_ERR_BOX
    assert b"replica 1" in lib.md_last_error()
    assert lib.md_batch_workspace_bytes(ctypes.byref(p), ok, 0) == 0
    g = ctypes.c_void_p()
    need = lib.md_batch_workspace_bytes(ctypes.byref(p), ok, 2)
    fake = ctypes.c_void_p(1 << 40)
    # a null stream cannot be captured: refused before any HIP call
    assert lib.md_batch_graph_create(ctypes.byref(p), ok, 2, fake, need, 10, 0, None, None, ctypes.byref(g)) \
        == _lib.MD_ERR_ARG
    assert lib.md_graph_destroy(None) == 0
    # per-replica wavefronts and tiles: valid values lay the workspace out the
    # same way, invalid ones are refused with the replica named
    knobs = _lib.replica_table([(100, 10.0, 0.0, 4, 192), (4000, 16.8, 0.0, 2, 0)])
    assert lib.md_batch_workspace_bytes(ctypes.byref(p), knobs, 2) == need
    for bad_knob in ((100, 10.0, 0.0, 3, 0), (100, 10.0, 0.0, 0, 100), (100, 10.0, 0.0, 0, 4096)):
        t = _lib.replica_table([(4000, 16.8), bad_knob])
        assert lib.md_batch_workspace_bytes(ctypes.byref(p), t, 2) == 0
        assert lib.md_batch_build(ctypes.byref(p), t, 2, None, 0, None, None, None) == _lib.MD_ERR_ARG
        assert b"replica 1" in lib.md_last_error()


def test_batch_replica_cell_min_on_host():
    """A replica's own cell_min replaces the shared one (0 keeps it); invalid
    values are refused with the replica's index, before any device work."""
    import ctypes
    import math

    lib = _lib.lib()
    p = md.make_params(1, 1.0)
    base = _lib.replica_table([(4000, 17.878), (4000, 17.878)])
    coarse = _lib.replica_table([(4000, 17.878), (4000, 17.878, 17.878 / 6.5)])
    assert lib.md_batch_workspace_bytes(ctypes.byref(p), coarse, 2) > 0
    assert lib.md_batch_workspace_bytes(ctypes.byref(p), coarse, 2) != \
        lib.md_batch_workspace_bytes(ctypes.byref(p), base, 2)  # fewer cells, larger buckets
    for badval in (-1.0, math.inf, math.nan):
        bad = _lib.replica_table([(4000, 17.878), (4000, 17.878, badval)])
        assert lib.md_batch_workspace_bytes(ctypes.byref(p), bad, 2) == 0
        assert lib.md_batch_build(ctypes.byref(p), bad, 2, None, 0, None, None, None) == _lib.MD_ERR_ARG
        assert b"replica 1" in lib.md_last_error()
        assert b"cell_min" in lib.md_last_error()


def test_grid_options_and_buckets():
    """The tuner's candidate grids: the default grid first, then coarser grids
    that md_cell_grid confirms, never below 2 cells per dimension or above the
    occupancy limit; members of one bucket share grid and occupancy."""
    from paper_0709_3225_amd.tune import bucket_key, grid_options

    L = 17.878  # N = 4000 at rho = 0.70: 7 cells of 2.554
    opts = grid_options(4000, L, extra=2)
    assert opts[0] == (7, 0.0)
    assert [nc for nc, _ in opts] == [7, 6, 5]
    for nc, cm in opts[1:]:
        got, side = md.md_cell_grid(md.make_params(4000, L, cell_min=cm))
        assert got == nc and side >= cm and side >= 2.5
    assert grid_options(500, 8.939, extra=2) == [(3, 0.0)]  # 2 cells would hold 62 atoms each
    assert grid_options(4000, L, extra=2, max_occupancy=20.0) == [(7, 0.0), (6, L / 6.5)]
    # a sparse system also gets the grid sized for about 14 atoms per cell
    Ls = (256000 / 0.1) ** (1.0 / 3.0)
    assert [nc for nc, _ in grid_options(256000, Ls)] == [54, 53, 26]
    assert bucket_key(4000, 7) == (7, 12)
    assert bucket_key(4000, 7) == bucket_key(4100, 7)

