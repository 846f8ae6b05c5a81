"""The C ABI: the library loads and exports every entry point include/dawn.h
declares; host-side argument checks work without a GPU (no compute calls)."""
import ctypes
import os
import re

import pytest

import paper_2306_07872_amd as dawn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dawn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(dawn_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dawn.LIB_PATH):
        from paper_2306_07872_amd import build
        build.build()
    return dawn.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    assert set(dawn.exported_symbols()) == set(names)


def test_status_strings_and_build_info(lib):
    assert lib.dawn_status_str(0) == b"ok"
    assert lib.dawn_status_str(3) == b"workspace too small"
    assert b"gfx950" in lib.dawn_build_info()


def test_tuning_roundtrip_and_range_checks(lib):
    t0 = dawn.get_tuning()
    assert t0["t_lane"] == 256 and t0["tile_k"] == 256
    prev = dawn.set_tuning(t_lane=8, tile_k=128)
    assert dawn.get_tuning()["t_lane"] == 8
    dawn.set_tuning(t_lane=4096, t_wave=4096)  # the lane tier's largest rows
    assert dawn.get_tuning()["t_lane"] == 4096
    dawn.set_tuning(t_lane=8, t_wave=2048)
    for bad in (dict(t_lane=0), dict(t_lane=4097, t_wave=8192), dict(t_lane=256, t_wave=128),
                dict(t_wave=10), dict(wg_threads=300), dict(wg_threads=128), dict(tile_k=100),
                dict(tile_k=1024), dict(mode=3), dict(t_chunk=8), dict(tile_t_wave=4),
                dict(tile_t_group=65), dict(tile_t_group=64, tile_t_wave=64),
                dict(tile_skip=2), dict(small_m=-1), dict(step_min_m=-1), dict(tile_pull=1002),
                dict(tile_pull_src=-1), dict(tile_pull_src=513), dict(ss_skip=2), dict(ss_pull=1002),
                dict(tile_sparse=513), dict(step_launches=-1), dict(step_launches=4097),
                dict(tile_step_launches=-1), dict(tile_step_launches=4097), dict(barrier_ms=-1),
                dict(barrier_ms=600001), dict(ss_tail_grid=-1)):
        with pytest.raises(dawn.DawnError) as e:
            dawn.set_tuning(**bad)
        assert e.value.status == 1
    dawn.set_tuning(**prev)
    dawn.set_tuning(reset=True)
    assert dawn.get_tuning() == t0


def test_host_side_validation_needs_no_gpu(lib):
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    # n < 1
    assert lib.dawn_sssp(fake, fake, fake, 0, 0, 0, 0, fake, null) == 1
    # m < 0
    assert lib.dawn_sssp(fake, fake, fake, 0, 5, -1, 0, fake, null) == 1
    # source out of range
    assert lib.dawn_sssp(fake, fake, fake, 0, 5, 3, 5, fake, null) == 1
    assert lib.dawn_sssp(fake, fake, fake, 0, 5, 3, -1, fake, null) == 1
    # bad weight type
    assert lib.dawn_sssp(fake, fake, fake, 7, 5, 3, 0, fake, null) == 1
    # null pointers
    assert lib.dawn_sssp(null, fake, fake, 0, 5, 3, 0, fake, null) == 1
    assert lib.dawn_sssp(fake, null, fake, 0, 5, 3, 0, fake, null) == 1
    assert lib.dawn_sssp(fake, fake, fake, 0, 5, 3, 0, null, null) == 1
    # k < 1
    assert lib.dawn_msssp(fake, fake, fake, 0, 5, 3, fake, 0, fake, null) == 1
    # workspace too small / misaligned
    need = lib.dawn_sssp_workspace_bytes(100, 1000)
    assert need > 0
    assert lib.dawn_sssp_ws(fake, fake, fake, 0, 100, 1000, 0, fake, ctypes.c_void_p(0x100000),
                            need - 1, null, null) == 3
    assert lib.dawn_sssp_ws(fake, fake, fake, 0, 100, 1000, 0, fake, ctypes.c_void_p(0x100010),
                            need, null, null) == 1
    assert b"aligned" in lib.dawn_last_error()
    assert lib.dawn_tile_bytes(100, 1000, 513) == 0
    assert lib.dawn_tile_bytes(100, 1000, 64) > 400 * 64


def test_workspace_sizes_grow_with_graph(lib):
    a = lib.dawn_sssp_workspace_bytes(1000, 8000)
    b = lib.dawn_sssp_workspace_bytes(4194304, 67108864)
    assert 0 < a < b
    # tile: the [n x K] distance tile dominates
    t = lib.dawn_msssp_workspace_bytes(1 << 20, 16 << 20, 256)
    assert t >= (1 << 20) * 256 * 4


def test_hop_count_entry_point_host_checks(lib):
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    need = lib.dawn_umsssp_workspace_bytes(100, 1000, 64)
    # no [n x K] distance tile: the reached-pairs bitset and ceil(log2 n) = 7
    # bit planes of n x K/64 words each
    assert 100 * 8 * 8 <= need < lib.dawn_msssp_workspace_bytes(100, 1000, 64)
    assert lib.dawn_umsssp_workspace_bytes(0, 10, 64) == 0

    assert lib.dawn_umsssp_workspace_bytes(100, 1000, 0) == 0
    # no weights needed; colidx is (m > 0)
    assert lib.dawn_umsssp_ws(fake, null, 100, 1000, null, fake, 4, fake, ws, need, null,
                              null) == 1
    assert lib.dawn_umsssp_ws(fake, fake, 100, 1000, null, fake, 0, fake, ws, need, null,
                              null) == 1
    assert lib.dawn_umsssp_ws(fake, fake, 100, 1000, null, null, 4, fake, ws, need, null,
                              null) == 1
    assert lib.dawn_umsssp_ws(fake, fake, 100, 1000, null, fake, 4, fake, ws, need - 1, null,
                              null) == 3
    assert lib.dawn_umsssp_ws(fake, fake, 100, 1000, ctypes.c_void_p(0x2010), fake, 4, fake, ws,
                              need, null, null) == 1
    assert b"aligned" in lib.dawn_last_error()


def test_int32_weights_are_single_source_only(lib):
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    # multi-source, all pairs, reverse-graph runs and tiles: unsupported (2)
    assert lib.dawn_msssp(fake, fake, fake, 2, 5, 3, fake, 4, fake, null) == 2
    assert lib.dawn_msssp_ws(fake, fake, fake, 2, 5, 3, fake, 4, fake, ws, 1 << 30, null,
                             null) == 2
    assert lib.dawn_apsp(fake, fake, fake, 2, 5, 3, fake, null) == 2
    assert b"single-source" in lib.dawn_last_error()
    # an unknown weight type stays invalid (1)
    assert lib.dawn_sssp(fake, fake, fake, 4, 5, 3, 0, fake, null) == 1
    # unit weights (3): not in batches or tile sessions
    h = ctypes.c_void_p()
    assert lib.dawn_tile_create(ctypes.byref(h), fake, fake, null, 3, 5, 3, 64, ws, 1 << 30,
                                null) == 2


def test_tile_session_takes_caller_workspace(lib):
    """dawn_tile_create allocates nothing: it needs a caller workspace of at
    least dawn_tile_bytes, 256-byte aligned (checked before any device call)."""
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    h = ctypes.c_void_p()
    need = lib.dawn_tile_bytes(100, 1000, 64)
    assert need > 100 * 64 * 4
    assert lib.dawn_tile_create(ctypes.byref(h), fake, fake, fake, 0, 100, 1000, 64, null, need,
                                null) == 1
    assert lib.dawn_tile_create(ctypes.byref(h), fake, fake, fake, 0, 100, 1000, 64,
                                ctypes.c_void_p(0x100010), need, null) == 1
    assert b"aligned" in lib.dawn_last_error()
    assert lib.dawn_tile_create(ctypes.byref(h), fake, fake, fake, 0, 100, 1000, 64,
                                ctypes.c_void_p(0x100000), need - 1, null) == 3
    assert h.value is None


def test_incomplete_status_code(lib):
    assert lib.dawn_status_str(5) == b"run did not converge"
    assert dawn.E_INCOMPLETE == 5


def test_noalloc_call_host_checks(lib):
    """dawn_sssp_noalloc rejects, before touching the device, graphs whose
    workspace exceeds its fixed scratch array (and the usual bad arguments)."""
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    cap = dawn.NOALLOC_SCRATCH_BYTES
    assert cap == 64 << 20
    n, m = 4_194_304, 67_108_864
    assert lib.dawn_sssp_workspace_bytes(n, m) > cap
    assert lib.dawn_sssp_noalloc(fake, fake, fake, 0, n, m, 0, fake, null) == 3
    assert b"dawn_sssp_ws" in lib.dawn_last_error()
    assert lib.dawn_sssp_workspace_bytes(2_097_152, 33_554_432) <= cap
    assert lib.dawn_sssp_noalloc(fake, fake, fake, 0, 0, 0, 0, fake, null) == 1
    assert lib.dawn_sssp_noalloc(fake, fake, fake, 0, 5, 3, 5, fake, null) == 1
    assert lib.dawn_sssp_noalloc(fake, fake, fake, 0, 5, 3, 0, null, null) == 1


def test_generic_workspace_size_dispatches_by_call(lib):
    # k = 1: the single-source call, whatever the weight type
    for wt in (0, 1, 2, 3):
        assert lib.dawn_workspace_bytes(1000, 8000, 1, wt) == lib.dawn_sssp_workspace_bytes(1000, 8000)
    # k > 1: the tile, or the hop-count tile for unit weights
    for wt in (0, 1):
        assert lib.dawn_workspace_bytes(1000, 8000, 300, wt) == lib.dawn_msssp_workspace_bytes(1000, 8000, 300)
    assert lib.dawn_workspace_bytes(1000, 8000, 300, 3) == lib.dawn_umsssp_workspace_bytes(1000, 8000, 300)
    # arguments no call accepts
    assert lib.dawn_workspace_bytes(1000, 8000, 300, 2) == 0   # int32 weights: single source only
    assert lib.dawn_workspace_bytes(0, 8000, 1, 0) == 0
    assert lib.dawn_workspace_bytes(1000, -1, 1, 0) == 0
    assert lib.dawn_workspace_bytes(1000, 8000, 0, 0) == 0
    assert lib.dawn_workspace_bytes(1000, 8000, 1, 9) == 0
