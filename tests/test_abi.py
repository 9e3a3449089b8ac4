"""C-ABI checks that need no GPU: symbols, argument validation, error paths, tuning table I/O.

Every call here either fails validation (which runs before any HIP call) or
is a host-only function, so nothing is enqueued on a device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "haar.h")


@pytest.fixture(scope="module")
def abi():
    from paper_1002_2184_amd import build as B
    B.build(force=False)
    from paper_1002_2184_amd import _abi
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(haar_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(abi):
    names = declared_functions()
    assert len(names) >= 20, names
    lib = ctypes.CDLL(abi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in haar.h but not exported"
    assert set(names) == set(abi.exported_names()), "binding and header disagree"


def test_binding_has_same_names(abi):
    for n in declared_functions():
        assert callable(getattr(abi, n)), n


def test_max_levels(abi):
    assert abi.haar_max_levels_1d(1) == 0
    assert abi.haar_max_levels_1d(2) == 1
    assert abi.haar_max_levels_1d(65536) == 16
    assert abi.haar_max_levels_1d(65537) == 17
    assert abi.haar_max_levels_1d(0) == -1
    assert abi.haar_max_levels_2d(4096, 4096) == 12
    assert abi.haar_max_levels_2d(3, 1000) == 10
    assert abi.haar_max_levels_2d(0, 5) == -1
    assert abi.haar_max_levels_3d(256, 256, 256) == 8
    assert abi.haar_max_levels_3d(3, 1000, 5) == 10
    assert abi.haar_max_levels_3d(1, 1, 1) == 0
    assert abi.haar_max_levels_3d(4, 0, 4) == -1


X, Y = 0x10000000, 0x20000000     # fake, non-overlapping device addresses (never dereferenced)


@pytest.mark.parametrize("call,code", [
    (lambda a: a.haar_fwd_1d(X, Y, 16, 2, 1, 7, 0), 2),          # dtype
    (lambda a: a.haar_fwd_1d(X, Y, 0, 0, 1, 0, 0), 3),           # length < 1
    (lambda a: a.haar_fwd_1d(X, Y, 16, 2, -1, 0, 0), 3),         # batch < 0
    (lambda a: a.haar_fwd_1d(X, Y, 16, 5, 1, 0, 0), 4),          # levels > log2
    (lambda a: a.haar_inv_1d(X, Y, 16, -1, 1, 0, 0), 4),         # levels < 0
    (lambda a: a.haar_fwd_1d(0, Y, 16, 2, 1, 0, 0), 1),          # NULL input
    (lambda a: a.haar_inv_1d(X, 0, 16, 2, 1, 0, 0), 1),          # NULL output
    (lambda a: a.haar_fwd_1d(X, X + 8, 16, 2, 1, 0, 0), 5),      # overlap
    (lambda a: a.haar_fwd_2d(X, Y, 0, 8, 1, 1, 0, 0), 3),
    (lambda a: a.haar_fwd_2d(X, Y, 8, 8, 4, 1, 0, 0), 4),
    (lambda a: a.haar_inv_2d(X, Y, 8, 8, 1, 1, 3, 0), 2),
    (lambda a: a.haar_inv_2d(X, X, 8, 8, 1, 1, 0, 0), 5),        # in place
    (lambda a: a.haar_fwd_2d(X, Y, 1 << 40, 1 << 40, 1, 1, 0, 0), 3),   # size overflow
    (lambda a: a.haar_shrink_1d(X, Y, 64, 2, 1, 0, 2, [1.0, 1.0], 0), 10),        # mode
    (lambda a: a.haar_shrink_1d(X, Y, 64, 2, 1, 0, 0, [1.0, -1.0], 0), 10),       # negative threshold
    (lambda a: a.haar_shrink_1d(X, Y, 64, 2, 1, 0, 1, [float("nan"), 1.0], 0), 10),
    (lambda a: a.haar_shrink_1d(X, Y, 64, 2, 1, 0, 0, None, 0), 1),               # no thresholds
    (lambda a: a.haar_shrink_1d(X, Y, 1 << 14, 13, 1, 0, 0, [1.0] * 13, 0), 9),   # beyond one chunk
    (lambda a: a.haar_shrink_1d(X, X + 4, 64, 2, 1, 0, 0, [1.0, 1.0], 0), 5),
    (lambda a: a.haar_shrink_2d(X, Y, 64, 64, 6, 1, 0, 0, [1.0] * 6, 0), 9),      # beyond one tile
    (lambda a: a.haar_shrink_2d(X, Y, 8, 8, 4, 1, 0, 0, [1.0] * 4, 0), 4),        # levels > log2
    (lambda a: a.haar_shrink_2d(X, Y, 8, 8, 2, 1, 5, 0, [1.0] * 2, 0), 2),        # dtype
    (lambda a: a.haar_direct_1d(X, Y, 64, 3, 1, 0, 0, 0, 0, 0), 1),                # no workspace
    (lambda a: a.haar_direct_1d(X, Y, 64, 3, 1, 0, 0, 0x30000000, 16, 0), 6),      # too small
    (lambda a: a.haar_direct_1d(X, Y, 64, 3, 1, 0, 0, 0x30000002, 1 << 20, 0), 6), # misaligned
    (lambda a: a.haar_direct_1d(X, Y, 64, 7, 1, 0, 0, 0x30000000, 1 << 20, 0), 4),  # levels
    (lambda a: a.haar_fwd_3d(X, Y, 0, 8, 8, 1, 1, 0, 0), 3),                        # depth < 1
    (lambda a: a.haar_fwd_3d(X, Y, 8, 8, 8, 4, 1, 0, 0), 4),                        # levels > log2
    (lambda a: a.haar_inv_3d(X, Y, 8, 8, 8, 1, 1, 3, 0), 2),                        # dtype
    (lambda a: a.haar_inv_3d(X, X + 64, 8, 8, 8, 1, 1, 0, 0), 5),                   # overlap
    (lambda a: a.haar_fwd_3d(X, Y, 1 << 30, 1 << 30, 1 << 30, 1, 1, 0, 0), 3),      # size overflow
    (lambda a: a.haar_fwd_3d(0, Y, 8, 8, 8, 1, 1, 0, 0), 1),                        # NULL input
    (lambda a: a.haar_l1_grad_2d(X, Y, 0x30000000, 64, 64, 6, 1, 0, 0), 9),         # beyond one tile
    (lambda a: a.haar_l1_grad_2d(X, Y, 0x30000000, 8, 8, 4, 1, 0, 0), 4),           # levels > log2
    (lambda a: a.haar_l1_grad_2d(X, Y, 0, 64, 64, 2, 1, 0, 0), 1),                  # no loss array
    (lambda a: a.haar_l1_grad_2d(X, X + 8, 0x30000000, 64, 64, 2, 1, 0, 0), 5),     # overlap
    (lambda a: a.haar_l1_grad_2d_noalloc(X, Y, 0x30000000, 64, 64, 6, 1, 0, 0), 9),  # beyond one tile
    (lambda a: a.haar_l1_grad_2d_noalloc(X, Y, 0x30000000, 8, 8, 4, 1, 0, 0), 4),    # levels > log2
    (lambda a: a.haar_l1_grad_2d_noalloc(X, Y, 0, 64, 64, 2, 1, 0, 0), 1),           # no loss array
    (lambda a: a.haar_l1_grad_2d_noalloc(X, X + 8, 0x30000000, 64, 64, 2, 1, 0, 0), 5),  # overlap
    (lambda a: a.haar_l1_grad_2d_noalloc(X, Y, 0x30000000, 64, 64, 2, 1, 7, 0), 2),  # dtype
])
def test_validation_codes(abi, call, code):
    assert call(abi) == code
    assert abi.haar_last_error() != ""


def test_overlap_detects_tail(abi, monkeypatch):
    # 8x8 f32 = 256 bytes: an output starting inside the input range overlaps
    assert abi.haar_fwd_2d(X, X + 252, 8, 8, 1, 1, 0, 0) == 5
    assert abi.haar_fwd_2d(X + 252, X, 8, 8, 1, 1, 0, 0) == 5
    # bf16: 128 bytes, so +128 does not overlap and passes validation; the
    # fault hook stops the call before anything is enqueued (fake pointers)
    monkeypatch.setenv("HAAR_FAULT_INJECT", "launch")
    assert abi.haar_fwd_2d(X, X + 128, 8, 8, 1, 1, 1, 0) == 7


# Fake device pointers far enough apart for multi-GiB shapes (validation only).
FAR_X, FAR_Y, FAR_LOSS = 1 << 40, 1 << 42, 1 << 44


@pytest.mark.parametrize("dt,tile", [(0, 32 * 128), (1, 32 * 256), (2, 32 * 256)])
def test_l1_grad_noalloc_limit(abi, monkeypatch, dt, tile):
    """The static loss-partial array holds 2^19 tiles: one more is refused
    before any HIP call; exactly the limit passes validation (the fault hook
    then stops it before anything is enqueued)."""
    limit = 1 << 19
    # one tile per item, then the limit plus one
    assert abi.haar_l1_grad_2d_noalloc(FAR_X, FAR_Y, FAR_LOSS, 32, tile // 32, 5, limit + 1, dt, 0) == 6
    assert "static scratch" in abi.haar_last_error()
    # ragged items: a 33 x (W + 1) image covers 4 tiles (2 x 2 with the edges)
    w = tile // 32 + 1
    assert abi.haar_l1_grad_2d_noalloc(FAR_X, FAR_Y, FAR_LOSS, 33, w, 5, limit // 4 + 1, dt, 0) == 6
    monkeypatch.setenv("HAAR_FAULT_INJECT", "launch")
    assert abi.haar_l1_grad_2d_noalloc(FAR_X, FAR_Y, FAR_LOSS, 32, tile // 32, 5, limit, dt, 0) == 7
    assert abi.haar_l1_grad_2d_noalloc(FAR_X, FAR_Y, FAR_LOSS, 33, w, 5, limit // 4, dt, 0) == 7


def test_shrink_accepts_infinite_threshold(abi, monkeypatch):
    monkeypatch.setenv("HAAR_FAULT_INJECT", "launch")     # valid call, stopped before any HIP call
    assert abi.haar_shrink_2d(X, Y, 64, 64, 2, 1, 0, 1, [float("inf"), 0.0], 0) == 7
    assert abi.haar_shrink_1d(X, Y, 64, 0, 1, 0, 0, None, 0) == 7        # levels 0: a copy


def test_direct_workspace_size(abi):
    # full-rate streams (low-pass as FP32 pairs) plus two pair buffers
    assert abi.haar_direct_workspace_size(64, 3) == (3 * 3 * 64 + 4 * 3 * 32) * 4
    assert abi.haar_direct_workspace_size(65, 1) == (3 * 65 + 4 * 33) * 4
    assert abi.haar_direct_workspace_size(0, 1) == 0


def test_batch_zero_is_a_noop(abi):
    assert abi.haar_shrink_1d(0, 0, 16, 2, 0, 0, 0, [1.0, 1.0], 0) == 0
    assert abi.haar_fwd_1d(0, 0, 16, 2, 0, 0, 0) == 0
    assert abi.haar_inv_2d(0, 0, 8, 8, 3, 0, 1, 0) == 0
    assert abi.haar_fwd_3d(0, 0, 8, 8, 8, 3, 0, 2, 0) == 0


def test_fault_injection_maps_to_hip_error(abi, monkeypatch):
    monkeypatch.setenv("HAAR_FAULT_INJECT", "launch")
    assert abi.haar_fwd_2d(X, Y, 64, 64, 3, 1, 0, 0) == 7
    assert "injected" in abi.haar_last_error()
    assert abi.haar_inv_1d(X, Y, 64, 3, 2, 1, 0) == 7


def test_status_strings(abi):
    assert abi.haar_status_string(0) == "HAAR_OK"
    assert abi.haar_status_string(5) == "HAAR_ERR_ALIAS"
    assert abi.haar_status_string(10) == "HAAR_ERR_ARG"
    assert abi.haar_status_string(99) == "HAAR_ERR_UNKNOWN"
    assert "gfx950" in abi.haar_version()


def test_python_check_raises(abi):
    with pytest.raises(abi.HaarError) as ei:
        abi.check(abi.haar_fwd_1d(X, Y, 16, 9, 1, 0, 0))
    assert ei.value.status == 4


def test_tuning_table_roundtrip(abi, tmp_path):
    src = tmp_path / "in.json"
    src.write_text('{\n  "format": "libhaar-tuning-1",\n  "2d:f32:fwd:L5:h12:w12": 2,\n'
                   '  "1d:bf16:inv:L10:n10": 3,\n  "2d:f32:fwd:L1:h1:w1": 99\n}\n')
    assert abi.haar_tune_load(str(src)) == 0
    out = tmp_path / "out.json"
    assert abi.haar_tune_save(str(out)) == 0
    text = out.read_text()
    assert '"2d:f32:fwd:L5:h12:w12": 2' in text
    assert '"1d:bf16:inv:L10:n10": 3' in text
    assert "99" not in text                       # out-of-range index rejected
    bad = tmp_path / "bad.json"
    bad.write_text("not a tuning file")
    assert abi.haar_tune_load(str(bad)) == 9
    assert abi.haar_tune_load(str(tmp_path / "missing.json")) == 9


def test_tuning_validation(abi):
    choice = ctypes.c_int32(-1)
    assert abi.haar_tune_2d(0, 0, 64, 64, 3, 1, 0, 0, 0, ctypes.byref(choice)) == 1
    assert abi.haar_tune_2d(0, 0, 64, 64, 9, 1, X, 1 << 20, 0, ctypes.byref(choice)) == 4
    assert abi.haar_tune_2d(0, 0, 64, 64, 3, 1, X, 100, 0, ctypes.byref(choice)) == 6
    assert abi.haar_tune_1d(5, 0, 64, 3, 1, X, 1 << 20, 0, ctypes.byref(choice)) == 2
    assert abi.haar_tune_candidates_2d(0) >= 2
    assert "tile" in abi.haar_tune_candidate_name(0, 0)
    assert abi.haar_force_config_2d(0, 99) == 9
    assert abi.haar_force_config_2d(0, -1) == 0


def _items2d(abi, shapes, levels):
    items = (abi.Item2D * len(shapes))()
    for i, (h, w) in enumerate(shapes):
        items[i] = abi.Item2D(X + i * (1 << 24), Y + i * (1 << 24), h, w, levels)
    return items


def test_plan_validation_and_sizes(abi, monkeypatch):
    plan = ctypes.c_void_p()
    items = _items2d(abi, [(64, 96), (33, 300)], 3)
    assert abi.haar_plan_create_2d(items, 2, 0, 0, ctypes.byref(plan)) == 0
    nb = ctypes.c_size_t()
    assert abi.haar_plan_workspace_size(plan, ctypes.byref(nb)) == 0
    assert nb.value % 256 == 0 and nb.value > 0
    tiles = ctypes.c_int64()
    assert abi.haar_plan_info(plan, ctypes.byref(tiles), None) == 0
    # 32x256 f32 tiles: 64x96 -> 2x1, 33x300 -> 2x2
    assert tiles.value == 6
    assert abi.haar_plan_execute(plan, X, 0) == 8          # not uploaded
    assert abi.haar_plan_set_config(plan, 10) == 9          # configs 0..9 (shape + 2 * schedule)
    assert abi.haar_plan_set_config(plan, -1) == 9
    assert abi.haar_plan_set_config(plan, 9) == 0
    monkeypatch.setenv("HAAR_FAULT_INJECT", "launch")
    assert abi.haar_plan_upload(plan, X, 0) == 7             # stopped before any HIP call
    assert abi.haar_plan_upload(plan, X + 8, 0) == 6         # misaligned workspace
    assert abi.haar_plan_destroy(plan) == 0
    bad = _items2d(abi, [(64, 96)], 6)                       # > 5 levels in a 2D plan
    assert abi.haar_plan_create_2d(bad, 1, 0, 0, ctypes.byref(plan)) == 4
    alias = (abi.Item2D * 1)(abi.Item2D(X, X + 4, 8, 8, 1))
    assert abi.haar_plan_create_2d(alias, 1, 0, 0, ctypes.byref(plan)) == 5
    assert abi.haar_plan_create_2d(items, 0, 0, 0, ctypes.byref(plan)) == 8
    assert abi.haar_plan_create_2d(items, 2, 4, 0, ctypes.byref(plan)) == 2


def test_plan_1d_validation(abi):
    plan = ctypes.c_void_p()
    items = (abi.Item1D * 3)(abi.Item1D(X, Y, 4096, 12), abi.Item1D(X + (1 << 26), Y + (1 << 26), 1 << 20, 20),
                             abi.Item1D(X + (2 << 26), Y + (2 << 26), 1000, 10))
    assert abi.haar_plan_create_1d(items, 3, 0, 0, ctypes.byref(plan)) == 0
    tiles = ctypes.c_int64()
    assert abi.haar_plan_info(plan, ctypes.byref(tiles), None) == 0
    assert tiles.value == 1 + 256 + 1
    assert abi.haar_plan_set_config(plan, 3) == 9           # 1D: schedules 0..2 only
    assert abi.haar_plan_set_config(plan, 2) == 0
    assert abi.haar_plan_destroy(plan) == 0
    deep = (abi.Item1D * 1)(abi.Item1D(X, Y + (1 << 40), 1 << 23, 23))
    assert abi.haar_plan_create_1d(deep, 1, 0, 0, ctypes.byref(plan)) == 9
    bad = (abi.Item1D * 1)(abi.Item1D(X, Y, 100, 8))
    assert abi.haar_plan_create_1d(bad, 1, 0, 0, ctypes.byref(plan)) == 4
