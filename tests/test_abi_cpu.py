"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects invalid requests before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1905_09345_amd import kp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kp_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(kp.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = kp.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_struct_layouts():
    assert ctypes.sizeof(kp.kp_problem) == 48
    assert kp.kp_problem.points_dev.offset == 24 and kp.kp_problem.seed.offset == 40
    assert ctypes.sizeof(kp.kp_tuning) == 40 and kp.kp_tuning.bound_codes.offset == 20
    assert kp.kp_tuning.timing_stages.offset == 24 and kp.kp_tuning.deterministic.offset == 28
    assert kp.kp_tuning.local_filter.offset == 32 and kp.kp_tuning.plain.offset == 36
    assert ctypes.sizeof(kp.kp_stage_time) == 40
    assert ctypes.sizeof(kp.kp_iter_stats) == 80 and kp.kp_iter_stats.point_filter_fail.offset == 8
    assert kp.kp_iter_stats.closed.offset == 64 and kp.kp_iter_stats.row_test.offset == 72


def _prob(**kw):
    base = dict(n=1000, d=32, k=16, g=4, precision=0, points_dev=4096, init_centroids_dev=8192, seed=0)
    base.update(kw)
    return kp.kp_problem(**base)


def test_workspace_bytes_valid_and_monotone():
    a = kp.kp_workspace_bytes([_prob()])
    b = kp.kp_workspace_bytes([_prob(n=2000)])
    c = kp.kp_workspace_bytes([_prob(precision=1)])
    assert 0 < a < b and a < c
    # several problems: their regions plus the batch header (descriptors and block tables)
    two = kp.kp_workspace_bytes([_prob(), _prob(n=2000)])
    assert a + b < two <= a + b + 64 * 1024


@pytest.mark.parametrize("bad", [dict(n=0), dict(k=0), dict(k=2000), dict(g=0), dict(g=17), dict(d=0),
                                 dict(d=2000), dict(precision=7), dict(points_dev=0),
                                 dict(init_centroids_dev=0), dict(points_dev=4100)])
def test_invalid_problem_rejected(bad):
    assert kp.kp_workspace_bytes([_prob(**bad)]) == 0
    assert kp.kp_last_error() != ""
    with pytest.raises(kp.KPError) as e:
        kp.kp_init([_prob(**bad)], 1 << 20, 1 << 30)
    assert e.value.status == kp.KP_ERR_INVALID


@pytest.mark.parametrize("field,value", [("timing", 7), ("chunk_depth", 2), ("chunk_depth", -1),
                                         ("waves_per_block", 5), ("use_graph", 3), ("bound_codes", 3),
                                         ("bound_codes", -1), ("timing_stages", 512), ("timing_stages", -1)])
def test_invalid_tuning_rejected(field, value):
    t = kp.kp_tuning(**{field: value})
    assert kp.kp_workspace_bytes([_prob()], t) == 0


def test_valid_tuning_accepted():
    for depth in (0, 1, 3):
        assert kp.kp_workspace_bytes([_prob()], kp.kp_tuning(chunk_depth=depth)) > 0
    for g in (-1, 1, 2):
        assert kp.kp_workspace_bytes([_prob()], kp.kp_tuning(use_graph=g)) > 0


def test_whole_call_graph_needs_timing_off():
    # one graph per kp_iterate call has no stage events to time
    assert kp.kp_workspace_bytes([_prob()], kp.kp_tuning(use_graph=2, timing=1)) == 0
    assert "timing" in kp.kp_last_error()


def test_fp16_bound_codes_shrink_bf16_workspace():
    # BF16 mode: 128-byte bound rows of roundup(g, 32) FP32 bounds or roundup(g, 64)
    # FP16 codes; FP32 mode keeps its FP32 bounds
    n, g = 4096, 100
    bf = _prob(precision=1, n=n, g=g, k=1024)
    fp32 = kp.kp_workspace_bytes([bf], kp.kp_tuning(bound_codes=1))
    fp16 = kp.kp_workspace_bytes([bf], kp.kp_tuning(bound_codes=2))
    want = n * (128 * 4 - 128 * 2)
    assert fp32 == kp.kp_workspace_bytes([bf]) and abs((fp32 - fp16) - want) <= 256
    f = _prob(precision=0)
    assert kp.kp_workspace_bytes([f], kp.kp_tuning(bound_codes=2)) == kp.kp_workspace_bytes([f])


def test_init_argument_errors_before_device_use():
    need = kp.kp_workspace_bytes([_prob()])
    with pytest.raises(kp.KPError) as e:
        kp.kp_init([_prob()], 256, need - 1)          # short workspace
    assert e.value.status == kp.KP_ERR_INVALID
    with pytest.raises(kp.KPError) as e:
        kp.kp_init([_prob()], 257, need)              # misaligned workspace
    assert e.value.status == kp.KP_ERR_INVALID
    with pytest.raises(kp.KPError) as e:
        kp.kp_init([_prob(d=300)], 256, 1 << 40)      # FP32 mode limit
    assert e.value.status == kp.KP_ERR_UNSUPPORTED
    L = kp.lib()
    assert L.kp_init(None, None, 0, None, 0, None, None) == kp.KP_ERR_INVALID


def test_null_ctx_calls():
    L = kp.lib()
    assert L.kp_iterate(None, 1) == kp.KP_ERR_INVALID
    assert L.kp_assign(None, 0, None) == kp.KP_ERR_INVALID
    assert L.kp_centroids(None, 0, None, None) == kp.KP_ERR_INVALID
    n = ctypes.c_int32(0)
    assert L.kp_stats(None, 0, None, 0, ctypes.byref(n)) == kp.KP_ERR_INVALID
    assert L.kp_stage_times(None, None, 0, ctypes.byref(n)) == kp.KP_ERR_INVALID
    assert L.kp_destroy(None) == kp.KP_OK
    assert L.kp_iterations(None) == -1
    assert L.kp_predict(None, 0, None, 10, None, None, 0) == kp.KP_ERR_INVALID
    assert L.kp_predict_scratch_bytes(None, 0, 10) == 0
    assert b"ctx" in L.kp_last_error()


def test_strerror():
    for s in range(6):
        assert kp.kp_strerror(s)
    assert kp.kp_strerror(99) == "unknown status"


def test_autotune_groups_argument_errors():
    lib = kp.lib()
    arr, n = kp._probs([_prob()])
    gs = (ctypes.c_int32 * 1)()
    assert lib.kp_autotune_groups(arr, n, None, 0, None, 4, None, None) == kp.KP_ERR_INVALID       # no output
    assert lib.kp_autotune_groups(arr, n, None, 0, None, 1, None, gs) == kp.KP_ERR_INVALID         # iters < 2
    assert lib.kp_autotune_groups(arr, 0, None, 0, None, 4, None, gs) == kp.KP_ERR_INVALID         # no problems
    assert lib.kp_autotune_groups(arr, n, None, 16, None, 4, None, gs) == kp.KP_ERR_INVALID        # workspace too small
    assert b"smaller" in lib.kp_last_error()


def test_autotune_argument_errors():
    lib = kp.lib()
    arr, n = kp._probs([_prob()])
    best = kp.kp_tuning()
    assert lib.kp_autotune(arr, n, None, 0, None, 4, None) == kp.KP_ERR_INVALID      # no output
    assert lib.kp_autotune(arr, n, None, 0, None, 1, ctypes.byref(best)) == kp.KP_ERR_INVALID   # iters < 2
    assert lib.kp_autotune(arr, 0, None, 0, None, 4, ctypes.byref(best)) == kp.KP_ERR_INVALID   # no problems
