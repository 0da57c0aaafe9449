"""The C ABI on a host without a GPU: the library loads, exports every entry
point include/sten4.h declares, and rejects bad arguments with the documented
codes before any device call."""
import ctypes
import os
import re

import pytest

import paper_1308_1343_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "sten4.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(s4_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared()
    assert len(names) >= 15
    L = S.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(S.EXPORTS) == names


def good_box(n=(8, 9, 10), g=2):
    return S.make_box(n, g, (1, n[0] + 2 * g, (n[0] + 2 * g) * (n[1] + 2 * g)), (0.1, 0.1, 0.1))


def test_check_boxes_codes():
    assert S.s4_check_boxes(good_box(), S.S4_OP_RK4) == S.S4_OK
    b = good_box(); b.n[1] = 0
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_EINVAL
    b = good_box(); b.ghost = 1
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_EGHOST
    b = good_box(); b.stride[0] = 2
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_ELAYOUT
    b = good_box(); b.stride[1] = 11
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_ELAYOUT
    b = good_box(); b.stride[2] = b.stride[1] * 12
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_ELAYOUT
    b = good_box(); b.dx[2] = 0.0
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_EINVAL
    b = good_box(); b.dx[0] = float("nan")
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_EINVAL
    b = good_box((2, 8, 8), 3)
    assert S.s4_check_boxes(b, S.S4_OP_FILL) == S.S4_EGHOST
    assert S.s4_check_boxes(b, S.S4_OP_WAVE_RHS) == S.S4_OK
    assert S.s4_check_boxes([good_box(), good_box()], S.S4_OP_ADJOINT_STEP) == S.S4_EINVAL
    assert S.s4_check_boxes(good_box(), 99) == S.S4_EINVAL
    assert "op" in S.s4_last_error()
    assert S.lib().s4_check_boxes(None, 1, S.S4_OP_RK4) == S.S4_EINVAL
    arr = (S.S4Box * 1)(good_box())
    assert S.lib().s4_check_boxes(arr, 0, S.S4_OP_RK4) == S.S4_EINVAL


def test_workspace_sizes():
    b = good_box()
    field = ((12 * 13 * 14 * 8 + 255) // 256) * 256
    ws = S.s4_workspace_size(b, S.S4_OP_RK4, S.S4_GRAPH)
    assert ws >= 6 * field
    assert S.s4_workspace_size([b, b, b], S.S4_OP_RK4, S.S4_BATCHED) >= 18 * field
    assert S.s4_workspace_size(b, S.S4_OP_ADJOINT_STEP) >= 6 * 12 * 13 * 14 * 8
    assert S.s4_workspace_size(b, S.S4_OP_WAVE_RHS) == 0
    with pytest.raises(S.Sten4Error) as e:
        S.s4_workspace_size(b, S.S4_OP_RK4, 7)
    assert e.value.code == S.S4_EINVAL


def test_entry_points_reject_null_context():
    L = S.lib()
    arr = (S.S4Box * 1)(good_box())
    p = (ctypes.c_void_p * 1)(256)
    assert L.s4_wave_rhs(None, arr, 1, p, None, p, None) == S.S4_EINVAL
    assert L.s4_fill_ghosts_periodic(None, arr, 1, p, None) == S.S4_EINVAL
    assert L.s4_rk4(None, arr, 1, p, p, None, 0.1, 1, 0, None, 0, None) == S.S4_EINVAL
    assert L.s4_rk4_adjoint_step(None, arr, None, None, None, 0.1, None, None, None, None, 0, None) == S.S4_EINVAL
    assert L.s4_rk4_step_to_y3(None, arr, p, p, None, 0.1, p, p, p, p, p, 1 << 20, None) == S.S4_EINVAL
    assert L.s4_rk4_step_to_y3(None, arr, p, p, None, 0.1, p, p, None, p, p, 1 << 20, None) == S.S4_EINVAL
    assert L.s4_rk4_adjoint_step_y3(None, arr, p, p, p, p, None, 0.1, p, p, None, p, 1 << 20, None) == S.S4_EINVAL
    # with c2_bar the stage state is required
    assert L.s4_rk4_adjoint_step_y3(None, arr, p, p, None, None, None, 0.1, p, p, p, p, 1 << 20, None) == \
        S.S4_EINVAL
    assert "u3" in S.s4_last_error()
    assert L.s4_copy(None, None, None, 16, None) == S.S4_EINVAL
    assert L.s4_tune(None, S.S4_OP_RK4, arr, 1, 0, None, 0, None) == S.S4_EINVAL
    out = (ctypes.c_int * 8)()
    assert L.s4_get_choice(None, S.S4_OP_RK4, arr, 1, out) == S.S4_EINVAL


def test_with_c2_modifier_on_tune_scratch():
    # one more field (the c^2 the timed step reads) per box; RK4 only
    b = good_box((16, 16, 16), 2)
    field = 8 * (16 + 4) * (16 + 4) * (16 + 4)
    plain = S.s4_tune_scratch_size(b, S.S4_OP_RK4)
    withc = S.s4_tune_scratch_size(b, S.S4_OP_RK4 | S.S4_WITH_C2)
    assert withc - plain >= field
    two = S.s4_tune_scratch_size([b, b], S.S4_OP_RK4 | S.S4_WITH_C2) - S.s4_tune_scratch_size([b, b], S.S4_OP_RK4)
    assert two == 2 * (withc - plain)
    with pytest.raises(S.Sten4Error):
        S.s4_tune_scratch_size(b, S.S4_OP_WAVE_RHS | S.S4_WITH_C2)
    assert "S4_WITH_C2" in S.s4_last_error()
