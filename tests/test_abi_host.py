"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/epic.h declares, rejects bad configurations before any
device work, and the workgroup partition used by the kernels is exact."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1904_11422_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epic.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(epic_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_config_struct_layout_matches_header():
    assert ctypes.sizeof(_lib.EpicConfig) == 48
    assert _lib.EpicConfig.kernel_sigma_cells.offset == 24
    assert _lib.EpicConfig.flags.offset == 44


def _init(cfg):
    L = _lib.load()
    ctx = ctypes.c_void_p()
    st = L.epic_init(ctypes.byref(cfg) if cfg is not None else None, 0, None, ctypes.byref(ctx))
    return st, ctx, L.epic_last_error(None).decode()


@pytest.mark.parametrize("field,value", [("grid_n", 48), ("grid_n", 256), ("n_pol", 3),
                                         ("n_ant", 0), ("n_chan", 0), ("kernel_support", 4),
                                         ("kernel_support", 17), ("kernel_sigma_cells", 0.0),
                                         ("cell_wavelengths", -0.5), ("precision", 5),
                                         ("flags", 64)])
def test_init_rejects_bad_config(field, value):
    cfg = _lib.EpicConfig(64, 4, 2, 256, 3, 0.5, 0.5, 0, 0)
    setattr(cfg, field, value)
    st, ctx, msg = _init(cfg)
    assert st == _lib.EPIC_E_INVALID
    assert ctx.value is None and msg


def test_init_null_config_and_null_out():
    L = _lib.load()
    ctx = ctypes.c_void_p()
    assert L.epic_init(None, 0, None, ctypes.byref(ctx)) == _lib.EPIC_E_INVALID
    cfg = _lib.EpicConfig(64, 4, 2, 256, 3, 0.5, 0.5, 0, 0)
    assert L.epic_init(ctypes.byref(cfg), 0, None, None) == _lib.EPIC_E_INVALID


def test_calls_on_null_context_are_rejected():
    L = _lib.load()
    assert L.epic_set_antennas(None, None, None) == _lib.EPIC_E_INVALID
    assert L.epic_image_accumulate(None, None, 1, None, None, 1) == _lib.EPIC_E_INVALID
    assert L.epic_image_backward(None, None, 1, None, None, None) == _lib.EPIC_E_INVALID
    assert L.epic_timing_history(None, 1, None) == _lib.EPIC_E_INVALID
    L.epic_destroy(None)
    assert L.epic_last_kernel_name(None) == b"none"


# The kernels split the flattened (channel, time) space into W contiguous
# ranges [w*total/W, (w+1)*total/W); the reducers find the workgroups of
# channel c with owner(f) = ceil((f+1) W / total) - 1 and store the partial of
# (w, c) in slot w + c.  Checked here by brute force.
def _begin(w, total, W):
    return (w * total) // W


def _owner(f, total, W):
    return ((f + 1) * W + total - 1) // total - 1


@pytest.mark.parametrize("C,T,W", [(1, 1, 1), (132, 1000, 256), (132, 1000, 512), (3, 7, 16),
                                   (5, 1, 8), (264, 200, 256), (16, 100000, 256), (2, 3, 6),
                                   (7, 13, 91)])
def test_partition_owner_and_slots(C, T, W):
    total = C * T
    W = min(W, total)
    starts = np.array([_begin(w, total, W) for w in range(W + 1)])
    assert starts[0] == 0 and starts[-1] == total
    assert np.all(np.diff(starts) >= 1)                  # W <= total: no empty range
    f = np.arange(total)
    own = np.searchsorted(starts, f, side="right") - 1
    for x in np.unique(np.r_[f[:50], f[-50:], np.random.default_rng(0).choice(f, 200)]):
        assert _owner(int(x), total, W) == own[x]
    slots = set()
    for w in range(W):
        cs = range(starts[w] // T, (starts[w + 1] - 1) // T + 1)
        for c in cs:
            assert (w + c) not in slots
            slots.add(w + c)
    assert max(slots) <= W + C - 2
