"""The C ABI on the CPU: the library loads, exports every symbol swept.h declares,
and validates arguments (no HIP call happens before validation finishes)."""
import ctypes
import os
import re

import pytest

from paper_2105_10332_amd import _lib
from paper_2105_10332_amd._lib import CODES, Problem, Tuning

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "swept.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char\*)\s+(\w+)\s*\(", text)))


def test_library_exports_all_declared_symbols():
    L = _lib.lib()
    names = declared_functions()
    assert "swept_advance" in names and "standard_advance" in names and len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def _ws(p, tile=0, wg=0):
    out = ctypes.c_size_t(0)
    rc = _lib.lib().swept_workspace_bytes(ctypes.byref(p), ctypes.byref(Tuning(tile, wg)), ctypes.byref(out))
    return rc, out.value


def heat(n=64, r=0.2, dtype=0):
    dx = 1.0 / n
    return Problem(0, dtype, n, n, 1.0, 1.0, r * dx * dx, 1.0, 1.4)


def euler(n=64, dtype=0):
    return Problem(1, dtype, n, n, 10.0, 10.0, 1e-3, 0.0, 1.4)


def test_workspace_size():
    rc, b = _ws(heat(64), 16)
    assert rc == 0 and b >= 64 * 64 * 8
    rc, b32 = _ws(heat(64, dtype=1), 16)
    assert rc == 0 and b32 >= 64 * 64 * 4 and b32 < b
    rc, be = _ws(euler(64), 16)
    assert rc == 0 and be >= 4 * 64 * 64 * 8


@pytest.mark.parametrize("prob,tile,wg,code", [
    (Problem(0, 0, 64, 32, 1.0, 1.0, 1e-5, 1.0, 1.4), 16, 0, "SWEPT_ESHAPE"),      # not square
    (heat(64), 12, 0, "SWEPT_ESHAPE"),                                             # 64 % 12
    (heat(64), 2, 0, "SWEPT_ESHAPE"),                                              # b = 2n
    (heat(64), 7, 0, "SWEPT_ESHAPE"),                                              # b % 2n
    (heat(64), 64, 0, "SWEPT_ESHAPE"),                                             # N < 2b
    (euler(64), 6, 0, "SWEPT_ESHAPE"),                                             # Euler b % 4
    (euler(256, dtype=0), 64, 0, "SWEPT_ESHAPE"),                                  # FP64 Euler b=64: LDS
    (heat(64, r=0.26), 16, 0, "SWEPT_EUNSTABLE"),                                  # 4r > 1
    (Problem(0, 0, 64, 64, 1.0, 1.0, -1.0, 1.0, 1.4), 16, 0, "SWEPT_EUNSTABLE"),   # dt <= 0
    (Problem(2, 0, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4), 16, 0, "SWEPT_EINVAL"),      # kind
    (Problem(0, 5, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4), 16, 0, "SWEPT_EINVAL"),      # dtype
    (Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 0.9), 16, 0, "SWEPT_EINVAL"),    # gamma <= 1
    (heat(64), 16, 100, "SWEPT_EINVAL"),                                           # wg not multiple of 64
    (euler(64), 16, 1088, "SWEPT_EINVAL"),                                         # wg > 1024
    (Problem(0, 0, 0, 0, 1.0, 1.0, 1e-5, 1.0, 1.4), 16, 0, "SWEPT_ESHAPE"),        # empty
    (Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, 4), 16, 0, "SWEPT_EINVAL"),  # unknown scheme bit
    (Problem(0, 0, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4, 1), 16, 0, "SWEPT_EINVAL"),    # heat has no variants
    (Problem(0, 0, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4, 0, 3), 16, 0, "SWEPT_EINVAL"),    # unknown boundary
    (Problem(0, 0, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4, 0, 1, float("nan")), 16, 0, "SWEPT_EINVAL"),  # NaN ghost
    (Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, 0, 1), 16, 0, "SWEPT_ENOTSUP"),  # Euler Dirichlet
    (Problem(0, 0, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4, 0, 3), 16, 0, "SWEPT_EINVAL"),    # heat slip wall
    (Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, 0, 4), 16, 0, "SWEPT_EINVAL"),  # unknown boundary
])
def test_validation_codes(prob, tile, wg, code):
    rc, _ = _ws(prob, tile, wg)
    assert rc == CODES[code], (rc, _lib.last_error())
    assert _lib.last_error()


def test_euler_lds_limits():
    """Euler keeps two state windows, a pressure plane and a face buffer in LDS:
    FP64 fits up to b = 32, FP32 b = 64 does not."""
    assert _ws(euler(256, dtype=0), 32)[0] == 0
    assert _ws(euler(256, dtype=1), 32)[0] == 0
    assert _ws(euler(256, dtype=1), 64)[0] == CODES["SWEPT_ESHAPE"]


def test_init_rejects_bad_pointers_and_small_workspace():
    L = _lib.lib()
    ctx = ctypes.c_void_p(0)
    p = heat(64)
    t = Tuning(16, 0)
    _, need = _ws(p, 16)
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first
    assert L.swept_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(t), None, fake, need, None) == CODES["SWEPT_EINVAL"]
    assert L.swept_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(t), fake, None, need, None) == CODES["SWEPT_EINVAL"]
    assert L.swept_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(t), fake, fake, need - 1, None) == \
        CODES["SWEPT_EWORKSPACE"]
    assert L.swept_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(t), ctypes.c_void_p(0x10004), fake, need,
                        None) == CODES["SWEPT_EINVAL"]
    assert ctx.value is None
    assert L.swept_advance(None, 5) == CODES["SWEPT_EINVAL"]
    assert L.standard_advance(None, 5) == CODES["SWEPT_EINVAL"]


def test_cfl_rejects_heat():
    L = _lib.lib()
    out = ctypes.c_double()
    fake = ctypes.c_void_p(0x10000)
    p = heat(64)
    assert L.swept_cfl_dt(ctypes.byref(p), fake, 0.4, fake, 1 << 30, None, ctypes.byref(out)) == CODES["SWEPT_ENOTSUP"]


def test_batch_tiles_follow_preferences():
    """Each problem of a batch takes the largest valid tile not above its kind's preference
    (the library's own validation decides validity)."""
    from paper_2105_10332_amd import tune

    specs = [("heat", 1024), ("heat", 160), ("heat", 96), ("euler", 512), ("euler", 288)]
    got = tune.batch_tiles(specs, "f32", {"heat": 64, "euler": 32})
    assert got == [64, 32, 48, 32, 32]
    got = tune.batch_tiles(specs, "f32", {"heat": 16, "euler": 16})
    assert got == [16, 16, 16, 16, 16]


def test_batch_count_and_dtype_validation():
    """A batch takes 1..256 problems of one dtype; anything else is rejected before any HIP call."""
    L = _lib.lib()
    out = ctypes.c_size_t(0)
    probs = (Problem * 257)(*[heat(32) for _ in range(257)])
    assert L.swept_batch_workspace_bytes(probs, None, 256, ctypes.byref(out)) == 0 and out.value > 0
    assert L.swept_batch_workspace_bytes(probs, None, 257, ctypes.byref(out)) == CODES["SWEPT_EINVAL"]
    assert L.swept_batch_workspace_bytes(probs, None, 0, ctypes.byref(out)) == CODES["SWEPT_EINVAL"]
    mixed = (Problem * 2)(heat(32, dtype=0), heat(32, dtype=1))
    assert L.swept_batch_workspace_bytes(mixed, None, 2, ctypes.byref(out)) == CODES["SWEPT_EINVAL"]
    variant = (Problem * 2)(heat(32), Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, 3))
    assert L.swept_batch_workspace_bytes(variant, None, 2, ctypes.byref(out)) == 0  # variants batch too
    for scheme in (1, 2, 3):  # the single-problem path takes every variant
        assert _ws(Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, scheme), 16)[0] == 0
    ewall = (Problem * 1)(Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, 0, 3))
    assert L.swept_batch_workspace_bytes(ewall, None, 1, ctypes.byref(out)) == CODES["SWEPT_ENOTSUP"]
    for bc in (2, 3):  # the single-problem Euler path takes zero-gradient and slip walls
        assert _ws(Problem(1, 0, 64, 64, 10.0, 10.0, 1e-3, 0.0, 1.4, 0, bc), 16)[0] == 0
    walls = (Problem * 1)(Problem(0, 0, 32, 32, 1.0, 1.0, 1e-4, 1.0, 1.4, 0, 1, 0.5))
    assert L.swept_batch_workspace_bytes(walls, None, 1, ctypes.byref(out)) == 0  # walls batch too
    for bc in (1, 2):  # the single-problem heat path takes both
        assert _ws(Problem(0, 0, 64, 64, 1.0, 1.0, 1e-5, 1.0, 1.4, 0, bc, 0.25), 16)[0] == 0


def test_batch_mode_validation():
    """swept_batch_set_mode checks its context before anything else."""
    L = _lib.lib()
    for mode in (0, 1, 2, -1):
        assert L.swept_batch_set_mode(None, mode) == CODES["SWEPT_EINVAL"]
    assert _lib.BATCH_COOPERATIVE == 0 and _lib.BATCH_PER_PHASE == 1
