"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every entry point that
include/ffbh.h declares, rejects bad parameters before touching a device, and its Morton code matches
the bit layout stated in the header (checked against an independent bit loop)."""
import os
import re

import numpy as np
import pytest

from paper_1212_2934_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ffbh.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const char \*\s*|bh_status\s+|int32_t\s+|uint64_t\s+|size_t\s+)(\w+)\s*\(",
                                 src, re.M)))


def test_every_declared_symbol_is_exported():
    L = binding.lib()
    names = _declared()
    assert "bh_field" in names and "md_step" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(binding.EXPORTED)


def test_workspace_bytes_validation():
    ok = binding.make_params(4096, 1, 16, 0.5, "fp64")
    assert binding.workspace_bytes(ok) > 0
    for bad in [dict(n=0), dict(batch=0), dict(leaf_size=0), dict(leaf_size=65), dict(theta=-0.1),
                dict(theta=float("nan")), dict(tuning_id=99)]:
        kw = dict(n=4096, batch=1, leaf_size=16, theta=0.5, precision="fp64")
        kw.update(bad)
        with pytest.raises(binding.BHError) as e:
            binding.workspace_bytes(binding.make_params(**kw))
        assert e.value.status == binding.BH_EINVAL


def test_create_rejects_missing_or_small_workspace():
    import ctypes as C
    L = binding.lib()
    p = binding.make_params(1000, 1, 16, 0.5, "fp32_mixed")
    h = C.c_void_p()
    assert L.bh_create(C.byref(p), None, 0, C.byref(h)) == binding.BH_EWORKSPACE
    assert L.bh_create(C.byref(p), C.c_void_p(256), 16, C.byref(h)) == binding.BH_EWORKSPACE
    assert L.bh_create(C.byref(p), C.c_void_p(257), 1 << 40, C.byref(h)) == binding.BH_EWORKSPACE
    assert L.bh_build(None, None, None) == binding.BH_EINVAL
    assert L.bh_field(None, None, None, None, None, None) == binding.BH_EINVAL


def test_caller_owned_handle_rejects_bad_memory_before_any_device_call():
    """bh_init checks the caller's handle memory, the parameters and the workspace before any HIP call;
    bh_fini and bh_destroy refuse null handles."""
    import ctypes as C
    L = binding.lib()
    hb = int(L.bh_handle_bytes())
    assert 0 < hb < 4096
    buf = (C.c_char * (hb + 64))()
    base = C.addressof(buf)
    mem = base + (-base) % 16
    p = binding.make_params(1000, 1, 16, 0.5, "fp32_mixed")
    ws = binding.workspace_bytes(p)
    h = C.c_void_p()
    EINVAL, EWS = binding.BH_EINVAL, binding.BH_EWORKSPACE
    assert L.bh_init(None, hb, C.byref(p), C.c_void_p(256), ws, None, C.byref(h)) == EINVAL
    assert L.bh_init(C.c_void_p(mem), hb - 1, C.byref(p), C.c_void_p(256), ws, None, C.byref(h)) == EINVAL
    assert L.bh_init(C.c_void_p(mem + 8), hb, C.byref(p), C.c_void_p(256), ws, None, C.byref(h)) == EINVAL
    bad = binding.make_params(0, 1, 16, 0.5, "fp32_mixed")
    assert L.bh_init(C.c_void_p(mem), hb, C.byref(bad), C.c_void_p(256), ws, None, C.byref(h)) == EINVAL
    assert L.bh_init(C.c_void_p(mem), hb, C.byref(p), C.c_void_p(256), ws, None, None) == EINVAL
    assert L.bh_init(C.c_void_p(mem), hb, C.byref(p), None, ws, None, C.byref(h)) == EWS
    assert L.bh_init(C.c_void_p(mem), hb, C.byref(p), C.c_void_p(257), ws, None, C.byref(h)) == EWS
    assert L.bh_init(C.c_void_p(mem), hb, C.byref(p), C.c_void_p(256), ws - 1, None, C.byref(h)) == EWS
    assert L.bh_fini(None) == EINVAL
    assert L.bh_destroy(None) == EINVAL


def test_workspace_grows_with_problem():
    a = binding.workspace_bytes(binding.make_params(1 << 12))
    b = binding.workspace_bytes(binding.make_params(1 << 16))
    c = binding.workspace_bytes(binding.make_params(1 << 12, batch=16))
    assert a < b and a < c


def _interleave_loop(qx, qy, qz):
    c = 0
    for k in range(21):
        c |= ((qx >> k) & 1) << (3 * k + 2)
        c |= ((qy >> k) & 1) << (3 * k + 1)
        c |= ((qz >> k) & 1) << (3 * k)
    return c


def test_morton_code_bit_layout():
    rng = np.random.default_rng(5)
    qs = rng.integers(0, 1 << 21, size=(200, 3))
    for qx, qy, qz in list(qs) + [(0, 0, 0), ((1 << 21) - 1,) * 3, (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        assert binding.morton_code(int(qx), int(qy), int(qz)) == _interleave_loop(int(qx), int(qy), int(qz))


def test_params_expansion_checked():
    """bh_params.expansion: 0 or 1 (the paper's cells) and 2 (with first moments) are valid, others not;
    order-2 cells keep their first moments in the workspace."""
    import ctypes as C
    L = binding.lib()
    out = C.c_size_t(0)
    sizes = {}
    for e in (0, 1, 2):
        p = binding.make_params(5000, 2, 16, 0.5, "fp64", -1, e)
        assert L.bh_workspace_bytes(C.byref(p), C.byref(out)) == 0
        sizes[e] = out.value
    assert sizes[0] == sizes[1] < sizes[2]
    for e in (-1, 3):
        p = binding.make_params(5000, 2, 16, 0.5, "fp64", -1, e)
        assert L.bh_workspace_bytes(C.byref(p), C.byref(out)) == -1


def test_allpairs_argument_checks():
    """Host-checkable errors return BH_EINVAL before anything is enqueued (no device needed).  Skipped
    where a GPU is present: the placeholder pointers must never reach a kernel."""
    import ctypes as C
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("host-only check")
    L = binding.lib()
    fake = C.c_void_p(4096)  # never dereferenced: every call below fails its checks first
    assert L.bh_allpairs(0, 1, 0, fake, fake, None, fake, None, None, None) == -1
    assert L.bh_allpairs(16, 0, 0, fake, fake, None, fake, None, None, None) == -1
    assert L.bh_allpairs(16, 70000, 0, fake, fake, None, fake, None, None, None) == -1
    assert L.bh_allpairs(16, 1, 7, fake, fake, None, fake, None, None, None) == -1
    assert L.bh_allpairs(16, 1, 0, None, fake, None, fake, None, None, None) == -1
    assert L.bh_allpairs(16, 1, 0, fake, fake, None, C.c_void_p(4097), None, None, None) == -1
