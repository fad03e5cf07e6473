"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/srot.h declares, and rejects bad arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srot.h")
LIB = os.path.join(ROOT, "paper_2103_05857_amd", "libsrot.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srot_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsrot.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"srot_init", "srot_step", "srot_gap", "srot_solve"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_default_options_and_workspace_size():
    from paper_2103_05857_amd import srot as S
    opt = S.srot_default_options()
    assert opt.w == 1.0 and opt.step_rule == S.SROT_ELS and opt.sampling == S.SROT_UNIFORM
    assert opt.eps == 1e-6 and opt.max_passes == 1000 and opt.gap_every == 1
    ws = S.srot_workspace_size(4096, 4096, opt)
    # dense FP64 plan dominates: 128 MiB plus support masks and small buffers
    assert 4096 * 4096 * 8 < ws < 4096 * 4096 * 8 + (16 << 20)
    assert ws % 256 == 0
    assert S.srot_workspace_size(0, 5, opt) == 0
    assert S.srot_workspace_size(5, -1, opt) == 0
    assert S.srot_workspace_size(3, 1, opt) > 0


def test_init_rejects_bad_arguments_on_host():
    from paper_2103_05857_amd import srot as S
    L = S.load()
    opt = S.srot_default_options()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(256)  # never dereferenced: checks fail first
    # m = 0
    assert L.srot_init(ctypes.byref(h), 0, 4, fake, None, None, fake, fake, fake, 1 << 20,
                       ctypes.byref(opt), None) == S.SROT_EINVAL
    # missing a
    assert L.srot_init(ctypes.byref(h), 4, 4, fake, None, None, None, fake, fake, 1 << 20,
                       ctypes.byref(opt), None) == S.SROT_EINVAL
    # stored cost without C
    assert L.srot_init(ctypes.byref(h), 4, 4, None, None, None, fake, fake, fake, 1 << 20,
                       ctypes.byref(opt), None) == S.SROT_EINVAL
    # fused cost without points
    o2 = S.srot_default_options(cost=S.SROT_COST_SQEUCLID)
    assert L.srot_init(ctypes.byref(h), 4, 4, None, None, None, fake, fake, fake, 1 << 20,
                       ctypes.byref(o2), None) == S.SROT_EINVAL
    # negative penalty weight, bad step rule, gap_every 0
    for bad in (dict(w=-1.0), dict(step_rule=7), dict(gap_every=0), dict(cost=9)):
        ob = S.srot_default_options(**bad)
        assert L.srot_init(ctypes.byref(h), 4, 4, fake, None, None, fake, fake, fake, 1 << 20,
                           ctypes.byref(ob), None) == S.SROT_EINVAL
    # unaligned workspace
    assert L.srot_init(ctypes.byref(h), 4, 4, fake, None, None, fake, fake, ctypes.c_void_p(264),
                       1 << 20, ctypes.byref(opt), None) == S.SROT_EINVAL
    # workspace too small
    assert L.srot_init(ctypes.byref(h), 64, 64, fake, None, None, fake, fake, fake, 1024,
                       ctypes.byref(opt), None) == S.SROT_ENOMEM
    assert b"workspace" in L.srot_last_error()
    assert h.value is None


def test_null_handle_is_rejected():
    from paper_2103_05857_amd import srot as S
    L = S.load()
    assert L.srot_step(None, 4, None, None, None) == S.SROT_EINVAL
    out = (ctypes.c_double * 3)()
    assert L.srot_gap(None, out, None, None) == S.SROT_EINVAL
    passes = ctypes.c_int64()
    assert L.srot_step_ga(None, 4, None, None, None, None, None) == S.SROT_EINVAL
    assert L.srot_solve_ga(None, 0.0, 1, out, ctypes.byref(passes)) == S.SROT_EINVAL
    assert L.srot_ga_reset(None, 1.0) == S.SROT_EINVAL
    assert L.srot_ga_refresh(None) == S.SROT_EINVAL
    assert L.srot_ga_weights(None, None) == S.SROT_EINVAL
    stats = (ctypes.c_int64 * 4)()
    assert L.srot_chain_stats(None, stats) == S.SROT_EINVAL
    assert L.srot_backward(None, 1.0, None, None, None, None, None) == S.SROT_EINVAL
    assert L.srot_backward_noalloc(None, 1.0, None, None, None, None, None) == S.SROT_EINVAL
    nnz = ctypes.c_int64()
    assert L.srot_get_plan_csr(None, None, None, None, 0, ctypes.byref(nnz)) == S.SROT_EINVAL
    assert L.srot_strerror(S.SROT_ECAPACITY) == b"output buffer too small"
    assert L.srot_strerror(S.SROT_ENONFINITE) == b"non-finite or negative input"


def test_binding_refuses_host_and_mistyped_tensors():
    """Every tensor handed to the library is dereferenced on the GPU, so the
    binding refuses host tensors, wrong dtypes, short and non-contiguous
    tensors before any call reaches the library."""
    import torch
    from paper_2103_05857_amd import srot as S
    with pytest.raises(S.SrotError):
        S._ptr(torch.zeros(4, dtype=torch.int32))                 # host memory
    with pytest.raises(S.SrotError):
        S.srot_step(None, 4, torch.zeros(4, dtype=torch.int32))
    with pytest.raises(S.SrotError):
        S._ptr([1, 2, 3])
    assert S._ptr(None) is None
