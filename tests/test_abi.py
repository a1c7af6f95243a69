"""The C-ABI library: every symbol declared in include/mi.h is exported (CPU), and every entry
point rejects bad arguments with the documented code before launching anything (GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1712_06913_amd", "libmi.so")


def _declared():
    text = open(os.path.join(ROOT, "include", "mi.h")).read()
    return sorted(set(re.findall(r"\b(mi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_six_hot_path_calls():
    names = _declared()
    for n in ("mi_grid", "mi_ifft2", "mi_dirty_image", "mi_dirty_beam", "mi_hogbom_clean", "mi_degrid"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libmi.so not built")
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_1712_06913_amd import _native
    assert set(_native.EXPORTS) == set(_declared())
    lib.mi_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.mi_version()


@pytest.mark.gpu
def test_bad_arguments_are_rejected_and_write_nothing():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06913_amd import api, _native as nat
    from paper_1712_06913_amd import synth
    wl = synth.random_instances(5, [64], m_range=(10, 10))
    vis, uv, w = api.workload_tensors(wl)
    sentinel = torch.full((64 * 64,), 7.0, device="cuda")

    def expect(code, **kw):
        b = api.Batch(kw.get("off", wl.vis_offset), kw.get("n", wl.n_img), kw.get("cell", wl.cell_rad),
                      kw.get("mode", wl.weight_mode))
        with pytest.raises(nat.MiError) as e:
            api.dirty_image(b, vis, uv, w, beam=False, out=sentinel)
        assert e.value.code == code
        torch.cuda.synchronize()
        assert torch.all(sentinel == 7.0)

    expect(nat.MI_ERR_SHAPE, n=np.array([100], np.int32))
    expect(nat.MI_ERR_SHAPE, n=np.array([32], np.int32))
    expect(nat.MI_ERR_ARG, cell=np.array([-1.0]))
    expect(nat.MI_ERR_ARG, mode=np.array([3], np.int8))
    expect(nat.MI_ERR_SHAPE, off=np.array([1, 10], np.int64))
    b = api.Batch.from_workload(wl)
    with pytest.raises(nat.MiError) as e:
        api.hogbom_clean(b, sentinel, torch.zeros(4 * 64 * 64, device="cuda"), [10], gain=1.5)
    assert e.value.code == nat.MI_ERR_ARG
    with pytest.raises(nat.MiError) as e:
        api.ifft2(torch.zeros(100, dtype=torch.complex64, device="cuda"), [10], [0])
    assert e.value.code == nat.MI_ERR_SHAPE
    with pytest.raises(nat.MiError) as e:
        api.steer_clean(b, sentinel, torch.zeros(4 * 64 * 64, device="cuda"), [10], trim=0.0)
    assert e.value.code == nat.MI_ERR_ARG
    with pytest.raises(nat.MiError) as e:
        api.hogbom_clean(b, sentinel, torch.zeros(4 * 64 * 64, device="cuda"), [10], no_alloc=True,
                         window=np.array([[0, 0, 8, 8]], np.int32))
    assert e.value.code == nat.MI_ERR_UNSUPPORTED
    with pytest.raises(nat.MiError) as e:
        api.set_tuning(b.ctx, 64, 0)
    assert e.value.code == nat.MI_ERR_ARG
    torch.cuda.synchronize()
    assert torch.all(sentinel == 7.0)
