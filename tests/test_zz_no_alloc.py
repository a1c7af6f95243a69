"""mi_hogbom_clean_noalloc (the CLEAN entry point that allocates nothing, working in the
library's fixed device scratch array) against mi_hogbom_clean, on two calls in a row, the
second with a smaller batch, and against the oracle's replay of its picks."""
import numpy as np
import pytest
import torch

from oracle import clean, imager
from paper_1712_06913_amd import synth
from tests.gpu_helpers import log, require_gpu

pytestmark = pytest.mark.gpu


def _maps(wl):
    d, b = [], []
    for i in range(wl.n_inst):
        v, uv, w = wl.instance(i)
        N, cell, mode = int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i])
        d.append(imager.dirty_image(v, uv, w, N, cell, mode).astype(np.float32))
        b.append(imager.dirty_beam(uv, w, N, cell, mode).astype(np.float32))
    return d, b


@pytest.mark.parametrize("restore_own_components", [False, True])
def test_noalloc_clean_matches_the_allocating_entry_point(restore_own_components):
    require_gpu()
    from paper_1712_06913_amd import api, _native as nat
    cases = [(synth.random_instances(91, [256, 256, 256], m_range=(200, 300)), [300, 150, 220]),
             (synth.random_instances(92, [128, 128], m_range=(100, 200)), [80, 120])]     # smaller second call
    for k, (wl, niter) in enumerate(cases):
        log(f"[no-alloc] call {k}: {wl.n_inst} x {int(wl.n_img[0])}^2, niter {niter}")
        niter = np.asarray(niter, np.int32)
        d, bm = _maps(wl)
        b = api.Batch.from_workload(wl)
        d_t = torch.from_numpy(np.concatenate([x.ravel() for x in d])).cuda()
        b_t = torch.from_numpy(np.concatenate([x.ravel() for x in bm])).cuda()
        ref = api.hogbom_clean(b, d_t, b_t, niter, restore=True)
        ref_status = b.status.clone()
        got = api.hogbom_clean(b, d_t, b_t, niter, restore=True, no_alloc=True,
                               want_components=not restore_own_components)
        torch.cuda.synchronize()
        assert torch.equal(b.status, ref_status)
        assert torch.equal(got["n_comp"], ref["n_comp"])
        # the same picks and the same fma sequence per pixel whatever the team shape
        assert torch.equal(got["residual"], ref["residual"])
        assert torch.equal(got["model"], ref["model"])
        assert torch.equal(got["cbeam"], ref["cbeam"])
        peak = float(d_t.abs().max())
        assert float((got["restored"] - ref["restored"]).abs().max()) <= 1e-6 * peak
        if not restore_own_components:
            assert torch.equal(got["comp_idx"], ref["comp_idx"]) and torch.equal(got["comp_flux"], ref["comp_flux"])
        ci, cf, off = ref["comp_idx"].cpu().numpy(), ref["comp_flux"].cpu().numpy(), ref["comp_off"]
        res = b.split(got["residual"])
        for i in range(wl.n_inst):
            n = int(got["n_comp"][i])
            ok, bad, R, _ = clean.replay(d[i].astype(np.float64), bm[i].astype(np.float64), ci[off[i]: off[i] + n],
                                         cf[off[i]: off[i] + n])
            assert ok, f"call {k} inst {i}: pick {bad} rejected"
            assert np.max(np.abs(res[i].cpu().numpy() - R)) <= 1e-4 * np.max(np.abs(d[i]))
    # sizes beyond the scratch array's limits are rejected before any launch
    wl = synth.random_instances(93, [64, 128], m_range=(50, 60))
    d, bm = _maps(wl)
    b = api.Batch.from_workload(wl)
    d_t = torch.from_numpy(np.concatenate([x.ravel() for x in d])).cuda()
    b_t = torch.from_numpy(np.concatenate([x.ravel() for x in bm])).cuda()
    with pytest.raises(nat.MiError):
        api.hogbom_clean(b, d_t, b_t, [10, 10], no_alloc=True)          # two image sizes
    wl = synth.random_instances(94, [256], m_range=(50, 60))
    d, bm = _maps(wl)
    b = api.Batch.from_workload(wl)
    with pytest.raises(nat.MiError):                                    # component lists beyond 8 MiB
        api.hogbom_clean(b, torch.from_numpy(d[0].ravel()).cuda(), torch.from_numpy(bm[0].ravel()).cuda(),
                         [2_000_000], no_alloc=True, want_components=False, want_model=False)
