"""The allocation-free smoothing entry point (vk_smooth_noalloc) against vk_smooth, through the C ABI.

Both run the same kernels in the same order on the same inputs, so the results must be bitwise
equal.  Three calls in a row share the library's fixed per-device scratch: a large input first,
then smaller ones (the array keeps the previous call's contents, which must not matter).
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_smooth_equals_smooth_on_successive_calls():
    import paper_2409_14222_amd as vk
    cases = [  # (k, n0, levels, level, store, smoother, weighting): largest input first
        (4, 4, 3, 2, vk.VK_STORE_FP64, vk.VK_SMOOTH_DAMPED, vk.VK_WEIGHT_MULTIPLICITY),   # N = 10,339
        (2, 4, 3, 1, vk.VK_STORE_FP64, vk.VK_SMOOTH_DAMPED, vk.VK_WEIGHT_MULTIPLICITY),   # N = 531
        (3, 2, 3, 1, vk.VK_STORE_FP32, vk.VK_SMOOTH_CHEBYSHEV, vk.VK_WEIGHT_NONE),        # N = 327, FP32
    ]
    for i, (k, n0, nl, level, store, sm, w) in enumerate(cases):
        print(f"[gpu-noalloc] call {i}: P{k}-P{k - 1} level {level} store {store} smoother {sm}", flush=True)
        H = vk.Hierarchy(k, n0, nl, store=store, smoother=sm, weighting=w).bind().setup()
        N = H.level_info(level).n_free
        b = torch.tensor(synth.vector(N, 50 + i), device="cuda")
        x0 = synth.vector(N, 60 + i)
        x_ref = torch.tensor(x0, device="cuda")
        x_new = torch.tensor(x0, device="cuda")
        assert vk.lib.vk_smooth(H.h, level, b.data_ptr(), x_ref.data_ptr(), 3) == vk.VK_OK
        st = vk.lib.vk_smooth_noalloc(H.h, level, b.data_ptr(), x_new.data_ptr(), 3)
        assert st == vk.VK_OK, vk.lib.vk_last_error()
        torch.cuda.synchronize()
        assert not torch.equal(x_new, torch.tensor(x0, device="cuda"))
        assert torch.equal(x_new, x_ref), i
        # the hierarchy's own buffers are untouched by the call: vk_smooth still gives the same bits
        x_again = torch.tensor(x0, device="cuda")
        assert vk.lib.vk_smooth(H.h, level, b.data_ptr(), x_again.data_ptr(), 3) == vk.VK_OK
        torch.cuda.synchronize()
        assert torch.equal(x_again, x_ref)
