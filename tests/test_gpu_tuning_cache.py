"""The autotuner's tuning cache (vk_autotune_cached): a miss tunes and appends, a hit restores the
same launch shapes for the same problem on the same device, other problems keep their own lines,
and the results stay bitwise those of the tuned hierarchy."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tuning_cache_miss_then_hit(tmp_path):
    import paper_2409_14222_amd as vk
    path = str(tmp_path / "vk_tuning.txt")
    H = vk.Hierarchy(2, 4, 3).bind().setup()
    t1 = H.autotune(reps=2, cache=path)
    assert not H.tuning_cache_hit
    lines = open(path).read().splitlines()
    assert len(lines) == 3
    N = H.level_info(2).n_free
    r = torch.tensor(synth.vector(N, 42), device="cuda")
    e1 = torch.empty_like(r)
    H.vcycle(r, e1, 2, 2)
    H2 = vk.Hierarchy(2, 4, 3).bind().setup()
    t2 = H2.autotune(reps=2, cache=path)
    assert H2.tuning_cache_hit and t2 == t1
    e2 = torch.empty_like(r)
    H2.vcycle(r, e2, 2, 2)
    torch.cuda.synchronize()
    assert torch.equal(e1, e2)
    # another problem (other order) misses and appends its own lines; the first key still hits
    H3 = vk.Hierarchy(3, 4, 3).bind().setup()
    H3.autotune(reps=2, cache=path)
    assert not H3.tuning_cache_hit
    assert len(open(path).read().splitlines()) == 6
    H4 = vk.Hierarchy(2, 4, 3).bind().setup()
    H4.autotune(reps=2, cache=path)
    assert H4.tuning_cache_hit
