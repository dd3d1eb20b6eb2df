"""gpbo_topk_noalloc through the C ABI: the same indices as gpbo_topk on two
calls in a row (the second with a smaller input, so stale scratch contents
from the first would show), and no device allocation through the context's
allocator or torch's during the calls."""
import numpy as np
import pytest
import torch

from paper_2403_08131_amd import gpbo as G

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def test_topk_noalloc_matches_topk_without_allocating():
    # the context hands torch's caching allocator to the library, so every
    # device allocation of the library is a torch allocation and shows in
    # torch's cumulative allocation count
    ctx = G.Context(0)
    r = np.random.default_rng(7)
    cases = [(1 << 20, 4096), (70001, 333)]  # second call: smaller m and k
    inputs = []
    for m, k in cases:
        v = np.round(r.normal(size=m), 2).astype(np.float32)  # many exact ties
        v[r.integers(0, m, 3)] = np.nan
        inputs.append((torch.tensor(v, device=DEV), k))
    outs = [torch.empty(k, dtype=torch.int64, device=DEV) for _, k in inputs]
    torch.cuda.synchronize()
    count = lambda: torch.cuda.memory_stats(DEV)["allocation.all.allocated"]
    before_count = count()
    before_bytes = torch.cuda.memory_allocated(DEV)
    for (v, k), o in zip(inputs, outs):
        G.topk_noalloc(ctx, v, k, idx=o)
    torch.cuda.synchronize()
    assert count() == before_count
    assert torch.cuda.memory_allocated(DEV) == before_bytes
    for (v, k), o in zip(inputs, outs):
        ref = G.topk(ctx, v, k)
        torch.cuda.synchronize()
        assert torch.equal(o, ref), (v.shape[0], k)
        vv = v.double().cpu().numpy()
        vv = np.where(np.isnan(vv), -np.inf, vv)
        want = np.lexsort((np.arange(vv.size), -vv))[:k]
        assert np.array_equal(o.cpu().numpy(), want)
    # the same sizes again in the opposite order
    for (v, k), o in reversed(list(zip(inputs, outs))):
        again = G.topk_noalloc(ctx, v, k)
        torch.cuda.synchronize()
        assert torch.equal(again, o)
    with pytest.raises(G.GpboError) as e:
        G.topk_noalloc(ctx, inputs[0][0], 8193)
    assert e.value.status == G.E_UNSUPPORTED
    ctx.close()
