"""hu_pipeline_noalloc, the hu_pipeline variant for callers that cannot allocate device memory
(its workspace is a fixed device array of the library), through the C-ABI against hu_pipeline:

* two calls in a row, the second on a smaller input (so it runs over what the first left in the
  shared array), each equal to hu_pipeline on the same inputs: fields, sign maps, counts and
  statistics bit-identical, bin counts exact, bin sums within 1e-12 (FP64 atomics may add in
  another order);
* a shape whose workspace exceeds the array is refused (HU_ERR_WORKSPACE) and one whose tables
  were never built is refused (HU_ERR_TABLES), both before anything is enqueued.
"""

import math

import numpy as np
import pytest
import torch

from paper_2509_08675_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08675_amd import hufield
    return hufield


def _say(*a):
    print(*a, flush=True)


CALLS = [
    ((512, 512), (32, 12), W.filt(p=4, semi=(3, 1), rot=math.pi / 6, alpha=4, k0=0.2, width=0.04), [41, 42, 43, 44]),
    ((96, 64, 32), (24, 1), W.filt(p=6, semi=(1, 2, 3), rot=0.2, alpha=2, k0=0.15, width=0.05), [45]),
]


def test_noalloc_matches_pipeline_twice(hf):
    for dims, bins, filt, seeds in CALLS:
        _say("noalloc", dims, len(seeds), bins)
        ref = hf.PipelineBuffers(dims, len(seeds), bins)
        hf.pipeline(ref, filt, seeds)                       # allocating call: builds the tables
        got = hf.PipelineBuffers(dims, len(seeds), bins)
        for t in (got.field, got.cont_sum, got.pm1_sum):
            t.fill_(float("nan"))
        for t in (got.pm1, got.counts, got.cont_cnt, got.pm1_cnt):
            t.fill_(7)
        hf.pipeline_noalloc(got, filt, seeds)
        torch.cuda.synchronize()
        assert torch.equal(got.field, ref.field)
        assert torch.equal(got.pm1, ref.pm1)
        assert torch.equal(got.counts, ref.counts)
        assert torch.equal(got.stats, ref.stats)
        assert torch.equal(got.cont_cnt, ref.cont_cnt) and torch.equal(got.pm1_cnt, ref.pm1_cnt)
        for a, b in ((got.cont_sum, ref.cont_sum), (got.pm1_sum, ref.pm1_sum)):
            np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-12, atol=0.0)


def test_noalloc_refusals(hf):
    with pytest.raises(hf.HuError) as e:
        hf.pipeline_noalloc(hf.PipelineBuffers((2048, 2048), 9, (16, 1), want=("field",)), W.C2["filt"], list(range(9)))
    assert e.value.code == hf.HU_ERR_WORKSPACE
    fresh = hf.PipelineBuffers((24, 48), 1, (11, 3), want=("field", "pm1"))
    with pytest.raises(hf.HuError) as e:
        hf.pipeline_noalloc(fresh, W.C2["filt"], [1])
    assert e.value.code == hf.HU_ERR_TABLES
