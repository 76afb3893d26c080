"""GPU tests of heterogeneous batches (one captured graph) and of the plan autotuner.

* every field of an uneven batch equals the same field generated alone (field and sign map
  bit-identical: the per-column arithmetic does not depend on the batch), and sampled fields
  match the FP64 oracle to the parity tolerances;
* the cached graph replays correctly several times in a row with other GPU work in between,
  for new seeds each time;
* an invalid job gets its error status and does not disturb the others;
* the half-width tile variants with every schedule switched give the same fields as the default
  plan and match the oracle;
* the autotuner writes a plan the library then reports;
* the full uneven 512-field batch in the benchmark's launch configuration: one field of every
  shape class (64^2 .. 1024^2, 64^3 .. 128^3) against the oracle to the parity tolerances.
"""

import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2509_08675_amd import workloads as W

import _parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08675_amd import hufield
    return hufield


def _say(*a):
    print(*a, flush=True)


def mixed_jobs(seed0=100):
    rng = np.random.default_rng(3)
    shapes = [((64, 64), (16, 1)), ((64, 64), (16, 1)), ((128, 128), (32, 6)), ((96, 64), (24, 4)),
              ((32, 48), (12, 1)), ((16, 16, 16), (16, 1)), ((16, 16, 16), (16, 1)), ((12, 24, 32), (16, 1)),
              ((24, 24, 24), (20, 1)), ((64, 64), None), ((8, 8), (4, 1)), ((48, 24, 12), (12, 1))]
    jobs = []
    for i, (dims, bins) in enumerate(shapes):
        k0 = float(rng.uniform(0.15, 0.35))
        f = W.filt(p=float(rng.uniform(1.5, 8)), semi=(float(rng.uniform(1, 3)), 1.0, 1.0),
                   rot=float(rng.uniform(0, math.pi)), alpha=float(rng.choice([2, 4, 6])), k0=k0, width=0.5 * k0)
        jobs.append(dict(dims=dims, filt=f, seed=seed0 + i, bins=bins))
    return jobs


def single(hf, job):
    bins = job["bins"] or (4, 1)
    b = hf.PipelineBuffers(job["dims"], 1, bins)
    hf.pipeline(b, job["filt"], [job["seed"]])
    return b


def _check_against_singles(hf, bb, jobs):
    for i, j in enumerate(jobs):
        s = single(hf, j)
        torch.cuda.synchronize()
        o = bb.out[i]
        assert torch.equal(o["field"], s.field[0]), (i, j["dims"])
        assert torch.equal(o["pm1"], s.pm1[0]), (i, j["dims"])
        assert torch.equal(o["counts"], s.counts[0])
        np.testing.assert_allclose(o["stats"].cpu().numpy(), s.stats[0].cpu().numpy(), rtol=1e-12)
        if j["bins"] is not None:
            assert torch.equal(o["cont_cnt"], s.cont_cnt[0]) and torch.equal(o["pm1_cnt"], s.pm1_cnt[0])
            # the bins are combined in a fixed order: the same bits whatever the schedule
            assert torch.equal(o["cont_sum"], s.cont_sum[0]), (i, j["dims"])
            assert torch.equal(o["pm1_sum"], s.pm1_sum[0]), (i, j["dims"])


def test_batch_matches_single_calls_and_oracle(hf):
    jobs = mixed_jobs()
    _say("batch of", len(jobs))
    bb = hf.BatchBuffers(jobs)
    st = hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    assert st == [0] * len(jobs)
    _check_against_singles(hf, bb, jobs)
    for i in (2, 7):
        j = jobs[i]
        P.compare_field("mixed_batch_job%d" % i, j["dims"], j["filt"], j["seed"], j["bins"], job_host(hf, bb, i))


def job_host(hf, bb, i):
    """Job i of BatchBuffers as host arrays, in the form _parity.compare_field takes."""
    o = bb.out[i]
    h = {k: (hf.u64_view(v) if k in ("counts", "cont_cnt", "pm1_cnt") else v.cpu().numpy()) for k, v in o.items()}
    return h


def test_whole_field_kernel_in_a_batch_equals_single_calls(hf):
    """The small 2D classes of a mixed batch under plan entry whole_field (one kernel per class,
    per-field parameters from the batch table) give the bits of single calls under the same entry,
    and agree with the oracle.  The same batch structure ran under the default plans in the tests
    above: the cached graph must follow the changed plan (a new capture)."""
    jobs = mixed_jobs(seed0=700)
    keys = set()
    for j in jobs:
        if len(j["dims"]) == 2 and max(j["dims"]) <= 128:
            keys.add((tuple(j["dims"]), j["bins"]))            # the batch classes
            keys.add((tuple(j["dims"]), j["bins"] or (4, 1)))  # the single calls
    def plans(v):
        for dims, bins in keys:
            for n in (1, 2, 8):                                 # every batch-size bucket used here
                hf.plan_set(dims, n, bins, v)
    plans([0] * 11 + [1, 0])
    try:
        bb = hf.BatchBuffers(jobs)
        st = hf.pipeline_batch(bb)
        torch.cuda.synchronize()
        assert st == [0] * len(jobs)
        _check_against_singles(hf, bb, jobs)
        for i in (0, 2):
            j = jobs[i]
            P.compare_field("whole_batch_job%d" % i, j["dims"], j["filt"], j["seed"], j["bins"], job_host(hf, bb, i))
    finally:
        plans([0] * 13)


def test_plane_kernels_in_a_batch_equal_single_calls(hf):
    """3D classes under plan entry plane (per-field parameters from the batch table) give the bits
    of single calls under the same entry, and agree with the oracle."""
    rng = np.random.default_rng(11)
    shapes = [((32, 64, 64), (16, 1)), ((32, 64, 64), (16, 1)), ((48, 32, 96), (12, 1)), ((16, 48, 32), (12, 1))]
    jobs = []
    for i, (dims, bins) in enumerate(shapes):
        k0 = float(rng.uniform(0.15, 0.35))
        f = W.filt(p=float(rng.uniform(1.5, 8)), semi=(float(rng.uniform(1, 3)), 1.0, 1.5),
                   rot=float(rng.uniform(0, math.pi)), alpha=float(rng.choice([2, 4])), k0=k0, width=0.5 * k0)
        jobs.append(dict(dims=dims, filt=f, seed=900 + i, bins=bins))
    on = [0] * 12 + [1]
    keys = {(tuple(j["dims"]), j["bins"]) for j in jobs}
    def plans(v):
        for dims, bins in keys:
            for n in (1, 2):
                hf.plan_set(dims, n, bins, v)
    plans(on)
    try:
        bb = hf.BatchBuffers(jobs)
        st = hf.pipeline_batch(bb)
        torch.cuda.synchronize()
        assert st == [0] * len(jobs)
        _check_against_singles(hf, bb, jobs)
        for i in (0, 2, 3):
            j = jobs[i]
            P.compare_field("plane_batch_job%d" % i, j["dims"], j["filt"], j["seed"], j["bins"], job_host(hf, bb, i))
    finally:
        plans([0] * 13)


def test_full_uneven_batch_sampled(hf):
    jobs = W.c4_jobs()
    _say("uneven batch of", len(jobs))
    bb = hf.BatchBuffers(jobs)
    st = hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    assert st == [0] * len(jobs)
    first = {}
    for i, j in enumerate(jobs):
        first.setdefault(tuple(j["dims"]), i)
    for dims, i in sorted(first.items()):
        j = jobs[i]
        rec = P.compare_field("c4_job%d" % i, dims, j["filt"], j["seed"], j["bins"], job_host(hf, bb, i))
        _say("   job", i, dims, "max err/rms %.3e" % rec["field_err_rms"], "flips", rec["flips"])


def test_batch_graph_replays(hf):
    jobs = mixed_jobs(seed0=500)
    bb = hf.BatchBuffers(jobs)
    for rep in range(3):
        _say("replay", rep)
        seeds = [900 + 37 * rep + i for i in range(len(jobs))]
        bb.set_seeds(seeds)
        for j, s in zip(jobs, seeds):
            j["seed"] = s
        hf.pipeline_batch(bb)
        x = torch.randn(1 << 20, device="cuda")          # unrelated eager work between replays
        y = (x * x).sum().item()
        assert y > 0
        torch.cuda.synchronize()
        _check_against_singles(hf, bb, jobs)


def test_batch_invalid_job_keeps_others(hf):
    jobs = mixed_jobs(seed0=50)[:4]
    bad = dict(jobs[1])
    bad["filt"] = dict(bad["filt"], p=0.0)
    jobs[1] = bad
    bb = hf.BatchBuffers(jobs)
    st = hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    assert st[1] == hf.HU_ERR_ARG and st[0] == 0 and st[2] == 0 and st[3] == 0
    good = [j for k, j in enumerate(jobs) if k != 1]
    for k, j in zip([0, 2, 3], good):
        s = single(hf, j)
        torch.cuda.synchronize()
        assert torch.equal(bb.out[k]["field"], s.field[0])


@pytest.mark.parametrize("dims,bins", [((256, 512), (32, 12)), ((2048, 64), (16, 4)), ((32, 64, 48), (24, 1)),
                                       ((96, 96, 96), (32, 1)), ((256, 32, 16), (24, 1))])
def test_half_width_variants_match(hf, dims, bins):
    _say("variants", dims)
    filt = W.filt(p=3, semi=(2, 1, 1.5), rot=0.4, alpha=4, k0=0.2, width=0.05)
    seeds = [11, 12]
    hf.plan_set(dims, 2, bins, [0] * 13)
    b0 = hf.PipelineBuffers(dims, 2, bins)
    hf.pipeline(b0, filt, seeds)
    switched = [1] * 8 + [0, 1, 1, 0, 0]                # every tile width, schedule and exchange
    hf.plan_set(dims, 2, bins, switched)
    b1 = hf.PipelineBuffers(dims, 2, bins)
    hf.pipeline(b1, filt, seeds)
    torch.cuda.synchronize()
    assert hf.plan_query(dims, 2, bins) == dict(zip(hf.PASS_NAMES, switched))
    assert torch.equal(b0.field, b1.field) and torch.equal(b0.pm1, b1.pm1)
    np.testing.assert_allclose(b0.pm1_sum.cpu().numpy(), b1.pm1_sum.cpu().numpy(), rtol=1e-10, atol=1e-9)
    ref = O.pipeline(dims, O.FilterParams(**filt), seeds[1], *bins)
    f = b1.field[1].double().cpu().numpy()
    assert np.max(np.abs(f - ref["f"])) <= 1e-5 * math.sqrt(float(np.mean(ref["f"] ** 2)))
    hf.plan_set(dims, 2, bins, [0] * 13)


def test_autotune_writes_plan(hf, tmp_path):
    dims, bins = (256, 256), (32, 6)
    path = str(tmp_path / "tune.json")
    _say("autotune", dims)
    plan, ms = hf.autotune(dims, 4, bins, path)
    assert set(plan.values()) <= {0, 1} and len(plan) == 13
    assert ms["default_ms"] > 0 and 0 < ms["tuned_ms"] <= ms["default_ms"]
    assert ms["flipped_ms"]["cols_filter"] > 0 and ms["flipped_ms"]["y_group"] == 0   # 2D: no y passes
    assert ms["flipped_ms"]["radix"] > 0                # 256 has an alternative radix list
    assert ms["flipped_ms"]["bin_exchange"] > 0 and ms["flipped_ms"]["filter_exchange"] > 0
    d = json.load(open(path))
    keys = [k for k in d["plans"] if "256x256x1" in k]
    assert keys and d["plans"][keys[0]] == [plan[n] for n in hf.PASS_NAMES]
    assert hf.plan_query(dims, 4, bins) == plan
    hf.plan_set(dims, 4, bins, [0] * 13)                # later tests run the default plan
