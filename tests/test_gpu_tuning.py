"""GPU tests of the autotuners: the batch tuner on a small plan and the
single-operator tuner.  Every configuration computes bit-identical results,
so the tuned plan's output must equal the default plan's, and the choice
must be one of the candidates timed."""
import numpy as np
import pytest
import torch

import synthetic as syn

pytestmark = pytest.mark.gpu
FP32, SPLIT = 0, 1


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def small_plan(dctf, prec, seed=3):
    rng = np.random.default_rng(seed)
    ops = dctf.dctf_build_operators([(syn.random_mask(rng, k, k), 8, b) for k in (3, 5, 7) for b in (0, 1)])
    jobs = []
    for i in range(24):
        B = int(rng.integers(1, 9000))
        X = torch.randn(B * 64, device="cuda") * 80
        jobs.append((ops[int(rng.integers(0, len(ops)))], X, torch.full_like(X, float("nan"))))
    return jobs


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_batch_autotune_choice_and_output(dctf, prec):
    jobs = small_plan(dctf, prec)
    b = dctf.dctf_batch_create(jobs, prec)
    cands = dctf.dctf_batch_autotune_candidates()
    best, table = dctf.dctf_batch_autotune(b, dctf.DCTF_RUN_REBUILD_OPERATORS, iters=2, rounds=1)
    assert 0 <= best < len(cands) and len(table) == len(cands)
    assert table[best][1] > 0 and all(t < 0 or t >= table[best][1] for _, t in table)
    cfg, resolved = dctf.dctf_batch_get_config(b)
    chosen = dict(cands[best])
    assert cfg["io"] == chosen["io"] and cfg["nt"] == chosen["nt"] and cfg["fronts"] == chosen["fronts"]
    assert resolved["io"] == chosen["io"]
    for _, _, Y in jobs:
        Y.fill_(float("nan"))
    dctf.dctf_batch_run(b)
    torch.cuda.synchronize()
    # the default plan's output, job by job
    for op, X, Y in jobs:
        Yd = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, Yd)
        torch.cuda.synchronize()
        assert torch.equal(Y, Yd)


def test_batch_config_replan_and_process_setting(dctf):
    jobs = small_plan(dctf, SPLIT, seed=4)
    want = []
    for op, X, _ in jobs:
        Yd = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, SPLIT, X, Yd)
        want.append(Yd)
    b = dctf.dctf_batch_create(jobs, SPLIT)
    saved = dctf.dctf_get_batch_config(SPLIT)
    try:
        for cfg in (dict(fronts=1, io=2, nt=1, groups_per_cu=1), dict(fronts=0, io=0, nt=0, groups_per_cu=0),
                    dict(fronts=5, io=1, nt=0, groups_per_cu=2)):
            dctf.dctf_batch_set_config(b, cfg)
            got, res = dctf.dctf_batch_get_config(b)
            assert got == cfg and res["io"] == cfg["io"]
            if cfg["groups_per_cu"]:
                assert res["groups_per_cu"] <= cfg["groups_per_cu"]
            for _, _, Y in jobs:
                Y.fill_(float("nan"))
            dctf.dctf_batch_run(b)
            torch.cuda.synchronize()
            for (_, _, Y), w in zip(jobs, want):
                assert torch.equal(Y, w), cfg
        # the process-wide setting reaches new plans
        dctf.dctf_set_batch_config(SPLIT, dict(fronts=3, io=2, nt=0, groups_per_cu=0))
        b2 = dctf.dctf_batch_create(jobs, SPLIT)
        assert dctf.dctf_batch_get_config(b2)[0] == dict(fronts=3, io=2, nt=0, groups_per_cu=0)
    finally:
        dctf.dctf_set_batch_config(SPLIT, saved)


def test_graph_after_replan(dctf):
    jobs = small_plan(dctf, SPLIT, seed=5)
    b = dctf.dctf_batch_create(jobs, SPLIT)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dctf.dctf_batch_capture(b, 0, s)
    dctf.dctf_batch_set_config(b, dict(fronts=2, io=2, nt=1, groups_per_cu=0))
    with pytest.raises(dctf.DctfError):           # the re-plan dropped the captured graph
        dctf.dctf_batch_launch_graph(b, s)
    with torch.cuda.stream(s):
        dctf.dctf_batch_capture(b, 0, s)
    for _, _, Y in jobs:
        Y.fill_(float("nan"))
    torch.cuda.synchronize()
    dctf.dctf_batch_launch_graph(b, s)
    s.synchronize()
    for op, X, Y in jobs:
        Yd = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, SPLIT, X, Yd)
        torch.cuda.synchronize()
        assert torch.equal(Y, Yd)


@pytest.mark.parametrize("N,prec", [(8, SPLIT), (16, FP32)])
def test_single_operator_autotune(dctf, N, prec):
    op = dctf.dctf_build_operator(syn.asym_mask_5x5(), N, 1)
    X = torch.randn(20000 * N * N, device="cuda") * 50
    Y = torch.empty_like(X)
    v0 = dctf.dctf_get_variant(N, prec)
    try:
        dctf.dctf_set_variant(N, prec, 0)
        Y0 = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, Y0)
        best, ms = dctf.dctf_autotune(op, prec, X, Y, iters=2)
        assert 0 <= best < dctf.dctf_variant_count(N, prec) and ms > 0
        assert dctf.dctf_get_variant(N, prec) == best
        dctf.dctf_filter_blocks(op, prec, X, Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, Y0)
    finally:
        dctf.dctf_set_variant(N, prec, v0)


def test_tuning_table_round_trip(dctf, tmp_path):
    from paper_1710_07193_amd import tuning
    saved = {p: dctf.dctf_get_batch_config(p) for p in (FP32, SPLIT)}
    v8 = dctf.dctf_get_variant(8, SPLIT)
    try:
        entry = tuning.tune_batch(SPLIT, images=4, blocks=4096, masks=3, iters=2, rounds=1)
        table = {"device": "test", "entries": {"batch/N8/split-bf16": entry,
                                               "filter/N8/split-bf16": {"variant": "dma_u1_w8_nt"}}}
        path = str(tmp_path / "t.json")
        tuning.save(table, path)
        out = tuning.apply_table(path)
        assert out["applied"]["batch/N8/split-bf16"] == entry["config"]
        assert dctf.dctf_get_batch_config(SPLIT) == entry["config"]
        assert dctf.dctf_variant_name(8, SPLIT, dctf.dctf_get_variant(8, SPLIT)) == "dma_u1_w8_nt"
    finally:
        for p in (FP32, SPLIT):
            dctf.dctf_set_batch_config(p, saved[p])
        dctf.dctf_set_variant(8, SPLIT, v8)
