"""GPU tests of the persistent batched launch and its HIP graph capture.

A batch mixes images of uneven block counts, several operators and both MFMA
block sizes (N = 8 and N = 16) in one launch.  Every job's output must be
bit-identical to filtering that job alone, and within the coefficient
tolerance of the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

Z, R = 0, 1
FP32, SPLIT = 0, 1
TOL = {FP32: 2e-3, SPLIT: 5e-3}


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_jobs(dctf, seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(8, 256, 264), (8, 512, 512), (8, 64, 72), (8, 8, 8), (8, 1000, 24),
              (16, 272, 256), (16, 96, 336), (16, 16, 16)]
    masks = [(syn.random_mask(rng, 5, 5), R), (syn.gaussian_mask(3), Z), (syn.random_mask(rng, 7, 7), Z),
             (syn.random_mask(rng, 3, 3, symmetric=True), R)]
    jobs = []
    for k, (N, h, w) in enumerate(shapes):
        W, border = masks[k % len(masks)]
        px = oracle.tile_u8(syn.image_u8(100 + k, h, w), N)
        X = dev(oracle.coeffs_fp32(px).reshape(-1))
        Y = torch.full_like(X, float("nan"))
        jobs.append(dict(N=N, W=W, border=border, px=px, X=X, Y=Y))
    specs = [(j["W"], j["N"], j["border"]) for j in jobs]
    ops = dctf.dctf_build_operators(specs)
    for j, op in zip(jobs, ops):
        j["op"] = op
    return jobs


def alone(dctf, j, prec):
    Y = torch.empty_like(j["X"])
    dctf.dctf_filter_blocks(j["op"], prec, j["X"], Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_batch_matches_alone_and_oracle(dctf, prec):
    jobs = make_jobs(dctf)
    batch = dctf.dctf_batch_create([(j["op"], j["X"], j["Y"]) for j in jobs], prec)
    g8, g16, threads = dctf.dctf_batch_info(batch)
    assert g8 >= 1 and g16 >= 1 and threads == 512
    dctf.dctf_batch_run(batch)
    torch.cuda.synchronize()
    for j in jobs:
        got = j["Y"].cpu().numpy()
        assert np.array_equal(got, alone(dctf, j, prec))
        Yref, _, _ = oracle.filter_pixels(j["px"], j["W"], j["border"])
        assert np.abs(got.reshape(Yref.shape) - Yref).max() <= TOL[prec]


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_batch_graph_replays(dctf, prec):
    jobs = make_jobs(dctf, seed=1)
    batch = dctf.dctf_batch_create([(j["op"], j["X"], j["Y"]) for j in jobs], prec)
    want = [alone(dctf, j, prec) for j in jobs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dctf.dctf_batch_capture(batch, dctf.DCTF_RUN_REBUILD_OPERATORS, s)
    torch.cuda.synchronize()
    for replay in range(3):
        for j in jobs:
            j["Y"].fill_(float("nan"))
        # unrelated eager work between replays
        dctf.dctf_filter_blocks(jobs[0]["op"], prec, jobs[0]["X"], torch.empty_like(jobs[0]["X"]))
        torch.cuda.synchronize()
        dctf.dctf_batch_launch_graph(batch, s)
        s.synchronize()
        for j, w in zip(jobs, want):
            assert np.array_equal(j["Y"].cpu().numpy(), w), replay


def test_filter_batch_oneshot_and_empty_jobs(dctf):
    jobs = make_jobs(dctf, seed=2)
    empty = torch.empty(0, dtype=torch.float32, device="cuda")
    triples = [(j["op"], j["X"], j["Y"]) for j in jobs] + [(jobs[0]["op"], empty, empty)]
    dctf.dctf_filter_batch(triples, SPLIT)
    for j in jobs:
        assert np.array_equal(j["Y"].cpu().numpy(), alone(dctf, j, SPLIT))
    dctf.dctf_filter_batch([], SPLIT)   # no jobs: no-op


def test_batch_only_one_block_size(dctf):
    jobs = [j for j in make_jobs(dctf, seed=3) if j["N"] == 16]
    batch = dctf.dctf_batch_create([(j["op"], j["X"], j["Y"]) for j in jobs], SPLIT)
    g8, g16, _ = dctf.dctf_batch_info(batch)
    assert g8 == 0 and g16 >= 1
    dctf.dctf_batch_run(batch)
    torch.cuda.synchronize()
    for j in jobs:
        assert np.array_equal(j["Y"].cpu().numpy(), alone(dctf, j, SPLIT))


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_batch_many_small_jobs(dctf, prec):
    """Hundreds of tiny jobs over 24 operators (more segments than usual,
    ragged tiles everywhere), for every N = 8 I/O variant the batch can use."""
    rng = np.random.default_rng(77)
    specs = [(syn.random_mask(rng, k, k), N, b) for N in (8, 16) for k in (3, 5, 7) for b in (Z, R)
             for _ in range(2)]
    ops = dctf.dctf_build_operators(specs)
    jobs = []
    for i in range(300):
        op = ops[int(rng.integers(0, len(ops)))]
        B = int(rng.integers(1, 60))
        X = torch.randn(B * op.N * op.N, device="cuda") * 100
        jobs.append((op, X, torch.empty_like(X)))
    want = []
    for op, X, _ in jobs:
        Y = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, Y)
        want.append(Y)
    fronts0 = dctf.dctf_get_batch_fronts()
    for order in (0, 1, 3):
        dctf.dctf_set_batch_fronts(order)
        for v in range(dctf.dctf_variant_count(8, prec)):
            dctf.dctf_set_variant(8, prec, v)
            try:
                for _, _, Y in jobs:
                    Y.fill_(float("nan"))
                dctf.dctf_filter_batch(jobs, prec)
                for (op, X, Y), w in zip(jobs, want):
                    assert torch.equal(Y, w), (order, dctf.dctf_variant_name(8, prec, v))
            finally:
                dctf.dctf_set_variant(8, prec, 0)
                dctf.dctf_set_batch_fronts(fronts0)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_batch_operator_changes_within_a_wave(dctf, prec):
    """Enough units that every wave walks through several jobs and operators
    (including a change right at its last unit), for each front setting."""
    rng = np.random.default_rng(91)
    ops = dctf.dctf_build_operators([(syn.random_mask(rng, k, k), 8, b) for k in (3, 5, 7) for b in (Z, R)
                                     for _ in range(4)])
    jobs = []
    for i in range(96):
        B = int(rng.integers(1, 12000))
        X = torch.randn(B * 64, device="cuda") * 100
        jobs.append((ops[int(rng.integers(0, len(ops)))], X, torch.empty_like(X)))
    want = []
    for op, X, _ in jobs:
        Y = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, Y)
        want.append(Y)
    fronts0 = dctf.dctf_get_batch_fronts()
    try:
        for fronts in (0, 1, 2, 5):
            dctf.dctf_set_batch_fronts(fronts)
            for _, _, Y in jobs:
                Y.fill_(float("nan"))
            dctf.dctf_filter_batch(jobs, prec)
            for k, ((op, X, Y), w) in enumerate(zip(jobs, want)):
                assert torch.equal(Y, w), (fronts, k)
    finally:
        dctf.dctf_set_batch_fronts(fronts0)


def test_batch_rejections(dctf):
    jobs = make_jobs(dctf, seed=4)
    a, b = jobs[0], jobs[1]
    with pytest.raises(dctf.DctfError):     # two jobs write the same memory
        dctf.dctf_batch_create([(a["op"], a["X"], a["Y"]), (a["op"], b["X"][: a["Y"].numel()], a["Y"])], SPLIT)
    with pytest.raises(dctf.DctfError):     # one job's output is another's input
        dctf.dctf_batch_create([(a["op"], a["X"], a["Y"]), (a["op"], a["Y"], b["Y"][: a["Y"].numel()])], SPLIT)
    small = dctf.dctf_build_operator(syn.box_mask(3), 4, Z)
    x4 = torch.zeros(16 * 4, device="cuda")
    with pytest.raises(dctf.DctfError):       # a side job's output overlapping a table job's input
        dctf.dctf_batch_create([(a["op"], a["X"], a["Y"]), (small, x4, a["X"][:x4.numel()])], SPLIT)


@pytest.mark.parametrize("prec", [FP32, SPLIT])
def test_batch_every_block_size(dctf, prec):
    """Jobs of N = 2, 4, 8, 16 and 32 in one batch (the N = 8 / 16 jobs in the
    persistent launch, the others one launch each after it): each output
    equals the job filtered alone, on a run with the operator rebuild, on
    graph replays and in the one-shot call, and the oracle within tolerance."""
    rng = np.random.default_rng(44)
    specs = [(2, 40, 36, syn.box_mask(3), Z), (4, 64, 52, syn.random_mask(rng, 5, 5), R),
             (8, 200, 264, syn.random_mask(rng, 5, 5), R), (16, 96, 128, syn.gaussian_mask(7), Z),
             (32, 160, 96, syn.random_mask(rng, 7, 7), Z), (32, 64, 64, syn.gaussian_mask(5), R),
             (4, 8, 8, syn.box_mask(3), R)]
    jobs = []
    for k, (N, h, w, W, border) in enumerate(specs):
        px = oracle.tile_u8(syn.image_u8(900 + k, h, w), N)
        X = dev(oracle.coeffs_fp32(px).reshape(-1))
        jobs.append(dict(N=N, W=W, border=border, px=px, X=X, Y=torch.full_like(X, float("nan"))))
    ops = dctf.dctf_build_operators([(j["W"], j["N"], j["border"]) for j in jobs])
    for j, op in zip(jobs, ops):
        j["op"] = op
    tol = {2: 2e-3, 4: 2e-3, 8: TOL[prec], 16: TOL[prec], 32: TOL[prec]}
    b = dctf.dctf_batch_create([(j["op"], j["X"], j["Y"]) for j in jobs], prec)
    dctf.dctf_batch_run(b, dctf.DCTF_RUN_REBUILD_OPERATORS)
    torch.cuda.synchronize()
    for j in jobs:
        got = j["Y"].cpu().numpy()
        assert np.array_equal(got, alone(dctf, j, prec)), j["N"]
        ref, _, _ = oracle.filter_pixels(j["px"], j["W"], j["border"])
        assert np.abs(got.reshape(ref.shape) - ref).max() <= tol[j["N"]], j["N"]
    first = [j["Y"].clone() for j in jobs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for j in jobs:
            j["Y"].fill_(float("nan"))
        dctf.dctf_batch_capture(b, dctf.DCTF_RUN_REBUILD_OPERATORS, s)
        for _ in range(3):
            dctf.dctf_batch_launch_graph(b, s)
            s.synchronize()
            for j, f in zip(jobs, first):
                assert torch.equal(j["Y"], f), j["N"]
                j["Y"].fill_(float("nan"))
    torch.cuda.synchronize()
    dctf.dctf_filter_batch([(j["op"], j["X"], j["Y"]) for j in jobs], prec)
    for j, f in zip(jobs, first):
        assert torch.equal(j["Y"], f), j["N"]
