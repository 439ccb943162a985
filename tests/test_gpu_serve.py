"""GPU tests of the continuous-batching server.

Requests of different sizes, block sizes and masks arrive while others are on
the GPU; each result must be bit-identical to the same request served alone
(and to a direct dctf_filter_blocks call), admission must respect the device
arena, and the operator cache must evict and rebuild correctly.
"""
import numpy as np
import pytest
import torch

import synthetic as syn

pytestmark = pytest.mark.gpu
SPLIT, FP32 = 1, 0


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def make_requests(n, seed, rate_hz, masks):
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for i in range(n):
        N = 16 if rng.random() < 0.25 else 8
        B = int(rng.integers(1, 3000))
        spec = masks[int(rng.integers(0, len(masks)))]
        X = torch.randn(B * N * N, device="cuda") * 60
        reqs.append(dict(arrival_s=t, mask=spec.mask, N=N, border=spec.border, X=X,
                         Y=torch.full_like(X, float("nan"))))
        t += float(rng.exponential(1.0 / rate_hz))
    return reqs


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_same_result_alone_and_in_the_mix(dctf, prec):
    masks = syn.mask_set_32()[:12]
    reqs = make_requests(48, 5, 200000.0, masks)        # arrivals ~5 us apart: they overlap
    server = dctf.dctf_server_create(arena_bytes=1 << 28, max_inflight=4, max_batch_jobs=8, prec=prec)
    res = dctf.dctf_server_run(server, reqs)
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in res)
    stats = dctf.dctf_server_stats(server)
    assert stats["batches"] >= 2
    mixed = [r["Y"].clone() for r in reqs]
    # alone: one request per run
    for i, r in enumerate(reqs):
        r["Y"].fill_(float("nan"))
        one = dict(r, arrival_s=0.0)
        res1 = dctf.dctf_server_run(server, [one])
        assert res1[0]["status"] == 0
        torch.cuda.synchronize()
        assert torch.equal(r["Y"], mixed[i]), i
    # and the direct single-operator call
    for i, r in enumerate(reqs[:10]):
        op = dctf.dctf_build_operator(r["mask"], r["N"], r["border"])
        Y = torch.empty_like(r["X"])
        dctf.dctf_filter_blocks(op, prec, r["X"], Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, mixed[i]), i
    for r in res:
        assert 0 <= r["admit_s"] <= r["launch_s"] <= r["done_s"]


def test_work_overlaps_on_the_device(dctf):
    masks = syn.mask_set_32()[:4]
    rng = np.random.default_rng(1)
    reqs = []
    for i in range(24):
        X = torch.randn(40000 * 64, device="cuda")       # 40k blocks: long enough to overlap
        reqs.append(dict(arrival_s=i * 2e-6, mask=masks[i % 4].mask, N=8, border=masks[i % 4].border, X=X))
    server = dctf.dctf_server_create(arena_bytes=1 << 30, max_inflight=4, max_batch_jobs=2)
    res = dctf.dctf_server_run(server, reqs)
    stats = dctf.dctf_server_stats(server)
    assert all(r["status"] == 0 for r in res)
    assert stats["peak_inflight_batches"] >= 2
    assert stats["batches"] >= 12


def test_admission_by_arena_bytes(dctf):
    masks = syn.mask_set_32()[:2]
    small = torch.randn(100 * 64, device="cuda")
    big = torch.randn(5000 * 64, device="cuda")
    arena = 3000 * 64 * 4                                 # smaller than `big`, room for ~2 smalls at once
    reqs = [dict(arrival_s=0.0, mask=masks[0].mask, N=8, border=0, X=small, Y=torch.empty_like(small)),
            dict(arrival_s=0.0, mask=masks[1].mask, N=8, border=1, X=big),
            dict(arrival_s=0.0, mask=masks[0].mask, N=8, border=0, X=small, Y=torch.empty_like(small))]
    server = dctf.dctf_server_create(arena_bytes=arena, max_inflight=2, max_batch_jobs=4)
    res = dctf.dctf_server_run(server, reqs)
    assert [r["status"] for r in res] == [0, dctf.DCTF_EBUSY, 0]
    stats = dctf.dctf_server_stats(server)
    assert stats["rejected"] == 1 and stats["peak_arena_bytes"] <= arena
    assert torch.equal(reqs[0]["Y"], reqs[2]["Y"])


def test_arena_limits_requests_in_flight(dctf):
    masks = syn.mask_set_32()[:1]
    X = torch.randn(2000 * 64, device="cuda")
    reqs = [dict(arrival_s=0.0, mask=masks[0].mask, N=8, border=0, X=X) for _ in range(6)]
    one = 2000 * 64 * 4
    server = dctf.dctf_server_create(arena_bytes=one + one // 2, max_inflight=4, max_batch_jobs=4)
    res = dctf.dctf_server_run(server, reqs)
    assert all(r["status"] == 0 for r in res)
    assert dctf.dctf_server_stats(server)["peak_arena_bytes"] <= one + one // 2
    # only one request fits at a time: every launch carries exactly one
    assert len({r["batch"] for r in res}) == 6


def test_operator_cache_evicts_and_rebuilds(dctf):
    masks = syn.mask_set_32()[8:12]
    X = torch.randn(300 * 64, device="cuda")
    reqs = []
    for i in range(16):
        m = masks[i % 4]
        reqs.append(dict(arrival_s=i * 1e-3, mask=m.mask, N=8, border=m.border, X=X, Y=torch.empty_like(X)))
    server = dctf.dctf_server_create(arena_bytes=1 << 26, max_inflight=1, max_batch_jobs=1, max_cached_ops=2)
    res = dctf.dctf_server_run(server, reqs)
    assert all(r["status"] == 0 for r in res)
    stats = dctf.dctf_server_stats(server)
    assert stats["cache_evictions"] > 0 and stats["cache_misses"] > 4
    for i in range(4, 16):
        assert torch.equal(reqs[i]["Y"], reqs[i - 4]["Y"])


def test_malformed_request_lists(dctf):
    masks = syn.mask_set_32()[:1]
    X = torch.randn(64, device="cuda")
    server = dctf.dctf_server_create(arena_bytes=1 << 20)
    bad_order = [dict(arrival_s=1.0, mask=masks[0].mask, N=8, border=0, X=X),
                 dict(arrival_s=0.5, mask=masks[0].mask, N=8, border=0, X=X)]
    with pytest.raises(dctf.DctfError):
        dctf.dctf_server_run(server, bad_order)
    with pytest.raises(dctf.DctfError):
        # N = 5 is no block size of the library
        dctf.dctf_server_run(server, [dict(arrival_s=0.0, mask=masks[0].mask, N=5, border=0,
                                           X=torch.randn(75, device="cuda"))])


def test_malformed_mask_runs_nothing(dctf):
    """A NaN in one request's mask makes the whole list malformed: nothing runs."""
    masks = syn.mask_set_32()[:1]
    X = torch.randn(300 * 64, device="cuda")
    Y = torch.full_like(X, float("nan"))
    bad = masks[0].mask.copy()
    bad[0, 0] = float("nan")
    server = dctf.dctf_server_create(arena_bytes=1 << 24)
    reqs = [dict(arrival_s=0.0, mask=masks[0].mask, N=8, border=0, X=X, Y=Y),
            dict(arrival_s=0.0, mask=bad, N=8, border=0, X=X)]
    with pytest.raises(dctf.DctfError) as e:
        dctf.dctf_server_run(server, reqs)
    assert e.value.status == dctf.DCTF_EINVAL
    torch.cuda.synchronize()
    assert torch.isnan(Y).all()
    assert dctf.dctf_server_stats(server)["batches"] == 0
    with pytest.raises(dctf.DctfError):
        dctf.dctf_server_submit(server, bad, 8, 0, X)
    # the server still serves after the rejected calls
    res = dctf.dctf_server_run(server, reqs[:1])
    assert res[0]["status"] == 0 and not torch.isnan(Y).any()


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_online_submit_and_poll(dctf, prec):
    """Requests submitted one by one while earlier ones are on the GPU: every
    request completes once, with the result of a single-operator call."""
    masks = syn.mask_set_32()
    rng = np.random.default_rng(8)
    server = dctf.dctf_server_create(arena_bytes=1 << 28, max_inflight=3, max_batch_jobs=6, prec=prec)
    reqs, done = [], []
    for i in range(40):
        N = 16 if i % 5 == 0 else 8
        X = torch.randn(int(rng.integers(1, 20000)) * N * N, device="cuda") * 50
        m = masks[int(rng.integers(0, len(masks)))]
        r = dctf.dctf_server_submit(server, m.mask, N, m.border, X, torch.full_like(X, float("nan")))
        reqs.append((r, m, N, X))
        if i % 3 == 0:
            done += dctf.dctf_server_poll(server)
    while len(done) < len(reqs):
        got = dctf.dctf_server_poll(server, wait_s=1.0)
        assert got, "no request completed within a second"
        done += got
    assert len({id(r) for r in done}) == len(reqs)
    assert dctf.dctf_server_poll(server) == []
    stats = dctf.dctf_server_stats(server)
    assert stats["batches"] >= 2 and stats["failed"] == 0
    torch.cuda.synchronize()
    for r, m, N, X in reqs:
        assert r.status == 0 and 0 <= r.admit_s <= r.launch_s <= r.done_s
        op = dctf.dctf_build_operator(m.mask, N, m.border)
        Y = torch.empty_like(X)
        dctf.dctf_filter_blocks(op, prec, X, Y)
        torch.cuda.synchronize()
        assert torch.equal(r.keep[2], Y)


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_served_outputs_match_oracle(dctf, prec):
    """Requests shaped like the serving workload (image sides that are
    multiples of 8, N = 8 or 16 with replication padding to whole blocks, the
    32-mask set): each served output against the FP64 oracle directly."""
    import oracle
    tol = 5e-3 if prec == SPLIT else 2e-3
    masks = syn.mask_set_32()
    rng = np.random.default_rng(31)
    reqs, refs = [], []
    for k in range(10):
        N = 16 if k % 3 == 0 else 8
        h, w = int(rng.choice(np.arange(256, 769, 8))), int(rng.choice(np.arange(256, 769, 8)))
        m = masks[(7 * k) % len(masks)]
        px = oracle.tile_u8(syn.image_u8(700 + k, h, w), N)
        X = torch.from_numpy(oracle.coeffs_fp32(px).reshape(-1)).cuda()
        reqs.append(dict(arrival_s=k * 2e-5, mask=m.mask, N=N, border=m.border, X=X,
                         Y=torch.full_like(X, float("nan"))))
        refs.append(oracle.filter_pixels(px, m.mask, m.border)[0])
    server = dctf.dctf_server_create(arena_bytes=1 << 28, max_inflight=4, max_batch_jobs=4, prec=prec)
    res = dctf.dctf_server_run(server, reqs)
    torch.cuda.synchronize()
    for r, q, ref in zip(res, reqs, refs):
        assert r["status"] == 0
        err = np.abs(q["Y"].cpu().numpy().reshape(ref.shape) - ref).max()
        assert err <= tol, err


@pytest.mark.parametrize("prec", [SPLIT, FP32])
def test_served_block_sizes_2_to_32(dctf, prec):
    """Requests of N = 2, 4 and 32 beside N = 8 and 16 in the same batches:
    each served output equals the single-operator call."""
    rng = np.random.default_rng(12)
    masks = {2: syn.box_mask(3), 4: syn.random_mask(rng, 5, 5), 8: syn.asym_mask_5x5(),
             16: syn.gaussian_mask(7), 32: syn.random_mask(rng, 7, 7)}
    reqs = []
    for k in range(20):
        N = (2, 4, 8, 16, 32)[k % 5]
        B = int(rng.integers(1, 600))
        X = torch.randn(B * N * N, device="cuda") * 40
        reqs.append(dict(arrival_s=k * 1e-5, mask=masks[N], N=N, border=k % 2, X=X,
                         Y=torch.full_like(X, float("nan"))))
    server = dctf.dctf_server_create(arena_bytes=1 << 28, max_inflight=3, max_batch_jobs=6, prec=prec)
    res = dctf.dctf_server_run(server, reqs)
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in res)
    for r in reqs:
        op = dctf.dctf_build_operator(r["mask"], r["N"], r["border"])
        Y = torch.empty_like(r["X"])
        dctf.dctf_filter_blocks(op, prec, r["X"], Y)
        torch.cuda.synchronize()
        assert torch.equal(r["Y"], Y), r["N"]
