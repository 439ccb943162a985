"""GPU parity of the benchmark's headline step at its full size.

The step is built by the benchmark's own function: 64 seeded 2048 x 2048 uint8
images through the library's forward DCT, the 16-mask pool (K in {3, 5, 7},
symmetric or not, border replication), one pool mask per image drawn with
seed 17, one job per image, and one persistent batch launch preceded by the
FP64 operator rebuild, with the launch configuration the benchmark takes
(the persisted tuning table, if there is one).  It runs in
split-BF16 and in FP32.  The coefficient input is checked against the
oracle's FP64 DCT rounded to FP32.  Every coefficient of every block of the
output is compared with the FP64 oracle's DCT(filter(pixels)) (absolute
tolerance 5e-3 split-BF16, 2e-3 FP32), and the uint8 pixels of the filtered
output (the library's inverse DCT and rounding, eq. 3 and Sec. III) with the
oracle's rounding of the spatially filtered pixels wherever the oracle's
value is not within 1e-3 of a .5 boundary.
"""
import numpy as np
import pytest
import torch

import bench
import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu

FP32, SPLIT = 0, 1
TOL = {FP32: 2e-3, SPLIT: 5e-3}
IMAGES, SIDE, N = 64, 2048, 8


@pytest.fixture(scope="module")
def dctf():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1710_07193_amd as m
    return m


def test_headline_batch_full_size(dctf):
    from paper_1710_07193_amd import tuning
    fronts0 = dctf.dctf_get_batch_fronts()
    v0 = {p: dctf.dctf_get_variant(N, p) for p in (FP32, SPLIT)}
    c0 = {p: dctf.dctf_get_batch_config(p) for p in (FP32, SPLIT)}
    # the launch configuration the bench runs: built-in defaults, then the persisted tuning table
    dctf.dctf_set_batch_fronts(-1)
    for p in (FP32, SPLIT):
        dctf.dctf_set_variant(N, p, 0)
    tuning.apply_table()
    try:
        X, Y, B, pool, draws, ops, jobs = bench.headline_jobs(dctf, torch, IMAGES, SIDE, N)
        assert B == 4194304 and len(jobs) == IMAGES
        per = (SIDE // N) ** 2 * N * N
        Yf = torch.full_like(X, float("nan"))
        jobs_f = [(op, Xi, Yf[i * per:(i + 1) * per]) for i, (op, Xi, _) in enumerate(jobs)]
        Y.fill_(float("nan"))
        out = {}
        for prec, js, Yp in ((SPLIT, jobs, Y), (FP32, jobs_f, Yf)):
            b = dctf.dctf_batch_create(js, prec)
            dctf.dctf_batch_run(b, dctf.DCTF_RUN_REBUILD_OPERATORS)
            pix = torch.empty(X.numel(), dtype=torch.uint8, device="cuda")
            dctf.dctf_idct_u8_verify(N, Yp, pix)
            torch.cuda.synchronize()
            out[prec] = (Yp.cpu().numpy().reshape(IMAGES, -1, N, N), pix.cpu().numpy().reshape(IMAGES, -1, N, N))
            del b, pix
        Xh = X.cpu().numpy().reshape(IMAGES, -1, N, N)
        del X, Y, Yf, jobs, jobs_f

        worst = {FP32: 0.0, SPLIT: 0.0}
        mism = {FP32: 0, SPLIT: 0}
        near = 0
        for i in range(IMAGES):
            px = oracle.tile_u8(syn.image_u8(1000 + i, SIDE, SIDE), N)
            # the coefficient input: the oracle's FP64 DCT rounded once to FP32, up to the
            # summation order of the FP64 sums (a few units in the last place)
            ref = oracle.coeffs_fp32(px)
            diff = np.abs(Xh[i].astype(np.float64) - ref)
            assert diff.max() <= 4 * np.spacing(np.float32(255 * N)), i
            big = np.abs(ref) > 1e-3
            assert np.all(diff[big] <= 2 * np.spacing(np.abs(ref[big]).astype(np.float32))), i
            spec = pool[draws[i]]
            Yref, u8ref, nh = oracle.filter_pixels(px, spec.mask, spec.border)
            near += int(nh.sum())
            for prec in (SPLIT, FP32):
                Yg, pg = out[prec][0][i], out[prec][1][i]
                err = np.abs(Yg - Yref)
                worst[prec] = max(worst[prec], float(err.max()))
                assert err.max() <= TOL[prec], (prec, i, float(err.max()), np.unravel_index(err.argmax(), err.shape))
                bad = (pg != u8ref) & ~nh
                mism[prec] += int(bad.sum())
        assert mism[SPLIT] == 0 and mism[FP32] == 0, mism
        print("headline parity: max |dY| split %.3g, fp32 %.3g; uint8 mismatches outside the band %s; "
              "oracle near-1/2 pixels %d of %d" % (worst[SPLIT], worst[FP32], mism, near, B * N * N))
    finally:
        dctf.dctf_set_batch_fronts(fronts0)
        for p in (FP32, SPLIT):
            dctf.dctf_set_variant(N, p, v0[p])
            dctf.dctf_set_batch_config(p, c0[p])
