"""CPU checks of the tuning table and the batch configuration calls (host
validation only; no device work)."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def dctf():
    import paper_1710_07193_amd as m
    return m


def test_persisted_table_is_valid(dctf):
    from paper_1710_07193_amd import tuning
    table = tuning.load()
    if table is None:
        pytest.skip("no persisted table")
    tuning.validate(table)
    for prec in ("split-bf16", "fp32"):
        assert "batch/N8/" + prec in table["entries"]
        e = table["entries"]["batch/N8/" + prec]
        cands = dctf.dctf_batch_autotune_candidates()
        timed = [c for c in e["candidates"] if c["ms"] > 0]
        assert min(c["ms"] for c in timed) == pytest.approx(e["ms_per_launch"])


def test_validate_rejects_bad_entries(dctf):
    from paper_1710_07193_amd import tuning
    with pytest.raises(ValueError):
        tuning.validate({"entries": {"batch/N8/split-bf16": {"config": dict(fronts=2, io=5, nt=0, groups_per_cu=0)}}})
    with pytest.raises(ValueError):
        tuning.validate({"entries": {"filter/N8/fp32": {"variant": "no_such_variant"}}})
    with pytest.raises(ValueError):
        tuning.validate({"entries": {"gemm/N8/fp32": {}}})
    tuning.validate({"entries": {"filter/N16/split-bf16": {"variant": dctf.dctf_variant_name(16, 1, 0)}}})


def test_batch_config_host_validation(dctf):
    lib = dctf.raw_library()
    saved = dctf.dctf_get_batch_config(1)
    try:
        for bad in ((-2, 0, 0, 0), (2, 3, 0, 0), (2, 1, 2, 0), (2, 1, 0, -1), (2, 1, 0, 65)):
            c = dctf._BatchConfig(*bad)
            assert lib.dctf_set_batch_config(1, ctypes.byref(c)) == -1, bad
        c = dctf._BatchConfig(1, 2, 1, 3)
        assert lib.dctf_set_batch_config(7, ctypes.byref(c)) == -1
        assert lib.dctf_set_batch_config(1, ctypes.byref(c)) == 0
        assert dctf.dctf_get_batch_config(1) == dict(fronts=1, io=2, nt=1, groups_per_cu=3)
        assert lib.dctf_batch_set_config(None, ctypes.byref(c)) == -1
        assert lib.dctf_batch_get_config(None, None, None) == -1
        assert lib.dctf_batch_autotune(None, 0, 1, 1, None, 0, None, None, None) == -1
    finally:
        dctf.dctf_set_batch_config(1, saved)


def test_builtin_candidates_cover_every_io_path(dctf):
    cands = dctf.dctf_batch_autotune_candidates()
    assert {(c["io"], c["nt"]) for c in cands} == {(0, 0), (1, 0), (1, 1), (2, 0), (2, 1)}
    assert {c["fronts"] for c in cands} == {1, 2, 3, 4, 6, 8}
    assert {c["groups_per_cu"] for c in cands} == {0, -1}


def test_kernel_source_hash_ignores_comments_only():
    """The traffic record is keyed by a hash of the kernel sources without
    their comments: a comment edit keeps it, a code edit changes it."""
    import bench
    code = 'int f(int x) { return x + 1; } // one\n/* two\n three */\nconst char *s = "a // b";\n'
    base = bench.strip_comments(code)
    assert "one" not in base and "three" not in base and '"a // b"' in base
    assert bench.strip_comments(code.replace("// one", "// other words")) == base
    assert bench.strip_comments(code.replace("x + 1", "x + 2")) != base
