"""CPU checks of the C ABI: the library builds, loads, exports every function
declared in include/fnlb.h, and validates parameters without touching a GPU."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fnlb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fnlb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1808_05168_amd import fnlb
    if not os.path.exists(fnlb.LIB_PATH):
        from paper_1808_05168_amd import build
        build.build()
    return fnlb.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1808_05168_amd import fnlb
    assert sorted(fnlb.EXPORTS) == declared_functions()


def test_error_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(lib.fnlb_strerror(code), bytes)


def test_bytes_required_and_validation(lib):
    import paper_1808_05168_amd as F
    s, a, w = F.bytes_required([W.parity_small()])
    # two state copies of 18 FP64 planes of 64 x 32
    assert s == 2 * 18 * 64 * 32 * 8
    # accumulators: 2 fields x 3 sums x 32 x 33 + pressure (2 + 32)
    assert a >= (6 * 32 * 33 + 34) * 8
    s32, _, _ = F.bytes_required([W.parity_small()], precision=F.FP32_DEV)
    assert s32 == s // 2
    bad = [dict(Lx=1), dict(Lz=1), dict(tau_s=0.5), dict(kT=-1.0), dict(grad_c0=0.04),
           dict(Lx=8192), dict(Lx=3000, Lz=10), dict(G=-1.0), dict(rho0=0.0)]
    for b in bad:
        rep = W.Replica(**{**W.parity_small().__dict__, **b})
        with pytest.raises(F.FnlbError):
            F.bytes_required([rep])
    with pytest.raises(F.FnlbError):
        F.bytes_required([W.parity_small()], precision=7)
    with pytest.raises(F.FnlbError):
        F.bytes_required([W.parity_small()], flags=64)
    # no replicas, negative sampling interval or row-range length
    for reps, kw in (([], {}), ([W.parity_small()], dict(sample_every=-1)),
                     ([W.parity_small()], dict(chunk_rows=-2))):
        with pytest.raises(F.FnlbError):
            F.bytes_required(reps, **kw)
    # a row range longer than the lattice is one work item per segment column
    assert F.bytes_required([W.parity_small()], chunk_rows=1000)[0] == s


def test_init_rejects_null_and_small_buffers(lib):
    from paper_1808_05168_amd import fnlb
    p = fnlb.replica_params([W.parity_small()])
    o = fnlb.Options(0, 0, fnlb.DEFAULT_FLAGS, 0)
    h = ctypes.c_void_p()
    rc = lib.fnlb_init(p, 1, ctypes.byref(o), None, 0, None, 0, None, 0, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert lib.fnlb_step(None, 1) == -1
    assert lib.fnlb_destroy(None) == 0


def test_tune_cache_file_round_trip(lib, tmp_path):
    """The autotuner's choices go to a text file keyed by GPU architecture,
    precision and the multiset of lattice shapes, and come back from it; entries
    of another architecture are kept but not used; other files are refused."""
    import paper_1808_05168_amd as F
    a = tmp_path / "a.txt"
    F.tune_cache_save(str(a))
    lines = a.read_text().splitlines()
    assert lines[0] == "fnlb-tune 1" and lines[1].startswith("# device ")
    arch = lines[1][len("# device "):]
    ens = W.batched_ensemble(96)
    key = "1|64x32*24|128x64*24|256x128*24|512x256*24"
    b = tmp_path / "b.txt"
    b.write_text(f"fnlb-tune 1\n{arch}\t{key}\t-32\nsome-other-gpu\t1|64x32*1\t7\n")
    F.tune_cache_load(str(b))
    assert F.tune_lookup(ens, F.FP32_DEV) == (2, 32)
    assert F.tune_lookup(ens, F.FP64) is None
    assert F.tune_lookup([W.parity_small()], F.FP32_DEV) is None
    c = tmp_path / "c.txt"
    c.write_text(f"fnlb-tune 1\nsome-other-gpu\t{key}\t5\n")
    F.tune_cache_save(str(c))
    text = c.read_text()
    assert f"{arch}\t{key}\t-32" in text and "some-other-gpu" in text
    bad = tmp_path / "bad.txt"
    bad.write_text("not a tuning file\n")
    with pytest.raises(F.FnlbError):
        F.tune_cache_load(str(bad))
    with pytest.raises(F.FnlbError):
        F.tune_cache_load(str(tmp_path / "missing.txt"))
