"""The entry point that allocates nothing (fnlb_init_static_work): a handle
over the library's static device workspace against one over a caller
workspace (fnlb_init), on the same seeded inputs, through the C ABI.  Two
handles in a row, the second on a smaller input, so that the second runs on
what the first left in the shared array."""
import numpy as np
import pytest

import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1808_05168_amd as F
    F.load()
    return F


def _run(F, reps, precision, every, flags, nsteps, static):
    lat = F.Lattice(reps, precision=precision, sample_every=every, flags=flags,
                    static_work=static)
    lat.step(nsteps)
    out = []
    for i in range(len(reps)):
        sq = [lat.read_structure_factor(i, fld) for fld in range(2)]
        out.append((lat.read_populations(i), sq, lat.read_pressure(i)))
    return lat, out


def _same(a, b):
    for (fa, sqa, pa), (fb, sqb, pb) in zip(a, b):
        np.testing.assert_array_equal(fa, fb)
        for (a2, re, im, n), (b2, bre, bim, m) in zip(sqa, sqb):
            assert n == m and n > 0
            np.testing.assert_array_equal(a2, b2)
            np.testing.assert_array_equal(re, bre)
            np.testing.assert_array_equal(im, bim)
        assert pa[0] == pb[0] and pa[1] == pb[1] and pa[3] == pb[3]
        np.testing.assert_array_equal(pa[2], pb[2])


CASES = [
    # larger first: three replicas, one ragged (direct transforms), FP32
    ("three replicas fp32-dev", [W.Replica(Lx=256, Lz=64, grad_c0=1e-3, kT=1e-5, G=0.5, seed=3),
                                 W.Replica(Lx=100, Lz=20, grad_c0=5e-3, kT=1e-4, G=0.5,
                                           tau_s=0.7, tau_d=0.8, seed=4),
                                 W.Replica(Lx=128, Lz=64, grad_c0=2e-3, kT=1e-5, seed=5)],
     1, 7, 60),
    # then a smaller one in FP64, on what the first left in the array
    ("64x32 fp64", [W.parity_small()], 0, 10, 45),
]


def test_static_work_matches_caller_work():
    import torch
    import paper_1808_05168_amd as F
    assert torch.cuda.is_available()
    for name, reps, prec, every, nsteps in CASES:
        say(f"case: static workspace vs caller workspace, {name}, {nsteps} steps every {every}")
        ls, got = _run(F, reps, prec, every, F.DEFAULT_FLAGS, nsteps, True)
        # one static handle per device at a time
        with pytest.raises(F.FnlbError):
            F.Lattice(reps, precision=prec, sample_every=every, static_work=True)
        ls.close()
        lc, ref = _run(F, reps, prec, every, F.DEFAULT_FLAGS, nsteps, False)
        lc.close()
        _same(got, ref)
    # a workspace beyond the static array's size is refused before any work
    big = W.Replica(Lx=4096, Lz=4096, grad_c0=1e-4, kT=1e-5, seed=9)
    assert F.bytes_required([big], precision=F.FP32_DEV, sample_every=10)[2] > \
        F.STATIC_WORK_BYTES
    with pytest.raises(F.FnlbError, match="smaller than required"):
        F.Lattice([big], precision=F.FP32_DEV, sample_every=10, static_work=True)
