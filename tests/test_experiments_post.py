"""Post-processing of the accumulated sums (mean row profiles from the k_x = 0
column, real-space correlations from S(q)), checked on CPU against direct
computations on the oracle's own sampled fields."""
import numpy as np
import pytest

import workloads as W
from paper_1808_05168_amd import experiments as X


def _random_state(ora, rep, seed):
    rng = np.random.default_rng(seed)
    _, w, _, _ = ora.tables()
    f = np.empty((2, 9, rep.Lz, rep.Lx))
    for s in range(2):
        for l in range(9):
            f[s, l] = w[l] * (0.5 + 0.05 * rng.standard_normal((rep.Lz, rep.Lx)))
    return f


@pytest.mark.parametrize("Lx,Lz", [(16, 8), (12, 10)])
def test_mean_row_profile_from_fourier_sums(ora, Lx, Lz):
    rep = W.Replica(Lx=Lx, Lz=Lz, grad_c0=0.01, G=0.3)
    flags = ora.DEFAULT_FLAGS | ora.VELOCITY
    acc = ora.Accum(Lx, Lz, nfields=4)
    rows = np.zeros((4, Lz))
    for k in range(3):
        f = _random_state(ora, rep, 10 + k)
        ora.sample(rep, f, acc, flags=flags)
        _, dphi = ora.fields(rep, f, flags=flags)
        rows += dphi.mean(axis=2)
    rows /= 3
    for fld in range(4):
        prof = X.mean_row_profile(acc.sq[fld, 1], acc.sq[fld, 2], acc.n_samples, Lx)
        np.testing.assert_allclose(prof, rows[fld], rtol=0, atol=1e-15)


@pytest.mark.parametrize("Lx,Lz", [(16, 8), (9, 7)])
def test_correlation_is_the_circular_autocorrelation(ora, Lx, Lz):
    rep = W.Replica(Lx=Lx, Lz=Lz, grad_c0=0.01)
    f = _random_state(ora, rep, 3)
    acc = ora.Accum(Lx, Lz)
    ora.sample(rep, f, acc)
    _, dphi = ora.fields(rep, f)
    for fld in range(2):
        # one sample: the raw |Phi|^2 is the periodogram of the field itself
        C = X.correlation(acc.sq[fld, 0], Lx)
        d = dphi[fld]
        direct = np.empty((Lz, Lx))
        for dz in range(Lz):
            for dx in range(Lx):
                direct[dz, dx] = np.mean(d * np.roll(np.roll(d, -dz, axis=0), -dx, axis=1))
        np.testing.assert_allclose(C, direct, rtol=0, atol=1e-14 * np.abs(direct).max())


def test_scan_replica_table():
    cfgs, reps = X.scan_replicas([8, 16], [0.01, 0.02], kT=1e-4, G=0.3, seeds=3, seed0=7)
    # per L: grads {0, 0.01, 0.02} x (1 cold + 3 thermal)
    assert len(reps) == 2 * 3 * 4
    assert [r.seed for r in reps] == list(range(7, 7 + len(reps)))
    assert all(r.Lx == 4 * r.Lz for r in reps)
    assert sum(1 for c in cfgs if c[2] == 0.0) == 6
    with pytest.raises(ValueError):
        X.scan_replicas([64], [0.02], kT=1e-4, G=0.3)      # L * grad >= 1
    with pytest.raises(ValueError):
        X.scan_replicas([8], [0.01], kT=0.0, G=0.3)
