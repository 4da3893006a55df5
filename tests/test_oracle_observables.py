"""Pins of the oracle's observables: the structure-factor transform against
numpy's FFT and Parseval (Appendix, Eqs. (A1)-(A4) with the lattice
normalisation), and the pressure against the equation of state (Eq. (24)) and
mechanical balance (Sec. IV.C)."""
import numpy as np
import pytest

import workloads as W


def _random_state(ora, rep, seed):
    rng = np.random.default_rng(seed)
    c, w, T, N = ora.tables()
    f = np.empty((2, 9, rep.Lz, rep.Lx))
    for s in range(2):
        for l in range(9):
            f[s, l] = w[l] * (0.5 + 0.05 * rng.standard_normal((rep.Lz, rep.Lx)))
    return f


@pytest.mark.parametrize("Lx,Lz", [(16, 8), (12, 10), (9, 7)])
def test_structure_factor_matches_fft_and_parseval(ora, Lx, Lz):
    rep = W.Replica(Lx=Lx, Lz=Lz, grad_c0=0.01)
    f = _random_state(ora, rep, Lx * Lz)
    flags = ora.DEFAULT_FLAGS | ora.VELOCITY
    acc = ora.Accum(Lx, Lz, nfields=4)
    ora.sample(rep, f, acc, flags=flags)
    _, dphi = ora.fields(rep, f, flags=flags)
    nkx = Lx // 2 + 1
    for fld in range(4):
        Phi = np.fft.fft2(dphi[fld]) / np.sqrt(Lx * Lz)   # [kz][kx]
        np.testing.assert_allclose(acc.sq[fld, 1], Phi.real[:, :nkx], atol=1e-15)
        np.testing.assert_allclose(acc.sq[fld, 2], Phi.imag[:, :nkx], atol=1e-15)
        np.testing.assert_allclose(acc.sq[fld, 0], np.abs(Phi[:, :nkx]) ** 2, rtol=1e-12,
                                   atol=1e-30)
        # Parseval over the full spectrum rebuilt from the half spectrum
        wgt = np.full(nkx, 2.0)
        wgt[0] = 1.0
        if Lx % 2 == 0:
            wgt[-1] = 1.0
        total = (acc.sq[fld, 0] * wgt).sum()
        assert abs(total / (dphi[fld] ** 2).sum() - 1) < 1e-12


def test_delta_fields_definition(ora):
    # delta c = rho^A / rho - c_0(z) (Fig. 1 profile) and delta rho = rho - rho_bar
    rep = W.Replica(Lx=6, Lz=5, grad_c0=0.02)
    f = _random_state(ora, rep, 2)
    rho, dphi = ora.fields(rep, f)
    z = np.arange(5) - 2.0
    np.testing.assert_allclose(dphi[0], rho[0] / (rho[0] + rho[1]) - (0.5 + 0.02 * z)[:, None],
                               atol=1e-16)
    np.testing.assert_allclose(dphi[1], rho[0] + rho[1] - 1.0, atol=1e-16)
    np.testing.assert_allclose(rho, f.sum(axis=1), atol=1e-16)


@pytest.mark.parametrize("G,ra,rb", [(0.0, 0.5, 0.5), (0.5, 0.6, 0.45), (1.3, 0.2, 0.9)])
def test_pressure_of_uniform_state_is_eos(ora, G, ra, rb):
    # Eq. (24): P = (rho^A + rho^B)/3 + G rho^A rho^B / 3 on a uniform state;
    # P_ref is the same EOS at rho^A = rho^B = rho_bar / 2.
    rep = W.Replica(Lx=8, Lz=6, G=G)
    c, w, T, N = ora.tables()
    f = np.empty((2, 9, 6, 8))
    for l in range(9):
        f[0, l] = w[l] * ra
        f[1, l] = w[l] * rb
    acc = ora.Accum(8, 6)
    ora.sample(rep, f, acc)
    expect = (ra + rb) / 3 + G * ra * rb / 3 - (1.0 / 3 + G / 12)
    assert abs(acc.pr[0] - expect) < 1e-15
    assert abs(acc.pr[1] - expect ** 2) < 1e-15
    np.testing.assert_allclose(acc.prof, expect, atol=1e-15)


def test_noise_free_pressure_is_homogeneous(ora):
    """Sec. IV.C: the total pressure of the steady state is z-independent.
    Noise-free run at G = 0.5 with grad c_0 = 0.01: the ideal and interaction
    parts each vary by ~7e-4 across the channel, their sum is flat in the bulk
    (three rows away from the ghost-row wall layers) to 1e-4 of that."""
    L, G, grad = 16, 0.5, 0.01
    rep = W.Replica(Lx=4, Lz=L, grad_c0=grad, G=G)
    f = ora.init_state(rep)
    ora.run(rep, f, 0, 20000)
    acc = ora.Accum(4, L)
    ora.sample(rep, f, acc)
    rho, _ = ora.fields(rep, f)
    ideal = (rho[0] + rho[1]).mean(axis=1) / 3
    bulk = acc.prof[3:-3]
    assert np.ptp(ideal) > 5e-4
    assert np.ptp(bulk) < 1e-4 * np.ptp(ideal)
    # and the concentration sits on the imposed profile
    z = np.arange(L) - 0.5 * (L - 1)
    c = (rho[0] / (rho[0] + rho[1])).mean(axis=1)
    assert np.abs(c - (0.5 + grad * z)).max() < 1e-5


def test_ideal_mixture_pressure_has_no_thermal_shift(ora):
    # Sec. IV.C: at G = 0 the mean pressure is not shifted by kT (mass is
    # conserved, P = rho/3).
    rep = W.Replica(Lx=16, Lz=8, grad_c0=0.01, kT=1e-4, seed=2)
    f = ora.init_state(rep)
    acc = ora.Accum(16, 8)
    ora.run(rep, f, 0, 200, acc, sample_every=10)
    assert acc.n_samples == 19
    assert abs(acc.pr[0]) < 1e-15 * acc.n_samples
