"""Pins of the oracle's time step against what the paper and the mathematics
fix: exact conservation, pure streaming with bounce-back, the noise-free
relaxation of the imposed concentration profile (diffusion with Neumann
walls), the critical coupling G_c = 2, and the equilibrium spectra predicted
by fluctuation-dissipation (Sec. IV.A)."""
import numpy as np
import pytest

import workloads as W


def test_species_mass_conserved(ora):
    # Per-species mass is an exact invariant (xi_0 = 0, F_0 = 0, bounce-back is
    # a permutation), with noise, non-ideal forcing, walls and the wall fix on.
    rep = W.Replica(Lx=24, Lz=12, grad_c0=5e-3, kT=1e-4, G=0.5, tau_s=0.7,
                    tau_d=0.8, seed=4)
    f = ora.init_state(rep)
    m0 = f.sum(axis=(1, 2, 3))
    ora.run(rep, f, 0, 1000)
    np.testing.assert_allclose(f.sum(axis=(1, 2, 3)), m0, rtol=1e-13, atol=0)


def test_streaming_and_bounce_back(ora):
    """A local equilibrium with a shared velocity field, no force, no noise and
    no wall fix is a fixed point of the collision, so one step is pure
    streaming: f_l(r + c_l) = f_l(r) inside, and a link that would leave
    through a wall comes back reversed at the same node."""
    Lx, Lz = 5, 4
    rep = W.Replica(Lx=Lx, Lz=Lz)
    rng = np.random.default_rng(1)
    c, w, T, N = ora.tables()
    f = np.zeros((2, 9, Lz, Lx))
    for j in range(Lz):
        for x in range(Lx):
            ux, uz = rng.uniform(-0.05, 0.05, 2)
            for s in range(2):
                f[s, :, j, x] = ora.equilibrium(rng.uniform(0.3, 0.7), ux, uz)
    g = f.copy()
    ora.run(rep, g, 1, 1, flags=ora.ASTAR)
    ref = np.zeros_like(f)
    opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
    for s in range(2):
        for l in range(9):
            for j in range(Lz):
                for x in range(Lx):
                    jd = j + c[l, 1]
                    if 0 <= jd < Lz:
                        ref[s, l, jd, (x + c[l, 0]) % Lx] = f[s, l, j, x]
                    else:
                        ref[s, opp[l], j, x] = f[s, l, j, x]
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-16)


def _profile_run(ora, flags, L=16, grad=1e-3):
    rep = W.Replica(Lx=4, Lz=L, grad_c0=grad)
    c, w, T, N = ora.tables()
    f = np.zeros((2, 9, L, 4))
    for s in range(2):
        for l in range(9):
            f[s, l] = w[l] * 0.5      # uniform c = 1/2, rho = 1, at rest
    z = np.arange(L) - 0.5 * (L - 1)
    ts, amps = [], []
    t = 0
    for _ in range(30):
        ora.run(rep, f, t, 50, flags=flags)
        t += 50
        rho, _ = ora.fields(rep, f)
        prof = (rho[0] / (rho[0] + rho[1])).mean(axis=1)
        amps.append(((prof - (0.5 + z * grad)) * np.sin(np.pi * z / L)).sum() * 2 / L)
        ts.append(t)
    ora.run(rep, f, t, 5000, flags=flags)
    rho, _ = ora.fields(rep, f)
    prof = (rho[0] / (rho[0] + rho[1])).mean(axis=1)
    return z, prof, np.array(ts), np.array(amps)


def test_noise_free_profile_relaxes_to_imposed_gradient(ora):
    """G = 0, kT = 0, start from c = 1/2: c - c_0 obeys the diffusion equation
    with zero flux at the walls (Eq. (26) with grad c_0 imposed by Eq. (12)),
    so the slowest mode decays at D (pi/L)^2 with D from Eq. (28), and the
    steady state is c = c_0(z) exactly (an exact discrete fixed point)."""
    L, grad = 16, 1e-3
    z, prof, ts, amps = _profile_run(ora, ora.DEFAULT_FLAGS, L, grad)
    np.testing.assert_allclose(prof, 0.5 + z * grad, rtol=0, atol=1e-13)
    rate = -np.polyfit(ts[5:], np.log(np.abs(amps[5:])), 1)[0]
    D = (1.0 - 0.5) / 3
    assert abs(rate / (D * (np.pi / L) ** 2) - 1) < 1e-3


def test_literal_first_order_forcing_misses_the_gradient(ora):
    # The same run with (F_1, F_2) = rho a (no (1 - lambda_d/2) factor) settles
    # at twice the imposed slope at tau = 1: the pin above rejects it.
    L, grad = 16, 1e-3
    z, prof, _, _ = _profile_run(ora, ora.DEFAULT_FLAGS | ora.FORCE_LITERAL, L, grad)
    slope = np.polyfit(z, prof, 1)[0]
    assert abs(slope / grad - 2) < 1e-6


def test_critical_coupling(ora, ):
    """Without the a_* correction the mixture demixes above G_c = 2 (Sec. IV.C:
    the critical point corresponds to G = 2) and stays mixed below."""
    stds = {}
    for G in (1.8, 2.3):
        rep = W.Replica(Lx=32, Lz=32, kT=1e-6, G=G, seed=3)
        f = ora.init_state(rep, flags=0)
        ora.run(rep, f, 0, 3000, flags=0)
        _, d = ora.fields(rep, f)
        stds[G] = d[0].std()
    thermal = np.sqrt(0.75e-6)
    assert stds[1.8] < 2 * thermal
    assert stds[2.3] > 0.05


def test_astar_keeps_concentration_ideal(ora):
    # With a_* both species feel the same non-ideal acceleration, so G no
    # longer drives demixing (reading R3): G = 2.3 stays at thermal level.
    rep = W.Replica(Lx=32, Lz=32, kT=1e-6, G=2.3, seed=3)
    f = ora.init_state(rep)
    ora.run(rep, f, 0, 3000)
    _, d = ora.fields(rep, f)
    assert d[0].std() < 1.2 * np.sqrt(0.75e-6)


def test_sampling_schedule(ora):
    # Samples are taken of f(t) for t >= 1 with t % every == 0, before the
    # collision of step t -> t+1.
    rep = W.Replica(Lx=8, Lz=4, kT=1e-5)
    f = ora.init_state(rep)
    acc = ora.Accum(8, 4)
    ora.run(rep, f, 0, 25, acc, sample_every=5)
    assert acc.n_samples == 4           # t = 5, 10, 15, 20
    ora.run(rep, f, 25, 6, acc, sample_every=5)
    assert acc.n_samples == 6           # t = 25, 30


def test_invalid_parameters_rejected(ora):
    ok = W.Replica(Lx=8, Lz=4)
    assert ora.check_params(ok)
    for bad in (dict(Lx=1), dict(Lz=1), dict(tau_d=0.5), dict(tau_s=0.4),
                dict(kT=-1.0), dict(grad_c0=0.3), dict(rho0=0.0), dict(G=-0.1)):
        rep = W.Replica(**{**ok.__dict__, **bad})
        assert not ora.check_params(rep)


@pytest.mark.parametrize("G", [0.0, 0.5])
def test_equilibrium_spectra_flat(ora, G):
    """Sec. IV.A, Eqs. (31)-(32): at grad c_0 = 0, S_c = 3 kT c(1-c)/rho = 3kT/4
    and S_Ux = kT/rho, independent of q (walls included).  S_Uz is checked with
    the wall fix off (test_density_spectrum_fdt_without_wall_fix): the fix
    zeroes U_z on the wall rows."""
    Lx, Lz, kT = 32, 16, 1e-4
    flags = ora.DEFAULT_FLAGS | ora.VELOCITY
    rep = W.Replica(Lx=Lx, Lz=Lz, kT=kT, G=G, seed=7)
    f = ora.init_state(rep, flags=flags)
    ora.run(rep, f, 0, 400, flags=flags)
    acc = ora.Accum(Lx, Lz, nfields=4)
    ora.run(rep, f, 400, 3000, acc, flags=flags, sample_every=10)
    S = ora.structure_factor(acc)
    mask = np.ones(S[0].shape, bool)
    mask[0, 0] = False
    assert abs(S[0][mask].mean() / (0.75 * kT) - 1) < 0.02
    # flat: the k_x-resolved means stay within sampling error of the level
    kx_means = S[0][:, 1:].mean(axis=0) / (0.75 * kT)
    assert np.all(np.abs(kx_means - 1) < 0.12)
    assert abs(S[2][mask].mean() / kT - 1) < 0.04
    # the velocity spectrum is flat along q = (q, 0) as well (at G > 0 the
    # non-ideal force lowers it by ~13% in the top third of the band, a lattice
    # effect of the forcing, so the band check runs on the ideal mixture),
    # except at k_x = Lx/2: there streaming flips the sign of the total
    # x-momentum mode and a force-free collision conserves it, so it keeps its
    # initial value 0
    if G == 0.0:
        assert np.all(np.abs(S[2][0, 1:Lx // 2].reshape(3, -1).mean(axis=1) / kT - 1) < 0.12)
        assert S[2][0, Lx // 2] < 1e-3 * kT
    # the velocity fields are the barycentric U of the state, wall fix applied
    _, dphi = ora.fields(rep, f, flags=flags)
    np.testing.assert_array_equal(dphi[2:], ora.velocity(rep, f, flags=flags))


def test_density_spectrum_fdt_without_wall_fix(ora):
    """Derived from the lattice FDT that Eqs. (22)-(23) encode: at G = 0 the
    total density spectrum is S_rho = 3 kT rho_bar (compressibility of the
    ideal EOS, Eq. (24)) for q != 0, and S_rho(0) = 0 by mass conservation.
    The wall U_z fix is a deterministic projection without matching noise, so
    this check runs with the fix off; so does the check of S_Uz = kT/rho
    (Eq. (31))."""
    Lx, Lz, kT = 32, 16, 1e-4
    flags = ora.ASTAR | ora.VELOCITY
    rep = W.Replica(Lx=Lx, Lz=Lz, kT=kT, seed=7)
    f = ora.init_state(rep, flags=flags)
    ora.run(rep, f, 0, 1000, flags=flags)
    acc = ora.Accum(Lx, Lz, nfields=4)
    ora.run(rep, f, 1000, 4000, acc, flags=flags, sample_every=10)
    S = ora.structure_factor(acc)
    mask = np.ones(S[1].shape, bool)
    mask[0, 0] = False
    assert abs(S[1][mask].mean() / (3 * kT) - 1) < 0.02
    assert S[1][0, 0] < 1e-20
    assert abs(S[2][mask].mean() / kT - 1) < 0.04
    assert abs(S[3][mask].mean() / kT - 1) < 0.04


def test_wall_rule_zeroes_normal_velocity(ora):
    """Sec. III.A: on the two wall rows the normal barycentric velocity is set
    to zero at every step by readjusting the rest population (reading R7).
    Checked from the populations the collision receives, recomputed here:
    rho U_z = sum_s sum_l c_lz f^S_l + (F^A_z + F^B_z)/2 vanishes on rows 0
    and L-1, each species keeps its mass, only f_0 and the bounced-back normal
    population (f_2 at the bottom, f_4 at the top) change, the change is split
    between species in proportion to rho^S/rho, and nothing changes in the
    bulk.  A sign slip in the fix at either wall doubles rho U_z there."""
    Lx, Lz = 12, 8
    rep = W.Replica(Lx=Lx, Lz=Lz, grad_c0=5e-3, kT=1e-4, G=0.5, tau_s=0.7, tau_d=0.8,
                    seed=11)
    c, w, T, N = ora.tables()
    cz = c[:, 1]
    f = ora.init_state(rep)
    ora.run(rep, f, 0, 40)
    # a state away from any stationary one, so that the walls carry momentum
    f = f + 1e-3 * np.random.default_rng(5).standard_normal(f.shape) * w[None, :, None, None]
    fl, F, U = ora.macros(rep, f)
    rho_s = f.sum(axis=1)
    jz = lambda g: np.einsum("l,slzx->zx", cz, g)
    Fz = F[0, 1] + F[1, 1]
    Pi_before = jz(f) + 0.5 * Fz
    Pi_after = jz(fl) + 0.5 * Fz
    # what is left is the rounding of these sums: a few ulps of the magnitudes
    # that enter them (about 3e-17 here, against >= 1e-7 before the fix)
    scale = np.einsum("l,slzx->zx", np.abs(cz), np.abs(fl)) + 0.5 * (np.abs(F[0, 1]) +
                                                                     np.abs(F[1, 1]))
    tol = 8 * np.finfo(float).eps * scale
    r = rho_s.sum(axis=0)
    for row in (0, Lz - 1):
        assert np.abs(Pi_before[row]).min() > 1e-7        # the fix has work to do
        assert (np.abs(Pi_after[row]) <= tol[row]).all()
        assert (np.abs(U[1, row]) <= tol[row] / r[row]).all()
    # the velocity the collision uses is that of the fixed populations
    assert (np.abs(U[1] - Pi_after / r) <= tol / r).all()
    np.testing.assert_allclose(fl.sum(axis=1), rho_s, rtol=0, atol=4e-16)
    np.testing.assert_array_equal(fl[:, :, 1:Lz - 1], f[:, :, 1:Lz - 1])
    for row, moved in ((0, 2), (Lz - 1, 4)):
        d = fl[:, :, row] - f[:, :, row]
        untouched = [l for l in range(9) if l not in (0, moved)]
        np.testing.assert_array_equal(d[:, untouched], 0.0)
        # the normal population loses rho^S/rho of the excess, f_0 gains it
        share = rho_s[:, row] / r[row]
        sign = -1.0 if row == 0 else 1.0
        np.testing.assert_allclose(d[:, moved], sign * share * Pi_before[row], rtol=1e-9,
                                   atol=1e-19)
        np.testing.assert_allclose(d[:, 0], -d[:, moved], rtol=0, atol=6e-17)
    # with the fix off nothing is touched and the walls keep their momentum
    fl0, _, U0 = ora.macros(rep, f, flags=ora.ASTAR)
    np.testing.assert_array_equal(fl0, f)
    assert np.abs(U0[1, 0]).min() > 1e-8 and np.abs(U0[1, Lz - 1]).min() > 1e-8
