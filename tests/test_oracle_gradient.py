"""The oracle's complex-step gradient of the structure-factor misfit agrees
with central finite differences of the oracle itself (a check of the
complex-step machinery that the GPU adjoint is compared against)."""
import dataclasses

import numpy as np
import pytest

import workloads as W

HORIZON, EVERY = 120, 10


def _case():
    rep = W.Replica(Lx=32, Lz=16, grad_c0=5e-3, kT=1e-4, G=0.5, tau_s=0.7, tau_d=0.8, seed=3)
    return rep


def target_and_weight(ora, rep, horizon=HORIZON, every=EVERY, field=0):
    # target spectrum: a twin run at (tau_s, tau_d, G) x (1.05, 0.95, 1.1), same noise
    twin = dataclasses.replace(rep, tau_s=rep.tau_s * 1.05, tau_d=rep.tau_d * 0.95, G=rep.G * 1.1)
    f = ora.init_state(twin)
    acc = ora.Accum(twin.Lx, twin.Lz)
    ora.run(twin, f, 0, horizon, acc, sample_every=every)
    S_t = ora.structure_factor(acc)[field]
    w = np.ones_like(S_t)
    w[:, 0] = 0.0
    return S_t, w


@pytest.mark.parametrize("which,name", [(0, "tau_s"), (1, "tau_d"), (2, "G")])
def test_complex_step_matches_central_differences(ora, which, name):
    rep = _case()
    S_t, w = target_and_weight(ora, rep)
    J0 = ora.sq_misfit(rep, HORIZON, EVERY, 0, S_t, w)
    assert J0 > 0
    cs = ora.sq_misfit_complex_step(rep, HORIZON, EVERY, 0, S_t, w, which)
    val = getattr(rep, name)
    h = 1e-4 * val
    jp = ora.sq_misfit(dataclasses.replace(rep, **{name: val + h}), HORIZON, EVERY, 0, S_t, w)
    jm = ora.sq_misfit(dataclasses.replace(rep, **{name: val - h}), HORIZON, EVERY, 0, S_t, w)
    fd = (jp - jm) / (2 * h)
    assert abs(cs - fd) <= 1e-6 * abs(cs) + 1e-12 * J0


def pressure_target_and_weight(ora, rep, horizon=HORIZON, every=EVERY):
    # target profile: a twin run at (tau_s, tau_d, G) x (1.05, 0.95, 1.1), same noise
    twin = dataclasses.replace(rep, tau_s=rep.tau_s * 1.05, tau_d=rep.tau_d * 0.95, G=rep.G * 1.1)
    f = ora.init_state(twin)
    acc = ora.Accum(twin.Lx, twin.Lz)
    ora.run(twin, f, 0, horizon, acc, sample_every=every)
    P_t = acc.prof / acc.n_samples
    w = np.linspace(0.5, 1.5, rep.Lz)
    return P_t, w


@pytest.mark.parametrize("which,name", [(0, "tau_s"), (1, "tau_d"), (2, "G")])
def test_pressure_misfit_complex_step_matches_central_differences(ora, which, name):
    rep = _case()
    P_t, w = pressure_target_and_weight(ora, rep)
    J0 = ora.p_misfit(rep, HORIZON, EVERY, P_t, w)
    assert J0 > 0
    cs = ora.p_misfit_complex_step(rep, HORIZON, EVERY, P_t, w, which)
    val = getattr(rep, name)
    h = 1e-4 * val
    jp = ora.p_misfit(dataclasses.replace(rep, **{name: val + h}), HORIZON, EVERY, P_t, w)
    jm = ora.p_misfit(dataclasses.replace(rep, **{name: val - h}), HORIZON, EVERY, P_t, w)
    fd = (jp - jm) / (2 * h)
    assert abs(cs - fd) <= 1e-6 * abs(cs) + 1e-12 * J0


def test_pressure_misfit_is_the_row_profile_misfit(ora):
    """J from the misfit routine equals the same sum formed from a plain run's
    pressure profile accumulator."""
    rep = _case()
    P_t, w = pressure_target_and_weight(ora, rep)
    f = ora.init_state(rep)
    acc = ora.Accum(rep.Lx, rep.Lz)
    ora.run(rep, f, 0, HORIZON, acc, sample_every=EVERY)
    J = float(np.sum(w * (acc.prof / acc.n_samples - P_t) ** 2))
    assert abs(ora.p_misfit(rep, HORIZON, EVERY, P_t, w) - J) <= 1e-14 * J
