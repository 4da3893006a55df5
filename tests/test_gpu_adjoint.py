"""GPU adjoint of the step (noise held fixed) against the oracle's
complex-step derivative and against central finite differences of the GPU
forward: gradient of J = sum_q w_q (S(q) - S*(q))^2 with respect to
(tau_s, tau_d, G), S* from a twin run at (tau_s, tau_d, G) x (1.05, 0.95, 1.1)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from gpu_util import say
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1808_05168_amd as F
    F.load()
    return F


def target(rep, horizon, every, field):
    twin = dataclasses.replace(rep, tau_s=rep.tau_s * 1.05, tau_d=rep.tau_d * 0.95, G=rep.G * 1.1)
    f = O.init_state(twin)
    acc = O.Accum(twin.Lx, twin.Lz)
    O.run(twin, f, 0, horizon, acc, sample_every=every)
    S = O.structure_factor(acc)[field]
    w = np.ones_like(S)
    w[:, 0] = 0.0
    return S, w


SMALL = W.Replica(Lx=32, Lz=16, grad_c0=5e-3, kT=1e-4, G=0.5, tau_s=0.7, tau_d=0.8, seed=3)


@pytest.mark.parametrize("field", [0, 1])
def test_adjoint_matches_complex_step_small(F, field):
    rep, H, every = SMALL, 120, 10
    say(f"case: adjoint 32x16 horizon {H} field {field}")
    S_t, w = target(rep, H, every, field)
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J, g = lat.sq_misfit_gradient(S_t, w, H, ckpt_every=25, field=field)
    J_o = O.sq_misfit(rep, H, every, field, S_t, w)
    assert abs(J - J_o) <= 1e-10 * abs(J_o)
    cs = np.array([O.sq_misfit_complex_step(rep, H, every, field, S_t, w, k) for k in range(3)])
    say(f"  adjoint {g}  complex-step {cs}")
    np.testing.assert_allclose(g, cs, rtol=1e-7, atol=1e-9 * np.abs(cs).max())


def test_adjoint_independent_of_checkpoint_interval(F):
    rep, H, every = SMALL, 60, 5
    S_t, w = target(rep, H, every, 0)
    res = []
    for K in (1, 7, 25, 60, 100):
        lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
        res.append(lat.sq_misfit_gradient(S_t, w, H, ckpt_every=K))
    for J, g in res[1:]:
        assert J == res[0][0]
        np.testing.assert_array_equal(g, res[0][1])


def test_adjoint_leaves_handle_untouched(F):
    rep, H, every = SMALL, 40, 5
    S_t, w = target(rep, H, every, 0)
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    lat.step(13)
    f = lat.read_populations(0)
    a2 = lat.read_structure_factor(0, 0)[0]
    lat.sq_misfit_gradient(S_t, w, H, ckpt_every=10)
    assert lat.time == 13
    np.testing.assert_array_equal(lat.read_populations(0), f)
    np.testing.assert_array_equal(lat.read_structure_factor(0, 0)[0], a2)


def test_autograd_function(F):
    import torch
    rep, H, every = SMALL, 60, 10
    S_t, w = target(rep, H, every, 0)
    theta = torch.tensor([rep.tau_s, rep.tau_d, rep.G], dtype=torch.float64, requires_grad=True)
    J = F.sq_misfit(theta, rep, S_t, w, H, every, ckpt_every=20)
    J.backward()
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J2, g = lat.sq_misfit_gradient(S_t, w, H, ckpt_every=20)
    assert float(J.detach()) == J2
    np.testing.assert_array_equal(theta.grad.numpy(), g)


def test_adjoint_256x128_horizon_2000(F):
    """256 x 128, G = 0.5, grad c0 = 1e-3, kT = 1e-5, tau_s = 0.7, tau_d = 0.8,
    2000 steps sampled every 10, checkpoints every 100: adjoint vs central
    differences of the GPU forward (h = 1e-6 relative) and vs the oracle's
    complex-step derivative."""
    rep, H, every = W.adjoint_256x128(), 2000, 10
    say("case: adjoint 256x128 horizon 2000")
    S_t, w = target(rep, H, every, 0)
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J, g = lat.sq_misfit_gradient(S_t, w, H, ckpt_every=100)
    fd = []
    for name in ("tau_s", "tau_d", "G"):
        v = getattr(rep, name)
        h = 1e-6 * v
        Js = []
        for sgn in (1, -1):
            r = dataclasses.replace(rep, **{name: v + sgn * h})
            lt = F.Lattice([r], precision=F.FP64, sample_every=every)
            Js.append(lt.sq_misfit_gradient(S_t, w, H, ckpt_every=100)[0])
        fd.append((Js[0] - Js[1]) / (2 * h))
    fd = np.array(fd)
    say(f"  adjoint {g}  central differences {fd}")
    np.testing.assert_allclose(g, fd, rtol=1e-5)
    cs = np.array([O.sq_misfit_complex_step(rep, H, every, 0, S_t, w, k) for k in range(3)])
    say(f"  complex-step {cs}")
    np.testing.assert_allclose(g, cs, rtol=1e-7)


# ------------------------------------------------- pressure-profile misfit

def p_target(rep, horizon, every):
    """Target row profile of P - P_ref from a twin run at (tau_s, tau_d, G) x
    (1.05, 0.95, 1.1); row weights 0.5 .. 1.5."""
    twin = dataclasses.replace(rep, tau_s=rep.tau_s * 1.05, tau_d=rep.tau_d * 0.95, G=rep.G * 1.1)
    f = O.init_state(twin)
    acc = O.Accum(twin.Lx, twin.Lz)
    O.run(twin, f, 0, horizon, acc, sample_every=every)
    return acc.prof / acc.n_samples, np.linspace(0.5, 1.5, rep.Lz)


def test_pressure_adjoint_matches_complex_step_small(F):
    rep, H, every = SMALL, 120, 10
    say(f"case: pressure adjoint 32x16 horizon {H}")
    P_t, w = p_target(rep, H, every)
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J, g = lat.pressure_misfit_gradient(P_t, w, H, ckpt_every=25)
    J_o = O.p_misfit(rep, H, every, P_t, w)
    assert abs(J - J_o) <= 1e-10 * abs(J_o)
    cs = np.array([O.p_misfit_complex_step(rep, H, every, P_t, w, k) for k in range(3)])
    say(f"  adjoint {g}  complex-step {cs}")
    np.testing.assert_allclose(g, cs, rtol=1e-7, atol=1e-9 * np.abs(cs).max())


def test_pressure_adjoint_256x128_horizon_2000(F):
    """256 x 128 over 2000 steps sampled every 10, checkpoints every 100:
    the pressure-profile gradient against central differences of the GPU
    forward (h = 1e-6 relative) and the oracle's complex-step derivative."""
    rep, H, every = W.adjoint_256x128(), 2000, 10
    say("case: pressure adjoint 256x128 horizon 2000")
    P_t, w = p_target(rep, H, every)
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J, g = lat.pressure_misfit_gradient(P_t, w, H, ckpt_every=100)
    fd = []
    for name in ("tau_s", "tau_d", "G"):
        v = getattr(rep, name)
        h = 1e-6 * v
        Js = []
        for sgn in (1, -1):
            r = dataclasses.replace(rep, **{name: v + sgn * h})
            lt = F.Lattice([r], precision=F.FP64, sample_every=every)
            Js.append(lt.pressure_misfit_gradient(P_t, w, H, ckpt_every=100)[0])
        fd.append((Js[0] - Js[1]) / (2 * h))
    fd = np.array(fd)
    say(f"  adjoint {g}  central differences {fd}")
    np.testing.assert_allclose(g, fd, rtol=1e-5)
    cs = np.array([O.p_misfit_complex_step(rep, H, every, P_t, w, k) for k in range(3)])
    say(f"  complex-step {cs}")
    np.testing.assert_allclose(g, cs, rtol=1e-7)


def test_pressure_autograd_function(F):
    import torch
    rep, H, every = SMALL, 60, 10
    P_t, w = p_target(rep, H, every)
    theta = torch.tensor([rep.tau_s, rep.tau_d, rep.G], dtype=torch.float64, requires_grad=True)
    J = F.p_misfit(theta, rep, P_t, w, H, every, ckpt_every=20)
    J.backward()
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J2, g = lat.pressure_misfit_gradient(P_t, w, H, ckpt_every=20)
    assert float(J.detach()) == J2
    np.testing.assert_array_equal(theta.grad.numpy(), g)


def test_step_vjp_dot_product(F):
    """Dot-product test of one adjoint step: for random y and x,
    <(df(t+1)/df(t))^T y, x> from the adjoint kernels equals <y, A x> with A x
    by central differences of the forward step (FP64, the noise of step t
    reused), and the parameter partials y . df(t+1)/dtheta equal central
    differences in tau_s, tau_d and G."""
    rep = SMALL
    say("case: step VJP dot product 32x16 at t = 30")
    lat = F.Lattice([rep], precision=F.FP64, sample_every=0)
    lat.step(30)
    t = lat.time
    f = lat.read_populations(0)
    _, wts, _, _ = O.tables()
    rng = np.random.default_rng(8)
    y = rng.standard_normal(f.shape)
    x = rng.standard_normal(f.shape) * 1e-3 * wts[None, :, None, None]
    ATy, dth = lat.step_vjp(y)
    assert lat.time == t
    np.testing.assert_array_equal(lat.read_populations(0), f)

    def one_step(g):
        lat.write_populations(0, g)
        lat.time = t
        lat.step(1)
        return lat.read_populations(0)

    eps = 1e-4
    Ax = (one_step(f + eps * x) - one_step(f - eps * x)) / (2 * eps)
    lhs, rhs = float(np.vdot(y, Ax)), float(np.vdot(ATy, x))
    say(f"  <y, Ax> = {lhs:.12e}  <A^T y, x> = {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)
    # parameter partials
    for k, name in enumerate(("tau_s", "tau_d", "G")):
        h = 1e-5 * max(abs(getattr(rep, name)), 1.0)
        outs = []
        for sgn in (1, -1):
            lat.reinit([dataclasses.replace(rep, **{name: getattr(rep, name) + sgn * h})])
            outs.append(one_step(f))
        fd = float(np.vdot(y, (outs[0] - outs[1]) / (2 * h)))
        say(f"  d/d{name}: adjoint {dth[k]:.10e}  differences {fd:.10e}")
        assert abs(dth[k] - fd) <= 1e-6 * abs(fd)


def test_misfit_forward_and_backward_halves(F):
    """fnlb_sq_misfit (J only) and fnlb_misfit_backward give exactly what the
    combined call gives, the backward half can be repeated, and it refuses
    once the handle's time has moved."""
    rep, H, every = SMALL, 60, 10
    S_t, w = target(rep, H, every, 0)
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    J2, g2 = lat.sq_misfit_gradient(S_t, w, H, ckpt_every=20)
    J = lat.sq_misfit(S_t, w, H, ckpt_every=20)
    assert J == J2
    np.testing.assert_array_equal(lat.misfit_backward(), g2)
    np.testing.assert_array_equal(lat.misfit_backward(), g2)
    lat.step(1)
    with pytest.raises(F.FnlbError):
        lat.misfit_backward()
    P_t, pw = p_target(rep, H, every)
    lat2 = F.Lattice([rep], precision=F.FP64, sample_every=every)
    Jp2, gp2 = lat2.pressure_misfit_gradient(P_t, pw, H, ckpt_every=20)
    assert lat2.pressure_misfit(P_t, pw, H, ckpt_every=20) == Jp2
    np.testing.assert_array_equal(lat2.misfit_backward(), gp2)


def test_reinit_equals_fresh_handle(F):
    """fnlb_reinit with new parameters and seed is a fresh start: the same
    populations and sums as a new handle, bit for bit, graphs included."""
    reps = [W.Replica(Lx=64, Lz=16, grad_c0=5e-3, kT=1e-4, G=0.5, seed=41),
            W.Replica(Lx=100, Lz=20, grad_c0=2e-3, kT=1e-4, seed=42)]
    new = [dataclasses.replace(reps[0], tau_s=0.7, G=0.3, seed=43),
           dataclasses.replace(reps[1], grad_c0=4e-3, kT=2e-5, seed=44)]
    for prec in (F.FP64, F.FP32_DEV):
        a = F.Lattice(reps, precision=prec, sample_every=5)
        a.step(27)
        a.reinit(new)
        assert a.time == 0
        a.step(33)
        b = F.Lattice(new, precision=prec, sample_every=5)
        b.step(33)
        for i in range(2):
            np.testing.assert_array_equal(a.read_populations(i), b.read_populations(i))
            for fld in range(2):
                for u, v in zip(a.read_structure_factor(i, fld), b.read_structure_factor(i, fld)):
                    np.testing.assert_array_equal(u, v)
        with pytest.raises(F.FnlbError):
            a.reinit([dataclasses.replace(reps[0], Lx=32), reps[1]])
        with pytest.raises(F.FnlbError):
            a.reinit(new[:1])
