"""The non-equilibrium pressure protocol of Sec. IV.C (Eqs. (41)-(42)) run on
the GPU as one batch, against the same protocol evaluated on the oracle's
runs; and the paper's statement that an ideal mixture (G = 0) shows no
non-equilibrium pressure."""
import numpy as np
import pytest

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


def _oracle_scan(Ls, grads, kT, G, seeds, warm, steps, every):
    from paper_1808_05168_amd import experiments as X
    cfgs, reps = X.scan_replicas(Ls, grads, kT, G, seeds=seeds)
    per = {}
    for c, r in zip(cfgs, reps):
        f = O.init_state(r)
        O.run(r, f, 0, warm)
        acc = O.Accum(r.Lx, r.Lz)
        O.run(r, f, warm, steps, acc, sample_every=every)
        n = acc.n_samples
        rho = X.mean_row_profile(acc.sq[1, 1], acc.sq[1, 2], n, r.Lx)
        per.setdefault(c[:3], []).append((acc.pr[0] / n, acc.prof / n, rho))
    return per


def test_pressure_protocol_matches_oracle(F):
    from paper_1808_05168_amd import experiments as X
    Ls, grads, kT, G, seeds, warm, steps, every = [8, 12], [0.02], 1e-4, 0.3, 2, 60, 100, 5
    say("case: pressure protocol L=8,12 grad=0.02 fp64")
    res = X.ne_pressure(Ls, grads, kT, G, seeds=seeds, warmup=warm, steps=steps,
                        sample_every=every, precision=F.FP64)
    per = _oracle_scan(Ls, grads, kT, G, seeds, warm, steps, every)
    mean = {k: np.mean([v[0] for v in vals]) for k, vals in per.items()}
    scale = max(abs(v) for v in mean.values()) + 1e-14
    for (L, g, T), m in mean.items():
        got = res.P_cold[(L, g)] if T == 0.0 else res.P_thermal[(L, g)][0]
        assert abs(got - m) <= 1e-12 * scale, (L, g, T, got, m)
        prof = np.mean([v[1] for v in per[(L, g, T)]], axis=0)
        # P - P_ref is a difference of O(1) quantities: its rounding is ~1e-16
        np.testing.assert_allclose(res.profiles[(L, g, T)]["pressure"], prof, rtol=0,
                                   atol=1e-12 * np.abs(prof).max() + 1e-14)
        rho = np.mean([v[2] for v in per[(L, g, T)]], axis=0)
        # delta rho is a difference of O(1) densities: its rounding is ~1e-16
        np.testing.assert_allclose(res.profiles[(L, g, T)]["density"], rho, rtol=0,
                                   atol=1e-12 * np.abs(rho).max() + 1e-14)
    for L in Ls:
        dpe = mean[(L, 0.0, kT)] - mean[(L, 0.0, 0.0)]
        assert abs(res.dP_eq[L][0] - dpe) <= 1e-12 * scale
        for g in grads:
            pne = mean[(L, g, kT)] - mean[(L, g, 0.0)] - dpe
            assert abs(res.P_ne[(L, g)][0] - pne) <= 1e-12 * scale
    say("  P_NE " + ", ".join(f"L={L}: {res.P_ne[(L, grads[0])][0]:.3e}" for L in Ls))


def test_ideal_mixture_has_no_pressure_shift(F):
    """Sec. IV.C: with an ideal equation of state (G = 0) the pressure is
    rho/3, whose spatial mean is fixed by mass conservation, so every P - P_ref
    and the non-equilibrium pressure vanish to rounding."""
    from paper_1808_05168_amd import experiments as X
    say("case: pressure protocol G=0")
    res = X.ne_pressure([16], [0.02], kT=1e-4, G=0.0, seeds=2, warmup=100, steps=200,
                        sample_every=10, precision=F.FP64)
    vals = [v for v in res.P_cold.values()] + [v[0] for v in res.P_thermal.values()]
    assert max(abs(v) for v in vals) < 1e-15
    assert abs(res.P_ne[(16, 0.02)][0]) < 1e-15


def test_ne_spectrum_matches_oracle(F):
    """The spectrum experiment of Sec. IV.B at a small size: ensemble mean of
    S_c(q, 0), wall-normal spectrum and measured bulk gradient against the same
    reduction of the oracle's runs."""
    import workloads as W
    from paper_1808_05168_amd import experiments as X
    L, Lx, kT, g, D, nu, nrep, warm, steps, every = 12, 24, 1e-4, 0.02, 0.02, 0.05, 3, 40, 120, 5
    say("case: ne_spectrum 24x12 x3 fp64")
    r = X.ne_spectrum(L=L, Lx=Lx, kT=kT, grad_c0=g, D=D, nu=nu, replicas=nrep, warmup=warm,
                      steps=steps, sample_every=every, precision=F.FP64, edge_rows=2)
    S, prof = [], []
    z = np.arange(L) - (L - 1) / 2.0
    for i in range(nrep):
        rep = W.Replica(Lx=Lx, Lz=L, grad_c0=g, kT=kT, tau_d=3 * D + 0.5, tau_s=3 * nu + 0.5,
                        seed=100 + i)
        f = O.init_state(rep)
        O.run(rep, f, 0, warm)
        acc = O.Accum(Lx, L)
        O.run(rep, f, warm, steps, acc, sample_every=every)
        S.append(O.structure_factor(acc)[0])
        # mean concentration profile straight from the oracle's field sums
        prof.append(X.mean_row_profile(acc.sq[0, 1], acc.sq[0, 2], acc.n_samples, Lx)
                    + 0.5 + z * g)
    S = np.array(S)
    np.testing.assert_allclose(r.S_c, S[:, 0, 1:].mean(axis=0), rtol=1e-10)
    np.testing.assert_allclose(r.S_c_wall_normal * r.S_eq, S[:, 1:L // 2 + 1, 0].mean(axis=0),
                               rtol=1e-10)
    c = np.mean(prof, axis=0)
    g_o = np.polyfit(z[2:-2], c[2:-2], 1)[0]
    assert abs(r.grad_measured - g_o) < 1e-12
    C = X.correlation(S.mean(axis=0), Lx)[0, : Lx // 2 + 1]
    C[0] -= r.S_eq
    np.testing.assert_allclose(r.C_x, C, rtol=0, atol=1e-10 * np.abs(C).max())
    assert np.allclose(r.q_tilde, 2 * np.pi * np.arange(1, Lx // 2 + 1) / Lx * L)


def test_gradient_scan_matches_oracle(F):
    """The grad c0 scan (S_c, S_rho band means, S_c(q_x, 0), mean pressure and
    its shift) against the same replicas run on the oracle."""
    from paper_1808_05168_amd import experiments as X
    Lx, Lz, grads, kT, G, warm, steps, every = 32, 16, [0.0, 5e-3, 1e-2], 1e-4, 0.5, 40, 120, 6
    say("case: gradient scan 32x16 fp64")
    res = X.gradient_scan(Lx, Lz, grads, kT=kT, G=G, warmup=warm, steps=steps,
                          sample_every=every, precision=F.FP64, seed=7)
    P = {}
    for g in grads:
        r = X._Run(Lx=Lx, Lz=Lz, grad_c0=g, kT=kT, G=G, seed=7)
        f = O.init_state(r)
        O.run(r, f, 0, warm)
        acc = O.Accum(Lx, Lz)
        O.run(r, f, warm, steps, acc, sample_every=every)
        n = acc.n_samples
        S = acc.sq[:, 0] / n - ((acc.sq[:, 1] / n) ** 2 + (acc.sq[:, 2] / n) ** 2)
        S_c, S_rho = S[0], S[1]
        scale = S_c[:, 1:].mean()
        assert abs(res.S_c_band[g] - S_c[:, 1:].mean()) <= 1e-12 * scale
        assert abs(res.S_rho_band[g] - S_rho[:, 1:].mean()) <= 1e-12 * S_rho[:, 1:].mean()
        np.testing.assert_allclose(res.S_c_qx[g], S_c[0, 1:], rtol=0, atol=1e-12 * scale)
        P[g] = acc.pr[0] / n
    scale = max(abs(v) for v in P.values()) + 1e-14
    for g in grads:
        assert abs(res.P_mean[g][0] - P[g]) <= 1e-12 * scale
        assert abs(res.P_shift[g][0] - (P[g] - P[grads[0]])) <= 2e-12 * scale


def test_run_description_end_to_end(F, tmp_path):
    """``experiments.run``: the sums it writes are those of the same batch run
    directly (and match the oracle), and a run resumed from its checkpoint
    image continues the accumulators exactly as an uninterrupted run."""
    from paper_1808_05168_amd import experiments as X
    cfg = {"precision": "fp64", "sample_every": 5, "warmup": 20, "steps": 40,
           "options": {"velocity": True}, "autotune": False,
           "replicas": [{"Lx": 24, "Lz": 12, "grad_c0": 5e-3, "kT": 1e-4, "G": 0.5,
                         "seed": 11, "copies": 2}]}
    say("case: run description, 2 x (24x12) fp64, 20 + 40 steps, checkpoint + resume")
    out1, ck = str(tmp_path / "a.npz"), str(tmp_path / "a.npy")
    info = X.run(cfg, out1, checkpoint=ck)
    assert info["samples"] == 8 and info["time"] == 60
    r1 = np.load(out1, allow_pickle=False)
    # the second replica (seed 12) against the oracle
    reps, *_ = X.run_config(cfg)
    f = O.init_state(reps[1], flags=O.DEFAULT_FLAGS | O.VELOCITY)
    O.run(reps[1], f, 0, 20, flags=O.DEFAULT_FLAGS | O.VELOCITY)
    acc = O.Accum(24, 12, nfields=4)
    O.run(reps[1], f, 20, 40, acc, flags=O.DEFAULT_FLAGS | O.VELOCITY, sample_every=5)
    assert acc.n_samples == 8
    for fld, name in enumerate(["c", "rho", "Ux", "Uz"]):
        sums = r1[f"rep1_{name}_sums"]
        scale = np.abs(acc.sq[fld]).max()
        assert np.abs(sums - acc.sq[fld]).max() <= 1e-12 * scale, name
    np.testing.assert_allclose(r1["rep1_P_profile"], acc.prof, rtol=0,
                               atol=1e-12 * np.abs(acc.prof).max())
    assert r1["rep1_P"][2] == 8
    # resumed for 40 more steps == one run of 20 + 80 steps
    out2 = str(tmp_path / "b.npz")
    X.run(cfg, out2, resume=ck)
    cfg_long = {**cfg, "steps": 80}
    out3 = str(tmp_path / "c.npz")
    X.run(cfg_long, out3)
    r2, r3 = np.load(out2, allow_pickle=False), np.load(out3, allow_pickle=False)
    assert int(r2["time"]) == int(r3["time"]) == 100 and int(r2["samples"]) == 16
    for k in r3.files:
        if k != "config":
            np.testing.assert_array_equal(r2[k], r3[k], err_msg=k)
