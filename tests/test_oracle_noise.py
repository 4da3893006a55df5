"""Pins of the oracle's noise: Philox4x32-10 words against rocRAND's own
implementation (a library routine compiled here for the host), Box-Muller
normals against the standard normal distribution, and the noise amplitudes
against the lattice fluctuation-dissipation relation (Eqs. (22)-(23))."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import workloads as W

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "philox_rocrand.cpp")


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                           HELPER, "-o", exe])

    def run(lines):
        inp = "\n".join(" ".join(str(v) for v in ln) for ln in lines) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
        return [[int(v) for v in row.split()] for row in out.stdout.strip().splitlines()]
    return run


def test_philox_matches_rocrand(ora, rocrand_philox):
    rng = np.random.default_rng(11)
    lines = [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6]
    lines += rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64).tolist()
    # counters of the shape the step uses: (node, t_lo, t_hi, call)
    lines += [[node, t, 0, call, 1, 0] for node in (0, 1, 2047) for t in (0, 1, 4999)
              for call in range(4)]
    ref = rocrand_philox(lines)
    got = [ora.philox(ln[:4], ln[4:]) for ln in lines]
    assert got == ref


def test_gaussians_are_standard_normal(ora):
    g = np.concatenate([ora.node_gaussians(5, node, t) for node in range(4000) for t in (3, 4)])
    assert g.size == 4000 * 2 * 14
    n = g.size
    assert abs(g.mean()) < 5 / np.sqrt(n)
    assert abs(g.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(g, fisher=False) - 3) < 5 * np.sqrt(24 / n)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # the 14 variates of a node are uncorrelated with each other
    G = g.reshape(-1, 14)
    C = np.corrcoef(G.T) - np.eye(14)
    assert np.abs(C).max() < 5 / np.sqrt(G.shape[0])


def _box_muller(w0, w1):
    u1 = (w0 + 0.5) * 2.0**-32
    u2 = (w1 + 0.5) * 2.0**-32
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)


@pytest.mark.parametrize("seed,node,t", [(1, 0, 0), (7, 513, 10), (3, 2047, 4998),
                                         (5, 9, 2**32 + 6)])
def test_shared_call_splits_between_two_steps(ora, seed, node, t):
    """Steps t (even) and t + 1 draw 28 words from seven Philox calls: calls
    0..2 of each step, and call 3 of step t, whose words 0, 1 go to step t and
    words 2, 3 to step t + 1 (as g_12, g_13)."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for step in (t, t + 1):
        g = ora.node_gaussians(seed, node, step)
        words = []
        for call in range(3):
            words += ora.philox([node, step & 0xFFFFFFFF, step >> 32, call], key)
        shared = ora.philox([node, t & 0xFFFFFFFF, t >> 32, 3], key)
        words += shared[0:2] if step == t else shared[2:4]
        expect = np.array([v for i in range(7) for v in _box_muller(words[2 * i], words[2 * i + 1])])
        np.testing.assert_allclose(g, expect, rtol=1e-13, atol=1e-15)


def test_two_steps_draw_independent_normals(ora):
    """The 28 variates of a node over an even step and the odd step after it
    are uncorrelated (the shared call gives each step words of its own)."""
    G = np.array([np.concatenate([ora.node_gaussians(4, node, 6), ora.node_gaussians(4, node, 7)])
                  for node in range(6000)])
    C = np.corrcoef(G.T) - np.eye(28)
    assert np.abs(C).max() < 5 / np.sqrt(G.shape[0])


def test_gaussians_depend_on_seed_node_and_time(ora):
    a = ora.node_gaussians(1, 10, 20)
    assert not np.array_equal(a, ora.node_gaussians(2, 10, 20))
    assert not np.array_equal(a, ora.node_gaussians(1, 11, 20))
    assert not np.array_equal(a, ora.node_gaussians(1, 10, 21))
    assert not np.array_equal(a, ora.node_gaussians(1, 10, 20 + (1 << 32)))
    np.testing.assert_array_equal(a, ora.node_gaussians(1, 10, 20))


def test_one_step_moment_variances_follow_fdt(ora):
    """From a state at rest with all lambda = 1, one collision replaces every
    non-conserved moment by its noise, so the sample variances after one step
    must equal the lattice FDT values: 3 kT rho^S N_a for a >= 3 (Eq. (23)) and
    kT rho^A rho^B / rho for the species momenta (Eq. (22)), with
    j^A + j^B = 0."""
    Lx, Lz, kT = 96, 64, 1e-4
    rep = W.Replica(Lx=Lx, Lz=Lz, kT=kT, seed=9)
    f = ora.init_state(rep, flags=ora.ASTAR)
    ora.run(rep, f, 1, 1, flags=ora.ASTAR)
    c, w, T, N = ora.tables()
    # undo streaming: post-collision population l of node r sits at r + c_l
    # (walls excluded: keep interior rows only)
    post = np.empty_like(f)
    for s in range(2):
        for l in range(9):
            post[s, l] = np.roll(np.roll(f[s, l], -c[l, 1], axis=0), -c[l, 0], axis=1)
    post = post[:, :, 2:-2, :]
    m = np.einsum("al,slzx->sazx", T, post)
    n = m[0, 0].size
    for s in range(2):
        for a in range(3, 9):
            expect = 3 * kT * 0.5 * N[a]
            assert abs(m[s, a].var() / expect - 1) < 6 * np.sqrt(2 / n)
        for a in (1, 2):
            assert abs(m[s, a].var() / (kT * 0.25) - 1) < 6 * np.sqrt(2 / n)
    np.testing.assert_allclose(m[0, 1] + m[1, 1], 0, atol=1e-16)
    np.testing.assert_allclose(m[0, 2] + m[1, 2], 0, atol=1e-16)
