"""GPU checks of the runtime around the step kernel: graph replay of whole
sampling periods is bit-identical to direct launches (checked after every
chunk of steps, with host reads in between), and the autotuner leaves state
and time untouched."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import compare_observables, dev_norm, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1808_05168_amd as F
    F.load()
    return F


def _same(a, b):
    for i in range(len(a.reps)):
        np.testing.assert_array_equal(a.read_populations(i), b.read_populations(i))
        for fld in range(2):
            ra, rb = a.read_structure_factor(i, fld), b.read_structure_factor(i, fld)
            assert ra[3] == rb[3]
            for x, y in zip(ra[:3], rb[:3]):
                np.testing.assert_array_equal(x, y)
        pa, pb = a.read_pressure(i), b.read_pressure(i)
        assert pa[0] == pb[0] and pa[1] == pb[1]
        np.testing.assert_array_equal(pa[2], pb[2])


@pytest.mark.parametrize("every,prec,two", [(5, 0, 0), (4, 1, 0), (0, 0, 0), (7, 1, 0),
                                            (4, 1, 1), (7, 1, 1), (0, 1, 1), (1, 1, 1),
                                            (2, 0, 0)])
def test_graph_replay_matches_direct_launches(F, every, prec, two):
    # block transforms for the first two, wavefront transforms for the third;
    # the step counts leave samples of a call in the spectrum slots of the
    # batched column pass in every phase, and replay both the graph of one
    # sampling period and the graph of sixteen
    reps = [W.Replica(Lx=96, Lz=20, grad_c0=2e-3, kT=1e-4, G=0.5, seed=51),
            W.Replica(Lx=300, Lz=9, grad_c0=1e-2, kT=1e-4, seed=52),
            W.Replica(Lx=64, Lz=32, grad_c0=5e-3, kT=1e-4, G=0.3, seed=54)]
    say(f"case: graph vs direct, every={every} precision={prec} two-step={two}")
    kern = F.TWO_STEP if two else F.ONE_STEP
    g = F.Lattice(reps, precision=prec, sample_every=every, flags=F.DEFAULT_FLAGS | kern)
    d = F.Lattice(reps, precision=prec, sample_every=every,
                  flags=F.DEFAULT_FLAGS | F.NO_GRAPH | kern)
    for n in (3, 7, 20, 1, 13, 40, 0, 17, 120):
        g.step(n)
        d.step(n)
        assert g.time == d.time
        _same(g, d)
    if prec == 0:
        for i, rep in enumerate(reps):
            f_o, acc = run_oracle(rep, g.time, every=every)
            assert dev_norm(g.read_populations(i), f_o, rep) <= 1e-12
            compare_observables(g, acc, i, rep, 1e-12)


def test_graph_after_time_reset_and_write(F):
    rep = W.Replica(Lx=64, Lz=16, grad_c0=5e-3, kT=1e-4, G=0.5, seed=53)
    say("case: graph after set_time/write_populations")
    g = F.Lattice([rep], sample_every=4)
    d = F.Lattice([rep], sample_every=4, flags=F.DEFAULT_FLAGS | F.NO_GRAPH)
    g.step(11)
    d.step(11)
    f = g.read_populations(0)
    for lat in (g, d):
        lat.write_populations(0, f)
        lat.time = 40
        lat.step(12)
    _same(g, d)


def test_autotune_keeps_state_and_results(F):
    rep = W.large_4096x1024()
    say("case: autotune 4096x1024 fp32-dev")
    a = F.Lattice([rep], precision=F.FP32_DEV, sample_every=10)
    b = F.Lattice([rep], precision=F.FP32_DEV, sample_every=10, chunk_rows=16)
    a.step(12)
    b.step(12)
    before = a.read_populations(0)
    chunk = a.autotune(5)
    assert chunk in (4, 8, 16, 32, 64, 128)
    assert a.time == 12
    np.testing.assert_array_equal(a.read_populations(0), before)
    a.step(21)
    b.step(21)
    _same(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpoint_resume_is_bit_identical(F, prec):
    """Save after 73 steps, continue 41 steps; a fresh handle loaded from the
    image and stepped 41 steps matches bit for bit (populations, structure-factor
    and pressure sums, sample count, time)."""
    import dataclasses
    precision = F.FP64 if prec == "fp64" else F.FP32_DEV
    reps = [W.Replica(Lx=70, Lz=12, grad_c0=5e-3, kT=1e-4, G=0.5, tau_s=0.7, seed=61),
            W.Replica(Lx=300, Lz=20, grad_c0=2e-3, kT=1e-4, seed=62)]
    say(f"case: checkpoint resume {prec}")
    a = F.Lattice(reps, precision=precision, sample_every=5)
    a.step(73)
    image = a.save()
    a.step(41)
    b = F.Lattice(reps, precision=precision, sample_every=5)
    b.load(image)
    assert b.time == 73
    b.step(41)
    assert b.time == a.time == 114
    for i in range(len(reps)):
        np.testing.assert_array_equal(b.read_populations(i), a.read_populations(i))
        for fld in range(2):
            for x, y in zip(b.read_structure_factor(i, fld), a.read_structure_factor(i, fld)):
                np.testing.assert_array_equal(x, y)
        for x, y in zip(b.read_pressure(i), a.read_pressure(i)):
            np.testing.assert_array_equal(x, y)
    # an image only loads into a handle of the same replicas and options
    other = [dataclasses.replace(reps[0], seed=99), reps[1]]
    with pytest.raises(F.FnlbError):
        F.Lattice(other, precision=precision, sample_every=5).load(image)
    with pytest.raises(F.FnlbError):
        F.Lattice(reps, precision=precision, sample_every=10).load(image)
    with pytest.raises(F.FnlbError):
        F.Lattice(reps, precision=precision, sample_every=5).load(image[:-8])


@pytest.mark.parametrize("flags", [W.DEFAULT_FLAGS, W.DEFAULT_FLAGS | W.SAMPLE_VELOCITY])
def test_sampling_leaves_fp32_trajectory_unchanged(F, flags):
    """With FP32-deviation storage a step that samples runs the same collision
    arithmetic as one that does not: the trajectories agree bit for bit."""
    reps = [W.Replica(Lx=100, Lz=20, grad_c0=5e-3, kT=1e-4, G=0.5, tau_s=0.7, tau_d=0.8, seed=71),
            W.Replica(Lx=600, Lz=9, grad_c0=1e-2, kT=1e-4, G=0.3, seed=72)]
    say(f"case: sampled vs unsampled fp32, flags={flags}")
    a = F.Lattice(reps, precision=F.FP32_DEV, sample_every=3, flags=flags)
    b = F.Lattice(reps, precision=F.FP32_DEV, sample_every=0, flags=flags)
    a.step(37)
    b.step(37)
    for i in range(len(reps)):
        np.testing.assert_array_equal(a.read_populations(i), b.read_populations(i))


def test_autotune_pick_reproduces_across_processes(F, tmp_path):
    """The benchmark ensemble's autotuned choice (kernel, rows per work item),
    saved to a tuning file, is what a fresh process finds stored and picks
    again when it tunes; a handle created there without a row-range length
    uses the stored choice."""
    import json
    import subprocess
    import sys
    reps = W.batched_ensemble(96)
    say("case: autotune, save, and tune again in a fresh process")
    lat = F.Lattice(reps, precision=F.FP32_DEV, sample_every=10)
    lat.autotune(20)
    pick = lat.launch_config()
    path = tmp_path / "tune.txt"
    F.tune_cache_save(str(path))
    code = (
        "import json, sys; sys.path.insert(0, %r)\n"
        "import paper_1808_05168_amd as F, workloads as W\n"
        "F.tune_cache_load(%r)\n"
        "reps = W.batched_ensemble(96)\n"
        "stored = F.tune_lookup(reps, F.FP32_DEV)\n"
        "lat = F.Lattice(reps, precision=F.FP32_DEV, sample_every=10)\n"
        "used = lat.launch_config()\n"
        "lat.autotune(20)\n"
        "print(json.dumps([stored, used, lat.launch_config()]))\n"
    ) % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), str(path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    stored, used, repick = json.loads(r.stdout.strip().splitlines()[-1])
    say(f"  pick {pick}, stored {stored}, used {used}, picked again {repick}")
    assert tuple(stored) == pick and tuple(used) == pick and tuple(repick) == pick
