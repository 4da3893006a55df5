"""The run description of ``experiments.run`` (CPU: parsing and checks)."""
import json

import pytest

from paper_1808_05168_amd import experiments as X
from paper_1808_05168_amd import fnlb as f


def test_defaults_copies_and_options():
    reps, prec, flags, every, warmup, steps, tune = X.run_config({
        "precision": "fp32", "steps": 100,
        "replicas": [{"Lx": 32, "Lz": 16, "kT": 1e-5, "seed": 5, "copies": 3},
                     {"Lx": 64, "Lz": 32, "grad_c0": 1e-3, "G": 0.5, "tau_s": 0.7}]})
    assert [r.seed for r in reps] == [5, 6, 7, 1]
    assert all((r.Lx, r.Lz, r.kT) == (32, 16, 1e-5) for r in reps[:3])
    assert (reps[3].grad_c0, reps[3].G, reps[3].tau_s, reps[3].tau_d) == (1e-3, 0.5, 0.7, 1.0)
    assert prec == f.FP32_DEV and flags == f.DEFAULT_FLAGS
    assert (every, warmup, steps, tune) == (10, 0, 100, True)
    _, prec, flags, *_ = X.run_config({
        "steps": 1, "options": {"velocity": True, "wall_uz_fix": False, "noise_loc": True},
        "replicas": [{"Lx": 8, "Lz": 8}]})
    assert prec == f.FP64
    assert flags == f.ASTAR | f.SAMPLE_VELOCITY | f.NOISE_LOC


@pytest.mark.parametrize("cfg", [
    {"steps": 1, "replicas": [{"Lx": 8, "Lz": 8}], "bogus": 1},
    {"steps": 1, "replicas": [{"Lx": 8, "Lz": 8}], "options": {"bogus": True}},
    {"steps": 1, "replicas": [{"Lx": 8, "Lz": 8}], "precision": "fp16"},
    {"steps": 1, "replicas": [{"Lz": 8}]},
    {"steps": 1, "replicas": [{"Lx": 8, "Lz": 8, "tau": 1.0}]},
    {"steps": 1, "replicas": [{"Lx": 8, "Lz": 8, "copies": 0}]},
    {"steps": 1, "replicas": []},
    {"steps": 0, "replicas": [{"Lx": 8, "Lz": 8}]},
    {"steps": 1, "sample_every": 0, "replicas": [{"Lx": 8, "Lz": 8}]},
    [1, 2],
])
def test_bad_descriptions_are_rejected(cfg):
    with pytest.raises(ValueError):
        X.run_config(cfg)


def test_json_and_yaml_files(tmp_path):
    cfg = {"precision": "fp64", "sample_every": 5, "warmup": 10, "steps": 20,
           "replicas": [{"Lx": 16, "Lz": 8, "kT": 1e-4, "seed": 3}]}
    pj = tmp_path / "run.json"
    pj.write_text(json.dumps(cfg))
    py = tmp_path / "run.yaml"
    py.write_text("precision: fp64\nsample_every: 5\nwarmup: 10\nsteps: 20\n"
                  "replicas:\n  - {Lx: 16, Lz: 8, kT: 1.0e-4, seed: 3}\n")
    assert X.load_run_config(str(pj)) == cfg
    assert X.load_run_config(str(py)) == cfg
