"""Host-side logic of bench.py that needs no GPU: the one-GPU guard, the
lookup of stored traffic counters (keyed by workload size and by the hash of
the kernel's sources), and the per-launch byte model of the spin sweep."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_lookup_by_size_and_source_hash(tmp_path, monkeypatch):
    k = "k_desc_angular<double>"
    good = bench.kernel_source_hash(k)
    d = {"workloads": [
        {"n_atoms": 1000, "kernels": {k: {"bytes_per_launch": 123, "source_hash": good}}},
        {"n_atoms": 2000, "kernels": {k: {"bytes_per_launch": 456, "source_hash": "stale"}}}]}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    # the hash is taken over the real sources, so point only the profile lookup at tmp_path
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: good)
    assert bench.traffic_from_profile(k, 1000) == 123
    assert bench.traffic_from_profile(k, 2000) is None      # measured on other sources
    assert bench.traffic_from_profile(k, 3000) is None      # another workload size
    assert bench.traffic_from_profile("k_none<double>", 1000) is None


def test_committed_traffic_matches_current_sources():
    """every kernel in the committed counter file was measured on the sources
    in the tree (or the bench reports traffic: null for it, by design)"""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    sizes = sorted(w["n_atoms"] for w in d["workloads"])
    assert sizes == [262144, 7077888]
    for w in d["workloads"]:
        stale = [k for k, v in w["kernels"].items() if v["source_hash"] != bench.kernel_source_hash(k)]
        assert not stale, f"{w['n_atoms']} atoms: counters older than the sources of {stale}"


def test_sweep_bytes_model():
    """per spin: its couplings (six reals, an index, the partner's spin) and
    its own records; per launch: one colour class"""
    pc = {"N_fe": 1024, "R_fefe": 1024 * 30}
    b64 = bench.sweep_bytes_per_launch(pc, 32, real_bytes=8)
    b32 = bench.sweep_bytes_per_launch(pc, 32, real_bytes=4)
    per_spin64 = 30 * (48 + 4 + 24) + 7 * 8 + 24 + 24 + 12 + 24
    assert b64 == pytest.approx(per_spin64 * 1024 / 32)
    assert b64 - b32 == pytest.approx((30 * 6 * 4 + 7 * 4) * 1024 / 32)


def test_pair_counts_of_the_crystal():
    """ordered pair counts of the B20 crystal per atom, which the work model
    scales from a small crystal to the large ones: 62 within 6 A (30 Fe-Fe
    per Fe); within 4.5 A about 29 (shells lie near that cutoff, so the
    0.02 A position noise moves a few pairs across it); the same per atom at
    two crystal sizes"""
    from paper_2606_14073_amd import workload as W
    a = bench.pair_counts(W.fege_lattice(4, 4, 4))
    b = bench.pair_counts(W.fege_lattice(6, 6, 6))
    for pc in (a, b):
        assert pc["R"] / pc["N"] == pytest.approx(62, abs=0.05)
        assert pc["R_fefe"] / pc["N_fe"] == 30
        assert pc["A"] / pc["N"] == pytest.approx(29, abs=0.5)
        assert pc["A_fe"] == pc["A_fefe"] + pc["A_fege"] // 2
    assert a["A"] / a["N"] == pytest.approx(b["A"] / b["N"], rel=0.01)


def test_sweep_kernel_named_by_class_size():
    """the bench names the sweep kernel by the lane layout the library's
    launcher takes for the largest colour class: 4 lanes per spin from
    32,768 spins up, 8 from 8,192, else 16"""
    import numpy as np
    small = np.repeat(np.arange(32), 4096)            # 262,144-atom crystal: 4,096 spins per colour
    large = np.repeat(np.arange(32), 110592)          # 7,077,888 atoms: 110,592 per colour
    ge = -np.ones(10, dtype=np.int64)                 # atoms without a spin carry no colour
    assert bench.kernel_name("sweep", "double", np.concatenate([small, ge])) == "k_sweep<double,16>"
    assert bench.kernel_name("sweep", "float", large) == "k_sweep<float,4>"
    assert bench.kernel_name("sweep", "double", np.repeat(np.arange(2), 32768)) == "k_sweep<double,4>"
    assert bench.kernel_name("sweep", "double", np.repeat(np.arange(2), 32767)) == "k_sweep<double,8>"
    assert bench.kernel_name("sweep", "double", np.repeat(np.arange(3), 8192)) == "k_sweep<double,8>"
    assert bench.kernel_name("sweep", "double", np.repeat(np.arange(3), 8191)) == "k_sweep<double,16>"
    assert bench.kernel_name("desc_angular", "double") == "k_desc_angular<double>"


def test_sweep_thresholds_match_the_library():
    """the bench's copy of the sweep launcher's class-size thresholds equals
    the constants in the kernel source"""
    import re
    src = open(os.path.join(ROOT, "paper_2606_14073_amd", "csrc", "kernels_int.hip")).read()
    wide = int(re.search(r"constexpr int SWEEP_WIDE_MIN = (\d+);", src).group(1))
    wider = int(re.search(r"constexpr int SWEEP_WIDER_MIN = (\d+);", src).group(1))
    assert (bench.SWEEP_WIDE_MIN, bench.SWEEP_WIDER_MIN) == (wide, wider)
