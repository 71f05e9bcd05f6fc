"""Host-side logic that needs no GPU: the synthetic workload recipes, the
benchmark's error statistics and counter summaries, and the one-GPU guard."""
import csv
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_workload_recipes():
    p = synth.config_plain_fp64()
    assert (p.nx, p.ny, p.ell, p.steps, p.v_rel) == (256, 128, 64, 2000, 0.3)
    p = synth.config_sif_fp32()
    assert (p.nx, p.ny, p.ell, p.steps) == (4096, 2048, 1024, 20000)
    assert p.K_C == pytest.approx(1.5 * 1e-3 * math.sqrt(math.pi * 1024))
    w = p.wdot0()
    assert w.shape == (2048, 4096) and abs(w.std() - 1e-6) < 1e-8
    np.testing.assert_array_equal(w, p.wdot0())  # seeded
    p = synth.config_precision()
    assert (p.nx, p.ny, p.ell, p.steps, p.v_rel) == (16384, 8192, 4096, 10000, 0.5)


def test_batched_recipe():
    plates = synth.config_batched()
    assert len(plates) == 64
    for k, p in enumerate(plates):
        assert (p.nx, p.ny) in synth.BATCH_SIZES and p.ell == p.nx // 4
        assert 5e-4 <= p.tau <= 2e-3
        if k % 2:
            assert p.growth == synth.GROW_SIF
            assert p.K_C == pytest.approx(1.5 * synth.k_static_edge(p.tau, p.ell))
        else:
            assert p.growth == synth.GROW_PRESCRIBED and 0.1 <= p.v_rel <= 0.7


def test_adjoint_recipe():
    p = synth.config_adjoint()
    s = synth.adjoint_sensors(p.nx, p.ny)
    assert len({tuple(x) for x in s}) == 32
    j0 = p.ny // 2 - 1
    assert np.all(np.abs(s[:, 1] - j0) > 2) and np.all(np.abs(s[:, 1] - (j0 + 1)) > 2)
    for d_tau, d_w in synth.adjoint_directions(50, (4, 6), count=5):
        assert (d_tau ** 2).sum() + (d_w ** 2).sum() == pytest.approx(1.0)
    h = synth.adjoint_target_history(1600)
    assert h[200] == pytest.approx(1.1e-3) and h[600] == pytest.approx(0.9e-3)


def test_k_static_edge_is_the_griffith_value():
    # edge crack of length ell at a free edge = Griffith crack of length 2 ell
    assert synth.k_static_edge(2e-3, 100.0) == pytest.approx(2e-3 * math.sqrt(math.pi * 100.0))


def test_k_error_statistics():
    K_ref = np.array([np.nan, 0.0, 1.0, 2.0, 4.0, 4.0, 4.0, 4.0, 4.0, 4.0, 4.0])
    K = K_ref.copy()
    K[3] += 0.02   # 1 % at a step with half the largest K
    K[-1] -= 0.004
    e = bench.k_errors(K, K_ref)
    assert e["K_err_rel_max"] == pytest.approx(0.02 / 4.0)
    assert e["K_err_rel_final"] == pytest.approx(0.001)
    assert e["K_err_rel_late_max"] == pytest.approx(0.001)
    assert e["K_err_rel_strong_max"] == pytest.approx(0.01)  # K_ref = 2 >= max / 2
    assert bench.k_errors(K, np.full(5, np.nan)) == {"K_err_rel_max": None}


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_counter_summary_scales_by_the_copy(tmp_path):
    copy = 1 << 30
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    p = synth.config_precision()
    alg = p.nx * p.ny * 28
    # FETCH_SIZE counts half the bytes (of the copy and of the kernel alike), WRITE_SIZE all;
    # the run also holds another storage's sweep with more launches (the record
    # storage a counter run times as well), which the summary must leave out
    own = "void lbmk::(anonymous namespace)::sweep_step<_Float16, float, float, 4, true, false, " \
          "false, true>(_Float16 const*, _Float16*, float const*, float*)"
    other = "void lbmk::(anonymous namespace)::sweep_step<_Float16, float, float, 4, true, true, " \
            "false, true>(_Float16 const*, _Float16*, float const*, float*)"
    _write_counters(fd, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy / 2 / 1024),
                                       (own, alg * 0.51 / 2 / 1024), (own, alg * 0.51 / 2 / 1024)]
                    + [(other, alg / 1024)] * 3)
    _write_counters(wd, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy / 1024),
                                       (own, alg * 0.5 / 1024)] + [(other, alg / 1024)] * 3)
    bench.summarize_pmc(fd, wd, "f16s", "precision", copy, "cmd", str(tmp_path))
    out = json.load(open(tmp_path / "sweep_f16s_precision_traffic.json"))
    assert out["FETCH_SIZE"]["factor"] == pytest.approx(2.0)
    assert out["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    assert out["traffic_over_algorithmic"] == pytest.approx(1.01)
    assert out["kernel_source_sha"] == bench.kernel_source_hash()


def test_counter_summary_sums_the_two_launches_of_a_t_step_sweep(tmp_path):
    """A T-step sweep is a fast launch (sweep_block_tall here) and a boundary
    launch (sweep_block_edges): the summary adds one of each per sweep, of this
    storage's instantiations only (the BF16 decoy has more launches)."""
    copy = 1 << 30
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    st = "f16s-eq-tb6-sr"
    p = synth.config_precision()
    alg = p.nx * p.ny * bench.sweep_bytes_per_site(st) * bench.time_block(st)
    tall = "_ZN4lbmk3blk16sweep_block_tallIDF16_ffLi4ELb1ELi16ELi32ELi6EEEvNS_9BlockArgsIT_T0_T1_EEiiNS0_8FastRunsE"
    edges = "_ZN4lbmk3blk17sweep_block_edgesIDF16_ffLi4ELb1ELi16ELi6EEEvNS_9BlockArgsIT_T0_T1_EEiiiiNS0_10SlowChunksE"
    decoy = "_ZN4lbmk3blk11sweep_blockIDF16bffLi4ELb1ELi16ELi6EEEvNS_9BlockArgsIT_T0_T1_EEiii"
    # FETCH_SIZE counts half the bytes: the fast launch fetches 1.1, the
    # boundary launch 0.1 of the algorithmic reads; writes 0.97 and 0.06
    _write_counters(fd, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy / 2 / 1024)]
                    + [(tall, alg / 2 * 1.1 / 2 / 1024), (edges, alg / 2 * 0.1 / 2 / 1024)] * 2
                    + [(decoy, alg / 1024)] * 3)
    _write_counters(wd, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy / 1024)]
                    + [(tall, alg / 2 * 0.97 / 1024), (edges, alg / 2 * 0.06 / 1024)] * 2
                    + [(decoy, alg / 1024)] * 3)
    bench.summarize_pmc(fd, wd, st, "precision", copy, "cmd", str(tmp_path))
    out = json.load(open(tmp_path / f"sweep_{st}_precision_traffic.json"))
    assert [k[1] for k in out["FETCH_SIZE"]["kernels"]] == [2, 2]
    assert out["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(alg / 2 * 1.2)
    assert out["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(alg / 2 * 1.03)
    assert out["traffic_over_algorithmic"] == pytest.approx((1.2 + 1.03) / 2)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_build_lists_every_source_and_the_traffic_hash_covers_the_sweeps():
    """Every HIP source in csrc is compiled, per-source flags name listed
    sources, and the hash that gates the stored traffic counters covers every
    sweep source and the build flags (a change to any of them voids them)."""
    from paper_2206_12412_amd import build as B
    srcs = sorted(f for f in os.listdir(B.CSRC) if f.endswith((".hip", ".cpp")))
    assert sorted(B.SOURCES) == srcs
    assert set(B.EXTRA) <= set(B.SOURCES)
    sweeps = {f for f in os.listdir(B.CSRC) if f.startswith("sweep")}
    assert sweeps | {"lbm_internal.hpp", "../build.py"} == set(bench.KERNEL_SOURCES)
