"""CPU tests of the benchmark's host logic: the roofline arithmetic, the
counter summary it reads, and the refusal of more than one GPU."""
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _stats(**kw):
    base = dict(minibatches=0, pairs=0, timed_launches=0, rows_in=0, rows_out=0,
                rows_out_single=0, ms=0.0, path=1, timed_minibatches=0, ms_update=0.0,
                ms_prep=0.0, ms_forward=0.0, ms_apply=0.0, ms_apply_first=0.0,
                update_blocks=64, us_phase=[0.0, 0.0, 0.0, 0.0])
    base.update(kw)
    return SimpleNamespace(**base)


def test_persistent_roofline_arithmetic():
    """Two calls of 128 minibatches (2 launches of 64 each): algorithmic bytes
    per launch = (2 x touched rows x d x 4 + 8 B per touch) per minibatch x 64;
    achieved = bytes / mean launch time; phases averaged over the timed
    minibatches."""
    d, K, P = 128, 5, 1024
    sts = [_stats(minibatches=128, pairs=128 * P, timed_launches=2, rows_in=128 * 1000,
                  rows_out=128 * 6000, rows_out_single=128 * 5800, ms=2.4,
                  timed_minibatches=128, ms_update=2.2, ms_prep=0.5,
                  us_phase=[7.0, 3.0, 1.0, 6.0]),
           _stats(minibatches=128, pairs=128 * P, timed_launches=2, rows_in=128 * 1000,
                  rows_out=128 * 6000, rows_out_single=128 * 5800, ms=2.4,
                  timed_minibatches=128, ms_update=2.4, ms_prep=0.5,
                  us_phase=[8.0, 3.0, 1.0, 6.0])]
    r = bench.sgns_roofline(sts, d, K, 256 * P)
    kern = "sgns_small_update_kernel<%d, %d>" % (d, K)
    assert r["kernel"] == kern and r["bound"] == "hbm" and r["unit"] == "GB/s"
    per_mb = 2 * 7000 * d * 4 + P * (K + 2) * 8
    k = r["kernels"][kern]
    assert k["minibatches_per_launch"] == 64
    assert k["algorithmic_bytes_per_launch"] == pytest.approx(per_mb * 64)
    avg_s = (2.2 + 2.4) / 1e3 / 4
    assert k["avg_launch_us"] == pytest.approx(avg_s * 1e6)
    assert r["achieved"] == pytest.approx(per_mb * 64 / avg_s / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    ph = k["phases_us_per_minibatch"]
    assert ph["forward"] == pytest.approx(7.5) and ph["barrier_2"] == pytest.approx(6.0)
    assert r["traffic"] is None          # the caller fills it from the counter summary


def test_counter_summary_matches_the_kernel_sources():
    """The committed counter summary was taken on the current sources of the
    persistent update, so the benchmark reports its measured traffic."""
    tr = bench.measured_traffic()
    assert tr is not None, ("profiles/sgns_small_update_rmat23w_counters.md was taken on "
                            "other sources: retake its FETCH_SIZE / WRITE_SIZE passes")
    assert tr["minibatches_per_launch"] == 64 and tr["bytes"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
