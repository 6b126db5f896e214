"""Host logic of bench.py and of the binding's load helpers (no GPU)."""

import os
import subprocess
import sys

import numpy as np

import bench
from paper_1905_09395_amd import stev, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_direct_dft_flop_count_by_hand():
    # 6-species set: 10 + 51 n_s; R1 irreversible with 4 participants (7 + 2*4),
    # R2 and R3 reversible with 3 and 4 (15 + 4*3, 15 + 4*4), R4 irreversible
    # with 4 (7 + 2*4); 185 per reversible reaction for the 13-point |DFT| at
    # bins 0 and 4-6 as direct sums
    assert bench.direct_dft_flops(synth.make_mech6()) == 10 + 51 * 6 + 15 + 27 + 31 + 15 + 2 * 185
    # the 19-species mechanism: 50 reversible reactions
    assert bench.direct_dft_flops(synth.make_mech19()) == 11995


def test_load_curve_counts_cells_still_integrating():
    """Sec 2.4 load: at each reported iteration count, the number of cells
    that take at least that many steps (cells placed on bin edges)."""
    edges = list(stev.load_bin_edges())
    iters = [edges[3], edges[3], edges[10], edges[40], edges[40], edges[40]]
    hist = np.zeros(len(edges), np.int64)
    for c in iters:
        hist[edges.index(c)] += 1
    want = [(e, sum(1 for c in iters if c >= e)) for e in (edges[3], edges[10], edges[40])]
    assert stev.load_curve(hist) == want


def test_cpu_baseline_record():
    mech = synth.make_mech6()
    T, P, Y = synth.make_cells_mech6(1024, seed=101)
    r = bench.cpu_baseline(mech, T, P, Y, 1e-4, budget_s=0.5)
    assert r["kind"] == "oracle" and r["unit"] == "cells/s" and r["cores"] >= 1
    assert r["value"] > 0 and r["one_thread_value"] > 0 and "1024-cell field" in r["sample"]
