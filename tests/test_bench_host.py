"""Host-side checks of bench.py: its algorithmic byte counts (the numerators of
the roofline figures) against closed forms, and its refusal of several GPUs.
No GPU is used: the mesh handle is set up on the host only."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import hdg  # noqa: E402
from paper_2302_10917_amd import inputs, mhdg  # noqa: E402


def test_apply_bytes_closed_form():
    """Plain at-scale mesh: 8 N^2 + 4 N per macro (factors and pivots once) plus
    32 bytes per trace unknown (gathered trace and written slots), N = 975:
    62,341,836,800 bytes per apply."""
    xy, tri = inputs.structured_mesh(64)
    m = mhdg.MacroMesh(xy, tri, 3, 3)
    s = m.sizes
    N = 3 * (24 + 1) * (24 + 2) // 2
    assert s.max_local == N == 975 and s.n_trace == 304000
    expect = 8192 * (8.0 * N * N + 4.0 * N) + 32.0 * s.n_trace
    assert bench.apply_bytes(m) == expect == 62341836800.0
    # flux eliminated: the Q x Q Schur block (Q = N / 3)
    Q = N // 3
    assert bench.apply_bytes(m, qelim=True) == 8192 * (8.0 * Q * Q + 4.0 * Q) + 32.0 * s.n_trace


def test_fold_bytes_matches_interior_face_counts():
    """8 L_K^2 per macro with L_K the trace dofs of its interior faces (counted
    here from the oracle's face topology), plus 32 bytes per trace unknown."""
    xy, tri = inputs.structured_mesh(4)
    for r in (2, inputs.random_levels(len(tri), (0, 1, 2), seed=3)):
        topo = hdg.Topology(xy, tri, r, 3)
        L = np.zeros(topo.n_macro)
        for f in range(topo.n_faces):
            if topo.interior[f]:
                for K, _ in topo.face_incid[f]:
                    L[K] += topo.face_nodes[f]
        expect = float(np.sum(8.0 * L * L)) + 32.0 * topo.n_trace
        assert bench.fold_bytes(tri, r, 3, topo.n_trace) == expect


def test_bench_refuses_several_gpus():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_cpu_baseline_reports_the_oracle_time_to_solve():
    """The CPU baseline on a small mesh (a bounded sample of macros): the apply
    rate, the whole-mesh factorisation time scaled from the sample, and the
    estimated time to solve = factorisation + applies / rate."""
    xy, tri = inputs.structured_mesh(3)
    w = {"r": 1, "p": 2, "kappa": 0.05, "beta": (1.0, 0.5)}
    cb = bench.cpu_baseline(xy, tri, w, n_sample=3, budget_s=0.2)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["factor_s_whole_mesh"] > 0
    bench.oracle_solve_estimate(cb, [100, 104], 0.5)
    expect = cb["factor_s_whole_mesh"] + 102.0 / cb["value"]
    assert abs(cb["time_to_solve_s_estimate"] - expect) <= 1e-12 * expect
    assert "102 applies" in cb["time_to_solve_estimate"]
