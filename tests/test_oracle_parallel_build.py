"""The OpenMP timing build of the oracle (the benchmark's all-cores CPU
baseline) computes the same step as the serial oracle: forces equal up to
summation order, trajectories and contact histories equal to rounding, and
the result does not depend on the number of threads."""
import os
import subprocess
import sys

import numpy as np

import workloads as W
from oracle import oracle_from_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(parallel):
    sc = W.dense_snapshot(n=4000, seed=13, polydisperse=0.2, n_types=2, K=7)
    o = oracle_from_scene(sc, parallel=parallel)
    o.step(30)
    F, T, _ = o.forces()
    return F, T, o.state()["pos"], o.contacts()[1]


def test_parallel_build_equals_serial_oracle(oracle_built):
    F0, T0, x0, d0 = _run(False)
    F1, T1, x1, d1 = _run(True)
    s = np.max(np.abs(F0))
    assert np.max(np.abs(F1 - F0)) <= 1e-12 * s
    assert np.max(np.abs(T1 - T0)) <= 1e-12 * np.max(np.abs(T0))
    assert np.max(np.abs(x1 - x0)) <= 1e-15
    assert np.max(np.abs(d1 - d0)) <= 1e-12 * np.max(np.abs(d0))


def test_parallel_build_is_deterministic_across_thread_counts(oracle_built):
    code = ("import sys, numpy as np; sys.path.insert(0, %r); "
            "from tests.test_oracle_parallel_build import _run; "
            "F, T, x, d = _run(True); sys.stdout.write(np.concatenate([F.ravel(), T.ravel(), "
            "x.ravel()]).tobytes().hex())") % ROOT
    outs = []
    for threads in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300, cwd=ROOT)
        assert r.returncode == 0, r.stderr
        outs.append(r.stdout)
    assert outs[0] == outs[1]
