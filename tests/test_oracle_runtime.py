"""The oracle as a program (CPU only): its OpenMP loops give the same bits on
one thread and on several, and a driver over every stage and option runs
clean under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2103_15196_amd import workloads as W
from tests.helpers import oracle_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_threads_give_the_same_bits(oracle_mod):
    """Every loop of the oracle runs over independent cells or faces and sums
    in a fixed order: one thread and four give identical fields and
    balances (river valley with inflow, per-cell soil, open side; second-order
    force and MC limiter in a second run)."""
    O = oracle_mod
    w = W.river_valley(n=96, ny=64, dx=5.0, amplitude=30.0, wavelength=300.0, width=30.0,
                       Q_base=20.0, Q_peak=100.0, t_peak=10.0, t_sigma=5.0)
    w.H = np.where(w.b < np.quantile(w.b, 0.2), 1.0, 0.0)
    n0 = O.threads()
    try:
        for over in ({}, dict(limiter=1, force_order=2)):
            out = []
            for nthr in (1, 4):
                O.set_threads(nthr)
                p, inp, s = oracle_case(O, w, **over)
                O.run(p, inp, s, 60)
                out.append((s.H.copy(), s.qx.copy(), s.qy.copy(), s.b.copy(), s.t, s.out_w, s.in_w))
            for a, b in zip(*out):
                assert np.array_equal(a, b), over
    finally:
        O.set_threads(n0)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_runs_clean_under_address_and_undefined_sanitizers():
    """tests/oracle_sanitize_driver.c includes the oracle source and runs 40
    steps of every limiter x speed estimate x force order x bedload law on
    small grids with all sources and forcing; built with
    -fsanitize=address,undefined (host code, gcc), any report fails it."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "drv")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                               os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
                               "-o", exe, "-lm"])
        # the driver's own runtime is linked statically into nothing else;
        # a library the environment preloads may come before it
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
