"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):

* the query planner of the runtime (paper_1805_00754_amd/csrc/plan.h, the
  Alg. 3 index math of every query) built with g++ into a checker that
  compares it with an enumeration of the rows on thousands of random stores
  and ranges (tests/hostcheck/plan_check.cpp);
* the oracle (oracle/zoom_oracle.c) built with gcc and every entry point run
  once on small inputs, in a child interpreter with the sanitizer runtime
  preloaded.

Any invalid access or undefined behaviour aborts the run (no recovery)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_00754_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc / g++")


def test_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *SAN, "-I", CSRC,
                    os.path.join(ROOT, "tests", "hostcheck", "plan_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "plan_check ok" in r.stdout


CHILD = r"""
import sys
sys.path.insert(0, %(root)r)
import numpy as np
import oracle
from paper_1805_00754_amd import synth
lib = oracle.load(%(so)r)
A = synth.sinusoid_mixture(1_210, 12, sources=4, seed=2, noise="iid", noise_sigma=0.1).A
oracle.svd(A[:90], lib=lib)
st = oracle.store(A, 100, 5, lib=lib)
stx = oracle.store(A, 100, 5, lib=lib, xi=0.9)
for ts, te in [(0, 1_210), (37, 1_163), (120, 180), (99, 101), (1_200, 1_210)]:
    oracle.query(st, ts, te, 4, lib=lib)
    oracle.query(stx, ts, te, 4, lib=lib)
    oracle.direct(A, ts, te, 4, lib=lib)
oracle.query_batch(st, np.array([0, 5, 300]), np.array([1_210, 6, 1_000]), 3, lib=lib)
oracle.direct_batch(A, np.array([0, 5]), np.array([700, 400]), 3, lib=lib)
oracle.partial_svd(st, 3, 10, 70, lib=lib)
oracle.xi_rank(np.array([3.0, 2.0, 1.0, 0.5]), 0.9, lib=lib)
oracle.query_blocks(37, 1_163, 100, lib=lib)
B = synth.sinusoid_mixture(330, 12, sources=4, seed=3, noise="iid", noise_sigma=0.1).A
oracle.append(st, B, lib=lib)
oracle.window_similarity(st, 900, 1_200, 50, 4, lib=lib)
print("oracle ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    so = str(tmp_path / "liboracle_san.so")
    flags = [f for f in oracle.CFLAGS if f != "-O3"] + ["-O1", "-g"] + SAN
    subprocess.run(["gcc", *flags, "-o", so, os.path.join(ROOT, "oracle", "zoom_oracle.c"), "-lm"],
                   check=True, capture_output=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD % dict(root=ROOT, so=so)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "oracle ok" in r.stdout
