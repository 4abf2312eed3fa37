"""The runtime's host code under address and undefined-behaviour
sanitizers: `lbm_host_check` (built by the package build from
csrc/host_check.cpp and a sanitized copy of csrc/lbm_api.hip, linked with
the product's kernels) drives every entry point of include/lbm.h for every
storage, temperature model, collision operator and wall family, launch
policies, graphs, state save/restore and batches, and must finish clean."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1510_08224_amd", "lbm_host_check")


def test_runtime_host_code_is_clean_under_sanitizers():
    assert os.path.exists(EXE), "lbm_host_check is missing: run the package build"
    # leaks of the (uninstrumented) HIP runtime are not ours to report
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "host check ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
