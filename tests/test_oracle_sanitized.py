"""Host sanitizer run of the oracle: the C source built with AddressSanitizer and UndefinedBehaviorSanitizer
(every report fatal, float-to-int overflow included) and with every uninitialised local filled with a NaN
pattern, then driven through each of its entry points in a child process. The child must exit cleanly and
give exactly the outputs of the normal build, so an out-of-bounds access, undefined behaviour or a value
read before it is written (which the NaN pattern would change) fails here. A rejected step's target read
for a particle that ended on the step limit was such a read."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan_and_pattern_init(tmp_path):
    from oracle import build
    if not os.path.exists(build.SAN_CC):
        pytest.skip("clang not available")
    build.build_sanitized(str(tmp_path))
    out = tmp_path / "san.npz"
    env = dict(os.environ, AVL_ORACLE_LIBDIR=str(tmp_path), LD_PRELOAD=build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]))
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "support", "sanitized_cases.py"), str(out)],
                         env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from support import sanitized_cases
    ref = sanitized_cases.run()
    got = np.load(out)
    assert sorted(got.files) == sorted(ref)
    for k, v in ref.items():
        assert np.array_equal(got[k], v, equal_nan=True), k
