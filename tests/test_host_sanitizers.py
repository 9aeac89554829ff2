"""The C++ runtime under the host sanitizers: the serving scheduler (its
threads, queues, cancellation and time-outs, with the fake executor) and the
C-ABI argument checks run against a build whose host code is instrumented
with AddressSanitizer or ThreadSanitizer (`python -m paper_2311_05646_amd.build
--sanitize address|thread`, about two minutes each, written to _build/).
Skipped when that build is absent."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SUITES = {"address": ["tests/test_serving_cpu.py", "tests/test_abi.py"],
          "thread": ["tests/test_serving_cpu.py"]}
OPTIONS = {"address": ("ASAN_OPTIONS", "detect_leaks=0:halt_on_error=1"),
           "thread": ("TSAN_OPTIONS", "halt_on_error=1:report_signal_unsafe=0")}


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_runtime_is_clean_under_sanitizer(kind):
    from paper_2311_05646_amd import build
    lib = os.path.join(build.SAN_DIR, f"libshapegrad_{build.SANITIZERS[kind]}.so")
    if not os.path.exists(lib):
        pytest.skip(f"no {kind}-sanitized build (python -m paper_2311_05646_amd.build --sanitize {kind})")
    runtime = build.sanitizer_runtime(kind)
    assert os.path.exists(runtime), runtime
    key, opts = OPTIONS[kind]
    env = dict(os.environ, SG_LIB_PATH=lib, LD_PRELOAD=runtime, **{key: opts})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider"] + SUITES[kind],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out, out[-4000:]
