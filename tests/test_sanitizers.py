"""CPU sanitizer runs (no GPU): the oracle and the library's host code built
with AddressSanitizer + UndefinedBehaviorSanitizer, and the host code with
ThreadSanitizer (tests/sanitize/build.py), each loaded into a pytest
subprocess that preloads the sanitizer runtime:

* ASan/UBSan: the C-ABI host tests (validation of malformed scenes, sizes,
  layouts and the walk of every collision plan), the scheduler tests on a
  fake executor, the acceptance-rule tests and the oracle's pins;
* TSan: the scheduler tests (submitting, waiting and the scheduler thread
  calling a caller's executor concurrently).

A sanitizer report ends the subprocess with an error status (halt on the
first report), which fails the test with the report's text."""
import os
import subprocess
import sys

import pytest

from tests.sanitize import build as sb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

ASAN_TESTS = ["tests/test_abi_cpu.py", "tests/test_server_cpu.py", "tests/test_parity_rule.py",
              "tests/test_oracle_geometry.py", "tests/test_oracle_motion_risk.py", "tests/test_oracle_pip.py",
              "tests/test_oracle_polygons.py", "tests/test_oracle_models.py", "tests/test_oracle_timeline.py"]
TSAN_TESTS = ["tests/test_server_cpu.py"]


def _instrumented(lib: str, symbol: str) -> bool:
    out = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    return symbol in out


def _run(kind: str, env_extra: dict, tests, tmp_path):
    report = str(tmp_path / f"{kind}_report")
    env = dict(os.environ)
    env.update(env_extra)
    env["MHC_NO_TORCH"] = "1"
    env["LD_PRELOAD"] = sb.runtime_library(kind)
    opts = f"halt_on_error=1:log_path={report}"
    if kind == "asan":
        env["ASAN_OPTIONS"] = "detect_leaks=0:" + opts
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:" + opts
    else:
        env["TSAN_OPTIONS"] = "report_signal_unsafe=0:" + opts
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = [f for f in os.listdir(tmp_path) if f.startswith(f"{kind}_report")]
    text = "".join(open(os.path.join(tmp_path, f)).read() for f in reports)
    assert r.returncode == 0 and not text, f"{kind} run failed ({r.returncode}):\n{text[:4000]}\n{r.stdout[-3000:]}"
    return r.stdout


def test_address_and_undefined_sanitizers(tmp_path):
    host = sb.build_host_library("asan")
    orc = sb.build_oracle()
    assert _instrumented(host, "__asan_init") and _instrumented(orc, "__asan_init")
    assert _instrumented(host, "__ubsan_handle") and _instrumented(orc, "__ubsan_handle")
    out = _run("asan", {"MHC_LIB_PATH": host, "ORACLE_LIB_PATH": orc}, ASAN_TESTS, tmp_path)
    assert " passed" in out


def test_thread_sanitizer_on_the_scheduler(tmp_path):
    host = sb.build_host_library("tsan")
    assert _instrumented(host, "__tsan_init")
    out = _run("tsan", {"MHC_LIB_PATH": host}, TSAN_TESTS, tmp_path)
    assert " passed" in out
