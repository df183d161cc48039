"""The host index planner under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): the check program csrc/plan_check.cpp plans grid matrices with every
option, rejects malformed inputs, plans from two threads at once, releases the
process-wide caches and plans again, then exits through the library's exit
handler (worker threads joined, cached blocks released).  Any sanitizer
report, leak or failed check makes the program exit non-zero."""
import importlib.util
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "amsp_build", os.path.join(ROOT, "paper_2606_04864_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_ubsan():
    exe = _build_module().build_plan_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "PASSED (0 failures)" in r.stdout, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.stdout.count("\nok ") + r.stdout.startswith("ok ") >= 18
