"""The host side of the library (argument checks, sizes, error strings, plan
and workspace bookkeeping reached without a GPU) built with AddressSanitizer
and UndefinedBehaviorSanitizer (host code only) and driven through its C ABI in
a separate process with the ASan runtime preloaded: every documented status
comes back and no sanitizer report appears."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    for clang in ("/opt/rocm/llvm/bin/clang", "clang"):
        try:
            out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                 capture_output=True, text=True, timeout=30).stdout.strip()
        except (OSError, subprocess.TimeoutExpired):
            continue
        if out and os.path.isabs(out) and os.path.exists(out):
            return out
    return None


def test_host_paths_under_sanitizers():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime in this toolchain")
    spec = importlib.util.spec_from_file_location(
        "_tn_build", os.path.join(ROOT, "paper_2504_08339_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    lib = build.build_host_sanitized()
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True,
                          text=True).stdout
    assert "__asan_report_load4" in syms and "__ubsan_handle_" in syms  # instrumented
    env = dict(os.environ, LD_PRELOAD=rt, HIP_VISIBLE_DEVICES="",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_san_driver.py"), lib,
                          ROOT], capture_output=True, text=True, env=env, timeout=300)
    report = res.stdout + res.stderr
    assert "AddressSanitizer" not in report and "runtime error:" not in report, report[-4000:]
    assert res.returncode == 0 and "host paths clean" in res.stdout, report[-4000:]
