"""The oracle and the host side of librs built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: GPU code is not instrumented)
and driven on the CPU: tests/sanitize/oracle_driver.c runs every oracle sort
against qsort, tests/sanitize/host_driver.cpp every host-side entry point
of librs that needs no GPU (argument checks, workspace sizes, the tuning
table and its JSON reader on truncated and corrupted files, options).  A
sanitizer report aborts the driver, which fails the test."""
import os
import shutil
import subprocess
import concurrent.futures as cf

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_09495_amd", "csrc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g"] + SAN + ["-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                      os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc to build the library")
def test_library_host_code_under_sanitizers(tmp_path):
    # host code instrumented: each -fsanitize= after -Xarch_host
    hsan = []
    for f in SAN:
        hsan += ["-Xarch_host", f]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops"] + hsan
    srcs = ["rs_lsd.hip", "rs_wide.hip", "rs_small.hip", "rs_seg.hip", "rs_blocks.hip", "rs_learned.hip",
            "rs_tune.hip", "rs_api.cpp"]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        _run(["hipcc"] + flags + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "host_driver.o")
    _run(["g++", "-O1", "-g", "-std=c++17"] + SAN + ["-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                                                    "-o", drv])
    exe = str(tmp_path / "host_driver")
    _run(["hipcc", "--offload-arch=gfx950"] + hsan[:4] + ["-o", exe, drv] + objs)
    files = tmp_path / "files"
    files.mkdir()
    r = _run([exe, str(files)], env=ENV, timeout=600)
    assert "host driver: ok" in r.stdout
