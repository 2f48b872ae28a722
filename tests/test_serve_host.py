"""The serving runtime's host code (csrc/serve.cpp) under AddressSanitizer with
UndefinedBehaviorSanitizer, and under ThreadSanitizer, built with g++ against host
stand-ins for the HIP runtime, the step and the device sampler (tests/serve_host/): a
stream of requests through 8 workers, every request borrowing its host arrays, both
precisions, one or two steps each.  The stand-in queues every asynchronous copy on its
stream and runs it only when the stream is synchronized (or by a later step on that
stream), so a source buffer that the host frees or reuses while its copy is still in
flight is reported.  Results must come back in request order."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_serving_host_code_is_clean_under_sanitizers(tmp_path, san):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no g++")
    src = os.path.join(ROOT, "paper_2101_12408_amd", "csrc")
    here = os.path.join(ROOT, "tests", "serve_host")
    exe = str(tmp_path / "serve_san")
    flags = [f"-fsanitize={san}", "-fno-omit-frame-pointer"]
    if san != "thread":
        flags.append("-fno-sanitize-recover=all")
    subprocess.run([cxx, "-std=c++17", "-O1", "-g", *flags, "-I", here, "-I", os.path.join(ROOT, "include"),
                    os.path.join(src, "serve.cpp"), os.path.join(src, "sampler.cpp"),
                    os.path.join(here, "stub_lib.cpp"), os.path.join(here, "driver.cpp"), "-o", exe, "-lpthread"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, "60"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "bad 0" in r.stdout
