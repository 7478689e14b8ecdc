"""The served form's host core (csrc/served_core.h: arena sub-allocator,
request queue, admission, stream slots and the request thread's loop) built
for the CPU with a simulated device, and run under AddressSanitizer +
UndefinedBehaviorSanitizer and under ThreadSanitizer
(tests/host/served_core_test.cpp lists what it checks: every ticket completes
once with its own result, per-controller order, EAGAIN, ESTATE, ENOMEM at
admission, EDEVICE, ETIMEDOUT, ECANCELED, the arena and controllers released)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "served_core_test.cpp")
INC = [os.path.join(ROOT, "include"), os.path.join(ROOT, "paper_2508_05773_amd", "csrc")]

SANITIZERS = {
    "asan_ubsan": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"],
                   {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"}),
    "tsan": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
}


@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_served_core_under_sanitizer(kind, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    flags, env_extra = SANITIZERS[kind]
    exe = str(tmp_path / f"served_core_{kind}")
    cmd = [gxx, "-std=c++17", "-O1", "-g", *flags, *sum((["-I", d] for d in INC), []), SRC, "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    print(r.stdout)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "served core: all checks passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
