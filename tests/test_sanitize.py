"""Host sanitizers on the FP64 oracle (CPU): the oracle's C sources and a
driver that calls every routine on small inputs (tests/sanitize_oracle.c) are
built with gcc's AddressSanitizer and UndefinedBehaviorSanitizer and run in a
child process; any report fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    srcs = [os.path.join(HERE, "sanitize_oracle.c")] + [
        os.path.join(ROOT, "oracle", f) for f in ("holo_oracle.c", "cnn_oracle.c", "phase_oracle.c")]
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-o", exe, *srcs, "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "SANITIZE_OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
