"""Build-level guard (CPU only): the gfx950 code of every kernel source has no
buffer store wider than 64 bits per lane.

A 16-byte buffer store with a scalar-register offset was seen, on gfx950, to
read its data registers after the next vector instruction had overwritten
them (some lanes, some blocks), and the compiler guards that hazard only for
the form without a scalar offset.  The kernels therefore store at most 8 bytes
per lane through buffer descriptors; this test compiles each source to AMD
assembly with the library's own flags and checks that the compiler did not
merge adjacent stores back into wider ones.
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2004_04049_amd"))
import build as holo_build  # noqa: E402  (the package's build script; imports nothing of the library)

WIDE = re.compile(r"^\s*buffer_store_dwordx[34]\b", re.M)


def _asm(src, out_dir):
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [holo_build.HIPCC, *holo_build.CFLAGS, "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    with open(out) as f:
        return os.path.basename(src), f.read()


@pytest.mark.skipif(not os.path.exists(holo_build.HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_no_wide_buffer_stores(tmp_path):
    srcs = holo_build.sources()
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        results = list(ex.map(lambda s: _asm(s, str(tmp_path)), srcs))
    bad = {name: len(WIDE.findall(text)) for name, text in results if WIDE.search(text)}
    assert not bad, f"buffer stores wider than 64 bits: {bad}"
