"""Build-level guard (CPU only): in the gfx950 code of every kernel source, a
buffer store wider than 64 bits per lane has a zero scalar offset, and the
next instruction does not overwrite its data registers.

A buffer store of more than 8 bytes per lane may read its data registers after
the next vector instruction has overwritten them.  The compiler inserts the
wait for the form without a scalar-register offset; with one, it leaves the
store unguarded, and on gfx950 such 16-byte stores were seen to lose data words
(some lanes, some blocks).  The kernels therefore pass the whole offset of a
16-byte store in the lane register.  This test compiles each source to AMD
assembly with the library's own flags and checks both properties, so that a
change of code or compiler that brings back the unguarded form fails here.

The same assembly also shows each kernel's scratch (private segment) size:
every kernel keeps its data in registers and LDS, so a nonzero size means a
register array the compiler could not promote, or spills.
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

WIDE = re.compile(r"^\s*buffer_store_dwordx[34]\s+(\S+),\s*(\S+),\s*(s\[\d+:\d+\]),\s*(\S+)")


def _vregs(spec):
    m = re.match(r"v\[(\d+):(\d+)\]$", spec)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", spec)
    return {int(m.group(1))} if m else set()


def _asm(src, out_dir):
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [holo_build.HIPCC, *holo_build.CFLAGS, "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    with open(out) as f:
        return os.path.basename(src), f.read().splitlines()


def _problems(lines):
    bad = []
    for i, line in enumerate(lines):
        m = WIDE.match(line)
        if not m:
            continue
        if m.group(4) != "0":
            bad.append(("scalar offset", line.strip()))
            continue
        j = i + 1
        while j < len(lines) and (not lines[j].strip() or lines[j].lstrip().startswith((";", "."))):
            j += 1
        nxt = lines[j].strip() if j < len(lines) else ""
        if nxt.startswith("v_"):
            dst = nxt.split(None, 1)[1].split(",")[0].strip()
            if _vregs(dst) & _vregs(m.group(1)):
                bad.append(("data overwritten", line.strip() + " / " + nxt))
    return bad


needs_hipcc = pytest.mark.skipif(not os.path.exists(holo_build.HIPCC) and shutil.which("hipcc") is None,
                                 reason="hipcc not available")


@pytest.fixture(scope="module")
def kernel_asm(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asm"))
    srcs = holo_build.sources()
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        return list(ex.map(lambda s: _asm(s, out), srcs))


@needs_hipcc
def test_wide_buffer_stores_are_guarded(kernel_asm):
    bad = {name: probs[:3] for name, lines in kernel_asm if (probs := _problems(lines))}
    assert not bad, f"unguarded wide buffer stores: {bad}"


def _scratch(lines):
    """(kernel, private segment bytes) for every kernel descriptor."""
    out, name = [], None
    for line in lines:
        t = line.split()
        if len(t) == 2 and t[0] == ".amdhsa_kernel":
            name = t[1]
        elif len(t) == 2 and t[0] == ".amdhsa_private_segment_fixed_size":
            out.append((name, int(t[1])))
    return out


@needs_hipcc
def test_no_kernel_uses_scratch(kernel_asm):
    sizes = [(src, k, n) for src, lines in kernel_asm for k, n in _scratch(lines)]
    assert len(sizes) > 100   # every source's kernels were found
    bad = [(src, k, n) for src, k, n in sizes if n != 0]
    assert not bad, f"kernels with scratch: {bad[:5]}"


def test_scratch_parser():
    lines = ["\t.amdhsa_kernel _Z1kv", "\t\t.amdhsa_private_segment_fixed_size 152", "\t.end_amdhsa_kernel",
             "\t.amdhsa_kernel _Z1jv", "\t\t.amdhsa_private_segment_fixed_size 0"]
    assert _scratch(lines) == [("_Z1kv", 152), ("_Z1jv", 0)]


def test_checker_flags_the_unguarded_forms():
    # the checker itself, on hand-written lines
    assert _problems(["buffer_store_dwordx4 v[2:5], v1, s[0:3], s77 offen", "v_mov_b32 v9, 0"])
    assert _problems(["buffer_store_dwordx4 v[2:5], v1, s[0:3], 0 offen", "v_mul_f32_e32 v2, 0.5, v0"])
    assert not _problems(["buffer_store_dwordx4 v[2:5], v1, s[0:3], 0 offen", "s_nop 1",
                          "v_mul_f32_e32 v2, 0.5, v0"])
    assert not _problems(["buffer_store_dwordx2 v[2:3], v1, s[0:3], s77 offen", "v_mov_b32 v2, 0"])
