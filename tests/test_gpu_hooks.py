"""Failure hooks and device-side hygiene, forced from the host (GPU).

  * HOLO_WORKSPACE_CAP forces HOLO_ENOMEM before anything is enqueued, and the
    library works again once it is lifted;
  * HOLO_DEBUG_FAIL=device makes every launch (direct or a cached graph)
    return HOLO_EDEVICE, after which the library still works;
  * HOLO_DEBUG_POISON=1 fills each call's workspace with NaN bytes first: a
    kernel that reads scratch it did not write would change the results, so
    poisoned runs must equal clean ones bit for bit;
  * every path run twice gives the same bits and NMSE (an LDS or ordering race
    would show as nondeterminism).
Every kernel exits normally in all of these: the hooks act on the host.
"""
import os

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

HOLO_ENOMEM, HOLO_EDEVICE = -3, -4


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    assert torch.cuda.is_available()
    return h


@pytest.fixture
def env():
    saved = {k: os.environ.get(k) for k in ("HOLO_WORKSPACE_CAP", "HOLO_DEBUG_FAIL", "HOLO_DEBUG_POISON")}
    yield os.environ
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def _runs(h, stream):
    """One OSPR frame, one batched pair of frames, a GS run and a replay of
    eight-level codes: (bits..., NMSE values...) as numpy arrays."""
    with torch.cuda.stream(stream):
        t = torch.from_numpy(synth.blob_target(256, 128, 31)).cuda()
        lut = h.Lut(10007, 1)
        bits, nm, _ = h.ospr_generate(t, 5, lut, 11)
        t2 = torch.from_numpy(synth.blob_target(128, 128, 32)).cuda()
        bb, nmb, _ = h.ospr_generate_batched([t, t2], [3, 4], lut, 5)
        tg = torch.from_numpy(synth.blob_target(128, 128, 33)).cuda()
        g = h.gs_iterate(tg, 6, h.Lut(4096, 1), 0, want_err=True)
        r8 = h.reconstruct_nmse(g["codes"].reshape(1, 128, 128), 8, 128, 128, 1, tg)
        torch.cuda.synchronize()
        return [bits.cpu().numpy(), nm, *[b.cpu().numpy() for b in bb], np.asarray(nmb),
                g["codes"].cpu().numpy(), g["field"].cpu().numpy(), g["nmse"], g["err"], g["nmse_final2"], r8]


def test_workspace_cap_forces_enomem(holo, env):
    t = torch.from_numpy(synth.blob_target(256, 256, 3)).cuda()
    lut = holo.Lut(10007, 1)
    env["HOLO_WORKSPACE_CAP"] = "4096"
    print("workspace cap 4096: ospr 256x256x4", flush=True)
    with pytest.raises(holo.HoloError) as e:
        holo.ospr_generate(t, 4, lut, 0)
    assert e.value.status == HOLO_ENOMEM and "HOLO_WORKSPACE_CAP" in str(e.value)
    with pytest.raises(holo.HoloError) as e:
        holo.gs_iterate(t, 2, lut, 0)
    assert e.value.status == HOLO_ENOMEM
    del env["HOLO_WORKSPACE_CAP"]
    _, nm, cur = holo.ospr_generate(t, 4, lut, 0)
    assert cur == 4 * 256 * 256 and 0.0 < nm[0] < 1.0


def test_debug_fail_forces_edevice(holo, env):
    s = torch.cuda.Stream()
    t = torch.from_numpy(synth.blob_target(128, 128, 4)).cuda()
    lut = holo.Lut(4096, 1)
    with torch.cuda.stream(s):
        ref = holo.gs_iterate(t, 3, lut, 0)          # captures and caches the GS graph
        _, nm_ref, _ = holo.ospr_generate(t, 2, lut, 0)
        env["HOLO_DEBUG_FAIL"] = "device"
        print("forced device failure: ospr, cached GS graph, batched", flush=True)
        for f in (lambda: holo.ospr_generate(t, 2, lut, 0),
                  lambda: holo.gs_iterate(t, 3, lut, 0),
                  lambda: holo.ospr_generate_batched([t], [2], lut, 0)):
            with pytest.raises(holo.HoloError) as e:
                f()
            assert e.value.status == HOLO_EDEVICE and "HOLO_DEBUG_FAIL" in str(e.value)
        del env["HOLO_DEBUG_FAIL"]
        again = holo.gs_iterate(t, 3, lut, 0)
        _, nm, _ = holo.ospr_generate(t, 2, lut, 0)
        torch.cuda.synchronize()
    assert np.array_equal(again["nmse"], ref["nmse"])
    assert np.array_equal(nm, nm_ref)


def test_poisoned_workspace_and_repeat_runs_are_identical(holo, env):
    s = torch.cuda.Stream()
    print("clean runs x2, then poisoned run", flush=True)
    a = _runs(holo, s)
    b = _runs(holo, s)
    env["HOLO_DEBUG_POISON"] = "1"
    c = _runs(holo, s)
    del env["HOLO_DEBUG_POISON"]
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y), "a repeated run differs"
        assert np.array_equal(x, z), "a run on a poisoned workspace differs"
    assert all(np.all(np.isfinite(np.asarray(x, dtype=np.complex128))) for x in a if x.dtype.kind in "fc")
