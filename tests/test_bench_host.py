"""Host logic of bench.py (CPU only): the canonical byte model per launch and
the gating of measured traffic on kernel sources and sub-frames per launch."""
import json

import bench


def test_byte_model_per_subframe():
    # per sub-frame: K1 writes 8 B/px, K2 reads 8 and writes 1/8 + 8, K3 reads 8;
    # the target (4 B/px) is read once per frame by K1 and once by K3
    nx = ny = 1024
    n = nx * ny
    n_sf = 24
    kb = bench.ospr_kernel_bytes(nx, ny, n_sf, 65536)
    total = sum(kb.values())
    assert total == n * (32.125 * n_sf + 8)
    assert kb["ospr_cols"] == n_sf * n * 16.125
    # chunked plans: K1 and K2 per launch of `chunk` sub-frames; K3 whole frame
    kc = bench.ospr_kernel_bytes(nx, ny, n_sf, 65536, chunk=8)
    assert kc["ospr_cols"] == 8 * n * 16.125
    assert kc["ospr_rows"] * 3 == kb["ospr_rows"]
    assert kc["recon_rows"] == kb["recon_rows"]
    # a table longer than 2^16 entries is charged to K1 (8 B per unique entry read)
    big = bench.ospr_kernel_bytes(nx, ny, n_sf, 1 << 20)
    assert big["ospr_rows"] - kb["ospr_rows"] == 8 * (1 << 20)
    huge = bench.ospr_kernel_bytes(nx, ny, n_sf, 1 << 30)
    assert huge["ospr_rows"] - kb["ospr_rows"] == 8 * n * n_sf


def test_measured_traffic_gating(tmp_path, monkeypatch):
    root = tmp_path
    (root / "profiles").mkdir()
    h = bench.source_hash()
    rec = {"w": {"ospr_cols": {"bytes_per_launch": 123, "source_hash": h, "sf_per_launch": 24}}}
    (root / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.measured_traffic("ospr_cols", "w", 24) == 123
    assert bench.measured_traffic("ospr_cols", "w", 12) is None        # other chunking
    assert bench.measured_traffic("ospr_rows", "w", 24) is None        # not profiled
    assert bench.measured_traffic("ospr_cols", "other", 24) is None
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)        # sources changed
    assert bench.measured_traffic("ospr_cols", "w", 24) is None


def test_committed_traffic_record_is_complete():
    # the committed profile summary names every OSPR kernel with its bytes, the
    # sources it was taken on and the sub-frames per launch (whether it still
    # applies is decided at run time: the bench reports null otherwise)
    with open(bench.os.path.join(bench.ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    entries = rec["ospr_1024x1024_sf24_lut65536"]
    assert set(entries) >= {"ospr_rows", "ospr_cols", "recon_rows"}
    for e in entries.values():
        assert len(e["source_hash"]) == 16 and e["sf_per_launch"] == 24
        assert abs(e["bytes_per_launch"] - e["fetch_bytes"] - e["write_bytes"]) <= 1   # rounded separately


def test_design_bytes_half_planes():
    # binary frames: half planes of (ny/2 + 1) rows, 8 B per complex value
    nx = ny = 1024
    n = nx * ny
    n_sf = 24
    half = (ny // 2 + 1) * nx * 8
    db = bench.ospr_design_bytes(nx, ny, n_sf, 65536)
    assert db["ospr_rows"] == n_sf * half + 4 * n
    assert db["ospr_cols"] == n_sf * (2 * half + n / 8)
    assert db["recon_rows"] == n_sf * half + 4 * n
    # about half the canonical bytes, never more
    kb = bench.ospr_kernel_bytes(nx, ny, n_sf, 65536)
    for k in db:
        assert 0.45 * kb[k] < db[k] < 0.55 * kb[k] + 8 * n
    # chunking and large tables behave as in the canonical model
    dc = bench.ospr_design_bytes(nx, ny, n_sf, 65536, chunk=8)
    assert dc["ospr_cols"] * 3 == db["ospr_cols"]
    big = bench.ospr_design_bytes(nx, ny, n_sf, 1 << 20)
    assert big["ospr_rows"] - db["ospr_rows"] == 8 * (1 << 20)
    # the committed K2 traffic agrees with the design bytes within the margin
    with open(bench.os.path.join(bench.ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    e = rec["ospr_1024x1024_sf24_lut65536"]["ospr_cols"]
    assert abs(e["bytes_per_launch"] / db["ospr_cols"] - 1) <= bench.TRAFFIC_MARGIN


def test_measured_batch_traffic_gating(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    h = bench.source_hash()
    rec = {"batched_64frames": {"fp32": {"bytes_per_batch": 7, "fetch_bytes": 4, "write_bytes": 3,
                                         "design_bytes": 100, "plans": {}, "source_hash": h, "frames": 64}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.measured_batch_traffic("fp32", 100)["bytes_per_batch"] == 7
    assert bench.measured_batch_traffic("fp32", 101) is None           # another batch layout
    assert bench.measured_batch_traffic("bf16", 100) is None           # not profiled
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)        # sources changed
    assert bench.measured_batch_traffic("fp32", 100) is None


def test_committed_batch_traffic_matches_the_benchmark_batch():
    # the committed batch record was taken on the benchmark's 64-frame layout
    import synth
    design = sum(sum(bench.ospr_design_bytes(n, n, k, 10007).values())
                 for n, k in synth.batch_layout(64, synth.SEED_BATCH))
    with open(bench.os.path.join(bench.ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)["batched_64frames"]
    assert set(rec) == {"fp32", "bf16", "fp16"}
    for e in rec.values():
        assert e["design_bytes"] == int(design) and e["frames"] == 64
        assert abs(e["bytes_per_batch"] - e["fetch_bytes"] - e["write_bytes"]) <= 1
        # measured bytes within 10% of the design bytes (row pitch, re-reads)
        assert 1.0 <= e["bytes_per_batch"] / design < 1.1
