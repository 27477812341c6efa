"""Host logic of bench.py: algorithmic bytes of the PCG iterations, and the
rule that a committed HBM-traffic figure is reported only while the machine
code of every kernel it was measured on is unchanged.  No GPU."""
import json

import bench


def test_pcg_bytes_counts_active_channels():
    # 48 bytes per vertex and iteration while any channel iterates, plus 24
    # per channel for its own iterations
    assert bench.pcg_bytes(10, [5]) == 10 * (48 * 5 + 24 * 5)
    assert bench.pcg_bytes(10, [5, 3, 0]) == 10 * (48 * 5 + 24 * 8)
    assert bench.pcg_bytes(7, []) == 0
    assert bench.pcg_bytes(3, [4] * 21) == 3 * 4 * (48 + 24 * 21)


def test_traffic_needs_the_measured_machine_code(tmp_path, monkeypatch):
    traffic = tmp_path / "traffic.json"
    code = tmp_path / "kernel_code.json"
    traffic.write_text(json.dumps({"workloads": {
        "w": {"bytes_per_launch": 123, "kernels": {"bs::k<1>": "aa", "bs::k<2>": "bb"}},
        "old": {"bytes_per_launch": 7}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    monkeypatch.setattr(bench, "KERNEL_CODE", str(code))
    code.write_text(json.dumps({"bs::k<1>": "aa", "bs::k<2>": "bb", "bs::k<3>": "cc"}))
    assert bench._measured_traffic("w") == 123
    assert bench._measured_traffic("old") is None          # no kernel digests recorded
    assert bench._measured_traffic("missing") is None
    code.write_text(json.dumps({"bs::k<1>": "aa", "bs::k<2>": "changed"}))
    assert bench._measured_traffic("w") is None
    code.write_text(json.dumps({"bs::k<1>": "aa"}))
    assert bench._measured_traffic("w") is None
    code.unlink()
    assert bench._measured_traffic("w") is None
