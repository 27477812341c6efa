"""Host logic of bench.py: algorithmic bytes of the matvec forms, and the
rule that a committed HBM-traffic figure is reported only while the machine
code of every kernel it was measured on is unchanged.  No GPU."""
import json

import bench


def test_matvec_bytes_counts_each_form():
    # every 4th iteration is the exact form (52 + 24C), the others the
    # recurrence (48 + 28C)
    for C in (1, 2, 21):
        assert bench.matvec_bytes(C, 4) == (52 + 24 * C) + 3 * (48 + 28 * C)
        assert bench.matvec_bytes(C, 3) == 3 * (48 + 28 * C)


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
