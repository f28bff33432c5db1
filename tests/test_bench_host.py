"""Host logic of the benchmark: the HBM traffic it reports comes from the
committed counter summary of the kernel it names, and only while that
summary was taken on the current kernel sources."""
import json
import os

import bench

CASES = [
    (bench.COUNTERS_FILE, bench.KERNEL_SOURCES, bench.KERNEL_I8),
    (bench.COUNTERS_FILE_F16, bench.KERNEL_SOURCES_F16, bench.KERNEL_F16),
]


def _record(path):
    text = open(path).read()
    return json.loads(text.split("```json", 1)[1].split("```", 1)[0])


def test_summaries_name_the_benched_kernels():
    for path, _, kernel in CASES:
        assert os.path.exists(path), path
        rec = _record(path)
        assert rec["kernel"] == kernel, path
        assert rec["traffic_bytes_per_launch"] > 0, path


def test_traffic_follows_kernel_and_sources():
    for path, sources, kernel in CASES:
        rec = _record(path)
        current = rec["kernel_source_sha"] == bench.kernel_source_sha(sources)
        want = rec["traffic_bytes_per_launch"] if current else None
        assert bench.measured_traffic(path, sources, kernel) == want, path
        # another kernel's name, or another kernel's sources, gives nothing
        other = [k for _, _, k in CASES if k != kernel][0]
        assert bench.measured_traffic(path, sources, other) is None, path
    assert bench.measured_traffic(bench.COUNTERS_FILE_F16, bench.KERNEL_SOURCES,
                                  bench.KERNEL_F16) is None


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    d = tmp_path / "paper_2009_05534_amd" / "csrc"
    d.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (d / "k.hip").write_text("int f() { return 1; }  // one\n")
    a = bench.kernel_source_sha(("k.hip",))
    (d / "k.hip").write_text("/* two */\nint f() {\n  return 1;\n}\n")
    assert bench.kernel_source_sha(("k.hip",)) == a
    (d / "k.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_sha(("k.hip",)) != a
