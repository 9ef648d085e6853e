"""Host-side bookkeeping of bench.py: which source family defines each kernel,
and measured HBM traffic reported only while that family's sources are
unchanged since the counters were taken."""
import json

import bench


def test_kernel_families():
    for k in ("k_pass1", "k_pass2", "k_hist", "k_scan", "k_bin_geo"):
        assert bench.kernel_sources(k) is bench.NUFFT_SOURCES, k
    for k in ("k_sym_topk", "k_gram_mfma", "k_lr_basis", "k_t_analyze", "k_syrk"):
        assert bench.kernel_sources(k) is bench.GEP_SOURCES, k
    assert bench.kernel_sources("k_no_such_kernel") is None


def test_traffic_follows_source_hash(tmp_path, monkeypatch):
    good = bench.sources_sha256(bench.NUFFT_SOURCES)
    recs = [{"kernel": "k_pass1", "bytes_per_launch": 123, "sources_sha256": good},
            {"kernel": "k_pass2", "bytes_per_launch": 456, "sources_sha256": "0" * 64}]
    f = tmp_path / "traffic.md"
    f.write_text("# t\n" + "".join("<!-- traffic " + json.dumps(r) + " -->\n" for r in recs))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("k_pass1") == 123
    assert bench.measured_traffic("k_pass2") is None       # sources changed since
    assert bench.measured_traffic("k_scatter") is None     # no record
