"""Host-side parts of bench.py, on the CPU: the algorithmic byte model and
the choice of the counter summary that backs the roofline's traffic field."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_bytes_model():
    b = _bench()
    n = 1 << 24
    # a scatter pass reads and writes every term once: key + amplitude
    assert b.kernel_bytes("radix_pass", 8, n, 0, 0) == 2 * 16 * n
    assert b.kernel_bytes("radix_pass", 16, n, 0, 0) == 2 * 24 * n
    assert b.kernel_bytes("radix_hist", 8, n, 0, 0) == 8 * n
    assert b.kernel_bytes("group_emit", 8, n, n // 2, 0) == 2 * 16 * (n // 2)
    assert b.kernel_bytes("group_hist", 16, n, n // 2, 0) == 24 * n + 24 * (n // 2)
    assert b.kernel_bytes("pick1", 8, n, n, n) == 0.0


def test_traffic_summary_matches_configuration():
    b = _bench()
    # no summary for configurations other than the committed one(s)
    assert b.measured_traffic("radix_pass", 1e-4, None) is None
    assert b.measured_traffic("radix_pass", 1e-4, "peaked48_K2e24_c128") is None
    assert b.measured_traffic("group_hist", 1e-4, "peaked48_K2e24_c64") is None
    # the committed complex64 summary: reported only while its source digest
    # matches the library sources
    from paper_2607_07816_amd import profsum
    path = os.path.join(ROOT, "profiles", "radix_pass_peaked48_K2e24_c64_hbm_traffic.txt")
    rec = profsum.read_traffic(path)
    got = b.measured_traffic("radix_pass", 1e-4, "peaked48_K2e24_c64")
    if rec.get("source_digest") == profsum.source_digest():
        assert abs(got - float(rec["traffic_bytes_per_launch"]) / 1e-4 / 1e9) < 1e-6
    else:
        assert got is None
