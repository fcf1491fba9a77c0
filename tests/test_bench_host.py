"""Host logic of bench.py that decides what its JSON line reports (no GPU).

The roofline's traffic comes from the committed counter profile only while the contraction
kernel's code and the band count match what was profiled; these tests pin that rule.
"""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_digest_ignores_comments_and_whitespace_only():
    b = _bench()
    src = "int f(int x) {\n  return x + 1;  // add one\n}\n"
    same = "int f(int x){return x+1;}\n// a note\n"
    changed = "int f(int x) {\n  return x + 2;  // add one\n}\n"
    assert b.kernel_code_digest(src) == b.kernel_code_digest(same)
    assert b.kernel_code_digest(src) != b.kernel_code_digest(changed)


def test_traffic_is_reported_only_for_the_profiled_launch():
    b = _bench()
    src = open(os.path.join(ROOT, "paper_1003_1140_amd", "csrc", "lw_mfma.hip")).read()
    for workload, prof in b.TRAFFIC_PROFILES.items():
        n = b.PROFILED_PARTICLES[workload]
        if not os.path.exists(prof):
            assert b.profiled_traffic("mfma_f16x3", 0, n, workload, 2) is None
            continue
        text = open(prof).read()
        fields = dict(line.split(":", 1) for line in text.splitlines() if ":" in line and not line.startswith(" "))
        profiled_bands = int(fields["bands"])
        if fields["kernel_code_sha256"].strip() != b.kernel_code_digest(src):
            # the kernel changed after the counters were taken: nothing may be reported
            assert b.profiled_traffic("mfma_f16x3", 0, n, workload, profiled_bands) is None
            continue
        got = b.profiled_traffic("mfma_f16x3", 0, n, workload, profiled_bands)
        assert got == float(fields["traffic_bytes_per_launch"])
        got = b.profiled_traffic("mfma_f16x3", 0, n, workload, profiled_bands, "spread")
        assert got == float(fields["spread_traffic_bytes_per_launch"])
        # any other launch gets none
        assert b.profiled_traffic("mfma_f16x3", 0, n, workload, profiled_bands + 1) is None
        assert b.profiled_traffic("mfma_bf16x3", 0, n, workload, profiled_bands) is None
        assert b.profiled_traffic("mfma_f16x3", 1, n, workload, profiled_bands) is None
        assert b.profiled_traffic("mfma_f16x3", 0, n // 2, workload, profiled_bands) is None
    assert b.profiled_traffic("mfma_f16x3", 0, 100_000, "other", 2) is None


def test_roofline_carries_the_dominant_kernels_traffic():
    """Both legs' `roofline` is re-copied from the dominant kernel after the traffic is
    attached, so it carries the same bytes as that kernel's own roofline."""
    b = _bench()
    for workload, bound, dominant in (("c2", "alu", "spread"), ("c3", "mfma", "contraction")):
        r = {"roofline_contraction": {"bound": "mfma", "traffic": None},
             "roofline_spread": {"bound": "alu", "traffic": None}}
        r["roofline"] = dict(r["roofline_" + dominant])
        b.attach_traffic(r, "mfma_f16x3", 0, b.PROFILED_PARTICLES[workload], workload, 2)
        assert r["roofline"]["bound"] == bound
        assert r["roofline"]["traffic"] == r["roofline_" + dominant]["traffic"]
        assert r["roofline"]["traffic"] == b.profiled_traffic("mfma_f16x3", 0, b.PROFILED_PARTICLES[workload],
                                                              workload, 2, dominant)


def test_spread_flop_model():
    b = _bench()
    # per band: 8W accumulation + 9W tap polynomials + 3 (z, z^2) + 4 demodulation + 6 FP64
    # (turn fraction, grid coordinate); per sample and direction, shared by a work-group's
    # bands: 35 integrand + 15 FP64 (kappa, retarded time)
    for w in (8, 10):
        per_band = 8 * w + 9 * w + 3 + 4 + 6
        assert b.spread_flops_per_unit(w) == per_band + 50  # one band: nothing shared
        assert b.spread_flops_per_unit(w, 2) == per_band + 25  # one work-group, two bands
        assert b.spread_flops_per_unit(w, 3) == per_band + 50 * 2 / 3  # groups of 2 and 1
        assert b.spread_flops_per_unit(w, 16) == per_band + 25
    assert b.spread_flops_per_unit(10, 2) == 208
    assert b.spread_width(3) == 10 and b.spread_width(1) == 8


def test_algorithmic_work_of_the_roofline():
    """frac uses the algorithmic work: 32 FLOP per (sample, direction, band) for the spread and
    one product's multiply-adds for the contraction, whatever the number of hi/lo products."""
    b = _bench()
    assert b.SPREAD_ALGO_FLOPS == 32
    assert b.C3_TERMS == 1e6 * 2048 * 16 * 2048 and abs(b.C3_TERMS / 6.7e13 - 1) < 0.01
