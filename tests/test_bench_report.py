"""Host logic of the benchmark report: the per-stage rates and the flop count
they are quoted on (no GPU)."""
import math

import bench


def _stages(ms=100.0):
    return {s: ms for s in ["cholesky", "reduce", "band", "bulge", "tridiag", "occ", "back_q2", "back_q1",
                            "backsub", "density", "refine"]}


def test_matrix_core_stages_sum_to_the_benchmark_flop_count():
    n, k, b = 32768, 8194, 64
    rep = bench.stage_roofline(_stages(), n, k, b)
    mfma = sum(v["flops"] for v in rep.values() if v.get("peak_of") == "fp64_mfma")
    assert math.isclose(mfma, bench.algorithmic_flops(n, k), rel_tol=1e-12)
    assert math.isclose(rep["bulge"]["flops"], 6.0 * b * n * n) and rep["bulge"]["peak_of"] == "fp64_valu"
    # the divide-and-conquer merges, occupations and refinement carry their time only
    for st in ("tridiag", "occ", "refine"):
        assert rep[st] == {"ms": 100.0}


def test_rates_and_peaks_per_precision():
    n, k, b = 1000, 300, 64
    st = _stages(ms=2.0)
    plain = bench.stage_roofline(st, n, k, b)
    mixed = bench.stage_roofline(st, n, k, b, mixed=True)
    assert math.isclose(plain["reduce"]["tflops"], n ** 3 / 2e-3 / 1e12)
    assert math.isclose(plain["reduce"]["frac"], plain["reduce"]["tflops"] / 78.6)
    # in the mixed mode full -> band and Q1 run on the FP32 matrix cores
    assert mixed["band"]["peak"] == 157.3 and mixed["back_q1"]["peak"] == 157.3
    assert mixed["band"]["peak_of"] == "fp32_mfma" and mixed["reduce"]["peak_of"] == "fp64_mfma"
    assert mixed["back_q2"]["peak"] == 78.6 and plain["band"]["peak"] == 78.6
    # a stage that did not run is reported by its time alone
    st["refine"] = 0.0
    assert bench.stage_roofline(st, n, k, b)["refine"] == {"ms": 0.0}


def test_tuner_buckets_and_samples():
    from paper_1705_11191_amd import tune

    # power-of-two upper bounds from 512 up to the first that covers the largest size
    assert tune.default_buckets([255, 300]) == [512]
    assert tune.default_buckets([256, 4095]) == [512, 1024, 2048, 4096]
    assert tune.default_buckets([4097]) == [512, 1024, 2048, 4096, 8192]
    # a bucket's sample spreads evenly over its members and never repeats one
    members = list(range(100, 140))
    s = tune._sample(members, 8)
    assert len(s) == 8 and len(set(s)) == 8 and all(x in members for x in s)
    assert s == sorted(s) and s[0] < 105 and s[-1] > 134
    assert tune._sample([3, 4], 8) == [3, 4]
    assert tune._sample([], 8) == []


def test_traffic_summary_round_trip_and_staleness(tmp_path, monkeypatch):
    """The HBM traffic figure is read back from the counter summary only while
    the GEMM source and the kernel's launch count per solve are those it was
    taken with; each counter is scaled by the calibration copy's reading."""
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    src = tmp_path / "gemm.hip"
    src.write_text("kernel source A")
    monkeypatch.setattr(bench, "GEMM_SRC", str(src))
    kern = "dgemm_kernel<128,128,0,true,false,false>"
    full = "void eg::(anonymous namespace)::dgemm_kernel<128, 128, 0, true, false, false>(int, int)"
    known_kib = bench.COPY_ELEMS * 8 / 1024

    def csv_file(name, counter, copy_kib, vals):
        rows = ["Counter_Name,Kernel_Name,Counter_Value", f'{counter},"void eg::neg_kernel(double*)",{copy_kib}']
        rows += [f'{counter},"{full}",{v}' for v in vals]
        path = tmp_path / name
        path.write_text("\n".join(rows) + "\n")
        return str(path)

    fetch = csv_file("f.csv", "FETCH_SIZE", known_kib / 2, [100.0, 300.0])   # reads back half: factor 2
    write = csv_file("w.csv", "WRITE_SIZE", known_kib, [40.0, 60.0])         # factor 1
    bench.summarize_pmc(fetch, write, kern, "wl", ["the two counter passes"])
    want = 200.0 * 1024 * 2 + 50.0 * 1024
    assert math.isclose(bench.load_traffic(kern, "wl", 2), want)
    assert bench.load_traffic(kern, "wl", 3) is None   # another mix of products
    assert bench.load_traffic(kern, "other", 2) is None
    src.write_text("kernel source B")
    assert bench.load_traffic(kern, "wl", 2) is None   # the GEMM changed since
