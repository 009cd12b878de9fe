"""Host-side checks of the rocprofv3 summariser (no GPU): interval union of
the busy fraction, the calibration of the traffic counters, and the per-kernel
averages of the matrix-core counters, on small hand-made CSV files."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2404_17133_amd"))

import profsum  # noqa: E402


def _write(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for r in rows:
            f.write(",".join('"%s"' % x if isinstance(x, str) else str(x) for x in r) + "\n")


def test_busy_union_and_tail(tmp_path):
    tr = tmp_path / "trace.csv"
    # [100, 300] (two overlapping kernels) + [400, 500]: 300 of a 400 ns span
    _write(tr, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [("a", 100, 200), ("b", 150, 300), ("c", 400, 500)])
    out = tmp_path / "b.md"
    profsum.busy(str(tr), str(out), "cmd")
    assert "= 75.0% of the span" in out.read_text()
    # only the last 150 ns: kernel c alone, fully busy
    profsum.busy(str(tr), str(out), "cmd", tail_s=150e-9)
    assert "1 kernels" in out.read_text() and "= 100.0% of the span" in out.read_text()


def test_pmc_calibration_and_rates(tmp_path):
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float>>"
    gemm = "void rid::(anonymous namespace)::gemm_nt_kernel<float, 64, 64, 32, 32, true, 3>(rid::GemmParams, int, long)"
    gram = "void rid::(anonymous namespace)::gram_part_kernel(double const*)"
    grid = 1024 * (1 << 20) // 16
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"]
    # the copy reads 1 GiB but the counter shows half: fetch factor 2
    _write(tmp_path / "f.csv", hdr, [(copy, "FETCH_SIZE", 524288, grid), (gemm, "FETCH_SIZE", 1000, 256),
                                     (gemm, "FETCH_SIZE", 3000, 256), (gram, "FETCH_SIZE", 500, 64)])
    _write(tmp_path / "w.csv", hdr, [(copy, "WRITE_SIZE", 1048576, grid), (gemm, "WRITE_SIZE", 100, 256),
                                     (gemm, "WRITE_SIZE", 100, 256), (gram, "WRITE_SIZE", 0, 64)])
    _write(tmp_path / "s.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [(gemm, 2, 2000000, 1000000), (gram, 1, 1000, 1000)])
    out = tmp_path / "t.md"
    profsum.pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "cmd", 1024, str(tmp_path / "s.csv"))
    text = out.read_text()
    assert "scale factors 2.0000 (fetch) and 1.0000 (write)" in text
    # gemm: (2000 KiB * 2 + 100 KiB) per dispatch = 4100 KiB = 0.0042 GB, over 1 ms
    assert "| gemm_nt<float,64x64,vec> [exch_w] | 2 | 2000 | 100 | 0.004 |" in text
    assert "| gemm_nt<float,64x64,vec> [exch_w] | 2 | 0.0042 | 1.0000 | 4 | 0.1% |" in text
    # gram: 1000 KiB over 1 us = 1024 GB/s
    assert "| gram_part_kernel | 1 | 0.0010 | 0.0010 | 1024 | 12.8% |" in text


def test_mfma_averages(tmp_path):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"]
    _write(tmp_path / "c.csv", hdr, [("k1", "MfmaUtil", 80.0, 1), ("k1", "SQ_INSTS_VALU_MFMA_MOPS_F32", 1e6, 1),
                                     ("k1", "MfmaUtil", 70.0, 1), ("k1", "SQ_INSTS_VALU_MFMA_MOPS_F32", 3e6, 1),
                                     ("k2", "MfmaUtil", 0.0, 1)])
    out = tmp_path / "m.md"
    profsum.mfma(str(tmp_path / "c.csv"), str(out), "cmd")
    text = out.read_text()
    assert "| k1 | 2 | 75.0 | 1.02, 0.00, 0.00 |" in text
    assert "| k2 |" not in text  # no matrix-core work


def test_short_names_of_gemm_kernels():
    from paper_2404_17133_amd.profsum import short_name

    base = "void rid::(anonymous namespace)::gemm_nt_kernel<float, 64, 64, 32, 32, %s>(rid::GemmParams, int, long)"
    assert short_name(base % "true, 3") == "gemm_nt<float,64x64,vec> [exch_w]"
    assert short_name(base % "true, false, 3") == "gemm_nt<float,64x64,vec> [exch_w]"
    assert short_name(base % "true, true, 5") == "gemm_nt<float,64x64,vec,il> [exch_wp]"
    assert short_name(base % "false, false, 2") == "gemm_nt<float,64x64,scalar> [exch_s]"
