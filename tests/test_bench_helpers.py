"""Host-side helpers of bench.py that turn kernel times into roofline figures:
the minimal HBM bytes of each flush variant and the recorded counter traffic."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import bench  # noqa: E402


def test_flush_minimal_bytes_per_variant():
    N, ld, n_mon = 16384, 16384, 64
    # whole block read and written once (the monitor rows by a kernel of their own);
    # upper triangle alone: half read, half written; complex128: 16-byte entries
    assert bench.flush_alg_bytes("w32_3m", "c64", N, ld, n_mon) == 16 * N * ld
    # complex128: the FP64 flush of the upper triangle and the monitor rows
    assert bench.flush_alg_bytes(None, "c128", N, ld, n_mon) == 16 * N * ld + 32 * n_mon * ld
    # the pair and band flushes also update the monitor rows (read and written once)
    for v in ("up_pair4_3m_nt", "up_pair4_3m_nt_x8", "up_band4_3m_nt", "up_bandseg4_3m_nt", "up_bandseg_s3"):
        assert bench.flush_covers_monitors(v)
        assert bench.flush_alg_bytes(v, "c64", N, ld, n_mon) == 8 * N * ld + 16 * n_mon * ld
    assert not bench.flush_covers_monitors("w32_3m")


def test_counter_traffic_lookup():
    # unrecorded kernels, workloads, variants or buckets give no traffic figure
    assert bench.pmc_traffic("k_flush_c64", "square128_c64", "w32") is None
    assert bench.pmc_traffic("k_rank1", "strip48x2048_c64", "2x1x1_nt") is None
    assert bench.flush_traffic("square128_c64", "up_bandseg_s3", []) is None
    assert bench.flush_traffic("square128_c64", "w32_3m", [64]) is None
    # a window's figure is the mean of its flushes' bucket records
    per = {b: bench.pmc_traffic("k_flush_c64", "square128_c64", "up_bandseg_s3", b) for b in (16, 32, 64, 128)}
    if all(v is not None for v in per.values()):
        got = bench.flush_traffic("square128_c64", "up_bandseg_s3", [128, 62, 3])
        assert abs(got - (per[128] + per[64] + per[16]) / 3) < 1.0
        # at least the tiles read and written once (the minimal 2.164 GB): within
        # 1.15x up to 64 terms; the 128-term form (one workgroup per compute unit,
        # twice the operand parts per tile) re-reads its operands, within 1.6x
        assert all(2.16e9 < per[b] < 1.15 * 2.165e9 for b in (16, 32, 64))
        assert 2.16e9 < per[128] < 1.6 * 2.165e9
    # the launcher's term buckets
    assert [bench.flush_bucket(t) for t in (1, 16, 17, 32, 33, 64, 65, 128)] == [16, 16, 32, 32, 64, 64, 128, 128]
    for rec in bench.PMC_TRAFFIC:
        assert rec["fetch_kib"] > 0 and rec["write_kib"] > 0
        assert os.path.exists(os.path.join(bench.ROOT, rec["source"]))


def test_flush_flops_count_the_folded_terms_only():
    N, ld, n_mon = 16384, 16384, 64
    nb = N // 64
    tiles = nb * (nb + 1) // 2 + ld // 64          # the triangle, then one band of monitor tiles
    f64 = bench.flush_mfma_flops("up_pair4_3m_nt", "c64", N, ld, n_mon, 64)
    assert f64 == 6.0 * 4096 * tiles * 64            # three real products of 2 flops each
    assert bench.flush_mfma_flops("up_pair4_3m_nt", "c64", N, ld, n_mon, 20) == f64 * 20 / 64
    # the non-symmetric form computes every tile of the block
    assert bench.flush_mfma_flops("w32_3m", "c64", N, ld, n_mon, 1) == 6.0 * 4096 * nb * (ld // 64)


def test_flush_roofline_bound_follows_the_terms():
    N, ld, n_mon = 16384, 16384, 64
    v = "up_pair4_3m_nt"
    # 64 terms per flush at 0.575 ms: matrix-core bound, below the FP32 peak
    r = bench.flush_roofline(v, "c64", N, ld, n_mon, [64, 64], [0.575, 0.575])
    assert r["bound"] == "mfma" and 0.5 < r["frac"] < 0.6 and r["launches"] == 2
    # a lone 20-term flush moves the same bytes for a third of the products: HBM bound
    r = bench.flush_roofline(v, "c64", N, ld, n_mon, [20], [0.40])
    assert r["bound"] == "hbm" and r["achieved"] == r["algorithmic_bytes_per_launch"] / 0.40e-3 / 1e9
    assert bench.flush_roofline(v, "c64", N, ld, n_mon, [], []) is None


def test_split_flush_counts_bf16_part_products():
    N, ld, n_mon = 16384, 16384, 64
    v = "up_bandseg_s3"
    # 17 to 128 terms: four real products per complex one, six BF16 part products each
    f = bench.flush_mfma_flops(v, "c64", N, ld, n_mon, 64)
    assert f == 8 * bench.flush_mfma_flops("up_pair4_3m_nt", "c64", N, ld, n_mon, 64)
    assert bench.flush_mfma_peak(v, "c64", 64) == bench.BF16_PEAK_TFLOPS
    # up to 16 terms the launcher runs the FP32 pair flush
    for t in (1, 16):
        assert bench.flush_mfma_flops(v, "c64", N, ld, n_mon, t) == bench.flush_mfma_flops(
            "up_pair4_3m_nt", "c64", N, ld, n_mon, t)
        assert bench.flush_mfma_peak(v, "c64", t) == bench.MFMA_PEAK_TFLOPS["c64"]
    # at 64 terms in 0.46 ms the bytes bind (0.17 ms of BF16 matrix work at peak)
    r = bench.flush_roofline(v, "c64", N, ld, n_mon, [64], [0.46])
    assert r["bound"] == "hbm" and 0.55 < r["frac"] < 0.65
    assert bench.flush_mfma_peak(v, "c64", 128) == bench.BF16_PEAK_TFLOPS
    # a window that mixes the two kernels: each flush's matrix work at its own
    # instructions' peak (both far below the bytes' time here)
    r = bench.flush_roofline(v, "c64", N, ld, n_mon, [16, 128], [0.4, 0.6])
    f16 = bench.flush_mfma_flops(v, "c64", N, ld, n_mon, 16)
    f128 = bench.flush_mfma_flops(v, "c64", N, ld, n_mon, 128)
    assert r["bound"] == "hbm" and r["mfma_flops_per_launch"] == (f16 + f128) / 2
    t_mfma = f16 / (bench.MFMA_PEAK_TFLOPS["c64"] * 1e12) + f128 / (bench.BF16_PEAK_TFLOPS * 1e12)
    assert t_mfma < 2 * r["algorithmic_bytes_per_launch"] / (bench.HBM_PEAK_GBS * 1e9)


def test_host_info_fields():
    h = bench.host_info()
    assert set(h) == {"cpu_model", "logical_cpus", "ram_gb", "blas", "blas_threads"}
    assert h["logical_cpus"] >= 1


def test_code_hash_ignores_comments_only(tmp_path):
    """A counter record stays valid across comment and whitespace edits of its
    source, and not across a code change."""
    a = tmp_path / "a.hip"
    a.write_text("// note\nint f(int x) {  /* twice */ return 2 * x; }\n")
    h = bench.code_hash(str(a))
    a.write_text("int f(int x) {\n  return 2 * x;  // doubled\n}\n")
    assert bench.code_hash(str(a)) == h
    a.write_text("int f(int x) { return 3 * x; }\n")
    assert bench.code_hash(str(a)) != h
