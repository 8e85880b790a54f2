"""Host-side helpers of bench.py that turn kernel times into roofline figures:
the minimal HBM bytes of each flush variant and the recorded counter traffic."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import bench  # noqa: E402


def test_flush_minimal_bytes_per_variant():
    N, ld, n_mon = 16384, 16384, 64
    # whole block read and written once; symmetric mirrored: half read, all written;
    # upper triangle alone: half read, half written; complex128: 16-byte entries
    assert bench.flush_alg_bytes("w32_pipe8_3m", "c64", N, ld) == 16 * N * ld
    assert bench.flush_alg_bytes("sym_pipe8_3m_nt", "c64", N, ld) == 12 * N * ld
    assert bench.flush_alg_bytes("up_pipe8_3m_nt", "c64", N, ld, n_mon) == 8 * N * ld
    assert bench.flush_alg_bytes(None, "c128", N, ld) == 32 * N * ld
    # the pair flush also updates the monitor rows (read and written once)
    assert bench.flush_covers_monitors("up_pair4_3m_nt")
    assert not bench.flush_covers_monitors("up_pipe8_3m_nt")
    assert bench.flush_alg_bytes("up_pair4_3m_nt", "c64", N, ld, n_mon) == 8 * N * ld + 16 * n_mon * ld


def test_counter_traffic_lookup():
    # unrecorded kernels, workloads or variants give no traffic figure
    assert bench.pmc_traffic("k_flush_c64", "square128_c64", "w32") is None
    assert bench.pmc_traffic("k_rank1", "strip48x2048_c64", "2x1x1_nt") is None
    for rec in bench.PMC_TRAFFIC:
        assert rec["fetch_kib"] > 0 and rec["write_kib"] > 0
        assert os.path.exists(os.path.join(bench.ROOT, rec["source"]))


def test_long_trajectory_workloads_flush_every_128():
    import workloads as W
    assert bench.LONG_TRAJECTORY_DELAY == {"strip48x2048_c64": 128}
    assert "strip48x2048_c64" in W.WORKLOADS
