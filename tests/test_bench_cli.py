"""Host-only checks of the benchmark's command line (no GPU is touched)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_is_keyed_to_the_sources():
    sys.path.insert(0, ROOT)
    import bench
    # records exist for the BF16 Gram of the chain FFNN (the 128x128 two-per-CU
    # kernel) and of the FFNN 100-400-400 (the wide-tile kernel); each is
    # reported only while the kernel, planner and tuning sources it was taken
    # with are unchanged, and then it is at least the launch's algorithmic
    # bytes (0.945 GB and 7.65 GB)
    t = bench.measured_traffic("k_gram_duo", "1")
    assert t is None or t > 0.945e9
    t = bench.measured_traffic("k_gram_wide", "2b")
    assert t is None or t > 7.65e9
    assert bench.measured_traffic("k_gram_wide", "1") is None
    assert bench.measured_traffic("k_gram_wide", "3") is None


def test_exact_heisenberg_energy_is_the_oracle_lanczos_value():
    """The VMC records report against the exact ground-state energy of the
    16-site ring; it is the oracle's Lanczos value on the zero-magnetisation
    sector (and 4 E0 rounds to the -28.57 of the paper's Sec. 3, Tab. 2)."""
    sys.path.insert(0, ROOT)
    import bench
    from oracle import vmc
    e16 = vmc.ground_state(16)[0]
    assert abs(bench.HEISENBERG_L16_E0 - e16) < 1e-9
    assert round(4 * bench.HEISENBERG_L16_E0, 2) == -28.57
