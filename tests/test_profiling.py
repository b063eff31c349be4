"""Host-side helpers of the measurement code: the per-kernel machine-code
digest read from the built library, and the summary parser the benchmark
uses to decide whether counter figures still describe the loaded kernel."""

import os

import pytest

from paper_2510_02873_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2510_02873_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("library not built")
    return _abi.LIB_PATH


def test_kernel_digest_names_whole_kernels():
    lib = _lib()
    d = profiling.kernel_digest("k_classic_f64", lib)
    assert len(d) == 16 and d == profiling.kernel_digest("k_classic_f64", lib)
    # k_classic_f64 must not match k_classic_f64_1, and the two differ
    assert profiling.kernel_digest("k_classic_f64_1", lib) != d
    # template kernels are found by their name
    assert profiling.kernel_digest("k_batch", lib)
    with pytest.raises(KeyError):
        profiling.kernel_digest("k_no_such_kernel", lib)


def test_committed_headline_summary_parses():
    prof = profiling.read_profile(os.path.join(ROOT, "profiles", "k_classic_f64_256cube_25radii.txt"))
    for key in ("kernel_digest", "traffic_bytes_per_launch", "fp64_flops_per_launch",
                "valu_instructions_per_wave_of_64_evals"):
        assert key in prof
    assert 1e9 < prof["traffic_bytes_per_launch"] < 2e9       # ~72 B per particle at 256^3
    assert 100 < prof["fp64_flops_per_eval"] < 300
    assert prof["fp64_flops_per_launch"] == pytest.approx(prof["fp64_flops_per_launch_from_instruction_counts"],
                                                          rel=1e-6)


def test_read_profile_missing_file_is_empty():
    assert profiling.read_profile(os.path.join(ROOT, "profiles", "no_such_file.txt")) == {}


def test_counter_table_takes_the_median_per_kernel(tmp_path):
    """The counters subcommand reads one --pmc run's CSV and reports, per
    kernel named exactly (k_x does not take k_x_1's rows), the median per
    dispatch and the figure per 64 evaluations."""
    from paper_2510_02873_amd import profiling
    d = tmp_path / "pmc" / "host"
    d.mkdir(parents=True)
    rows = [("pino::k_x(int)", "C_A", v) for v in (10.0, 1000.0, 1000.0)]
    rows += [("pino::k_x_1(int)", "C_A", 5.0), ("pino::k_x(int)", "C_B", 64.0)]
    with open(d / "run_counter_collection.csv", "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for k, c, v in rows:
            f.write(f'"{k}",{c},{v}\n')
    out = tmp_path / "t.txt"
    profiling.counter_table(str(tmp_path / "pmc"), str(out), "cmd", ["k_x"], evals_per_launch=128)
    text = out.read_text()
    line = [ln for ln in text.splitlines() if ln.startswith("k_x |")][0]
    assert "| 3 |" in line and "1.0000e+03" in line and "6.4000e+01" in line
    assert "k_x: C_A 500.00, C_B 32.00" in text
