"""Host logic of bench.py, on the CPU.

Three parts are checked: the refusal of more than one GPU, the gate that takes
HBM traffic from a counter summary only when that summary was taken on the
current kernel source, and the two error measures of the parity fields.  The
first is the maximum relative error against the oracle.  The second is Eq. (1)
against a tight-tolerance run, with the weights atol + rtol |y| of Sec. 2.1.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       timeout=300, env={**os.environ, **env})
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _fake_tree(tmp_path, kernel):
    csrc = tmp_path / "paper_1607_03884_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES[kernel]:
        (csrc / f).write_text(f"// {f}\n")
    (tmp_path / "profiles").mkdir()
    return tmp_path


def test_traffic_only_from_a_summary_of_the_current_source(tmp_path, monkeypatch):
    kernel = "radau_group_kernel64"
    root = _fake_tree(tmp_path, kernel)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic(kernel, "cfg3") is None          # no summary yet
    h = bench.source_hash(kernel)
    prof = root / "profiles" / f"{kernel}_cfg3.md"
    prof.write_text(f"# summary\n\ntraffic_bytes_per_dispatch: 946234061\nsource_sha256_16: {h}\n")
    assert bench.measured_traffic(kernel, "cfg3") == 946234061.0
    assert bench.measured_traffic(kernel, "cfg2") is None          # another workload
    assert bench.measured_traffic("no_such_kernel", "cfg3") is None
    # any of the kernel's sources changing voids the summary
    for f in bench.KERNEL_SOURCES[kernel]:
        p = root / "paper_1607_03884_amd" / "csrc" / f
        old = p.read_text()
        p.write_text(old + "// edited\n")
        assert bench.source_hash(kernel) != h
        assert bench.measured_traffic(kernel, "cfg3") is None
        p.write_text(old)
    assert bench.measured_traffic(kernel, "cfg3") == 946234061.0
    # a summary without the traffic line gives nothing
    prof.write_text(f"source_sha256_16: {h}\n")
    assert bench.measured_traffic(kernel, "cfg3") is None


def test_max_rel_err_on_T_and_resolved_mass_fractions():
    K = 3
    # rows: T, Y_1..Y_K, P
    ref = np.array([[1500.0, 0.6, 0.4, 5e-9, 101325.0],
                    [900.0, 0.2, 0.8, 0.0, 101325.0]])
    got = ref.copy()
    assert bench.max_rel_err(got, ref, K) == 0.0
    got[0, 0] = 1500.0 * (1 + 2e-7)
    assert bench.max_rel_err(got, ref, K) == pytest.approx(2e-7, rel=1e-6)
    got[1, 2] = 0.8 * (1 - 3e-6)
    assert bench.max_rel_err(got, ref, K) == pytest.approx(3e-6, rel=1e-6)
    # mass fractions at or below 1e-8 in the reference are not relative-error terms
    got[0, 3] = 5e-8
    got[1, 3] = 1e-9
    assert bench.max_rel_err(got, ref, K) == pytest.approx(3e-6, rel=1e-6)
    # pressure (the last column) is not compared
    got[:, K + 1] *= 2.0
    assert bench.max_rel_err(got, ref, K) == pytest.approx(3e-6, rel=1e-6)


def test_eq1_error_weights_and_norms():
    K = 3
    N = K + 1
    atol, rtol = 1e-10, 1e-6
    truth = np.array([[1000.0, 0.5, 0.25, 0.25, 101325.0],
                      [2000.0, 0.1, 0.0, 0.9, 101325.0]])
    got = truth.copy()
    # state 0: T off by one weight (atol + rtol * 1000)
    got[0, 0] += atol + rtol * 1000.0
    # state 1: a zero mass fraction off by 3 atol (its weight is atol alone),
    # and Y_3 off by 4 of its weights
    got[1, 2] += 3 * atol
    got[1, 3] += 4 * (atol + rtol * 0.9)
    r = bench.eq1_error(got, truth, K, atol, rtol)
    assert r["two_norm_max"] == pytest.approx(5.0, rel=1e-9)            # sqrt(3^2 + 4^2)
    assert r["rms_max"] == pytest.approx(5.0 / np.sqrt(N), rel=1e-9)
    # the pressure column does not enter
    got[:, N] += 1.0
    assert bench.eq1_error(got, truth, K, atol, rtol)["two_norm_max"] == pytest.approx(5.0, rel=1e-9)
