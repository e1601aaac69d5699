"""bench.py contract pieces that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_traffic_is_keyed_by_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2512_23116_amd.rocprof_summary import kernel_source_sha
    path = os.path.join(ROOT, "profiles", "hbm_traffic_step_kernels_forced_hit_100_800.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows, "no counter rows"
    for key, sha, fetch, write, fam, *_ in rows:
        got = bench.counter_traffic(key, fam)
        if sha == kernel_source_sha(fam):
            assert got == float(fetch) + float(write)
        else:
            assert got is None
    assert bench.counter_traffic("no_such_lattice") is None


def test_precision_errors_compare_common_snapshots_after_the_start():
    sys.path.insert(0, ROOT)
    import bench
    ref = {"kt_series": [dict(step=0, mean=1.0, var=1e-21, flat=3.0),
                         dict(step=500, mean=2.0, var=4.0, flat=3.0),
                         dict(step=1000, mean=2.0, var=4.0, flat=3.0)],
           "spectrum_final": [0.0] + [1.0] * 40}
    run = {"kt_series": [dict(step=0, mean=1.5, var=5e-21, flat=9.0),
                         dict(step=500, mean=2.2, var=4.0, flat=3.0),
                         dict(step=1000, mean=2.02, var=3.6, flat=3.3)],
           "spectrum_final": [0.0] + [1.0] * 8 + [1.5] + [1.0] * 31}
    e = bench.precision_errors(run, ref, 40)
    assert abs(e["kt_rel_err_max"]["mean"] - 0.1) < 1e-12       # step 0 is left out
    assert abs(e["kt_rel_err_last"]["mean"] - 0.01) < 1e-12
    assert abs(e["kt_rel_err_max"]["var"] - 0.1) < 1e-12
    assert abs(e["kt_rel_err_max"]["flat"] - 0.1) < 1e-12
    assert e["spectrum_rel_err_last"]["k<=8"] == 0.0
    assert abs(e["spectrum_rel_err_last"]["k<=32"] - 0.5) < 1e-12
    assert set(e["spectrum_rel_err_last"]) == {"k<=8", "k<=32", "k<=10"}
