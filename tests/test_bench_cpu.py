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


def test_counter_traffic_is_keyed_by_kernel_code():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2512_23116_amd.rocprof_summary import kernel_code_sha
    path = os.path.join(ROOT, "profiles", "hbm_traffic_step_kernels_forced_hit_100_800.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows, "no counter rows"
    for key, sha, fetch, write, fam, *_ in rows:
        got = bench.counter_traffic(key, fam)
        if sha == kernel_code_sha(fam):
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


def test_kernel_code_sha_follows_the_kernel_machine_code(tmp_path, monkeypatch):
    """The profile-table key hashes each step-kernel family's gfx950 code and
    descriptors: it sees every instantiation, changes when one byte of that code
    changes, and stays put when only another kernel's code changes."""
    import shutil
    from paper_2512_23116_amd import lbm
    from paper_2512_23116_amd import rocprof_summary as R
    if not os.path.exists(lbm.LIB_PATH):
        raise AssertionError("liblbm.so is not built (run __graft_entry__.build())")
    syms = R.kernel_symbols("k_step")
    names = [nm.decode() for nm, _, _ in syms]
    for codec in ("CdF64", "CdF32", "CdF16", "CdBF16"):
        for pat in (0, 1, 2):
            mangled = f"_ZN3lbm6k_stepINS_{len(codec)}{codec}ELi{pat}ELi0EEEvNS_11LatticeArgsE"
            assert mangled in names and mangled + ".kd" in names
    assert len(R.kernel_symbols("k_step_tb2")) >= 4
    base = {f: R.kernel_code_sha(f) for f in R.KERNEL_FAMILIES}
    assert base == {f: R.kernel_code_sha(f) for f in R.KERNEL_FAMILIES}

    def flipped(off):
        p = tmp_path / f"lib_{off}.so"
        shutil.copy(lbm.LIB_PATH, p)
        with open(p, "r+b") as fh:
            fh.seek(off)
            b = fh.read(1)
            fh.seek(off)
            fh.write(bytes([b[0] ^ 0x01]))
        return str(p)

    _, off, size = next(s for s in syms if not s[0].endswith(b".kd"))
    lib1 = flipped(off + size // 2)
    assert R.kernel_code_sha("k_step", lib1) != base["k_step"]
    assert R.kernel_code_sha("k_step_tb2", lib1) == base["k_step_tb2"]
    monkeypatch.setitem(R.KERNEL_FAMILIES, "k_stream", "8k_streamI")
    _, off, size = R.kernel_symbols("k_stream")[0]
    lib2 = flipped(off + size // 2)
    assert {f: R.kernel_code_sha(f, lib2) for f in ("k_step", "k_step_tb2")} == \
        {f: base[f] for f in ("k_step", "k_step_tb2")}


def test_profile_rows_are_keyed_by_lattice_pattern_and_storage():
    """The profile summary names each step launch by its lattice: edge from the
    grid, AA (patterns 0, 1) or A/B (pattern 2), storage from the codec."""
    sys.path.insert(0, ROOT)
    from paper_2512_23116_amd.rocprof_summary import lattice_key
    assert lattice_key("k_step<CdF32, 2, 0>(LatticeArgs)", 1000192, "fp32", 800) == \
        ("k_step", "100_fp32_ab")
    assert lattice_key("k_step<CdF32, 1, 0>(LatticeArgs)", 1000192, "fp32", 800) == \
        ("k_step", "100_fp32_aa")
    assert lattice_key("k_step<CdF16, 0, 0>(LatticeArgs)", 512000000, "fp32", 800) == \
        ("k_step", "800_fp16_aa")
    assert lattice_key("k_step_tb2<CdBF16, 16>(TB2Args)", 3178496, "fp32", 800) == \
        ("k_step_tb2", "800_bf16_ab_tb2")
    assert lattice_key("k_moments<CdF32, 0>(LatticeArgs, double*, double*)", 1000192, "fp32",
                       800) is None


def test_the_committed_profiles_cover_the_default_headline():
    """The default headline lattice (100^3 FP32 A/B) has a row in the committed
    trace table and in the counter table; whether it is current is the code
    sha's business (bench.py prints null for a stale row)."""
    for table in ("durations_step_kernels_forced_hit_100_800.txt",
                  "hbm_traffic_step_kernels_forced_hit_100_800.txt"):
        keys = [l.split()[0] for l in open(os.path.join(ROOT, "profiles", table))
                if l.strip() and not l.startswith("#")]
        assert "100_fp32_ab" in keys, table
