"""Summarise rocprofv3 output for the step kernels.

    python -m paper_2512_23116_amd.rocprof_summary --trace DIR [--fetch DIR --write DIR]
        [--cmd "the profiled command"] [--traffic-out profiles/hbm_traffic_step_kernels_forced_hit_100_800.txt]

``--trace`` is a ``rocprofv3 --kernel-trace --stats --output-format csv`` output
directory: per-kernel launch counts and durations are listed per grid size
(lattice), so even and odd AA steps and the 100^3 / 800^3 lattices are apart.

``--fetch`` / ``--write`` are ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc
WRITE_SIZE`` runs of ``bench.py --profile``.  That command first copies 1 GiB
with a known-size copy kernel; the counters' reading for it calibrates the
counters to bytes (FETCH_SIZE reads half of the true bytes on MI355X), and the
calibrated bytes per step launch are compared with the algorithmic 2*19*b*N^3.
With ``--traffic-out`` one line per lattice is appended for bench.py:
``<N>_<precision>_<streaming>[_tb2] <kernel code sha> <fetch bytes> <write bytes>``,
the sha taken over that kernel family's gfx950 machine code in the built library
(kernel_code_sha).
With ``--durations-out`` the trace's mean duration per step launch is written
the same way (``<key> <sha> <mean us> <launches> <family>``), so that bench.py can
print the profile's figure beside its own live HIP-event mean.
"""
import argparse
import collections
import csv
import glob
import hashlib
import os
import statistics
import struct

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


# Mangled-name marker of each step-kernel family in the gfx950 code objects.
KERNEL_FAMILIES = {"k_step": "6k_stepI", "k_step_tb2": "10k_step_tb2I"}
LIB_PATH = os.path.join(HERE, "liblbm.so")
_BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
_GFX950 = b"hipv4-amdgcn-amd-amdhsa--gfx950"


def _elf_sections(d):
    """{name: (file offset, size, address)} of an ELF64 little-endian image."""
    shoff, = struct.unpack_from("<Q", d, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", d, 0x3A)
    hdrs = []
    for i in range(shnum):
        name, _, _, addr, off, size = struct.unpack_from("<IIQQQQ", d, shoff + i * shentsize)
        hdrs.append((name, off, size, addr))
    stroff = hdrs[shstrndx][1]
    out = {}
    for i, (name, off, size, addr) in enumerate(hdrs):
        end = d.index(b"\0", stroff + name)
        out[d[stroff + name:end].decode()] = (off, size, addr, i)
    return out


def gfx950_code_objects(lib_path=LIB_PATH):
    """(file offset, bytes) of the gfx950 code objects inside a HIP shared
    library: its .hip_fatbin section holds one clang offload bundle per
    translation unit (magic string, entry count, then offset / size / target
    triple of each entry)."""
    d = open(lib_path, "rb").read()
    base, size, _, _ = _elf_sections(d)[".hip_fatbin"]
    fat = d[base:base + size]
    objs, pos = [], fat.find(_BUNDLE_MAGIC)
    while pos >= 0:
        n, = struct.unpack_from("<Q", fat, pos + len(_BUNDLE_MAGIC))
        q, end = pos + len(_BUNDLE_MAGIC) + 8, pos
        for _ in range(n):
            eoff, esize, tlen = struct.unpack_from("<QQQ", fat, q)
            triple = fat[q + 24:q + 24 + tlen]
            q += 24 + tlen
            end = max(end, pos + eoff + esize)
            if triple == _GFX950 and esize:
                obj = fat[pos + eoff:pos + eoff + esize]
                if obj[:4] != b"\x7fELF":
                    raise ValueError("compressed or unknown code object in the offload bundle")
                objs.append((base + pos + eoff, obj))
        pos = fat.find(_BUNDLE_MAGIC, end)
    return objs


def kernel_symbols(family="k_step", lib_path=LIB_PATH):
    """(mangled name, file offset in the library, size) of the machine code and
    kernel descriptor of every instantiation of a step-kernel family."""
    marker = KERNEL_FAMILIES[family].encode()
    found = []
    for obj_off, obj in gfx950_code_objects(lib_path):
        sec = _elf_sections(obj)
        by_index = {v[3]: v for v in sec.values()}
        symoff, symsize, _, _ = sec[".symtab"]
        stroff = sec[".strtab"][0]
        for q in range(symoff, symoff + symsize, 24):
            name, _, _, shndx, value, size = struct.unpack_from("<IBBHQQ", obj, q)
            nm = obj[stroff + name:obj.index(b"\0", stroff + name)]
            if marker not in nm or not size or shndx not in by_index:
                continue
            s_off, _, s_addr, _ = by_index[shndx]
            found.append((nm, obj_off + s_off + value - s_addr, size))
    return sorted(found)


def kernel_code_sha(family="k_step", lib_path=LIB_PATH):
    """sha256[:16] over the gfx950 machine code and kernel descriptors of every
    instantiation of a step-kernel family in the built library (symbol names and
    bytes, in name order): a profile taken on this library stays valid while
    this value is unchanged, whatever else in the library or its headers changes."""
    syms = kernel_symbols(family, lib_path)
    if not syms:
        raise ValueError(f"no {family} kernels in {lib_path}")
    d = open(lib_path, "rb").read()
    h = hashlib.sha256()
    for nm, off, size in syms:
        h.update(nm + b"\0" + d[off:off + size])
    return h.hexdigest()[:16]


CODEC_PRECISION = {"CdF64": "fp64", "CdF32": "fp32", "CdF16": "fp16", "CdBF16": "bf16"}
PRECISION_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def kernel_precision(kernel, default):
    """Storage precision named by a step kernel's codec template argument."""
    for codec, p in CODEC_PRECISION.items():
        if f"<{codec}," in short(kernel) or f"<{codec}>" in short(kernel):
            return p
    return default


def lattice_key(kernel, grid, precision, tb2_n):
    """(family, traffic key) of a step-kernel launch, or None for other kernels.

    k_step launches one thread per cell (grid = N^3 rounded up to 256); the
    pattern template argument tells AA (0, 1) from A/B (2), the codec argument
    the storage precision (`precision` when it names none).  The two-step
    kernel's grid counts tiles, so its lattice edge is given (tb2_n)."""
    k = short(kernel)
    precision = kernel_precision(kernel, precision)
    if k.startswith("k_step_tb2"):
        return "k_step_tb2", f"{tb2_n}_{precision}_ab_tb2"
    if not k.startswith("k_step<"):
        return None
    pattern = k.split(",")[1].strip()
    N = round(grid ** (1 / 3))
    return "k_step", f"{N}_{precision}_{'ab' if pattern == '2' else 'aa'}"


def _csv(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(files[0])))


def short(name):
    return name.replace("(lbm::LatticeArgs)", "").replace("void ", "").replace("lbm::", "")


def trace_table(d):
    rows = _csv(d, "_kernel_trace.csv")
    by = collections.defaultdict(list)
    for r in rows:
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        by[(short(r["Kernel_Name"]), g)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = []
    for (k, g), v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        out.append((k, g, len(v), statistics.mean(v) / 1e3, statistics.median(v) / 1e3,
                    min(v) / 1e3, max(v) / 1e3))
    return out


def counters(d, name):
    rows = _csv(d, "_counter_collection.csv")
    by = collections.defaultdict(list)
    for r in rows:
        if r["Counter_Name"] != name:
            continue
        by[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return by


def calibration(by):
    """KiB the counter reports for the 1 GiB copy launches (largest copy grid)."""
    copies = [(g, v) for (k, g), v in by.items() if "copyBuffer" in k or "copy" in k.lower()]
    g, v = max(copies, key=lambda gv: gv[0])
    return statistics.mean(v)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--streaming", default="aa")
    ap.add_argument("--sq", help="rocprofv3 --pmc run of SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
                                  "SQ_INSTS_VALU SQ_WAIT_ANY SQ_INSTS_LDS GRBM_GUI_ACTIVE")
    ap.add_argument("--traffic-out")
    ap.add_argument("--durations-out")
    ap.add_argument("--tb2-n", type=int, default=800,
                    help="lattice edge of the two-step kernel launches in the counter runs")
    a = ap.parse_args()
    if a.cmd:
        print(f"command: {a.cmd}")
    for fam in KERNEL_FAMILIES:
        print(f"{fam} gfx950 code sha256[:16]: {kernel_code_sha(fam)}")
    if a.trace:
        print("\nkernel trace (durations in us; grid = threads launched)")
        print(f"{'kernel':58s} {'grid':>11s} {'calls':>6s} {'mean':>10s} {'median':>10s} "
              f"{'min':>10s} {'max':>10s}")
        table = trace_table(a.trace)
        for k, g, n, mean, med, lo, hi in table:
            print(f"{k[:58]:58s} {g:11d} {n:6d} {mean:10.2f} {med:10.2f} {lo:10.2f} {hi:10.2f}")
        per_key = collections.defaultdict(lambda: [0.0, 0, ""])
        for k, g, n, mean, med, lo, hi in table:
            lk = lattice_key(k, g, a.precision, a.tb2_n)
            if lk is None:
                continue
            fam, key = lk
            acc = per_key[key]
            acc[0] += mean * n
            acc[1] += n
            acc[2] = fam
        print("\nmean duration per step launch (all launches of the lattice, even and odd)")
        for key, (tot, n, fam) in sorted(per_key.items()):
            print(f"{key:>16s} {fam:>10s} {n:6d} launches {tot / n:10.2f} us")
        if a.durations_out:
            write_table(a.durations_out, {k: (v[0] / v[1], v[1], v[2]) for k, v in per_key.items()},
                        lambda key, val: f"{key} {kernel_code_sha(val[2])} {val[0]:.3f} "
                                         f"{val[1]} {val[2]}\n", fam_col=4)
    if a.fetch and a.write:
        fb = counters(a.fetch, "FETCH_SIZE")
        wb = counters(a.write, "WRITE_SIZE")
        fcal = COPY_BYTES / 1024 / calibration(fb)
        wcal = COPY_BYTES / 1024 / calibration(wb)
        print(f"\ncounter calibration on a 1 GiB copy: FETCH_SIZE x {fcal:.4f}, "
              f"WRITE_SIZE x {wcal:.4f}")
        print(f"{'kernel':40s} {'lattice':>16s} {'fetch GB':>9s} {'write GB':>9s} "
              f"{'step alg GB':>11s} {'ratio':>6s}")
        per_key = collections.defaultdict(lambda: [0.0, 0.0, 0, ""])
        for (k, g), v in sorted(fb.items()):
            lk = lattice_key(k, g, a.precision, a.tb2_n)
            if lk is None:
                continue
            fam, key = lk
            N = int(key.split("_")[0])
            f = statistics.mean(v) * 1024 * fcal
            w = statistics.mean(wb[(k, g)]) * 1024 * wcal
            kb = PRECISION_BYTES[key.split("_")[1]]
            alg = 2 * 19 * kb * N ** 3     # one read and one write of every population
            print(f"{short(k)[:40]:40s} {key:>16s} {f / 1e9:9.4f} {w / 1e9:9.4f} {alg / 1e9:11.4f} "
                  f"{(f + w) / alg:6.3f}")
            acc = per_key[key]
            acc[0] += f
            acc[1] += w
            acc[2] += 1
            acc[3] = fam
        if a.traffic_out:
            write_traffic(a.traffic_out, per_key)
    if a.sq:
        sq_table(a.sq, a.precision, a.tb2_n)


def sq_table(d, precision, tb2_n, simds=1024, clock_ghz=2.4):
    """Per step kernel and lattice: VALU instructions per cell update, an estimate
    of how busy the SIMDs' VALUs were, the share of wave time spent waiting, and
    the launch duration from the busy cycles.

    VALU per cell update = SQ_INSTS_VALU (wave instructions) x 64 lanes / cell
    updates of the launch (N^3, or 2 N^3 for the two-step kernel).  GRBM_GUI_ACTIVE
    sums the busy cycles of the 8 XCDs, so /8 is one XCD's.  VALU busy (estimate) =
    4 cycles x SQ_INSTS_VALU / (SIMDs x one XCD's busy cycles), a lower bound where
    instructions take more than 4 cycles."""
    rows = _csv(d, "_counter_collection.csv")
    by = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        k = r["Kernel_Name"]
        g = int(r["Grid_Size"])
        by[(k, g)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    print("\nSQ counters (means over the launches of each kernel and lattice)")
    print(f"{'kernel':40s} {'lattice':>16s} {'launches':>8s} {'VALU/update':>11s} "
          f"{'VALU busy':>9s} {'wait/wave':>9s} {'LDS/update':>10s} {'us':>9s}")
    for (k, g), c in sorted(by.items()):
        lk = lattice_key(k, g, precision, tb2_n)
        if lk is None and not short(k).startswith("k_stream<"):
            continue
        if lk is None:
            N = round(g ** (1 / 3))
            key, updates = f"{N}_stream", N ** 3
        else:
            fam, key = lk
            N = int(key.split("_")[0])
            updates = N ** 3 * (2 if fam == "k_step_tb2" else 1)
        need = ("SQ_INSTS_VALU", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "GRBM_GUI_ACTIVE")
        if not all(n in c for n in need):
            continue
        valu = statistics.mean(c["SQ_INSTS_VALU"])
        gui = statistics.mean(c["GRBM_GUI_ACTIVE"]) / 8
        wait = statistics.mean(c["SQ_WAIT_ANY"]) / statistics.mean(c["SQ_WAVE_CYCLES"])
        lds = statistics.mean(c["SQ_INSTS_LDS"]) * 64 / updates if "SQ_INSTS_LDS" in c else float("nan")
        print(f"{short(k)[:40]:40s} {key:>16s} {len(c['SQ_INSTS_VALU']):8d} "
              f"{valu * 64 / updates:11.1f} {4 * valu / (simds * gui):9.2f} {wait:9.2f} "
              f"{lds:10.1f} {gui / (clock_ghz * 1e3):9.1f}")


def write_table(path, per_key, fmt, fam_col):
    """Rewrite a per-lattice table: its comment lines, the earlier entries that
    were taken on the current machine code of their kernel and not measured again
    now, then the new entries.  Entries of older code are dropped."""
    current = {fam: kernel_code_sha(fam) for fam in KERNEL_FAMILIES}
    head, keep = [], []
    if os.path.exists(path):
        for ln in open(path):
            if ln.startswith("#"):
                head.append(ln)
                continue
            parts = ln.split()
            if len(parts) > fam_col and parts[0] not in per_key \
                    and current.get(parts[fam_col]) == parts[1]:
                keep.append(ln)
    with open(path, "w") as fh:
        fh.writelines(head + keep)
        for key, val in sorted(per_key.items()):
            fh.write(fmt(key, val))


def write_traffic(path, per_key):
    write_table(path, per_key,
                lambda key, v: f"{key} {kernel_code_sha(v[3])} {v[0] / v[2]:.6e} "
                               f"{v[1] / v[2]:.6e} {v[3]} mean over {v[2]} kernels\n", fam_col=4)


if __name__ == "__main__":
    main()
