"""Summaries of rocprofv3 runs of the benchmark (text, for profiles/).

    python -m paper_2510_02873_amd.profiling summarize --kernel k_classic_f64 \
        --trace DIR --fetch DIR --write DIR [--flops DIR --evals-per-launch N] \
        --calib-mib 1024 --out profiles/X.txt --command "..."
    python -m paper_2510_02873_amd.profiling table --trace DIR --out profiles/Y.txt

DIRs are rocprofv3 output directories written with --output-format csv
(kernel trace with --stats; one --pmc FETCH_SIZE run; one --pmc WRITE_SIZE
run; optionally one --pmc run of the FP64 FLOP counters).  HBM bytes per
dispatch are the counters (KiB) scaled by what the same counter reads for
the benchmark's calibration copy of known size.  The summary records a
digest of the kernel's machine code (read from the built library); the
benchmark reports counter-derived figures only while the loaded library's
kernel still has that digest.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import struct

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _elf_sections(blob):
    """{name: (addr, offset, size)} of a little-endian ELF64 image."""
    if blob[:4] != b"\x7fELF" or blob[4] != 2:
        raise ValueError("not an ELF64 image")
    shoff, = struct.unpack_from("<Q", blob, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", blob, 0x3A)
    heads = [struct.unpack_from("<IIQQQQIIQQ", blob, shoff + k * shentsize) for k in range(shnum)]
    names_off = heads[shstrndx][4]

    def name(off):
        end = blob.index(b"\0", names_off + off)
        return blob[names_off + off:end].decode()

    return {name(h[0]): (h[3], h[4], h[5], h[1]) for h in heads}, heads


def _device_code_object(lib_path):
    """The gfx950 code object embedded in a hipcc-built shared library
    (clang offload bundle in the .hip_fatbin section)."""
    blob = open(lib_path, "rb").read()
    secs, _ = _elf_sections(blob)
    _, off, size, _ = secs[".hip_fatbin"]
    fat = blob[off:off + size]
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    if not fat.startswith(magic):
        raise ValueError("unexpected fat binary format")
    n, = struct.unpack_from("<Q", fat, len(magic))
    pos = len(magic) + 8
    for _ in range(n):
        eoff, esize, tlen = struct.unpack_from("<QQQ", fat, pos)
        triple = fat[pos + 24:pos + 24 + tlen].decode()
        pos += 24 + tlen
        if "gfx950" in triple:
            return fat[eoff:eoff + esize]
    raise ValueError("no gfx950 code object in " + lib_path)


def kernel_digest(kernel, lib_path=None):
    """sha256 (16 hex digits) over the machine code and kernel descriptor of
    the kernel named `kernel` (the first template instance for a template;
    the descriptor's code-entry offset, which moves with other kernels, is
    left out)."""
    if lib_path is None:
        lib_path = os.path.join(HERE, "libpino_collapse.so")
    co = _device_code_object(lib_path)
    secs, heads = _elf_sections(co)
    symtab = [h for h in heads if h[1] == 2]  # SHT_SYMTAB
    if not symtab:
        raise ValueError("code object has no symbol table")
    st = symtab[0]
    strtab = heads[st[6]]
    # the name as a whole mangled component (length prefix, then the end of
    # the nested name or a template argument list), so k_x does not match k_x_1;
    # "k_x<true>" / "k_x<false>" name one instance of a bool template
    inst = re.fullmatch(r"(\w+)<(true|false)>", kernel)
    if inst:
        pat = re.compile(r"\d" + re.escape(inst.group(1)) + r"ILb" + ("1" if inst.group(2) == "true" else "0") + "E")
    else:
        pat = re.compile(r"\d" + re.escape(kernel) + r"[EI]")
    found = {}
    for k in range(st[5] // 24):
        st_name, st_info, _, st_shndx, st_value, st_size = struct.unpack_from("<IBBHQQ", co, st[4] + 24 * k)
        end = co.index(b"\0", strtab[4] + st_name)
        nm = co[strtab[4] + st_name:end].decode()
        if pat.search(nm) and st_size and st_shndx < len(heads):
            sec = heads[st_shndx]
            start = sec[4] + (st_value - sec[3])
            found.setdefault(nm, co[start:start + st_size])
    funcs = sorted(n for n in found if not n.endswith(".kd"))
    if not funcs:
        raise KeyError(f"kernel {kernel} not in the library")
    h = hashlib.sha256()
    h.update(funcs[0].encode())
    h.update(found[funcs[0]])
    kd = bytearray(found.get(funcs[0] + ".kd", b""))
    if len(kd) >= 24:
        kd[16:24] = bytes(8)  # kernel_code_entry_byte_offset: depends on where the code was placed
    h.update(bytes(kd))
    return h.hexdigest()[:16]


def _csv(directory, suffix):
    hits = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return list(csv.DictReader(open(hits[0])))


def _named(kernel):
    """Regex for a kernel's demangled name (followed by its argument or
    template list, so k_x does not match k_x_1)."""
    return re.compile(re.escape(kernel) + r"[(<]")


def _counter(rows, counter, kernel):
    pat = _named(kernel)
    return [(float(r["Counter_Value"]), r) for r in rows if r["Counter_Name"] == counter and pat.search(r["Kernel_Name"])]


FLOP_COUNTERS = ("SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP64_TRANS", "SQ_INSTS_VALU_ADD_F64",
                 "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU",
                 "SQ_WAVES")


def _mean_counter(rows, counter, kernel):
    v = [x for x, _ in _counter(rows, counter, kernel)]
    return float(np.mean(v)) if v else None


def summarize(kernel, trace, fetch, write, calib_mib, out, command, flops=None, evals_per_launch=None, extra=None):
    stats = _csv(trace, "kernel_stats.csv")
    ks = [r for r in stats if _named(kernel).search(r["Name"])]
    try:
        digest = kernel_digest(kernel)
    except (KeyError, ValueError):
        digest = "-"  # not in the collapse library (the benchmark's probes)
    lines = [f"# rocprofv3 summary: {kernel}", f"command: {command}", f"kernel_digest: {digest}", ""]
    lines.append("kernel stats (--kernel-trace --stats):")
    for r in ks:
        lines.append(f"  {r['Name']}: calls={r['Calls']} total_ns={r['TotalDurationNs']} "
                     f"average_ns={float(r['AverageNs']):.1f} min_ns={r['MinNs']} max_ns={r['MaxNs']}")
    avg_ns = float(ks[0]["AverageNs"]) if ks else None
    calib_kib = calib_mib * 1024.0
    res = {}
    for label, d, counter in (("fetch", fetch, "FETCH_SIZE"), ("write", write, "WRITE_SIZE")):
        rows = _csv(d, "counter_collection.csv")
        kvals = _counter(rows, counter, kernel)
        # the calibration copy is the largest dispatch of a kernel named *copy*
        # (torch's copy of calib_mib MiB); the benchmark's own copy probe has
        # another size and is not it
        allv = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter
                  and re.search("copy", r["Kernel_Name"], re.I) and not re.search("probe", r["Kernel_Name"])]
        ref = max(copies) if copies else max(allv)
        factor = calib_kib / ref
        per = np.array([v for v, _ in kvals]) * factor * 1024.0
        res[label] = (factor, per)
        lines.append(f"{counter}: {len(per)} dispatches of {kernel}; calibration copy of {calib_mib} MiB "
                     f"read {ref:.0f} KiB -> scale {factor:.4f}; bytes per dispatch mean {per.mean():.4e} "
                     f"min {per.min():.4e} max {per.max():.4e}")
    fetch_mean = float(res["fetch"][1].mean())
    write_mean = float(res["write"][1].mean())
    tail = ["", f"traffic_bytes_per_launch: {fetch_mean + write_mean:.6e}",
            f"fetch_bytes_per_launch: {fetch_mean:.6e}", f"write_bytes_per_launch: {write_mean:.6e}"]
    if avg_ns:
        tail.append(f"traffic_GBps_at_average_duration: {(fetch_mean + write_mean) / avg_ns:.1f}")
    if flops:
        rows = _csv(flops, "counter_collection.csv")
        c = {k: _mean_counter(rows, k, kernel) for k in FLOP_COUNTERS}
        lines.append("FP64 counters (mean per dispatch): " + ", ".join(
            f"{k}={v:.6e}" for k, v in c.items() if v is not None))
        # The SQ instruction counters count wave instructions.  FLOPS_FP64
        # weighs each FP64 VALU instruction by its operations (FMA 2, ADD,
        # MUL and transcendental 1; its TRANS part is a subset), per wave:
        # times 64 lanes it is the FLOP count with every lane active.  The
        # instruction counts give the same figure independently.
        fl = 64.0 * (c["SQ_INSTS_VALU_FLOPS_FP64"] or 0.0)
        fl_instr = 64.0 * sum((c[k] or 0.0) * w for k, w in (("SQ_INSTS_VALU_ADD_F64", 1), ("SQ_INSTS_VALU_MUL_F64", 1),
                                                              ("SQ_INSTS_VALU_TRANS_F64", 1),
                                                              ("SQ_INSTS_VALU_FMA_F64", 2)))
        tail.append(f"fp64_flops_per_launch: {fl:.6e}")
        tail.append(f"fp64_flops_per_launch_from_instruction_counts: {fl_instr:.6e}")
        if evals_per_launch:
            tail.append(f"fp64_flops_per_eval: {fl / evals_per_launch:.2f}")
            if c["SQ_INSTS_VALU"]:
                tail.append(f"valu_instructions_per_wave_of_64_evals: {c['SQ_INSTS_VALU'] * 64.0 / evals_per_launch:.1f}")
        if avg_ns:
            tail.append(f"fp64_TFLOPs_at_average_duration: {fl / avg_ns / 1e3:.3f}")
    if extra:
        # every counter of one more --pmc run, mean per dispatch of the kernel
        rows = _csv(extra, "counter_collection.csv")
        names = sorted({r["Counter_Name"] for r in rows})
        vals = {k: _mean_counter(rows, k, kernel) for k in names}
        lines.append("more counters (mean per dispatch): " + ", ".join(
            f"{k}={v:.6e}" for k, v in vals.items() if v is not None))
        waves = vals.get("SQ_WAVES")
        if evals_per_launch:
            for k in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD"):
                if vals.get(k) is not None:
                    tail.append(f"{k.lower()}_per_64_evals: {vals[k] * 64.0 / evals_per_launch:.1f}")
        if vals.get("SQ_INSTS_VALU_MFMA_MOPS_BF16") is not None and avg_ns:
            # MOPS counts 512-flop units of matrix work
            tail.append(f"bf16_mfma_TFLOPs_at_average_duration: "
                        f"{vals['SQ_INSTS_VALU_MFMA_MOPS_BF16'] * 512.0 / avg_ns / 1e3:.3f}")
        if waves:
            tail.append(f"waves_per_dispatch: {waves:.0f}")
    lines += tail
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def kernel_table(trace, out, command, pattern=r"pino::|k_probe"):
    """Per-kernel duration statistics of one --kernel-trace --stats run, for
    every kernel whose name matches `pattern`, with each kernel's digest."""
    stats = _csv(trace, "kernel_stats.csv")
    lines = ["# rocprofv3 kernel statistics", f"command: {command}", "",
             "kernel | calls | average_ns | min_ns | max_ns | total_ns | kernel_digest"]
    for r in stats:
        if not re.search(pattern, r["Name"]):
            continue
        short = re.sub(r"\(.*", "", r["Name"].replace("(anonymous namespace)::", ""))
        short = short.replace("pino::", "").replace("void ", "")
        try:
            dig = kernel_digest(short.split("<")[0].strip())
        except (KeyError, ValueError):
            dig = "-"
        lines.append(f"{r['Name']} | {r['Calls']} | {float(r['AverageNs']):.1f} | {r['MinNs']} | {r['MaxNs']} | "
                     f"{r['TotalDurationNs']} | {dig}")
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counter_table(pmc, out, command, kernels, evals_per_launch=None):
    """Median per dispatch of every counter of one rocprofv3 --pmc run, one
    row per kernel (with its digest), and per 64 evaluations when the
    launches' evaluation count is given.  The median, so that a few smaller
    dispatches of the same kernel (a benchmark's table fills) do not move
    the figure of its full-size launches."""
    rows = _csv(pmc, "counter_collection.csv")
    names = sorted({r["Counter_Name"] for r in rows})
    lines = ["# rocprofv3 counters per kernel", f"command: {command}", "",
             "kernel | kernel_digest | dispatches | " + " | ".join(f"{n} (median)" for n in names)]
    per64 = []
    for k in kernels:
        vals = {}
        for n in names:
            v = [x for x, _ in _counter(rows, n, k)]
            vals[n] = float(np.median(v)) if v else None
        count = len(_counter(rows, names[0], k)) if names else 0
        try:
            dig = kernel_digest(k)
        except (KeyError, ValueError):
            dig = "-"
        lines.append(f"{k} | {dig} | {count} | " + " | ".join("-" if vals[n] is None else f"{vals[n]:.4e}"
                                                              for n in names))
        if evals_per_launch:
            per64.append(f"{k}: " + ", ".join(f"{n} {vals[n] * 64.0 / evals_per_launch:.2f}"
                                              for n in names if vals[n] is not None))
    if per64:
        lines += ["", f"per 64 evaluations ({evals_per_launch:.0f} evaluations per launch):"] + per64
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_profile(path):
    """The key: value figures of a summary (floats where they parse), or {}."""
    if not os.path.exists(path):
        return {}
    out = {}
    for line in open(path):
        m = re.match(r"^([a-z0-9_A-Z]+): (\S+)\s*$", line)
        if m:
            try:
                out[m.group(1)] = float(m.group(2))
            except ValueError:
                out[m.group(1)] = m.group(2)
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summarize")
    s.add_argument("--kernel", required=True)
    s.add_argument("--trace", required=True)
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--calib-mib", type=int, default=1024)
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    s.add_argument("--flops", default=None, help="rocprofv3 --pmc output of the FP64 counters")
    s.add_argument("--evals-per-launch", type=float, default=None)
    s.add_argument("--extra", default=None, help="one more rocprofv3 --pmc output (any counters)")
    t = sub.add_parser("table")
    t.add_argument("--trace", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", default="")
    c = sub.add_parser("counters")
    c.add_argument("--pmc", required=True, help="rocprofv3 --pmc output directory")
    c.add_argument("--kernels", required=True, help="comma-separated kernel names")
    c.add_argument("--evals-per-launch", type=float, default=None)
    c.add_argument("--out", required=True)
    c.add_argument("--command", default="")
    d = sub.add_parser("digest")
    d.add_argument("kernel")
    a = ap.parse_args()
    if a.cmd == "digest":
        print(kernel_digest(a.kernel))
        return
    if a.cmd == "table":
        kernel_table(a.trace, a.out, a.command)
        return
    if a.cmd == "counters":
        counter_table(a.pmc, a.out, a.command, a.kernels.split(","), a.evals_per_launch)
        return
    summarize(a.kernel, a.trace, a.fetch, a.write, a.calib_mib, a.out, a.command, a.flops, a.evals_per_launch,
              a.extra)


if __name__ == "__main__":
    main()
