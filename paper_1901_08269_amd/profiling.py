"""Summaries of rocprofv3 result databases as short markdown.

Five reports:

``stats``    per-kernel call counts and durations from a ``--kernel-trace --stats`` run.
``kernels``  the solve kernels of such a run against the HBM roofline: algorithmic bytes
             per interior point (each operand read or written once), GB/s from the average
             launch duration, fraction of the 8 TB/s peak.
``mfma``     MFMA busy share and BF16 matrix FLOP rate of the network's kernels from one ``--pmc`` run.
``counters`` counters of chosen kernels from one or more ``--pmc`` passes, with derived
             figures (resident waves, wait shares, cache latencies, address-unit load).
``traffic``  HBM bytes per launch of one kernel (or several counted together, as the
             instantiations of one kernel template) on the problem's grid from two ``--pmc`` runs
             (``FETCH_SIZE`` and ``WRITE_SIZE``, each in its own pass), each counter scaled by
             what the same counter reads for a plain device copy of known size (the
             calibration runs).  The report
             ends with machine-readable ``key: value`` lines, including a hash of the kernel
             sources, so a reader can tell whether the counters still describe the code.

Usage::

    python -m paper_1901_08269_amd.profiling stats DB --title T --cmd C [--top 20]
    python -m paper_1901_08269_amd.profiling kernels DB --points P --title T --cmd C
    python -m paper_1901_08269_amd.profiling mfma DB --title T --cmd C
    python -m paper_1901_08269_amd.profiling counters DB [DB ...] --kernel NAME [--kernel ...] --title T --cmd C
    python -m paper_1901_08269_amd.profiling traffic --fetch DB --write DB \\
        --copy-fetch DB --copy-write DB --copy-bytes B --kernel NAME=BYTES_PER_UNIT [--kernel ...] --units U \\
        --title T --cmd C
"""
import argparse
import hashlib
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
# what defines the measured sweep kernel: the data layout header, and in sweeps.hip the
# Chebyshev section from its heading to the end of k_cheb4 (its helpers and the kernel);
# a traffic report is stale once any of it changes
KERNEL_HEADER = "csrc/cps_device.h"
KERNEL_FILE = "csrc/sweeps.hip"
KERNEL_START = "// Chebyshev-Jacobi steps on K phi = rho"
KERNEL_NAME = " k_cheb4("
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source():
    """The source text the sweep kernel is compiled from (see KERNEL_*)."""
    with open(os.path.join(HERE, KERNEL_FILE)) as fh:
        src = fh.read()
    a = src.index(KERNEL_START)
    b = src.index("\n}\n", src.index(KERNEL_NAME, a)) + 3
    with open(os.path.join(HERE, KERNEL_HEADER)) as fh:
        return fh.read() + src[a:b]


def source_hash():
    return hashlib.sha256(kernel_source().encode()).hexdigest()[:16]


def short_name(n):
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(cps::Geom.*", "", n)
    n = re.sub(r"\(.*", "", n)
    return n.replace("void ", "")


def kernel_stats(db):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name,total_calls,total_duration,average,percentage from top_kernels"))
    con.close()
    return rows


def _problem_grid(groups):
    """Pick the launches on the problem's grid from {key: [(duration, value), ...]} groups of
    one kernel by launch grid.  A multigrid kernel runs on every level, one launch grid per
    level, and the problem's grid is the one whose launches take longest; two levels can
    share a launch grid, so within a group the launches shorter than 0.4 of its 90th
    percentile duration (a much smaller level) are left out."""
    best = None
    for key, items in groups.items():
        d = sorted(x[0] for x in items)
        cut = 0.4 * d[min(len(d) - 1, int(0.9 * len(d)))]
        kept = [x for x in items if x[0] >= cut]
        mean = sum(x[0] for x in kept) / len(kept)
        if best is None or mean > best[0]:
            best = (mean, kept)
    return best[1]


def pmc_per_kernel(db):
    """{short kernel name: (dispatches, mean counter value, mean duration ns)} over each
    kernel's dispatches on the problem's grid (see _problem_grid)."""
    con = sqlite3.connect(db)
    acc = {}
    rows = con.execute("select p.name, p.counter_value, p.duration, k.grid_x * k.grid_y * k.grid_z "
                       "from pmc_events p join kernels k on p.dispatch_id = k.dispatch_id")
    for name, val, dur, size in rows:
        acc.setdefault(short_name(name), {}).setdefault(size, []).append((dur, val))
    con.close()
    out = {}
    for n, groups in acc.items():
        kept = _problem_grid(groups)
        out[n] = (len(kept), sum(v for _, v in kept) / len(kept), sum(d for d, _ in kept) / len(kept))
    return out


def stats_report(db, title, cmd, top=20):
    out = [f"# {title}", "", "Command (run from the repository root on an MI355X):", "", "```", cmd, "```", "",
           "Kernel statistics from `rocprofv3 --kernel-trace --stats` (durations in microseconds):", "",
           "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a, p in kernel_stats(db)[:top]:
        out.append(f"| `{short_name(n)}` | {c} | {t:.1f} | {a:.2f} | {p:.1f} |")
    return "\n".join(out) + "\n"


HBM_PEAK_GBS = 8000.0
_SIZE = {"float": 4, "double": 8}


def algorithmic_bytes(name):
    """Bytes per interior point that a solve kernel must move (each operand once), or None.

    k_cheb4       one Chebyshev step: x_k, x_{k-1}, rho in, x_{k+1} out (no x_{k-1}: first step)
    k_first4      p = r + beta (p - omega v) (P) or s = r - alpha v (S), and x_1 = c p / diag K
    k_apply4      y = B x with a second operand (V, T), y = B x (plain), r = b - B x (residual)
    k_update4     x += alpha p^ + omega s^, r = s - omega t, with (r0, r)
    k_resid4      r = rho - K x (multigrid): x, rho in, r out
    k_mg_restrict fine r in; coarse rho and first step out, coarse diagonal in (1/8 of a
                  value each per fine point)
    k_mg_resid_restrict  x, rho in; coarse rho and first step out, coarse diagonal in
    k_mg_prolong_add  x += P e: x in and out, the coarse e in (1/8 per fine point)
    """
    n = short_name(name)
    m = re.match(r"cps::(k_cheb4|k_first4|k_apply4|k_update4|k_resid4|k_mg_restrict|k_mg_resid_restrict"
                 r"|k_mg_prolong_add)<(.*)>$", n)
    if not m:
        return None
    kern, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
    t = _SIZE.get(args[0])
    if t is None:
        return None
    if kern == "k_cheb4":
        return (3 if args[1] == "true" else 4) * t
    if kern == "k_resid4":
        return 3 * t
    if kern == "k_mg_restrict":
        return t + 3 * t / 8
    if kern == "k_mg_resid_restrict":
        return 2 * t + 3 * t / 8
    if kern == "k_mg_prolong_add":
        return 2 * t + t / 8
    if kern == "k_first4":
        return (5 if args[1] == "0" else 4) * t
    if kern == "k_update4":
        return 8 * t
    to, mode = _SIZE[args[1]], int(args[2])
    if mode == 0:
        return t + to
    if mode in (1, 2):
        return 2 * t + to
    return t + 8 + to       # residual: x and b (FP64) in, r out


def fine_grid_launches(db):
    """Per solve kernel, its launches on the problem's grid (see _problem_grid).
    [(name, calls, avg us)]"""
    con = sqlite3.connect(db)
    groups = {}
    for name, gx, gy, gz, dur in con.execute("select name, grid_x, grid_y, grid_z, duration from kernels"):
        groups.setdefault(name, {}).setdefault(gx * gy * gz, []).append((dur, 0.0))
    con.close()
    rows = []
    for name, g in groups.items():
        kept = _problem_grid(g)
        rows.append((name, len(kept), sum(d for d, _ in kept) / len(kept) / 1e3))
    return sorted(rows, key=lambda r: -r[1] * r[2])


def kernels_report(db, points, title, cmd, exclude=()):
    """exclude: short kernel names that have no launch over the problem's grid in the run (a
    kernel that only runs on coarser grids, or only over the irregular rows there), whose
    longest launches would otherwise be taken for it."""
    out = [f"# {title}", "", "Command (run from the repository root on an MI355X):", "", "```", cmd, "```", "",
           f"Solve kernels from `rocprofv3 --kernel-trace --stats`, launches on the problem's grid only "
           f"({points} interior points per launch; a multigrid kernel's launches on coarser grids are left "
           "out); algorithmic bytes count each operand once per point (tables, halos, bits and the "
           f"irregular rows as overhead); GB/s = bytes per launch / average duration; peak "
           f"{HBM_PEAK_GBS:.0f} GB/s."]
    if exclude:
        out.append("Left out, as they make no launch over the problem's grid: "
                   + ", ".join(f"`{n}`" for n in exclude) + ".")
    out += ["", "| kernel | calls | avg us | B / point | GB/s | of peak |", "|---|---:|---:|---:|---:|---:|"]
    for n, c, a in fine_grid_launches(db):
        b = algorithmic_bytes(n)
        if b is None or short_name(n) in exclude:
            continue
        gbs = b * points / (a * 1e-6) / 1e9
        out.append(f"| `{short_name(n)}` | {c} | {a:.2f} | {b:g} | {gbs:.0f} | {gbs / HBM_PEAK_GBS:.2f} |")
    return "\n".join(out) + "\n"


def traffic_report(a):
    """Calibrated FETCH_SIZE + WRITE_SIZE of one kernel or of several (a.kernel: "NAME=B" items,
    B the algorithmic bytes per unit of that kernel): the per-launch figures are averages over
    all their launches on the problem's grid."""
    cf = pmc_per_kernel(a.copy_fetch)[COPY_KERNEL]
    cw = pmc_per_kernel(a.copy_write)[COPY_KERNEL]
    kib = a.copy_bytes / 1024.0
    sf, sw = kib / cf[1], kib / cw[1]
    fetch, write = pmc_per_kernel(a.fetch), pmc_per_kernel(a.write)
    kernels = [(k.rsplit("=", 1)[0], float(k.rsplit("=", 1)[1])) for k in a.kernel]
    rows, nf, nw, rd_sum, wr_sum, alg_sum, dur_sum = [], 0, 0, 0.0, 0.0, 0.0, 0.0
    for name, ub in kernels:
        f, w = fetch[name], write[name]
        rd, wr, alg = f[1] * sf * 1024.0, w[1] * sw * 1024.0, a.units * ub
        rows.append(f"| `{name}` | {f[0]} / {w[0]} | {f[1]:.1f} | {w[1]:.1f} | {rd + wr:.4g} | {alg:.4g} | "
                    f"{(rd + wr) / alg:.3f} | {f[2] / 1e3:.1f} |")
        nf += f[0]
        nw += w[0]
        rd_sum += f[0] * rd
        wr_sum += w[0] * wr
        alg_sum += f[0] * alg
        dur_sum += f[0] * f[2]
    rd, wr, alg = rd_sum / nf, wr_sum / nw, alg_sum / nf
    names = ", ".join(n for n, _ in kernels)
    out = [f"# {a.title}", "", "Commands (run from the repository root on an MI355X, each counter in its own pass):",
           "", "```", a.cmd, "```", "",
           f"Calibration: a device copy of {a.copy_bytes} bytes (`{COPY_KERNEL}`) reads "
           f"FETCH_SIZE = {cf[1]:.1f} KiB and WRITE_SIZE = {cw[1]:.1f} KiB per dispatch, so the counters are "
           f"scaled by {sf:.4f} (fetch) and {sw:.4f} (write).", "",
           "| kernel | dispatches (fetch / write pass) | FETCH_SIZE raw KiB | WRITE_SIZE raw KiB | "
           "HBM traffic per launch, B | algorithmic per launch, B | traffic / algorithmic | mean us under counters |",
           "|---|---:|---:|---:|---:|---:|---:|---:|", *rows, "",
           f"Over all {nf} launches: HBM read {rd:.4g} B and write {wr:.4g} B per launch (scaled), traffic "
           f"{rd + wr:.4g} B against {alg:.4g} algorithmic ({a.units} units per launch): "
           f"{(rd + wr) / alg:.3f}; mean duration under counters {dur_sum / nf / 1e3:.1f} us.", "",
           "Machine-readable:", "", "```",
           f"kernel: {names}",
           f"traffic_bytes_per_launch: {rd + wr:.6g}",
           f"read_bytes_per_launch: {rd:.6g}",
           f"write_bytes_per_launch: {wr:.6g}",
           f"algorithmic_bytes_per_launch: {alg:.6g}",
           f"kernel_source_sha256_16: {source_hash()}",
           "```", ""]
    return "\n".join(out)


SIMDS = 256 * 4                 # MI355X: 256 compute units of 4 SIMDs
BF16_PEAK_TFLOPS = 2500.0       # dense BF16 matrix peak


def mfma_report(db, title, cmd):
    """Per network kernel (one --pmc pass of SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE and
    SQ_INSTS_VALU_MFMA_MOPS_BF16): dispatches, mean duration, MFMA busy share (busy cycles
    over active cycles times the SIMD count, as rocprofv3's MfmaUtil) and BF16 matrix FLOPs
    (512 per MOPS unit) per second against the dense BF16 peak."""
    con = sqlite3.connect(db)
    acc = {}
    for name, disp, dur, cname, val in con.execute(
            "select name, dispatch_id, duration, counter_name, counter_value from pmc_events"):
        if "cpsnet" not in name:
            continue
        k = acc.setdefault(short_name(name), {})
        d = k.setdefault(disp, {"dur": dur})
        d[cname] = d.get(cname, 0.0) + val
    con.close()
    out = [f"# {title}", "", "Command (run from the repository root on an MI355X):", "", "```", cmd, "```", "",
           f"MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x {SIMDS} SIMDs); BF16 TFLOP/s = "
           f"512 x SQ_INSTS_VALU_MFMA_MOPS_BF16 / duration, against {BF16_PEAK_TFLOPS:.0f} TFLOP/s dense.", "",
           "| kernel | dispatches | mean us | MFMA busy % | BF16 TFLOP/s | of peak |",
           "|---|---:|---:|---:|---:|---:|"]
    rows = []
    tot_dur = tot_fl = tot_busy = tot_act = 0.0
    for n, disps in acc.items():
        ds = list(disps.values())
        dur = sum(d["dur"] for d in ds)
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in ds)
        act = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in ds)
        fl = 512.0 * sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) for d in ds)
        rows.append((dur, n, len(ds), busy, act, fl))
        tot_dur += dur
        tot_fl += fl
        tot_busy += busy
        tot_act += act
    for dur, n, c, busy, act, fl in sorted(rows, reverse=True):
        tf = fl / (dur * 1e-9) / 1e12 if dur else 0.0
        util = 100.0 * busy / (act * SIMDS) if act else 0.0
        out.append(f"| `{n}` | {c} | {dur / c / 1e3:.2f} | {util:.1f} | {tf:.1f} | {tf / BF16_PEAK_TFLOPS:.4f} |")
    tf = tot_fl / (tot_dur * 1e-9) / 1e12 if tot_dur else 0.0
    util = 100.0 * tot_busy / (tot_act * SIMDS) if tot_act else 0.0
    out.append(f"| all network kernels | {sum(r[2] for r in rows)} | {tot_dur / 1e3:.1f} total | {util:.1f} | "
               f"{tf:.1f} | {tf / BF16_PEAK_TFLOPS:.4f} |")
    return "\n".join(out) + "\n"


def counters_report(dbs, kernels, title, cmd):
    """Per kernel (matched by its short name), the mean over dispatches of each counter summed
    over its hardware instances, from one or more ``--pmc`` passes of the same program, and the
    figures derived from them where their counters are present:

    * waves resident per SIMD: 4 SQ_WAVE_CYCLES (quad-cycles, summed over the shader engines)
      over the busy cycles of one engine (SQ_BUSY_CYCLES summed over the engines, divided by
      their count) and the SIMD count;
    * the share of wave time spent waiting (SQ_WAIT_ANY), waiting for issue
      (SQ_WAIT_INST_ANY) and executing (SQ_ACTIVE_INST_ANY), each over SQ_WAVE_CYCLES;
    * instructions per wave (SQ_INSTS_* over SQ_WAVES);
    * mean L1-to-L2 read latency in cycles (TCP_TCC_READ_REQ_LATENCY_sum over
      TCP_TCC_READ_REQ_sum) and mean L2-to-memory read latency (TCC_EA0_RDREQ_LEVEL_sum over
      TCC_EA0_RDREQ_sum), the L2 hit share (TCC_HIT_sum over TCC_HIT_sum + TCC_MISS_sum);
    * the share of active GPU cycles (GRBM_GUI_ACTIVE) in which the address unit is busy
      (TA_BUSY_avr) or its address path is stalled by the cache (TA_ADDR_STALLED_BY_TC_CYCLES
      per TA instance)."""
    acc = {}
    for db in dbs:
        con = sqlite3.connect(db)
        for name, disp, dur, cname, val in con.execute(
                "select name, dispatch_id, duration, counter_name, counter_value from pmc_events"):
            n = short_name(name)
            if n not in kernels:
                continue
            d = acc.setdefault(n, {}).setdefault(cname, {}).setdefault((db, disp), [0.0, 0, dur])
            d[0] += val
            d[1] += 1
        con.close()
    names = []
    for n in kernels:
        for c in acc.get(n, {}):
            if c not in names:
                names.append(c)

    def mean(n, c):
        ds = acc.get(n, {}).get(c)
        return None if not ds else sum(v[0] for v in ds.values()) / len(ds)

    def inst(n, c):
        ds = acc.get(n, {}).get(c)
        return None if not ds else sum(v[1] for v in ds.values()) / len(ds)

    out = [f"# {title}", "", "Commands (run from the repository root on an MI355X, one counter set per pass):", "",
           "```", cmd, "```", "", "Each counter summed over its hardware instances, mean over dispatches:", "",
           "| counter | " + " | ".join(f"`{n}`" for n in kernels) + " |",
           "|---|" + "---:|" * len(kernels)]
    rows = [("dispatches", lambda n: max((len(v) for v in acc.get(n, {}).values()), default=0)),
            ("mean us under counters", lambda n: next(
                (sum(v[2] for v in ds.values()) / len(ds) / 1e3 for ds in acc.get(n, {}).values()), None))]
    for c in names:
        rows.append((c, lambda n, c=c: mean(n, c)))

    def fmt(v):
        if v is None:
            return "-"
        return f"{v:.4g}" if abs(v) < 1e6 else f"{v:.4e}"
    for label, f in rows:
        out.append(f"| {label} | " + " | ".join(fmt(f(n)) for n in kernels) + " |")

    def ratio(a, b, scale=1.0):
        return None if a is None or not b else scale * a / b

    def derived(n):
        W, B, S = mean(n, "SQ_WAVE_CYCLES"), mean(n, "SQ_BUSY_CYCLES"), inst(n, "SQ_BUSY_CYCLES")
        waves = mean(n, "SQ_WAVES")
        res = None if W is None or not B or not S else 4.0 * W / (B / S) / SIMDS
        hit, miss = mean(n, "TCC_HIT_sum"), mean(n, "TCC_MISS_sum")
        gui = mean(n, "GRBM_GUI_ACTIVE")
        stall, ta_n = mean(n, "TA_ADDR_STALLED_BY_TC_CYCLES"), inst(n, "TA_ADDR_STALLED_BY_TC_CYCLES")
        return [("waves resident per SIMD", res),
                ("wave time waiting, %", ratio(mean(n, "SQ_WAIT_ANY"), W, 100.0)),
                ("wave time waiting for issue, %", ratio(mean(n, "SQ_WAIT_INST_ANY"), W, 100.0)),
                ("wave time executing, %", ratio(mean(n, "SQ_ACTIVE_INST_ANY"), W, 100.0)),
                ("VALU instructions per wave", ratio(mean(n, "SQ_INSTS_VALU"), waves)),
                ("vector loads per wave", ratio(mean(n, "SQ_INSTS_VMEM_RD"), waves)),
                ("L1-to-L2 read latency, cycles",
                 ratio(mean(n, "TCP_TCC_READ_REQ_LATENCY_sum"), mean(n, "TCP_TCC_READ_REQ_sum"))),
                ("L2-to-memory read latency, cycles",
                 ratio(mean(n, "TCC_EA0_RDREQ_LEVEL_sum"), mean(n, "TCC_EA0_RDREQ_sum"))),
                ("L2 hit share, %", None if hit is None or miss is None or not hit + miss else 100.0 * hit / (hit + miss)),
                ("address unit busy, % of active cycles", ratio(mean(n, "TA_BUSY_avr"), gui, 100.0)),
                ("address path stalled by the cache, % of active cycles",
                 None if stall is None or not ta_n or not gui else 100.0 * stall / ta_n / gui)]
    table = [derived(n) for n in kernels]
    if table and any(v is not None for row in table for _, v in row):
        out += ["", "Derived:", "", "| figure | " + " | ".join(f"`{n}`" for n in kernels) + " |",
                "|---|" + "---:|" * len(kernels)]
        for q in range(len(table[0])):
            if all(t[q][1] is None for t in table):
                continue
            out.append(f"| {table[0][q][0]} | " + " | ".join(fmt(t[q][1]) for t in table) + " |")
    return "\n".join(out) + "\n"


def read_traffic(path):
    """The machine-readable lines of a traffic report, or None if absent."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        m = re.match(r"^([a-z_0-9]+): (.+)$", line.strip())
        if m:
            kv[m.group(1)] = m.group(2)
    return kv or None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--top", type=int, default=20)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--points", type=int, required=True)
    k.add_argument("--title", required=True)
    k.add_argument("--cmd", required=True)
    k.add_argument("--exclude", action="append", default=[],
                   help="short kernel name without a launch over the problem's grid (repeatable)")
    mf = sub.add_parser("mfma")
    mf.add_argument("db")
    mf.add_argument("--title", required=True)
    mf.add_argument("--cmd", required=True)
    cn = sub.add_parser("counters")
    cn.add_argument("db", nargs="+")
    cn.add_argument("--kernel", action="append", required=True, help="short kernel name (repeatable)")
    cn.add_argument("--title", required=True)
    cn.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "title", "cmd"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--kernel", action="append", required=True,
                   help="NAME=BYTES_PER_UNIT (repeat for several kernels counted together)")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--units", type=int, required=True)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        print(stats_report(a.db, a.title, a.cmd, a.top), end="")
    elif a.mode == "kernels":
        print(kernels_report(a.db, a.points, a.title, a.cmd, tuple(a.exclude)), end="")
    elif a.mode == "mfma":
        print(mfma_report(a.db, a.title, a.cmd), end="")
    elif a.mode == "counters":
        print(counters_report(a.db, a.kernel, a.title, a.cmd), end="")
    else:
        print(traffic_report(a), end="")


if __name__ == "__main__":
    main()
