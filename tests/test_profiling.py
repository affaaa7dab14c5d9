"""Host-side checks of the rocprofv3 summary tool: the counter scaling of the traffic report
and the parsing that the benchmark relies on, on small synthetic result databases."""
import argparse
import sqlite3

from paper_1901_08269_amd import profiling


def _pmc_db(path, rows):
    """rows: (name, counter value, duration) or (name, counter value, duration, grid_x)."""
    con = sqlite3.connect(path)
    con.execute("create table pmc_events (name text, counter_value real, duration real, dispatch_id int)")
    con.execute("create table kernels (dispatch_id int, grid_x int, grid_y int, grid_z int)")
    for q, r in enumerate(rows):
        con.execute("insert into pmc_events values (?,?,?,?)", (r[0], r[1], r[2], q))
        con.execute("insert into kernels values (?,?,1,1)", (q, r[3] if len(r) > 3 else 256))
    con.commit()
    con.close()
    return str(path)


def test_traffic_report_scales_by_copy_calibration(tmp_path):
    copy_bytes = 1 << 20                       # 1024 KiB copied
    cf = _pmc_db(tmp_path / "cf.db", [(profiling.COPY_KERNEL, 512.0, 10.0)] * 3)     # counter reads half
    cw = _pmc_db(tmp_path / "cw.db", [(profiling.COPY_KERNEL, 1024.0, 10.0)] * 3)    # counter exact
    k = "void cps::k_cheb<float, false>(cps::Geom, int)"
    # the shorter launches of another launch grid (a coarser multigrid level) are left out
    f = _pmc_db(tmp_path / "f.db", [(k, 100.0, 2000.0), (k, 300.0, 4000.0), ("other", 9.0, 1.0),
                                    (k, 7.0, 100.0, 512), (k, 5.0, 100.0, 512)])
    w = _pmc_db(tmp_path / "w.db", [(k, 50.0, 2000.0)] * 2)
    a = argparse.Namespace(fetch=f, write=w, copy_fetch=cf, copy_write=cw, copy_bytes=copy_bytes,
                           kernel=["cps::k_cheb<float, false>=16"], units=1000, title="t", cmd="c")
    rep = profiling.traffic_report(a)
    p = tmp_path / "rep.md"
    p.write_text(rep)
    kv = profiling.read_traffic(str(p))
    # fetch: mean 200 KiB x 2 = 400 KiB; write: 50 KiB x 1
    assert abs(float(kv["read_bytes_per_launch"]) - 400 * 1024) < 1
    assert abs(float(kv["write_bytes_per_launch"]) - 50 * 1024) < 1
    assert abs(float(kv["traffic_bytes_per_launch"]) - 450 * 1024) < 1
    assert float(kv["algorithmic_bytes_per_launch"]) == 16000.0
    assert kv["kernel_source_sha256_16"] == profiling.source_hash()
    assert len(profiling.source_hash()) == 16


def test_traffic_report_averages_several_kernels_over_their_launches(tmp_path):
    """Two instantiations counted together: per-launch figures are launch-weighted means."""
    copy_bytes = 1 << 20
    cf = _pmc_db(tmp_path / "cf.db", [(profiling.COPY_KERNEL, 1024.0, 10.0)])
    cw = _pmc_db(tmp_path / "cw.db", [(profiling.COPY_KERNEL, 1024.0, 10.0)])
    a_, b_ = "cps::k_cheb<float, true>", "cps::k_cheb<float, false>"
    f = _pmc_db(tmp_path / "f.db", [(a_, 100.0, 10.0)] * 2 + [(b_, 400.0, 10.0)])     # 2 + 1 launches
    w = _pmc_db(tmp_path / "w.db", [(a_, 10.0, 10.0)] * 2 + [(b_, 40.0, 10.0)])
    a = argparse.Namespace(fetch=f, write=w, copy_fetch=cf, copy_write=cw, copy_bytes=copy_bytes,
                           kernel=[a_ + "=12", b_ + "=16"], units=100, title="t", cmd="c")
    p = tmp_path / "rep.md"
    p.write_text(profiling.traffic_report(a))
    kv = profiling.read_traffic(str(p))
    assert abs(float(kv["read_bytes_per_launch"]) - (2 * 100 + 400) / 3 * 1024) < 1.0
    assert abs(float(kv["write_bytes_per_launch"]) - (2 * 10 + 40) / 3 * 1024) < 1.0
    assert abs(float(kv["algorithmic_bytes_per_launch"]) - (2 * 1200 + 1600) / 3) < 1e-2   # 6 digits printed
    assert kv["kernel"] == f"{a_}, {b_}"


def test_read_traffic_missing(tmp_path):
    assert profiling.read_traffic(str(tmp_path / "none.md")) is None


def test_stats_report(tmp_path):
    db = tmp_path / "s.db"
    con = sqlite3.connect(db)
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, average real, percentage real)")
    con.execute("insert into top_kernels values ('void cps::k_update<float>(cps::Geom, int)', 4, 400.0, 100.0, 55.0)")
    con.commit()
    con.close()
    rep = profiling.stats_report(str(db), "T", "cmd")
    assert "| `cps::k_update<float>` | 4 | 400.0 | 100.00 | 55.0 |" in rep


def test_algorithmic_bytes_per_kernel():
    ab = profiling.algorithmic_bytes
    assert ab("void cps::k_cheb4<float, false>(cps::Geom, int)") == 16
    assert ab("void cps::k_cheb4<float, true>(cps::Geom, int)") == 12
    assert ab("void cps::k_cheb4<double, false>(cps::Geom, int)") == 32
    assert ab("void cps::k_first4<float, 0>(cps::Geom)") == 20
    assert ab("void cps::k_first4<float, 1>(cps::Geom)") == 16
    assert ab("void cps::k_update4<double>(cps::Geom)") == 64
    assert ab("void cps::k_apply4<float, float, 1>(cps::Geom)") == 12
    assert ab("void cps::k_apply4<double, float, 3>(cps::Geom)") == 20
    assert ab("void cps::k_apply4<double, double, 0>(cps::Geom)") == 16
    assert ab("void cps::k_finalize<0>(double const*, int, cps::DevState*)") is None
    assert ab("void cps::k_resid4<float>(cps::Geom)") == 12
    assert ab("void cps::(anonymous namespace)::k_mg_prolong_add<double>(int, int)") == 17
    # fused residual + restriction: x and rho per fine point, three coarse values per 8 points
    assert ab("void cps::(anonymous namespace)::k_mg_resid_restrict<float, false>(cps::Geom)") == 9.5
    assert ab("void cps::(anonymous namespace)::k_mg_resid_restrict<double, true>(cps::Geom)") == 19
    assert ab("void cps::(anonymous namespace)::k_mg_restrict<float>(int)") == 5.5


def test_kernels_report(tmp_path):
    """Only each kernel's launches on the problem's grid (its longest launches) are reported."""
    db = tmp_path / "s.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, grid_y int, grid_z int, duration real)")
    sweep = "void cps::k_cheb4<float, false>(cps::Geom, int)"
    for _ in range(10):
        con.execute("insert into kernels values (?, 79872, 4, 1, 40000.0)", (sweep,))
    for _ in range(7):                                   # a coarse level: shorter launches, left out
        con.execute("insert into kernels values (?, 135168, 4, 1, 12000.0)", (sweep,))
    con.execute("insert into kernels values ('void cps::(anonymous namespace)::k_mg_restrict<float>(int)', "
                "64, 128, 128, 20000.0)")
    con.execute("insert into kernels values ('void cps::k_fill<float>(unsigned long, float*, float)', 256, 1, 1, 2e4)")
    con.commit()
    con.close()
    rep = profiling.kernels_report(str(db), 1000000, "T", "cmd")
    # 16 B x 1e6 points in 40 us = 400 GB/s = 0.05 of 8 TB/s
    assert "| `cps::k_cheb4<float, false>` | 10 | 40.00 | 16 | 400 | 0.05 |" in rep
    # restriction: 5.5 B per fine point in 20 us = 275 GB/s
    assert "| `cps::k_mg_restrict<float>` | 1 | 20.00 | 5.5 | 275 | 0.03 |" in rep
    assert "k_fill" not in rep
    # a kernel without launches over the problem's grid is left out by name
    rep = profiling.kernels_report(str(db), 1000000, "T", "cmd", exclude=("cps::k_mg_restrict<float>",))
    assert "| `cps::k_mg_restrict<float>`" not in rep and "Left out" in rep
    assert "| `cps::k_cheb4<float, false>` | 10 | 40.00 | 16 | 400 | 0.05 |" in rep


def test_kernels_report_separates_levels_sharing_a_launch_grid(tmp_path):
    """Two multigrid levels can launch the sweep with the same grid (a coarse level's latency
    tiling): the much shorter launches of the smaller level are left out."""
    db = tmp_path / "s.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, grid_y int, grid_z int, duration real)")
    sweep = "void cps::k_cheb4<float, false>(cps::Geom, int)"
    for _ in range(10):
        con.execute("insert into kernels values (?, 65536, 4, 1, 40000.0)", (sweep,))
        con.execute("insert into kernels values (?, 65536, 4, 1, 5000.0)", (sweep,))
    con.commit()
    con.close()
    rep = profiling.kernels_report(str(db), 1000000, "T", "cmd")
    assert "| `cps::k_cheb4<float, false>` | 10 | 40.00 | 16 | 400 | 0.05 |" in rep


def test_counters_report_sums_instances_and_derives_figures(tmp_path):
    """Counters summed over their instances per dispatch, averaged over dispatches, from two
    passes; resident waves = 4 wave quad-cycles / (busy cycles of one engine) / SIMDs."""
    k = "cps::k_x<float>"
    dbs = []
    for q, rows in enumerate([
        # pass A: two engines report each SQ counter; two dispatches
        [(7, "SQ_WAVES", 10.0), (7, "SQ_WAVES", 14.0), (7, "SQ_WAVE_CYCLES", 512.0), (7, "SQ_WAVE_CYCLES", 512.0),
         (7, "SQ_BUSY_CYCLES", 100.0), (7, "SQ_BUSY_CYCLES", 100.0), (7, "SQ_WAIT_ANY", 256.0),
         (7, "SQ_WAIT_ANY", 256.0),
         (9, "SQ_WAVES", 12.0), (9, "SQ_WAVES", 12.0), (9, "SQ_WAVE_CYCLES", 512.0), (9, "SQ_WAVE_CYCLES", 512.0),
         (9, "SQ_BUSY_CYCLES", 100.0), (9, "SQ_BUSY_CYCLES", 100.0), (9, "SQ_WAIT_ANY", 256.0),
         (9, "SQ_WAIT_ANY", 256.0)],
        # pass B: cache counters, one dispatch
        [(3, "TCC_HIT_sum", 30.0), (3, "TCC_MISS_sum", 70.0), (3, "TCP_TCC_READ_REQ_LATENCY_sum", 5000.0),
         (3, "TCP_TCC_READ_REQ_sum", 10.0)]]):
        db = str(tmp_path / f"p{q}.db")
        con = sqlite3.connect(db)
        con.execute("create table pmc_events (name text, dispatch_id int, duration real, counter_name text, "
                    "counter_value real)")
        for disp, c, v in rows:
            con.execute("insert into pmc_events values (?,?,?,?,?)", (f"void {k}(cps::Geom, int)", disp, 2000.0, c, v))
        con.execute("insert into pmc_events values (?,?,?,?,?)", ("void cps::k_other(int)", 1, 5.0, "SQ_WAVES", 1e9))
        con.commit()
        con.close()
        dbs.append(db)
    rep = profiling.counters_report(dbs, [k], "t", "c")
    lines = {l.split("|")[1].strip(): l.split("|")[2].strip() for l in rep.splitlines() if l.startswith("| ")}
    assert lines["SQ_WAVES"] == "24"                     # 10 + 14 and 12 + 12
    assert lines["dispatches"] == "2"
    assert lines["mean us under counters"] == "2"
    # 4 x 1024 quad-cycles / (200 cycles / 2 engines) / 1024 SIMDs
    assert abs(float(lines["waves resident per SIMD"]) - 4.0 * 1024 / 100.0 / profiling.SIMDS) < 1e-12
    assert float(lines["wave time waiting, %"]) == 50.0
    assert float(lines["L2 hit share, %"]) == 30.0
    assert float(lines["L1-to-L2 read latency, cycles"]) == 500.0
    assert "k_other" not in rep
