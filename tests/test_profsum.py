"""The rocprofv3 summariser used for profiles/: counter selection and copy
calibration on a synthetic results database."""
import sqlite3

from paper_2607_07816_amd import profsum


def _make_db(path, counter, rows):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (dispatch_id int, kernel_name text, grid_size int, "
               "counter_name text, value real)")
    db.execute("create table kernels (name text, start int, duration int)")
    for did, name, grid, vals in rows:
        for v in vals:  # several dimension rows per dispatch are summed
            db.execute("insert into counters_collection values (?,?,?,?,?)", (did, name, grid, counter, v))
        db.execute("insert into kernels values (?,?,?)", (name, did, 1000 * did))
    db.commit()
    db.close()


def test_traffic_calibration(tmp_path, capsys):
    f = tmp_path / "f_results.db"
    w = tmp_path / "w_results.db"
    copy = "__amd_rocclr_copyBuffer"
    kern = "void k_radix_pass<float2>(PassBufs)"
    # calibration copy of 2 MiB reads as 1 MiB FETCH and 2 MiB WRITE; small blits are ignored
    _make_db(f, "FETCH_SIZE", [(1, copy, 512, [0.5]), (2, copy, 4096, [512.0, 512.0]),
                               (3, kern, 100, [1.0]), (4, kern, 800, [300.0, 100.0]),
                               (5, kern, 800, [200.0, 200.0])])
    _make_db(w, "WRITE_SIZE", [(1, copy, 512, [0.7]), (2, copy, 4096, [2048.0]),
                               (3, kern, 100, [1.0]), (4, kern, 800, [500.0]), (5, kern, 800, [700.0])])
    profsum.main(["traffic", "--fetch", str(f), "--write", str(w), "--copy-bytes", str(2 << 20),
                  "--kernel", "k_radix_pass"])
    out = capsys.readouterr().out
    path = tmp_path / "t.txt"
    path.write_text(out)
    rec = profsum.read_traffic(str(path))
    # steady dispatches (grid 800): FETCH 400 KiB x scale 2, WRITE 600 KiB x scale 1
    assert float(rec["fetch_bytes_per_launch"]) == 400 * 1024 * 2
    assert float(rec["write_bytes_per_launch"]) == 600 * 1024
    assert float(rec["traffic_bytes_per_launch"]) == 1400 * 1024
    assert rec["source_digest"] == profsum.source_digest()


def test_kernel_rows_steady_tail(tmp_path):
    db = tmp_path / "k_results.db"
    _make_db(db, "X", [(i, "void k_tile_emit<float2, 2>(x)", 1, [0.0]) for i in range(1, 11)])
    rows = profsum.kernel_rows(str(db), last=0.5)
    (name, calls, tot, avg, lo, hi, steady), = rows
    assert name.startswith("k_tile_emit") and calls == 10
    assert avg == 5500 and steady == 8000 and lo == 1000 and hi == 10000


def test_short_kernel_names():
    from paper_2607_07816_amd.profsum import short
    assert short("void (anonymous namespace)::k_radix_pass<1>(unsigned long const*)") == "k_radix_pass<c64>"
    assert short("_ZN12_GLOBAL__N_112k_radix_passILi2EEEvPKyS2_PyS3_") == "k_radix_pass<c128>"
    assert short("void sts_group::k_tile_hist<HIP_vector_type<float, 2u>, 2>(GateArg, PassBufs)") == "k_tile_hist<c64>"
    assert short("void sts_group::k_tile_emit<HIP_vector_type<double, 2u>, 3>(GateArg, PassBufs)") == "k_tile_emit<c128>"
    assert short("(anonymous namespace)::k_radix_count(unsigned long const*)") == "k_radix_count"


def test_counters_per_dispatch_and_wave(tmp_path, capsys):
    a = tmp_path / "a_results.db"
    b = tmp_path / "b_results.db"
    kern = "void sts_group::k_tile_emit<HIP_vector_type<float, 2u>, 2>(GateArg, PassBufs)"
    other = "k_pick1(PassBufs, int, int, int)"
    _make_db(a, "SQ_WAVES", [(1, kern, 100, [4.0]), (2, kern, 800, [16.0, 16.0]), (3, other, 256, [4.0])])
    _make_db(b, "SQ_INSTS_VALU", [(1, kern, 100, [9.0]), (2, kern, 800, [3200.0]), (3, other, 256, [1.0])])
    profsum.main(["counters", str(a), str(b), "--kernel", "k_tile_emit", "--command", "x", "--command", "y"])
    out = capsys.readouterr().out
    assert "k_tile_emit<c64>" in out and "k_pick1" not in out
    line = [l for l in out.splitlines() if "SQ_INSTS_VALU" in l][0]
    # steady dispatch only (grid 800): 3200 instructions over 32 waves
    assert "3200" in line and "100.0 per wave" in line
    assert "# command 2: y" in out
