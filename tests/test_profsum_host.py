"""Host tests of the rocprofv3 summariser (paper_2411_06405_amd.profsum) on
small synthetic databases: kernel names, per-kernel counter means, and the
copy-calibrated HBM bytes per launch and per decomposition."""
import json
import sqlite3

from paper_2411_06405_amd import profsum


def test_short_strips_namespace_parameters_and_templates():
    assert profsum.short("hotruss::k_level<1024u, 2048u>(hotruss::Dev const*, unsigned int)") \
        == "k_level"
    assert profsum.short("void k_support_init<64, 1>") == "k_support_init"
    assert profsum.short("hotruss::k_support(hotruss::Dev const*)") == "k_support"
    assert profsum.short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def _pmc_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?)", rows)
    c.commit()
    c.close()


def test_counters_summary_means_per_kernel(tmp_path):
    lv = "hotruss::k_level<1024u, 2048u>(hotruss::Dev const*, unsigned int)"
    sp = "hotruss::k_support(hotruss::Dev const*)"
    db = tmp_path / "pmc.db"
    _pmc_db(db, [(lv, "SQ_INSTS_LDS", 10.0), (lv, "SQ_INSTS_LDS", 30.0),
                 (lv, "SQ_LDS_BANK_CONFLICT", 4.0), (lv, "SQ_LDS_BANK_CONFLICT", 0.0),
                 (sp, "TCC_HIT_sum", 7.0)])
    profsum.counters_main(str(db), str(tmp_path / "out"), "w", "cmd")
    lines = (tmp_path / "out" / "counters_w.txt").read_text().splitlines()
    assert lines[0].startswith("# rocprofv3 --pmc SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT TCC_HIT_sum")
    body = {ln.split()[0]: ln.split()[1:] for ln in lines[2:]}
    # dispatches, then the means in counter-name order; absent counters read 0
    assert body["k_level"] == ["2", "20.0", "2.0", "0.0"]
    assert body["k_support"] == ["1", "0.0", "0.0", "7.0"]


def test_traffic_scaled_by_copy_calibration(tmp_path):
    """A kernel's bytes per launch are its FETCH_SIZE and WRITE_SIZE means
    (KiB) scaled by what the same counters read for the 256 MiB copy."""
    copy_kib = profsum.COPY_BYTES / 1024
    lv = "hotruss::k_level<1024u, 2048u>(hotruss::Dev const*, unsigned int)"
    init = "hotruss::k_init_ctl(hotruss::Dev)"
    trace = tmp_path / "trace.db"
    c = sqlite3.connect(trace)
    c.execute("create table kernels (name text, start integer, end integer)")
    c.executemany("insert into kernels values (?, ?, ?)", [(lv, 0, 2000), (lv, 0, 4000)])
    c.commit()
    c.close()
    fetch, write = tmp_path / "fetch.db", tmp_path / "write.db"
    # the copy reads about half its bytes on FETCH_SIZE (as on the GPU: a
    # little more than half) and all of them on WRITE_SIZE
    fcopy = copy_kib / 2 * 1.0001
    sf = copy_kib / fcopy
    _pmc_db(fetch, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", fcopy),
                    (lv, "FETCH_SIZE", 100.0), (lv, "FETCH_SIZE", 300.0),
                    (init, "FETCH_SIZE", 1.0)])
    _pmc_db(write, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", copy_kib),
                    (lv, "WRITE_SIZE", 50.0), (lv, "WRITE_SIZE", 50.0),
                    (init, "WRITE_SIZE", 0.0)])
    out = tmp_path / "out"
    profsum.main(str(trace), str(fetch), str(write), str(out), "w", "cmd")
    rec = json.loads((out / "traffic_k_level_w.txt").read_text())
    assert rec["launches"] == 2
    assert abs(rec["fetch_scale"] - sf) < 1e-12 and rec["write_scale"] == 1.0
    assert abs(rec["bytes_per_launch"] - (200.0 * sf + 50.0) * 1024) < 1e-6
    whole = json.loads((out / "traffic_whole_w.txt").read_text())
    assert whole["decompositions"] == 1
    # every library kernel (k_ prefix) of the run: k_level twice, k_init_ctl once
    assert abs(whole["bytes_per_decomposition"] - ((400.0 + 1.0) * sf + 100.0) * 1024) < 1e-6
    kt = (out / "kernels_w.txt").read_text().splitlines()
    assert kt[2].split()[:2] == ["k_level", "2"]
