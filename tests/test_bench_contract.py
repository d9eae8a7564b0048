"""The benchmark's contract, on the CPU (no GPU is touched): more than one
GPU is refused with a message, the stored HBM counter summary was taken on
the fused kernels as they are (their source hash), and the oracle leg runs."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr and "--gpus 4" in r.stderr
    assert r.stdout == ""


def test_counter_summary_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.PMC_SUMMARY) as f:
        pm = json.load(f)
    assert pm["kernel_sha256_16"] == bench.kernel_hash()
    assert pm["hbm_bytes_per_launch"] > 0



def test_cpu_baseline_leg_on_a_small_field():
    """The oracle leg of the benchmark (whole steps with every OpenMP thread,
    then one step on one thread) on a 64^2 field of the same mixture: the
    fields the bench line reports are there and positive."""
    sys.path.insert(0, ROOT)
    import bench
    r = bench.cpu_baseline(64, budget_s=0.2, gpu_check=False)
    assert r["kind"] == "oracle" and r["unit"] == "CSU/s"
    assert r["value"] > 0 and r["one_thread"]["value"] > 0
    assert r["cores"] >= 1 and "64x64" in r["sample"]


def _db(tmp_path, name, schema, rows):
    import sqlite3
    path = str(tmp_path / name)
    db = sqlite3.connect(path)
    db.execute(schema)
    table = schema.split()[2]
    marks = ",".join("?" * len(rows[0]))
    db.executemany("insert into %s values (%s)" % (table, marks), rows)
    db.commit()
    db.close()
    return path


def test_profile_summaries_read_rocprofv3_databases(tmp_path, capsys):
    """The summaries that write profiles/ (kernel trace, roctx ranges, SQ
    counters) on small databases in rocprofv3's table layout, with known
    answers: the timed window is the `steps` dispatches before the last
    `steady` ones, ranges are grouped by their roctx message, counters are
    medians per dispatch of the fused kernel."""
    sys.path.insert(0, ROOT)
    import bench
    k = "void (anonymous namespace)::k_fused_d2q9_ws<10, double>(FusedItem const*)"
    # 3 tuning launches of 900 ns, 2 timed of 400 ns, 3 steady of 300 ns
    durs = [900, 900, 900, 400, 400, 300, 300, 300]
    rows, t = [], 0
    for d in durs:
        rows.append((k, t, t + d * 1000))
        t += d * 1000 + 10
    rows.append(("void k_diag_final(double const*)", t, t + 5000))
    trace = _db(tmp_path, "trace.db", "create table kernels (name text, start int, end int)", rows)
    bench.trace_summary(trace, 2, 3)
    out = capsys.readouterr().out
    line = [l for l in out.splitlines() if "k_fused_d2q9_ws" in l][0].split("|")
    assert [c.strip() for c in line[2:9]] == ["8", "550.0", "2", "400.0", "400.0", "400.0", "300.0"]
    assert "| `k_diag_final` | 1 | 5.0 | | | | | |" in out

    regions = [(1000, 3001000, '{"message":"fuglbm_step_n"}', "MARKER_CORE_RANGE_API"),
               (4000000, 5000000, '{"message":"fuglbm_step_n"}', "MARKER_CORE_RANGE_API"),
               (0, 2000000, '{"message":"fuglbm_init_fields"}', "MARKER_CORE_RANGE_API")]
    mk = _db(tmp_path, "mk.db", "create table regions (start int, end int, extdata text, category text)",
             regions)
    bench.marker_summary(mk)
    out = capsys.readouterr().out
    assert "| `fuglbm_step_n` | 2 | 4.00 | 2.000 | 3.000 |" in out
    assert "| `fuglbm_init_fields` | 1 | 2.00 | 2.000 | 2.000 |" in out

    cc = [(k, "SQ_WAVE_CYCLES", v) for v in (1000, 1200, 1100)] + \
         [(k, "SQ_WAIT_ANY", v) for v in (500, 600, 550)] + \
         [("void k_other(int)", "SQ_WAVE_CYCLES", 9)]
    sq = _db(tmp_path, "sq.db",
             "create table counters_collection (kernel_name text, counter_name text, value real)", cc)
    bench.sq_summary([sq])
    out = capsys.readouterr().out
    assert "| SQ_WAVE_CYCLES | 1100 |" in out
    assert "| SQ_WAIT_ANY / SQ_WAVE_CYCLES | 0.500 |" in out
