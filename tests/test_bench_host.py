"""Host-side arithmetic of the benchmark (CPU): the filter's useful-op model,
the pair buckets, the fused kernel's algorithmic bytes, and the summaries of
rocprofv3 counter and kernel-trace CSVs, each on small hand-worked inputs."""
import csv

import numpy as np

import bench


def _host(cand_offsets, read_E, approx):
    return {"cand_offsets": np.asarray(cand_offsets, np.uint64), "read_E": np.asarray(read_E, np.uint16),
            "approx": np.asarray(approx, np.uint16)}


def test_useful_ops_by_hand():
    # read 0: m = 150, E = 7 (15 rows, 3 words), approx 0 and 9 (walks of 1 and 8 steps);
    # read 1: m = 70, E = 3 (7 rows, 2 words), approx 2 (3 steps); read 2 has no candidate
    host = _host([0, 2, 3, 3], [7, 3, 5], [0, 9, 2])
    got = bench.useful_ops(host, [150, 70, 100]).tolist()
    assert got == [270 + 120 * 1, 270 + 120 * 8, 84 + 56 * 3]


def test_pair_buckets_by_hand():
    # E <= 7, <= 15, <= 31, then long pairs by the 64-base blocks of read and window they stage
    host = _host([0, 1, 2, 3, 4, 5, 6], [7, 15, 31, 50, 500, 500], [0] * 6)
    lengths = [150, 300, 250, 1000, 10000, 40000]
    # m = 1000, E = 50: 16 + 1 + 20 + 2 = 39 blocks (<= 96); m = 10000, E = 500: 157 + 1 + 174 + 2 = 334
    # (<= 384); m = 40000, E = 500: 625 + 1 + 643 + 2 = 1271 (general)
    assert bench.pair_bucket(host, lengths).tolist() == [0, 1, 2, 3, 5, 7]
    assert bench.BUCKET_NAMES[5] == "long<=384"


def test_fused_algorithmic_bytes():
    stats = {"fused_bases": 1500, "fused_minimizers": 200, "fused_occ": 30, "fused_window_blocks": 40,
             "fused_cands": 25, "fused_reads": 10}
    assert bench.fused_alg_bytes(stats) == 1500 + 16 * 200 + 8 * 30 + 16 * 40 + 19 * 25 + 11 * 10


def _write_csv(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_counter_summary_adds_rows_of_a_dispatch(tmp_path):
    """Rows of one dispatch (one per hardware block) add up; dispatches are averaged;
    launches of the long-read filter are kept apart by workgroup size."""
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "LDS_Block_Size", "Workgroup_Size"]
    rows = []
    for did, base in ((1, 100.0), (2, 300.0)):
        for part in (0.25, 0.75):
            rows.append(dict(Dispatch_Id=did, Kernel_Name="void mt::k_fused<16, true>(mt::FusedArgs)",
                             Counter_Name="SQ_INSTS_VALU", Counter_Value=base * part, LDS_Block_Size=0,
                             Workgroup_Size=256))
    for did, wg in ((3, 256), (4, 512), (5, 512)):
        rows.append(dict(Dispatch_Id=did, Kernel_Name="mt::k_filter_long(mt::FilterArgs)", Counter_Name="SQ_WAVES",
                         Counter_Value=float(wg), LDS_Block_Size=0, Workgroup_Size=wg))
    p = tmp_path / "c.csv"
    _write_csv(p, fields, rows)
    out = bench.counter_summary([str(p)])
    assert out["void mt::k_fused<16, true>"] == {"SQ_INSTS_VALU": 200.0, "dispatches": 2}
    assert out["mt::k_filter_long [lds 0, wg 256]"] == {"SQ_WAVES": 256.0, "dispatches": 1}
    assert out["mt::k_filter_long [lds 0, wg 512]"] == {"SQ_WAVES": 512.0, "dispatches": 2}


def test_trace_overlap_by_hand(tmp_path):
    """Queue 1 runs [0, 10) and [20, 30), queue 2 runs [5, 25): busy 30 ns, two queues at once
    during [5, 10) and [20, 25), every dispatch overlapping the other queue."""
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Queue_Id"]
    rows = [dict(Kernel_Name="mt::k_fused<16, false>", Start_Timestamp=a, End_Timestamp=b, Queue_Id=q)
            for a, b, q in ((0, 10, 1), (20, 30, 1), (5, 25, 2))]
    rows.append(dict(Kernel_Name="mt::k_reduce", Start_Timestamp=0, End_Timestamp=100, Queue_Id=3))
    p = tmp_path / "t.csv"
    _write_csv(p, fields, rows)
    out = bench.trace_overlap(str(p))
    assert out["dispatches"] == 3 and out["queues"] == 2
    assert out["busy_ns"] == 30 and out["ns_with_two_or_more_queues_running"] == 10
    assert out["dispatches_overlapping_another_queue"] == 3
    assert out["share_of_busy_time_overlapped"] == round(10 / 30, 4)
