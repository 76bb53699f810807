"""Host logic of bench.py that needs no GPU: the fragment count of the compacted products and
the join of a kernel trace with per-step active columns (--step-table)."""

import csv
import json

import pytest

import bench


@pytest.mark.parametrize("nact,R,work", [
    (132, 132, 8.25),    # eight fragments and the narrow ninth (4 active)
    (128, 132, 8.0),
    (129, 132, 8.25),
    (133, 144, 9.0),     # 5 active in the ninth: a full fragment
    (0, 132, 0.0),
    (20, 132, 1.25),
    (264, 264, 17.0),    # two groups: 9 + 8
    (140, 264, 9.0),     # every active position in the first group
    (148, 264, 9.25),    # 4 in the second group
    (36, 40, 2.25),
])
def test_fragment_work(nact, R, work):
    assert bench.fragment_work(nact, R) == work


def test_step_table_joins_trace_and_active_counts(tmp_path):
    # two E-steps of 4 steps each; the table must use the launches after the last k_cg_init
    T, R = 2, 132
    active = {"T": T, "R": R, "active": [
        [[132, 132]] * 4,
        [[132, 132], [132, 128], [128, 128], [0, 20]],
    ]}
    rows, ts = [], 0

    def launch(name, us):
        nonlocal ts
        rows.append({"Kernel_Name": "void " + name + "(double*)", "Start_Timestamp": str(ts),
                     "End_Timestamp": str(ts + int(us * 1e3))})
        ts += int(us * 1e3) + 100

    for e, durs in enumerate(([100, 100, 100, 100], [165, 161, 160, 13])):
        launch("cmtcs::k_cg_init<double, 1024, 4, false>", 5)
        for d in durs:
            launch("cmtcs::k_phi_v_lds<double, 1>", d)
            launch("cmtcs::k_phit_w_lds<double, 1>", 2 * d)
            launch("cmtcs::k_cg_update<double, 1024, 4, false>", 3)
    trace = tmp_path / "kernel_trace.csv"
    with open(trace, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        wr.writeheader()
        wr.writerows(rows)
    act = tmp_path / "active.json"
    act.write_text(json.dumps(active))
    table = bench.step_table(str(trace), str(act)).splitlines()
    body = [[c.strip() for c in ln.strip("|").split("|")] for ln in table[2:]]
    # steps sorted by fragments: 1.25 (last step), 16.0, 16.25 (132 + 128), 16.5
    frags = [float(r[2]) for r in body]
    assert frags == sorted(frags) and frags[0] == 1.25 and frags[-1] == 16.5
    fwd = {float(r[2]): float(r[3]) for r in body}
    assert fwd[1.25] == 13.0 and fwd[16.5] == 165.0 and fwd[16.0] == 160.0
    adj = {float(r[2]): float(r[4]) for r in body}
    assert adj[16.25] == 322.0
