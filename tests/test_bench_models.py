"""The measurement code of bench.py on the CPU: the smoother's byte model counted by
hand on a tiny level, the per-node V-cycle byte figures, the selection of the
finest level's dispatches from a profile, and the copy-kernel scaling of the
traffic counters."""
import numpy as np

import bench


def _level(n):
    # a 5 x 5 grid with inside nodes (1,1), (2,1), (2,2) and ghosts (3,1), (1,2);
    # compact order: inside nodes, then ghosts; grid index i + n*j
    inside = [(1, 1), (2, 1), (2, 2)]
    ghosts = [(3, 1), (1, 2)]
    c2g = np.array([i + n * j for i, j in inside + ghosts])
    return c2g, len(inside), len(ghosts)


def test_smoother_bytes_hand_count():
    n, P = 5, 4
    c2g, ni, ng = _level(n)
    b0, b1 = bench.smoother_bytes(c2g, ni, ng, n, 2, P)
    # colours (i + j) & 1: inside (1,1) 0, (2,1) 1, (2,2) 0; ghosts (3,1) 0, (1,2) 1
    # colour 0 updates 2 inside nodes and reads the corrections of the 2 active nodes of colour 1
    s_c = 2 * P * (ni + ng)
    assert b0 == s_c + 2 * P * 2 + (2 * P + 1) * 2 + 2 * P * 2
    # colour 1 updates 1 inside node, reads the 3 active nodes of colour 0, and
    # snapshots every ghost's correction (index 4 B, value read and written)
    assert b1 == s_c + 2 * P * 3 + (2 * P + 1) * 1 + 2 * P * 1 + ng * (4 + 2 * P)


def test_smoother_bytes_3d_has_no_ghost_snapshot():
    n, P = 5, 8
    c2g = np.array([1 + n * 1 + n * n * 1, 2 + n * 1 + n * n * 1, 3 + n * 1 + n * n * 1])
    b0, b1 = bench.smoother_bytes(c2g, 2, 1, n, 3, P)
    # colours: (1,1,1) 1, (2,1,1) 0, ghost (3,1,1) 1
    assert b0 == 2 * P * 3 + 2 * P * 2 + (2 * P + 1) * 1 + 2 * P * 1
    assert b1 == 2 * P * 3 + 2 * P * 1 + (2 * P + 1) * 1 + 2 * P * 1


def test_fused_sweep_bytes_hand_count():
    n, P = 5, 4
    c2g, ni, ng = _level(n)
    # black (colour 1) active nodes: (2,1) and ghost (1,2); red ghosts: (3,1)
    expect = (2 * P + 1) * (ni + ng) + 2 * P * ni + 2 * P * (2 + 1) + 2 * P * (ni + ng) + ng * (4 + 2 * P)
    assert bench.fused_sweep_bytes(c2g, ni, ng, n, P) == expect


def test_vcycle_bytes_per_node():
    # 63 values per finest node in 2-D, 55 in 3-D; mixed: FP32 values plus the FP64 refinement
    assert bench.vcycle_bytes_per_node(2, False) == 504
    assert bench.vcycle_bytes_per_node(2, True) == 63 * 4 + 70
    assert bench.vcycle_bytes_per_node(3, False) == 440
    assert bench.vcycle_bytes_per_node(3, True) == 55 * 4 + 70


def test_finest_dispatch_selection():
    rows = [dict(Kernel_Name="void lsmg::k_smooth_colour<float, 2>(...)", Grid_Size=str(g)) for g in
            (2709248, 2756608, 1360256, 690944, 2709056)]
    rows.append(dict(Kernel_Name="void lsmg::k_defect<float, 2, 9>(...)", Grid_Size="5465600"))
    sel = bench._finest(rows, "Grid_Size")
    assert sorted(int(r["Grid_Size"]) for r in sel) == [2709056, 2709248, 2756608]


def test_copy_probe_scale(tmp_path):
    # the copy kernel's dispatches of about the probe's size set the scale; small
    # dispatches in the same profile (torch's own fills) are left out
    d = tmp_path / "copy" / "x"
    d.mkdir(parents=True)
    lines = ["Counter_Name,Counter_Value"] + ["FETCH_SIZE,262144"] * 3 + ["FETCH_SIZE,12"]
    (d / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")
    assert bench._pmc_copy(str(tmp_path / "copy"), "FETCH_SIZE", 512) == 2.0


def test_request_workloads_are_the_served_requests():
    # the single-request workloads step requests of the served stream (seed 0) alone,
    # request 10 on its plain (creased) union
    import lsmg_inputs as I
    reqs = {r["id"]: r for r in I.serving_requests(24, seed=0)}
    for name, smooth in (("request22", 0.02), ("request10_creased", 0.0)):
        w = bench.WORKLOADS[name]
        r = reqs[w["id"]]
        assert (w["n"], w["dt"], w["smooth"]) == (r["n"], r["dt"], smooth)
        if w["n"] <= 65:
            phi = bench.levelset(w)
            assert np.array_equal(phi, I.ellipsoids(r["n"], r["centres"], r["semi"], smooth=smooth))
