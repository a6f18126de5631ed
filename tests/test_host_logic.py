"""Host-side logic without a GPU: surrogate features and dataset masking, trajectory files, the
counter summary of bench.py."""
import csv
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_0807_0602_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_features_and_dataset_masking(tmp_path):
    from paper_0807_0602_amd import surrogate as S
    cases = S.draw_cases(3, seed=4, steps=500, every=100)
    for c in cases:
        H = c.geom.ny - 2
        L = c.geom.x1 - c.geom.x0
        assert 20 <= H <= 160 and 512 <= L <= 4096 and L % 4 == 0 and -0.3 <= c.params.gw[0] <= 0.3
        assert tuple(c.params.tau) in inputs.TAU_FOR_RATIO.values()
    f = S.features(cases[0], np.array([100.0, 1000.0]), with_length=True)
    c0 = cases[0]
    np.testing.assert_allclose(f[:, 0], c0.params.gw[0], rtol=1e-6)
    np.testing.assert_allclose(f[:, 1], math.log(c0.params.tau[1] / c0.params.tau[0]), rtol=1e-6)
    np.testing.assert_allclose(f[:, 2], c0.geom.ny - 2)
    np.testing.assert_allclose(f[:, 3], np.log([100.0, 1000.0]), rtol=1e-6)
    np.testing.assert_allclose(f[:, 4], math.log(c0.geom.x1 - c0.geom.x0), rtol=1e-6)
    # trajectories: t, z, p, flags, unstable-so-far
    ns = 6
    traj = np.zeros((3, ns, 5))
    traj[:, :, 0] = np.arange(ns) * 100
    traj[:, :, 1] = 2.0
    traj[:, :, 2] = 3.0
    traj[1, 3, 1] = np.nan            # missing front: dropped
    traj[2, 4:, 4] = 1.0              # unstable from sample 4 on: dropped
    traj[0, 2, 3] = 2.0               # flag bit 1 alone does not drop (the unstable column does)
    traj[1, 5, 3] = 1.0               # reservoir drained at sample 5: dropped from there on
    X, T, w, k = S.dataset(cases, traj)
    assert X.shape == (3 * ns, 4) and T.shape == (3 * ns, 2)
    keep = k.reshape(3, ns)
    assert not keep[:, 0].any()       # t = 0 < t_min
    assert keep[0, 1:].all() and not keep[1, 3] and keep[1, 4] and not keep[1, 5]
    assert not keep[2, 4:].any()
    traj[1, 5, 3] = 0.0
    traj[1, 4, 3] = 3.0               # both bits at sample 4: dropped from sample 4 on
    keep = S.dataset(cases, traj)[3].reshape(3, ns)
    assert keep[1, 2] and not keep[1, 4:].any()
    traj[1, 4, 3] = 0.0
    # a precursor faster than one node per step is the draining reservoir: dropped from there on;
    # 90 nodes in 100 steps stays, and a missing precursor in between is skipped, not a jump
    traj[0, 2, 2] = 93.0
    traj[0, 3, 2] = np.nan
    traj[0, 4, 2] = 183.0
    traj[0, 5, 2] = 273.0
    keep = S.dataset(cases, traj)[3].reshape(3, ns)
    assert keep[0, 1] and keep[0, 2] and not keep[0, 3] and keep[0, 4] and keep[0, 5]
    traj[0, 5, 2] = 500.0
    keep = S.dataset(cases, traj)[3].reshape(3, ns)
    assert keep[0, 4] and not keep[0, 5]
    assert not S.precursor_jumped(traj[0, :, 0], traj[0, :, 2])[:5].any()
    traj[0, 2:, 2] = 3.0
    H = np.repeat([c.geom.ny - 2 for c in cases], ns)
    np.testing.assert_allclose(w, H * H)
    np.testing.assert_allclose(T[k, 0], (2.0 / H)[k], rtol=1e-6)
    # file round trip
    p = str(tmp_path / "t.npz")
    S.save_trajectories(p, cases, traj, 500, 100)
    c2, t2 = S.load_trajectories(p)
    for a, b in zip(cases, c2):
        assert a.geom == b.geom and a.params == b.params and a.seed == b.seed
    assert np.array_equal(np.isnan(t2), np.isnan(traj))
    np.testing.assert_allclose(np.nan_to_num(t2), np.nan_to_num(traj), rtol=1e-6)


def _counter_csv(path, kernel, counter, values):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for v in values:
            w.writerow({"Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": v})


def test_bench_counter_summary(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    files = []
    for name, kern, ctr, vals in [("f", "k_step_fused<256>", "FETCH_SIZE", [600000, 600000]),
                                  ("w", "k_step_fused<256>", "WRITE_SIZE", [1179000]),
                                  ("fc", "__amd_rocclr_copyBuffer", "FETCH_SIZE", [524288]),
                                  ("wc", "__amd_rocclr_copyBuffer", "WRITE_SIZE", [1048576])]:
        p = str(tmp_path / f"{name}.csv")
        _counter_csv(p, kern, ctr, vals)
        files.append(p)

    class A:
        summarize_counters = files
        workload = "roofline"
        tile = bench.parse_tile([256, 16, 1])
    assert A.tile == (256, 16, 1, 1)
    assert bench.summarize_counters(A) == 0
    t = json.load(open(tmp_path / "traffic.json"))
    # keyed by the kernels together with the runtime that plans their tiles
    assert t["kernel_sha256_16"] == bench.kernel_hash() != bench.kernel_hash(bench.KERNEL_SRC)
    e = t["schedules"][0]
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["read_bytes_per_launch"] == 600000 * 2 * 1024 and e["write_bytes_per_launch"] == 1179000 * 1024
    cells = 16384 * 1024
    assert bench.measured_traffic(cells, {"bx": 256, "cy": 16, "order": 1}) == e["bytes_per_launch"]
    assert bench.measured_traffic(cells, {"bx": 256, "cy": 16, "order": 1, "fuse": 1}) == e["bytes_per_launch"]
    assert bench.measured_traffic(cells, {"bx": 256, "cy": 16, "order": 1, "fuse": 2}) is None
    assert bench.measured_traffic(cells, {"bx": 256, "cy": 8, "order": 1}) is None
    # a two-step schedule reads the counters of k_step_fused2 only
    files2 = []
    for name, kern, ctr, vals in [("f2", "k_step_fused2<256, false>", "FETCH_SIZE", [900000]),
                                  ("w2", "k_step_fused2<256, false>", "WRITE_SIZE", [1179000])]:
        p = str(tmp_path / f"{name}.csv")
        _counter_csv(p, kern, ctr, vals)
        files2.append(p)

    class B:
        summarize_counters = files2 + files[2:]
        workload = "roofline"
        tile = bench.parse_tile([256, 16, 1, 2])
    assert bench.summarize_counters(B) == 0
    t = json.load(open(tmp_path / "traffic.json"))
    assert len(t["schedules"]) == 2
    assert bench.measured_traffic(cells, {"bx": 256, "cy": 16, "order": 1, "fuse": 2}) == (900000 * 2 + 1179000) * 1024
    # the two-kernel variant: one k_density and one k_collide launch per step, summed
    files4 = []
    for name, kern, ctr, vals in [("f4", "k_density(scf::Chan const*)", "FETCH_SIZE", [700000]),
                                  ("f4", None, None, None),
                                  ("w4", "k_collide(scf::Chan const*)", "WRITE_SIZE", [1179000])]:
        if kern is None:
            continue
        p = str(tmp_path / f"{name}.csv")
        _counter_csv(p, kern, ctr, vals)
        files4.append(p)
    with open(files4[0], "a", newline="") as f:
        csv.writer(f).writerow(["k_collide(scf::Chan const*)", "FETCH_SIZE", 900000])
    with open(files4[1], "a", newline="") as f:
        csv.writer(f).writerow(["k_density(scf::Chan const*)", "WRITE_SIZE", 131000])

    class T:
        summarize_counters = files4 + files[2:]
        workload = "roofline"
        variant = "two_kernel"
        tile = None
    assert bench.summarize_counters(T) == 0
    assert bench.measured_traffic(cells, {"variant": "two_kernel"}, keys=("variant",)) == \
        ((700000 + 900000) * 2 + 1179000 + 131000) * 1024
    assert bench.measured_traffic(cells, {"bx": 256, "cy": 16, "order": 1, "fuse": 2}) == (900000 * 2 + 1179000) * 1024
    # the 3-D duct: k3_fused counters into their own file, keyed by the rows per tile
    monkeypatch.setattr(bench, "TRAFFIC3_FILE", str(tmp_path / "traffic3.json"))
    files3 = []
    for name, kern, ctr, vals in [("f3", "k3_fused<4>", "FETCH_SIZE", [2900000]),
                                  ("w3", "k3_fused<4>", "WRITE_SIZE", [2490000]),
                                  ("fo", "k3_density", "FETCH_SIZE", [1])]:
        p = str(tmp_path / f"{name}.csv")
        _counter_csv(p, kern, ctr, vals)
        files3.append(p)

    class D:
        summarize_counters = files3[:2] + files[2:]
        workload = "duct3d"
        cy3 = 16
        tile = None
    assert bench.summarize_counters(D) == 0
    t3 = json.load(open(tmp_path / "traffic3.json"))
    assert t3["cells"] == 512 * 182 * 182 and t3["schedules"][0]["schedule"] == {"cy": 16}
    assert bench.measured_traffic(512 * 182 * 182, {"cy": 16}, bench.TRAFFIC3_FILE, bench.KERNEL3_SRC,
                                  ("cy",)) == (2900000 * 2 + 2490000) * 1024
    assert bench.measured_traffic(512 * 182 * 182, {"cy": 8}, bench.TRAFFIC3_FILE, bench.KERNEL3_SRC,
                                  ("cy",)) is None


def test_wetting_circle_fit_and_contour():
    """Host analysis of the sessile-droplet estimator on a synthetic circular cap: the contour
    points of a signed-distance field and the algebraic circle fit recover the cap's angle."""
    from paper_0807_0602_amd import wetting as W
    ny, nx = 60, 120
    xc, yc, R = 59.5, -6.0, 30.0            # centre below the wall plane y = 0.5: angle < 90
    Y, X = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    phi = R - np.hypot(X - xc, Y - yc)
    phi[0, :] = -1.0
    pts = W._contour_points(phi, 5)
    cx, cy, cr = W.fit_circle(pts)
    assert abs(cx - xc) < 0.05 and abs(cy - yc) < 0.05 and abs(cr - R) < 0.05
    assert abs((0.5 - cy) / cr - (0.5 - yc) / R) < 2e-3
    # exact circle through three points
    t = np.array([0.3, 1.7, 2.9])
    p3 = np.stack([2 + 5 * np.cos(t), -1 + 5 * np.sin(t)], axis=1)
    assert np.allclose(W.fit_circle(p3), (2.0, -1.0, 5.0))


def test_wetting_match_and_pressure():
    from oracle import physics
    from paper_0807_0602_amd import wetting as W
    assert W.match_coupling([0.1, 0.2, 0.3], [0.1, 0.2, 0.35], 0.275) == pytest.approx(0.25)
    with pytest.raises(ValueError):
        W.match_coupling([0.1, 0.2], [0.1, 0.2], 0.5)
    rng = np.random.default_rng(3)
    a, b = rng.uniform(0, 2, 50), rng.uniform(0, 2, 50)
    assert np.allclose(W.eos_pressure(a, b, 0.9), physics.pressure(a, b, 0.9))


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on exactly one GPU and says so when asked for more (before touching one)."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_meniscus_radius_of_a_synthetic_arc():
    """A concave meniscus of radius 45 spanning H = 60 rows (centre of curvature on the gas side):
    the circle fit recovers R and the apparent cos(theta) = H / (2 R)."""
    from paper_0807_0602_amd import wetting
    H, R, xc = 60, 45.0, 160.0
    ny, nx = H + 2, 260
    yc = (ny - 1) / 2.0
    Y, X = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    d = np.hypot(X - xc, Y - yc)
    phi = np.where(X < xc, np.tanh((d - R) / 2.0), -1.0)   # liquid (phi > 0) left of the arc
    nA, nB = 1.0 + 0.5 * phi, 1.0 - 0.5 * phi
    m = wetting.meniscus_radius(nA, nB, x_front=xc - R, H=H, skip=6)
    assert m["npts"] > 30
    assert abs(m["R"] - R) < 0.02 * R
    assert abs(m["cos"] - H / (2 * R)) < 0.02
