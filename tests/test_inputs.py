"""The seeded input generator (no model arithmetic): SplitMix64 and the field recipes."""
import numpy as np

from paper_0807_0602_amd import inputs


def test_splitmix64_published_sequence():
    # First two outputs of SplitMix64 started from state 0: the generator adds the golden
    # gamma before mixing, so outputs k = 1, 2 are splitmix64(0), splitmix64(gamma).
    out = inputs.splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_uniform_range_and_moments():
    Y, X = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    u = inputs.uniform_pm1(7, 0, Y, X)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 3.0) < 0.01
    assert not np.array_equal(u, inputs.uniform_pm1(7, 1, Y, X))


def test_window_regenerates_exactly():
    case = inputs.capillary_roofline(seed=3)
    a_full, b_full = inputs.capillary_small(3).fields()
    # a window of a small case equals the same columns of the full field
    small = inputs.capillary_small(3)
    a_win, b_win = small.fields(40, 90)
    assert np.array_equal(a_win, a_full[:, 40:90]) and np.array_equal(b_win, b_full[:, 40:90])
    # windows wrap around x
    a_wrap, _ = small.fields(190, 210)
    assert np.array_equal(a_wrap[:, :10], a_full[:, 190:]) and np.array_equal(a_wrap[:, 10:], a_full[:, :10])
    assert case.geom.nx == 16384


def test_capillary_layout():
    c = inputs.capillary_small(1)
    a, b = c.fields()
    g = c.geom
    solid = g.solid_mask()
    assert solid.sum() == 2 * (g.x1 - g.x0)
    assert np.all(a[solid] == 0) and np.all(b[solid] == 0)
    fluid = ~solid
    assert np.all(np.abs(a[:, :50][fluid[:, :50]] - 2.0) <= 1e-3)
    assert np.all(np.abs(a[:, 50:][fluid[:, 50:]] - 0.06) <= 1e-3)
    assert np.all(np.abs(b[:, 50:][fluid[:, 50:]] - 2.0) <= 1e-3)


def test_sweep_draws_cover_the_sets():
    d = inputs.sweep_draws(64, seed=0)
    assert len(d) == 64
    Hs = {c.geom.ny - 2 for c in d}
    Ls = {c.geom.x1 - c.geom.x0 for c in d}
    assert Hs <= {20, 40, 80, 160} and Ls <= {512, 1024, 2048, 4096}
    for c in d:
        assert -0.3 <= c.params.gw[0] <= 0.3 and c.params.gw[1] == -c.params.gw[0]
        assert c.geom.nx == 3 * (c.geom.x1 - c.geom.x0) // 2


def test_rough_mask_geometry():
    case = inputs.capillary_rough(seed=1)
    g = case.geom
    m = g.solid_mask()
    rows = inputs.Geometry(g.nx, g.ny, g.x0, g.x1).solid_mask()
    assert np.all(m[rows])                                  # contains the wall rows
    assert not m[:, :g.x0].any() and not m[:, g.x1:].any()   # reservoirs stay free
    assert m[6:10, 96:100].all()                             # the post
    assert not m[g.ny // 2 - 1:g.ny // 2 + 1].any()           # centre line free
    assert np.array_equal(m, inputs.capillary_rough(seed=1).geom.solid_mask())
    a, b = case.fields()
    assert np.all(a[m] == 0) and np.all(b[m] == 0) and np.all(a[~m] > 0)
    assert g == inputs.Geometry(g.nx, g.ny, g.x0, g.x1)      # the mask is not part of equality


def test_instability_golden_case_is_the_sweep_channel():
    """The oracle-written golden file describes the channel the sweep recipe draws today."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sweep_instability_H20_L512_r2.json")))
    c = inputs.sweep_draws(64, seed=0)[ref["case"]["index"]]
    g = c.geom
    assert (c.name, g.nx, g.ny, g.x0, g.x1, c.seed) == (ref["case"]["name"], ref["case"]["nx"], ref["case"]["ny"],
                                                      ref["case"]["x0"], ref["case"]["x1"], ref["case"]["noise_seed"])
    assert list(c.params.tau) == ref["case"]["tau"] and list(c.params.gw) == ref["case"]["gw"]


def test_instability_golden_regenerates_from_the_oracle(tmp_path, monkeypatch):
    """The stored instability record is what the oracle-only script writes: rerunning it (to the
    recorded step) reproduces the first unstable observation and every stored front exactly."""
    import importlib.util
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    ref = json.load(open(os.path.join(here, "sweep_instability_H20_L512_r2.json")))
    spec = importlib.util.spec_from_file_location("make_sweep_instability",
                                                  os.path.join(here, "make_sweep_instability.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(mod, "HERE", str(tmp_path))
    mod.main()
    new = json.load(open(tmp_path / "sweep_instability_H20_L512_r2.json"))
    assert new["first_unstable_t"] == ref["first_unstable_t"]
    assert new["z_every_1000"] == ref["z_every_1000"]


def test_density_ratio_golden_regenerates_from_the_oracle(tmp_path, monkeypatch):
    """The stored density-ratio drop record is what the oracle-only script writes (its smallest
    drop, rerun here: the same numbers to the last digit)."""
    import importlib.util
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    ref = json.load(open(os.path.join(here, "density_ratio_droplets.json")))
    spec = importlib.util.spec_from_file_location("make_density_ratio_droplets",
                                                  os.path.join(here, "make_density_ratio_droplets.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(mod, "HERE", str(tmp_path))
    monkeypatch.setattr(mod, "RADII", (10,))
    mod.main()
    new = json.load(open(tmp_path / "density_ratio_droplets.json"))
    assert new["drops"][0] == ref["drops"][0]
