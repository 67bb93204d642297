"""Host side of the robustness and funnelling studies: the k-nearest-neighbour density
concentration ratio against closed forms and invariances, the success rate, and the
perturbation generators (level 0 reproduces the design; draws are seeded)."""
import numpy as np
import pytest

from paper_2509_15180_amd import robustness as Rb
from paper_2509_15180_amd import workloads as W


def test_ratio_of_evenly_spaced_points_is_one():
    a = 2 * np.pi * np.arange(40) / 40
    pts = np.stack([np.cos(a), np.sin(a)], 1)
    assert Rb.knn_density_ratio(pts, k=4) == pytest.approx(1.0, abs=1e-12)


def test_ratio_on_a_line_closed_form():
    # points 0..5 on a line, k = 2: the two ends have r_2 = 1.5, the others 1, so
    # p_end = 2 / (pi 2.25), p_in = 2 / pi; the top decile holds the four inner points
    pts = np.stack([np.arange(6.0), np.zeros(6)], 1)
    assert Rb.knn_density_ratio(pts, k=2) == pytest.approx(108.0 / 88.0, rel=1e-12)


def test_ratio_invariant_under_similarity():
    rng = np.random.default_rng(1)
    pts = rng.normal(size=(60, 2))
    base = Rb.knn_density_ratio(pts)
    c, s = np.cos(0.7), np.sin(0.7)
    moved = 3.5 * pts @ np.array([[c, -s], [s, c]]).T + np.array([10.0, -4.0])
    assert Rb.knn_density_ratio(moved) == pytest.approx(base, rel=1e-9)
    assert base >= 1.0


def test_ratio_of_a_tight_cluster_tends_to_ten():
    # 10 of 100 points in a cluster of width eps, 90 on a wide ring: the top decile is
    # the cluster, so the ratio is 100 P_c / (10 P_c + 90 P_r) -> 10 as eps -> 0
    a = 2 * np.pi * np.arange(90) / 90
    ring = 10.0 * np.stack([np.cos(a), np.sin(a)], 1)
    prev = 0.0
    for eps in (1e-1, 1e-3, 1e-5):
        b = 2 * np.pi * np.arange(10) / 10
        cl = eps * np.stack([np.cos(b), np.sin(b)], 1)
        r = Rb.knn_density_ratio(np.concatenate([cl, ring]), k=3)
        assert prev <= r <= 10.0
        prev = r
    assert prev > 9.99


def test_success_rate():
    tips = np.array([[0.0, 0.0], [0.1, 0.0], [0.3, 0.4]])
    assert Rb.success_rate(tips, (0.0, 0.0), 0.1) == pytest.approx(2 / 3)
    assert Rb.success_rate(tips, (0.3, 0.4), 0.01) == pytest.approx(1 / 3)


def test_perturbation_level_zero_is_the_design_and_draws_are_seeded():
    w = W.config2(3)
    for i in range(3):
        p = W.perturbed(w, i, 4)
        base = w.instance(i)
        for t in range(4):
            it = p.instance(t)
            assert np.array_equal(it["obs"], base["obs"]) and np.array_equal(it["spam"], base["spam"])
            assert np.array_equal(it["d"], base["d"])
    a = W.perturbed(w, 1, 5, 0.1, 0.1, tag=3)
    b = W.perturbed(w, 1, 5, 0.1, 0.1, tag=3)
    c = W.perturbed(w, 1, 5, 0.1, 0.1, tag=4)
    assert np.array_equal(a.obs_d, b.obs_d) and np.array_equal(a.spam, b.spam)
    assert not np.array_equal(a.obs_d, c.obs_d)


def test_perturbed_obstacles_stay_clear_of_the_base_and_sizes_positive():
    w = W.config2(2)
    p = W.perturbed(w, 0, 50, sigma_env=0.3, sigma_act=0.3)
    base = w.instance(0)
    l, R, psi = base["d"][0], base["d"][1], base["d"][5]
    for t in range(50):
        it = p.instance(t)
        for kd, (cx, cy, a, b) in zip(it["kind"], it["obs"]):
            assert a > 0 and (b > 0 or kd == W.CIRCLE)
            assert not W._meets_first_link(int(kd), cx, cy, a, b, l, R, psi)
        sp = it["spam"]
        assert np.all(sp[:, 3] >= 0) and np.all(sp[:, 1] > sp[:, 0])
        assert np.all(sp[:, 1] <= base["n"] * l + 1e-15)


def test_start_angles_spread_evenly():
    w = W.config2(1)
    s = W.start_angles(w, 0, 5, 0.4)
    psi = w.inst_d[0, 5]
    assert np.allclose(s.inst_d[:, 5], psi + np.array([-0.2, -0.1, 0.0, 0.1, 0.2]))
