"""Host tests of the App. D harness (tuning grids, the reached / censored
logic, the optimum per instance and its average, and the a N^alpha + b fit)
on scripted inputs whose answers are known by construction."""
import os

import numpy as np
import pytest

from paper_2501_17267_amd import tuning as tu
from paper_2501_17267_amd import tteps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appd_tuning_grids.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, *vals = line.split()
        out[name] = [float(v) for v in vals]
    return out


def _check_range(values, first, bound, step):
    # first value, increments, and the last value within the bound
    assert values[0] == pytest.approx(first)
    assert np.allclose(np.diff(values), step)
    assert values[-1] <= bound + 1e-9 and values[-1] + step > bound + 1e-9


def test_sa_grid_is_app_d_grid():
    g = _golden()
    bmin, bmax = tu.appd_sa_grid()
    _check_range(bmin, *g["sa_beta_min"])
    _check_range(bmax, *g["sa_beta_max"])
    assert (len(bmin), len(bmax)) == (16, 25)


def test_pt_grid_is_app_d_grid():
    g = _golden()
    bmin, bmax, sweeps, temps = tu.appd_pt_grid()
    _check_range(bmin, *g["pt_beta_min"])
    _check_range(bmax, *g["pt_beta_max"])
    _check_range(sweeps, *g["pt_sweeps"])
    _check_range(temps, *g["pt_temperatures"])
    # 0.1 + 0.2 k stays below 2.8 up to 2.7: 14 values
    assert len(bmin) == 14 and bmin[-1] == pytest.approx(2.7)


def test_alpha_study_sizes_and_targets():
    g = _golden()
    assert list(tu.TARGETS) == g["targets"]
    import inspect
    assert list(inspect.signature(tu.run).parameters["sa_sizes"].default) == g["sa_sizes"]
    assert list(inspect.signature(tu.run).parameters["pt_sizes"].default) == g["pticm_sizes"]


def test_sweep_grid():
    assert tu.sweep_grid(16, 64, 2) == [16, 23, 32, 45, 64]
    g = tu.sweep_grid(1, 40, 4)
    assert g[:8] == [1, 2, 3, 4, 5, 6, 7, 8]        # duplicates from rounding dropped
    assert all(b > a for a, b in zip(g, g[1:])) and g[-1] <= 40
    assert tteps.sweep_grid is tu.sweep_grid


def test_first_reached_and_censoring():
    # three items, scripted mean eps per sweep count: item 0 reaches 5 % at
    # S = 32 and 3 % at 64; item 1 dips below 5 % at 16 and never below 3 %
    # (censored there); item 2 never reaches 5 %
    table = [(16, np.array([0.09, 0.049, 0.2])),
             (32, np.array([0.05, 0.06, 0.2])),
             (64, np.array([0.03, 0.04, 0.1]))]
    r = tu.first_reached(table, (0.03, 0.05))
    assert r[0.05] == [32, 16, None]
    assert r[0.03] == [64, None, None]
    assert tu.first_reached([], (0.01,)) == {0.01: []}


def test_instance_optimum_centroid_of_ties():
    params = [(0.3, 3.0), (0.5, 3.0), (0.3, 5.0), (3.3, 27.0)]
    opt = tu.instance_optimum([40, 32, 32, None], params)
    assert opt["sweeps"] == 32 and opt["tied"] == 2
    assert opt["beta_min"] == pytest.approx(0.4) and opt["beta_max"] == pytest.approx(4.0)
    assert tu.instance_optimum([None, None], params[:2]) is None
    avg = tu.average_optimum([opt, None, {"sweeps": 64, "beta_min": 0.8, "beta_max": 6.0}])
    assert avg["instances"] == 2 and avg["censored"] == 1
    assert avg["beta_min"] == pytest.approx(0.6) and avg["beta_max"] == pytest.approx(5.0)
    assert avg["mean_sweeps"] == pytest.approx(48.0)


def test_pt_optimum_minimises_temperatures_times_sweeps():
    costs = [(2, 0.1, 3.0, 9), (3, 0.5, 4.0, 6), (2, 0.3, 5.0, 9), (4, 0.1, 3.0, 4), (3, 0.1, 3.0, None)]
    o = tu.pt_instance_optimum(costs)
    # cost 16 (T=4, 4 sweeps) is the least; a tie at 18 would not matter
    assert o["T"] == 4 and o["cost"] == 16 and o["sweeps"] == 4
    costs = [(2, 0.1, 3.0, 6), (3, 0.5, 4.0, 4), (2, 0.3, 5.0, 6)]
    o = tu.pt_instance_optimum(costs)
    # cost 12 reached by T=2 twice and T=3 once: T = 2, centroid of its betas
    assert o["T"] == 2 and o["tied"] == 3
    assert o["beta_min"] == pytest.approx(0.2) and o["beta_max"] == pytest.approx(4.0)
    a = tu.pt_average_optimum([o, {"T": 3, "beta_min": 1.0, "beta_max": 6.0}, None,
                               {"T": 3, "beta_min": 0.4, "beta_max": 3.0}])
    assert a["T"] == 3 and a["censored"] == 1 and a["T_votes"] == {"2": 1, "3": 2}
    assert a["beta_min"] == pytest.approx((0.2 + 1.0 + 0.4) / 3)
    assert tu.pt_instance_optimum([(2, 0.1, 3.0, None)]) is None


@pytest.mark.parametrize("a,alpha,b", [(0.5, 1.3, 0.02), (2.0, 0.8, 0.5), (0.01, 2.0, 0.0)])
def test_fit_recovers_known_exponent(a, alpha, b):
    N = np.array([20, 30, 40, 50, 56], np.float64) ** 3
    T = a * (N / N.min()) ** alpha + b
    f = tu.fit_alpha(N, T)
    assert f["alpha"] == pytest.approx(alpha, rel=1e-4)
    assert f["a_at_N0"] == pytest.approx(a, rel=1e-4)
    assert f["b"] == pytest.approx(b, abs=1e-6 + 1e-4 * abs(b))
    assert tu.fit_alpha(N[:2], T[:2]) is None


def test_alpha_table_reads_the_fits():
    res = {"sa_alpha": {"fits": {"0.03": {"plain": {"alpha": 1.4}, "batched": None}}},
           "pticm_alpha": {"fits": {"0.05": {"plain": {"alpha": 1.1}, "batched": {"alpha": 1.2}}}}}
    rows = {r["eps"]: r for r in tu.alpha_table(res)}
    assert rows[0.03]["sa_alpha_plain"] == 1.4 and rows[0.03]["sa_alpha_batched"] is None
    assert rows[0.05]["pticm_alpha_batched"] == 1.2 and rows[0.04]["pticm_alpha_plain"] is None
