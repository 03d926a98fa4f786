"""Host logic of the variance harness (CPU): the relative efficiency of
Sec. 7, the signal part per operator (Table 2) and the averaging over
configurations and operator groups."""
import numpy as np

from paper_1903_06986_amd import variance as Vh


def test_relative_efficiency_definition():
    # RE = (1/dy^2 - 1) x 100: equal error bars give 0, half the error bar
    # (a quarter of the variance) gives 300
    assert Vh.relative_efficiency(1.0, 1.0) == 0.0
    assert abs(Vh.relative_efficiency(0.5, 1.0) - 300.0) < 1e-12
    assert abs(Vh.relative_efficiency(2.0, 1.0) + 75.0) < 1e-12
    np.testing.assert_allclose(Vh.relative_efficiency([0.1, 1 / 3], [1.0, 1.0]), [9900.0, 800.0])


def test_signal_parts():
    assert Vh.signal_part(0) == 0
    assert all(Vh.signal_part(c) == 1 for c in range(1, 9))


def test_summarize_averages_and_groups():
    thetas = (0, 1, 2, 5)
    q_list = (0, 4)
    c1 = {"NS": np.array([4.0, 2.0, 2.0, 8.0]), "PS": np.array([2.0, 1.0, 1.0, 4.0]),
          "POLY": np.array([2.0, 1.0, 1.0, 4.0])}
    c2 = {k: 3 * v for k, v in c1.items()}
    for c in (c1, c2):
        c[("ES", 0)], c[("HFES", 0)], c[("HFPS", 0)], c[("HFPOLY", 0)] = c["NS"], c["NS"], c["PS"], c["POLY"]
        c[("ES", 4)] = c["NS"] * 2
        c[("HFES", 4)] = c["NS"] / 2
        c[("HFPS", 4)] = c["PS"] / 2
        c[("HFPOLY", 4)] = c["PS"] / 4
    s = Vh.summarize([c1, c2], thetas, q_list)
    assert s["configs"] == 2
    # mean over configurations = 2 x c1; groups: scalar (0), local (1, 2), point-split (5)
    assert s["error"]["NS"] == {"scalar": 8.0, "local_vector": 4.0, "point_split": 16.0}
    assert s["error_vs_Q"]["HFES"]["4"]["scalar"] == 4.0
    # HFES at Q = 4 halves the NS error bar: RE vs NS = 300; HFPOLY = PS / 4 -> RE vs PS = 1500
    assert abs(s["RE_at_Qmax"]["NS"]["HFES"]["local_vector"] - 300.0) < 1e-9
    assert abs(s["RE_at_Qmax"]["PS"]["HFPOLY"]["point_split"] - 1500.0) < 1e-9
    assert abs(s["RE_at_Qmax"]["PS"]["POLY"]["scalar"]) < 1e-12
    # ES doubling the NS error bar: RE vs NS = -75
    assert abs(s["RE_at_Qmax"]["NS"]["ES"]["scalar"] + 75.0) < 1e-9
