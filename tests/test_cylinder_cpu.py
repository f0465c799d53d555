"""Host post-processing of the cylinder case on synthetic data: the shedding
frequency estimator and the wake-axis interpolation."""
import numpy as np

from paper_2007_07347_amd import cylinder


def test_dominant_frequency_recovers_a_sinusoid():
    rng = np.random.default_rng(0)
    for f0 in (0.0137, 0.01523, 0.0166):
        t = 600.0 + 0.37 * np.arange(1400)
        x = 0.3 * np.sin(2 * np.pi * f0 * t + 0.4) + 0.01 * np.sin(2 * np.pi * 2 * f0 * t) + 1e-3 * rng.standard_normal(len(t))
        assert abs(cylinder.dominant_frequency(t, x) - f0) <= 2e-3 * f0


def test_axis_velocity_is_exact_for_linear_fields():
    rng = np.random.default_rng(1)
    cx, cy = rng.uniform(0.5, 10, 4000), rng.uniform(-1, 1, 4000)
    u = 0.1 * (cx - 3.0) + 0.02 * cy
    xs = np.linspace(0.6, 9.0, 50)
    assert np.abs(cylinder.axis_velocity(cx, cy, u, xs) - 0.1 * (xs - 3.0)).max() <= 1e-12


def test_golden_paper_cylinder_values():
    """The transcribed paper values are consistent with what the paper says
    of them: drag falls and the bubble grows with Re over the steady range, and
    the Strouhal numbers follow the experimental fit it cites
    (St = -3.3265/Re + 0.1816 + 1.6e-4 Re) to within 2 %."""
    from conftest import read_cylinder_golden
    g = read_cylinder_golden()
    assert sorted(g["steady"]) == [10, 20, 40] and sorted(g["unsteady"]) == [60, 80, 100]
    cd = [g["steady"][r][0] for r in (10, 20, 40)]
    lr = [g["steady"][r][1] for r in (10, 20, 40)]
    assert cd[0] > cd[1] > cd[2] and lr[0] < lr[1] < lr[2]
    for re_, (cd_u, lr_u, st) in g["unsteady"].items():
        fit = -3.3265 / re_ + 0.1816 + 1.6e-4 * re_
        assert abs(st - fit) <= 0.02 * fit, (re_, st, fit)
        assert cd_u < cd[2]
