"""Post-processing of front time series (front.py), on synthetic series with
known answers: the sampled velocity of a sinusoidal swing, its period and
the crossing count, the band wavelength mean(v) x period, and the
classification of a front as steady, oscillating or transient."""
import numpy as np

from paper_2303_09671_amd.front import front_state, oscillation


def _series(t, v, T):
    return dict(n=np.arange(len(t)), t=t[:, None], z=np.cumsum(v)[:, None], v=v[:, None], T=T[:, None])


def test_sinusoid_period_and_wavelength():
    t = np.arange(0.0, 1000.0, 0.5)
    v = 0.3 + 0.2 * np.sin(2 * np.pi * t / 100.0 + 0.3)
    T = 0.01 * np.cos(2 * np.pi * t / 100.0)
    o = oscillation(_series(t, v, T))
    assert abs(o["period"] - 100.0) < 0.5
    assert o["crossings"] in (9, 10)
    assert abs(o["v_mean"] - 0.3) < 1e-3 and abs(o["v_max"] - 0.5) < 1e-3 and abs(o["v_min"] - 0.1) < 1e-3
    assert abs(o["wavelength"] - 30.0) < 0.2
    assert abs(o["T_max"] - 0.01) < 1e-6 and abs(o["T_min"] + 0.01) < 1e-6


def test_window_start_and_steady_front():
    t = np.arange(0.0, 400.0, 1.0)
    v = np.where(t < 200.0, 0.3 + 0.1 * np.sin(2 * np.pi * t / 40.0), 0.27)
    o = oscillation(_series(t, v, np.zeros_like(t)), t_from=200.0)
    assert o["crossings"] == 0 and np.isnan(o["period"])
    assert o["v_min"] == o["v_max"] == 0.27


def test_front_state():
    t = np.arange(0.0, 3000.0, 10.0)
    V = 0.1
    steady = V * (1.0 + 0.005 * np.sin(2 * np.pi * t / 300.0))
    swing = V * (1.0 + 0.4 * np.sin(2 * np.pi * t / 300.0))
    approach = V * (1.0 - 0.3 * np.exp(-t / 2000.0))  # slow monotone approach
    overshoot = V * (1.0 + 0.2 * np.exp(-t / 800.0))
    ringing = V * (1.0 + 0.2 * np.exp(-t / 500.0) * np.sin(2 * np.pi * t / 300.0))  # damped
    z = np.zeros_like(t)
    assert front_state(_series(t, steady, z), 0, V, t_from=1000.0) == "steady"
    assert front_state(_series(t, swing, z), 0, V, t_from=1000.0) == "oscillating"
    assert front_state(_series(t, approach, z), 0, V, t_from=1000.0) == "transient"
    assert front_state(_series(t, ringing, z), 0, V, t_from=1000.0) == "transient"
    assert front_state(_series(t, overshoot, z), 0, V, t_from=1000.0) == "transient"
    assert front_state(_series(t, overshoot, z), 0, V, t_from=2500.0) == "steady"
