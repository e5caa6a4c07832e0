"""The host-side FIR checks of paper_2407_03323_amd.stability against closed forms."""
import numpy as np

import workloads as wl
from paper_2407_03323_amd import stability as st


def test_binomial_filter_magnitude_is_a_power_of_sine():
    """delta/2^16 (1 - e^{-j theta})^16 has magnitude delta sin^16(theta/2) (eq:FIRmagnitude)."""
    th = np.linspace(0.0, np.pi, 97)
    got = st.fir_magnitude(wl.binomial_highpass(17, 0.01), th)
    assert np.allclose(got, 0.01 * np.sin(th / 2) ** 16, rtol=0, atol=1e-16)


def test_paper_fir2_magnitude_and_report():
    th = np.linspace(0.0, np.pi, 97)
    assert np.allclose(st.fir_magnitude([0.05, -0.05], th), 0.1 * np.abs(np.sin(th / 2)), atol=1e-16)
    r = st.fir_report([0.05, -0.05])
    assert abs(r["delta"] - 0.1) < 1e-15 and r["linear_phase"] and r["group_delay_steps"] == 0.5


def test_report_of_the_workload_filter():
    r = st.fir_report(wl.binomial_highpass(17, wl.FIR17_DELTA))
    assert abs(r["delta"] - wl.FIR17_DELTA) < 1e-15           # eq:RegReq1
    assert r["group_delay_steps"] == 8.0
    assert r["max_magnitude_below_0.9pi"] < wl.FIR17_DELTA
