"""The oracle's feedback and CR-Hall arithmetic, coupled to a minimal 1D gas
model, against the linear growth of the Bell instability (App. B.2): growth
rate and phase speed of the box mode from the dispersion relation with the
CR-Hall term (App. C).  The paper's own runs agree within 2 %; the TSC
gather and deposit at 32 cells per wavelength account for about 1 % here."""
import pytest

from bell_harness import BellSetup, OracleBackend, dispersion, measured_rates, run

TOL = 0.02


@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
def test_bell_growth_without_hall(eps):
    st = BellSetup(eps=eps)
    ts, amps = run(st, OracleBackend(st), t_end=0.8, dt=st.dt_max)
    growth, omega_r = measured_rates(ts, amps, t0=0.1)
    g_exact, vph_exact = dispersion(st)
    # without the Hall term the closed form of App. B.2 is exact
    assert abs(g_exact / st.growth - 1.0) < 1e-9 and abs(vph_exact - st.phase_speed) < 1e-9
    assert abs(growth / g_exact - 1.0) < TOL, (growth, g_exact)
    assert abs(omega_r / st.km / vph_exact - 1.0) < TOL, (omega_r / st.km, vph_exact)


@pytest.mark.parametrize("lam,t_end", [(0.5, 0.4), (2.0, 0.4), (5.0, 0.25)])
def test_bell_growth_with_hall(lam, t_end):
    st = BellSetup(eps=0.01, hall_lambda=lam)
    ts, amps = run(st, OracleBackend(st), t_end=t_end, dt=st.dt_max)
    growth, omega_r = measured_rates(ts, amps, t0=0.05)
    g_exact, vph_exact = dispersion(st)
    assert abs(growth / g_exact - 1.0) < TOL, (growth, g_exact)
    assert abs(omega_r / st.km / vph_exact - 1.0) < TOL, (omega_r / st.km, vph_exact)
