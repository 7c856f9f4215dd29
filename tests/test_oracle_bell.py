"""The oracle's feedback and CR-Hall arithmetic, coupled to a minimal 1D gas
model, against the linear growth of the Bell instability (App. B.2): growth
rate and phase speed of the box mode from the dispersion relation with the
CR-Hall term (App. C), over the paper's range eps = 0.1..0.9 without it and
Lambda = 0.2..20 with it.  The paper's growth rates agree within 0.5 % at 32
cells per wavelength.  Here the particles couple to the gas through a TSC
deposit and a TSC gather, whose transfer function sinc(k dx/2)^6 is 0.990 at
32 cells per wavelength (about -1 % in both rates) and 0.9976 at 64; the
runs use 64 cells, and the rates are fitted once the mode dominates
(2 to 4.5 e-folding times)."""
import pytest

from bell_harness import BellSetup, OracleBackend, dispersion, measured_rates, run

TOL = 0.005
NX = 64


def _rates(st):
    g0, _ = dispersion(st)
    ts, amps = run(st, OracleBackend(st), t_end=4.5 / g0, dt=st.dt_max)
    return measured_rates(ts, amps, t0=2.0 / g0)


@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
def test_bell_growth_without_hall(eps):
    st = BellSetup(eps=eps, nx=NX)
    growth, omega_r = _rates(st)
    g_exact, vph_exact = dispersion(st)
    # without the Hall term the closed form of App. B.2 is exact
    assert abs(g_exact / st.growth - 1.0) < 1e-9 and abs(vph_exact - st.phase_speed) < 1e-9
    assert abs(growth / g_exact - 1.0) < TOL, (growth, g_exact)
    assert abs(omega_r / st.km / vph_exact - 1.0) < TOL, (omega_r / st.km, vph_exact)


@pytest.mark.parametrize("lam", [0.2, 0.5, 2.0, 5.0, 20.0])
def test_bell_growth_with_hall(lam):
    st = BellSetup(eps=0.01, hall_lambda=lam, nx=NX)
    growth, omega_r = _rates(st)
    g_exact, vph_exact = dispersion(st)
    assert abs(growth / g_exact - 1.0) < TOL, (growth, g_exact)
    assert abs(omega_r / st.km / vph_exact - 1.0) < TOL, (omega_r / st.km, vph_exact)


def test_bell_error_at_32_cells_is_the_tsc_transfer_function():
    """Without the Hall term both rates of the box mode scale with the CR
    current the gas sees; at 32 cells per wavelength that current comes
    through a TSC deposit and a TSC gather, so both rates come out low by
    1 - sinc(pi/32)^6 = 0.96 %."""
    import math
    st = BellSetup(eps=0.5, nx=32)
    growth, omega_r = _rates(st)
    g_exact, vph_exact = dispersion(st)
    x = math.pi / 32
    filt = (math.sin(x) / x) ** 6 - 1.0
    assert abs((growth / g_exact - 1.0) - filt) < 0.001, (growth / g_exact - 1.0, filt)
    assert abs((omega_r / st.km / vph_exact - 1.0) - filt) < 0.001
