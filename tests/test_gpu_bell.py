"""The Bell-instability check (App. B.2) with the HIP library as the particle
side: the coupled run must follow the oracle's run step for step (the
library's deposits and feedback are bit-identical to the oracle's, and the
gas model is the same), and grow at the rate of the dispersion relation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from bell_harness import (BellSetup, GpuBackend, OracleBackend, dispersion,  # noqa: E402
                          measured_rates, run)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("eps,lam", [(0.1, 0.0), (0.01, 20.0)])
def test_bell_growth_on_the_gpu_follows_the_oracle(eps, lam):
    _need_gpu()
    st = BellSetup(eps=eps, hall_lambda=lam, nx=64)
    g0, _ = dispersion(st)
    ts, a_gpu = run(st, GpuBackend(st), t_end=4.5 / g0, dt=st.dt_max)
    _, a_ora = run(st, OracleBackend(st), t_end=4.5 / g0, dt=st.dt_max)
    assert np.array_equal(a_gpu, a_ora)
    growth, omega_r = measured_rates(ts, a_gpu, t0=2.0 / g0)
    g_exact, vph_exact = dispersion(st)
    assert abs(growth / g_exact - 1.0) < 0.005, (growth, g_exact)
    assert abs(omega_r / st.km / vph_exact - 1.0) < 0.005, (omega_r / st.km, vph_exact)
