"""Pins of oracle.quanta against the quantization errors printed in Fig. 4."""
import math

import pytest

from oracle import kernels, quanta
from tests import fig4

F = fig4.load()
KAP = kernels.kappa("cubic")
KAPP = kernels.kappa_prime("cubic")
RATIO = quanta.fig4_sigma_ratio("cubic")


@pytest.mark.parametrize("D", [2, 3, 4, 5, 6])
def test_fig4_quantization_error(D):
    tau = quanta.optimal_tau("cubic", D, RATIO, KAP, KAPP)
    assert abs(quanta.Q("cubic", D, tau, RATIO, KAP, KAPP) / F["Q"][D] - 1) < 1e-12


@pytest.mark.parametrize("K,D", sorted(F["C"]))
def test_fig4_combined_error(K, D):
    # sqrt(E^2 + Q^2) with the printed E and this Q must give the printed combined value
    tau = quanta.optimal_tau("cubic", D, RATIO, KAP, KAPP)
    q = quanta.Q("cubic", D, tau, RATIO, KAP, KAPP)
    assert abs(math.hypot(F["E"][(K, D)], q) / F["C"][(K, D)] - 1) < 1e-11


@pytest.mark.parametrize("D", [1, 2, 3, 6])
def test_tau_is_the_minimiser(D):
    tau = quanta.optimal_tau("cubic", D, RATIO, KAP, KAPP)
    q0 = quanta.Q("cubic", D, tau, RATIO, KAP, KAPP)
    for f in (1 - 1e-4, 1 + 1e-4, 0.5, 2.0):
        assert quanta.Q("cubic", D, tau * f, RATIO, KAP, KAPP) >= q0
    # and the derivative of Q^2 vanishes there (relative to its two parts)
    d = quanta.dQ2_dtau("cubic", D, tau, RATIO, KAP, KAPP)
    scale = KAPP * KAPP * tau / (8 * KAP * KAP)
    assert abs(d) < 1e-12 * scale


def test_sigma_is_amax_over_intmax():
    assert quanta.int_max(64) == 2 ** 63 - 1
    assert quanta.sigma_from_amax(2.0 ** 63, 64) == 2.0 ** 63 / float(2 ** 63 - 1)


def test_choose_quanta_scales_with_representatives():
    # tau / h_repr depends only on sigma / phi_repr (Sec. 5.2)
    t1, s1 = quanta.choose_quanta("cubic", 3, 1e5, 0.01, 7.0)
    t2, s2 = quanta.choose_quanta("cubic", 3, 2e5, 0.02, 14.0)
    assert abs(t2 / t1 - 2.0) < 1e-12 and abs(s2 / s1 - 2.0) < 1e-15
