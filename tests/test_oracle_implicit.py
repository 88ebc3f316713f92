"""Pins of the oracle's linearly implicit Euler step for the 0-D
constant-pressure reactor ((I - dt Jf) dx = dt f(x), the stiff integration
Sec. 4 calls for), against facts that do not use its own formula: the closed
form of backward Euler for a first-order isothermal reaction, conservation of
total mass fraction and of elements, an equilibrium state as a fixed point,
agreement with the (separately pinned) explicit step to second order in dt,
and boundedness at step sizes a hundred times past explicit stability."""

import math

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import synth
from tests.test_oracle_pins import _equilibrium_state, _Mech, _nasa

MILD = dict(ln_A_range=(8.0, 16.0), Ea_range=(20000.0, 60000.0))


def _mild():
    return synth.make_mechanism(9, 21, **MILD)


@pytest.mark.parametrize("kdt", [1e-3, 1.0, 250.0])
def test_first_order_reaction_is_backward_euler(kdt):
    # A -> B, irreversible, first order with k = A (beta = 0, E = 0), both
    # species with the same molar mass and the same NASA-7 set: the enthalpy
    # does not change, so T stays put, and dY_A/dt = -k Y_A is linear, for
    # which one linearly implicit step is backward Euler, Y_A / (1 + k dt).
    k = 2.5e4
    m = _Mech([20.0, 20.0], [[1, 0]], [[0, 1]], [math.log(k)], [0.0], [0.0],
              _nasa([3.5, 3.5], [-1200.0, -1200.0]), rev=[0])
    Y = np.array([[0.7], [0.3]])
    dt = kdt / k
    T1, Y1 = oracle.integrate_implicit(m, [1400.0], [2e5], Y, dt, 1, precision="ld")
    assert T1[0] == 1400.0
    np.testing.assert_allclose(Y1[:, 0], [0.7 / (1 + kdt), 0.3 + 0.7 - 0.7 / (1 + kdt)],
                               rtol=1e-13)
    # three steps: (1 + k dt)^-3
    T3, Y3 = oracle.integrate_implicit(m, [1400.0], [2e5], Y, dt, 3, precision="ld")
    assert Y3[0, 0] == pytest.approx(0.7 / (1 + kdt) ** 3, rel=1e-12)


def test_conservation_at_stiff_step_sizes():
    m = _mild()
    T, P, Y = synth.make_states(m, 16, 6, (1000.0, 2500.0), 1.0, 0.5)
    # dt a hundred times the explicit stability limit of this mechanism
    T1, Y1 = oracle.integrate_implicit(m, T, P, Y, 1e-12, 20, precision="ld")
    assert np.all(np.isfinite(T1)) and np.all(np.abs(T1 - T) > 1e-3)
    assert np.abs(Y1.sum(axis=0) - Y.sum(axis=0)).max() < 1e-12
    el0 = m.atoms.T.astype(float) @ (Y / m.W[:, None])
    el1 = m.atoms.T.astype(float) @ (Y1 / m.W[:, None])
    assert np.abs(el1 - el0).max() <= 1e-12 * np.abs(el0).max()


def test_equilibrium_state_is_a_fixed_point():
    m = _mild()
    P, Y = _equilibrium_state(m, 1500.0, [-10.0, -12.0, -11.0])
    T1, Y1 = oracle.integrate_implicit(m, np.array([1500.0]), [P], Y[:, None], 1e-9, 5,
                                       precision="ld")
    assert abs(T1[0] - 1500.0) < 1e-9
    assert np.abs(Y1[:, 0] - Y).max() < 1e-12 * Y.max()


def test_agrees_with_explicit_to_second_order():
    # x_impl - x_expl = O(dt^2): halving dt quarters the difference
    m = _mild()
    T, P, Y = synth.make_states(m, 8, 7, (1000.0, 2500.0), 1.0, 0.5)
    d = []
    for dt in (2e-16, 1e-16):
        Ti, Yi = oracle.integrate_implicit(m, T, P, Y, dt, 1, precision="ld")
        Te, Ye = oracle.integrate_euler(m, T, P, Y, dt, 1, precision="ld")
        d.append(np.abs(Yi - Ye).max())
    assert 3.5 < d[0] / d[1] < 4.5


def test_bounded_where_explicit_diverges():
    m = _mild()
    T, P, Y = synth.make_states(m, 8, 8, (1000.0, 2500.0), 1.0, 0.5)
    dt = 1e-11
    Te, Ye = oracle.integrate_euler(m, T, P, Y, dt, 5)
    assert not (np.all(np.isfinite(Ye)) and np.abs(Ye).max() < 10.0)
    Ti, Yi = oracle.integrate_implicit(m, T, P, Y, dt, 50)
    assert np.all(np.isfinite(Yi)) and np.all(np.isfinite(Ti))
    assert Yi.min() > -1e-3 and Yi.max() < 1.0 + 1e-3
    assert np.all((Ti > 200.0) & (Ti < 6000.0))
