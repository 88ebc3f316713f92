"""Pins of the oracle's 0-D constant-pressure reactor (forward Euler, the
paper's 0-D ignition test, Sec. 3.1), against properties that do not use
its own update formula: one step equals the update built from the
separately pinned source term and temperature source; total mass fraction
and element amounts are conserved; the mixture enthalpy drifts at first
order in dt (halving dt halves the drift over a fixed time); the global
error is first order; an equilibrium state stays put."""

import numpy as np

import oracle
from paper_2008_08483_amd import synth

# a mechanism mild enough for explicit steps of 1e-14 s (the benchmark's
# mechanisms have Jacobian eigenvalues near 1e20 1/s)
MILD = dict(ln_A_range=(8.0, 16.0), Ea_range=(20000.0, 60000.0))


def _mech():
    return synth.make_mechanism(9, 21, **MILD)


def test_one_step_is_the_update_of_the_pinned_rates():
    m = _mech()
    T, P, Y = synth.make_states(m, 32, 5, (1000.0, 2500.0), 1.0, 0.5)
    dt = 1e-14
    T1, Y1 = oracle.integrate_euler(m, T, P, Y, dt, 1, precision="ld")
    om = oracle.source(m, T, P, Y, precision="ld").astype(float)
    omT = oracle.temp_source(m, T, P, Y, precision="ld").astype(float)
    # rho = P W_mix / (Ru T), W_mix = sum(Y) / sum(Y / W) for Y >= 0
    rho = P * Y.sum(axis=0) / (8314.46261815324 * T * (Y / m.W[:, None]).sum(axis=0))
    np.testing.assert_allclose(Y1, Y + dt * m.W[:, None] * om / rho, rtol=1e-13, atol=1e-30)
    np.testing.assert_allclose(T1, T + dt * omT, rtol=1e-15)


def test_conservation_along_a_trajectory():
    m = _mech()
    T, P, Y = synth.make_states(m, 32, 6, (1000.0, 2500.0), 1.0, 0.5)
    T1, Y1 = oracle.integrate_euler(m, T, P, Y, 1e-14, 2000, precision="ld")
    assert np.all(np.abs(T1 - T) > 1e-3)          # the state did move
    assert np.abs(Y1.sum(axis=0) - Y.sum(axis=0)).max() < 1e-13
    el0 = m.atoms.T.astype(float) @ (Y / m.W[:, None])
    el1 = m.atoms.T.astype(float) @ (Y1 / m.W[:, None])
    assert np.abs(el1 - el0).max() <= 1e-13 * np.abs(el0).max()


def _enthalpy(m, T, Y):
    """Mixture enthalpy per unit mass, J/kg: sum_k Y_k H_k(T) / W_k."""
    out = np.zeros(T.shape[0])
    for i in range(T.shape[0]):
        h, _, _ = oracle.thermo(m, T[i], precision="ld")
        out[i] = float((Y[:, i] * h.astype(float) * 8314.46261815324 * T[i] / m.W).sum())
    return out


def test_enthalpy_drift_and_global_error_are_first_order():
    m = _mech()
    T, P, Y = synth.make_states(m, 16, 7, (1000.0, 2500.0), 1.0, 0.5)
    t_end = 2e-11
    h0 = _enthalpy(m, T, Y)
    ref_T, _ = oracle.integrate_euler(m, T, P, Y, t_end / 16000, 16000, precision="ld")
    drift, err = [], []
    for steps in (2000, 4000):
        T1, Y1 = oracle.integrate_euler(m, T, P, Y, t_end / steps, steps, precision="ld")
        drift.append(np.abs(_enthalpy(m, T1, Y1) - h0).max())
        err.append(np.abs(T1 - ref_T).max())
    # halving dt halves the drift (first order); the error against the run
    # with dt/8 then shrinks by (1 - 1/8) / (1/2 - 1/8) = 2.33
    assert 1.7 < drift[0] / drift[1] < 2.3, drift
    assert 1.9 < err[0] / err[1] < 2.8, err


def test_equilibrium_state_is_a_fixed_point():
    from test_oracle_pins import _equilibrium_state
    m = _mech()
    P, Y = _equilibrium_state(m, 1500.0, [-10.0, -12.0, -11.0])
    T = np.array([1500.0])
    T1, Y1 = oracle.integrate_euler(m, T, [P], Y[:, None], 1e-12, 100, precision="ld")
    assert abs(T1[0] - 1500.0) < 1e-9
    assert np.abs(Y1[:, 0] - Y).max() < 1e-12 * Y.max()
