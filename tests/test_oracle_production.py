"""Pins of the oracle's stoichiometric contraction omega = nu r (Eq. 2 with
the rates of progress given), against facts other than its own product: a
hand-balanced reaction in closed form, agreement with the separately pinned
source term when r is that cell's q_f - q_r, and conservation of mass and of
every element for arbitrary rates (each reaction is balanced)."""

import numpy as np

import oracle
from paper_2008_08483_amd import synth
from tests.test_oracle_pins import _Mech, _nasa


def test_hand_reaction_closed_form():
    # 2 H2 + O2 -> 2 H2O and H2O -> H + OH, at rates 3 and -0.5
    m = _Mech([2.016, 31.998, 18.015, 1.008, 17.007],
              [[2, 1, 0, 0, 0], [0, 0, 1, 0, 0]],
              [[0, 0, 2, 0, 0], [0, 0, 0, 1, 1]],
              [0.0, 0.0], [0.0, 0.0], [0.0, 0.0], _nasa([3.5] * 5, [0.0] * 5))
    om = oracle.production(m, np.array([[3.0], [-0.5]]))
    np.testing.assert_array_equal(om[:, 0], [-6.0, -3.0, 6.5, -0.5, -0.5])


def test_matches_source_at_the_cells_rates():
    m = synth.make_mechanism(9, 21, seed=3)
    T, P, Y = synth.make_states(m, 6, 4, (1000.0, 2500.0), 1.0, 0.5)
    om = oracle.source(m, T, P, Y)
    for i in range(T.shape[0]):
        q = oracle.rates(m, T[i], P[i], Y[:, i])
        r = (q["qf"] - q["qr"])[:, None]
        scale = np.abs(m.nu_r - m.nu_f).T.astype(float) @ (q["qf"] + q["qr"])
        got = oracle.production(m, r)[:, 0]
        assert np.all(np.abs(got - om[:, i]) <= 1e-13 * scale + 1e-300)


def test_mass_and_elements_conserved_for_any_rates():
    m = synth.make_mechanism(53, 325, seed=1)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((325, 17)) * 10.0 ** rng.uniform(-20, 10, (325, 17))
    om = oracle.production(m, r)
    gross = np.abs((m.nu_r - m.nu_f).T.astype(float)) @ np.abs(r)
    mass = m.W @ om
    assert np.all(np.abs(mass) <= 1e-13 * (m.W @ gross))
    el = m.atoms.T.astype(float) @ om
    assert np.all(np.abs(el) <= 1e-13 * (m.atoms.T.astype(float) @ gross + 1e-300))
