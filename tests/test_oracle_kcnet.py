"""Pins of the oracle's ln K_c pieces: ln K_c alone (Eq. 8), the source term
with a given ln K_c in place of Eq. 8 (the drop-in of Sec. 2.3), and the
approximate ln K_c network of Sec. 2.3 (Architecture 2: standardized ln T in,
elu hidden layers, Eqs. 12 and 14, a linear output layer to N_R standardized
outputs).  Each is checked against closed forms, 50-digit brute force or the
separately pinned source term."""

import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import synth
from tests.test_oracle_pins import PREF, RU, RU_MOL, _golden, _Mech, _nasa


def _example2():
    g = _golden()["example2"]
    W = np.array(g["W"])
    X = np.array(g["X"])
    Y = X * W / (X * W).sum()
    m = _Mech(W, [[1, 1, 0]], [[0, 0, 1]], [math.log(g["A_cgs"])], [g["beta"]],
              [g["Ea_cal"]], _nasa(g["nasa_a1"], g["nasa_a6"]))
    return g, m, Y


def test_lnkc_hand_example_2():
    g, m, _ = _example2()
    got = oracle.lnkc(m, [g["T"]], precision="ld")
    assert got.shape == (1, 1)
    assert abs(float(got[0, 0]) - 8.611472607251978) < 1e-12


def _mp_lnkc(mech, T):
    mp.mp.dps = 50
    T = mp.mpf(T)
    ns, nr = mech.nu_f.shape[1], mech.nu_f.shape[0]
    H, S = [], []
    for k in range(ns):
        a = mech.nasa_high[k] if T >= mech.T_mid[k] else mech.nasa_low[k]
        a = [mp.mpf(float(x)) for x in a]
        H.append(a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5 + a[5] / T)
        S.append(a[0] * mp.log(T) + a[1] * T + a[2] * T ** 2 / 2 + a[3] * T ** 3 / 3 + a[4] * T ** 4 / 4 + a[6])
    out = []
    for j in range(nr):
        nu = [int(mech.nu_r[j, k]) - int(mech.nu_f[j, k]) for k in range(ns)]
        out.append(sum(nu) * mp.log(PREF / (RU * T)) + sum(n * (S[k] - H[k]) for k, n in enumerate(nu)))
    return out


def test_lnkc_brute_force_tiny_mechanism():
    mech = synth.make_mechanism(6, 9, seed=4)
    T = np.array([650.0, 999.999, 1000.0, 2750.5])
    got = oracle.lnkc(mech, T, precision="ld")
    for i, t in enumerate(T):
        ref = _mp_lnkc(mech, t)
        for j in range(mech.n_reactions):
            assert abs(float(got[j, i]) - float(ref[j])) <= 1e-15 * (1 + abs(float(ref[j]))), (i, j)


def test_source_with_given_lnkc_hand_example_2():
    # omega_AB = q_f - k_f exp(-L) C_AB with an arbitrary L in place of ln K_c
    g, m, Y = _example2()
    T, P = g["T"], g["P"]
    L = 3.25
    mp.mp.dps = 50
    T_ = mp.mpf(T)
    kf = mp.mpf(10) ** 10 * T_ ** mp.mpf("0.5") * mp.exp(-mp.mpf(10000) * mp.mpf("4.184") / RU_MOL / T_)
    Ct = mp.mpf(P) / (RU * T_)
    CA, CB, CAB = [mp.mpf(x) * Ct for x in g["X"]]
    expect = float(kf * CA * CB - kf * mp.exp(-mp.mpf(L)) * CAB)
    om = oracle.source_lnkc(m, [T], [P], Y[:, None], np.array([[L]]), precision="ld")[:, 0]
    for k, sgn in ((0, -1), (1, -1), (2, 1)):
        assert abs(float(om[k]) - sgn * expect) <= 1e-14 * abs(expect), k


def test_source_with_exact_lnkc_is_the_source():
    mech = synth.make_mechanism(9, 21)
    T, P, Y = synth.make_states(mech, 32, 9, (800.0, 2800.0), (1.0, 20.0), 0.3)
    a, S, _ = oracle.source(mech, T, P, Y, scales=True)
    b = oracle.source_lnkc(mech, T, P, Y, oracle.lnkc(mech, T))
    assert np.all(np.abs(a - b) <= 1e-14 * S)


def test_lnkc_shift_scales_the_reverse_rate():
    # ln K_c of reaction j raised by d: q_r,j -> q_r,j e^-d, so
    # omega_k changes by nu_kj q_r,j (1 - e^-d) and nothing else changes
    mech = synth.make_mechanism(9, 21)
    T, P, Y = synth.make_states(mech, 4, 10, (800.0, 2800.0), (1.0, 20.0), 0.3)
    K = oracle.lnkc(mech, T)
    base = oracle.source_lnkc(mech, T, P, Y, K, precision="ld").astype(float)
    nu = (mech.nu_r.astype(int) - mech.nu_f.astype(int))
    for j, d in ((0, 0.7), (5, -1.3), (20, 2.0)):
        K2 = K.copy()
        K2[j] += d
        got = oracle.source_lnkc(mech, T, P, Y, K2, precision="ld").astype(float)
        for i in range(4):
            qr = float(oracle.rates(mech, T[i], P[i], Y[:, i], precision="ld")["qr"][j])
            expect = nu[j] * qr * (1.0 - math.exp(-d))
            scale = np.abs(base[:, i]).max() + abs(qr)
            assert np.all(np.abs(got[:, i] - base[:, i] - expect) <= 1e-12 * scale), (j, i)


def test_given_lnkc_ignored_by_irreversible_reactions():
    mech = synth.make_mechanism(9, 21)
    mech.reversible = mech.reversible.copy()
    mech.reversible[[2, 7]] = 0
    T, P, Y = synth.make_states(mech, 8, 11, (800.0, 2800.0), (1.0, 20.0), 0.3)
    K = oracle.lnkc(mech, T)
    K[[2, 7]] = np.nan
    got = oracle.source_lnkc(mech, T, P, Y, K)
    assert np.all(np.isfinite(got))
    a, S, _ = oracle.source(mech, T, P, Y, scales=True)
    assert np.all(np.abs(got - a) <= 1e-14 * S)


class _Net:
    def __init__(self, weights, biases, x_mean, x_std, y_mean, y_std):
        self.weights, self.biases = weights, biases
        self.x_mean, self.x_std, self.y_mean, self.y_std = x_mean, x_std, y_mean, y_std


def _hand_net():
    # z = (ln T - 7) / 0.5; one hidden layer of two neurons, three outputs
    return _Net([np.array([[2.0, -3.0]]), np.array([[1.0, 0.0, 2.0], [4.0, -1.0, 0.5]])],
                [np.array([0.5, 1.0]), np.array([0.0, 1.0, -1.0])],
                7.0, 0.5, np.array([10.0, -5.0, 0.0]), np.array([2.0, 3.0, 4.0]))


def test_kcnet_closed_form():
    net = _hand_net()
    T = math.exp(7.5)                     # z = 1: pre-activations 2.5 and -2
    e = math.expm1(-2.0)                  # elu(-2) = e^-2 - 1
    out = [2.5 + 4.0 * e, -e + 1.0, 5.0 + 0.5 * e - 1.0]
    expect = [o * s + m for o, s, m in zip(out, (2.0, 3.0, 4.0), (10.0, -5.0, 0.0))]
    got, mag = oracle.kcnet(net, [T], bound=True)
    assert got.shape == (3, 1)
    np.testing.assert_allclose(got[:, 0], expect, rtol=1e-15, atol=1e-14)
    # running magnitude: |z||W0| + |b0| = (2.5, 4); then |.||W1| + |b1|, times |std|, + |mean|
    h = [2.5, 4.0]
    m1 = [h[0] * 1 + h[1] * 4 + 0, h[0] * 0 + h[1] * 1 + 1, h[0] * 2 + h[1] * 0.5 + 1]
    np.testing.assert_allclose(mag[:, 0], [m1[0] * 2 + 10, m1[1] * 3 + 5, m1[2] * 4 + 0],
                               rtol=1e-15)


def test_kcnet_elu_branches():
    # one neuron, identity readout: elu(w z) at z of both signs, and at 0
    net = _Net([np.array([[1.0]]), np.array([[1.0]])], [np.array([0.0]), np.array([0.0])],
               0.0, 1.0, np.array([0.0]), np.array([1.0]))
    T = np.exp([-3.0, -1e-9, 0.0, 1e-9, 2.0])
    z = np.log(T)                           # the inputs exactly as the network sees them
    got = oracle.kcnet(net, T)[0]
    expect = [math.expm1(z[0]), math.expm1(z[1]), 0.0, z[3], z[4]]
    assert z[1] < 0.0 < z[3] and z[2] == 0.0
    np.testing.assert_allclose(got, expect, rtol=1e-15, atol=0)


def test_kcnet_identity_hidden_layers():
    # extra hidden layers that are the identity on positive activations
    # (W = I, bias 0, inputs kept positive by a large first bias) leave the
    # output unchanged: depth is counted as N_L hidden layers + 1 readout
    rng = np.random.default_rng(3)
    w0 = rng.uniform(-1, 1, (1, 8))
    b0 = np.full(8, 10.0)
    wo = rng.normal(size=(8, 5))
    bo = rng.normal(size=5)
    ym, ys = rng.normal(size=5), rng.uniform(0.5, 2.0, 5)
    T = rng.uniform(300.0, 3000.0, 20)
    one = oracle.kcnet(_Net([w0, wo], [b0, bo], 7.0, 0.6, ym, ys), T)
    three = oracle.kcnet(_Net([w0, np.eye(8), np.eye(8), wo], [b0, np.zeros(8), np.zeros(8), bo],
                              7.0, 0.6, ym, ys), T)
    np.testing.assert_allclose(three, one, rtol=1e-14, atol=1e-13)


def test_euler_with_given_lnkc_is_euler_when_exact():
    # the composition with the exact ln K_c reproduces the (pinned) Euler
    # integrator of the oracle, step for step
    mech = synth.make_mechanism(9, 21, ln_A_range=(8.0, 16.0), Ea_range=(20000.0, 60000.0))
    T, P, Y = synth.make_states(mech, 6, 12, (1000.0, 2500.0), 1.0, 0.5)
    a = oracle.integrate_euler_lnkc(mech, lambda t: oracle.lnkc(mech, t), T, P, Y, 1e-14, 20)
    b = oracle.integrate_euler(mech, T, P, Y, 1e-14, 20)
    assert np.abs(a[0] - T).max() > 1e-3
    np.testing.assert_allclose(a[0], b[0], rtol=1e-13)
    assert np.abs(a[1] - b[1]).max() <= 1e-13
