"""Pins of the oracle's pressure-dependent reactions (Sec. 2.4 of the paper:
third-body reactions through M = C E added to the log forward rate, falloff
reactions through a separate, non-matrix blending function).

Each pin checks the oracle against something other than its own formula:
* a third-body reaction equals the sum of elementary reactions
  A + B + S_k <=> AB + S_k with rate constants eff_k k (the definition of
  [M] = sum_k eff_k C_k, evaluated by the oracle's elementary code path);
* Lindemann falloff equals the harmonic blend 1/(1/k_inf + 1/(k_0 [M])) at
  every pressure, with k_inf and k_0 [M] taken from elementary and
  third-body copies of the reaction;
* Troe falloff with a centre broadening Fc = 1 reduces to Lindemann, and at
  the centre of the falloff curve (log10 Pr = -c) the broadening equals Fc,
  for parameters whose Fc is 1/2 or 3/4 by construction;
* detailed balance and atom conservation hold for a synthetic mechanism
  with 20 % pressure-dependent reactions.
(The oracle's analytic Jacobian does not cover these reactions.)
"""

import math

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import synth


class _Mech:
    def __init__(self, W, nu_f, nu_r, ln_A, beta, Ea, a6, **extra):
        self.W = np.asarray(W, float)
        ns = self.W.shape[0]
        self.nu_f = np.asarray(nu_f, np.int8)
        self.nu_r = np.asarray(nu_r, np.int8)
        nr = self.nu_f.shape[0]
        self.ln_A = np.asarray(ln_A, float)
        self.beta = np.asarray(beta, float)
        self.Ea = np.asarray(Ea, float)
        low = np.zeros((ns, 7))
        low[:, 0] = 2.5
        low[:, 5] = a6
        self.nasa_low = low
        self.nasa_high = low
        self.T_mid = np.full(ns, 1000.0)
        self.reversible = np.ones(nr, np.uint8)
        for k, v in extra.items():
            setattr(self, k, v)


# A + B (+M) <=> AB (+M) with an inert partner X; W = (1, 16, 17, 40)
W4 = [1.0, 16.0, 17.0, 40.0]
A6 = [0.0, 0.0, -40000.0, 0.0]
NU_F = [[1, 1, 0, 0]]
NU_R = [[0, 0, 1, 0]]
KINF = dict(ln_A=[math.log(1e13)], beta=[0.5], Ea=[10000.0])
K0 = dict(ln_A=[math.log(1e13) + 11.0], beta=[-0.3], Ea=[6000.0])


def _states(n, seed, ns=4):
    rng = np.random.default_rng(seed)
    T = rng.uniform(900.0, 2500.0, n)
    P = rng.uniform(0.5, 30.0, n) * 101325.0
    Y = rng.dirichlet(np.full(ns, 0.7), n).T.copy()
    return T, P, Y


def test_third_body_equals_sum_of_elementary_reactions():
    eff = np.array([[1.0, 2.5, 0.3, 0.0]])
    tb = _Mech(W4, NU_F, NU_R, a6=A6, rtype=np.array([1], np.uint8), eff=eff, **KINF)
    # expanded: one elementary reaction A + B + S_k <=> AB + S_k per partner
    # with eff_k > 0, rate constant eff_k k (same reaction order 3)
    nf, nr_, lnA = [], [], []
    for k in range(4):
        if eff[0, k] == 0:
            continue
        f = np.array(NU_F[0]); r = np.array(NU_R[0])
        f[k] += 1
        r[k] += 1
        nf.append(f); nr_.append(r)
        lnA.append(KINF["ln_A"][0] + math.log(eff[0, k]))
    m = len(nf)
    el = _Mech(W4, nf, nr_, lnA, [0.5] * m, [10000.0] * m, a6=A6)
    T, P, Y = _states(40, 1)
    om_tb, S, _ = oracle.source(tb, T, P, Y, precision="ld", scales=True)
    om_el = oracle.source(el, T, P, Y, precision="ld")
    # the inert partner X (efficiency 0) takes no part
    assert np.all(om_tb[3] == 0) and np.all(S[3] == 0)
    # ln A + ln eff_k rounds in double: a few 1e-15 of relative difference
    rel = np.abs((om_tb - om_el)[:3].astype(float)) / S[:3].astype(float)
    assert rel.max() < 1e-14, rel.max()
    # [M] with unit efficiencies is the total concentration P/(Ru T)
    one = _Mech(W4, NU_F, NU_R, a6=A6, rtype=np.array([1], np.uint8),
                eff=np.ones((1, 4)), **KINF)
    plain = _Mech(W4, NU_F, NU_R, a6=A6, **KINF)
    for Ti, Pi in ((1200.0, 101325.0), (2000.0, 5e6)):
        y = np.array([0.1, 0.4, 0.3, 0.2])
        k1 = oracle.rates(one, Ti, Pi, y, precision="ld")["kf"][0]
        k_el = oracle.rates(plain, Ti, Pi, y, precision="ld")["kf"][0]
        # the elementary copy counts A as second order: one order more is 1e-3
        ctot = np.longdouble(Pi) / (np.longdouble(8314.46261815324) * np.longdouble(Ti))
        assert abs(k1 / (k_el * np.longdouble(1e-3) * ctot) - 1) < 1e-16


def _falloff(rtype, troe=None):
    return _Mech(W4, NU_F, NU_R, a6=A6, rtype=np.array([rtype], np.uint8),
                 eff=np.array([[1.0, 1.0, 2.0, 0.5]]), low_ln_A=K0["ln_A"],
                 low_beta=K0["beta"], low_Ea=K0["Ea"],
                 troe=None if troe is None else np.array([troe], float), **KINF)


def _limits(T, P, y):
    """k_inf (elementary copy) and k_0 [M] (third-body copy of the low-
    pressure parameters) at one state."""
    el = _Mech(W4, NU_F, NU_R, a6=A6, **KINF)
    tb = _Mech(W4, NU_F, NU_R, a6=A6, rtype=np.array([1], np.uint8),
               eff=np.array([[1.0, 1.0, 2.0, 0.5]]), **K0)
    kinf = oracle.rates(el, T, P, y, precision="ld")["kf"][0]
    k0M = oracle.rates(tb, T, P, y, precision="ld")["kf"][0]
    return kinf, k0M


@pytest.mark.parametrize("T", [1000.0, 1700.0, 2400.0])
def test_lindemann_is_the_harmonic_blend(T):
    y = np.array([0.2, 0.3, 0.4, 0.1])
    lind = _falloff(2)
    for P in (1e-2, 1e2, 1e4, 1e5, 1e6, 1e8, 1e11):
        kinf, k0M = _limits(T, P, y)
        k = oracle.rates(lind, T, P, y, precision="ld")["kf"][0]
        ref = 1 / (1 / kinf + 1 / k0M)
        assert abs(k / ref - 1) < 1e-16, (P, k, ref)
    # the two limits
    kinf, k0M = _limits(T, 1e16, y)
    assert abs(oracle.rates(lind, T, 1e16, y, precision="ld")["kf"][0] / kinf - 1) < 1e-6
    kinf, k0M = _limits(T, 1e-10, y)
    assert abs(oracle.rates(lind, T, 1e-10, y, precision="ld")["kf"][0] / k0M - 1) < 1e-6


def test_troe_with_unit_centre_is_lindemann():
    y = np.array([0.25, 0.25, 0.25, 0.25])
    lind = _falloff(2)
    # Fc = 0 * exp(-T/T3) + 1 * exp(-T/1e30) = 1 (no T2 term): F = 1
    troe = _falloff(3, [1.0, 100.0, 1e30, 0.0])
    for T in (950.0, 1800.0):
        for P in (1e3, 1e5, 1e7):
            a = oracle.rates(lind, T, P, y, precision="ld")["kf"][0]
            b = oracle.rates(troe, T, P, y, precision="ld")["kf"][0]
            assert abs(b / a - 1) < 1e-17


@pytest.mark.parametrize("case", ["half", "three_quarters"])
def test_troe_centre_broadening_equals_fc(case):
    # Fc by construction: T3 = T1 = T / ln 2 make both exponentials 1/2;
    # with alpha = 1/2 and no T2 term Fc = 1/2; with alpha = 1/4 and
    # T2 = T ln 4 (exp(-T2/T) = 1/4) Fc = 3/4
    T = 1500.0
    if case == "half":
        troe, fc = [0.5, T / math.log(2.0), T / math.log(2.0), 0.0], 0.5
    else:
        troe, fc = [0.25, T / math.log(2.0), T / math.log(2.0), T * math.log(4.0)], 0.75
    m = _falloff(3, troe)
    y = np.array([0.1, 0.2, 0.3, 0.4])
    # centre of the falloff curve: log10 Pr + c = 0, c = -0.4 - 0.67 log10 Fc
    c = -0.4 - 0.67 * math.log10(fc)
    # Pr is proportional to P (k_0 [M] / k_inf): find P with Pr = 10^-c
    P1 = 1e5
    kinf, k0M = _limits(T, P1, y)
    P = P1 * (10.0 ** (-c)) * float(kinf / k0M)
    kinf, k0M = _limits(T, P, y)
    pr = k0M / kinf
    assert abs(float(np.log10(pr)) + c) < 1e-12
    k = oracle.rates(m, T, P, y, precision="ld")["kf"][0]
    F = float(k / (kinf * pr / (1 + pr)))
    assert abs(F - fc) < 1e-12, (F, fc)
    # width of the curve: where (log10 Pr + c) / (n - 0.14 (log10 Pr + c))
    # is +1 or -1, i.e. log10 Pr + c = n / 1.14 or -n / 0.86 with
    # n = 0.75 - 1.27 log10 Fc, the broadening is sqrt(Fc)
    n = 0.75 - 1.27 * math.log10(fc)
    for x in (n / 1.14, -n / 0.86):
        Px = P * 10.0 ** x
        kinf, k0M = _limits(T, Px, y)
        pr = k0M / kinf
        assert abs(float(np.log10(pr)) + c - x) < 1e-12
        F = float(oracle.rates(m, T, Px, y, precision="ld")["kf"][0] / (kinf * pr / (1 + pr)))
        assert abs(F - math.sqrt(fc)) < 1e-12, (x, F, math.sqrt(fc))
    # away from the centre the broadening is closer to one than Fc
    for s in (1e-3, 1e3):
        kinf, k0M = _limits(T, P * s, y)
        pr = k0M / kinf
        F = float(oracle.rates(m, T, P * s, y, precision="ld")["kf"][0] / (kinf * pr / (1 + pr)))
        assert fc < F < 1


def test_pressure_dependent_detailed_balance_and_conservation():
    from test_oracle_pins import _equilibrium_state
    mech = synth.with_pressure_dependence(synth.make_mechanism(9, 21), frac=0.5)
    assert set(np.unique(mech.rtype)) >= {1, 2, 3}
    rng = np.random.default_rng(2)
    for T in (1000.0, 1600.0, 2400.0):
        lam = rng.uniform(-14.0, -8.0, mech.n_elements)
        P, Y = _equilibrium_state(mech, T, lam)
        om, S, _ = oracle.source(mech, [T], [P], Y[:, None], precision="ld", scales=True)
        assert float((np.abs(om[:, 0]) / S[:, 0]).max()) < 1e-14
    T, P, Y = synth.make_states(mech, 200, 3)
    om, S, _ = oracle.source(mech, T, P, Y, precision="ld", scales=True)
    om = om.astype(float)
    scale = (mech.W[:, None] * S.astype(float)).sum(axis=0)
    assert np.all(np.abs((mech.W[:, None] * om).sum(axis=0)) <= 1e-14 * scale)
    for e in range(mech.n_elements):
        a = mech.atoms[:, e].astype(float)[:, None]
        assert np.all(np.abs((a * om).sum(axis=0)) <= 1e-14 * (a * S.astype(float)).sum(axis=0) + 1e-300)


def test_jacobian_not_claimed_for_pressure_dependent_reactions():
    mech = synth.with_pressure_dependence(synth.make_mechanism(9, 21), frac=0.5)
    T, P, Y = synth.make_states(mech, 4, 3)
    with pytest.raises(NotImplementedError):
        oracle.jacobian(mech, T, P, Y)
