"""Pins of the test oracle against facts fixed by the paper and by mathematics.

The oracle (``oracle/``) evaluates the source term of Barwey & Raman, Sec. 2,
in the classical form.  Each test here checks it against something other
than itself: closed forms of hand-worked reactions, detailed balance at a
constructed equilibrium state, conservation laws, homogeneity, thermodynamic
identities, special cases and 50-digit brute force.
"""

import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
mp.mp.dps = 50
RU = mp.mpf("8314.46261815324")
RU_MOL = mp.mpf("8.31446261815324")
PREF = mp.mpf(100000)


class _Mech:
    """Minimal mechanism container for hand-built cases."""

    def __init__(self, W, nu_f, nu_r, ln_A, beta, Ea, low, high=None, T_mid=1000.0, rev=None):
        self.W = np.asarray(W, float)
        self.nu_f = np.asarray(nu_f, np.int8)
        self.nu_r = np.asarray(nu_r, np.int8)
        self.ln_A = np.asarray(ln_A, float)
        self.beta = np.asarray(beta, float)
        self.Ea = np.asarray(Ea, float)
        self.nasa_low = np.asarray(low, float)
        self.nasa_high = np.asarray(low if high is None else high, float)
        ns = self.W.shape[0]
        self.T_mid = np.full(ns, float(T_mid))
        nr = self.nu_f.shape[0]
        self.reversible = np.ones(nr, np.uint8) if rev is None else np.asarray(rev, np.uint8)


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _nasa(a1, a6):
    low = np.zeros((len(a1), 7))
    low[:, 0] = a1
    low[:, 5] = a6
    return low


# --------------------------------------------------------------------------
# hand-worked reactions, closed forms


def test_hand_example_1_closed_form():
    g = _golden()["example1"]
    m = _Mech(g["W"], [[1, 0]], [[0, 1]], [math.log(g["A_cgs"])], [g["beta"]], [g["Ea_cal"]],
              _nasa(g["nasa_a1"], g["nasa_a6"]))
    T, P = g["T"], g["P"]
    om = oracle.source(m, [T], [P], np.array(g["Y"])[:, None], precision="ld")[:, 0]
    mp.mp.dps = 50
    C = mp.mpf(P) / (RU * T) / 2
    qf = mp.mpf(g["A_cgs"]) * C
    qr = qf / mp.e
    expect = float(qf - qr)
    assert abs(float(om[1]) - expect) <= 1e-15 * expect
    assert abs(float(om[0]) + expect) <= 1e-15 * expect
    # same value as printed in the hand derivation
    assert abs(expect - 3.851699055298052e7) < 1e-6


def test_hand_example_2_closed_form():
    g = _golden()["example2"]
    W = np.array(g["W"])
    X = np.array(g["X"])
    Y = X * W / (X * W).sum()
    m = _Mech(W, [[1, 1, 0]], [[0, 0, 1]], [math.log(g["A_cgs"])], [g["beta"]],
              [g["Ea_cal"]], _nasa(g["nasa_a1"], g["nasa_a6"]))
    T, P = g["T"], g["P"]
    mp.mp.dps = 50
    T_ = mp.mpf(T)
    kf = mp.mpf(10) ** 10 * T_ ** mp.mpf("0.5") * mp.exp(-mp.mpf(10000) * mp.mpf("4.184") / RU_MOL / T_)
    lnKc = -mp.log(PREF / (RU * T_)) + 40000 / T_ + mp.mpf("2.5") - mp.mpf("2.5") * mp.log(T_)
    Ctot = mp.mpf(P) / (RU * T_)
    CA, CB, CAB = [mp.mpf(x) * Ctot for x in g["X"]]
    qf = kf * CA * CB
    qr = kf / mp.exp(lnKc) * CAB
    expect = float(qf - qr)
    om = oracle.source(m, [T], [P], Y[:, None], precision="ld")[:, 0]
    for k, sgn in ((0, -1), (1, -1), (2, 1)):
        assert abs(float(om[k]) - sgn * expect) <= 1e-14 * expect, k
    r = oracle.rates(m, T, P, Y, precision="ld")
    assert abs(float(mp.log(r["Kc"][0])) - float(lnKc)) < 1e-14 * 10
    assert abs(float(lnKc) - 8.611472607251978) < 1e-12
    assert abs(float(mp.log(kf)) - 24.31020449221767) < 1e-12
    # mass conservation for this reaction: sum W_k omega_k = 0
    assert abs(float((W * om.astype(float)).sum())) <= 1e-14 * float(W @ np.abs(om.astype(float)))


def test_hand_example_scales_closed_form():
    """Gross and net rate scales S = sum_j |nu| (q_f + q_r), N = sum_j |nu|
    |q_f - q_r| in closed form: examples 1 and 2 (|nu| = 1) and example 3
    (2 A <=> B, |nu_A| = 2)."""
    g = _golden()
    mp.mp.dps = 50
    # example 1
    e = g["example1"]
    m = _Mech(e["W"], [[1, 0]], [[0, 1]], [math.log(e["A_cgs"])], [e["beta"]], [e["Ea_cal"]],
              _nasa(e["nasa_a1"], e["nasa_a6"]))
    _, S, N = oracle.source(m, [e["T"]], [e["P"]], np.array(e["Y"])[:, None], precision="ld",
                            scales=True)
    C = mp.mpf(e["P"]) / (RU * e["T"]) / 2
    qf = mp.mpf(e["A_cgs"]) * C
    qr = qf / mp.e
    for k in range(2):
        assert abs(float(S[k, 0]) - float(qf + qr)) <= 1e-15 * float(qf + qr)
        assert abs(float(N[k, 0]) - float(qf - qr)) <= 1e-15 * float(qf - qr)
    # example 2
    e = g["example2"]
    W = np.array(e["W"])
    X = np.array(e["X"])
    Y = X * W / (X * W).sum()
    m = _Mech(W, [[1, 1, 0]], [[0, 0, 1]], [math.log(e["A_cgs"])], [e["beta"]], [e["Ea_cal"]],
              _nasa(e["nasa_a1"], e["nasa_a6"]))
    T_ = mp.mpf(e["T"])
    kf = mp.mpf(10) ** 10 * T_ ** mp.mpf("0.5") * mp.exp(-mp.mpf(10000) * mp.mpf("4.184") / RU_MOL / T_)
    lnKc = -mp.log(PREF / (RU * T_)) + 40000 / T_ + mp.mpf("2.5") - mp.mpf("2.5") * mp.log(T_)
    Ct = mp.mpf(e["P"]) / (RU * T_)
    qf = kf * (mp.mpf(X[0]) * Ct) * (mp.mpf(X[1]) * Ct)
    qr = kf / mp.exp(lnKc) * (mp.mpf(X[2]) * Ct)
    _, S, N = oracle.source(m, [e["T"]], [e["P"]], Y[:, None], precision="ld", scales=True)
    for k in range(3):
        assert abs(float(S[k, 0]) - float(qf + qr)) <= 1e-14 * float(qf + qr)
        assert abs(float(N[k, 0]) - float(qf - qr)) <= 1e-14 * float(qf - qr)
    # example 3: 2 A <=> B
    e = g["example3"]
    W = np.array(e["W"])
    X = np.array(e["X"])
    Y = X * W / (X * W).sum()
    low = np.zeros((2, 7))
    low[:, 0] = e["nasa_a1"]
    low[:, 5] = e["nasa_a6"]
    low[:, 6] = e["nasa_a7"]
    m = _Mech(W, [[2, 0]], [[0, 1]], [math.log(e["A_cgs"])], [e["beta"]], [e["Ea_cal"]], low)
    T_ = mp.mpf(e["T"])
    a1 = mp.mpf(e["nasa_a1"][0])
    dH = (a1 + mp.mpf(e["nasa_a6"][1]) / T_) - 2 * a1
    dS = (a1 * mp.log(T_) + mp.mpf(e["nasa_a7"][1])) - 2 * (a1 * mp.log(T_) + mp.mpf(e["nasa_a7"][0]))
    lnKc = -mp.log(PREF / (RU * T_)) + dS - dH
    Ct = mp.mpf(e["P"]) / (RU * T_)
    kf = mp.mpf(e["A_cgs"]) * mp.mpf("1e-3")
    qf = kf * (mp.mpf(X[0]) * Ct) ** 2
    qr = kf / mp.exp(lnKc) * (mp.mpf(X[1]) * Ct)
    om, S, N = oracle.source(m, [e["T"]], [e["P"]], Y[:, None], precision="ld", scales=True)
    for k, nu in ((0, -2), (1, 1)):
        assert abs(float(om[k, 0]) - float(nu * (qf - qr))) <= 1e-14 * float(abs(nu) * (qf + qr))
        assert abs(float(S[k, 0]) - float(abs(nu) * (qf + qr))) <= 1e-14 * float(abs(nu) * (qf + qr))
        assert abs(float(N[k, 0]) - float(abs(nu) * abs(qf - qr))) <= 1e-14 * float(abs(nu) * (qf + qr))
    r = oracle.rates(m, e["T"], e["P"], Y, precision="ld")
    assert abs(float(mp.log(r["Kc"][0])) - float(lnKc)) < 1e-13


def test_hand_example_1_temperature_source_closed_form():
    """omega_T = T omega_B / (3.5 C_tot) for example 1 (see the golden file)."""
    e = _golden()["example1"]
    m = _Mech(e["W"], [[1, 0]], [[0, 1]], [math.log(e["A_cgs"])], [e["beta"]], [e["Ea_cal"]],
              _nasa(e["nasa_a1"], e["nasa_a6"]))
    mp.mp.dps = 50
    T, P = e["T"], e["P"]
    Ct = mp.mpf(P) / (RU * T)
    qf = mp.mpf(e["A_cgs"]) * Ct / 2
    omB = qf - qf / mp.e
    expect = float(mp.mpf(T) * omB / (mp.mpf("3.5") * Ct))
    got = float(oracle.temp_source(m, [T], [P], np.array(e["Y"])[:, None], precision="ld")[0])
    assert abs(got - expect) <= 1e-15 * abs(expect)
    # the double build agrees to rounding
    got64 = float(oracle.temp_source(m, [T], [P], np.array(e["Y"])[:, None])[0])
    assert abs(got64 - expect) <= 1e-13 * abs(expect)


def test_irreversible_flag_drops_reverse_rate():
    g = _golden()["example2"]
    W = np.array(g["W"])
    X = np.array(g["X"])
    Y = X * W / (X * W).sum()
    m = _Mech(W, [[1, 1, 0]], [[0, 0, 1]], [math.log(g["A_cgs"])], [g["beta"]],
              [g["Ea_cal"]], _nasa(g["nasa_a1"], g["nasa_a6"]), rev=[0])
    r = oracle.rates(m, g["T"], g["P"], Y)
    assert r["qr"][0] == 0.0
    om = oracle.source(m, [g["T"]], [g["P"]], Y[:, None])[:, 0]
    assert om[2] == pytest.approx(r["qf"][0], rel=1e-15)


def test_tmid_tie_uses_high_range():
    # species B differs between ranges only in a6; at T == T_mid the high set applies
    low = _nasa([3.5, 3.5], [0.0, -1000.0])
    high = _nasa([3.5, 3.5], [0.0, -2000.0])
    m = _Mech([2.0, 2.0], [[1, 0]], [[0, 1]], [math.log(1e10)], [0.0], [0.0], low, high)
    for T, a6 in ((1000.0, -2000.0), (999.9999, -1000.0)):
        r = oracle.rates(m, T, 101325.0, [0.5, 0.5], precision="ld")
        assert float(np.log(r["Kc"][0])) == pytest.approx(-a6 / T, rel=1e-15)


def test_arrhenius_special_cases():
    # beta = 0, E = 0: kf = A (unit conversion by reaction order, cgs -> SI kmol)
    low = _nasa([3.5] * 3, [0.0] * 3)
    for nu_f, nu_r, order in (([[1, 0, 0]], [[0, 1, 0]], 1), ([[1, 1, 0]], [[0, 0, 1]], 2),
                              ([[2, 1, 0]], [[0, 0, 1]], 3)):
        m = _Mech([1.0, 1.0, 2.0], nu_f, nu_r, [math.log(5e11)], [0.0], [0.0], low)
        r = oracle.rates(m, 1234.0, 2e5, [0.3, 0.3, 0.4], precision="ld")
        assert float(r["kf"][0]) == pytest.approx(5e11 * 1e-3 ** (order - 1), rel=1e-15)
    # general: kf = A T^b exp(-E/RT) vs the Arrhenius layer's log form (Eq. 6)
    m = _Mech([1.0, 1.0, 2.0], [[1, 1, 0]], [[0, 0, 1]], [30.0], [-1.3], [25000.0], low)
    for T in (300.0, 800.0, 1500.0, 2999.0):
        r = oracle.rates(m, T, 2e5, [0.3, 0.3, 0.4], precision="ld")
        ln_kf = 30.0 + math.log(1e-3) - 1.3 * math.log(T) - 25000.0 * 4.184 / 8.31446261815324 / T
        assert math.log(float(r["kf"][0])) == pytest.approx(ln_kf, abs=1e-13)


# --------------------------------------------------------------------------
# thermodynamics: NASA-7 definitions and identities


def test_thermo_single_coefficient_forms():
    # a species with one nonzero cp coefficient a_n: cp/R = a_n T^(n-1),
    # h/RT = a_n T^(n-1)/n, s/R = a_n T^(n-1)/(n-1) (a1: ln T); a6 -> h/RT += a6/T; a7 -> s/R += a7
    T = 1700.0
    for n in range(1, 6):
        low = np.zeros((1, 7))
        low[0, n - 1] = 0.7
        low[0, 5] = 123.0
        low[0, 6] = -4.5
        m = _Mech([1.0], [[1]], [[1]], [0.0], [0.0], [0.0], low)
        h, s, cp = oracle.thermo(m, T, precision="ld")
        assert float(cp[0]) == pytest.approx(0.7 * T ** (n - 1), rel=1e-15)
        assert float(h[0]) == pytest.approx(0.7 * T ** (n - 1) / n + 123.0 / T, rel=1e-15)
        s_exp = 0.7 * (math.log(T) if n == 1 else T ** (n - 1) / (n - 1)) - 4.5
        assert float(s[0]) == pytest.approx(s_exp, rel=1e-14)


@pytest.mark.parametrize("T", [450.0, 800.0, 1300.0, 2600.0])
def test_thermo_identities(T):
    mech = synth.make_mechanism(53, 325)
    d = 1e-3
    hp, sp, _ = oracle.thermo(mech, T + d, precision="ld")
    hm, sm, _ = oracle.thermo(mech, T - d, precision="ld")
    _, _, cp = oracle.thermo(mech, T, precision="ld")
    # d(H/R)/dT = cp/R with H/R = T h/RT; dS/dT = cp/T
    dH = ((T + d) * hp - (T - d) * hm) / (2 * d)
    dS = (sp - sm) / (2 * d)
    np.testing.assert_allclose(dH.astype(float), cp.astype(float), rtol=1e-9)
    np.testing.assert_allclose((dS * T).astype(float), cp.astype(float), rtol=1e-9)


def test_vant_hoff():
    mech = synth.make_mechanism(9, 21)
    T, P = 1500.0, 3e5
    Y = np.full(9, 1 / 9)
    d = 1e-3
    rp = oracle.rates(mech, T + d, P, Y, precision="ld")
    rm = oracle.rates(mech, T - d, P, Y, precision="ld")
    h, _, _ = oracle.thermo(mech, T, precision="ld")
    nu = (mech.nu_r - mech.nu_f).astype(float)
    dlnKc = (np.log(rp["Kc"]) - np.log(rm["Kc"])) / (2 * d)
    expect = (nu @ h.astype(float) - nu.sum(axis=1)) / T
    np.testing.assert_allclose(dlnKc.astype(float), expect, rtol=1e-8, atol=1e-12)


# --------------------------------------------------------------------------
# invariants on synthetic mechanisms


def _equilibrium_state(mech, T, lam):
    """State with ln(C_k/C0) = -G_k + sum_e a_ke lam_e: every atom-balanced
    reaction then has zero affinity (detailed balance)."""
    mp.mp.dps = 50
    h, s, _ = oracle.thermo(mech, T, precision="ld")
    G = (h - s).astype(np.longdouble)
    C0 = np.longdouble(1e5) / (np.longdouble(8314.46261815324) * np.longdouble(T))
    lnC = np.log(C0) - G + mech.atoms.astype(np.longdouble) @ np.asarray(lam, np.longdouble)
    C = np.exp(lnC)
    P = float(np.longdouble(8314.46261815324) * T * C.sum())
    Y = C * mech.W.astype(np.longdouble)
    Y = (Y / Y.sum()).astype(float)
    return P, Y


@pytest.mark.parametrize("ns,nr", [(9, 21), (53, 325)])
def test_detailed_balance(ns, nr):
    mech = synth.make_mechanism(ns, nr)
    rng = np.random.default_rng(7)
    for T in (900.0, 1000.0, 1600.0, 2500.0):
        lam = rng.uniform(-14.0, -8.0, mech.n_elements)
        P, Y = _equilibrium_state(mech, T, lam)
        om, S, _ = oracle.source(mech, [T], [P], Y[:, None], precision="ld", scales=True)
        rel = np.abs(om[:, 0]) / S[:, 0]
        assert float(rel.max()) < 1e-14, (T, float(rel.max()))
        # and the rates themselves are far from zero
        r = oracle.rates(mech, T, P, Y)
        assert np.all(r["qf"] > 0)
        np.testing.assert_allclose(r["qr"], r["qf"], rtol=1e-9)


def test_hand_example_2_equilibrium():
    # A + B <=> AB at 2000 K with lam_A = lam_B = -17.6 (element potentials)
    g = _golden()["example2"]
    m = _Mech(g["W"], [[1, 1, 0]], [[0, 0, 1]], [math.log(g["A_cgs"])], [g["beta"]],
              [g["Ea_cal"]], _nasa(g["nasa_a1"], g["nasa_a6"]))
    m.atoms = np.array([[1, 0], [0, 1], [1, 1]], np.int8)
    P, Y = _equilibrium_state(m, 2000.0, [-17.6, -17.6])
    assert P / 101325.0 == pytest.approx(4.288, abs=2e-3)
    om, S, _ = oracle.source(m, [2000.0], [P], Y[:, None], precision="ld", scales=True)
    assert float(np.abs(om[:, 0] / S[:, 0]).max()) < 1e-15


@pytest.mark.parametrize("wl", ["c0", "c1"])
def test_atom_and_mass_conservation(wl):
    mech, T, P, Y = synth.workload(wl, n_cells=256)
    om, S, _ = oracle.source(mech, T, P, Y, scales=True)
    Wm = mech.W[:, None]
    mass = (Wm * om).sum(axis=0)
    assert np.all(np.abs(mass) <= 1e-13 * (Wm * S).sum(axis=0))
    A = mech.atoms.astype(float)
    for e in range(A.shape[1]):
        at = (A[:, e:e + 1] * om).sum(axis=0)
        assert np.all(np.abs(at) <= 1e-13 * (A[:, e:e + 1] * S).sum(axis=0) + 1e-300)


def test_homogeneous_in_Y():
    mech, T, P, Y = synth.workload("c1", n_cells=64)
    om, S, _ = oracle.source(mech, T, P, Y, scales=True)
    for lam in (0.37, 3.0):
        om2 = oracle.source(mech, T, P, lam * Y)
        assert np.all(np.abs(om2 - om) <= 1e-13 * S)


def test_zero_mass_fraction_is_exact_zero_concentration():
    mech, T, P, Y = synth.workload("c0", n_cells=8)
    Y = Y.copy()
    Y[2, :] = 0.0
    Y[5, 3] = -1e-9            # negative values clamp to zero
    r = oracle.rates(mech, float(T[3]), float(P[3]), Y[:, 3])
    assert r["C"][2] == 0.0 and r["C"][5] == 0.0
    uses2 = mech.nu_f[:, 2] > 0
    assert np.all(r["qf"][uses2] == 0.0)
    om = oracle.source(mech, T, P, Y)
    assert np.all(np.isfinite(om))


def test_ld_and_f64_agree():
    mech, T, P, Y = synth.workload("c1", n_cells=128)
    a, S, _ = oracle.source(mech, T, P, Y, scales=True)
    b = oracle.source(mech, T, P, Y, precision="ld")
    assert np.all(np.abs(a - b.astype(float)) <= 1e-13 * S)


# --------------------------------------------------------------------------
# 50-digit brute force on tiny mechanisms (Eqs. 2, 3, 5, 7, 8 directly)


def _brute_force_rates(mech, T, P, Y):
    """q_f and q_r of every reaction at 50 digits, straight from Eqs. 3, 5, 7, 8
    with the ideal-gas concentrations and the NASA-7 forms, at the caller's
    working precision (numerical differentiation raises it)."""
    T = mp.mpf(T)
    ns, nr = mech.nu_f.shape[1], mech.nu_f.shape[0]
    y = [max(mp.mpf(v), 0) / mp.mpf(float(w)) for v, w in zip(Y, mech.W)]
    C = [mp.mpf(P) / (RU * T) * v / sum(y) for v in y]
    H, S = [], []
    for k in range(ns):
        a = mech.nasa_high[k] if T >= mech.T_mid[k] else mech.nasa_low[k]
        a = [mp.mpf(float(x)) for x in a]
        H.append(a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5 + a[5] / T)
        S.append(a[0] * mp.log(T) + a[1] * T + a[2] * T ** 2 / 2 + a[3] * T ** 3 / 3 + a[4] * T ** 4 / 4 + a[6])
    qf, qr = [], []
    for j in range(nr):
        order = int(mech.nu_f[j].sum())
        A = mp.exp(mp.mpf(float(mech.ln_A[j]))) * mp.mpf("1e-3") ** (order - 1)
        kf = A * T ** mp.mpf(float(mech.beta[j])) * mp.exp(-mp.mpf(float(mech.Ea[j])) * mp.mpf("4.184") / RU_MOL / T)
        nu = [int(mech.nu_r[j, k]) - int(mech.nu_f[j, k]) for k in range(ns)]
        Kc = (PREF / (RU * T)) ** sum(nu) * mp.exp(sum(n * (S[k] - H[k]) for k, n in enumerate(nu)))
        qf.append(kf * mp.fprod(C[k] ** int(mech.nu_f[j, k]) for k in range(ns)))
        rev = mech.reversible is None or int(mech.reversible[j])
        qr.append(kf / Kc * mp.fprod(C[k] ** int(mech.nu_r[j, k]) for k in range(ns)) if rev else mp.mpf(0))
    return qf, qr


def _brute_force_scales(mech, T, P, Y):
    """(omega, S, N) at 50 digits from _brute_force_rates."""
    qf, qr = _brute_force_rates(mech, T, P, Y)
    ns, nr = mech.nu_f.shape[1], mech.nu_f.shape[0]
    om, S, N = [mp.mpf(0)] * ns, [mp.mpf(0)] * ns, [mp.mpf(0)] * ns
    for j in range(nr):
        for k in range(ns):
            nu = int(mech.nu_r[j, k]) - int(mech.nu_f[j, k])
            om[k] += nu * (qf[j] - qr[j])
            S[k] += abs(nu) * (qf[j] + qr[j])
            N[k] += abs(nu) * abs(qf[j] - qr[j])
    return om, S, N


def _brute_force_omega(mech, T, P, Y):
    mp.mp.dps = 50
    T = mp.mpf(T)
    ns, nr = mech.nu_f.shape[1], mech.nu_f.shape[0]
    y = [max(mp.mpf(float(v)), 0) / mp.mpf(float(w)) for v, w in zip(Y, mech.W)]
    C = [mp.mpf(P) / (RU * T) * v / sum(y) for v in y]
    H, S = [], []
    for k in range(ns):
        a = mech.nasa_high[k] if T >= mech.T_mid[k] else mech.nasa_low[k]
        a = [mp.mpf(float(x)) for x in a]
        H.append(a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5 + a[5] / T)
        S.append(a[0] * mp.log(T) + a[1] * T + a[2] * T ** 2 / 2 + a[3] * T ** 3 / 3 + a[4] * T ** 4 / 4 + a[6])
    om = [mp.mpf(0)] * ns
    for j in range(nr):
        order = int(mech.nu_f[j].sum())
        A = mp.exp(mp.mpf(float(mech.ln_A[j]))) * mp.mpf("1e-3") ** (order - 1)
        kf = A * T ** mp.mpf(float(mech.beta[j])) * mp.exp(-mp.mpf(float(mech.Ea[j])) * mp.mpf("4.184") / RU_MOL / T)
        nu = [int(mech.nu_r[j, k]) - int(mech.nu_f[j, k]) for k in range(ns)]
        Kc = (PREF / (RU * T)) ** sum(nu) * mp.exp(sum(n * (S[k] - H[k]) for k, n in enumerate(nu)))
        qf = kf * mp.fprod(C[k] ** int(mech.nu_f[j, k]) for k in range(ns))
        qr = kf / Kc * mp.fprod(C[k] ** int(mech.nu_r[j, k]) for k in range(ns))
        for k in range(ns):
            om[k] += nu[k] * (qf - qr)
    return om


def _ld_to_mp(x):
    return mp.mpf(np.format_float_scientific(np.longdouble(x), precision=24, unique=False))


@pytest.mark.parametrize("seed", [3, 6])
def test_brute_force_scales_tiny_mechanisms(seed):
    """The oracle's S and N against 50-digit brute force (with irreversible
    reactions, whose reverse rate is zero)."""
    mech = synth.make_mechanism(4, 3, seed=seed)
    mech.reversible = np.array([1, 0, 1], np.uint8)
    rng = np.random.default_rng(seed + 100)
    for _ in range(3):
        T = float(rng.uniform(600, 2900))
        P = float(rng.uniform(0.5, 30) * 101325)
        Y = rng.dirichlet(np.full(4, 0.7))
        om, S, N = oracle.source(mech, [T], [P], Y[:, None], precision="ld", scales=True)
        bo, bS, bN = _brute_force_scales(mech, T, P, Y)
        for k in range(4):
            assert abs(_ld_to_mp(om[k, 0]) - bo[k]) <= mp.mpf("1e-17") * bS[k] + mp.mpf("1e-300")
            assert abs(_ld_to_mp(S[k, 0]) - bS[k]) <= mp.mpf("1e-17") * bS[k] + mp.mpf("1e-300")
            assert abs(_ld_to_mp(N[k, 0]) - bN[k]) <= mp.mpf("1e-17") * bS[k] + mp.mpf("1e-300")


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_brute_force_tiny_mechanisms(seed):
    mech = synth.make_mechanism(4, 3, seed=seed)
    rng = np.random.default_rng(seed)
    for _ in range(4):
        T = float(rng.uniform(600, 2900))
        P = float(rng.uniform(0.5, 30) * 101325)
        Y = rng.dirichlet(np.full(4, 0.7))
        om, S, _ = oracle.source(mech, [T], [P], Y[:, None], precision="ld", scales=True)
        ref = _brute_force_omega(mech, T, P, Y)
        for k in range(4):
            err = abs(_ld_to_mp(om[k, 0]) - ref[k])
            assert err <= mp.mpf("1e-17") * _ld_to_mp(S[k, 0]) + mp.mpf("1e-300"), (k, err)


def test_brute_force_c0_cells():
    mech, T, P, Y = synth.workload("c0", n_cells=1024)
    idx = np.random.default_rng(11).choice(1024, 25, replace=False)
    om, S, _ = oracle.source(mech, T[idx], P[idx], Y[:, idx], scales=True)
    for c, i in enumerate(idx):
        ref = _brute_force_omega(mech, T[i], P[i], Y[:, i])
        for k in range(mech.n_species):
            # double rounding in exponent arguments of magnitude ~50 gives a few 1e-15
            assert abs(float(ref[k]) - om[k, c]) <= 5e-14 * S[k, c]


# --------------------------------------------------------------------------
# Jacobian


def _fd_jacobian(mech, T, P, Y):
    """Central differences of the oracle (f64), h = 1e-6 |x| per input."""
    ns = mech.n_species
    x0 = np.concatenate([Y, [T]])
    J = np.zeros((ns + 1, ns + 1))
    for c in range(ns + 1):
        h = 1e-6 * abs(x0[c])
        xp, xm = x0.copy(), x0.copy()
        xp[c] += h
        xm[c] -= h
        fp = np.concatenate([oracle.source(mech, [xp[ns]], [P], xp[:ns, None])[:, 0],
                             oracle.temp_source(mech, [xp[ns]], [P], xp[:ns, None])])
        fm = np.concatenate([oracle.source(mech, [xm[ns]], [P], xm[:ns, None])[:, 0],
                             oracle.temp_source(mech, [xm[ns]], [P], xm[:ns, None])])
        J[:, c] = (fp - fm) / (xp[c] - xm[c])
    return J


@pytest.mark.parametrize("wl,n", [("c0", 6), ("c1", 2)])
def test_jacobian_vs_finite_differences(wl, n):
    mech, T, P, Y = synth.workload(wl, n_cells=n)
    Ja = oracle.jacobian(mech, T, P, Y)
    ns = mech.n_species
    for i in range(n):
        Jf = _fd_jacobian(mech, float(T[i]), float(P[i]), Y[:, i])
        # scale: per row, the largest entry magnitude times the column's input size
        x = np.concatenate([Y[:, i], [T[i]]])
        scale = np.abs(Ja[i] * x[None, :]).max(axis=1, keepdims=True) / np.abs(x)[None, :]
        err = np.abs(Ja[i] - Jf) / scale
        assert float(err.max()) < 1e-5, (i, float(err.max()))
        assert ns + 1 == Ja.shape[1]


def test_jacobian_conservation_and_homogeneity():
    mech, T, P, Y = synth.workload("c1", n_cells=4)
    J = oracle.jacobian(mech, T, P, Y)
    ns = mech.n_species
    A = mech.atoms.astype(float)
    for i in range(4):
        Ji = J[i, :ns, :]
        mag = np.abs(Ji).max()
        # element rows: sum_k a_ke dω_k/dx = 0
        assert np.abs(A.T @ Ji).max() <= 1e-12 * mag * np.abs(A).max() * ns
        # degree-0 homogeneity in Y: J_Y . Y = 0
        JY = Ji[:, :ns] @ Y[:, i]
        assert np.abs(JY).max() <= 1e-12 * (np.abs(Ji[:, :ns]) @ np.abs(Y[:, i])).max()


@pytest.mark.parametrize("ns,nr", [(9, 21), (53, 325)])
def test_jacobian_at_equilibrium(ns, nr):
    """At detailed balance q_f = q_r = q for every reaction, so
    d omega / d ln C = -nu^T diag(q) nu (symmetric, negative semidefinite);
    the composition block of the (Y, T) Jacobian is that matrix times
    d ln C_l / d Y_m = delta_lm / Y_m - 1 / (sigma W_m), sigma = sum Y / W."""
    mech = synth.make_mechanism(ns, nr)
    rng = np.random.default_rng(11)
    for T in (1000.0, 2200.0):
        lam = rng.uniform(-14.0, -8.0, mech.n_elements)
        P, Y = _equilibrium_state(mech, T, lam)
        J = np.asarray(oracle.jacobian(mech, [T], [P], Y[:, None], precision="ld"), float)[0]
        q = np.asarray(oracle.rates(mech, T, P, Y, precision="ld")["qf"], float)
        nu = (mech.nu_r - mech.nu_f).astype(float)             # [reaction][species]
        K = -(nu.T * q) @ nu
        assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
        assert np.linalg.eigvalsh(K).max() <= 1e-10 * np.abs(K).max()
        W = mech.W.astype(float)
        sigma = float((Y / W).sum())
        dlnC = np.diag(1.0 / Y) - 1.0 / (sigma * W)[None, :]   # [l][m]
        expect = K @ dlnC
        got = J[:ns, :ns]
        scale = np.abs(K).max(axis=1, keepdims=True) * np.abs(dlnC).max()
        assert float((np.abs(got - expect) / scale).max()) < 1e-10, T


@pytest.mark.parametrize("case", ["example2", "tiny"])
def test_jacobian_gross_scale_definition(case):
    """The oracle's Jacobian gross scale S^J_kc = sum_j |nu_kj| (|d q_f/d x_c| +
    |d q_r/d x_c|) against the same definition evaluated with 50-digit
    numerical derivatives (mpmath) of the brute-force q_f and q_r of each
    reaction, x = (Y_1..Y_NS, T) at fixed P; the scale also bounds the
    entry: |J_kc| <= S^J_kc, and the temperature row's scale bounds its entry."""
    if case == "example2":
        g = _golden()["example2"]
        W = np.array(g["W"])
        X = np.array(g["X"])
        Y = X * W / (X * W).sum()
        mech = _Mech(W, [[1, 1, 0]], [[0, 0, 1]], [math.log(g["A_cgs"])], [g["beta"]],
                     [g["Ea_cal"]], _nasa(g["nasa_a1"], g["nasa_a6"]))
        T, P = g["T"], g["P"]
    else:
        mech = synth.make_mechanism(4, 3, seed=3)
        rng = np.random.default_rng(5)
        T, P, Y = 1700.0, 3.0e5, rng.dirichlet(np.full(4, 0.7))
    ns, nr = mech.nu_f.shape[1], mech.nu_f.shape[0]
    J, Ja = oracle.jacobian(mech, [T], [P], Y[:, None], precision="ld", scales=True)
    J, Ja = J[0], Ja[0]
    mp.mp.dps = 50
    x0 = [mp.mpf(float(v)) for v in Y] + [mp.mpf(T)]

    def rates_at(c, xc):
        x = list(x0)
        x[c] = xc
        return _brute_force_rates(mech, x[ns], P, x[:ns])

    dqf = [[None] * (ns + 1) for _ in range(nr)]
    dqr = [[None] * (ns + 1) for _ in range(nr)]
    for c in range(ns + 1):
        for j in range(nr):
            dqf[j][c] = mp.diff(lambda v: rates_at(c, v)[0][j], x0[c])
            dqr[j][c] = mp.diff(lambda v: rates_at(c, v)[1][j], x0[c])
    for k in range(ns):
        for c in range(ns + 1):
            sj = mp.mpf(0)
            for j in range(nr):
                nu = abs(int(mech.nu_r[j, k]) - int(mech.nu_f[j, k]))
                sj += nu * (abs(dqf[j][c]) + abs(dqr[j][c]))
            assert abs(_ld_to_mp(Ja[k, c]) - sj) <= mp.mpf("1e-15") * sj + mp.mpf("1e-300"), (k, c)
            assert abs(float(J[k, c])) <= float(Ja[k, c]) * (1 + 1e-15)
    for c in range(ns + 1):
        assert abs(float(J[ns, c])) <= float(Ja[ns, c]) * (1 + 1e-15)


def test_jacobian_ld_matches_f64():
    mech, T, P, Y = synth.workload("c0", n_cells=16)
    a = oracle.jacobian(mech, T, P, Y)
    b = oracle.jacobian(mech, T, P, Y, precision="ld").astype(float)
    scale = np.abs(b).max(axis=2, keepdims=True)
    assert float((np.abs(a - b) / scale).max()) < 1e-12
