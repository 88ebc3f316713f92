"""CHEMKIN mechanism files (the mechanism a kinetics code reads "through the
mechanism files", Sec. 2.2; pressure-dependent entries as in Sec. 2.4): the
parser against a hand-written file whose arrays are spelled out below, the
units keywords against their definitions, the refusals, and the round trip
write -> parse of the synthetic mechanisms (arrays, and the oracle's source
term on both).  Every rate constant and NASA coefficient here is invented.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2008_08483_amd import chemkin, synth

R_CAL = 8.31446261815324 / 4.184
N_A = 6.02214076e23


def _record(name, comp, tmid, hi, lo):
    """One fixed-format NASA-7 record (four 80-column lines)."""
    cf = "".join(f"{e:<2s}{n:>3d}" for e, n in comp)
    l1 = f"{name:<18s}INVENT{cf:<20s}G{300.0:10.3f}{5000.0:10.3f}{tmid:8.2f}"
    c = list(hi) + list(lo)
    fmt = lambda xs: "".join(f"{x:15.8E}" for x in xs)  # noqa: E731
    return [l1.ljust(79) + "1", fmt(c[0:5]).ljust(79) + "2", fmt(c[5:10]).ljust(79) + "3",
            fmt(c[10:14]).ljust(79) + "4"]


_SPECIES = ["H2", "O2", "H", "O", "OH", "H2O", "HO2", "N2", "AR"]
_COMP = {"H2": [("H", 2)], "O2": [("O", 2)], "H": [("H", 1)], "O": [("O", 1)],
         "OH": [("O", 1), ("H", 1)], "H2O": [("H", 2), ("O", 1)], "HO2": [("H", 1), ("O", 2)],
         "N2": [("N", 2)], "AR": [("AR", 1)]}


def _coeffs(k):
    hi = [3.1 + 0.1 * k, 1.25e-3, -3.5e-7, 4.5e-11, -2.5e-15, -950.0 * k - 100.0, 4.5 - 0.25 * k]
    lo = [3.3 + 0.05 * k, -2.5e-4, 1.5e-6, -7.5e-10, 1.25e-13, -975.0 * k - 50.0, 2.5 + 0.5 * k]
    return [float(f"{x:.8e}") for x in hi], [float(f"{x:.8e}") for x in lo]


def _thermo_block(t_mid_of=lambda k: 1000.0):
    out = ["THERMO ALL", "   300.000  1000.000  5000.000"]
    for k, s in enumerate(_SPECIES):
        hi, lo = _coeffs(k)
        out += _record(s, _COMP[s], t_mid_of(k), hi, lo)
    out.append("END")
    return out


_REACTIONS = """\
REACTIONS KCAL/MOLE
H + O2 <=> O + OH            3.1E+13   0.25   12.5   ! chain branching
O + H2 = H + OH              4.0E+04   2.5     5.75
2O + M <=> O2 + M            2.5E+17  -1.25    0.0
   H2/2.5/ H2O/12.0/ AR/0.75/
H + O2 (+M) <=> HO2 (+M)     3.5E+12   0.5     0.0
   LOW / 5.0E+19 -1.5 0.25 /
   TROE / 0.625 95.0 2750.0 6500.0 /
   H2O/10.5/ O2/0.875/
H + OH (+AR) <=> H2O (+AR)   1.5E+13   0.0     0.0
   LOW / 2.25E+18 -1.0 0.0 /
OH + OH => H2O + O           2.5E+04   2.25   -1.75
HO2 + H <=> 2OH              6.5E+13   0.0     0.375
DUPLICATE
HO2 + H <=> 2OH              1.25E+13  0.0     0.0
DUP
H + O2 (+M) <=> HO2 (+M)     1.0E+12   0.75    0.0
   LOW / 4.0E+18 -1.25 0.0 /
   TROE / 0.5 1.0E-30 1.0E+30 /
DUP
END
"""


def _text(reactions=_REACTIONS, thermo=None):
    head = ["! invented test mechanism", "ELEMENTS", "H O N AR", "END", "SPECIES",
            " ".join(_SPECIES), "END"]
    return "\n".join(head + (thermo or _thermo_block()) + [reactions])


def _idx(s):
    return _SPECIES.index(s)


def test_thermo_record_columns():
    # the fixed format: phase letter in column 45, T_mid in 66-73, line number in 80
    l1 = _record("H2O", _COMP["H2O"], 1000.0, *_coeffs(5))[0]
    assert len(l1) == 80 and l1[44] == "G" and l1[79] == "1"
    assert l1[24:34] == "H   2O   1" and float(l1[65:73]) == 1000.0


def test_hand_written_mechanism():
    m = chemkin.parse(_text(), name="invented")
    ns, nr = 9, 9
    assert m.species == _SPECIES and m.n_species == ns and m.n_reactions == nr
    # molecular weights: compositions times the conventional atomic weights
    aw = {"H": 1.008, "O": 15.999, "N": 14.007, "AR": 39.948}
    W = [sum(n * aw[e] for e, n in _COMP[s]) for s in _SPECIES]
    np.testing.assert_allclose(m.W, W, rtol=1e-15)
    # NASA-7: high range first in the file; T_mid from columns 66-73
    for k in range(ns):
        hi, lo = _coeffs(k)
        assert list(m.nasa_high[k]) == hi and list(m.nasa_low[k]) == lo
    assert np.all(m.T_mid == 1000.0)
    nu_f = np.zeros((nr, ns), int)
    nu_r = np.zeros((nr, ns), int)

    def put(nu, j, **c):
        for s, n in c.items():
            nu[j, _idx(s)] = n

    put(nu_f, 0, H=1, O2=1), put(nu_r, 0, O=1, OH=1)
    put(nu_f, 1, O=1, H2=1), put(nu_r, 1, H=1, OH=1)
    put(nu_f, 2, O=2), put(nu_r, 2, O2=1)
    put(nu_f, 3, H=1, O2=1), put(nu_r, 3, HO2=1)
    put(nu_f, 4, H=1, OH=1), put(nu_r, 4, H2O=1)
    put(nu_f, 5, OH=2), put(nu_r, 5, H2O=1, O=1)
    for j in (6, 7):
        put(nu_f, j, HO2=1, H=1), put(nu_r, j, OH=2)
    put(nu_f, 8, H=1, O2=1), put(nu_r, 8, HO2=1)
    assert np.array_equal(m.nu_f, nu_f) and np.array_equal(m.nu_r, nu_r)
    A = [3.1e13, 4.0e4, 2.5e17, 3.5e12, 1.5e13, 2.5e4, 6.5e13, 1.25e13, 1.0e12]
    assert np.array_equal(m.ln_A, np.log(A))
    assert list(m.beta) == [0.25, 2.5, -1.25, 0.5, 0.0, 2.25, 0.0, 0.0, 0.75]
    # KCAL/MOLE: E in cal/mol is 1000 times the file's number
    assert list(m.Ea) == [12500.0, 5750.0, 0.0, 0.0, 0.0, -1750.0, 375.0, 0.0, 0.0]
    assert list(m.reversible) == [1, 1, 1, 1, 1, 0, 1, 1, 1]
    # Sec. 2.4 entries: 1 third body, 2 Lindemann, 3 Troe
    assert list(m.rtype) == [0, 0, 1, 3, 2, 0, 0, 0, 3]
    eff = np.ones((nr, ns))
    eff[2, [_idx("H2"), _idx("H2O"), _idx("AR")]] = [2.5, 12.0, 0.75]
    eff[3, [_idx("H2O"), _idx("O2")]] = [10.5, 0.875]
    eff[4, :] = 0.0
    eff[4, _idx("AR")] = 1.0               # (+AR): only argon is the collider
    for j in (2, 3, 4, 8):
        assert np.array_equal(m.eff[j], eff[j]), j
    assert np.array_equal(m.low_ln_A[[3, 4, 8]], np.log([5.0e19, 2.25e18, 4.0e18]))
    assert list(m.low_beta[[3, 4, 8]]) == [-1.5, -1.0, -1.25]
    assert list(m.low_Ea[[3, 4, 8]]) == [250.0, 0.0, 0.0]
    assert list(m.troe[3]) == [0.625, 95.0, 2750.0, 6500.0]
    assert list(m.troe[8]) == [0.5, 1.0e-30, 1.0e30, 0.0]   # three numbers: no T**


def test_mechanism_without_pressure_dependence_has_no_tables():
    rx = "REACTIONS\nH + O2 <=> O + OH  3.1E+13 0.25 12500.0\nEND\n"
    m = chemkin.parse(_text(rx))
    assert m.rtype is None and m.eff is None and m.n_reactions == 1
    assert m.Ea[0] == 12500.0                      # default unit: cal/mol


@pytest.mark.parametrize("unit,factor", [("CAL/MOLE", 1.0), ("KCAL/MOLE", 1000.0),
                                         ("JOULES/MOLE", 1.0 / 4.184),
                                         ("KJOULES/MOLE", 1000.0 / 4.184),
                                         ("KELVINS", R_CAL)])
def test_energy_units(unit, factor):
    rx = f"REACTIONS {unit}\nH + O2 <=> O + OH  3.1E+13 0.25 12.5\nEND\n"
    m = chemkin.parse(_text(rx))
    assert m.Ea[0] == pytest.approx(12.5 * factor, rel=1e-15)


def test_molecules_unit():
    # A per molecule: times N_A^(order - 1), the order counting [M] for a third
    # body; a falloff LOW is one order above its k_inf
    rx = """REACTIONS MOLECULES KELVINS
H + O2 <=> O + OH            5.0E-11  0.0  8000.0
2O + M <=> O2 + M            5.0E-33  0.0  0.0
H + O2 (+M) <=> HO2 (+M)     2.0E-12  0.0  0.0
   LOW / 4.0E-32 0.0 0.0 /
OH => H + O                  3.0E+09  0.0  0.0
END
"""
    m = chemkin.parse(_text(rx))
    got = np.exp(m.ln_A)
    np.testing.assert_allclose(got, [5.0e-11 * N_A, 5.0e-33 * N_A**2, 2.0e-12 * N_A, 3.0e9],
                               rtol=1e-14)
    assert math.exp(m.low_ln_A[2]) == pytest.approx(4.0e-32 * N_A**2, rel=1e-14)
    assert m.Ea[0] == pytest.approx(8000.0 * R_CAL, rel=1e-15)


def test_element_weights_from_the_elements_block():
    text = _text().replace("H O N AR", "H/1.5/ O N AR")
    m = chemkin.parse(text)
    assert m.W[_idx("H2")] == 3.0 and m.W[_idx("OH")] == 1.5 + 15.999


def test_global_t_mid_and_record_t_mid():
    th = _thermo_block(lambda k: 1200.0 if k == 3 else 1000.0)
    m = chemkin.parse(_text(thermo=th))
    assert m.T_mid[3] == 1200.0 and m.T_mid[0] == 1000.0


_BAD = {
    "unknown species": "REACTIONS\nH + XX <=> O + OH  1.0E+13 0 0\nEND\n",
    "not supported": "REACTIONS\nH + O2 <=> O + OH  1.0E+13 0 0\n  PLOG / 1.0 1.0E+13 0 0 /\nEND\n",
    "falloff reaction without LOW": "REACTIONS\nH + O2 (+M) <=> HO2 (+M)  1.0E+12 0 0\nEND\n",
    "non-integer coefficient": "REACTIONS\n1.5H2 + O <=> H2O + H  1.0E+12 0 0\nEND\n",
    "unbalanced third body": "REACTIONS\n2O + M <=> O2  1.0E+12 0 0\nEND\n",
    "unbalanced falloff collider": "REACTIONS\nH + O2 (+M) <=> HO2 (+AR)  1.0E+12 0 0\n"
                                   "  LOW / 1.0E+18 0 0 /\nEND\n",
    "without [M]": "REACTIONS\nH + O2 <=> O + OH  1.0E+13 0 0\n  H2O/2.0/\nEND\n",
    "unknown REACTIONS unit": "REACTIONS FURLONGS\nH + O2 <=> O + OH  1.0E+13 0 0\nEND\n",
    "A <= 0": "REACTIONS\nH + O2 <=> O + OH  0.0 0 0\nEND\n",
    "no reactions": "REACTIONS\nEND\n",
}


@pytest.mark.parametrize("what", sorted(_BAD))
def test_refusals(what):
    with pytest.raises(chemkin.ChemkinError, match=what.replace("[", r"\[").replace("]", r"\]")):
        chemkin.parse(_text(_BAD[what]))


def test_missing_thermo_record():
    th = _thermo_block()
    i = th.index(next(ln for ln in th if ln.startswith("HO2 ")))
    del th[i:i + 4]
    with pytest.raises(chemkin.ChemkinError, match="no THERMO record for HO2"):
        chemkin.parse(_text(thermo=th))


def test_text_outside_a_block():
    with pytest.raises(chemkin.ChemkinError, match="outside a block"):
        chemkin.parse("H2 O2\n" + _text())


@pytest.mark.parametrize("pdep", [False, True])
def test_round_trip_of_the_synthetic_mechanisms(tmp_path, pdep):
    src = synth.make_mechanism(53, 325)
    if pdep:
        src = synth.with_pressure_dependence(src, frac=0.3)
    path = tmp_path / "mech.inp"
    path.write_text(chemkin.write(src))
    m = chemkin.load(str(path))
    assert m.name == "mech" and m.species == src.species
    for a in ("nu_f", "nu_r", "reversible", "atoms", "W", "T_mid", "ln_A", "beta", "Ea"):
        assert np.array_equal(getattr(m, a), getattr(src, a)), a
    # the THERMO format keeps 9 significant digits
    for a in ("nasa_low", "nasa_high"):
        np.testing.assert_allclose(getattr(m, a), getattr(src, a), rtol=1e-8, atol=0)
    if pdep:
        assert np.array_equal(m.rtype, src.rtype)
        p = src.rtype > 0
        f = src.rtype >= 2
        assert np.array_equal(m.eff[p], src.eff[p])
        assert np.array_equal(m.low_ln_A[f], src.low_ln_A[f])
        assert np.array_equal(m.low_beta[f], src.low_beta[f])
        assert np.array_equal(m.low_Ea[f], src.low_Ea[f])
        assert np.array_equal(m.troe[src.rtype == 3], src.troe[src.rtype == 3])
    else:
        assert m.rtype is None
    # the oracle's source term on both: equal up to the rounding of the NASA
    # coefficients (Eq. 10 -> Kc), i.e. to about 1e-8 of the gross rate
    T, P, Y = synth.make_states(src, 64, 5, (800.0, 2800.0), (1.0, 20.0), 0.3)
    a, S, _ = oracle.source(src, T, P, Y, scales=True)
    b = oracle.source(m, T, P, Y)
    assert np.max(np.abs(a - b) / np.maximum(S, 1e-300)) < 1e-6
