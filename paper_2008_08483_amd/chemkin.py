"""CHEMKIN-format mechanism files: the mechanism a kinetics code takes "through
the mechanism files" (Sec. 2.2: Arrhenius A, beta, E per reaction; Eq. 10's
NASA-7 polynomials per species), read into the arrays ``annkin.Mechanism``
loads, and written back from them.

Read: the ELEMENTS block (optional ``X/weight/`` atomic weights), SPECIES,
THERMO (NASA-7 records, fixed format: name and composition on the first line,
T_low / T_high / T_mid in columns 46-73, then 14 coefficients in 15-column
fields, high range first), and REACTIONS with the units keywords CAL/MOLE,
KCAL/MOLE, JOULES/MOLE, KJOULES/MOLE, KELVINS, MOLES and MOLECULES.  Reaction
lines carry the equation (``<=>`` or ``=`` reversible, ``=>`` irreversible,
integer stoichiometric prefixes such as ``2O``), then A, beta, E.  ``+M``
marks a third-body reaction and ``(+M)`` (or ``(+species)``) a falloff one;
the auxiliary lines ``species/efficiency/ ...``, ``LOW / A beta E /``,
``TROE / alpha T3 T1 [T2] /`` and ``DUPLICATE`` follow it (Sec. 2.4).  Other
auxiliary keywords (REV, PLOG, CHEB, SRI, FORD, ...) are refused, as are
non-integer coefficients.  '!' starts a comment.

Molecular weights come from the THERMO compositions and the atomic weights:
the ELEMENTS block's own, else the table below (IUPAC conventional values).
Units: A stays in cgs (mol, cm^3, s) and E in cal/mol, the descriptor's units
(``include/annkin.h``); MOLECULES multiplies A by N_A^(order-1).
"""

from __future__ import annotations

import math
import re

import numpy as np

from .synth import Mechanism

ATOMIC_WEIGHTS = {"H": 1.008, "D": 2.014, "HE": 4.0026, "C": 12.011, "N": 14.007,
                  "O": 15.999, "F": 18.998, "NE": 20.180, "SI": 28.085, "S": 32.06,
                  "CL": 35.45, "AR": 39.948, "KR": 83.798, "XE": 131.29}
CAL = 4.184                    # J per cal
R_CAL = 8.31446261815324 / CAL  # gas constant, cal/(mol K)
N_A = 6.02214076e23

_ENERGY = {"CAL/MOLE": 1.0, "KCAL/MOLE": 1000.0, "JOULES/MOLE": 1.0 / CAL,
           "KJOULES/MOLE": 1000.0 / CAL, "KELVINS": R_CAL, "EVOLTS": 96485.33212 / CAL}
_UNSUPPORTED = ("REV", "PLOG", "CHEB", "SRI", "FORD", "RORD", "HIGH", "UNITS", "LT", "RLT",
                "JAN", "FIT1", "TDEP", "XSMI", "EXCI", "MOME", "PCHEB", "TCHEB")


class ChemkinError(ValueError):
    pass


def _strip(text: str) -> list[str]:
    return [ln.split("!", 1)[0].rstrip() for ln in text.splitlines()]


def _sections(lines):
    """(keyword, header tokens, body lines) per block."""
    keys = {"ELEM": "ELEMENTS", "ELEMENTS": "ELEMENTS", "SPEC": "SPECIES", "SPECIES": "SPECIES",
            "THER": "THERMO", "THERMO": "THERMO", "REAC": "REACTIONS", "REACTIONS": "REACTIONS"}
    out, cur = [], None
    for ln in lines:
        toks = ln.split()
        head = toks[0].upper() if toks else ""
        if head in keys:
            cur = [keys[head], toks[1:], []]
            out.append(cur)
        elif head == "END" and len(toks) == 1:
            cur = None
        elif cur is not None:
            cur[2].append(ln)
        elif toks:
            raise ChemkinError(f"text outside a block: {ln!r}")
    return out


def _elements(tokens):
    names, weights = [], {}
    for t in tokens:
        m = re.fullmatch(r"([A-Za-z]+)(?:/\s*([-+0-9.eEdD]+)\s*/)?", t)
        if not m:
            raise ChemkinError(f"bad element entry {t!r}")
        e = m.group(1).upper()
        names.append(e)
        if m.group(2):
            weights[e] = float(m.group(2).replace("D", "E").replace("d", "e"))
    return names, weights


def _thermo(lines, header):
    """NASA-7 records: name -> (composition dict, T_mid, low[7], high[7])."""
    body = [ln for ln in lines if ln.strip()]
    i = 0
    t_mid_default = 1000.0
    # optional line of global T_low, T_mid, T_high
    if body and re.fullmatch(r"\s*[-+0-9.eE]+\s+[-+0-9.eE]+\s+[-+0-9.eE]+\s*", body[0]):
        t_mid_default = float(body[0].split()[1])
        i = 1
    out = {}
    while i < len(body):
        if i + 3 >= len(body):
            raise ChemkinError(f"truncated THERMO record at {body[i]!r}")
        l1, l2, l3, l4 = (body[i + q].ljust(80) for q in range(4))
        name = l1[:18].split()[0]
        comp = {}
        fields = [l1[24 + 5 * q:29 + 5 * q] for q in range(4)] + [l1[73:78]]
        for f in fields:
            el, cnt = f[:2].strip(), f[2:].strip()
            if el and el != "0" and cnt:
                n = int(float(cnt))
                if n:
                    comp[el.upper()] = comp.get(el.upper(), 0) + n
        t_mid = l1[65:73].strip()
        t_mid = float(t_mid) if t_mid else t_mid_default
        coef = []
        for ln in (l2, l3, l4):
            for q in range(5):
                s = ln[15 * q:15 * q + 15].strip()
                if s:
                    coef.append(float(s.replace("D", "E").replace("d", "e")))
        if len(coef) < 14:
            raise ChemkinError(f"THERMO record of {name} has {len(coef)} coefficients")
        out[name.upper()] = (name, comp, t_mid, np.array(coef[7:14]), np.array(coef[0:7]))
        i += 4
    return out


def _side(text, index):
    """{species index: count} of one side of an equation."""
    out = {}
    for term in text.split("+"):
        term = term.strip()
        if not term:
            raise ChemkinError(f"empty term in {text!r}")
        if re.fullmatch(r"\d*\.\d*\s*\S.*", term) and term.upper() not in index:
            raise ChemkinError(f"non-integer coefficient in {term!r}")
        m = re.fullmatch(r"(\d+)\s*(\S.*)", term)
        if m and m.group(2).upper() in index:
            n, sp = int(m.group(1)), m.group(2)
        else:
            n, sp = 1, term
        k = index.get(sp.upper())
        if k is None:
            raise ChemkinError(f"unknown species {sp!r}")
        out[k] = out.get(k, 0) + n
    return out


def parse(text: str, name: str = "mechanism") -> Mechanism:
    """A mechanism from CHEMKIN text (see the module docstring)."""
    secs = _sections(_strip(text))
    el_names, el_w = [], {}
    species = []
    thermo = {}
    reac_lines, reac_head = [], []
    for key, head, body in secs:
        toks = head + [t for ln in body for t in ln.split()]
        if key == "ELEMENTS":
            n, w = _elements(toks)
            el_names += n
            el_w.update(w)
        elif key == "SPECIES":
            species += toks
        elif key == "THERMO":
            thermo.update(_thermo(body, head))
        else:
            reac_head, reac_lines = head, body
    if not species:
        raise ChemkinError("no SPECIES block")
    index = {s.upper(): k for k, s in enumerate(species)}
    if len(index) != len(species):
        raise ChemkinError("a species is listed twice")
    ns = len(species)
    # thermo and molecular weights
    low = np.zeros((ns, 7))
    high = np.zeros((ns, 7))
    t_mid = np.zeros(ns)
    elements = list(dict.fromkeys(el_names))
    comps = []
    for k, s in enumerate(species):
        rec = thermo.get(s.upper())
        if rec is None:
            raise ChemkinError(f"no THERMO record for {s}")
        _, comp, tm, lo, hi = rec
        low[k], high[k], t_mid[k] = lo, hi, tm
        for e in comp:
            if e not in elements:
                elements.append(e)
        comps.append(comp)
    weights = []
    for e in elements:
        if e in el_w:
            weights.append(el_w[e])
        elif e in ATOMIC_WEIGHTS:
            weights.append(ATOMIC_WEIGHTS[e])
        else:
            raise ChemkinError(f"no atomic weight for element {e}")
    atoms = np.zeros((ns, len(elements)), dtype=np.int64)
    for k, comp in enumerate(comps):
        for e, n in comp.items():
            atoms[k, elements.index(e)] = n
    W = atoms.astype(np.float64) @ np.array(weights)
    if np.any(W <= 0):
        raise ChemkinError("a species has no atoms")
    # units of the REACTIONS block
    e_unit, molecules = 1.0, False
    for t in reac_head:
        u = t.upper()
        if u in _ENERGY:
            e_unit = _ENERGY[u]
        elif u == "MOLES":
            molecules = False
        elif u == "MOLECULES":
            molecules = True
        else:
            raise ChemkinError(f"unknown REACTIONS unit {t!r}")
    rx = []
    for ln in reac_lines:
        if not ln.strip():
            continue
        m = re.fullmatch(r"\s*(.*\S)\s+(\S+)\s+(\S+)\s+(\S+)\s*", ln)
        if m and "=" in m.group(1) and "/" not in m.group(1):
            try:
                A, beta, E = (float(x.replace("D", "E").replace("d", "e"))
                              for x in m.group(2, 3, 4))
            except ValueError:
                A = None
            if A is not None:
                rx.append({"eq": m.group(1), "A": A, "beta": beta, "E": E, "aux": []})
                continue
        if not rx:
            raise ChemkinError(f"auxiliary line before any reaction: {ln!r}")
        rx[-1]["aux"].append(ln)
    nr = len(rx)
    if nr == 0:
        raise ChemkinError("no reactions")
    nu_f = np.zeros((nr, ns), dtype=np.int64)
    nu_r = np.zeros((nr, ns), dtype=np.int64)
    ln_A = np.zeros(nr)
    beta = np.zeros(nr)
    Ea = np.zeros(nr)
    rev = np.ones(nr, dtype=np.uint8)
    rtype = np.zeros(nr, dtype=np.uint8)
    eff = np.ones((nr, ns))
    low_ln_A = np.zeros(nr)
    low_beta = np.zeros(nr)
    low_Ea = np.zeros(nr)
    troe = np.zeros((nr, 4))
    for j, r in enumerate(rx):
        eq = r["eq"]
        for sep, reversible in (("<=>", 1), ("=>", 0), ("=", 1)):
            if sep in eq:
                lhs, rhs = eq.split(sep, 1)
                break
        rev[j] = reversible
        third = None
        fo = re.compile(r"\(\s*\+\s*([^)\s]+)\s*\)")
        ml, mr = fo.search(lhs), fo.search(rhs)
        if ml or mr:
            if not (ml and mr) or ml.group(1).upper() != mr.group(1).upper():
                raise ChemkinError(f"unbalanced falloff collider in {eq!r}")
            third = ml.group(1).upper()
            lhs, rhs = fo.sub("", lhs), fo.sub("", rhs)
            rtype[j] = 2
        else:
            pl = [t.strip().upper() for t in lhs.split("+")]
            pr = [t.strip().upper() for t in rhs.split("+")]
            if "M" in pl or "M" in pr:
                if not ("M" in pl and "M" in pr):
                    raise ChemkinError(f"unbalanced third body in {eq!r}")
                lhs = "+".join(t for t in lhs.split("+") if t.strip().upper() != "M")
                rhs = "+".join(t for t in rhs.split("+") if t.strip().upper() != "M")
                third = "M"
                rtype[j] = 1
        f = _side(lhs, index)
        b = _side(rhs, index)
        for k, n in f.items():
            nu_f[j, k] = n
        for k, n in b.items():
            nu_r[j, k] = n
        order = sum(f.values()) + (1 if rtype[j] == 1 else 0)
        A = r["A"] * (N_A ** (order - 1) if molecules else 1.0)
        if A <= 0:
            raise ChemkinError(f"A <= 0 in {eq!r}")
        ln_A[j] = math.log(A)
        beta[j] = r["beta"]
        Ea[j] = r["E"] * e_unit
        if third not in (None, "M"):
            eff[j, :] = 0.0
            if third not in index:
                raise ChemkinError(f"unknown collider {third} in {eq!r}")
            eff[j, index[third]] = 1.0
        aux = " ".join(r["aux"])
        for m in re.finditer(r"([^\s/]+)\s*(?:/([^/]*)/)?", aux):
            key, val = m.group(1).upper(), m.group(2)
            if key in ("DUP", "DUPLICATE"):
                continue
            if key in _UNSUPPORTED:
                raise ChemkinError(f"{key} is not supported ({eq!r})")
            nums = [float(x.replace("D", "E").replace("d", "e")) for x in (val or "").split()]
            if key == "LOW":
                if rtype[j] < 2 or len(nums) != 3:
                    raise ChemkinError(f"LOW needs a falloff reaction and 3 numbers ({eq!r})")
                A0 = nums[0] * (N_A ** order if molecules else 1.0)
                low_ln_A[j], low_beta[j], low_Ea[j] = math.log(A0), nums[1], nums[2] * e_unit
                r["low"] = True
            elif key == "TROE":
                if rtype[j] < 2 or len(nums) not in (3, 4):
                    raise ChemkinError(f"TROE needs a falloff reaction and 3-4 numbers ({eq!r})")
                troe[j, :len(nums)] = nums
                rtype[j] = 3
            elif key.upper() in index:
                if rtype[j] == 0 or val is None or len(nums) != 1:
                    raise ChemkinError(f"efficiency {key} on a reaction without [M] ({eq!r})")
                eff[j, index[key]] = nums[0]
            else:
                raise ChemkinError(f"unknown auxiliary entry {key!r} ({eq!r})")
        if rtype[j] >= 2 and not r.get("low"):
            raise ChemkinError(f"falloff reaction without LOW ({eq!r})")
    pdep = bool(rtype.any())
    return Mechanism(
        name=name, W=W, atoms=atoms.astype(np.int8), nu_f=nu_f.astype(np.int8),
        nu_r=nu_r.astype(np.int8), ln_A=ln_A, beta=beta, Ea=Ea, nasa_low=low, nasa_high=high,
        T_mid=t_mid, reversible=rev, species=list(species),
        rtype=rtype if pdep else None, eff=eff if pdep else None,
        low_ln_A=low_ln_A if pdep else None, low_beta=low_beta if pdep else None,
        low_Ea=low_Ea if pdep else None, troe=troe if pdep else None)


def load(path: str) -> Mechanism:
    """parse() of a file (one file with all blocks)."""
    with open(path) as f:
        text = f.read()
    import os
    return parse(text, name=os.path.splitext(os.path.basename(path))[0])


def _e15(x: float) -> str:
    return f"{x:15.8E}"


def write(mech, elements=None, element_weights=None, t_low: float = 200.0,
          t_high: float = 6000.0) -> str:
    """CHEMKIN text of a mechanism's arrays (A in cgs, E in cal/mol).  The
    element names and weights default to the synthetic generator's; they go
    into the ELEMENTS block as ``X/weight/``."""
    from . import synth
    elements = list(elements or synth.ELEMENT_NAMES)
    weights = list(element_weights if element_weights is not None else synth.ELEMENT_MASSES)
    ns, nr = mech.n_species, mech.n_reactions
    names = list(mech.species) if mech.species else [f"S{k}" for k in range(ns)]
    out = ["ELEMENTS " + " ".join(f"{e}/{float(w)!r}/" for e, w in zip(elements, weights)), "END",
           "SPECIES"]
    for q in range(0, ns, 8):
        out.append("  " + " ".join(names[q:q + 8]))
    out += ["END", "THERMO"]
    for k in range(ns):
        comp = [(e, int(n)) for e, n in zip(elements, mech.atoms[k]) if n]
        if len(comp) > 4:
            raise ValueError("more than four elements in a species")
        cf = "".join(f"{e:<2s}{n:3d}" for e, n in comp).ljust(20)
        l1 = f"{names[k]:<18s}{'':6s}{cf}G{t_low:10.3f}{t_high:10.3f}{float(mech.T_mid[k]):8.2f}"
        out.append(l1.ljust(79) + "1")
        c = list(mech.nasa_high[k]) + list(mech.nasa_low[k])
        out.append("".join(_e15(x) for x in c[0:5]).ljust(79) + "2")
        out.append("".join(_e15(x) for x in c[5:10]).ljust(79) + "3")
        out.append("".join(_e15(x) for x in c[10:14]).ljust(79) + "4")
    out += ["END", "REACTIONS CAL/MOLE MOLES"]
    rtype = mech.rtype if getattr(mech, "rtype", None) is not None else np.zeros(nr, np.uint8)

    def side(nu, extra):
        terms = [f"{int(n) if n > 1 else ''}{names[k]}" for k, n in enumerate(nu) if n]
        return " + ".join(terms) + extra

    for j in range(nr):
        extra = " (+M)" if rtype[j] >= 2 else (" + M" if rtype[j] == 1 else "")
        sep = " <=> " if mech.reversible[j] else " => "
        eq = side(mech.nu_f[j], extra) + sep + side(mech.nu_r[j], extra)
        out.append(f"{eq}  {math.exp(mech.ln_A[j]):.15e} {float(mech.beta[j])!r} "
                   f"{float(mech.Ea[j])!r}")
        if rtype[j]:
            effs = [f"{names[k]}/{float(mech.eff[j, k])!r}/" for k in range(ns) if mech.eff[j, k] != 1.0]
            if effs:
                out.append("    " + " ".join(effs))
        if rtype[j] >= 2:
            out.append(f"    LOW / {math.exp(mech.low_ln_A[j]):.15e} {float(mech.low_beta[j])!r} "
                       f"{float(mech.low_Ea[j])!r} /")
        if rtype[j] == 3:
            t = mech.troe[j]
            vals = [repr(float(x)) for x in (t if t[3] != 0.0 else t[:3])]
            out.append("    TROE / " + " ".join(vals) + " /")
    out.append("END")
    return "\n".join(out) + "\n"
