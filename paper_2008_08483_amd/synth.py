"""Seeded synthetic inputs: mechanisms, cell states and request traces.

This module is shared by the test oracle and the HIP path as an *input*
source only.  It draws random numbers and does composition bookkeeping
(atom balance, molecular weights); it evaluates none of the source-term
arithmetic (no rate constants, no thermodynamic polynomials, no rates).

Mechanism form (Barwey & Raman, Sec. 2, Eq. 1): NS species, NR reversible
reactions  sum_k nu'_kj S_k <=> sum_k nu''_kj S_k.  Parameters are kept in
the units a CHEMKIN-style mechanism file carries:

* ``ln_A``   natural log of the pre-exponential factor in cgs units,
             (cm^3/mol)^(n-1) / s with n the reaction order (Eq. 5);
* ``beta``   temperature exponent (Eq. 5);
* ``Ea``     activation energy in cal/mol (Eq. 5);
* ``nasa_low``, ``nasa_high`` NASA 7-coefficient sets a1..a7 per species,
             split at ``T_mid`` (the temperature cutoff noted under Eq. 10).

Arrays use these layouts (row-major numpy):

* ``nu_f``, ``nu_r``  int8 [NR, NS]: reaction-major copies of the paper's
  NS x NR matrices nu' and nu'' (entry [j, k] is nu'_kj);
* ``atoms``           int8 [NS, NE];
* ``W``               float64 [NS], kg/kmol.

States: T [n] in K, P [n] in Pa, Y [NS, n] mass fractions (species-major,
cell index fastest: the transpose of the paper's N_C x N_S layout, with the
batch N_C as the leading dimension, Sec. 2.1).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Element masses, kg/kmol, for the three synthetic elements (H, C, O).
ELEMENT_MASSES = np.array([1.008, 12.011, 15.999])
ELEMENT_NAMES = ("H", "C", "O")
ATM = 101325.0

# Seeds for the fixed workloads.
MECH_SEEDS = {(9, 21): 0, (53, 325): 1, (111, 784): 2}


@dataclass
class Mechanism:
    """A synthetic, atom-balanced mechanism (all reactions reversible)."""

    name: str
    W: np.ndarray            # [NS] float64 kg/kmol
    atoms: np.ndarray        # [NS, NE] int8
    nu_f: np.ndarray         # [NR, NS] int8
    nu_r: np.ndarray         # [NR, NS] int8
    ln_A: np.ndarray         # [NR] float64, cgs units
    beta: np.ndarray         # [NR] float64
    Ea: np.ndarray           # [NR] float64, cal/mol
    nasa_low: np.ndarray     # [NS, 7] float64
    nasa_high: np.ndarray    # [NS, 7] float64
    T_mid: np.ndarray        # [NS] float64, K
    reversible: np.ndarray   # [NR] uint8
    species: list = field(default_factory=list)
    # pressure-dependent reactions (Sec. 2.4); None = all elementary
    rtype: np.ndarray | None = None      # [NR] uint8: 0 elementary, 1 third body, 2 Lindemann, 3 Troe
    eff: np.ndarray | None = None        # [NR, NS] third-body efficiencies
    low_ln_A: np.ndarray | None = None   # [NR] low-pressure limit (falloff), cgs of order + 1
    low_beta: np.ndarray | None = None
    low_Ea: np.ndarray | None = None
    troe: np.ndarray | None = None       # [NR, 4] alpha, T***, T*, T** (0: absent)

    @property
    def n_species(self) -> int:
        return int(self.W.shape[0])

    @property
    def n_reactions(self) -> int:
        return int(self.nu_f.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.atoms.shape[1])

    def arrays(self) -> dict:
        return {
            "W": self.W, "atoms": self.atoms, "nu_f": self.nu_f, "nu_r": self.nu_r,
            "ln_A": self.ln_A, "beta": self.beta, "Ea": self.Ea,
            "nasa_low": self.nasa_low, "nasa_high": self.nasa_high,
            "T_mid": self.T_mid, "reversible": self.reversible,
        }

    def save(self, path: str) -> None:
        np.savez(path, name=np.array(self.name), species=np.array(self.species),
                 **self.arrays())

    @staticmethod
    def load(path: str) -> "Mechanism":
        z = np.load(path, allow_pickle=False)
        kw = {k: z[k] for k in ("W", "atoms", "nu_f", "nu_r", "ln_A", "beta", "Ea",
                                "nasa_low", "nasa_high", "T_mid", "reversible")}
        return Mechanism(name=str(z["name"]), species=[str(s) for s in z["species"]], **kw)


def _compositions(ns: int, rng: np.random.Generator) -> np.ndarray:
    """Distinct compositions in {0,1,2}^3 minus the zero vector, repeated as
    isomers (same composition, independent thermodynamics) past 26."""
    base = [c for c in np.ndindex(3, 3, 3) if any(c)]
    base = np.array(base, dtype=np.int8)
    rng.shuffle(base)
    reps = int(math.ceil(ns / len(base)))
    comp = np.concatenate([base] * reps, axis=0)[:ns]
    return comp


def _nasa_sets(ns: int, n_atoms: np.ndarray, rng: np.random.Generator):
    """NASA-7 coefficient sets: an ideal-gas heat-capacity baseline that rises
    from about 3.5 R at 300 K to about 6 R at 3000 K (more for bigger
    molecules), each of a1..a5 scaled by (1 + U[-0.1, 0.1]) independently per
    range.  a6 and a7 are drawn directly; the two ranges are not forced to
    join at T_mid (each range is a separate set of Gibbs-layer weights)."""
    scale = 1.0 + 0.08 * (n_atoms - 2)
    # cp/R baseline per range as a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4
    lo_base = np.array([3.30, 1.10e-3, -2.0e-7, 8.0e-11, -1.2e-14])
    hi_base = np.array([3.60, 1.10e-3, -2.6e-7, 3.0e-11, -2.5e-15])
    low = np.zeros((ns, 7))
    high = np.zeros((ns, 7))
    for k in range(ns):
        low[k, :5] = lo_base * scale[k] * (1.0 + rng.uniform(-0.1, 0.1, 5))
        high[k, :5] = hi_base * scale[k] * (1.0 + rng.uniform(-0.1, 0.1, 5))
        a6 = rng.uniform(-6000.0, 6000.0)
        a7 = rng.uniform(-2.0, 12.0)
        low[k, 5] = a6
        low[k, 6] = a7
        high[k, 5] = a6 + rng.uniform(-150.0, 150.0)
        high[k, 6] = a7 + rng.uniform(-0.3, 0.3)
    return low, high


# reaction-side shapes: tuple of stoichiometric coefficients of its species,
# with a drawing weight
_SHAPES = (((1,), 0.22), ((2,), 0.04), ((1, 1), 0.60), ((2, 1), 0.10), ((2, 2), 0.04))


def make_mechanism(ns: int, nr: int, seed: int | None = None, name: str | None = None,
                   max_tries: int = 200, ln_A_range=(20.0, 35.0),
                   Ea_range=(0.0, 40000.0)) -> Mechanism:
    """Random atom-balanced reversible mechanism with ns species, nr reactions.

    Reactions have 1-2 reactant species and 1-2 product species with
    stoichiometric coefficients 1 or 2, reactant and product sides share the
    same atom vector, the two sides have no species in common, no reaction is
    drawn twice (in either direction), and every species takes part in at
    least one reaction.  Arrhenius: ln A ~ U[20, 35] (cgs), beta ~ U[-2, 2],
    Ea ~ U[0, 40000] cal/mol (``ln_A_range`` and ``Ea_range`` change the
    first and last).
    """
    if seed is None:
        seed = MECH_SEEDS.get((ns, nr), 0)
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        comp = _compositions(ns, rng)
        m = _try_reactions(ns, nr, comp, rng)
        if m is not None:
            nu_f, nu_r = m
            break
    else:  # pragma: no cover
        raise RuntimeError("could not draw a mechanism covering every species")
    n_atoms = comp.sum(axis=1)
    W = comp.astype(np.float64) @ ELEMENT_MASSES
    low, high = _nasa_sets(ns, n_atoms, rng)
    ln_A = rng.uniform(ln_A_range[0], ln_A_range[1], nr)
    beta = rng.uniform(-2.0, 2.0, nr)
    Ea = rng.uniform(Ea_range[0], Ea_range[1], nr)
    species = []
    count = {}
    for k in range(ns):
        key = tuple(int(x) for x in comp[k])
        count[key] = count.get(key, 0) + 1
        nm = "".join(f"{e}{n if n > 1 else ''}" for e, n in zip(ELEMENT_NAMES, key) if n)
        species.append(nm + ("" if count[key] == 1 else f"_i{count[key] - 1}"))
    return Mechanism(
        name=name or f"synthetic_{ns}sp_{nr}rxn_seed{seed}",
        W=W, atoms=comp.astype(np.int8), nu_f=nu_f, nu_r=nu_r,
        ln_A=ln_A, beta=beta, Ea=Ea, nasa_low=low, nasa_high=high,
        T_mid=np.full(ns, 1000.0), reversible=np.ones(nr, dtype=np.uint8),
        species=species)


def _try_reactions(ns, nr, comp, rng):
    shapes = [s for s, _ in _SHAPES]
    wts = np.array([w for _, w in _SHAPES])
    wts = wts / wts.sum()
    seen = set()
    # index of sides by atom vector, built lazily per shape pair
    by_atoms: dict = {}
    sides_all = []
    for shape in shapes:
        if len(shape) == 1:
            for a in range(ns):
                sides_all.append(((a, shape[0]),))
        else:
            for a in range(ns):
                for b in range(ns):
                    if a == b:
                        continue
                    if shape[0] == shape[1] and b < a:
                        continue
                    sides_all.append(((a, shape[0]), (b, shape[1])))
    for side in sides_all:
        vec = tuple(int(x) for x in sum(nu * comp[sp].astype(np.int64) for sp, nu in side))
        by_atoms.setdefault(vec, []).append(side)
    shape_of = {}
    for side in sides_all:
        shape_of.setdefault(tuple(nu for _, nu in side), []).append(side)
    reactions = []
    attempts = 0
    while len(reactions) < nr and attempts < 200 * nr:
        attempts += 1
        shp = shapes[rng.choice(len(shapes), p=wts)]
        pool = shape_of[shp]
        lhs = pool[rng.integers(len(pool))]
        vec = tuple(int(x) for x in sum(nu * comp[sp].astype(np.int64) for sp, nu in lhs))
        cands = by_atoms[vec]
        rhs = cands[rng.integers(len(cands))]
        if {s for s, _ in lhs} & {s for s, _ in rhs}:
            continue
        key = (tuple(sorted(lhs)), tuple(sorted(rhs)))
        rkey = (key[1], key[0])
        if key in seen or rkey in seen:
            continue
        seen.add(key)
        reactions.append((lhs, rhs))
    if len(reactions) < nr:
        return None
    nu_f = np.zeros((nr, ns), dtype=np.int8)
    nu_r = np.zeros((nr, ns), dtype=np.int8)
    for j, (lhs, rhs) in enumerate(reactions):
        for sp, nu in lhs:
            nu_f[j, sp] += nu
        for sp, nu in rhs:
            nu_r[j, sp] += nu
    if not np.all((nu_f + nu_r).sum(axis=0) > 0):
        return None
    return nu_f, nu_r


def with_pressure_dependence(mech: Mechanism, frac: float = 0.2, seed: int = 11,
                             types=(0.5, 0.2, 0.3)) -> Mechanism:
    """A copy of ``mech`` in which a fraction ``frac`` of the reactions are
    pressure dependent (Sec. 2.4): third-body (+M), Lindemann falloff or Troe
    falloff, in the proportions ``types``.  Reactions with one molecule on
    one side and two on the other (dissociation / recombination, the usual
    form of such reactions) are taken first.  Efficiencies are 1 except for
    those of one of three efficiency profiles drawn for the mechanism, as real
    mechanisms share a few (each: five species at 0, 0.5, 2 or 5; the first
    profile is taken by half of the reactions).  A third-body reaction's
    ln A, one order more, gets U[5, 10] added (termolecular constants are
    larger in cgs units); for falloff the drawn
    parameters are the high-pressure limit and the low-pressure limit gets
    ln A0 = ln A + U[8, 14] (one order more, so that the reduced pressure
    k0 [M] / k_inf spans the falloff region at 1-20 atm), beta0 = beta +
    U[-1, 0], E0 = E U[0.5, 1]; Troe: alpha ~ U[0.1, 0.9], T3 ~ U[50, 500] K,
    T1 ~ U[1000, 5000] K, T2 ~ U[2000, 8000] K for half of them (else
    absent)."""
    rng = np.random.default_rng(seed)
    nr, ns = mech.nu_f.shape
    nf = mech.nu_f.sum(axis=1)
    nb = mech.nu_r.sum(axis=1)
    pref = np.nonzero(((nf == 1) & (nb == 2)) | ((nf == 2) & (nb == 1)))[0]
    rest = np.setdiff1d(np.arange(nr), pref)
    cand = np.concatenate([rng.permutation(pref), rng.permutation(rest)])
    chosen = np.sort(cand[:int(round(frac * nr))])
    rtype = np.zeros(nr, np.uint8)
    kinds = rng.choice(3, size=chosen.size, p=np.asarray(types) / np.sum(types)) + 1
    rtype[chosen] = kinds
    profiles = np.ones((3, ns))
    for q in range(3):
        special = rng.choice(ns, size=min(5, ns), replace=False)
        profiles[q, special] = rng.choice([0.0, 0.5, 2.0, 5.0], size=special.size)
    eff = np.ones((nr, ns))
    for j in chosen:
        eff[j] = profiles[rng.choice(3, p=[0.5, 0.25, 0.25])]
    low_ln_A = mech.ln_A + rng.uniform(8.0, 14.0, nr)
    low_beta = mech.beta + rng.uniform(-1.0, 0.0, nr)
    low_Ea = mech.Ea * rng.uniform(0.5, 1.0, nr)
    troe = np.zeros((nr, 4))
    troe[:, 0] = rng.uniform(0.1, 0.9, nr)
    troe[:, 1] = rng.uniform(50.0, 500.0, nr)
    troe[:, 2] = rng.uniform(1000.0, 5000.0, nr)
    troe[:, 3] = np.where(rng.random(nr) < 0.5, rng.uniform(2000.0, 8000.0, nr), 0.0)
    fall = rtype >= 2
    ln_A = np.where(rtype == 1, mech.ln_A + rng.uniform(5.0, 10.0, nr), mech.ln_A)
    return Mechanism(
        name=mech.name + f"_pdep{int(round(100 * frac))}", W=mech.W, atoms=mech.atoms,
        nu_f=mech.nu_f, nu_r=mech.nu_r, ln_A=ln_A, beta=mech.beta, Ea=mech.Ea,
        nasa_low=mech.nasa_low, nasa_high=mech.nasa_high, T_mid=mech.T_mid,
        reversible=mech.reversible, species=list(mech.species), rtype=rtype,
        eff=np.where(rtype[:, None] > 0, eff, 1.0),
        low_ln_A=np.where(fall, low_ln_A, 0.0), low_beta=np.where(fall, low_beta, 0.0),
        low_Ea=np.where(fall, low_Ea, 0.0), troe=np.where((rtype == 3)[:, None], troe, 0.0))


# ----------------------------------------------------------------------------
# cell states

def make_states(mech: Mechanism, n_cells: int, seed: int, T_range=(800.0, 2800.0),
                P_atm=(1.0, 20.0), alpha: float = 0.3, floor: float = 1e-12,
                dtype=np.float64):
    """Random cell states: T ~ U[T_range], P ~ U[P_atm] atm (a scalar P_atm
    fixes P), Y ~ Dirichlet(alpha) floored at ``floor`` then renormalised.
    Returns (T [n], P [n], Y [NS, n]) in ``dtype``."""
    rng = np.random.default_rng(seed)
    ns = mech.n_species
    T = rng.uniform(T_range[0], T_range[1], n_cells)
    if np.isscalar(P_atm):
        P = np.full(n_cells, float(P_atm) * ATM)
    else:
        P = rng.uniform(P_atm[0], P_atm[1], n_cells) * ATM
    Y = rng.dirichlet(np.full(ns, alpha), size=n_cells)
    Y = np.maximum(Y, floor)
    Y /= Y.sum(axis=1, keepdims=True)
    Y = np.ascontiguousarray(Y.T)
    return T.astype(dtype), P.astype(dtype), Y.astype(dtype)


# Workload definitions (sizes and state distributions of the paper's
# mechanism classes, Tab. 1, scaled to the benchmark sizes).
WORKLOADS = {
    "c0": dict(ns=9, nr=21, n_cells=1024, T_range=(1000.0, 2500.0), P_atm=1.0, alpha=0.5,
               state_seed=1000),
    "c1": dict(ns=53, nr=325, n_cells=65536, T_range=(800.0, 2800.0), P_atm=(1.0, 20.0),
               alpha=0.3, state_seed=1001),
    "c1_full": dict(ns=53, nr=325, n_cells=1 << 20, T_range=(800.0, 2800.0),
                    P_atm=(1.0, 20.0), alpha=0.3, state_seed=1001),
    "c2": dict(ns=111, nr=784, n_cells=1 << 20, T_range=(800.0, 2800.0), P_atm=(1.0, 20.0),
               alpha=0.3, state_seed=1002),
    "c4": dict(ns=53, nr=325, n_cells=65536, T_range=(800.0, 2800.0), P_atm=(1.0, 20.0),
               alpha=0.3, state_seed=1004),
}


def workload(name: str, n_cells: int | None = None, dtype=np.float64):
    """(mechanism, T, P, Y) for a named workload, optionally truncated."""
    w = WORKLOADS[name]
    mech = make_mechanism(w["ns"], w["nr"])
    n = w["n_cells"] if n_cells is None else n_cells
    T, P, Y = make_states(mech, n, w["state_seed"], w["T_range"], w["P_atm"], w["alpha"],
                          dtype=dtype)
    return mech, T, P, Y


# ----------------------------------------------------------------------------
# request traces for the serving loop

def make_trace(n_requests: int, rate_per_s: float, seed: int = 2000,
               lo: int = 64, hi: int = 65536, n_mechs: int = 2):
    """Poisson arrivals at ``rate_per_s``; n_cells log-uniform in [lo, hi]
    (rounded); mechanism index uniform over ``n_mechs``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    t = np.cumsum(gaps)
    n = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(np.int64)
    mech = rng.integers(0, n_mechs, n_requests)
    return t, n, mech
