"""Seeded synthetic chemical mechanisms (input data only).

The paper's own mechanisms (a 9-species H2/O2 set and GRI-Mech 3.0) are not
available, so the workloads use synthetic stand-ins of the same shape: a
9-species H/O/N species set with 21 reversible Arrhenius reactions and a
21-species C/H/O/N set with 84 reactions.  This module only *draws numbers*:
species compositions, molecular weights from atomic weights, single-range
NASA-7 style polynomial coefficients, and candidate Arrhenius parameters.
It evaluates none of the method's formulas (no thermodynamics, no rates).

Which candidate draws make up a mechanism is decided once by a screening
script that lives with the test fixtures; the accepted (reaction, attempt)
pairs are stored as JSON and read back here by ``build``.
"""
import itertools
import json
import os

import numpy as np

# atomic weights, kg/mol
ATOMIC_WEIGHT = {"H": 1.008e-3, "C": 12.011e-3, "N": 14.007e-3, "O": 15.999e-3}

SPECIES_SETS = {
    # H/O/N-shaped set of nine species (N2 is an inert bath gas)
    "HON9": [
        ("H2", {"H": 2}), ("O2", {"O": 2}), ("H", {"H": 1}), ("O", {"O": 1}),
        ("OH", {"O": 1, "H": 1}), ("H2O", {"H": 2, "O": 1}),
        ("HO2", {"H": 1, "O": 2}), ("H2O2", {"H": 2, "O": 2}), ("N2", {"N": 2}),
    ],
    # C/H/O/N-shaped set of 21 species
    "CHON21": [
        ("H2", {"H": 2}), ("O2", {"O": 2}), ("H", {"H": 1}), ("O", {"O": 1}),
        ("OH", {"O": 1, "H": 1}), ("H2O", {"H": 2, "O": 1}),
        ("HO2", {"H": 1, "O": 2}), ("H2O2", {"H": 2, "O": 2}),
        ("CO", {"C": 1, "O": 1}), ("CO2", {"C": 1, "O": 2}),
        ("HCO", {"H": 1, "C": 1, "O": 1}), ("CH2O", {"C": 1, "H": 2, "O": 1}),
        ("CH3", {"C": 1, "H": 3}), ("CH4", {"C": 1, "H": 4}),
        ("CH2", {"C": 1, "H": 2}), ("CH", {"C": 1, "H": 1}),
        ("C2H2", {"C": 2, "H": 2}), ("C2H4", {"C": 2, "H": 4}),
        ("C2H6", {"C": 2, "H": 6}), ("CH3O", {"C": 1, "H": 3, "O": 1}),
        ("N2", {"N": 2}),
    ],
}

ELEMENTS = ("H", "C", "N", "O")

# Arrhenius parameter ranges (config): A in [1e8, 1e14] (CGS-mole units of the
# forward order), Ea in [0, 40] kcal/mol, b range per mechanism kind.
KIND = {
    "mech9": dict(species="HON9", nr=21, b=(-1.0, 2.0), le=None, bulk=0.0),
    "mech21": dict(species="CHON21", nr=84, b=(-2.0, 3.0), le=None, bulk=0.0),
    # test-only variant: non-unity Lewis numbers and bulk viscosity exercise
    # the correction-velocity and bulk-viscosity code paths
    "mech9le": dict(species="HON9", nr=21, b=(-1.0, 2.0), le=(0.8, 1.2), bulk=0.6),
}

CAL = 4.184
T_LO, T_HI = 200.0, 3500.0


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def composition_matrix(species):
    return np.array([[sp[1].get(e, 0) for e in ELEMENTS] for sp in species], dtype=np.int64)


def molecular_weights(species):
    return np.array([sum(n * ATOMIC_WEIGHT[e] for e, n in comp.items()) for _, comp in species])


def candidate_reactions(species):
    """All element-balanced reactions with one or two reactants and one or two
    products (a species may appear twice, giving a coefficient of 2), listed
    once per unordered pair of sides, with no species on both sides."""
    ns = len(species)
    comp = composition_matrix(species)
    sides = [(a,) for a in range(ns)] + [tuple(c) for c in itertools.combinations_with_replacement(range(ns), 2)]
    out = []
    for r, p in itertools.combinations(sides, 2):
        if set(r) & set(p):
            continue
        if not np.array_equal(comp[list(r)].sum(0), comp[list(p)].sum(0)):
            continue
        out.append((r, p))
    return out


def cp_polynomial(rng):
    """Coefficients a1..a5 of a smooth c_p/R(T) that increases monotonically
    from c_lo at T_LO to c_hi at T_HI, with 2.5 <= c_lo < c_hi <= 7."""
    c_lo = rng.uniform(2.5, 4.5)
    c_hi = rng.uniform(c_lo + 0.5, 7.0)
    w = rng.dirichlet(np.ones(4))
    # monotone basis on s in [0,1]: s, 2s-s^2, 3s^2-2s^3, s^4
    poly_s = np.array([0.0, w[0] + 2 * w[1], -w[1] + 3 * w[2], -2 * w[2], w[3]])
    poly_s *= (c_hi - c_lo)
    poly_s[0] += c_lo
    # substitute s = (T - T_LO)/(T_HI - T_LO)
    sub = np.polynomial.Polynomial([-T_LO / (T_HI - T_LO), 1.0 / (T_HI - T_LO)])
    poly_t = np.polynomial.Polynomial([0.0])
    for i, c in enumerate(poly_s):
        poly_t = poly_t + c * sub ** i
    a = np.zeros(5)
    a[: len(poly_t.coef)] = poly_t.coef
    return a


def species_data(kind, seed):
    spec = KIND[kind]
    species = SPECIES_SETS[spec["species"]]
    ns = len(species)
    nasa = np.zeros((ns, 7))
    le = np.ones(ns)
    for k in range(ns):
        rng = _rng(seed, 11, k)
        nasa[k, :5] = cp_polynomial(rng)
        nasa[k, 5] = rng.uniform(-6000.0, 4000.0)   # enthalpy constant a6, K
        nasa[k, 6] = rng.uniform(2.0, 12.0)         # entropy constant a7
        if spec["le"] is not None:
            le[k] = rng.uniform(*spec["le"])
    return species, molecular_weights(species), nasa, le


def candidate_order(kind, seed):
    species = SPECIES_SETS[KIND[kind]["species"]]
    cands = candidate_reactions(species)
    perm = _rng(seed, 17).permutation(len(cands))
    return cands, perm


def draw_arrhenius(kind, seed, cand_index, attempt):
    """One candidate draw (A_SI, b, Ea in J/mol) for candidate reaction
    ``cand_index``; ``attempt`` indexes independent redraws."""
    spec = KIND[kind]
    rng = _rng(seed, 23, cand_index, attempt)
    log10a = rng.uniform(8.0, 14.0)
    b = rng.uniform(*spec["b"])
    ea = rng.uniform(0.0, 40.0) * 1000.0 * CAL
    return log10a, b, ea


def assemble(kind, seed, chosen):
    """Mechanism dict from the list of chosen (candidate index, attempt)."""
    spec = KIND[kind]
    species, W, nasa, le = species_data(kind, seed)
    cands, _ = candidate_order(kind, seed)
    ns = len(species)
    nr = len(chosen)
    nu_f = np.zeros((nr, ns), dtype=np.int32)
    nu_r = np.zeros((nr, ns), dtype=np.int32)
    A = np.zeros(nr)
    b = np.zeros(nr)
    Ea = np.zeros(nr)
    for j, (ci, att) in enumerate(chosen):
        r, p = cands[ci]
        for s in r:
            nu_f[j, s] += 1
        for s in p:
            nu_r[j, s] += 1
        log10a, bj, ea = draw_arrhenius(kind, seed, ci, att)
        order = int(nu_f[j].sum())
        # CGS-mole units ((cm^3/mol)^(n-1)/s) converted to SI (m^3/mol)
        A[j] = 10.0 ** (log10a - 6.0 * (order - 1))
        b[j] = bj
        Ea[j] = ea
    return dict(
        kind=kind, seed=int(seed), species=[s[0] for s in species], ns=ns, nr=nr,
        W=W, nasa=nasa, Tlo=T_LO, Thi=T_HI, A=A, b=b, Ea=Ea, nu_f=nu_f, nu_r=nu_r,
        Le=le, mu_ref=1.8e-5, T_ref=300.0, mu_exp=0.7, Pr=0.7, bulk_ratio=spec["bulk"],
        m47=3557.0 / 44100.0, m48=-2083.0 / 117600.0,
        composition=composition_matrix(species), chosen=[list(c) for c in chosen],
    )


MANIFEST_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "tests", "golden", "manifest")


def load(kind):
    """Mechanism ``kind`` from its stored reaction selection."""
    if kind in SUBSETS:
        base, names = SUBSETS[kind]
        return subset(load(base), names, kind)
    with open(os.path.join(MANIFEST_DIR, f"{kind}.json")) as f:
        sel = json.load(f)
    return assemble(kind, sel["seed"], [tuple(c) for c in sel["chosen"]])


# mechanisms that keep a subset of another's species and the reactions among
# them (element balance and the screening carry over): a CO/H2/O2-shaped
# 12-species set from the 21-species mechanism
SUBSETS = {
    "mech12": ("mech21", ["H2", "O2", "H", "O", "OH", "H2O", "HO2", "H2O2", "CO", "CO2", "HCO", "N2"]),
}


def subset(m, names, kind):
    """Mechanism ``m`` restricted to the species ``names`` (in that order)
    and to the reactions whose reactants and products are all among them."""
    idx = [m["species"].index(s) for s in names]
    keep = np.zeros(m["ns"], bool)
    keep[idx] = True
    rows = [j for j in range(m["nr"]) if not ((m["nu_f"][j] > 0) | (m["nu_r"][j] > 0))[~keep].any()]
    out = dict(m)
    out.update(
        kind=kind, species=list(names), ns=len(idx), nr=len(rows),
        W=np.asarray(m["W"])[idx], nasa=np.asarray(m["nasa"])[idx], Le=np.asarray(m["Le"])[idx],
        A=np.asarray(m["A"])[rows], b=np.asarray(m["b"])[rows], Ea=np.asarray(m["Ea"])[rows],
        nu_f=np.ascontiguousarray(np.asarray(m["nu_f"])[rows][:, idx]),
        nu_r=np.ascontiguousarray(np.asarray(m["nu_r"])[rows][:, idx]),
        composition=np.asarray(m["composition"])[idx],
        chosen=[m["chosen"][j] for j in rows],
    )
    return out


def small_test_mechanism(seed=5, ns_keep=None):
    """Unscreened mechanism over the HON9 species with every candidate
    reaction and mild fixed rate parameters, for pointwise invariant tests."""
    species, W, nasa, le = species_data("mech9", seed)
    cands, perm = candidate_order("mech9", seed)
    chosen = [(int(ci), 0) for ci in perm[:8]]
    m = assemble("mech9", seed, chosen)
    return m
