"""Seeded synthetic inputs: reaction mechanisms and per-cell thermochemical fields.

This module is shared by the HIP path, the CPU oracle and the benchmark.  It
only draws random numbers and assembles input arrays; it contains none of the
method's arithmetic (no thermodynamics, kinetics, mixture fraction or
integration).  Every array it returns is plain numpy.

The paper runs a 54-species/269-reaction n-dodecane skeletal mechanism on an
OpenFOAM shear layer and an ECN spray (Sec. 4.1, 4.2).  Neither the mechanism
nor the cases are available, so these generators stand in for them with
mechanisms of the same size class and fields whose stiffness mix (a few hot,
igniting cells among many cold, near-reactant or near-oxidiser cells) has the
same structure as the paper's workloads (Sec. 2.3, 4.1).

Workloads (cells, species, reactions):
  small  :   4096 cells, 10 species / 20 reactions / 3 elements, no third body
  flame  :  65536 cells, 53 species / 325 reactions / 4 elements, 20% third body,
            10% hot igniting cells stored contiguously (worst static imbalance)
  mapped : 262144 cells, same 53-species mechanism, 60% cold near-oxidiser,
            30% mixing layer, 10% igniting, shuffled; 10 consecutive steps
  large  : 131072 cells, 130 species / 1000 reactions, bimodal like flame
  surrogate: 1048576 cells from the mapped distribution
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

ELEMENT_MASS = (1.008, 12.011, 15.999, 14.007)  # H, C, O, N  [g/mol]
P_ATM = 1.01325e6                                # dyn/cm^2

FUEL, OXIDISER, INERT = 0, 1, 2                  # reserved species indices


@dataclass
class Mechanism:
    """Host description of a synthetic mechanism (all arrays numpy, C order)."""
    n_elements: int
    n_species: int
    n_reactions: int
    elem_mass: np.ndarray          # [E] float64
    composition: np.ndarray        # [N, E] int32 atom counts
    W: np.ndarray                  # [N] float64 molar mass g/mol
    nasa: np.ndarray               # [N, 7] float64 (a1..a7), single range
    reactants: np.ndarray          # [R, 2] int32, -1 padded
    products: np.ndarray           # [R, 3] int32, -1 padded
    A: np.ndarray                  # [R] float64, CGS (cm^3/mol)^(order-1)/s
    b: np.ndarray                  # [R] float64 temperature exponent
    Ea: np.ndarray                 # [R] float64 J/mol
    third_body: np.ndarray         # [R] int32 0/1
    eff_reaction: np.ndarray       # [n_eff] int32  non-default third-body efficiencies
    eff_species: np.ndarray        # [n_eff] int32
    eff_value: np.ndarray          # [n_eff] float64
    seed: int = 0
    name: str = ""
    falloff: np.ndarray = None     # [R] int32 0 none, 1 Lindemann, 2 Troe (third-body reactions)
    fo_params: np.ndarray = None   # [R, 7] A0 (CGS), b0, Ea0 (J/mol), a, T3, T1, T2 (<= 0: absent)
    plog_count: np.ndarray = None  # [R] int32 0, or 2..8 tabulated pressures (PLOG reactions)
    plog_params: np.ndarray = None # [R, 8, 4] p_i (dyn/cm^2, increasing), A_i (CGS), b_i, Ea_i (J/mol)

    def arrays(self):
        keys = ["elem_mass", "composition", "W", "nasa", "reactants", "products",
                "A", "b", "Ea", "third_body", "eff_reaction", "eff_species", "eff_value"]
        if self.falloff is not None:
            keys += ["falloff", "fo_params"]
        if self.plog_count is not None:
            keys += ["plog_count", "plog_params"]
        return {k: getattr(self, k) for k in keys}

    def save(self, path):
        np.savez(path, n_elements=self.n_elements, n_species=self.n_species,
                 n_reactions=self.n_reactions, seed=self.seed, name=self.name,
                 **self.arrays())

    @staticmethod
    def load(path) -> "Mechanism":
        z = np.load(path, allow_pickle=False)
        kw = {k: z[k] for k in z.files if k not in ("n_elements", "n_species",
                                                    "n_reactions", "seed", "name")}
        return Mechanism(int(z["n_elements"]), int(z["n_species"]),
                         int(z["n_reactions"]), seed=int(z["seed"]),
                         name=str(z["name"]), **kw)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _draw_compositions(rng, n_species, n_elements, derived_frac):
    """Atom-count matrix [N, E] with counts 0..3, rows distinct and non-zero.

    Species 0 (fuel) carries carbon (element 1); the oxidiser (1) and the inert
    (2) carry none, so fuel and oxidiser streams differ in at least one element.
    A fraction of the remaining species is the sum of two earlier ones (when the
    sum stays within 0..3), which seeds association/dissociation pairs.
    """
    E = n_elements
    comp = []
    seen = set()

    def push(c):
        t = tuple(int(x) for x in c)
        if sum(t) == 0 or t in seen:
            return False
        seen.add(t)
        comp.append(np.array(t, dtype=np.int32))
        return True

    # fuel: carbon >= 1
    while True:
        c = rng.integers(0, 4, size=E)
        c[1] = rng.integers(1, 4)
        if push(c):
            break
    # oxidiser: no carbon, oxygen >= 1
    while True:
        c = rng.integers(0, 4, size=E)
        c[1] = 0
        c[2] = rng.integers(1, 4)
        if push(c):
            break
    # inert: no carbon, no oxygen (nitrogen-like when E == 4, else hydrogen-like)
    while True:
        c = np.zeros(E, dtype=np.int64)
        c[E - 1 if E == 4 else 0] = rng.integers(1, 4)
        if push(c):
            break
    while len(comp) < n_species:
        if len(comp) >= 4 and rng.random() < derived_frac:
            # sum of two earlier non-inert species, when it stays within 0..3
            cand = [(i, j) for i in range(len(comp)) for j in range(i, len(comp))
                    if i != INERT and j != INERT and (comp[i] + comp[j]).max() <= 3
                    and tuple(int(x) for x in comp[i] + comp[j]) not in seen]
            if cand:
                i, j = cand[int(rng.integers(0, len(cand)))]
                push(comp[i] + comp[j])
                continue
        c = rng.integers(0, 4, size=E)
        push(c)
    return np.stack(comp).astype(np.int32)


def _balanced_pairs(comp, inert):
    """All element-balanced (reactants, products) pairs.

    Reactant multisets have 1-2 species, product multisets 1-3, the two sides
    share no species, the inert species takes no part, and each reversible
    reaction is listed once (canonical orientation: the side usable as reactants
    with the smaller sorted tuple comes first when both orientations are valid).
    """
    N = comp.shape[0]
    species = [k for k in range(N) if k != inert]
    react_sets = [(a,) for a in species] + list(itertools.combinations_with_replacement(species, 2))
    prod_sets = react_sets + list(itertools.combinations_with_replacement(species, 3))
    by_comp = {}
    for ps in prod_sets:
        key = tuple(comp[list(ps)].sum(axis=0))
        by_comp.setdefault(key, []).append(ps)
    pairs = set()
    for rs in react_sets:
        key = tuple(comp[list(rs)].sum(axis=0))
        for ps in by_comp.get(key, ()):
            if ps == rs or set(ps) & set(rs):
                continue
            if len(ps) <= 2 and ps < rs:
                pair = (ps, rs)        # the reverse orientation is also valid
            else:
                pair = (rs, ps)
            pairs.add(pair)
    return sorted(pairs)


def make_mechanism(n_species: int, n_reactions: int, n_elements: int, seed: int,
                   third_body_frac: float = 0.2, name: str = "",
                   falloff_frac: float = 0.0, plog_frac: float = 0.0) -> Mechanism:
    """Seeded synthetic reversible mechanism (see module docstring).

    Thermo: a1 ~ U(2.5, 4.5) + (atoms - 1)/2; a2..a5 = u a1 / (8 T_MAX^(m-1)),
    u ~ U(-1, 1), so the cp polynomial stays within a1 +- a1/2 (cp > 0) up to
    T_MAX = 10000 K; a6 ~ U(-3e4, 3e4) K (heat-of-formation offset); a7 ~ U(0, 8).
    Each reaction is written in the direction in which its heat-of-formation
    offsets decrease (sum of nu_k a6_k < 0), as kinetic mechanisms are usually
    written, so reverse rates derived from equilibrium constants stay within
    physical bounds; pairs whose exothermic direction would need three reactants
    are not used.  Rates: A log-uniform in [1e6, 1e14], b ~ U(-1, 1),
    Ea ~ U(0, 200) kJ/mol.  Third-body reactions are association/dissociation
    pairs; up to three species per third-body reaction get an efficiency
    ~ U(0.5, 5), all others 1.
    Fall-off (falloff_frac of the third-body reactions, half Lindemann, half
    Troe): the reaction's Arrhenius form is the high-pressure limit, the
    low-pressure limit has A0 = A 10^U(4, 8) cm^3/mol (so Pr = k0 [M] / k_inf
    spans the fall-off region at 1 atm), b0 ~ U(-2, 0), Ea0 = Ea U(0.5, 1);
    Troe a ~ U(0.2, 0.9), T3 = 10^U(1.5, 3) K, T1 = 10^U(3, 4) K and, for half
    of them, T2 = 10^U(3, 4) K (else absent).  These draws come after all
    others, so a mechanism without fall-off is unchanged by the option.
    Pressure dependence by tabulation (PLOG; plog_frac of the reactions without
    a third body): 2 to 5 pressures log-uniform in [0.1, 100] atm, at each an
    Arrhenius form A 10^U(-1, 1), b + U(-0.3, 0.3), Ea U(0.8, 1.2).  These draws
    come last.
    """
    rng = _rng(seed)
    T_MAX = 10000.0
    n_tb_want = int(round(third_body_frac * n_reactions))
    for attempt in range(64):
        comp = _draw_compositions(rng, n_species, n_elements,
                                  derived_frac=min(0.9, 0.5 + 0.1 * attempt))
        atoms = comp.sum(axis=1)
        nasa = np.zeros((n_species, 7))
        nasa[:, 0] = rng.uniform(2.5, 4.5, size=n_species) + 0.5 * (atoms - 1)
        for m in range(1, 5):
            u = rng.uniform(-1.0, 1.0, size=n_species)
            nasa[:, m] = u * 0.5 * nasa[:, 0] / (4.0 * T_MAX ** m)
        nasa[:, 5] = rng.uniform(-3.0e4, 3.0e4, size=n_species)
        nasa[:, 6] = rng.uniform(0.0, 8.0, size=n_species)
        pairs = []
        for rs, ps in _balanced_pairs(comp, INERT):
            d = sum(nasa[k, 5] for k in ps) - sum(nasa[k, 5] for k in rs)
            if d < 0.0:
                pairs.append((rs, ps))
            elif len(ps) <= 2:
                pairs.append((ps, rs))
        n_assoc = sum(1 for rs, ps in pairs if (len(rs), len(ps)) in ((2, 1), (1, 2)))
        if len(pairs) >= n_reactions and n_assoc >= n_tb_want:
            break
    else:
        raise RuntimeError(f"could not find {n_reactions} balanced reactions")

    elem_mass = np.array(ELEMENT_MASS[:n_elements], dtype=np.float64)
    W = np.array([float(sum(int(comp[k, e]) * elem_mass[e] for e in range(n_elements)))
                  for k in range(n_species)])

    n_tb = n_tb_want
    assoc = [i for i, (rs, ps) in enumerate(pairs)
             if (len(rs), len(ps)) in ((2, 1), (1, 2))]
    n_tb = min(n_tb, len(assoc))
    tb_idx = list(rng.choice(np.array(assoc), size=n_tb, replace=False)) if n_tb else []
    rest = np.array(sorted(set(range(len(pairs))) - set(int(i) for i in tb_idx)))
    other_idx = list(rng.choice(rest, size=n_reactions - n_tb, replace=False))
    chosen = [(int(i), True) for i in tb_idx] + [(int(i), False) for i in other_idx]
    order = rng.permutation(len(chosen))
    chosen = [chosen[i] for i in order]

    R = n_reactions
    reactants = -np.ones((R, 2), dtype=np.int32)
    products = -np.ones((R, 3), dtype=np.int32)
    third = np.zeros(R, dtype=np.int32)
    eff_r, eff_s, eff_v = [], [], []
    for j, (pi, tb) in enumerate(chosen):
        rs, ps = pairs[pi]
        reactants[j, :len(rs)] = rs
        products[j, :len(ps)] = ps
        if tb:
            third[j] = 1
            n_eff = int(rng.integers(0, 4))
            for s in sorted(rng.choice(n_species, size=n_eff, replace=False)):
                eff_r.append(j)
                eff_s.append(int(s))
                eff_v.append(float(rng.uniform(0.5, 5.0)))
    A = 10.0 ** rng.uniform(6.0, 14.0, size=R)
    b = rng.uniform(-1.0, 1.0, size=R)
    Ea = rng.uniform(0.0, 200.0e3, size=R)
    falloff = fo_params = None
    if falloff_frac > 0.0:
        tbj = np.nonzero(third)[0]
        n_fo = int(round(falloff_frac * tbj.size))
        pick = np.sort(rng.choice(tbj, size=n_fo, replace=False))
        falloff = np.zeros(R, dtype=np.int32)
        fo_params = np.zeros((R, 7))
        for q, j in enumerate(pick):
            troe = q % 2 == 1
            falloff[j] = 2 if troe else 1
            fo_params[j, 0] = A[j] * 10.0 ** rng.uniform(4.0, 8.0)
            fo_params[j, 1] = rng.uniform(-2.0, 0.0)
            fo_params[j, 2] = Ea[j] * rng.uniform(0.5, 1.0)
            if troe:
                fo_params[j, 3] = rng.uniform(0.2, 0.9)
                fo_params[j, 4] = 10.0 ** rng.uniform(1.5, 3.0)
                fo_params[j, 5] = 10.0 ** rng.uniform(3.0, 4.0)
                fo_params[j, 6] = 10.0 ** rng.uniform(3.0, 4.0) if rng.uniform() < 0.5 else 0.0
    plog_count = plog_params = None
    if plog_frac > 0.0:
        free = np.nonzero(third == 0)[0]
        pick = np.sort(rng.choice(free, size=int(round(plog_frac * free.size)), replace=False))
        plog_count = np.zeros(R, dtype=np.int32)
        plog_params = np.zeros((R, 8, 4))
        for j in pick:
            cnt = int(rng.integers(2, 6))
            while True:
                e = np.sort(rng.uniform(-1.0, 2.0, size=cnt))
                if np.all(np.diff(e) > 0.05):
                    break
            plog_count[j] = cnt
            plog_params[j, :cnt, 0] = P_ATM * 10.0 ** e
            plog_params[j, :cnt, 1] = A[j] * 10.0 ** rng.uniform(-1.0, 1.0, size=cnt)
            plog_params[j, :cnt, 2] = b[j] + rng.uniform(-0.3, 0.3, size=cnt)
            plog_params[j, :cnt, 3] = Ea[j] * rng.uniform(0.8, 1.2, size=cnt)
    return Mechanism(n_elements, n_species, R, elem_mass, comp, W, nasa,
                     reactants, products, A, b, Ea, third,
                     np.array(eff_r, dtype=np.int32), np.array(eff_s, dtype=np.int32),
                     np.array(eff_v, dtype=np.float64), seed=seed, name=name,
                     falloff=falloff, fo_params=fo_params,
                     plog_count=plog_count, plog_params=plog_params)


# ----------------------------------------------------------------------------
# Named mechanisms and fields
# ----------------------------------------------------------------------------
MECH_SPECS = {
    "small": dict(n_species=10, n_reactions=20, n_elements=3, seed=1, third_body_frac=0.0),
    "mech53": dict(n_species=53, n_reactions=325, n_elements=4, seed=2, third_body_frac=0.2),
    "mech130": dict(n_species=130, n_reactions=1000, n_elements=4, seed=3, third_body_frac=0.2),
    # the two sides of the boundary between the one-wavefront integrator
    # (n = N + 1 <= 64) and the workgroup integrator
    "mech63": dict(n_species=63, n_reactions=400, n_elements=4, seed=4, third_body_frac=0.2),
    "mech64": dict(n_species=64, n_reactions=400, n_elements=4, seed=5, third_body_frac=0.2),
    # fall-off kinetics (Lindemann and Troe) on half of the third-body reactions
    "mech53fo": dict(n_species=53, n_reactions=325, n_elements=4, seed=6, third_body_frac=0.2,
                     falloff_frac=0.5),
    "mech64fo": dict(n_species=64, n_reactions=400, n_elements=4, seed=7, third_body_frac=0.2,
                     falloff_frac=0.5),
    # the two fall-off mechanisms with tabulated pressure dependence (PLOG) on
    # a fifth of the reactions without a third body (drawn last, so everything
    # else equals mech53fo / mech64fo)
    "mech53pl": dict(n_species=53, n_reactions=325, n_elements=4, seed=6, third_body_frac=0.2,
                     falloff_frac=0.5, plog_frac=0.2),
    "mech64pl": dict(n_species=64, n_reactions=400, n_elements=4, seed=7, third_body_frac=0.2,
                     falloff_frac=0.5, plog_frac=0.2),
}

_MECH_CACHE = {}


def mechanism(name: str) -> Mechanism:
    if name not in _MECH_CACHE:
        _MECH_CACHE[name] = make_mechanism(name=name, **MECH_SPECS[name])
    return _MECH_CACHE[name]


def stream_fuel(mech: Mechanism) -> np.ndarray:
    Y = np.zeros(mech.n_species)
    Y[FUEL] = 1.0
    return Y


def stream_oxidiser(mech: Mechanism) -> np.ndarray:
    """Oxidiser stream: 23% oxidiser species, 77% inert by mass (air analogue)."""
    Y = np.zeros(mech.n_species)
    Y[OXIDISER] = 0.23
    Y[INERT] = 0.77
    return Y


@dataclass
class Field:
    """Per-cell state, species-major (structure of arrays)."""
    T: np.ndarray          # [cells]
    p: np.ndarray          # [cells] dyn/cm^2
    Y: np.ndarray          # [N, cells]
    dt: float
    n_steps: int = 1
    cls: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int8))  # cell class
    class_names: tuple = ()

    @property
    def n_cells(self):
        return self.T.shape[0]


def _dirichlet(rng, alpha, n, cells):
    return rng.dirichlet(np.full(n, alpha), size=cells).T.copy()   # [n, cells]


def _hot_cells(rng, mech, cells):
    """Igniting, radical-rich cells: half a fuel/oxidiser mix, half Dirichlet(0.5)."""
    N = mech.n_species
    Z = rng.uniform(0.1, 0.9, size=cells)
    mix = np.outer(stream_fuel(mech), Z) + np.outer(stream_oxidiser(mech), 1.0 - Z)
    Y = 0.5 * mix + 0.5 * _dirichlet(rng, 0.5, N, cells)
    T = rng.uniform(1200.0, 2600.0, size=cells)
    return T, Y


def field_small(n_cells=4096, seed=101) -> Field:
    mech = mechanism("small")
    rng = _rng(seed)
    T = rng.uniform(800.0, 2000.0, size=n_cells)
    Y = _dirichlet(rng, 0.5, mech.n_species, n_cells)
    return Field(T, np.full(n_cells, P_ATM), Y, 1e-6, 1,
                 np.zeros(n_cells, np.int8), ("random",))


def field_bimodal(mech_name="mech53", n_cells=65536, seed=102, dt=1e-6, shuffle=False,
                  hot_last=False) -> Field:
    """10% hot igniting cells first (contiguous), 90% cold near-reactant cells;
    shuffle permutes the cells, hot_last puts the hot block at the end of the
    index range (the worst order for a launch that starts cells in index order)."""
    mech = mechanism(mech_name)
    N = mech.n_species
    rng = _rng(seed)
    n_hot = n_cells // 10
    n_cold = n_cells - n_hot
    Th, Yh = _hot_cells(rng, mech, n_hot)
    Ymix = np.zeros(N)
    Ymix[FUEL], Ymix[OXIDISER], Ymix[INERT] = 0.06, 0.22, 0.72
    eps = 1e-3
    Yc = (1.0 - eps) * Ymix[:, None] + eps * _dirichlet(rng, 0.5, N, n_cold)
    Tc = rng.uniform(300.0, 700.0, size=n_cold)
    T = np.concatenate([Th, Tc])
    Y = np.concatenate([Yh, Yc], axis=1)
    cls = np.concatenate([np.full(n_hot, 2, np.int8), np.zeros(n_cold, np.int8)])
    if shuffle:
        perm = rng.permutation(n_cells)
        T, Y, cls = T[perm], Y[:, perm], cls[perm]
    elif hot_last:
        perm = np.concatenate([np.arange(n_hot, n_cells), np.arange(n_hot)])
        T, Y, cls = T[perm], Y[:, perm], cls[perm]
    return Field(T, np.full(n_cells, P_ATM), np.ascontiguousarray(Y), dt, 1, cls,
                 ("cold", "mixing", "igniting"))


def field_mapped(n_cells=262144, seed=103, mech_name="mech53", n_steps=10) -> Field:
    """60% cold near-oxidiser (mappable), 30% mixing layer, 10% igniting; shuffled."""
    mech = mechanism(mech_name)
    N = mech.n_species
    rng = _rng(seed)
    n_cold = (6 * n_cells) // 10
    n_mix = (3 * n_cells) // 10
    n_hot = n_cells - n_cold - n_mix
    Yox, Yf = stream_oxidiser(mech), stream_fuel(mech)
    delta = rng.uniform(0.0, 5e-6, size=n_cold)
    Yc = (1.0 - delta)[None, :] * Yox[:, None] + delta[None, :] * _dirichlet(rng, 0.5, N, n_cold)
    Tc = rng.uniform(300.0, 500.0, size=n_cold)
    Z = rng.uniform(0.0, 1.0, size=n_mix)
    Ym = np.outer(Yox, 1.0 - Z) + np.outer(Yf, Z) + 1e-4 * _dirichlet(rng, 0.5, N, n_mix)
    Ym /= Ym.sum(axis=0, keepdims=True)
    Tm = (1.0 - Z) * 900.0 + Z * 400.0
    Th, Yh = _hot_cells(rng, mech, n_hot)
    T = np.concatenate([Tc, Tm, Th])
    Y = np.concatenate([Yc, Ym, Yh], axis=1)
    cls = np.concatenate([np.zeros(n_cold, np.int8), np.ones(n_mix, np.int8),
                          np.full(n_hot, 2, np.int8)])
    perm = rng.permutation(n_cells)
    return Field(T[perm], np.full(n_cells, P_ATM), np.ascontiguousarray(Y[:, perm]),
                 1e-6, n_steps, cls[perm], ("cold", "mixing", "igniting"))


# Load-balancing benchmark (Sec. 3): a fraction x of the processes (here the
# persistent slots) holds heavy problems at ratio theta; the rest hold light
# problems only; heavy problems are 1/5 of all problems in every layout.
UNIT_LAYOUTS = {"C1": (0.2, 1.0), "C2": (0.25, 0.8), "C3": (0.5, 0.4), "C4": (1.0, 0.2)}


def field_unit(layout, heavy, light, n_slots, n_per_slot, dt=1e-6):
    """Heavy/light pseudo-problem field: slot s owns cells [s B, (s + 1) B),
    B = n_per_slot; the first round(x n_slots) slots start with
    round(theta B) copies of the heavy problem, every other cell is a copy of
    the light problem.  heavy and light are (T, p, Y[N], h) tuples.  Returns
    (Field, h, is_heavy)."""
    x, theta = UNIT_LAYOUTS[layout]
    n = n_slots * n_per_slot
    is_heavy = np.zeros(n, bool)
    n_theta = int(round(x * n_slots))
    n_heavy = int(round(theta * n_per_slot))
    for s in range(n_theta):
        is_heavy[s * n_per_slot: s * n_per_slot + n_heavy] = True
    pick = lambda a, b: np.where(is_heavy, a, b)
    T = pick(heavy[0], light[0]).astype(np.float64)
    p = pick(heavy[1], light[1]).astype(np.float64)
    Y = np.where(is_heavy[None, :], np.asarray(heavy[2])[:, None], np.asarray(light[2])[:, None])
    h = pick(heavy[3], light[3]).astype(np.float64)
    f = Field(T, p, np.ascontiguousarray(Y, dtype=np.float64), dt, 1,
              is_heavy.astype(np.int8), ("light", "heavy"))
    return f, h, is_heavy


WORKLOADS = {
    "small": dict(mech="small", field=lambda n=4096: field_small(n)),
    "flame": dict(mech="mech53", field=lambda n=65536: field_bimodal("mech53", n, 102)),
    "flame_shuffled": dict(mech="mech53", field=lambda n=65536: field_bimodal("mech53", n, 102, shuffle=True)),
    "flame_hot_last": dict(mech="mech53", field=lambda n=65536: field_bimodal("mech53", n, 102, hot_last=True)),
    # the same field recipe with richer kinetics: fall-off, and fall-off plus PLOG
    "flame_falloff": dict(mech="mech53fo", field=lambda n=65536: field_bimodal("mech53fo", n, 102)),
    "flame_plog": dict(mech="mech53pl", field=lambda n=65536: field_bimodal("mech53pl", n, 102)),
    "mapped": dict(mech="mech53", field=lambda n=262144: field_mapped(n, 103)),
    "large": dict(mech="mech130", field=lambda n=131072: field_bimodal("mech130", n, 104, dt=2e-6)),
    "surrogate": dict(mech="mech53", field=lambda n=1048576: field_mapped(n, 105, n_steps=1)),
}


def subsample(f: Field, idx) -> Field:
    idx = np.asarray(idx)
    return Field(f.T[idx].copy(), f.p[idx].copy(), np.ascontiguousarray(f.Y[:, idx]), f.dt,
                 f.n_steps, f.cls[idx].copy() if f.cls.size else f.cls, f.class_names)


def stratified_indices(f: Field, per_class: int, seed: int = 7):
    """Seeded sample of up to per_class cells of every class present."""
    rng = _rng(seed)
    out = []
    for c in np.unique(f.cls):
        ids = np.nonzero(f.cls == c)[0]
        take = min(per_class, ids.size)
        out.append(np.sort(rng.choice(ids, size=take, replace=False)))
    return np.concatenate(out)


# ------------------------------------------------------- surrogate inputs ---
SUR_DIMS = (64, 256, 256, 256, 256, 64)   # padded layer widths of the surrogate network


def surrogate_params(n_species: int, seed: int = 0, weight_scale: float = 1.0,
                     out_sd=(4.0, 4.0), zero_output_weights=False, out_bias=None,
                     box=None) -> np.ndarray:
    """Seeded float32 parameter blob in the surrogate's layout, for tests.

    Layer l: W [out x in] ~ N(0, weight_scale^2 / in) on the live rows and
    columns (n_species + 3 inputs, n_species + 1 outputs), zero on the padding;
    b ~ N(0, 0.1^2) on live outputs.  zero_output_weights makes the output
    layer's W zero, so the network output equals its bias exactly; out_bias
    (n_species + 1 values) replaces that bias.  Normalisation: features
    centred on (ln 1000 K, ln 1 atm, 0.02, ln 1e-6 s) with spreads
    (0.5, 1, 0.1, 1); outputs with mean 0 and spreads out_sd = (species, T).
    box = (xmin, xmax) arrays of the N + 3 live features, or None for an
    unbounded box."""
    N = int(n_species)
    rng = _rng(seed)
    nfeat, nout = N + 3, N + 1
    blob = []
    for l in range(5):
        ni, no = SUR_DIMS[l], SUR_DIMS[l + 1]
        live_i = nfeat if l == 0 else ni
        live_o = nout if l == 4 else no
        W = np.zeros((no, ni))
        b = np.zeros(no)
        if not (l == 4 and zero_output_weights):
            W[:live_o, :live_i] = rng.standard_normal((live_o, live_i)) * weight_scale / np.sqrt(ni)
        b[:live_o] = rng.standard_normal(live_o) * 0.1
        if l == 4 and out_bias is not None:
            b[:nout] = out_bias
        blob += [W.ravel(), b]
    mu_x = np.zeros(64)
    sd_x = np.ones(64)
    mu_x[0], sd_x[0] = np.log(1000.0), 0.5
    mu_x[1], sd_x[1] = np.log(P_ATM), 1.0
    mu_x[2:2 + N], sd_x[2:2 + N] = 0.02, 0.1
    mu_x[2 + N], sd_x[2 + N] = np.log(1e-6), 1.0
    mu_o = np.zeros(64)
    sd_o = np.ones(64)
    sd_o[:N] = out_sd[0]
    sd_o[N] = out_sd[1]
    xmin = np.full(64, -1e30)
    xmax = np.full(64, 1e30)
    if box is not None:
        xmin[:nfeat] = box[0]
        xmax[:nfeat] = box[1]
    blob += [mu_x, sd_x, mu_o, sd_o, xmin, xmax]
    return np.concatenate(blob).astype(np.float32)


def surrogate_increment_bias(n_species: int, seed: int, dY_sd: float, dT_sd: float) -> np.ndarray:
    """Output-layer bias that, with zero output weights and unit output
    spreads, makes the network predict fixed increments dY ~ N(0, dY_sd^2) per
    species and dT ~ N(0, dT_sd^2): the increments in the output scale,
    asinh(dY / 1e-12) and asinh(dT / 1e-6 K)."""
    rng = _rng(seed)
    dY = rng.standard_normal(n_species) * dY_sd
    dT = rng.standard_normal() * dT_sd
    return np.r_[np.arcsinh(dY / 1e-12), np.arcsinh(dT / 1e-6)]


def surrogate_pairs_field(n_cells: int, seed: int = 900) -> Field:
    """Initial states for solver-generated training pairs: the mixed
    cold / mixing-layer / igniting distribution with its own seed."""
    return field_mapped(n_cells, seed, n_steps=1)


def surrogate_dt(n: int, seed: int, dt0=1e-6, lo=2.5e-7, hi=4e-6, levels=16):
    """Per-sample steps: half exactly dt0, half drawn uniformly from `levels`
    log-spaced values spanning [lo, hi] (a discrete log-uniform law, so that
    the solver runs one call per distinct step)."""
    rng = _rng(seed)
    dt = np.full(n, dt0)
    k = rng.permutation(n)[: n // 2]
    grid = np.exp(np.linspace(np.log(lo), np.log(hi), levels))
    dt[k] = grid[rng.integers(0, levels, size=k.size)]
    return dt
