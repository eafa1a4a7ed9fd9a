"""Seeded synthetic inputs for the batched rMD / SCPS stepping workloads.

This module only *draws* inputs: chain conformations on a cubic lattice,
charges, masses, parameter sets and replica layouts.  It contains none of the
method's arithmetic (no contact function, no forces, no noise, no
integration), so both the FP64 CPU oracle (test infrastructure) and the HIP
library can consume the same inputs without sharing any computation.

Units for the protein-shaped workloads: Angstrom, picosecond, kJ/mol,
elementary charge.  Masses are given in kJ/mol * ps^2 / A^2 so that the
acceleration is simply F/m (1 amu = 0.01 in these units).  The small 20-bead
chain uses reduced units (kT = 1).

The paper's systems (Fip35 in an all-atom implicit-solvent force field, the
serpin fold) are not available; these chains stand in for them with the
sizes, contact-set sizes and step counts of the paper's protocol (section
"Realistic all-atom protein folding simulations", SCPS implementation steps
2-4).  Native conformations are compact self-avoiding walks on a 3.8 A cubic
lattice randomised by backbite moves; the reference contact map is whatever
the contact function gives on them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

SEED0 = 20170502
LATTICE = 3.8            # lattice spacing = bond length (A)
AMU = 0.01               # 1 amu in kJ/mol * ps^2 / A^2
KB_KJ = 0.0083144626     # Boltzmann constant, kJ/mol/K
KE_KJ = 1389.35458       # Coulomb constant, kJ * A / (mol * e^2)

_NEIGH = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0],
                   [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.int64)


# ---------------------------------------------------------------------------
# lattice conformations
# ---------------------------------------------------------------------------
def _boustrophedon(L: int, Lz: int) -> np.ndarray:
    """Hamiltonian path that snakes through an L x L x Lz box."""
    sites = []
    for z in range(Lz):
        rows = range(L) if z % 2 == 0 else range(L - 1, -1, -1)
        for k, y in enumerate(rows):
            xs = range(L) if (k + z * L) % 2 == 0 else range(L - 1, -1, -1)
            for x in xs:
                sites.append((x, y, z))
    return np.array(sites, dtype=np.int64)


def _backbite(path: np.ndarray, dims: np.ndarray, n_moves: int,
              rng: np.random.Generator) -> np.ndarray:
    """Randomise a Hamiltonian path of a box with backbite moves.

    A move picks one end of the path and a lattice neighbour of that end.
    If the neighbour is inside the box and is not the end's own path
    neighbour, the bond end-neighbour is added and the path is re-opened
    next to it, which reverses a prefix (or suffix) of the path.  Every
    site stays visited exactly once.  Sites are handled as integer ids of
    the box with a precomputed neighbour table.
    """
    n = len(path)
    L0, L1, L2 = (int(d) for d in dims)
    sid = (path[:, 0] * L1 + path[:, 1]) * L2 + path[:, 2]
    nsite = L0 * L1 * L2
    index = np.full(nsite, -1, dtype=np.int64)
    index[sid] = np.arange(n)
    g = np.arange(nsite)
    cx, cy, cz = g // (L1 * L2), (g // L2) % L1, g % L2
    neigh = np.full((nsite, 6), -1, dtype=np.int64)
    for k, (dx, dy, dz) in enumerate(_NEIGH):
        x, y, z = cx + dx, cy + dy, cz + dz
        inside = (x >= 0) & (x < L0) & (y >= 0) & (y < L1) & (z >= 0) & (z < L2)
        neigh[inside, k] = ((x * L1 + y) * L2 + z)[inside]
    neigh = neigh.tolist()
    ends = rng.random(n_moves) < 0.5
    dirs = rng.integers(6, size=n_moves)
    for end_first, dk in zip(ends.tolist(), dirs.tolist()):
        e = 0 if end_first else n - 1
        u = neigh[int(sid[e])][dk]
        if u < 0:
            continue
        j = int(index[u])
        if end_first:
            if j <= 1:
                continue
            seg = sid[:j][::-1].copy()
            sid[:j] = seg
            index[seg] = np.arange(j)
        else:
            if j >= n - 2:
                continue
            seg = sid[j + 1:][::-1].copy()
            sid[j + 1:] = seg
            index[seg] = np.arange(j + 1, n)
    return np.stack([sid // (L1 * L2), (sid // L2) % L1, sid % L2], axis=1)


def compact_native(n: int, seed: int) -> np.ndarray:
    """Compact self-avoiding chain of n beads, float64 [3][n] in Angstrom."""
    rng = np.random.default_rng(seed)
    L = max(2, int(math.ceil(n ** (1.0 / 3.0))))
    Lz = max(1, int(math.ceil(n / (L * L))))
    path = _boustrophedon(L, Lz)
    path = _backbite(path, np.array([L, L, Lz]), 10 * n, rng)
    xyz = path[:n].astype(np.float64) * LATTICE
    xyz -= xyz.mean(axis=0)
    return np.ascontiguousarray(xyz.T)


def straight_start(n: int, seed: int, jitter: float = 0.05) -> np.ndarray:
    """Extended chain along x with bond length 3.8 A plus seeded jitter."""
    rng = np.random.default_rng(seed)
    xyz = np.zeros((n, 3))
    xyz[:, 0] = np.arange(n) * LATTICE
    xyz += rng.normal(0.0, jitter, size=xyz.shape)
    xyz -= xyz.mean(axis=0)
    return np.ascontiguousarray(xyz.T)


def persistent_start(n: int, seed: int, persistence: float = 10.0,
                     jitter: float = 0.05) -> np.ndarray:
    """Self-avoiding lattice walk that keeps its direction for about
    `persistence` bonds before turning, plus seeded jitter.

    Non-bonded beads stay at least one lattice spacing apart, so the start
    carries no overlapping pairs; its extent is a few hundred Angstrom.
    """
    rng = np.random.default_rng(seed)
    p_turn = 1.0 / persistence
    steps = [tuple(int(c) for c in row) for row in _NEIGH]
    while True:
        cur = (0, 0, 0)
        pos = [cur]
        occ = {cur}
        d = steps[int(rng.integers(6))]
        ok = True
        for _ in range(n - 1):
            cand = []
            if rng.random() >= p_turn:
                cand.append(d)
            back = (-d[0], -d[1], -d[2])
            cand += [steps[k] for k in rng.permutation(6).tolist() if steps[k] != back]
            for c in cand:
                nxt = (cur[0] + c[0], cur[1] + c[1], cur[2] + c[2])
                if nxt not in occ:
                    pos.append(nxt)
                    occ.add(nxt)
                    cur = nxt
                    d = c
                    break
            else:
                ok = False
                break
        if ok:
            break
    xyz = np.array(pos, dtype=np.float64) * LATTICE
    xyz += rng.normal(0.0, jitter, size=xyz.shape)
    xyz -= xyz.mean(axis=0)
    return np.ascontiguousarray(xyz.T)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
@dataclass
class System:
    n: int
    contact_idx: np.ndarray      # int32 ascending local indices
    mass: np.ndarray             # float32 [n]
    charge: np.ndarray           # float32 [n]
    native: np.ndarray           # float64 [3][n]
    start: np.ndarray            # float64 [3][n]


@dataclass
class Workload:
    name: str
    params: Dict[str, float]
    systems: List[System]
    replica_system: np.ndarray   # int32 [R]
    n_steps: int
    record_every: int = 0
    iterations: int = 1
    notes: Dict[str, object] = field(default_factory=dict)

    # -- flat layouts shared by both consumers --------------------------------
    @property
    def n_replicas(self) -> int:
        return int(len(self.replica_system))

    def replica_sizes(self) -> np.ndarray:
        return np.array([self.systems[s].n for s in self.replica_system], dtype=np.int64)

    def replica_offsets(self) -> np.ndarray:
        """Start of each replica's [3][N_r] block, in particles (x3 floats)."""
        sz = self.replica_sizes()
        off = np.zeros(len(sz) + 1, dtype=np.int64)
        off[1:] = np.cumsum(sz)
        return off

    def initial_x(self) -> np.ndarray:
        """float32 flat buffer: replica r occupies [3*off_r, 3*off_{r+1}) as [3][N_r].  Every replica
        starts from its system's start state unless notes["replica_starts"] gives one per replica."""
        own = self.notes.get("replica_starts")
        if own is not None:
            blocks = [np.asarray(own[r], dtype=np.float32).ravel() for r in range(self.n_replicas)]
        else:
            blocks = [self.systems[s].start.astype(np.float32).ravel() for s in self.replica_system]
        return np.ascontiguousarray(np.concatenate(blocks))

    def initial_v(self, seed: int) -> np.ndarray:
        """Maxwell-Boltzmann velocities drawn with numpy (an input, not the method's noise)."""
        rng = np.random.default_rng(seed)
        kT = self.params["kT"]
        out = []
        for s in self.replica_system:
            m = self.systems[s].mass.astype(np.float64)
            out.append((rng.normal(size=(3, len(m))) * np.sqrt(kT / m)).astype(np.float32).ravel())
        return np.ascontiguousarray(np.concatenate(out))

    def initial_cvstate(self) -> np.ndarray:
        """float64 [R][8]; running minima start at +inf so the first evaluation sets them."""
        cv = np.zeros((self.n_replicas, 8), dtype=np.float64)
        cv[:, 1] = np.inf
        cv[:, 5] = np.inf
        cv[:, 6] = np.inf
        return cv


def _base_params(**kw) -> Dict[str, float]:
    p = dict(integrator=1, bias_mode=0, dt=0.002, gamma=1.0, kT=KB_KJ * 300.0,
             k_bond=100.0, r_bond=LATTICE, lj_eps=1.0, lj_sigma=4.0,
             dh_prefactor=KE_KJ / 80.0, dh_kappa=0.1, nb_excl=2, min_seq_sep=0,
             r0_contact=7.5, r_cut_contact=0.0, r_cut_nb=0.0, k_R=1e-4, lam=13.5, k_s=2.5,
             k_w=2.5e-4, seed=SEED0)
    p.update(kw)
    return p


def config1(n_replicas: int = 16, n_steps: int = 1000) -> Workload:
    """20-bead chain, reduced units, overdamped Langevin, FP64-feasible."""
    cfg = 1
    n = 20
    sys0 = System(
        n=n,
        contact_idx=np.arange(n, dtype=np.int32),
        mass=np.ones(n, dtype=np.float32),
        charge=np.zeros(n, dtype=np.float32),
        native=compact_native(n, SEED0 + 1000 * cfg),
        start=straight_start(n, SEED0 + 3000 * cfg),
    )
    # m * gamma = 10 (mass 1, gamma 10): the overdamped chain with k = 100 is
    # stable at dt = 0.01 only for m*gamma well above 2.
    params = _base_params(integrator=0, dt=0.01, gamma=10.0, kT=1.0, dh_prefactor=0.0,
                          k_R=0.01, seed=SEED0 + cfg)
    return Workload("chain20_overdamped", params, [sys0],
                    np.zeros(n_replicas, dtype=np.int32), n_steps)


def config2(n_replicas: int = 256, n_steps: int = 10000) -> Workload:
    """560-particle chain (35 groups of 16), contacts over the 280 heavy particles."""
    cfg = 2
    n = 560
    local = np.arange(n) % 16
    heavy = local < 8
    rng = np.random.default_rng(SEED0 + 2000 * cfg)
    sys0 = System(
        n=n,
        contact_idx=np.nonzero(heavy)[0].astype(np.int32),
        mass=np.where(heavy, 12.011, 1.008).astype(np.float32) * AMU,
        charge=rng.normal(0.0, 0.3, size=n).astype(np.float32),
        native=compact_native(n, SEED0 + 1000 * cfg),
        start=straight_start(n, SEED0 + 3000 * cfg),
    )
    params = _base_params(seed=SEED0 + cfg)
    return Workload("chain560_fip35_shaped", params, [sys0],
                    np.zeros(n_replicas, dtype=np.int32), n_steps)


def config3(n_replicas: int = 512, n_steps: int = 1000, n_min: int = 200,
            n_max: int = 3000) -> Workload:
    """Uneven batch: every replica is its own chain with N ~ U{n_min..n_max}."""
    cfg = 3
    rng = np.random.default_rng(SEED0 + 4000 * cfg)
    sizes = rng.integers(n_min, n_max + 1, size=n_replicas)
    systems = []
    for s, n in enumerate(sizes):
        n = int(n)
        crng = np.random.default_rng(SEED0 + 2000 * cfg + s)
        systems.append(System(
            n=n,
            contact_idx=np.arange(n, dtype=np.int32),
            mass=np.full(n, 12.011 * AMU, dtype=np.float32),
            charge=crng.normal(0.0, 0.3, size=n).astype(np.float32),
            native=compact_native(n, SEED0 + 1000 * cfg + s),
            start=persistent_start(n, SEED0 + 3000 * cfg + s),
        ))
    params = _base_params(seed=SEED0 + cfg)
    return Workload("uneven_chains_200_3000", params, systems,
                    np.arange(n_replicas, dtype=np.int32), n_steps)


def config4(n_chains: int = 64, n: int = 3000) -> Workload:
    """Differentiation workload: chains of 3000 particles, no stepping."""
    cfg = 4
    systems = []
    for s in range(n_chains):
        systems.append(System(
            n=n,
            contact_idx=np.arange(n, dtype=np.int32),
            mass=np.full(n, 12.011 * AMU, dtype=np.float32),
            charge=np.zeros(n, dtype=np.float32),
            native=compact_native(n, SEED0 + 1000 * cfg + s),
            start=persistent_start(n, SEED0 + 3000 * cfg + s),
        ))
    params = _base_params(seed=SEED0 + cfg, dh_prefactor=0.0)
    return Workload("autograd_chains_3000", params, systems,
                    np.arange(n_chains, dtype=np.int32), 0)


def config5(n_replicas: int = 32, n: int = 6000, n_steps: int = 10000,
            record_every: int = 200, iterations: int = 5) -> Workload:
    """Serpin-scale chain (400 residues x 15 particles), SCPS iterations."""
    cfg = 5
    rng = np.random.default_rng(SEED0 + 2000 * cfg)
    sys0 = System(
        n=n,
        contact_idx=np.arange(n, dtype=np.int32),
        mass=np.full(n, 12.011 * AMU, dtype=np.float32),
        charge=rng.normal(0.0, 0.3, size=n).astype(np.float32),
        native=compact_native(n, SEED0 + 1000 * cfg),
        start=persistent_start(n, SEED0 + 3000 * cfg),
    )
    params = _base_params(seed=SEED0 + cfg)
    return Workload("chain6000_serpin_shaped", params, [sys0],
                    np.zeros(n_replicas, dtype=np.int32), n_steps,
                    record_every=record_every, iterations=iterations)


def config6(n_replicas: int = 32, n: int = 6000, r_cut: float = 12.0) -> Workload:
    """Cutoff variant: config 5's chain under rMD with the contact and the
    nonbonded terms cut at r_cut (the paper's 1.2 nm), started from compact
    states (the native fold with 0.05 A of seeded jitter per coordinate, one
    draw per replica), where a cutoff removes the fewest pairs."""
    cfg = 6
    base = config5(n_replicas=1, n=n)
    sy = base.systems[0]
    rng = np.random.default_rng(SEED0 + 3000 * cfg)
    starts = [sy.native + rng.normal(0.0, 0.05, size=sy.native.shape) for _ in range(n_replicas)]
    sys0 = System(n=n, contact_idx=sy.contact_idx, mass=sy.mass, charge=sy.charge, native=sy.native,
                  start=starts[0])
    params = _base_params(seed=SEED0 + cfg, r_cut_contact=r_cut, r_cut_nb=r_cut)
    return Workload("chain6000_cutoff", params, [sys0], np.zeros(n_replicas, dtype=np.int32), 1000,
                    notes={"replica_starts": np.stack(starts)})


def funnel_params(**kw) -> Dict[str, float]:
    """The toy model's parameters: Table 1 of the paper (the asymmetric funnel
    of eq (U)), kT = 0.3 and the overdamped step gamma dt = 0.02 (read as
    dt / (m gamma)), rMD with k_R = 70 on z = |X|, the tube variables with
    lambda = 0.3 and k_s = k_w = 3; start (0, 5) on the outer ring."""
    p = dict(A1=30.0, A2=20.0, A3=6.0, s1=1.0, s2=2.0, s3=0.5, w=0.03, xm=1.5, ym=0.0,
             kT=0.3, mob_dt=0.02, bias_mode=0, k_R=70.0, lam=0.3, k_s=3.0, k_w=3.0, seed=SEED0 + 7)
    p.update(kw)
    return p


FUNNEL_START = (0.0, 5.0)


def random_coil(n: int, seed: int) -> np.ndarray:
    """A non-native state: a persistent lattice walk, float64 [3][n]."""
    return persistent_start(n, seed)
