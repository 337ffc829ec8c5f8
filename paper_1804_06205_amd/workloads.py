"""Seeded synthetic inputs for the DPD step: fluids, diblock melts, peptide-like
chains in solvent, the alpha-helix deck, and the replica request stream.

This module only draws inputs (positions, velocities, types, bond lists,
parameters, arrival times).  It holds none of the method's arithmetic: no
force, integrator or binning code lives here.  Both the HIP library's tests and
the oracle's tests take their inputs from it.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` in FP64:

* positions uniform in [0, L)^3;
* velocities N(0, kT) per component, minus their mean (zero net momentum);
* chains: first bead uniform, every next bead the previous one plus ``b``
  times a uniform unit vector, wrapped into the box;
* tags are the generation order: chain beads first, then solvent.

The paper's workloads are synthetic boxes at reduced density 3 (performance
section; alpha-helix section); these generators stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Bond type codes shared with the C ABI (include/dpd.h).
BOND_HARMONIC = 1      # Eq. (6) of the paper
BOND_MORSE_PAPER = 2   # Eq. (7) of the paper, modified Morse with |r - r_e|
BOND_MORSE = 3         # standard Morse U = D[(1 - e^{-alpha(r - r0)})^2 - 1]


@dataclasses.dataclass
class Workload:
    """A complete DPD input: box, state, types, pair table, bonds, parameters."""
    name: str
    L: tuple
    pos: np.ndarray            # (n, 3) float64, in [0, L)
    vel: np.ndarray            # (n, 3) float64
    types: np.ndarray          # (n,) uint8
    ntypes: int
    a: np.ndarray              # (ntypes, ntypes) float64, symmetric
    gamma: float = 4.5
    sigma: float = 3.0
    kT: float = 1.0
    dt: float = 0.04
    lam: float = 0.65
    seed: int = 1
    steps: int = 100
    btype: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    bi: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int64))
    bj: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int64))
    r_e: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.float64))
    k: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.float64))
    alpha: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.float64))
    precision: str = "mixed"   # "fp64" or "mixed"

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nbonds(self) -> int:
        return int(self.btype.shape[0])

    def params(self) -> dict:
        return dict(a=self.a, gamma=self.gamma, sigma=self.sigma, kT=self.kT,
                    dt=self.dt, lam=self.lam)

    def bonds(self) -> dict:
        return dict(btype=self.btype, bi=self.bi, bj=self.bj, r_e=self.r_e,
                    k=self.k, alpha=self.alpha)

    def copy(self) -> "Workload":
        return dataclasses.replace(
            self, pos=self.pos.copy(), vel=self.vel.copy(), types=self.types.copy(),
            a=self.a.copy(), btype=self.btype.copy(), bi=self.bi.copy(),
            bj=self.bj.copy(), r_e=self.r_e.copy(), k=self.k.copy(),
            alpha=self.alpha.copy())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _into_box(x: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Reduce coordinates into [0, L) (input preparation only)."""
    x = np.mod(x, L)
    x = np.where(x >= L, x - L, x)
    return np.where(x < 0, 0.0, x)


def _velocities(rng: np.random.Generator, n: int, kT: float) -> np.ndarray:
    v = rng.normal(0.0, math.sqrt(kT), size=(n, 3))
    v -= v.mean(axis=0, keepdims=True)
    return v


def _unit_vectors(rng: np.random.Generator, m: int) -> np.ndarray:
    z = rng.uniform(-1.0, 1.0, size=m)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=m)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def _walk(rng: np.random.Generator, nchains: int, nbeads: int, b: float,
          L: np.ndarray) -> np.ndarray:
    """Random-walk chains, (nchains*nbeads, 3), chain-major bead order."""
    start = rng.uniform(0.0, 1.0, size=(nchains, 1, 3)) * L
    steps = _unit_vectors(rng, nchains * (nbeads - 1)).reshape(nchains, nbeads - 1, 3) * b
    pos = np.concatenate([start, start + np.cumsum(steps, axis=1)], axis=1)
    return _into_box(pos.reshape(-1, 3), L)


def _quantize(rng: np.random.Generator, pos: np.ndarray, L: np.ndarray, q: int) -> np.ndarray:
    """Round positions down to multiples of 2^-q and redraw duplicate sites."""
    scale = float(2 ** q)
    grid = np.floor(pos * scale).astype(np.int64)
    ncell = (np.asarray(L) * scale).astype(np.int64)
    while True:
        key = (grid[:, 2] * ncell[1] + grid[:, 1]) * ncell[0] + grid[:, 0]
        _, first = np.unique(key, return_index=True)
        dup = np.ones(len(key), bool)
        dup[first] = False
        if not dup.any():
            break
        grid[dup] = np.floor(rng.uniform(0.0, 1.0, size=(int(dup.sum()), 3)) * ncell).astype(np.int64)
    return grid.astype(np.float64) / scale


def _bond_arrays(records):
    if not records:
        return (np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0, np.int64),
                np.zeros(0), np.zeros(0), np.zeros(0))
    rec = list(zip(*records))
    return (np.asarray(rec[0], np.int32), np.asarray(rec[1], np.int64),
            np.asarray(rec[2], np.int64), np.asarray(rec[3], np.float64),
            np.asarray(rec[4], np.float64), np.asarray(rec[5], np.float64))


def _box(L) -> np.ndarray:
    """Box edges from a scalar (cubic box) or three edges."""
    Lv = np.asarray(L, np.float64).reshape(-1)
    return np.repeat(Lv, 3) if Lv.shape[0] == 1 else Lv.copy()


def _box_name(Lv: np.ndarray) -> str:
    if Lv[0] == Lv[1] == Lv[2]:
        return f"{Lv[0]:g}"
    return "x".join(f"{v:g}" for v in Lv)


def fluid(L=10.0, rho: float = 3.0, seed: int = 1, kT: float = 1.0,
          a: float = 25.0, quantize: int | None = None, precision: str = "mixed",
          name: str | None = None, **kw) -> Workload:
    """Single-species fluid: N = round(rho * V) beads uniform in the box (L a
    scalar for a cubic box, or three edges)."""
    Lv = _box(L)
    n = int(round(rho * float(np.prod(Lv))))
    rng = _rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(n, 3)) * Lv
    pos = _into_box(pos, Lv)
    if quantize is not None:
        pos = _quantize(rng, pos, Lv, quantize)
    vel = _velocities(rng, n, kT)
    return Workload(name=name or f"fluid_L{_box_name(Lv)}", L=tuple(float(v) for v in Lv),
                    pos=pos, vel=vel, types=np.zeros(n, np.uint8), ntypes=1,
                    a=np.array([[a]]), kT=kT, seed=seed, precision=precision, **kw)


def melt(L: float = 32.0, rho: float = 3.0, seed: int = 2, nbeads: int = 10,
         b: float = 0.7, k: float = 4.0, a_same: float = 25.0, a_cross: float = 40.0,
         **kw) -> Workload:
    """A5B5 diblock melt: floor(N/10) chains of 10 beads with harmonic springs
    (k, r0 = 0) between neighbours, plus N mod 10 free A beads."""
    Lv = np.array([L, L, L], np.float64)
    n = int(round(rho * L ** 3))
    nchains = n // nbeads
    nfree = n - nchains * nbeads
    rng = _rng(seed)
    chain = _walk(rng, nchains, nbeads, b, Lv)
    free = _into_box(rng.uniform(0.0, 1.0, size=(nfree, 3)) * Lv, Lv)
    pos = np.concatenate([chain, free])
    vel = _velocities(rng, n, 1.0)
    half = nbeads // 2
    types = np.zeros(n, np.uint8)
    per = np.concatenate([np.zeros(half, np.uint8), np.ones(nbeads - half, np.uint8)])
    types[:nchains * nbeads] = np.tile(per, nchains)
    base = np.arange(nchains, dtype=np.int64)[:, None] * nbeads
    bi = (base + np.arange(nbeads - 1)).ravel()
    nb = bi.shape[0]
    return Workload(name=f"melt_L{L:g}", L=(L, L, L), pos=pos, vel=vel, types=types,
                    ntypes=2, a=np.array([[a_same, a_cross], [a_cross, a_same]]),
                    seed=seed, btype=np.full(nb, BOND_HARMONIC, np.int32), bi=bi,
                    bj=bi + 1, r_e=np.zeros(nb), k=np.full(nb, k), alpha=np.zeros(nb),
                    **kw)


# Peptide-like chain model: solvent W, chain types P and H.
PEPTIDE_A = np.array([[25.0, 25.0, 40.0],
                      [25.0, 25.0, 30.0],
                      [40.0, 30.0, 25.0]])


def peptide_chain_types(nbeads: int) -> np.ndarray:
    """Bead k of a chain is H (type 2) when k mod 7 is 0, 3 or 4, else P (type 1)."""
    k = np.arange(nbeads)
    return np.where(np.isin(k % 7, (0, 3, 4)), 2, 1).astype(np.uint8)


def peptide_chain_bonds(offset: int, nbeads: int):
    """Backbone 1-2 harmonic (k=4, r0=0.5), 1-3 and 1-5 standard Morse
    (D=5, alpha=2, r0=0.7 and 1.0) for one chain starting at tag ``offset``."""
    rec = [(BOND_HARMONIC, offset + i, offset + i + 1, 0.5, 4.0, 0.0) for i in range(nbeads - 1)]
    rec += [(BOND_MORSE, offset + i, offset + i + 2, 0.7, 5.0, 2.0) for i in range(nbeads - 2)]
    rec += [(BOND_MORSE, offset + i, offset + i + 4, 1.0, 5.0, 2.0) for i in range(nbeads - 4)]
    return rec


def peptide(L=40.0, rho: float = 3.0, seed: int = 4, nchains: int = 400,
            nbeads: int = 20, b: float = 0.5, name: str | None = None, **kw) -> Workload:
    """Peptide-like chains in solvent: nchains chains of nbeads beads, rest
    solvent (L a scalar for a cubic box, or three edges)."""
    Lv = _box(L)
    n = int(round(rho * float(np.prod(Lv))))
    nchain_beads = nchains * nbeads
    if nchain_beads > n:
        raise ValueError("more chain beads than particles")
    rng = _rng(seed)
    chain = _walk(rng, nchains, nbeads, b, Lv) if nchains else np.zeros((0, 3))
    solvent = _into_box(rng.uniform(0.0, 1.0, size=(n - nchain_beads, 3)) * Lv, Lv)
    pos = np.concatenate([chain, solvent])
    vel = _velocities(rng, n, 1.0)
    types = np.zeros(n, np.uint8)
    if nchains:
        types[:nchain_beads] = np.tile(peptide_chain_types(nbeads), nchains)
    rec = []
    for c in range(nchains):
        rec += peptide_chain_bonds(c * nbeads, nbeads)
    bt, bi, bj, re, kk, al = _bond_arrays(rec)
    return Workload(name=name or f"peptide_L{_box_name(Lv)}", L=tuple(float(v) for v in Lv),
                    pos=pos, vel=vel, types=types, ntypes=3, a=PEPTIDE_A.copy(), seed=seed, btype=bt,
                    bi=bi, bj=bj, r_e=re, k=kk, alpha=al, **kw)


def helix(L: float = 20.0, rho: float = 3.0, seed: int = 6, beads: int = 60,
          b: float = 0.6, **kw) -> Workload:
    """The paper's alpha-helix deck (Fig. 3b and the protein section): one chain
    of 60 skeletal beads S in water W, a_SS = a_WW = 50, a_SW = 55, 1-2 harmonic
    (C=160, r_e=0.6), 1-3 harmonic (C=80, r_e=1.2), 1-3 modified Morse (K_M=12,
    alpha=8, r_e=0.9), 1-5 modified Morse (K_M=12, alpha=8, r_e=0.6), kT=1,
    gamma=4.2, lambda=0.65, dt=0.02.  sigma follows sigma^2 = 2 gamma kT."""
    Lv = np.array([L, L, L], np.float64)
    n = int(round(rho * L ** 3))
    rng = _rng(seed)
    chain = _walk(rng, 1, beads, b, Lv)
    water = _into_box(rng.uniform(0.0, 1.0, size=(n - beads, 3)) * Lv, Lv)
    pos = np.concatenate([chain, water])
    vel = _velocities(rng, n, 1.0)
    types = np.zeros(n, np.uint8)
    types[:beads] = 1
    bt, bi, bj, re, kk, al = _bond_arrays(helix_records(0, beads))
    gamma = 4.2
    return Workload(name="helix_L20", L=(L, L, L), pos=pos, vel=vel, types=types,
                    ntypes=2, a=np.array([[50.0, 55.0], [55.0, 50.0]]), gamma=gamma,
                    sigma=math.sqrt(2.0 * gamma * 1.0), dt=0.02, seed=seed,
                    steps=10000, btype=bt, bi=bi, bj=bj, r_e=re, k=kk, alpha=al, **kw)


def helix_records(offset: int, beads: int):
    """The bond records of one chain of the alpha-helix deck (Fig. 3b) starting
    at tag `offset`: 1-2 harmonic (C=160, r_e=0.6), 1-3 harmonic (C=80,
    r_e=1.2), 1-3 modified Morse (K_M=12, alpha=8, r_e=0.9), 1-5 modified Morse
    (K_M=12, alpha=8, r_e=0.6)."""
    o = offset
    rec = [(BOND_HARMONIC, o + i, o + i + 1, 0.6, 160.0, 0.0) for i in range(beads - 1)]
    rec += [(BOND_HARMONIC, o + i, o + i + 2, 1.2, 80.0, 0.0) for i in range(beads - 2)]
    rec += [(BOND_MORSE_PAPER, o + i, o + i + 2, 0.9, 12.0, 8.0) for i in range(beads - 2)]
    rec += [(BOND_MORSE_PAPER, o + i, o + i + 4, 0.6, 12.0, 8.0) for i in range(beads - 4)]
    return rec


def sweep_box(N: int, chains: bool = False, seed: int = 11, beads: int = 60,
              fraction: float = 0.03) -> Workload:
    """A box of the paper's benchmark sweep (performance section, Tables 1-3):
    N beads at rho = 3 in a cubic box of edge (N/3)^(1/3), a = 25, gamma = 4.5,
    sigma = 3.  With chains (Table 3), ceil(fraction N / beads) chains of the
    alpha-helix deck's bonds (60 beads, Fig. 3b records, b = 0.6 random walk)
    replace solvent beads; every pair keeps a = 25, so the pair work equals
    Table 1's, and dt = 0.02 (the deck's step; its Morse terms need it)."""
    L = (N / 3.0) ** (1.0 / 3.0)
    if not chains:
        return fluid(L, seed=seed, name=f"sweep_N{N}")
    Lv = _box(L)
    n = int(round(3.0 * L ** 3))
    nchains = int(math.ceil(fraction * n / beads))
    rng = _rng(seed)
    chain = _walk(rng, nchains, beads, 0.6, Lv)
    solvent = _into_box(rng.uniform(0.0, 1.0, size=(n - nchains * beads, 3)) * Lv, Lv)
    pos = np.concatenate([chain, solvent])
    vel = _velocities(rng, n, 1.0)
    types = np.zeros(n, np.uint8)
    types[:nchains * beads] = 1
    rec = []
    for c in range(nchains):
        rec += helix_records(c * beads, beads)
    bt, bi, bj, re, kk, al = _bond_arrays(rec)
    return Workload(name=f"sweep_N{N}_chains", L=tuple(float(v) for v in Lv), pos=pos,
                    vel=vel, types=types, ntypes=2, a=np.full((2, 2), 25.0), dt=0.02,
                    seed=seed, btype=bt, bi=bi, bj=bj, r_e=re, k=kk, alpha=al)


# The five benchmark workloads by name.
def cfg_fluid_L10(**kw) -> Workload:
    """Single-species fluid, FP64: L=10, N=3000, a=25, gamma=4.5, sigma=3, dt=0.04."""
    return fluid(10.0, seed=1, precision="fp64", steps=100, name="fluid_L10", **kw)


def cfg_melt_L32(**kw) -> Workload:
    """A5B5 melt, FP32 forces: L=32, N=98304, harmonic k=4, a_AB=40, 1000 steps."""
    return melt(32.0, seed=2, steps=1000, **kw)


def cfg_fluid_L96(**kw) -> Workload:
    """Large fluid, FP32 forces / FP64 positions: L=96, N=2,654,208, 500 steps."""
    return fluid(96.0, seed=3, steps=500, name="fluid_L96", **kw)


def cfg_peptide_L40(**kw) -> Workload:
    """Peptide-like chains: L=40, N=192000, 400 chains of 20 beads, 2000 steps."""
    return peptide(40.0, seed=4, steps=2000, **kw)


@dataclasses.dataclass
class Request:
    """One replica simulation request of the serving stream."""
    rid: int
    arrival: float          # seconds after the stream starts
    L: int
    nbeads: int
    steps: int
    seed: int


def replica_stream(nreq: int = 512, rate: float = 200.0, seed: int = 5,
                   L_range=(6, 12), beads_range=(10, 40),
                   steps_range=(1000, 10000)) -> list:
    """Poisson arrivals (exponential gaps, mean 1/rate) of replica requests with
    integer L uniform in L_range, chain length uniform in beads_range and step
    count uniform in steps_range; replica r uses seed 1000 + r."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=nreq)
    nb = rng.integers(beads_range[0], beads_range[1] + 1, size=nreq)
    st = rng.integers(steps_range[0], steps_range[1] + 1, size=nreq)
    return [Request(r, float(t[r]), int(Ls[r]), int(nb[r]), int(st[r]), 1000 + r)
            for r in range(nreq)]


def replica(req: Request) -> Workload:
    """The workload of one request: one peptide-like chain in solvent at rho=3."""
    return peptide(float(req.L), seed=req.seed, nchains=1, nbeads=req.nbeads,
                   name=f"replica_{req.rid}", steps=req.steps)
