"""Seeded synthetic inputs for the one-band Hubbard sector problems.

This module produces *inputs only*: site numbering, bond lists, per-bond hopping
amplitudes, per-site U and on-site energies, and the seeds handed to the solver.
It contains none of the method's arithmetic (no bases, no hopping signs, no
matrix elements), so both the CPU oracle and the GPU library can consume it
without sharing any code with each other.

Parameter draws use SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) in counter mode: draw ``k`` of a
stream with seed ``s`` is the SplitMix64 output for state ``s + (k+1)*gamma``.
Draws are consumed in the order the bonds (or sites) are listed.

Lattices follow the Hamiltonian of Eq. (count1): nearest-neighbour bonds with
amplitude ``t_ij`` and on-site repulsion ``U``.  The generalisation to per-bond
``t_ij``, per-site ``U_i`` and on-site energies ``eps_i`` is the one needed for
the Anderson impurity model of Sec. VIII.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

PARAMS_SEED = 1307
START_SEED = 7542


def _splitmix64_out(state: int) -> int:
    z = state & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def draw_uniform(seed: int, k: int, lo: float, hi: float) -> float:
    """k-th draw of the counter-based SplitMix64 stream `seed`, mapped to [lo, hi)."""
    u = (_splitmix64_out(seed + (k + 1) * GAMMA) >> 11) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def draw_int(seed: int, k: int, lo: int, hi: int) -> int:
    """k-th draw mapped to the integers lo..hi inclusive."""
    u = (_splitmix64_out(seed + (k + 1) * GAMMA) >> 11) * (1.0 / 9007199254740992.0)
    return lo + min(int(u * (hi - lo + 1)), hi - lo)


@dataclass
class Model:
    """One-band Hubbard / Anderson model on an arbitrary bond graph.

    Sites are 0-based; site ``i`` is bit ``i`` of an occupation integer.
    Each bond (i, j) carries amplitude ``t`` so that the hopping operator is
    ``-t (c+_i c_j + c+_j c_i)`` for each spin.
    """

    name: str
    n_sites: int
    bonds: List[Tuple[int, int]]
    t: List[float]
    U: List[float]
    eps: List[float]
    n_up: int
    n_dn: int
    meta: dict = field(default_factory=dict)

    @property
    def n_bonds(self) -> int:
        return len(self.bonds)

    def with_params(self, *, t=None, U=None, eps=None, n_up=None, n_dn=None, name=None) -> "Model":
        return Model(
            name=name or self.name,
            n_sites=self.n_sites,
            bonds=list(self.bonds),
            t=list(self.t if t is None else t),
            U=list(self.U if U is None else U),
            eps=list(self.eps if eps is None else eps),
            n_up=self.n_up if n_up is None else n_up,
            n_dn=self.n_dn if n_dn is None else n_dn,
            meta=dict(self.meta),
        )

    def bond_arrays(self):
        bi = [min(i, j) for i, j in self.bonds]
        bj = [max(i, j) for i, j in self.bonds]
        return bi, bj


def ring(M: int, *, t: float = 1.0, U: float = 4.0, n_up: int = None, n_dn: int = None) -> Model:
    """Periodic 1D chain of M >= 3 sites, bonds (i, i+1 mod M) in order of i."""
    if M < 3:
        raise ValueError("periodic ring needs M >= 3")
    bonds = [(i, (i + 1) % M) for i in range(M)]
    n_up = M // 2 if n_up is None else n_up
    n_dn = M // 2 if n_dn is None else n_dn
    return Model(f"ring{M}", M, bonds, [t] * M, [U] * M, [0.0] * M, n_up, n_dn)


def square_periodic(Lx: int, Ly: int, *, t_lo: float = 0.9, t_hi: float = 1.1, U: float = 4.0,
                    n_up: int = 7, n_dn: int = 7, seed: int = PARAMS_SEED, uniform_t: float = None) -> Model:
    """Lx x Ly torus, site = Lx*y + x.  For each site in row-major order the bond to
    the right neighbour, then the bond to the neighbour below (both periodic).
    t_ij ~ uniform(t_lo, t_hi) drawn in bond-list order unless `uniform_t` is given."""
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            s = Lx * y + x
            bonds.append((s, Lx * y + (x + 1) % Lx))
            bonds.append((s, Lx * ((y + 1) % Ly) + x))
    if uniform_t is not None:
        t = [uniform_t] * len(bonds)
    else:
        t = [draw_uniform(seed, k, t_lo, t_hi) for k in range(len(bonds))]
    M = Lx * Ly
    return Model(f"square{Lx}x{Ly}", M, bonds, t, [U] * M, [0.0] * M, n_up, n_dn,
                 meta={"seed": seed})


def ladder(L: int, *, t_leg: float = 1.0, rung_lo: float = 0.5, rung_hi: float = 1.5, U: float = 6.0,
           n_up: int = None, n_dn: int = None, seed: int = PARAMS_SEED) -> Model:
    """Two-leg ladder of L rungs, periodic along the legs, site = 2*x + leg.
    Bond list: leg 0 bonds (x, x+1 mod L), then leg 1 bonds, then the L rungs.
    One rung amplitude drawn per rung, uniform(rung_lo, rung_hi), in rung order."""
    bonds, t = [], []
    for leg in (0, 1):
        for x in range(L):
            bonds.append((2 * x + leg, 2 * ((x + 1) % L) + leg))
            t.append(t_leg)
    for x in range(L):
        bonds.append((2 * x, 2 * x + 1))
        t.append(draw_uniform(seed, x, rung_lo, rung_hi))
    M = 2 * L
    n_up = L if n_up is None else n_up
    n_dn = L if n_dn is None else n_dn
    return Model(f"ladder2x{L}", M, bonds, t, [U] * M, [0.0] * M, n_up, n_dn, meta={"seed": seed})


def dimer(*, t: float = 1.0, U: float = 4.0) -> Model:
    """Two sites joined by one bond, one electron of each spin."""
    return Model("dimer", 2, [(0, 1)], [t], [U, U], [0.0, 0.0], 1, 1)


def anderson_impurity(V: Sequence[float], eps_bath: Sequence[float], U: float, *,
                      eps_imp: float = None, name: str = "aim") -> Model:
    """Star-geometry Anderson impurity model: impurity = site 0, bath sites 1..n_b.

    Hybridisation +V_k (c+_0 c_k + h.c.) is expressed through the bond amplitude
    t_0k = -V_k.  U acts on the impurity only; eps_imp defaults to -U/2 and the
    sector is half filling per spin: N_up = ceil(M/2), N_dn = floor(M/2)."""
    n_b = len(V)
    M = 1 + n_b
    bonds = [(0, k + 1) for k in range(n_b)]
    t = [-float(v) for v in V]
    Us = [float(U)] + [0.0] * n_b
    e0 = -0.5 * U if eps_imp is None else eps_imp
    eps = [e0] + [float(e) for e in eps_bath]
    return Model(name, M, bonds, t, Us, eps, (M + 1) // 2, M // 2)


def aim_batch(count: int = 64, *, seed: int = PARAMS_SEED) -> List[Model]:
    """Batch of impurity problems.  Per problem p the draws of stream `seed + p`
    are consumed in this order: n_b ~ U{5..11}, U ~ U(2, 8), then for each bath
    site k: V_k ~ U(0.1, 1), eps_k ~ U(-2, 2)."""
    out = []
    for p in range(count):
        s = seed + 1000 + p
        n_b = draw_int(s, 0, 5, 11)
        U = draw_uniform(s, 1, 2.0, 8.0)
        V, eb = [], []
        for k in range(n_b):
            V.append(draw_uniform(s, 2 + 2 * k, 0.1, 1.0))
            eb.append(draw_uniform(s, 3 + 2 * k, -2.0, 2.0))
        out.append(anderson_impurity(V, eb, U, name=f"aim{p}"))
    return out


def random_graph(M: int, n_bonds: int, *, seed: int, U: float = 3.0, n_up: int = None, n_dn: int = None,
                 with_eps: bool = True, site_U: bool = False) -> Model:
    """Random simple graph on M sites (distinct bonds, no self loops) with random t,
    optional random on-site energies and per-site U.  For property tests."""
    pairs = [(i, j) for i in range(M) for j in range(i + 1, M)]
    chosen = []
    k = 0
    while len(chosen) < min(n_bonds, len(pairs)):
        idx = draw_int(seed, k, 0, len(pairs) - 1)
        k += 1
        if pairs[idx] not in chosen:
            chosen.append(pairs[idx])
    # randomly orient each bond so canonicalisation is exercised
    bonds = []
    for n, (i, j) in enumerate(chosen):
        bonds.append((j, i) if draw_int(seed + 7, n, 0, 1) else (i, j))
    t = [draw_uniform(seed + 1, n, -1.5, 1.5) for n in range(len(bonds))]
    if site_U:
        Us = [draw_uniform(seed + 2, i, 0.0, 6.0) for i in range(M)]
    else:
        Us = [U] * M
    eps = [draw_uniform(seed + 3, i, -1.0, 1.0) for i in range(M)] if with_eps else [0.0] * M
    n_up = M // 2 if n_up is None else n_up
    n_dn = (M - 1) // 2 if n_dn is None else n_dn
    return Model(f"rand{M}_{seed}", M, bonds, t, Us, eps, n_up, n_dn, meta={"seed": seed})


def config(name: str) -> Model:
    """Named workloads.

    ring8      : periodic chain M=8, t=1, U=4, N=4/4 (dim 4900)
    ring14_uX  : periodic chain M=14, t=1, U=X in {2,4,8}, N=7/7 (dim 11,778,624)
    square4x4  : 4x4 torus, 32 bonds t~U(0.9,1.1), U=4, N=7/7 (dim 130,873,600)
    ladder2x9  : 2x9 ladder, t_leg=1, t_rung~U(0.5,1.5), U=6, N=9/9 (dim 2,363,904,400)
    """
    if name == "ring8":
        return ring(8, U=4.0, n_up=4, n_dn=4)
    if name.startswith("ring14"):
        U = float(name.split("_u")[1]) if "_u" in name else 4.0
        return ring(14, U=U, n_up=7, n_dn=7).with_params(name=f"ring14_u{U:g}")
    if name == "ring16":
        return ring(16, U=4.0, n_up=8, n_dn=8)
    if name == "square4x4":
        return square_periodic(4, 4)
    if name == "ladder2x9":
        return ladder(9)
    raise KeyError(name)


def start_seed() -> int:
    return START_SEED
