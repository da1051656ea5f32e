"""Parameter layout of the correlator-product-state (CPS) times pfaffian ansatz, Sec. II.C.

A correlator acting on k spin orbitals carries one parameter per occupation pattern of
those orbitals, 2^k in all; a pair correlator covers 2 sites (4 spin orbitals, 16
parameters) and an n x n plaquette covers n^2 sites (2n^2 spin orbitals).  The pfaffian
pairing matrix f_ij, i < j over all spin orbitals, adds C(2 n_sites, 2) parameters.
Translation-invariant correlators share one parameter set across all their translates.

The layouts below are built from the lattice geometry of the paper's examples
(Sec. III.A, III.B, III.C); the test suite checks the totals the paper prints.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations


@dataclass(frozen=True)
class Correlator:
    sites: tuple            # lattice sites covered (each site = 2 spin orbitals)
    shared: bool = False    # True: parameters shared by all translates (translation invariant)

    @property
    def n_spin_orbitals(self) -> int:
        return 2 * len(self.sites)

    @property
    def n_params(self) -> int:
        return 2 ** self.n_spin_orbitals


@dataclass
class CpsLayout:
    n_sites: int
    correlators: list = field(default_factory=list)   # distinct parameter sets

    @property
    def n_correlator_params(self) -> int:
        return sum(c.n_params for c in self.correlators)

    @property
    def n_pairing_params(self) -> int:
        m = 2 * self.n_sites
        return m * (m - 1) // 2

    @property
    def n_params(self) -> int:
        return self.n_correlator_params + self.n_pairing_params


def _site(x, y, lx):
    return y * lx + x


def _plaquettes(lx, ly, n, periodic):
    """All n x n plaquettes of an lx x ly lattice, as tuples of sites."""
    xs = range(lx) if periodic else range(lx - n + 1)
    ys = range(ly) if periodic else range(ly - n + 1)
    out = []
    for y0 in ys:
        for x0 in xs:
            out.append(tuple(sorted(_site((x0 + dx) % lx, (y0 + dy) % ly, lx)
                                    for dy in range(n) for dx in range(n))))
    return out


def hubbard_4x4_layout() -> CpsLayout:
    """Sec. III.A: periodic 4x4 lattice, two translation-invariant 3x3 correlators (one
    anchored on each sublattice) plus the pfaffian."""
    lx = ly = 4
    anchors = [(0, 0), (1, 0)]   # one anchor on each sublattice of the bipartite lattice
    cors = []
    for ax, ay in anchors:
        sites = tuple(sorted(_site((ax + dx) % lx, (ay + dy) % ly, lx) for dy in range(3) for dx in range(3)))
        cors.append(Correlator(sites, shared=True))
    return CpsLayout(n_sites=lx * ly, correlators=cors)


def hydrogen_4x4_layout() -> CpsLayout:
    """Sec. III.C: open 4x4 lattice, every 2x2 plaquette and every long-range pair, plus the
    pfaffian.  Reading: a pair whose two sites already share a plaquette is not repeated."""
    lx = ly = 4
    plaqs = _plaquettes(lx, ly, 2, periodic=False)
    covered = set()
    for p in plaqs:
        covered.update(combinations(p, 2))
    pairs = [pr for pr in combinations(range(lx * ly), 2) if pr not in covered]
    cors = [Correlator(p) for p in plaqs] + [Correlator(pr) for pr in pairs]
    return CpsLayout(n_sites=lx * ly, correlators=cors)


def hubbard_8x8_plaquette_layout() -> CpsLayout:
    """Correlator shape of Sec. III.B used for the synthetic CPS-shaped matrices: the 64
    overlapping 2x2 plaquettes of a periodic 8x8 lattice, each with its own parameters
    (2^8 = 256 each), plus the pfaffian over 128 spin orbitals (8128 parameters)."""
    lx = ly = 8
    return CpsLayout(n_sites=lx * ly, correlators=[Correlator(p) for p in _plaquettes(lx, ly, 2, periodic=True)])
