"""Virtual-pair decomposition of E2 — oracle only (test infrastructure).

The paper's "Implementation" subsection notes, without implementing it, that
V can be split into terms over virtual orbitals whose actions on Psi0 are
mutually orthogonal, so that the Hylleraas functional can be minimised for
each term on its own and E2 is the sum.  With Dyall's H0 the split is by
virtual occupation pattern (H0 keeps the pattern, so the first-order
equation is block diagonal over patterns).  Reading used here: the terms are
the unordered virtual pairs a <= b.  Pair (a, b), a < b, owns every pattern
with one electron in a and one in b; pair (a, a) owns the patterns with one
or two electrons in a, which carries the singles.

Each pair is solved as a problem on the active orbitals plus its virtual
orbitals (a, then b), with the integrals restricted to them and the Psi1
configurations restricted to the pair's occupancy on those sites.
"""
from __future__ import annotations

import numpy as np


def pairs(k_v):
    return [(a, b) for a in range(k_v) for b in range(a, k_v)]


def occupancy(a, b):
    """Allowed electron counts on the pair's virtual sites."""
    return [{1}, {1}] if a < b else [{1, 2}]


def restrict(h, eri, k_a, eps_virt, a, b):
    """h, eri and the virtual energies on the active orbitals plus a (and b)."""
    orbs = list(range(k_a)) + [k_a + a] + ([k_a + b] if a != b else [])
    hp = h[np.ix_(orbs, orbs)]
    ep = eri[np.ix_(orbs, orbs, orbs, orbs)]
    ev = np.array([eps_virt[a]] + ([eps_virt[b]] if a != b else []))
    return hp, ep, ev


def owner(pattern):
    """The pair that owns a virtual pattern, given as the key of the
    factorised sum over states: ((a, sig),) or ((a, sig), (b, tau))."""
    orbs = sorted(p[0] for p in pattern)
    return (orbs[0], orbs[-1])


def pair_e2(contrib):
    """Per-pair E2: sum of the pattern contributions each pair owns."""
    out = {}
    for pat, e in contrib.items():
        key = owner(pat)
        out[key] = out.get(key, 0.0) + e
    return out
