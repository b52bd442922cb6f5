"""M-scheme basis of the oracle (test infrastructure; see package docstring).

Follows the paper's Sec. 2 (Slater determinants as bit strings, Eq. for
|M_i>) and App. A (Table 1 ordering, partitions Gamma = (N^p, N^n, M^p) and the
product form |M_i> = |p_i> (x) |n_i>).

Readings (the paper fixes them only through Table 1):
  * m-states: orbit order as given, then 2m ascending; bit s is state s.
  * species sector order: occupation partitions in descending lexicographic
    order; inside a partition, occupied-state tuples in ascending
    lexicographic order. Table 1 is exactly this for d5/2 + s1/2.
  * product basis: blocks by 2M_p ascending, then proton parity + before -,
    then neutron parity + before -; inside a block proton-major:
    index = offset + p * D_n + n.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass


def m_states(orbits):
    """[(orbit index, 2m)] in orbit order, 2m ascending."""
    out = []
    for k, (_n, _l, twoj) in enumerate(orbits):
        for twom in range(-twoj, twoj + 1, 2):
            out.append((k, twom))
    return out


def species_sectors(orbits, n_part):
    """All SDs of ``n_part`` identical nucleons keyed by (2M, parity).

    Each value is a list of (bitmask, partition) in Table-1 order.
    """
    states = m_states(orbits)
    norb = len(orbits)
    sectors = {}
    for occ in itertools.combinations(range(len(states)), n_part):
        twoM = sum(states[s][1] for s in occ)
        par = 1
        part = [0] * norb
        for s in occ:
            part[states[s][0]] += 1
            if orbits[states[s][0]][1] % 2:
                par = -par
        key = (twoM, par)
        sectors.setdefault(key, []).append((tuple(-x for x in part), occ))
    out = {}
    for key, lst in sectors.items():
        lst.sort()
        out[key] = [(sum(1 << s for s in occ), tuple(-x for x in negpart)) for negpart, occ in lst]
    return out


def _orbit_subsets(orbits, o, k):
    """Subsets of k m-states of orbit o as (bitmask, 2M), in ascending lexicographic order of
    the state-index tuples (itertools.combinations order)."""
    states = m_states(orbits)
    idx = [s for s, (oo, _m) in enumerate(states) if oo == o]
    out = []
    for sub in itertools.combinations(idx, k):
        out.append((sum(1 << s for s in sub), sum(states[s][1] for s in sub)))
    return out


def sector_words(orbits, n_part, twoM, parity):
    """Words of one species sector (2M, parity) in Table-1 order, without visiting the other
    sectors: for large spaces where ``species_sectors`` (all subsets) is too slow.

    Same order as ``species_sectors``: partitions (occupation per orbit) in descending
    lexicographic order; inside a partition the occupied-state tuples ascend
    lexicographically, which is the nested order with orbit 0 outermost and each orbit's
    subsets in combinations order. Subsets are combined orbit by orbit (numpy outer
    products in that nested order), dropping partial words whose 2M can no longer reach
    the target.
    """
    import numpy as np
    norb = len(orbits)
    caps = [tj + 1 for (_n, _l, tj) in orbits]

    def mmax(o, k):  # largest 2M of k particles in orbit o
        tj = orbits[o][2]
        return sum(range(tj, tj - 2 * k, -2))

    parts = []

    def rec(o, left, cur):
        if o == norb:
            if left == 0:
                parts.append(tuple(cur))
            return
        for k in range(min(caps[o], left), -1, -1):  # descending occupation first
            rec(o + 1, left - k, cur + [k])

    rec(0, n_part, [])
    chunks = []
    for part in parts:  # generated in descending lexicographic order
        par = 1
        for o, k in enumerate(part):
            if orbits[o][1] % 2 and k % 2:
                par = -par
        if parity != 0 and par != parity:
            continue
        rest = [0] * (norb + 1)
        for o in range(norb - 1, -1, -1):
            rest[o] = rest[o + 1] + mmax(o, part[o])
        words = np.zeros(1, dtype=np.uint64)
        ms = np.zeros(1, dtype=np.int64)
        for o, k in enumerate(part):
            sub = _orbit_subsets(orbits, o, k)
            sw = np.array([w for w, _ in sub], dtype=np.uint64)
            sm = np.array([m for _, m in sub], dtype=np.int64)
            words = (words[:, None] | sw[None, :]).ravel()
            ms = (ms[:, None] + sm[None, :]).ravel()
            keep = np.abs(twoM - ms) <= rest[o + 1]
            words, ms = words[keep], ms[keep]
        chunks.append(words[ms == twoM])
    return np.concatenate(chunks) if chunks else np.zeros(0, dtype=np.uint64)


def _sectors_for(orbits, n_part, n_other, twoM, parity):
    """species_sectors(orbits, n_part), or for large species only the sectors that pair with
    a sector of the other species (found from the counts) to total 2M and parity, listed by
    ``sector_words`` (the partition entry is not filled in there)."""
    from math import comb
    if comb(len(m_states(orbits)), n_part) <= 2_000_000:
        return species_sectors(orbits, n_part)
    other = count_sds(orbits, n_other)
    out = {}
    for (tm, par), _c in sorted(count_sds(orbits, n_part).items()):
        if any(tm + to == twoM and (parity == 0 or par * po == parity) for (to, po) in other):
            out[(tm, par)] = [(int(w), None) for w in sector_words(orbits, n_part, tm, par)]
    return out


@dataclass
class Block:
    twoMp: int
    parp: int
    twoMn: int
    parn: int
    dp: int
    dn: int
    offset: int


class ProductBasis:
    """Proton x neutron M-scheme basis for fixed 2M (and optionally parity)."""

    def __init__(self, orbits, n_prot, n_neut, twoM, parity=0):
        self.orbits = tuple(orbits)
        self.nstates = len(m_states(orbits))
        self.n_prot, self.n_neut, self.twoM, self.parity = n_prot, n_neut, twoM, parity
        self.psec = _sectors_for(orbits, n_prot, n_neut, twoM, parity)
        self.nsec = _sectors_for(orbits, n_neut, n_prot, twoM, parity)
        keys = []
        for (tmp, pp) in self.psec:
            for (tmn, pn) in self.nsec:
                if tmp + tmn != twoM:
                    continue
                if parity != 0 and pp * pn != parity:
                    continue
                keys.append((tmp, -pp, -pn, tmn, pp, pn))
        keys.sort()
        self.blocks = []
        off = 0
        for tmp, _a, _b, tmn, pp, pn in keys:
            dp, dn = len(self.psec[(tmp, pp)]), len(self.nsec[(tmn, pn)])
            self.blocks.append(Block(tmp, pp, tmn, pn, dp, dn, off))
            off += dp * dn
        self.dim = off

    def states(self):
        """(proton bitmask, neutron bitmask) for every basis index, in order."""
        out = []
        for b in self.blocks:
            plist = self.psec[(b.twoMp, b.parp)]
            nlist = self.nsec[(b.twoMn, b.parn)]
            for pw, _ in plist:
                for nw, _ in nlist:
                    out.append((pw, nw))
        return out

    def combined_words(self):
        """One word per basis state: proton bits low, neutron bits shifted by the state count."""
        ns = self.nstates
        return [pw | (nw << ns) for pw, nw in self.states()]

    def combined_words_array(self):
        """combined_words() as a uint64 array, built block by block (same order; for large spaces)."""
        import numpy as np
        ns = np.uint64(self.nstates)
        out = np.empty(self.dim, dtype=np.uint64)
        for b in self.blocks:
            pw = np.array([w for w, _ in self.psec[(b.twoMp, b.parp)]], dtype=np.uint64)
            nw = np.array([w for w, _ in self.nsec[(b.twoMn, b.parn)]], dtype=np.uint64)
            out[b.offset:b.offset + b.dp * b.dn] = (pw[:, None] | (nw[None, :] << ns)).ravel()
        return out


def count_sds(orbits, n_part):
    """Number of SDs by (2M, parity) for ``n_part`` nucleons, by dynamic programming over orbits.

    Independent of the enumeration in ``species_sectors``: each orbit contributes
    subsets of its own m-states, and the counts are convolved orbit by orbit.
    """
    table = {(0, 0, 1): 1}  # (particles, 2M, parity) -> count
    for (_n, l, twoj) in orbits:
        ms = list(range(-twoj, twoj + 1, 2))
        orb = {}
        for k in range(len(ms) + 1):
            for sub in itertools.combinations(ms, k):
                key = (k, sum(sub))
                orb[key] = orb.get(key, 0) + 1
        new = {}
        for (n0, m0, p0), c0 in table.items():
            for (k, m), c in orb.items():
                if n0 + k > n_part:
                    continue
                key = (n0 + k, m0 + m, p0 * ((-1) ** (l * k)))
                new[key] = new.get(key, 0) + c0 * c
        table = new
    return {(m, p): c for (n, m, p), c in table.items() if n == n_part}


def count_dim(orbits_p, n_prot, orbits_n, n_neut, twoM, parity=0):
    """M-scheme dimension from per-species DP counts (no enumeration)."""
    cp = count_sds(orbits_p, n_prot) if n_prot or orbits_p else {(0, 1): 1}
    cn = count_sds(orbits_n, n_neut) if n_neut or orbits_n else {(0, 1): 1}
    tot = 0
    for (mp, pp), a in cp.items():
        for (mn, pn), b in cn.items():
            if mp + mn == twoM and (parity == 0 or pp * pn == parity):
                tot += a * b
    return tot
