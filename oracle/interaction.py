"""J-coupled two-body matrix elements -> m-scheme terms (oracle, test infrastructure).

Hamiltonian of Sec. 2:  H = sum_a e_a n_a + sum_{a<b, c<d} h_abcd c+_a c+_b c_d c_c,
written here over *combined* single-particle states: proton m-states 0..Ns-1,
neutron m-states Ns..2Ns-1 (protons first).

Readings of the silent parts of the paper:
  * Pair states are normalised and antisymmetrised, Condon-Shortley CG, orbit a
    coupled before b, proton before neutron in the pn channel:
      A+_JM(ab) = (1+delta_ab)^(-1/2) sum_{ma mb} <ja ma jb mb|J M> c+_a,ma c+_b,mb
      H2 = sum_{(ab),(cd)} sum_J V_J(ab,cd) sum_M A+_JM(ab) A_JM(cd)
    so for ordered m-states alpha<beta in (ab), gamma<delta in (cd):
      h = sum_J N_ab N_cd <..|JM><..|JM> V_J(ab,cd),  N_ab = sqrt(1+delta_ab) (pp, nn), 1 (pn).
  * Reordered identical-particle pairs: V_J(ba,cd) = -(-1)^(ja+jb-J) V_J(ab,cd).
  * Each element is listed once; the mirror V_J(cd,ab) = V_J(ab,cd) is implied.
"""
from __future__ import annotations

from .basis import m_states
from .cg import cg

CH_PP, CH_NN, CH_PN = 0, 1, 2


def _canonical(orbits, ch, a, b, c, d, twoJ, v):
    """Reorder identical-particle pairs to a<=b, c<=d with the exchange phase."""
    if ch != CH_PN:
        if a > b:
            a, b = b, a
            v *= -((-1) ** ((orbits[a][2] + orbits[b][2] - twoJ) // 2))
        if c > d:
            c, d = d, c
            v *= -((-1) ** ((orbits[c][2] + orbits[d][2] - twoJ) // 2))
    return a, b, c, d, v


def _pair_mstates(orbits, states, ch, a, b, ns):
    """Ordered combined-index pairs (s1 < s2, 2m1, 2m2, weight N_ab) of the orbit pair (a,b)."""
    out = []
    if ch == CH_PN:
        for s1, (o1, m1) in enumerate(states):
            if o1 != a:
                continue
            for s2, (o2, m2) in enumerate(states):
                if o2 == b:
                    out.append((s1, s2 + ns, m1, m2, 1.0))
        return out
    off = 0 if ch == CH_PP else ns
    norm = 2.0 ** 0.5 if a == b else 1.0
    for s1, (o1, m1) in enumerate(states):
        if o1 != a:
            continue
        for s2, (o2, m2) in enumerate(states):
            if o2 == b and s2 > s1:
                out.append((s1 + off, s2 + off, m1, m2, norm))
    return out


def mscheme_terms(orbits, tbme):
    """Dict {(alpha, beta, gamma, delta): h} over combined states, alpha<beta, gamma<delta."""
    states = m_states(orbits)
    ns = len(states)
    terms = {}
    for (ch, a, b, c, d, twoJ, v) in tbme:
        a, b, c, d, v = _canonical(orbits, ch, a, b, c, d, twoJ, v)
        pairs = [((a, b), (c, d))]
        if (a, b) != (c, d):
            pairs.append(((c, d), (a, b)))
        for (x, y), (z, w) in pairs:
            left = _pair_mstates(orbits, states, ch, x, y, ns)
            right = _pair_mstates(orbits, states, ch, z, w, ns)
            jx, jy, jz, jw = orbits[x][2], orbits[y][2], orbits[z][2], orbits[w][2]
            for (s1, s2, m1, m2, n1) in left:
                c1 = cg(jx, m1, jy, m2, twoJ, m1 + m2)
                if c1 == 0.0:
                    continue
                for (s3, s4, m3, m4, n2) in right:
                    if m3 + m4 != m1 + m2:
                        continue
                    c2 = cg(jz, m3, jw, m4, twoJ, m3 + m4)
                    if c2 == 0.0:
                        continue
                    key = (s1, s2, s3, s4)
                    terms[key] = terms.get(key, 0.0) + n1 * n2 * c1 * c2 * v
    return terms


def one_body(orbits, spe_p, spe_n):
    """Single-particle energy of every combined state (protons then neutrons)."""
    states = m_states(orbits)
    return [spe_p[o] for o, _ in states] + [spe_n[o] for o, _ in states]
