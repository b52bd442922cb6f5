"""The regrouping of H by spectator cores that the GPU pair-block kernels use, checked on the CPU
against the oracle's explicit H (no library code).

App. B applies every pn term as a proton one-body jump times a neutron one-body jump. The pair
blocks group the same terms by the nucleons they leave in place: a proton core K_p (the target's
protons minus the created one) and a neutron core K_n. Each term application then belongs to
exactly one core pair (for a proton number operator n_x: the core target - x), and its
Jordan-Wigner sign factorises into sigma(K_p, x) sigma(K_p, y) sigma(K_n, u) sigma(K_n, v),
sigma(K, s) = (-1)^(occupied states of K below s). So
    (H_pn)[t, s] = sum over the core pairs of t of  sigma_t * h((x,u); (y,v)) * sigma_s.
For one species the cores hold n - 2 nucleons and the sign is sigma(L,a) sigma(L,b) sigma(L,c)
sigma(L,d) for the term c+_a c+_b c_d c_c on L + c + d. Both identities are rebuilt here term by
term, in plain Python loops over small spaces, from the oracle's m-scheme coefficients, and
compared with the oracle's dense H of the same terms."""
import numpy as np
import pytest

from oracle.basis import m_states
from oracle.hamiltonian import Model as OracleModel
from oracle.interaction import mscheme_terms
from workloads import PF_ORBITS, SD_ORBITS, random_tbme

MIXED_PAR = ((0, 1, 1), (0, 2, 5), (0, 1, 3))


def _sigma(K, s):
    return -1.0 if bin(K & ((1 << s) - 1)).count("1") & 1 else 1.0


def _bits(w):
    out = []
    while w:
        low = w & -w
        out.append(low.bit_length() - 1)
        w ^= low
    return out


@pytest.mark.parametrize("case", [
    # orbits, Z, N, 2M, parity, seed
    (SD_ORBITS, 2, 2, 0, 0, 1),
    (SD_ORBITS, 3, 2, 1, 0, 2),
    (MIXED_PAR, 2, 2, 0, 1, 3),
    (PF_ORBITS, 2, 1, 1, 0, 4),
], ids=["sd22", "sd32_odd", "mixpar_pos", "pf21"])
def test_pn_part_by_core_pairs(case):
    orbits, z, n, twoM, par, seed = case
    tb = [e for e in random_tbme(orbits, seed) if e[0] == 2]  # pn elements only
    zero = [0.0] * len(orbits)
    o = OracleModel(orbits, z, n, twoM, tb, zero, zero, par)
    H = o.dense()
    ns = len(m_states(orbits))
    rows = {}  # target pair (x, u) -> [(y, v, h)]
    for (al, be, ga, de), h in mscheme_terms(orbits, tb).items():
        assert al < ns <= be and ga < ns <= de  # c+_x(p) c+_u(n) c_v(n) c_y(p)
        rows.setdefault((al, be - ns), []).append((ga, de - ns, h))
    index = {int(w): i for i, w in enumerate(o.words)}
    Hc = np.zeros_like(H)
    core_pairs = 0
    for t, w in enumerate(o.words):
        p, q = int(w) & ((1 << ns) - 1), int(w) >> ns
        for x in _bits(p):
            Kp = p & ~(1 << x)
            for u in _bits(q):
                Kn = q & ~(1 << u)
                core_pairs += 1
                st = _sigma(Kp, x) * _sigma(Kn, u)
                for y, v, h in rows.get((x, u), ()):
                    if (Kp >> y) & 1 or (Kn >> v) & 1:
                        continue
                    s = index.get((Kp | (1 << y)) | ((Kn | (1 << v)) << ns))
                    if s is not None:
                        Hc[t, s] += st * _sigma(Kp, y) * _sigma(Kn, v) * h
    assert core_pairs == o.dim * z * n  # n_prot * n_neut core pairs (slots) per basis state
    assert np.abs(Hc - H).max() <= 1e-12 * np.abs(H).max()


@pytest.mark.parametrize("case", [
    (SD_ORBITS, 3, 0, 1, 0, 5),
    (SD_ORBITS, 0, 4, 0, 0, 6),
    (MIXED_PAR, 0, 3, 1, 0, 7),
], ids=["sd_z3", "sd_n4", "mixpar_n3"])
def test_single_species_two_body_by_cores(case):
    orbits, z, n, twoM, par, seed = case
    ch = 0 if z else 1
    tb = [e for e in random_tbme(orbits, seed) if e[0] == ch]
    zero = [0.0] * len(orbits)
    o = OracleModel(orbits, z, n, twoM, tb, zero, zero, par)
    H = o.dense()
    ns = len(m_states(orbits))
    off = 0 if z else ns
    rows = {}  # target pair (a, b), a < b -> [(c, d, h)]
    for (al, be, ga, de), h in mscheme_terms(orbits, tb).items():
        assert al < be and ga < de
        rows.setdefault((al - off, be - off), []).append((ga - off, de - off, h))
    index = {int(w): i for i, w in enumerate(o.words)}
    Hc = np.zeros_like(H)
    npart = z + n
    for t, w in enumerate(o.words):
        word = (int(w) >> off) & ((1 << ns) - 1)
        occ = _bits(word)
        for i, a in enumerate(occ):
            for b in occ[i + 1:]:
                L = word & ~(1 << a) & ~(1 << b)
                st = _sigma(L, a) * _sigma(L, b)
                for c, d, h in rows.get((a, b), ()):
                    if (L >> c) & 1 or (L >> d) & 1:
                        continue
                    s = index.get((L | (1 << c) | (1 << d)) << off)
                    if s is not None:
                        Hc[t, s] += st * _sigma(L, c) * _sigma(L, d) * h
    assert len(occ) == npart
    assert np.abs(Hc - H).max() <= 1e-12 * np.abs(H).max()
