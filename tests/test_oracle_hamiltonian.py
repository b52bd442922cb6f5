"""Pins of the oracle's Hamiltonian against closed forms and independent constructions (CPU only).

Each pin is chosen so a plausible slip fails it:
  * Fock-space matrices obeying the canonical anticommutation relations -> any
    Jordan-Wigner sign or operator-order slip;
  * rows (adjoint terms) against columns (terms) -> a missing mirror element;
  * seniority formula for pairing in one j-shell -> the sqrt(2) pair normalisation;
  * J^2 written as an interaction -> CG phases in every channel incl. pn;
  * M=1 spectrum inside the M=0 spectrum for a random interaction -> CG phases of
    off-diagonal elements;
  * single-particle energies only -> the one-body diagonal;
  * reordered pair input expanded from scratch -> the exchange phase.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.basis import ProductBasis, count_dim, m_states
from oracle.cg import cg
from oracle.hamiltonian import Model
from oracle.interaction import mscheme_terms
from workloads import (PF_ORBITS, SD_ORBITS, SD_SPE, jsquared_spe, jsquared_tbme, pairing_tbme,
                       random_tbme)

F72 = ((0, 3, 7),)
H112 = ((0, 5, 11),)
P_ORBITS = ((0, 1, 1), (0, 1, 3))


def _fock_ops(nmodes):
    """Annihilators c_s on the 2^nmodes Fock space from tensor products (mode 0 leftmost)."""
    a = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    z = sp.csr_matrix(np.diag([1.0, -1.0]))
    eye = sp.identity(2, format="csr")
    ops = []
    for s in range(nmodes):
        m = sp.identity(1, format="csr")
        for t in range(nmodes):
            m = sp.kron(m, z if t < s else (a if t == s else eye), format="csr")
        ops.append(m)
    return ops


def test_fock_space_construction_matches():
    orbits = P_ORBITS
    tb = random_tbme(orbits, 5)
    spe = (0.7, -1.3)
    zp, zn, twoM = 2, 1, 1
    model = Model(orbits, zp, zn, twoM, tb, spe, spe)
    ns = len(m_states(orbits))
    S = 2 * ns
    c = _fock_ops(S)
    cd = [x.T.tocsr() for x in c]
    dimF = 2 ** S
    # canonical anticommutation relations
    for s in range(S):
        for t in range(S):
            acomm = (c[s] @ cd[t] + cd[t] @ c[s]).toarray()
            assert np.allclose(acomm, np.eye(dimF) if s == t else 0.0)
            assert abs(c[s] @ c[t] + c[t] @ c[s]).sum() == 0
    vac = np.zeros(dimF)
    vac[0] = 1.0
    basis_vecs = []
    for pw, nw in model.basis.states():
        occ = [s for s in range(ns) if pw >> s & 1] + [ns + s for s in range(ns) if nw >> s & 1]
        v = vac
        for s in reversed(occ):           # c+_{s1} c+_{s2} ... |0>, s1 < s2 < ...
            v = cd[s] @ v
        basis_vecs.append(v)
    B = np.array(basis_vecs).T
    e = np.array(list(spe[o] for o, _ in m_states(orbits)) * 2)
    Hop = sp.csr_matrix((dimF, dimF))
    for s in range(S):
        Hop = Hop + e[s] * (cd[s] @ c[s])
    for (a, b, cc, d), h in mscheme_terms(orbits, tb).items():
        Hop = Hop + h * (cd[a] @ cd[b] @ c[d] @ c[cc])
    want = B.T @ (Hop @ B)
    assert np.allclose(B.T @ B, np.eye(model.dim))
    assert np.abs(model.dense() - want).max() < 1e-12


def test_rows_equal_columns_transposed():
    for orbits, z, n, seed in ((SD_ORBITS, 2, 2, 1), (PF_ORBITS, 2, 1, 2), (SD_ORBITS, 3, 2, 3)):
        twoM = (z + n) % 2
        spe_p = [0.3 * k - 1.0 for k in range(len(orbits))]
        spe_n = [0.1] * len(orbits)
        m = Model(orbits, z, n, twoM, random_tbme(orbits, seed), spe_p, spe_n)
        idx = np.arange(m.dim)
        pr, cr, vr = m.rows(idx)
        Hr = sp.csr_matrix((vr, cr, pr), shape=(m.dim, m.dim))
        pc, cc, vc = m.columns(idx)
        Hc = sp.csr_matrix((vc, cc, pc), shape=(m.dim, m.dim))
        assert abs(Hr - Hc.T).max() < 1e-13
        assert abs(Hr - Hr.T).max() < 1e-13


def _mzero_count(twoj, k):
    ms = range(-twoj, twoj + 1, 2)
    return sum(1 for sub in itertools.combinations(ms, k) if sum(sub) == 0)


@pytest.mark.parametrize("orbits,n", [(F72, 4), (H112, 6), (F72, 2), (H112, 4)])
def test_seniority_single_shell(orbits, n):
    """Pairing V_0 = -G*Omega: E = -(G/4)(n-v)(2 Omega - n - v + 2), M=0 multiplicity d(v)-d(v-2)."""
    G = 1.0
    twoj = orbits[0][2]
    omega = (twoj + 1) // 2
    m = Model(orbits, n, 0, 0, pairing_tbme(orbits, G), (0.0,), (0.0,))
    ev = np.linalg.eigvalsh(m.dense())
    want = []
    for v in range(n % 2, n + 1, 2):
        mult = _mzero_count(twoj, v) - (_mzero_count(twoj, v - 2) if v >= 2 else 0)
        want += [-(G / 4) * (n - v) * (2 * omega - n - v + 2)] * mult
    assert len(want) == m.dim
    assert np.allclose(np.sort(want), ev, atol=1e-12)


def test_seniority_two_species_f72():
    m = Model(F72, 4, 4, 0, pairing_tbme(F72, 1.0), (0.0,), (0.0,))
    ev = np.linalg.eigvalsh(m.dense())
    assert m.dim == 390
    assert ev[0] == pytest.approx(-12.0, abs=1e-12) and ev[1] > -11.9
    assert np.allclose(ev[1:7], -8.0, atol=1e-12) and ev[7] > -7.9


@pytest.mark.parametrize("orbits,z,n", [(SD_ORBITS, 2, 2), (SD_ORBITS, 3, 2), (PF_ORBITS, 2, 2)])
def test_jsquared_eigenvalues(orbits, z, n):
    """J^2 as an interaction: every eigenvalue is J(J+1), multiplicity D(M=J) - D(M=J+1)."""
    twoM = (z + n) % 2
    spe = jsquared_spe(orbits)
    m = Model(orbits, z, n, twoM, jsquared_tbme(orbits), spe, spe)
    ev = np.linalg.eigvalsh(m.dense())
    tJ = np.rint(np.sqrt(4 * ev + 1) - 1).astype(int)          # 2J from J(J+1)
    assert np.allclose(ev, tJ / 2 * (tJ / 2 + 1), atol=1e-10)
    for t in sorted(set(tJ)):
        mult = count_dim(orbits, z, orbits, n, t) - count_dim(orbits, z, orbits, n, t + 2)
        assert int(np.sum(tJ == t)) == mult


def test_rotational_invariance_random():
    """Every M=1 eigenvalue of a random rotationally invariant H is an M=0 eigenvalue."""
    tb = random_tbme(SD_ORBITS, 11)
    e0 = np.linalg.eigvalsh(Model(SD_ORBITS, 2, 2, 0, tb, SD_SPE, SD_SPE).dense())
    m1 = Model(SD_ORBITS, 2, 2, 2, tb, SD_SPE, SD_SPE)
    e1 = np.linalg.eigvalsh(m1.dense())
    assert m1.dim == 594
    d = np.array([np.min(np.abs(e0 - x)) for x in e1])
    assert d.max() < 1e-10
    unmatched = sum(1 for x in e0 if np.min(np.abs(e1 - x)) > 1e-8)
    assert unmatched == 640 - 594


def test_single_particle_energies_only():
    """H = sum e_a n_a: eigenvalues are occupation sums, multiplicity = number of such M=0 states."""
    orbits, spe_p, spe_n = SD_ORBITS, (-3.9, -3.2, 2.1), (-1.0, 0.25, 3.0)
    m = Model(orbits, 2, 2, 0, [], spe_p, spe_n)
    ev = np.linalg.eigvalsh(m.dense())
    ms = [(o, tm) for o, (_n, _l, tj) in enumerate(orbits) for tm in range(-tj, tj + 1, 2)]
    want = []
    for po in itertools.combinations(range(len(ms)), 2):
        for no in itertools.combinations(range(len(ms)), 2):
            if sum(ms[s][1] for s in po) + sum(ms[s][1] for s in no) == 0:
                want.append(sum(spe_p[ms[s][0]] for s in po) + sum(spe_n[ms[s][0]] for s in no))
    assert np.allclose(np.sort(want), ev, atol=1e-12)
    # ground value of the sd22 workload's energies: all four nucleons in d5/2
    m2 = Model(orbits, 2, 2, 0, [], SD_SPE, SD_SPE)
    ev2 = np.linalg.eigvalsh(m2.dense())
    assert ev2[0] == pytest.approx(-15.6, abs=1e-12)
    assert int(np.sum(np.abs(ev2 + 15.6) < 1e-9)) == 29


def test_reordered_pair_matches_direct_expansion():
    """An element given as (ba,cd) expanded operator by operator equals the oracle's phase rule."""
    orbits = SD_ORBITS
    states = m_states(orbits)
    for (ch, a, b, c, d, twoJ, v) in [(0, 0, 2, 0, 2, 2, 0.7), (1, 1, 2, 0, 1, 4, -1.1), (0, 0, 2, 1, 2, 2, 0.3)]:
        # reordered element V_J(ba, dc) as a user might list it
        given = (ch, b, a, d, c, twoJ, v)
        terms = mscheme_terms(orbits, [given])
        # direct: A+_JM(ba) = sum CG(jb mb ja ma|JM) c+_b c+_a (a != b), A_JM(dc) its adjoint,
        # H = v (A+(ba) A(dc) + A+(dc) A(ba)); normal-order each product to alpha<beta, gamma<delta
        off = 0 if ch == 0 else len(states)
        direct = {}

        def add(x, y, z, w, val):
            sgn = 1.0
            if x > y:
                x, y, sgn = y, x, -sgn
            if z > w:
                z, w, sgn = w, z, -sgn
            direct[(x, y, z, w)] = direct.get((x, y, z, w), 0.0) + sgn * val

        prods = [((b, a), (d, c))] + ([((d, c), (b, a))] if (b, a) != (d, c) else [])
        for (p1, p2), (q1, q2) in prods:
            for s1, (o1, m1) in enumerate(states):
                for s2, (o2, m2) in enumerate(states):
                    if o1 != p1 or o2 != p2:
                        continue
                    c1 = cg(orbits[p1][2], m1, orbits[p2][2], m2, twoJ, m1 + m2)
                    for s3, (o3, m3) in enumerate(states):
                        for s4, (o4, m4) in enumerate(states):
                            if o3 != q1 or o4 != q2 or m3 + m4 != m1 + m2:
                                continue
                            c2 = cg(orbits[q1][2], m3, orbits[q2][2], m4, twoJ, m3 + m4)
                            # c+_s1 c+_s2 c_s4 c_s3
                            add(s1 + off, s2 + off, s3 + off, s4 + off, v * c1 * c2)
        keys = set(terms) | set(direct)
        for k in keys:
            assert terms.get(k, 0.0) == pytest.approx(direct.get(k, 0.0), abs=1e-13)


def test_hermitian_trace_and_sparse_rows():
    tb = random_tbme(SD_ORBITS, 1)
    m = Model(SD_ORBITS, 2, 2, 0, tb, SD_SPE, SD_SPE)
    H = m.dense()
    ev = np.linalg.eigvalsh(H)
    assert np.trace(H) == pytest.approx(ev.sum(), rel=1e-12)
    rng = np.random.default_rng(0)
    V = rng.standard_normal((m.dim, 3))
    idx = rng.choice(m.dim, 50, replace=False)
    assert np.allclose(m.apply_rows(V, idx), (H @ V)[idx], atol=1e-12)


def _move_linked_pairs(words):
    """Pairs (i, j) of basis states whose occupations differ by at most two particles moved
    (i == j included): every pair a one- plus two-body H can link, allowed J or not."""
    w = np.asarray(words, dtype=np.uint64)
    cnt = 0
    for x in w:
        diff = np.bitwise_xor(w, x)
        nbits = np.array([bin(int(d)).count("1") for d in diff])
        cnt += int(np.count_nonzero(nbits <= 4))  # a move clears one bit and sets another
    return cnt


@pytest.mark.parametrize("orbits,z,n,twoM,seed,nnz", [
    (SD_ORBITS, 2, 2, 0, 1, 54112),   # sd22 workload: 54,112 = non-zeros of H
    (SD_ORBITS, 3, 2, 1, 4, None),    # odd A
])
def test_row_nnz_counts_the_nonzeros(orbits, z, n, twoM, seed, nnz):
    """Model.row_nnz (the structural count behind the H.V flop count) counts, per row, the
    distinct columns some term reaches, diagonal included: the non-zeros of H, plus entries whose
    terms cancel exactly (none in sd22; two in this odd-A space). Pairs linked by a move of at
    most two particles but with no common allowed J (sd22: 54,624 such pairs) have no matrix
    element and are not counted."""
    tb = random_tbme(orbits, seed)
    m = Model(orbits, z, n, twoM, tb, SD_SPE, SD_SPE)
    H = m.dense()
    rn = m.row_nnz()
    nz = np.count_nonzero(H, axis=1)
    ptr, col, val = m.rows(np.arange(m.dim))
    zeros = np.add.reduceat((val == 0.0).astype(np.int64), ptr[:-1])
    assert np.array_equal(rn, nz + zeros)
    if nnz is not None:
        assert rn.sum() == nnz and zeros.sum() == 0
    linked = _move_linked_pairs(m.words)
    assert linked >= rn.sum()
    if nnz is not None:
        assert linked == 54624


def test_rows_generated_are_the_term_applications():
    """rows_generated lists, per row, the single-particle diagonal plus one entry per m-scheme
    term whose adjoint maps the row's state into the basis: pinned against a pure-Python
    application of every term to every state, and merged it gives rows()."""
    orbits = SD_ORBITS
    tb = random_tbme(orbits, 6)
    m = Model(orbits, 2, 1, 1, tb, SD_SPE, SD_SPE)
    terms = mscheme_terms(orbits, tb)
    words = [int(x) for x in m.words]
    index = {w: i for i, w in enumerate(words)}

    def op(w, s, create, sign):
        bit = 1 << s
        if bool(w & bit) == create:
            return None, sign
        sign *= -1 if bin(w & (bit - 1)).count("1") % 2 else 1
        return (w | bit) if create else (w & ~bit), sign

    ptr, col, val = m.rows_generated(np.arange(m.dim))
    for i, w in enumerate(words):
        expect = []
        for (a, b, c, d), h in terms.items():
            # adjoint of c+_a c+_b c_d c_c acting on <i|: remove a and b, then create d and c
            x, sg = w, 1
            for s, cr in ((a, False), (b, False), (d, True), (c, True)):
                x, sg = op(x, s, cr, sg)
                if x is None:
                    break
            if x is not None and x in index:
                expect.append((index[x], sg * h))
        got = sorted(zip(col[ptr[i] + 1:ptr[i + 1]].tolist(), val[ptr[i] + 1:ptr[i + 1]].tolist()))
        assert col[ptr[i]] == i  # the one-body diagonal comes first
        assert len(got) == len(expect)
        for (cg_, vg), (ce, ve) in zip(got, sorted(expect)):
            assert cg_ == ce and abs(vg - ve) <= 1e-14 * max(1.0, abs(ve))
    # merged by column, the generated entries are the rows of H
    pr, cr_, vr = m.rows(np.arange(m.dim))
    for i in range(m.dim):
        acc = {}
        for j, v in zip(col[ptr[i]:ptr[i + 1]], val[ptr[i]:ptr[i + 1]]):
            acc[int(j)] = acc.get(int(j), 0.0) + v
        assert sorted(acc) == cr_[pr[i]:pr[i + 1]].tolist()
        for j, v in zip(cr_[pr[i]:pr[i + 1]], vr[pr[i]:pr[i + 1]]):
            assert abs(acc[int(j)] - v) <= 1e-13 * max(1.0, abs(v))
