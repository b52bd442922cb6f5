"""Pins of the oracle's basis against numbers the paper prints (CPU only)."""
import os

import numpy as np

import pytest

from oracle.basis import ProductBasis, count_dim, count_sds, sector_words, species_sectors
from workloads import PF_ORBITS, SD_ORBITS, SNSB_ORBITS, TABLE1_ORBITS, random_tbme

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ORB = {"sd": SD_ORBITS, "pf": PF_ORBITS, "snsb": SNSB_ORBITS}


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if line:
            out.append(line.split())
    return out


def test_table1_order_bit_exact():
    """Table 1: the nine 3-particle d5/2+s1/2 determinants at M=1/2, serial order and partitions."""
    sec = species_sectors(TABLE1_ORBITS, 3)[(1, 1)]
    rows = _rows("table1.txt")
    assert len(sec) == len(rows) == 9
    for (word, part), row in zip(sec, rows):
        bits = "".join("1" if word >> s & 1 else "0" for s in range(8))
        assert bits == row[1]
        assert part == (int(row[2]), int(row[3]))


@pytest.mark.parametrize("row", _rows("dimensions.txt"), ids=lambda r: r[0])
def test_printed_dimensions_dp(row):
    name, orb, z, n, par, dim = row[0], row[1], int(row[2]), int(row[3]), int(row[4]), int(row[5])
    o = ORB[orb]
    assert count_dim(o, z, o, n, 0, par) == dim


@pytest.mark.parametrize("row", [r for r in _rows("dimensions.txt") if int(r[5]) < 10_000_000],
                         ids=lambda r: r[0])
def test_printed_dimensions_enumerated(row):
    o = ORB[row[1]]
    b = ProductBasis(o, int(row[2]), int(row[3]), 0, int(row[4]))
    assert b.dim == int(row[5])


def test_sector_words_matches_full_enumeration():
    """The per-sector enumerator (used for large species) gives every sector of the full
    subset enumeration in the same Table-1 order."""
    for orbits, n in ((TABLE1_ORBITS, 3), (SD_ORBITS, 3), (PF_ORBITS, 4), (SNSB_ORBITS, 3), (SNSB_ORBITS, 4)):
        for (tm, par), lst in species_sectors(orbits, n).items():
            want = np.array([w for w, _ in lst], dtype=np.uint64)
            assert np.array_equal(sector_words(orbits, n, tm, par), want), (n, tm, par)


def test_sn112_words_are_the_sector():
    """112Sn (Sec. 4.2): the enumerated positive-parity M = 0 sector has the printed dimension,
    and every word is a distinct 12-neutron determinant with 2M = 0 and parity +."""
    w = sector_words(SNSB_ORBITS, 12, 0, 1)
    assert len(w) == 6210638
    assert len(np.unique(w)) == len(w)
    states = [(o, tm) for o, (_n, _l, tj) in enumerate(SNSB_ORBITS) for tm in range(-tj, tj + 1, 2)]
    rng = np.random.default_rng(0)
    for word in w[rng.integers(0, len(w), 200)]:
        occ = [s for s in range(len(states)) if int(word) >> s & 1]
        assert len(occ) == 12
        assert sum(states[s][1] for s in occ) == 0
        assert sum(SNSB_ORBITS[states[s][0]][1] for s in occ) % 2 == 0


def test_dp_matches_enumeration_all_sectors():
    for orbits, n in ((SD_ORBITS, 3), (PF_ORBITS, 4), (SNSB_ORBITS, 2)):
        enum = {k: len(v) for k, v in species_sectors(orbits, n).items()}
        assert enum == count_sds(orbits, n)


@pytest.mark.parametrize("row", _rows("partitions.txt"), ids=lambda r: r[0])
def test_partition_counts(row):
    """Partitions Gamma = (N^p, N^n, M^p) with a non-empty product space (App. A, App. C.1)."""
    o = ORB[row[1]]
    z, n, want = int(row[2]), int(row[3]), int(row[4])
    ps, ns = species_sectors(o, z), species_sectors(o, n)
    pkeys = {(part, m) for (m, _p), lst in ps.items() for _w, part in lst}
    nkeys = {(part, m) for (m, _p), lst in ns.items() for _w, part in lst}
    cnt = sum(1 for (_a, m) in pkeys for (_b, mn) in nkeys if m + mn == 0)
    assert cnt == want


def test_product_basis_layout():
    b = ProductBasis(SD_ORBITS, 2, 2, 0)
    st = b.states()
    assert len(st) == len(set(st)) == b.dim
    keys = [(blk.twoMp, -blk.parp, -blk.parn) for blk in b.blocks]
    assert keys == sorted(keys)
    for blk in b.blocks:
        plist = b.psec[(blk.twoMp, blk.parp)]
        nlist = b.nsec[(blk.twoMn, blk.parn)]
        assert blk.twoMp + blk.twoMn == 0
        for p in range(blk.dp):
            for n in range(blk.dn):
                assert st[blk.offset + p * blk.dn + n] == (plist[p][0], nlist[n][0])


def test_tbme_counts_pn_formalism():
    """Independent pn-formalism elements: sd 30+30+98, pf 94+94+330."""
    for orbits, want in ((SD_ORBITS, (30, 30, 98)), (PF_ORBITS, (94, 94, 330))):
        t = random_tbme(orbits, 1)
        got = tuple(sum(1 for x in t if x[0] == ch) for ch in (0, 1, 2))
        assert got == want


def test_combined_words_array_matches_list():
    """The block-wise uint64 construction gives the same words, in the same order, as the plain one."""
    from oracle.basis import ProductBasis
    from workloads import PF_ORBITS, SD_ORBITS
    for orbits, z, n, twoM, par in ((SD_ORBITS, 2, 2, 0, 0), (SD_ORBITS, 3, 2, 1, -1), (PF_ORBITS, 2, 3, 1, 0)):
        b = ProductBasis(orbits, z, n, twoM, par)
        arr = b.combined_words_array()
        assert arr.dtype == np.uint64 and len(arr) == b.dim
        assert [int(x) for x in arr] == b.combined_words()
