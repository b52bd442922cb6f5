"""Bit-exact basis indexing of the library (host and device kernels) against the oracle (GPU)."""
import numpy as np
import pytest

from gpu_common import pair, say
from oracle.basis import ProductBasis
from workloads import PF_ORBITS, SD_ORBITS, TABLE1_ORBITS, random_tbme

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1902_02064_amd as trbl

MIXED_PAR = ((0, 1, 1), (0, 2, 5), (0, 1, 3))


@pytest.mark.parametrize("orbits,z,n,twoM,par", [
    (SD_ORBITS, 2, 2, 0, 0), (SD_ORBITS, 3, 2, 1, 0), (PF_ORBITS, 4, 4, 0, 0), (PF_ORBITS, 3, 2, -3, 0),
    (MIXED_PAR, 2, 2, 0, 1), (MIXED_PAR, 2, 1, 1, 0), (TABLE1_ORBITS, 3, 0, 1, 0), (SD_ORBITS, 6, 6, 0, 0)],
    ids=["sd22", "sd32", "pf44", "pf32m3", "mix_pos", "mix_both", "table1", "sd66"])
def test_unrank_rank_bit_exact(orbits, z, n, twoM, par):
    say("basis", orbits, z, n, twoM, par)
    g = trbl.Model(orbits, z, n, twoM, par)
    b = ProductBasis(orbits, z, n, twoM, par)
    assert g.dim == b.dim
    st = b.states()
    pw = np.array([p for p, _ in st], dtype=np.uint64).view(np.int64)
    nw = np.array([q for _, q in st], dtype=np.uint64).view(np.int64)
    idx = torch.arange(g.dim, dtype=torch.int64, device="cuda")
    p, q = g.unrank_dev(idx)
    assert np.array_equal(p.cpu().numpy(), pw) and np.array_equal(q.cpu().numpy(), nw)
    r = g.rank_dev(torch.from_numpy(pw).cuda(), torch.from_numpy(nw).cuda())
    assert torch.equal(r, idx)
    # host-side calls on a sample
    for i in np.linspace(0, g.dim - 1, 50).astype(int):
        assert g.unrank(i) == st[i]
        assert g.rank(*st[i]) == i
    # states outside the basis rank to -1 (wrong M, wrong particle number, stray high bit)
    bad_p = torch.tensor([int(pw[0]) ^ 1, 0, int(pw[0]) | (1 << 62)], dtype=torch.int64, device="cuda")
    bad_n = torch.tensor([int(nw[0]), int(nw[0]), int(nw[0])], dtype=torch.int64, device="cuda")
    assert torch.all(g.rank_dev(bad_p, bad_n) == -1)


def test_empty_space_rejected():
    with pytest.raises(trbl.TrblError):
        trbl.Model(SD_ORBITS, 2, 2, 1, 0)  # even A with odd 2M
