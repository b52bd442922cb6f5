"""trbl_expect_noalloc (the entry point that allocates nothing, for callers that cannot) against
trbl_expect through the C ABI (GPU): two calls in a row, the second with fewer columns, on a
space that takes 16-column products and on one that takes 2-column products."""
import numpy as np
import pytest

from gpu_common import pair, say
from workloads import WORKLOADS, random_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dot_bound(X, HX):
    """Two summations of the same D products in different orders: each within gamma_D of
    sum |x| |Hx| (the products themselves are the same H X columns, bit for bit)."""
    u = 2.0 ** -53
    D = X.shape[0]
    return 2 * D * u / (1 - D * u) * np.sum(np.abs(X) * np.abs(HX), axis=0) + 1e-300


@pytest.mark.parametrize("wname,ncols", [("sd66", (21, 5)), ("pf44", (7, 3))])
def test_expect_noalloc_matches_expect(wname, ncols):
    w = WORKLOADS[wname]
    say("no-alloc expect", wname)
    g, _ = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, w.tbme(), w.spe, w.spe, oracle=False)
    for call, n in enumerate(ncols):
        X = torch.from_numpy(random_block(300 + call, g.dim, n)).cuda()
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        g.expect_noalloc(X, out)
        got = out.cpu().numpy()
        ref = g.expect(X)
        HX = g.apply(X).cpu().numpy()
        bound = _dot_bound(X.cpu().numpy(), HX)
        say("call", call, "n", n, "max |diff| / bound", np.max(np.abs(got - ref) / bound))
        assert np.all(np.isfinite(got))
        assert np.all(np.abs(got - ref) <= bound)


def test_expect_noalloc_errors():
    import paper_1902_02064_amd as trbl
    w = WORKLOADS["sd66"]
    g, _ = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, w.tbme(), w.spe, w.spe, oracle=False)
    lib = trbl.load()
    assert lib.trbl_expect_noalloc(g._h, 0, None, None, None) == -1
    m = trbl.Model(w.orbits, w.n_prot, w.n_neut, w.twoM)
    X = torch.zeros((m.dim, 2), dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert lib.trbl_expect_noalloc(m._h, 2, trbl._ptr(X), trbl._ptr(out), trbl._stream()) == -7  # no H yet
