"""Parity of the HIP block H.V (trbl_apply) with the oracle's explicit H (GPU)."""
import numpy as np
import pytest

import os

from gpu_common import fp32_bound, fp64_bound, pair, say, term_bound
from workloads import PF_ORBITS, SD_ORBITS, SD_SPE, PF_SPE, WORKLOADS, random_block, random_tbme

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIXED_PAR = ((0, 1, 1), (0, 2, 5), (0, 1, 3))  # p1/2 d5/2 p3/2: both parities present

CASES = [
    # name, orbits, Z, N, 2M, parity, seed, nb
    ("sd22_nb4", SD_ORBITS, 2, 2, 0, 0, 1, 4),
    ("sd32_odd_nb3", SD_ORBITS, 3, 2, 1, 0, 2, 3),
    ("sd22_m2_nb1", SD_ORBITS, 2, 2, 2, 0, 3, 1),
    ("pf22_nb16", PF_ORBITS, 2, 2, 0, 0, 4, 16),
    ("pf31_nb64", PF_ORBITS, 3, 1, 0, 0, 5, 64),
    ("mixpar_pos_nb5", MIXED_PAR, 2, 2, 0, 1, 6, 5),
    ("mixpar_neg_nb8", MIXED_PAR, 2, 1, 1, -1, 7, 8),
    ("mixpar_both_nb2", MIXED_PAR, 1, 2, 1, 0, 8, 2),
    ("sd_protons_only", SD_ORBITS, 3, 0, 1, 0, 9, 4),
    ("sd_neutrons_only", SD_ORBITS, 0, 4, 0, 0, 10, 4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_apply_matches_dense_oracle(case):
    name, orbits, z, n, twoM, par, seed, nb = case
    say("case", name)
    spe = [(-1.5 + 0.7 * k) for k in range(len(orbits))]
    spn = [(0.3 - 0.4 * k) for k in range(len(orbits))]
    g, o = pair(orbits, z, n, twoM, random_tbme(orbits, seed), spe, spn, par)
    assert g.dim == o.dim
    H = o.dense()
    nnz = int(np.max(np.count_nonzero(H, axis=1)))
    V = random_block(100 + seed, o.dim, nb)
    ref = H @ V
    # per-term bound: the FP64 product sums the pn terms of each core pair unmerged
    ex = z * n + 64  # slot sum and pair blocks of the pn kernel
    bound = term_bound(o, np.arange(o.dim), V, extra=ex)
    W = g.apply(torch.from_numpy(V).cuda()).cpu().numpy()
    assert np.all(np.abs(W - ref) <= bound), np.max(np.abs(W - ref) / bound)
    # mixed precision: FP32 vectors, FP32 coefficients, FP32 accumulation (per-term bound, as above)
    V32 = V.astype(np.float32)
    ref32 = H @ V32.astype(np.float64)
    W32 = g.apply(torch.from_numpy(V32).cuda()).cpu().numpy().astype(np.float64)
    b32 = term_bound(o, np.arange(o.dim), V32, fp32=True, extra=ex)
    assert np.all(np.abs(W32 - ref32) <= b32), np.max(np.abs(W32 - ref32) / b32)


PATH_CASES = [
    # name, orbits, Z, N, 2M, parity, seed, nb: the pn part by core-pair blocks (one 16-column
    # tile summed by the own-row kernel, several tiles, narrower tiles) against the jump-list kernel
    ("pf22_nb16", PF_ORBITS, 2, 2, 0, 0, 4, 16),
    ("pf31_nb40", PF_ORBITS, 3, 1, 0, 0, 5, 40),
    ("sd32_odd_nb5", SD_ORBITS, 3, 2, 1, 0, 2, 5),
    ("mixpar_neg_nb12", MIXED_PAR, 2, 1, 1, -1, 7, 12),
    ("sd22_nb1", SD_ORBITS, 2, 2, 0, 0, 8, 1),
    ("pf22_nb3", PF_ORBITS, 2, 2, 2, 0, 9, 3),
]


@pytest.mark.parametrize("case", PATH_CASES, ids=lambda c: c[0])
def test_pair_blocks_match_jump_lists(case):
    """The two pn kernels (pair blocks on the matrix cores, and the jump-list rows kernel
    selected with TRBL_PN_TILES=0 at set-up) agree within the sum of their rounding bounds, and
    each matches the oracle, in FP64 and in FP32."""
    name, orbits, z, n, twoM, par, seed, nb = case
    say("case", name)
    tb = random_tbme(orbits, seed)
    spe = [(-1.5 + 0.7 * k) for k in range(len(orbits))]
    old = os.environ.get("TRBL_PN_TILES")
    try:
        os.environ["TRBL_PN_TILES"] = "2"  # pair blocks at every width
        g, o = pair(orbits, z, n, twoM, tb, spe, spe, par)
        os.environ["TRBL_PN_TILES"] = "0"  # jump lists
        g0, _ = pair(orbits, z, n, twoM, tb, spe, spe, par, oracle=False)
    finally:
        if old is None:
            del os.environ["TRBL_PN_TILES"]
        else:
            os.environ["TRBL_PN_TILES"] = old
    V = random_block(300 + seed, o.dim, nb)
    Vt = torch.from_numpy(V).cuda()
    W1 = g.apply(Vt).cpu().numpy()
    W0 = g0.apply(Vt).cpu().numpy()
    idx = np.arange(o.dim)
    ex = z * n + 64  # slot sum and pair blocks of the pn kernel
    bound = term_bound(o, idx, V, extra=ex)
    ref = o.apply_rows(V, idx)
    assert np.all(np.abs(W1 - ref) <= bound)
    assert np.all(np.abs(W0 - ref) <= bound)
    assert np.all(np.abs(W1 - W0) <= 2 * bound)
    # FP32 (mixed-precision) products of both kernels
    V32 = V.astype(np.float32)
    V32t = torch.from_numpy(V32).cuda()
    X1 = g.apply(V32t).cpu().numpy().astype(np.float64)
    X0 = g0.apply(V32t).cpu().numpy().astype(np.float64)
    b32 = term_bound(o, idx, V32, fp32=True, extra=ex)
    ref32 = o.apply_rows(V32.astype(np.float64), idx)
    assert np.all(np.abs(X1 - ref32) <= b32)
    assert np.all(np.abs(X0 - ref32) <= b32)


def test_apply_deterministic_and_linear():
    g, o = pair(SD_ORBITS, 2, 2, 0, random_tbme(SD_ORBITS, 1), SD_SPE, SD_SPE, oracle=False)
    V = torch.from_numpy(random_block(5, g.dim, 4)).cuda()
    W1 = g.apply(V)
    W2 = g.apply(V)
    assert torch.equal(W1, W2)
    # nb columns are independent: the single-column product equals the corresponding column
    W3 = g.apply(V[:, 2:3].contiguous())
    assert torch.equal(W3[:, 0], W1[:, 2])


@pytest.mark.parametrize("wname,nrows", [("pf44", 300), ("sd66", 300)])
def test_apply_full_size_sampled_rows(wname, nrows):
    """Full-size workload in the bench's launch configuration; oracle rows computed one by one."""
    w = WORKLOADS[wname]
    say("case", wname, "full size")
    g, o = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, w.tbme(), w.spe, w.spe)
    assert g.dim == o.dim
    V = random_block(2000, g.dim, w.nb)
    W = g.apply(torch.from_numpy(V).cuda()).cpu().numpy()
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(g.dim, nrows, replace=False), [0, g.dim - 1]]))
    ref = o.apply_rows(V, idx)
    ptr, col, val = o.rows(idx)
    nnz = int(np.max(np.diff(ptr)))
    ex = w.n_prot * w.n_neut + 64  # slot sum and pair blocks of the pn kernel
    assert np.all(np.abs(W[idx] - ref) <= term_bound(o, idx, V, extra=ex))
    # FP32 path on the same rows
    V32 = V.astype(np.float32)
    W32 = g.apply(torch.from_numpy(V32).cuda()).cpu().numpy().astype(np.float64)
    ref32 = o.apply_rows(V32.astype(np.float64), idx)
    assert np.all(np.abs(W32[idx] - ref32) <= term_bound(o, idx, V32, fp32=True, extra=ex))


def test_apply_pf66_sampled_rows():
    """pf shell 6+6 (D = 109,954,620; neutron sectors up to 3,952 SDs, so the widest source rows go
    through the 144 KB single row buffer, 4 targets per lane, and the columns kernel takes a
    narrower tile): 60 sampled rows against the oracle. nb = 8 (FP64 tile of 4 columns, FP32 of
    8), host-side input 7 GB."""
    w = WORKLOADS["pf66"]
    say("case pf66 full size, nb=8")
    g, o = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, w.tbme(), w.spe, w.spe)
    assert g.dim == o.dim == 109954620
    V = random_block(2000, g.dim, 8)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.choice(g.dim, 60, replace=False), [0, g.dim - 1]]))
    ref = o.apply_rows(V, idx)
    ptr, col, val = o.rows(idx)
    absHV = np.zeros_like(ref)
    for r in range(len(idx)):
        sl = slice(ptr[r], ptr[r + 1])
        absHV[r] = np.abs(val[sl]) @ np.abs(V[col[sl]])
    nnz = int(np.max(np.diff(ptr)))
    Vd = torch.from_numpy(V).cuda()
    W = g.apply(Vd)[torch.from_numpy(idx).cuda()].cpu().numpy()
    say("pf66 fp64 max err", np.abs(W - ref).max())
    assert np.all(np.abs(W - ref) <= fp64_bound(absHV, nnz))
    del Vd
    V32 = V.astype(np.float32)
    del V
    W32 = g.apply(torch.from_numpy(V32).cuda())[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    ref32 = o.apply_rows(V32.astype(np.float64), idx)
    assert np.all(np.abs(W32 - ref32) <= fp32_bound(absHV * 1.0001, nnz))
