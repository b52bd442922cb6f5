"""Single-species spaces with the identical-particle part generated per element (GPU).

Small spaces are forced onto that path (TRBL_FLY=1 at model creation) and compared with the
oracle's explicit H; the 112Sn-shaped space (Sec. 4.2, D = 6,210,638) takes it by itself and
is checked on sampled rows against the oracle, and through a short solve whose Ritz pairs
are checked with the oracle's rows of H.
"""
import os

import numpy as np
import pytest

from gpu_common import pair, say, term_bound
from oracle.hamiltonian import Model as OracleModel
from workloads import SD_ORBITS, SNSB_ORBITS, WORKLOADS, jsquared_spe, jsquared_tbme, random_block, random_tbme

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIXED_PAR = ((0, 1, 1), (0, 2, 5), (0, 1, 3))

CASES = [
    # name, orbits, Z, N, 2M, parity, seed, nb
    ("sd_n4", SD_ORBITS, 0, 4, 0, 0, 21, 4),
    ("sd_z3_odd", SD_ORBITS, 3, 0, 1, 0, 22, 5),
    ("mixpar_n3_both", MIXED_PAR, 0, 3, 1, 0, 23, 16),
    ("mixpar_z2_neg", MIXED_PAR, 2, 0, 0, -1, 24, 1),
    ("snsb_n4_pos", SNSB_ORBITS, 0, 4, 0, 1, 25, 20),
]


def _forced(orbits, z, n, twoM, tb, spe, par):
    os.environ["TRBL_FLY"] = "1"
    try:
        return pair(orbits, z, n, twoM, tb, spe, spe, par)
    finally:
        del os.environ["TRBL_FLY"]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_fly_matches_dense_oracle(case):
    name, orbits, z, n, twoM, par, seed, nb = case
    say("fly case", name)
    spe = [(-0.8 + 0.5 * k) for k in range(len(orbits))]
    tb = random_tbme(orbits, seed)
    g, o = _forced(orbits, z, n, twoM, tb, spe, par)
    assert g.dim == o.dim
    H = o.dense()
    rows = np.arange(o.dim)
    V = random_block(200 + seed, o.dim, nb)
    ref = H @ V
    W = g.apply(torch.from_numpy(V).cuda()).cpu().numpy()
    # the pair-block path sums blocks of at most 64 pairs, then the C(n, 2) core slots
    npart = z + n
    ex = npart * (npart - 1) // 2 + 64
    bound = term_bound(o, rows, V, extra=ex)
    say("fp64 max err / bound", np.max(np.abs(W - ref) / bound))
    assert np.all(np.abs(W - ref) <= bound)
    V32 = V.astype(np.float32)
    W32 = g.apply(torch.from_numpy(V32).cuda()).cpu().numpy()
    ref32 = H @ V32.astype(np.float64)
    b32 = term_bound(o, rows, V32, fp32=True, extra=ex)
    say("fp32 max err / bound", np.max(np.abs(W32 - ref32) / b32))
    assert np.all(np.abs(W32 - ref32) <= b32)


@pytest.mark.parametrize("case", CASES[:3] + CASES[4:], ids=lambda c: c[0])
def test_fly_pair_blocks_match_per_element_kernel(case):
    """The single-species two-body part by pair blocks (the default) and by the per-element kernel
    (TRBL_PN_TILES=0 at set-up): both within the per-term bound of the oracle, FP64 and FP32."""
    name, orbits, z, n, twoM, par, seed, nb = case
    say("fly paths", name)
    spe = [(-0.8 + 0.5 * k) for k in range(len(orbits))]
    tb = random_tbme(orbits, seed)
    g1, o = _forced(orbits, z, n, twoM, tb, spe, par)
    os.environ["TRBL_PN_TILES"] = "0"
    try:
        g0, _ = _forced(orbits, z, n, twoM, tb, spe, par)
    finally:
        del os.environ["TRBL_PN_TILES"]
    H = o.dense()
    rows = np.arange(o.dim)
    npart = z + n
    ex = npart * (npart - 1) // 2 + 64
    for dt, fp32 in ((np.float64, False), (np.float32, True)):
        V = random_block(400 + seed, o.dim, nb).astype(dt)
        ref = H @ V.astype(np.float64)
        bound = term_bound(o, rows, V, fp32=fp32, extra=ex)
        Vt = torch.from_numpy(V).cuda()
        for g in (g0, g1):
            W = g.apply(Vt).cpu().numpy().astype(np.float64)
            assert np.all(np.abs(W - ref) <= bound)


def test_fly_same_as_staged_path():
    """The same small space through both paths: equal to rounding."""
    tb = random_tbme(SNSB_ORBITS, 26)
    spe = (0.0, 0.2, 1.5, 1.8, 2.4)
    g1, _ = _forced(SNSB_ORBITS, 0, 3, 1, tb, spe, 0)
    g0, _ = pair(SNSB_ORBITS, 0, 3, 1, tb, spe, spe, 0, oracle=False)
    V = torch.from_numpy(random_block(31, g0.dim, 8)).cuda()
    a, b = g0.apply(V).cpu().numpy(), g1.apply(V).cpu().numpy()
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


@pytest.fixture(scope="module")
def sn112():
    w = WORKLOADS["sn112"]
    tb = w.tbme()
    say("building sn112 (library, then oracle)")
    g, _ = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, tb, w.spe, w.spe, w.parity, oracle=False)
    o = OracleModel(w.orbits, w.n_prot, w.n_neut, w.twoM, tb, w.spe, w.spe, w.parity)
    return w, g, o


def test_sn112_sampled_rows(sn112):
    """112Sn shape (D = 6,210,638): sampled rows of H V (FP64, 16 columns) against the oracle's
    rows of H, including both ends of the space."""
    w, g, o = sn112
    assert g.dim == o.dim == 6210638
    V = random_block(41, g.dim, 16)
    W = g.apply(torch.from_numpy(V).cuda()).cpu().numpy()
    rows = np.unique(np.concatenate([[0, 1, g.dim - 2, g.dim - 1],
                                     np.random.default_rng(5).integers(0, g.dim, 300)]))
    ref = o.apply_rows(V, rows)
    bound = term_bound(o, rows, V, extra=w.n_neut * (w.n_neut - 1) // 2 + 64)
    err = np.abs(W[rows] - ref)
    say("sn112 rows", len(rows), "max err/bound", np.max(err / bound))
    assert np.all(err <= bound)


def test_sn112_solve_ritz_pairs(sn112):
    """A short FP64 solve of the 112Sn shape; every returned Ritz pair is checked on sampled
    rows with the oracle's H: |(H x)_i - theta x_i| small against |H| |x|."""
    w, g, o = sn112
    say("solve sn112")
    ev, X, info = g.solve(w.nb, w.n_eig, w.l_s, w.l_m, w.tol, "fp64", vectors=True, check_every=-1)
    say("sn112", info.iterations, "iterations, ev", ev[:4])
    assert info.converged
    assert np.all(np.diff(ev) >= -1e-9)
    Xh = X.cpu().numpy()
    rows = np.random.default_rng(6).integers(0, g.dim, 200)
    HX = o.apply_rows(Xh, rows)
    hn = np.abs(ev).max()
    r = np.abs(HX - Xh[rows] * ev[None, :]).max()
    say("sampled residual", r, "scale", hn)
    assert r <= 1e-7 * hn
    # rotational invariance through the same generated-per-element path: J^2 as an interaction
    import paper_1902_02064_amd as trbl
    gj = trbl.Model(w.orbits, w.n_prot, w.n_neut, w.twoM, w.parity)
    gj.set_hamiltonian(jsquared_spe(w.orbits), jsquared_spe(w.orbits), jsquared_tbme(w.orbits))
    j2 = gj.expect(X)
    J = (-1 + np.sqrt(1 + 4 * j2)) / 2
    say("sn112 <J^2>", np.round(j2, 6))
    assert np.abs(J - np.round(J)).max() <= 1e-5


def test_fly_gradient_reports_error():
    """The gradient contracts the stored identical-particle operator: a space on the per-element
    path reports an error instead of a wrong answer."""
    import paper_1902_02064_amd as trbl
    tb = random_tbme(SD_ORBITS, 28)
    g, _ = _forced(SD_ORBITS, 0, 4, 0, tb, [0.0, 0.5, 1.0], 0)
    with pytest.raises(trbl.TrblError):
        g.tbme_grad(np.ones(2), nb=2, tol=1e-8)
