"""Full-size solves (GPU): sd66 and pf44 against the oracle TRBL's stored eigenvalues (sd66 also
with restarts that keep more than 208 vectors), and the mixed-precision pf44 solve against the
FP64 one."""
import os

import numpy as np
import pytest

from gpu_common import pair, say
from workloads import WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_eigs.txt")
    if not os.path.exists(path):
        pytest.skip(f"{name}_eigs.txt not generated (oracle TRBL run of several hours)")
    return np.array([float(x) for x in open(path) if x.strip() and not x.startswith("#")])


def _model(w):
    g, _ = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, w.tbme(), w.spe, w.spe, w.parity, oracle=False)
    return g


@pytest.fixture(scope="module")
def pf44():
    w = WORKLOADS["pf44"]
    g = _model(w)
    say("solve pf44 fp64")
    ev, X, info = g.solve(w.nb, w.n_eig, w.l_s, w.l_m, w.tol, "fp64", check_every=-1)
    say("pf44 fp64", info.iterations, "iterations", info.t_total, "s")
    return w, g, ev, info


def test_sd66_matches_oracle_trbl():
    """sd shell 6+6 (D = 93,710), 20 lowest at tol 1e-10: relative error <= 1e-8 per eigenvalue."""
    ref = _golden("sd66")
    w = WORKLOADS["sd66"]
    g = _model(w)
    ev, _, info = g.solve(w.nb, w.n_eig, w.l_s, w.l_m, w.tol, "fp64", check_every=-1)
    assert info.converged
    rel = np.abs(ev - ref) / np.abs(ref)
    say("sd66 max rel err", rel.max(), "iterations", info.iterations)
    assert rel.max() <= 1e-8


@pytest.mark.parametrize("l_s,l_m", [(216, 232), (220, 236)])
def test_sd66_restart_keeps_more_than_208_vectors(l_s, l_m):
    """Thick restarts that keep more than 208 vectors: the restart product Q U is then computed
    in place by row chunks through a work buffer. With (220, 236) and nb = 8 the block moved to
    column l_s at the first restart (from column 224) overlaps its destination. FP64 against the
    oracle TRBL's eigenvalues (<= 1e-8 relative), mixed precision <= 1e-6."""
    ref = _golden("sd66")
    w = WORKLOADS["sd66"]
    g = _model(w)
    ev, _, info = g.solve(w.nb, w.n_eig, l_s, l_m, w.tol, "fp64", check_every=-1)
    rel = np.abs(ev - ref) / np.abs(ref)
    say("sd66 l_s", l_s, "l_m", l_m, "fp64", info.iterations, "iterations", info.restarts, "restarts, max rel err",
        rel.max())
    assert info.converged and info.restarts >= 1
    assert rel.max() <= 1e-8
    evm, _, im = g.solve(w.nb, w.n_eig, l_s, l_m, w.tol, "mixed", check_every=-1)
    relm = np.abs(evm - ref) / np.abs(ref)
    say("mixed", im.iterations, "iterations", im.restarts, "restarts, max rel err", relm.max())
    assert im.converged and im.restarts >= 1
    assert relm.max() <= 1e-6


def test_pf44_fp64_matches_oracle_trbl(pf44):
    """pf shell 4+4 (D = 1,963,461), 100 lowest: relative error <= 1e-8 per eigenvalue."""
    w, g, ev, info = pf44
    assert info.converged
    ref = _golden("pf44")
    rel = np.abs(ev - ref) / np.abs(ref)
    say("pf44 max rel err", rel.max())
    assert rel.max() <= 1e-8


def test_pf44_residuals_and_ordering(pf44):
    """Properties at full size that need no stored values: ascending, converged residuals."""
    w, g, ev, info = pf44
    assert info.converged and np.all(np.diff(ev) >= -1e-12 * np.abs(ev).max())
    assert info.resid.max() <= w.tol * np.abs(ev).max() * 10


def test_pf44_mixed_vs_fp64(pf44):
    """Mixed precision (FP32 vectors and H.V, FP64 refinement): <= 1e-6 relative per eigenvalue."""
    w, g, ev, info = pf44
    evm, _, im = g.solve(w.nb, w.n_eig, w.l_s, w.l_m, w.tol, "mixed", check_every=-1)
    assert im.converged
    rel = np.abs(evm - ev) / np.abs(ev)
    say("pf44 mixed max rel err", rel.max(), "median", np.median(rel), im.iterations, "iterations")
    assert rel.max() <= 1e-6


def test_pf66_mixed_restart_and_refinement():
    """pf shell 6+6 (D = 109,954,620), mixed precision, nb = 32, 200 wanted, l_s = 384, l_m = 448
    (the FP32 basis takes 197 GB). A full solve is beyond a test's time. 14 iterations from one start include the first restart (iteration 13: the product Q U
    keeps 384 vectors and goes through the work buffer in chunks of 16.9 million rows, whose
    copies exceed 2^32 elements). The FP64 Rayleigh-Ritz refinement of the 200 Ritz vectors then
    recomputes H in FP64 from the restarted basis: its values agree with the unrefined Ritz values
    only if the restart wrote every row."""
    w = WORKLOADS["pf66"]
    g = _model(w)
    say("pf66 mixed, 14 iterations without and with refinement")
    e0, _, i0 = g.solve(32, 200, 384, 448, 1e-5, "mixed", max_iter=14, refine=False, check_every=1)
    e1, _, i1 = g.solve(32, 200, 384, 448, 1e-5, "mixed", max_iter=14, refine=True, check_every=1)
    d = np.abs(e1 - e0).max()
    say("pf66 lowest Ritz value", e0[0], "refined", e1[0], "max |refined - Ritz|", d, "t", i0.t_total, i1.t_total)
    assert not i0.converged and i0.iterations == 14 and i0.restarts == 1 and i1.restarts == 1
    assert np.all(np.isfinite(e0)) and np.all(np.isfinite(e1))
    # Each stored FP32 vector (rounded to within 2^-24 relative) perturbs the projected matrix by
    # at most 2^-24 |H| in norm, the basis holds at most l_m of them, and by Weyl's theorem an
    # eigenvalue moves by at most the norm of the perturbation: |refined - Ritz| <= l_m 2^-24 |H|.
    assert d <= 448 * 2.0 ** -24 * np.abs(e0).max()


def test_pf66_fp64_vs_mixed_same_start():
    """pf shell 6+6 has no CPU oracle run; its precision parity is GPU FP64 against GPU mixed.
    nb = 32, 8 wanted, l_s = 64, l_m = 128 (the FP64 basis then fits: 113 GB), 12 iterations
    (9 restarts) from the same start block: the 8 lowest values, mixed with its FP64 refinement,
    agree with FP64 to <= 1e-6 relative."""
    w = WORKLOADS["pf66"]
    g = _model(w)
    say("pf66 fp64 and mixed, 12 iterations")
    e64, _, i64 = g.solve(32, 8, 64, 128, 1e-5, "fp64", max_iter=12, check_every=1, seed=1000)
    e32, _, i32 = g.solve(32, 8, 64, 128, 1e-5, "mixed", max_iter=12, check_every=1, seed=1000)
    rel = np.abs(e32 - e64) / np.abs(e64)
    say("pf66 fp64", e64[:4], "mixed max rel", rel.max(), "t", i64.t_total, i32.t_total)
    assert i64.iterations == i32.iterations == 12 and i64.restarts == i32.restarts >= 1
    assert rel.max() <= 1e-6


def test_pf44_ritz_vectors_have_integer_j():
    """pf44 at full size: <J^2> of the 100 Ritz vectors is J(J+1) with integer J."""
    from workloads import jsquared_spe, jsquared_tbme
    w = WORKLOADS["pf44"]
    g = _model(w)
    ev, X, info = g.solve(w.nb, w.n_eig, w.l_s, w.l_m, w.tol, "fp64", vectors=True, check_every=-1)
    assert info.converged
    gj, _ = pair(w.orbits, w.n_prot, w.n_neut, w.twoM, jsquared_tbme(w.orbits), jsquared_spe(w.orbits),
                 jsquared_spe(w.orbits), oracle=False)
    j2 = gj.expect(X)
    J = (-1 + np.sqrt(1 + 4 * j2)) / 2
    say("pf44 J values", np.round(J, 4)[:20], "max dev", np.abs(J - np.round(J)).max())
    assert np.abs(J - np.round(J)).max() <= 1e-4


@pytest.mark.parametrize("nb", [32, 64])
def test_sd66_wide_block_large_basis(nb):
    """Blocks of 32 and 64 vectors with the basis at the eigensolver's limit (l_m - nb = 640):
    the projected updates there exceed the LDS tile of one pass over the basis and run in
    chunks of its columns. FP64 against the oracle TRBL's eigenvalues (<= 1e-8 relative)."""
    ref = _golden("sd66")
    w = WORKLOADS["sd66"]
    g = _model(w)
    ev, _, info = g.solve(nb, w.n_eig, 64, 640 + nb, w.tol, "fp64", check_every=-1)
    rel = np.abs(ev - ref) / np.abs(ref)
    say("sd66 nb", nb, "iterations", info.iterations, "restarts", info.restarts, "max rel err", rel.max())
    assert info.converged
    assert rel.max() <= 1e-8
