"""Pins of the oracle's TRBL and gradient (CPU only).

The lowest eigenvalues have a plain definition, so the oracle TRBL is pinned to
dense diagonalisation of the explicit H; the gradient is pinned to central
finite differences and to Euler's identity for a Hamiltonian that is
homogeneous of degree one in its parameters.
"""
import numpy as np
import pytest

from oracle.grad import spe_gradient, tbme_gradient
from oracle.hamiltonian import Model
from oracle.trbl import fix_signs, trbl
from workloads import SD_ORBITS, SD_SPE, WORKLOADS, grad_weights, random_block, random_tbme


@pytest.fixture(scope="module")
def sd22():
    w = WORKLOADS["sd22"]
    m = Model(w.orbits, 2, 2, 0, w.tbme(), w.spe, w.spe)
    H = m.dense()
    e, U = np.linalg.eigh(H)
    return w, m, H, e, U


def test_trbl_matches_dense(sd22):
    w, m, H, e, U = sd22
    V1 = random_block(1000, m.dim, w.nb)
    ev, X, info = trbl(m.apply, m.dim, V1, w.n_eig, w.l_s, w.l_m, w.tol)
    assert info["converged"] and info["restarts"] > 0
    assert np.max(np.abs(ev - e[:w.n_eig]) / np.abs(e[:w.n_eig])) < 1e-12
    # eigenvectors: spectral projector of the 10 lowest (span, not individual vectors)
    P1 = X @ X.T
    P0 = U[:, :w.n_eig] @ U[:, :w.n_eig].T
    assert np.linalg.norm(P1 - P0, 2) < 1e-6
    assert np.max(np.linalg.norm(H @ X - X * ev, axis=0)) <= 1.01 * w.tol * np.max(np.abs(e))


def test_trbl_reduces_to_lanczos(sd22):
    """p = 1 and a large l_m: plain Lanczos with full reorthogonalisation (Alg. 1)."""
    w, m, H, e, U = sd22
    V1 = random_block(7, m.dim, 1)
    ev, X, info = trbl(m.apply, m.dim, V1, 6, 6, 400, 1e-10)
    assert info["restarts"] == 0
    assert np.max(np.abs(ev - e[:6])) < 1e-10


def test_trbl_m1_companion():
    tb = random_tbme(SD_ORBITS, 1)
    m = Model(SD_ORBITS, 2, 2, 2, tb, SD_SPE, SD_SPE)
    e = np.linalg.eigvalsh(m.dense())
    ev, X, info = trbl(m.apply, m.dim, random_block(3, m.dim, 4), 10, 20, 60, 1e-9)
    assert np.max(np.abs(ev - e[:10])) < 1e-10


def test_trbl_breakdown_duplicated_start(sd22):
    """Rank-deficient start block (duplicated columns) and Krylov exhaustion still converge."""
    w, m, H, e, U = sd22
    V = random_block(5, m.dim, 2)
    V1 = np.concatenate([V, V], axis=1)
    ev, X, info = trbl(m.apply, m.dim, V1 + 1e-14, 8, 16, 48, 1e-9)
    assert info["converged"]
    assert np.max(np.abs(ev - e[:8])) < 1e-9
    tiny = Model(((0, 3, 7),), 2, 2, 0, [(0, 0, 0, 0, 0, 2, 0.5), (2, 0, 0, 0, 0, 4, -1.0)], (0.0,), (0.0,))
    et = np.linalg.eigvalsh(tiny.dense())
    evt, _, it = trbl(tiny.apply, tiny.dim, random_block(9, tiny.dim, 2), 3, 4, min(tiny.dim, 12), 1e-10)
    assert np.max(np.abs(evt - et[:3])) < 1e-9


def test_fix_signs():
    X = np.array([[0.1, -0.2], [-0.9, 0.2], [0.3, 0.1]])
    Y = fix_signs(X)
    assert Y[1, 0] > 0 and Y[0, 1] > 0 and Y[1, 1] < 0  # tie |-0.2| = |0.2|: lowest index wins


def test_gradient_fd_and_euler(sd22):
    w, m, H, e, U = sd22
    tb = w.tbme()
    n = w.n_eig
    wt = grad_weights(n)
    g = tbme_gradient(m, tb, U[:, :n], wt)
    gs = spe_gradient(m, U[:, :n], wt)
    v = np.array([x[6] for x in tb])
    spe = np.array(list(w.spe) * 2)
    assert v @ g + spe @ gs == pytest.approx(wt @ e[:n], rel=1e-12)
    h = 1e-5
    for i in (0, 17, 40, 77, 120, 157):
        tp = [list(x) for x in tb]
        tm = [list(x) for x in tb]
        tp[i][6] += h
        tm[i][6] -= h
        ep = np.linalg.eigvalsh(m.with_interaction([tuple(x) for x in tp], w.spe, w.spe).dense())[:n]
        em = np.linalg.eigvalsh(m.with_interaction([tuple(x) for x in tm], w.spe, w.spe).dense())[:n]
        fd = (wt @ ep - wt @ em) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(g[i]), 1e-3 * np.max(np.abs(g)))


def test_trbl_checkpoint_resume(sd22, tmp_path):
    """A run stopped after some restarts and resumed from its checkpoint takes the same iterates."""
    w, o = sd22[0], sd22[1]
    V1 = random_block(1000, o.dim, w.nb)
    ev_ref, _, info_ref = trbl(o.apply, o.dim, V1, w.n_eig, w.l_s, w.l_m, 1e-10)
    assert info_ref["restarts"] >= 2
    trbl(o.apply, o.dim, V1, w.n_eig, w.l_s, w.l_m, 1e-10, max_iter=25, checkpoint=str(tmp_path))
    ev, _, info = trbl(o.apply, o.dim, V1, w.n_eig, w.l_s, w.l_m, 1e-10, checkpoint=str(tmp_path))
    assert info["iterations"] == info_ref["iterations"]
    assert np.array_equal(ev, ev_ref)
