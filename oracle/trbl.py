"""Thick-restart block Lanczos for the oracle (test infrastructure).

Takes the steps of Alg. 4 (Sec. 3.4) in the paper's order and notation:
  W := H V_k ;  alpha_k := V_k^T W  (symmetrised) ; T block (k,k) := alpha_k ;
  orthogonalise W against v_1 .. v_{k_x + p k}  (classical Gram-Schmidt, twice) ;
  V_{k+1} beta_k := QR(W)  (diag(beta_k) >= 0) ; T blocks (k+1,k), (k,k+1) := beta_k, beta_k^T ;
  diagonalise T^(k) and test convergence ;
and the restart equations of Sec. 3.4 when the next block would not fit in l_m:
  v_k := sum_j v_j U_jk (k <= l_s),  V_1 := V_{k_m+1},
  r := beta_{k_m} U[last block rows, 1:l_s],  T := [E r^T; r .],  k_x := l_s.

Readings (listed in the design doc):
  * convergence: residual norm rho_i = || beta_k U[last block rows, i] || <= tol * ||H||_est
    for the n_eig lowest Ritz pairs, with ||H||_est the largest |Ritz value| seen;
    the test runs after the QR step because rho_i needs beta_k.
  * l_m counts every stored vector including V_{k+1}; restart when V_{k+2} would not fit.
  * breakdown: a column of V_{k+1} whose R diagonal is below 1e-10 of the largest is
    replaced by a random vector orthogonal to everything stored, with a zero beta row.
"""
from __future__ import annotations

import numpy as np


def _qr_pos(W):
    Qm, R = np.linalg.qr(W)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Qm * s, R * s[:, None]


def fix_signs(X):
    """Eigenvector sign convention: largest-magnitude component positive (lowest index on ties)."""
    X = np.array(X, copy=True)
    for j in range(X.shape[1]):
        i = int(np.argmax(np.abs(X[:, j])))
        if X[i, j] < 0:
            X[:, j] = -X[:, j]
    return X


def _save_state(path, Q, T, kx, k, hnorm, it, info, rng):
    """Resumable state after a restart (long runs only; no arithmetic here)."""
    import json
    import os
    np.save(os.path.join(path, "Q.npy.tmp.npy"), Q)
    np.save(os.path.join(path, "T.npy.tmp.npy"), T)
    os.replace(os.path.join(path, "Q.npy.tmp.npy"), os.path.join(path, "Q.npy"))
    os.replace(os.path.join(path, "T.npy.tmp.npy"), os.path.join(path, "T.npy"))
    meta = {"kx": kx, "k": k, "hnorm": hnorm, "it": it, "info": info, "rng": rng.bit_generator.state}
    with open(os.path.join(path, "meta.json.tmp"), "w") as f:
        json.dump(meta, f)
    os.replace(os.path.join(path, "meta.json.tmp"), os.path.join(path, "meta.json"))


def trbl(apply, dim, V1, n_eig, l_s, l_m, tol, max_iter=10000, seed=12345, history=None, checkpoint=None):
    """Lowest ``n_eig`` eigenpairs of the symmetric operator ``apply`` (D x p -> D x p).

    V1: D x p start block (orthonormalised here). Returns (evals, evecs, info).
    checkpoint: optional directory; the state is saved after every restart and a run
    started with a saved state there continues from it (same iterates).
    """
    import json
    import os
    p = V1.shape[1]
    if not (n_eig <= l_s and l_s + 2 * p <= l_m and l_m <= dim):
        raise ValueError("need n_eig <= l_s, l_s + 2p <= l_m <= D")
    rng = np.random.default_rng(seed)
    it0 = 1
    if checkpoint and os.path.exists(os.path.join(checkpoint, "meta.json")):
        with open(os.path.join(checkpoint, "meta.json")) as f:
            meta = json.load(f)
        Q = np.load(os.path.join(checkpoint, "Q.npy"))
        T = np.load(os.path.join(checkpoint, "T.npy"))
        kx, k, hnorm, info = meta["kx"], meta["k"], meta["hnorm"], meta["info"]
        rng.bit_generator.state = meta["rng"]
        it0 = meta["it"] + 1
    else:
        Q = np.zeros((dim, l_m))
        T = np.zeros((l_m, l_m))
        Q[:, :p], _ = _qr_pos(np.asarray(V1, dtype=np.float64))
        kx, k = 0, 0
        hnorm = 0.0
        info = {"iterations": 0, "restarts": 0, "converged": False}
    for it in range(it0, max_iter + 1):
        k += 1
        c0 = kx + (k - 1) * p
        m = c0 + p
        Vk = Q[:, c0:m]
        W = apply(Vk)
        alpha = Vk.T @ W
        alpha = 0.5 * (alpha + alpha.T)
        T[c0:m, c0:m] = alpha
        for _ in range(2):
            W -= Q[:, :m] @ (Q[:, :m].T @ W)
        Vn, beta = _qr_pos(W)
        dmax = np.max(np.abs(np.diag(beta))) if p else 0.0
        for j in range(p):
            if abs(beta[j, j]) <= 1e-10 * max(dmax, 1e-300):
                x = rng.standard_normal(dim)
                for _ in range(2):
                    x -= Q[:, :m] @ (Q[:, :m].T @ x)
                    others = np.delete(Vn, j, axis=1)
                    x -= others @ (others.T @ x)
                Vn[:, j] = x / np.linalg.norm(x)
                beta[j, :] = 0.0
        theta, U = np.linalg.eigh(T[:m, :m])
        hnorm = max(hnorm, float(np.max(np.abs(theta))))
        nchk = min(n_eig, m)
        rho = np.linalg.norm(beta @ U[m - p:m, :nchk], axis=0)
        info["iterations"] = it
        if history is not None:
            history.append((it, theta[:nchk].copy(), rho.copy()))
        if nchk == n_eig and np.all(rho <= tol * hnorm):
            info["converged"] = True
            info["resid"] = rho
            X = Q[:, :m] @ U[:, :n_eig]
            return theta[:n_eig], X, info
        Q[:, m:m + p] = Vn
        T[m:m + p, c0:m] = beta
        T[c0:m, m:m + p] = beta.T
        if m + 2 * p > l_m:
            Y = Q[:, :m] @ U[:, :l_s]
            r = beta @ U[m - p:m, :l_s]
            Q[:, :l_s] = Y
            Q[:, l_s:l_s + p] = Vn
            Q[:, l_s + p:] = 0.0
            T[:] = 0.0
            T[np.arange(l_s), np.arange(l_s)] = theta[:l_s]
            T[l_s:l_s + p, :l_s] = r
            T[:l_s, l_s:l_s + p] = r.T
            kx, k = l_s, 0
            info["restarts"] += 1
            if checkpoint:
                _save_state(checkpoint, Q, T, kx, k, hnorm, it, info, rng)
    info["resid"] = rho
    X = Q[:, :m] @ U[:, :n_eig]
    return theta[:n_eig], X, info
