"""Gradient of a weighted eigenvalue sum for the oracle (test infrastructure).

H is linear in the single-particle energies and the J-coupled elements, so by
Hellmann-Feynman  d(sum_k w_k E_k)/d theta = sum_k w_k psi_k^T (dH/d theta) psi_k,
where dH/d theta is the Hamiltonian built from that one parameter set to 1 and
every other parameter set to 0. For an element listed once with (ab) != (cd)
this includes its implied mirror V_J(cd,ab), i.e. both entries of H.
"""
from __future__ import annotations

import numpy as np


def tbme_gradient(model, tbme, evecs, weights):
    """d(sum w_k E_k)/dV for every listed element; evecs D x n (orthonormal columns)."""
    X = np.ascontiguousarray(evecs, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    zero = [0.0] * len(model.orbits)
    g = np.zeros(len(tbme))
    for t, el in enumerate(tbme):
        unit = [tuple(el[:6]) + (1.0,)]
        Ht = model.with_interaction(unit, zero, zero)
        HX = Ht.apply(X)
        g[t] = float(np.sum(w * np.einsum("ik,ik->k", X, HX)))
    return g


def spe_gradient(model, evecs, weights):
    """d(sum w_k E_k)/d e_a for proton orbits then neutron orbits."""
    X = np.ascontiguousarray(evecs, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    norb = len(model.orbits)
    out = []
    for species in (0, 1):
        for a in range(norb):
            ep = [0.0] * norb
            en = [0.0] * norb
            (ep if species == 0 else en)[a] = 1.0
            Ht = model.with_interaction([], ep, en)
            HX = Ht.apply(X)
            out.append(float(np.sum(w * np.einsum("ik,ik->k", X, HX))))
    return np.array(out)
