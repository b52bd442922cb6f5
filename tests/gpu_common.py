"""Shared helpers of the GPU tests: build the same workload for the oracle and the library."""
import sys

import numpy as np

import paper_1902_02064_amd as trbl
from oracle.hamiltonian import Model as OracleModel


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair(orbits, z, n, twoM, tbme, spe_p, spe_n, parity=0, oracle=True):
    g = trbl.Model(orbits, z, n, twoM, parity)
    g.set_hamiltonian(spe_p, spe_n, tbme)
    o = OracleModel(orbits, z, n, twoM, tbme, spe_p, spe_n, parity) if oracle else None
    return g, o


def fp64_bound(absH_absV, nnz):
    """Rounding bound for a sum of nnz products in FP64 (gamma_{nnz+1} |H||V|)."""
    u = 2.0 ** -53
    k = nnz + 1
    return k * u / (1 - k * u) * absH_absV + 1e-300


def fp32_bound(absH_absV, nnz):
    """FP32 inputs, coefficients and accumulation against an FP64 product of the rounded inputs."""
    u = 2.0 ** -24
    k = nnz + 2
    return k * u / (1 - k * u) * absH_absV + 1e-30


def term_bound(o, idx, V, fp32=False, extra=0):
    """Rounding bound for rows idx of a per-element H V (a kernel that adds, for each row, the k
    generated terms one product at a time, unmerged) against the oracle.

    With S = sum_t |h_t| |V[j_t]| over the row's generated terms (oracle rows_generated):
      FP64: the kernel's sum of k products errs by at most gamma_k S; its coefficients, built
            by another Clebsch-Gordan code, by gamma_4 S; the oracle's merging of terms into H
            and its product with V by gamma_k S each (merged counts are <= k and |H||V| <= S):
            gamma_{3k+4} S in all.
      FP32: coefficients rounded to FP32 (u32 each) and a k-term FP32 sum, against an FP64
            reference of the same rounded V: gamma32_{k+2} S (the FP64 parts are far below).
    extra: further additions on a term's rounding chain (the pair-block product sums its terms in
    blocks of at most 64 pairs, then the n_prot * n_neut slots: extra = n_prot * n_neut + 64)."""
    ptr, col, val = o.rows_generated(idx)
    k = np.diff(ptr).astype(np.float64)
    absV = np.abs(np.asarray(V, dtype=np.float64))
    S = np.zeros((len(idx), absV.shape[1]))
    for r in range(len(idx)):
        sl = slice(ptr[r], ptr[r + 1])
        S[r] = np.abs(val[sl]) @ absV[col[sl]]
    if fp32:
        u, kk, tiny = 2.0 ** -24, k + 2 + extra, 1e-30
    else:
        u, kk, tiny = 2.0 ** -53, 3 * k + 4 + extra, 1e-300
    return (kk * u / (1 - kk * u))[:, None] * S + tiny
