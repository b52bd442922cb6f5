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
