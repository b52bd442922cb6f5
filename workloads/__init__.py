"""Seeded synthetic inputs for the shell-model TRBL eigensolver.

This module only *draws inputs*: orbit sets, the five workload records, random
J-coupled two-body matrix elements and random vector blocks. It contains none
of the method's arithmetic (no Clebsch-Gordan coupling, no basis, no
Hamiltonian action); both the CPU oracle and the GPU library consume what it
produces.

Random numbers come from a counter-based generator: the c-th output of
splitmix64 seeded with ``seed`` (Steele, Lea and Flood, OOPSLA 2014; the
finaliser constants are Vigna's published ones), turned into normals by the
Box-Muller transform. The c-th output can be computed directly, so the GPU
library can implement the same stream independently for its internal start
block.

Two-body matrix elements follow the proton-neutron formalism: channel 0 = pp,
1 = nn, 2 = pn; each independent element V_J(ab,cd) is listed once with the
pair (ab) not after (cd); the Hamiltonian implies the mirror V_J(cd,ab).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Orbits as (n, l, 2j).
SD_ORBITS = ((0, 2, 5), (1, 0, 1), (0, 2, 3))            # 0d5/2 1s1/2 0d3/2
PF_ORBITS = ((0, 3, 7), (1, 1, 3), (0, 3, 5), (1, 1, 1))  # 0f7/2 1p3/2 0f5/2 1p1/2
# 50-82 neutron shell used for the 112Sn dimension: 0g7/2 1d5/2 1d3/2 2s1/2 0h11/2
SNSB_ORBITS = ((0, 4, 7), (1, 2, 5), (1, 2, 3), (2, 0, 1), (0, 5, 11))
# two orbits of Table 1: 0d5/2 1s1/2
TABLE1_ORBITS = ((0, 2, 5), (1, 0, 1))

CH_PP, CH_NN, CH_PN = 0, 1, 2

_MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, counter: int) -> int:
    """The counter-th output (0-based) of splitmix64 started from state ``seed``."""
    z = (seed + (counter + 1) * _GOLDEN) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _splitmix64_np(seed: int, counters: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + (counters.astype(np.uint64) + np.uint64(1)) * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1]: top 53 bits of the splitmix64 output, plus one ulp."""
    bits = _splitmix64_np(seed, counters) >> np.uint64(11)
    return (bits.astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def normal(seed: int, index: np.ndarray) -> np.ndarray:
    """Standard normals; normal k uses uniforms 2k and 2k+1 (Box-Muller, cosine branch)."""
    index = np.asarray(index, dtype=np.uint64)
    u1 = uniform01(seed, index * np.uint64(2))
    u2 = uniform01(seed, index * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def normal_scalar(seed: int, k: int) -> float:
    """normal(seed, k) evaluated one draw at a time with the C library's log and cos (numpy's
    vectorised log and cos may differ from them by one unit in the last place)."""
    u1 = ((splitmix64(seed, 2 * k) >> 11) + 1.0) * (1.0 / 9007199254740992.0)
    u2 = ((splitmix64(seed, 2 * k + 1) >> 11) + 1.0) * (1.0 / 9007199254740992.0)
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def random_block(seed: int, rows: int, cols: int) -> np.ndarray:
    """A rows x cols row-major block of standard normals; entry (i, c) is normal #(i*cols+c)."""
    idx = np.arange(rows * cols, dtype=np.uint64)
    return normal(seed, idx).reshape(rows, cols)


def _pair_list(orbits, channel):
    """Canonical orbit pairs of one channel: (a<=b) for pp/nn, every (a,b) for pn (a proton, b neutron)."""
    n = len(orbits)
    if channel == CH_PN:
        return [(a, b) for a in range(n) for b in range(n)]
    return [(a, b) for a in range(n) for b in range(a, n)]


def _pair_allows(orbits, channel, a, b, twoJ):
    ja, jb = orbits[a][2], orbits[b][2]
    if twoJ < abs(ja - jb) or twoJ > ja + jb:
        return False
    if channel != CH_PN and a == b and (twoJ // 2) % 2 == 1:
        return False  # two identical nucleons in one j-shell couple to even J only
    return True


def tbme_blocks(orbits):
    """(channel, 2J, parity, [pairs]) for every non-empty J-pi block, in drawing order."""
    jmax2 = 2 * max(o[2] for o in orbits)
    out = []
    for ch in (CH_PP, CH_NN, CH_PN):
        pairs = _pair_list(orbits, ch)
        for twoJ in range(0, jmax2 + 1, 2):
            for par in (+1, -1):
                blk = [(a, b) for (a, b) in pairs
                       if (-1) ** (orbits[a][1] + orbits[b][1]) == par and _pair_allows(orbits, ch, a, b, twoJ)]
                if blk:
                    out.append((ch, twoJ, par, blk))
    return out


def random_tbme(orbits, seed: int, sigma: float = 1.0):
    """i.i.d. Gaussian J-coupled elements, one per independent (ab)<=(cd) in every block.

    Returns a list of (channel, a, b, c, d, 2J, v) drawn in block order
    (channel, 2J, parity +/-) and, inside a block, over pairs i<=j of the
    block's pair list; draw number k uses normal_scalar(seed, k).
    """
    out = []
    k = 0
    for ch, twoJ, _par, blk in tbme_blocks(orbits):
        for i in range(len(blk)):
            for j in range(i, len(blk)):
                v = sigma * normal_scalar(seed, k)
                k += 1
                (a, b), (c, d) = blk[i], blk[j]
                out.append((ch, a, b, c, d, twoJ, v))
    return out


def pairing_tbme(orbits, strength: float):
    """Pure J=0 pairing in each identical channel for a single orbit: V_0(jj,jj) = -G*Omega."""
    assert len(orbits) == 1
    omega = (orbits[0][2] + 1) / 2.0
    return [(CH_PP, 0, 0, 0, 0, 0, -strength * omega), (CH_NN, 0, 0, 0, 0, 0, -strength * omega)]


def jsquared_tbme(orbits):
    """Two-body part of total J^2 written as a J-coupled interaction (diagonal in the pair basis).

    2 j1.j2 on a pair coupled to J equals J(J+1) - ja(ja+1) - jb(jb+1); the one-body
    part j(j+1) goes into the single-particle energies (see ``jsquared_spe``).
    """
    out = []
    for ch, twoJ, _par, blk in tbme_blocks(orbits):
        J = twoJ / 2.0
        for (a, b) in blk:
            ja, jb = orbits[a][2] / 2.0, orbits[b][2] / 2.0
            out.append((ch, a, b, a, b, twoJ, J * (J + 1) - ja * (ja + 1) - jb * (jb + 1)))
    return out


def jsquared_spe(orbits):
    return [o[2] / 2.0 * (o[2] / 2.0 + 1) for o in orbits]


@dataclass
class Workload:
    """One synthetic workload: model space, Hamiltonian recipe and solver settings."""
    name: str
    orbits: tuple
    n_prot: int
    n_neut: int
    twoM: int
    spe: tuple
    nb: int
    n_eig: int
    l_s: int
    l_m: int
    tol: float
    precision: str            # "fp64" or "mixed"
    seed: int = 1             # interaction seed
    parity: int = 0           # 0 = both, +1, -1
    sigma: float = 1.0
    extra: dict = field(default_factory=dict)

    def tbme(self):
        return random_tbme(self.orbits, self.seed, self.sigma)


SD_SPE = (-3.9, -3.2, 2.1)
PF_SPE = (0.0, 2.0, 4.0, 6.0)
SNSB_SPE = (0.0, 0.2, 1.5, 1.8, 2.4)

WORKLOADS = {
    # sd shell, 2+2 nucleons (20Ne shape, D = 640)
    "sd22": Workload("sd22", SD_ORBITS, 2, 2, 0, SD_SPE, nb=4, n_eig=10, l_s=20, l_m=60,
                     tol=1e-8, precision="fp64"),
    # pf shell, 4+4 nucleons (48Cr shape, D = 1,963,461)
    "pf44": Workload("pf44", PF_ORBITS, 4, 4, 0, PF_SPE, nb=16, n_eig=100, l_s=200, l_m=400,
                     tol=1e-8, precision="fp64"),
    # mixed-precision form of sd22
    "sd22_mixed": Workload("sd22_mixed", SD_ORBITS, 2, 2, 0, SD_SPE, nb=4, n_eig=10, l_s=20, l_m=60,
                           tol=1e-8, precision="mixed"),
    # sd shell, 6+6 nucleons (28Si shape, D = 93,710): gradient workload
    "sd66": Workload("sd66", SD_ORBITS, 6, 6, 0, SD_SPE, nb=8, n_eig=20, l_s=40, l_m=120,
                     tol=1e-10, precision="fp64", extra={"grad_weight_seed": 7, "fd_step": 1e-5}),
    # 50-82 neutron shell, 12 neutrons, positive parity (112Sn shape, D = 6,210,638): one
    # species only, the identical-particle part generated per element
    "sn112": Workload("sn112", SNSB_ORBITS, 0, 12, 0, SNSB_SPE, nb=8, n_eig=10, l_s=40, l_m=120,
                      tol=1e-8, precision="fp64", parity=1),
    # pf shell, 6+6 nucleons (D = 109,954,620), mixed precision
    "pf66": Workload("pf66", PF_ORBITS, 6, 6, 0, PF_SPE, nb=32, n_eig=200, l_s=400, l_m=560,
                     tol=1e-5, precision="mixed"),
}


def grad_weights(n: int, seed: int = 7) -> np.ndarray:
    """Weights w_k ~ U[0,1) of the eigenvalue sum whose gradient is taken."""
    return uniform01(seed, np.arange(n, dtype=np.uint64)) - 2.0 ** -53
