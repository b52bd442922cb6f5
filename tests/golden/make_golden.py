"""Write the stored expected values of the full-size workloads, calling only the oracle.

  python tests/golden/make_golden.py [sd22] [sd66] [pf44]
  python tests/golden/make_golden.py --nnz-only sn112

Outputs (text, one value per line, header comments):
  <name>_nnz.txt     structural non-zero count of H (merged matrix elements)
  <name>_eigs.txt    lowest eigenvalues from the oracle TRBL (Alg. 4) with residual norms
  sd66_grad.txt      d(sum w_k E_k)/dV for every listed element, then the 6 orbit energies
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.grad import spe_gradient, tbme_gradient  # noqa: E402
from oracle.hamiltonian import model_from_workload  # noqa: E402
from oracle.trbl import trbl  # noqa: E402
from workloads import WORKLOADS, grad_weights, random_block  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def write(name, header, values, fmt="%.17g"):
    with open(os.path.join(HERE, name), "w") as f:
        for h in header:
            f.write("# " + h + "\n")
        for v in np.atleast_1d(values):
            f.write((fmt % v) + "\n")


def run(wname, nnz_only=False):
    w = WORKLOADS[wname]
    t0 = time.time()
    m = model_from_workload(w)
    nnz = int(m.row_nnz().sum())
    write(f"{wname}_nnz.txt", [f"{wname}: structural non-zeros of H (oracle rows, merged)", f"D = {m.dim}"],
          [nnz], "%d")
    print(wname, "D", m.dim, "nnz", nnz, flush=True)
    if nnz_only:
        return
    V1 = random_block(1000, m.dim, w.nb)
    tol = min(w.tol, 1e-10)
    hist = []
    ckpt = os.environ.get("TRBL_GOLDEN_CKPT")  # optional directory: resumable long runs
    if ckpt:
        ckpt = os.path.join(ckpt, wname)
        os.makedirs(ckpt, exist_ok=True)
    ev, X, info = trbl(m.apply, m.dim, V1, w.n_eig, w.l_s, w.l_m, tol, history=hist, checkpoint=ckpt)
    print(wname, "iterations", info["iterations"], "restarts", info["restarts"], "converged", info["converged"],
          "%.0f s" % (time.time() - t0), flush=True)
    write(f"{wname}_eigs.txt",
          [f"{wname}: {w.n_eig} lowest eigenvalues, oracle TRBL nb={w.nb} l_s={w.l_s} l_m={w.l_m} tol={tol}",
           f"interaction seed {w.seed}, start block workloads.random_block(1000, D, nb)",
           f"iterations {info['iterations']} restarts {info['restarts']} converged {info['converged']}",
           f"max residual {np.max(info['resid']):.3e}"], ev)
    if wname == "sd66":
        wt = grad_weights(w.n_eig, w.extra["grad_weight_seed"])
        g = tbme_gradient(m, w.tbme(), X, wt)
        gs = spe_gradient(m, X, wt)
        write("sd66_grad.txt",
              ["sd66: d(sum_k w_k E_k)/dV_t for the listed elements (workloads.random_tbme order),",
               "then d/de_a for proton orbits then neutron orbits; w = workloads.grad_weights(20, 7)"],
              np.concatenate([g, gs]))


if __name__ == "__main__":
    args = sys.argv[1:]
    only = "--nnz-only" in args
    names = [x for x in args if x != "--nnz-only"]
    for name in (names or ["sd22", "sd66", "pf44"]):
        run(name, only)
