#!/usr/bin/env python3
"""Benchmark of the TRBL shell-model eigensolver on one MI355X.

A step is one complete thick-restart block Lanczos solve (Alg. 4 with the
restart of Sec. 3.4): random start block -> block H.V, projections, block
Gram-Schmidt, Cholesky QR, projected eigenproblem and restarts, until the 100
lowest eigenpairs of the pf-shell 4+4 workload (D = 1,963,461; the 48Cr shape
of Sec. 4.1) have converged. Inputs (basis tables, interaction, start block)
are resident in HBM before the timed region.

Printed: one JSON line. value = seconds per solve in FP64 (lower is better);
the mixed-precision solve, the H.V kernel's own timing, the roofline of the
dominant kernel and the CPU oracle baseline are extra fields.

Other modes (one JSON line each, not the benchmark line): --workload sn112 runs the
same benchmark on the single-species 112Sn shape of Sec. 4.2 (--workload pf66 --hv-only times
the pf 6+6 block H.V); --sweep measures the
block-size trade-off of Sec. 4.2; --truncated-start compares start vectors from a
particle-hole truncated space with a random start block (Sec. 4.2); --hv-only times
the block H.V alone (for profilers).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s to N converged eigenpairs + block H·V HBM GB/s, FP64 vs mixed FP32"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="pf44")
    p.add_argument("--hv-launches", type=int, default=20)
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--hv-only", action="store_true", help="only the H.V timing loop (for profilers)")
    p.add_argument("--calib-copy", action="store_true",
                   help="with --hv-only: also run a plain 1 GiB device copy (counter calibration)")
    p.add_argument("--check-every", type=int, default=-1, help="convergence-test period; -1 = adaptive")
    p.add_argument("--truncated-start", action="store_true",
                   help="start vectors from a truncated subspace (Sec. 4.2) instead of the benchmark: nb vectors "
                        "of the space with at most --trunc-max nucleons in --trunc-orbits start the full solve, "
                        "against a random start of the same block size")
    p.add_argument("--trunc-orbits", default="2,3,4", help="orbit indices of the truncation (sn112: above N = 64)")
    p.add_argument("--trunc-max", type=int, default=4)
    p.add_argument("--trunc-nb", type=int, default=16)
    p.add_argument("--trunc-spe", default="",
                   help="comma-separated single-particle energies for the truncated-start run (default: the "
                        "workload's); e.g. a wide gap above the truncation orbits")
    p.add_argument("--sweep", action="store_true",
                   help="block-size sweep instead of the benchmark: H.V time and TRBL solve for the 32 lowest, "
                        "nb = 1..32, l_s = 40, l_m = max(200, 40 + 10 nb)")
    return p.parse_args()


def stored_nnz(name):
    path = os.path.join(ROOT, "tests", "golden", f"{name}_nnz.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            return int(line)
    return None


HV_SOURCES = ("hv.hip", "hv_kern.h", "hv_f64.hip", "hv_f32.hip")


def hv_source_digest():
    """Digest of the block H.V sources (a stored counter summary is valid only for these)."""
    import hashlib
    h = hashlib.sha256()
    for f in HV_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1902_02064_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(name):
    """Measured HBM bytes per H.V launch from the committed counter summary, if it matches the source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hv_{name}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    digest = hv_source_digest()
    if kv.get("hv_source_sha256_16") != digest:
        return None
    return float(kv["fp64_bytes_per_launch"])


def hv_timing(model, nb, dtype, launches, torch):
    """Average duration of one block H.V launch, HIP events on the launching stream."""
    s = torch.cuda.current_stream()
    V = torch.randn(model.dim, nb, dtype=dtype, device="cuda")
    W = torch.empty_like(V)
    for _ in range(3):
        model.apply(V, W)
    s.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(launches):
        model.apply(V, W)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / launches


def cpu_baseline(w, iterations, seconds_target=12.0):
    """The oracle's block H.V on a bounded sample of rows, scaled to one solve's H.V work."""
    import numpy as np

    from oracle.hamiltonian import model_from_workload, threads
    from workloads import random_block
    m = model_from_workload(w)
    V = random_block(2000, m.dim, w.nb)
    rng = np.random.default_rng(0)
    n = 2000
    t0 = time.perf_counter()
    m.apply_rows(V, rng.choice(m.dim, n, replace=False))
    t1 = time.perf_counter() - t0
    n2 = int(min(m.dim, max(n, n * seconds_target / max(t1, 1e-6))))
    idx = rng.choice(m.dim, n2, replace=False)
    t0 = time.perf_counter()
    m.apply_rows(V, idx)
    t2 = time.perf_counter() - t0
    per_hv = t2 * m.dim / n2
    return {
        "value": per_hv * iterations,
        "unit": "s",
        "cores": threads(),
        "kind": "oracle",
        "sample": (f"oracle block H.V (nb={w.nb}) on {n2} random rows of {m.dim} ({t2:.1f} s), scaled to the "
                   f"full matrix ({per_hv:.1f} s per H.V) and to the {iterations} block iterations of the GPU "
                   f"solve; H.V only, so a lower bound on the oracle's time to {w.n_eig} eigenpairs"),
    }


def sweep(model, w, torch, np):
    """Trade-off of Sec. 4.2: block H.V time against nb (a line whose intercept is the fixed
    generation cost) and iterations / time to the 32 lowest eigenpairs against nb."""
    rows = []
    for nb in (1, 2, 4, 8, 16, 32):
        t_hv = hv_timing(model, nb, torch.float64, 10, torch)
        lm = max(200, 40 + 10 * nb)  # room for ten blocks between restarts
        ev, _, info = model.solve(nb, 32, 40, lm, 1e-8, "fp64", max_iter=20000, seed=1000, check_every=-1)
        r = {"nb": nb, "l_m": lm, "hv_ms": t_hv * 1e3, "hv_ms_per_vector": t_hv * 1e3 / nb, "iterations": info.iterations,
             "restarts": info.restarts, "converged": info.converged, "t_total_s": info.t_total, "t_hv_s": info.t_hv,
             "t_orth_s": info.t_orth, "t_qr_s": info.t_qr, "t_eig_s": info.t_eig, "t_restart_s": info.t_restart,
             "e0": float(ev[0]), "e31": float(ev[31])}
        print("# " + json.dumps(r), file=sys.stderr, flush=True)
        rows.append(r)
    x = np.array([r["nb"] for r in rows], dtype=float)
    y = np.array([r["hv_ms"] for r in rows])
    slope, icpt = np.polyfit(x, y, 1)
    print(json.dumps({"sweep": rows, "hv_fit_ms": {"intercept": icpt, "slope_per_vector": slope},
                      "workload": w.name, "n_eig": 32, "l_s": 40, "l_m": "max(200, 40 + 10 nb)", "tol": 1e-8}))


def truncated_start(model, w, a, torch):
    """Sec. 4.2: nb start vectors from the truncated space (at most trunc_max nucleons in the
    given orbits) against a random start block, for the workload's lowest n_eig."""
    nb = a.trunc_nb
    orbs = [int(x) for x in a.trunc_orbits.split(",") if x != ""]
    spe = list(w.spe)
    if a.trunc_spe:
        spe = [float(x) for x in a.trunc_spe.split(",")]
        model.set_hamiltonian(spe, spe, w.tbme())
    ls, lm = 4 * nb, 16 * nb
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mask = model.occupation_mask(orbs, a.trunc_max)
    kept = int(mask.sum().item())
    print(f"# truncated space: {kept} of {model.dim} states; solving for {nb} vectors", file=sys.stderr, flush=True)
    et, Xt, it_t = model.solve(nb, nb, ls, lm, 1e-4, "fp64", max_iter=2000, vectors=True, mask=mask, check_every=-1)
    print(f"# truncated solve: {it_t.iterations} iterations, converged {it_t.converged}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_trunc = time.perf_counter() - t0
    del mask
    runs = {}
    for name, v0 in (("truncated_start", Xt.contiguous()), ("random_start", None)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        print(f"# full solve, {name}", file=sys.stderr, flush=True)
        ev, _, info = model.solve(nb, w.n_eig, ls, lm, w.tol, "fp64", max_iter=2000, v0=v0, check_every=-1)
        torch.cuda.synchronize()
        runs[name] = {"s": time.perf_counter() - t0, "iterations": info.iterations, "restarts": info.restarts,
                      "converged": info.converged, "e0": float(ev[0]), "e_last": float(ev[-1])}
        print("# " + name + " " + json.dumps(runs[name]), file=sys.stderr, flush=True)
    print(json.dumps({"truncated_start": {
        "workload": w.name, "D": model.dim, "spe": spe,
        "truncation": {"orbits": orbs, "max_nucleons": a.trunc_max, "kept": kept},
        "nb": nb, "n_eig": w.n_eig, "l_s": ls, "l_m": lm, "tol": w.tol,
        "truncated_solve": {"s": t_trunc, "iterations": it_t.iterations, "converged": it_t.converged, "tol": 1e-4,
                            "e0": float(et[0]), "e_last": float(et[-1])},
        "full": runs,
        "speedup_incl_truncated": runs["random_start"]["s"] / (runs["truncated_start"]["s"] + t_trunc)}}))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU path is a design note, "
              "not part of this build", file=sys.stderr)
        sys.exit(2)
    from workloads import WORKLOADS

    w = WORKLOADS[a.workload]
    if w.name == "pf66" and not a.hv_only:
        print("pf66: only --hv-only here (its FP64 basis does not fit one GPU and a mixed solve to 200 "
              "eigenpairs takes about an hour; the pf66 tests cover restarts and FP64 against mixed)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1902_02064_amd as trbl
    torch.cuda.init()
    t_setup = time.perf_counter()
    model = trbl.Model(w.orbits, w.n_prot, w.n_neut, w.twoM, w.parity)
    model.set_hamiltonian(w.spe, w.spe, w.tbme())
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"# setup {t_setup:.2f} s, D = {model.dim}", file=sys.stderr, flush=True)

    nnz = stored_nnz(a.workload)
    hv64 = hv_timing(model, w.nb, torch.float64, a.hv_launches, torch)
    hv32 = hv_timing(model, w.nb, torch.float32, a.hv_launches, torch)
    print(f"# H.V fp64 {hv64 * 1e3:.3f} ms, fp32 {hv32 * 1e3:.3f} ms", file=sys.stderr, flush=True)
    if a.hv_only:
        if a.calib_copy:
            src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
        return

    if a.sweep:
        sweep(model, w, torch, np)
        return
    if a.truncated_start:
        truncated_start(model, w, a, torch)
        return

    def solve(prec):
        return model.solve(w.nb, w.n_eig, w.l_s, w.l_m, w.tol, prec, max_iter=3000, seed=1000,
                           check_every=a.check_every)

    for i in range(a.warmup):
        ev, _, info = solve("fp64")
        print(f"# warmup {i}: {info.iterations} it, {info.t_total:.3f} s, conv {info.converged}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        ev, _, info = solve("fp64")
        infos.append(info)
        print(f"# step {i}: {info.iterations} it, {info.restarts} restarts, {info.t_total:.3f} s, "
              f"conv {info.converged}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / a.steps
    inf = infos[-1]
    its = inf.iterations

    mixed = None
    if not a.no_mixed:
        evm, _, im = solve("mixed")
        torch.cuda.synchronize()
        t0m = time.perf_counter()
        evm, _, im = solve("mixed")
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0m
        rel = np.abs(evm - ev) / np.abs(ev)
        mixed = {"s_per_solve": tm, "iterations": im.iterations, "converged": im.converged,
                 "max_rel_err_vs_fp64": float(rel.max()), "median_rel_err_vs_fp64": float(np.median(rel)),
                 "t_hv": im.t_hv, "t_orth": im.t_orth, "t_eig": im.t_eig, "t_refine": im.t_refine}

    # per-phase device time of one FP64 solve (HIP events inside the library, on the solve's stream)
    phases = {"hv": inf.t_hv, "orth": inf.t_orth, "qr": inf.t_qr, "eig": inf.t_eig, "restart": inf.t_restart}
    hv_launch = inf.t_hv / max(its, 1)
    D = model.dim
    bytes_min = 2.0 * D * w.nb * 8
    if nnz:
        flops = 2.0 * w.nb * nnz
        traffic = stored_traffic(a.workload)
        roof = {"bound": "alu", "achieved": flops / hv_launch / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / hv_launch / 1e12 / PEAK_FP64_TFLOPS, "traffic": traffic,
                "kernel": ("block H.V, FP64: fly_kernel (single species, generated per element) + two row permutations"
                           if (w.n_prot == 0) != (w.n_neut == 0) and D > 2048 else
                           "block H.V, FP64: hv_rows_kernel (one launch per sector-width bin) + hv_cols_kernel"),
                "measured_GBs": (traffic / hv_launch / 1e9) if traffic else None,
                "per_launch": {"elements": nnz, "flops": flops, "compulsory_bytes": bytes_min,
                               "avg_duration_s": hv_launch}}
    else:
        roof = None
    out = {
        "metric": METRIC, "value": t, "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {w.n_prot}+{w.n_neut} nucleons, orbits {list(w.orbits)}, 2M={w.twoM}, "
                               f"D={D}, random J-coupled TBMEs sigma={w.sigma} seed {w.seed}; TRBL nb={w.nb}, "
                               f"{w.n_eig} lowest, l_s={w.l_s}, l_m={w.l_m}, tol={w.tol}",
                   "D": D, "nb": w.nb, "n_eig": w.n_eig, "l_s": w.l_s, "l_m": w.l_m, "tol": w.tol,
                   "check_every": a.check_every},
        "iterations": its, "restarts": inf.restarts, "phases_s": phases,
        "hv": {"fp64_ms": hv64 * 1e3, "fp32_ms": hv32 * 1e3,
               "fp64_compulsory_GBs": bytes_min / hv64 / 1e9, "fp32_compulsory_GBs": bytes_min / 2 / hv32 / 1e9,
               "fp64_TFLOPs": (2.0 * w.nb * nnz / hv64 / 1e12) if nnz else None,
               "fp32_TFLOPs": (2.0 * w.nb * nnz / hv32 / 1e12) if nnz else None},
        "mixed": mixed, "roofline": roof, "setup_s": t_setup,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, its)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
