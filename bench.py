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
    p.add_argument("--large-solve", action="store_true",
                   help="pf66 only: one TRBL solve for the 200 lowest (nb = 32, tol 1e-5 relative) with the basis "
                        "sized to the free HBM; prints time to the 200 eigenpairs")
    p.add_argument("--large-precision", default="mixed", choices=["mixed", "fp64"])
    p.add_argument("--large-nb", type=int, default=32)
    p.add_argument("--large-ls", type=int, default=320)
    p.add_argument("--large-lm", type=int, default=0, help="0: as many as fit")
    p.add_argument("--large-max-s", type=float, default=1000.0,
                   help="stop after about this many seconds of iterations (max_iter from the measured rate)")
    p.add_argument("--cpu-baseline-full", action="store_true",
                   help="host only: the oracle's block H.V (median of 5) on the sd 2+2 and sd 6+6 workloads in full "
                        "and on a row sample of pf44, and the oracle TRBL time to N on sd 2+2 and sd 6+6")
    p.add_argument("--sweep", action="store_true",
                   help="block-size sweep instead of the benchmark: H.V time against nb = 1..32 and TRBL solves "
                        "for the 32 lowest with 160 or 320 new vectors per restart cycle and without restarts")
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


HV_SOURCES = ("hv.hip", "hv_kern.h", "hv_f64.hip", "hv_f32.hip", "pntile.hip", "tilecore.h")


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


def host_info():
    """Host cores and CPU model (the oracle runs on these)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline_full():
    """The oracle timed on the host cores: block H.V (median of 5) on sd 2+2 and sd 6+6 in full and
    on a 20,000-row sample of pf44 (scaled to the full matrix), and the oracle TRBL (Alg. 4) time to
    the wanted eigenpairs on sd 2+2 and sd 6+6 with the GPU bench's parameters."""
    import numpy as np

    from oracle.hamiltonian import model_from_workload, threads
    from oracle.trbl import trbl
    from workloads import WORKLOADS, random_block
    res = {"host": host_info(), "oracle_threads": threads(), "hv": {}, "time_to_n": {}}
    for name in ("sd22", "sd66", "pf44"):
        w = WORKLOADS[name]
        t0 = time.perf_counter()
        m = model_from_workload(w)
        t_build = time.perf_counter() - t0
        V = random_block(2000, m.dim, w.nb)
        if name == "pf44":
            idx = np.sort(np.random.default_rng(0).choice(m.dim, 20000, replace=False))
        else:
            idx = np.arange(m.dim)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            m.apply_rows(V, idx)
            ts.append(time.perf_counter() - t0)
        med = float(np.median(ts))
        res["hv"][name] = {"D": m.dim, "nb": w.nb, "rows_timed": len(idx), "median_s": med,
                           "per_full_hv_s": med * m.dim / len(idx), "build_s": t_build}
        print(f"# oracle H.V {name}: {med:.4f} s for {len(idx)} rows -> {med * m.dim / len(idx):.3f} s per H.V",
              file=sys.stderr, flush=True)
        if name in ("sd22", "sd66"):
            t0 = time.perf_counter()
            ev, _, info = trbl(m.apply, m.dim, random_block(1000, m.dim, w.nb), w.n_eig, w.l_s, w.l_m, w.tol)
            t = time.perf_counter() - t0
            res["time_to_n"][name] = {"n_eig": w.n_eig, "nb": w.nb, "l_s": w.l_s, "l_m": w.l_m, "tol": w.tol,
                                      "s": t, "iterations": info["iterations"], "converged": bool(info["converged"])}
            print(f"# oracle TRBL {name}: {t:.2f} s, {info['iterations']} iterations", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


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
        **host_info(),
        "kind": "oracle",
        "sample": (f"oracle block H.V (nb={w.nb}) on {n2} random rows of {m.dim} ({t2:.1f} s), scaled to the "
                   f"full matrix ({per_hv:.1f} s per H.V) and to the {iterations} block iterations of the GPU "
                   f"solve; H.V only, so a lower bound on the oracle's time to {w.n_eig} eigenpairs"),
    }


def sweep(model, w, torch, np):
    """Trade-off of Sec. 4.1 / 4.2: block H.V time against nb (a line whose intercept is the fixed
    generation cost), and iterations / time to the 32 lowest eigenpairs against nb for three restart
    settings: a fixed number of new vectors per restart cycle (l_m - l_s = 160 and 320) and no
    restart at all (l_m at the device eigensolver's limit, which the solve does not reach)."""
    nbs = (1, 2, 4, 8, 16, 32)
    hv = {}
    for nb in nbs:
        hv[nb] = hv_timing(model, nb, torch.float64, 10, torch)
        print(f"# H.V nb={nb}: {hv[nb] * 1e3:.3f} ms", file=sys.stderr, flush=True)
    x = np.array(nbs, dtype=float)
    slope, icpt = np.polyfit(x, np.array([hv[nb] * 1e3 for nb in nbs]), 1)
    settings = [("cycle160", 40, lambda nb: 200), ("cycle320", 64, lambda nb: 384),
                ("largest", 40, lambda nb: 640 + nb)]
    rows = []
    for name, ls, lmf in settings:
        for nb in nbs:
            lm = lmf(nb)
            ev, _, info = model.solve(nb, 32, ls, lm, 1e-8, "fp64", max_iter=20000, seed=1000, check_every=-1)
            r = {"setting": name, "nb": nb, "l_s": ls, "l_m": lm, "hv_ms": hv[nb] * 1e3,
                 "iterations": info.iterations, "matvecs": info.iterations * nb, "restarts": info.restarts,
                 "converged": info.converged, "t_total_s": info.t_total, "t_hv_s": info.t_hv,
                 "t_orth_s": info.t_orth, "t_qr_s": info.t_qr, "t_eig_s": info.t_eig, "t_restart_s": info.t_restart,
                 "e0": float(ev[0]), "e31": float(ev[31])}
            print("# " + json.dumps(r), file=sys.stderr, flush=True)
            rows.append(r)
    print(json.dumps({"sweep": rows, "hv_fit_ms": {"intercept": icpt, "slope_per_vector": slope},
                      "workload": w.name, "n_eig": 32, "tol": 1e-8}))


def large_solve(model, w, a, torch, np, t_setup, hv64, hv32):
    """One TRBL solve of the large space for its wanted eigenpairs, the basis sized to the free
    HBM: the stored vectors take what is left after the packed block, the FP64 work block (FP64
    only), the final FP64 check or refinement chunks (8 GB each) and a 6 GB margin. l_m - nb is
    capped at 640, the largest projected matrix of the device eigensolver. Progress lines of the
    solver go to stderr; the eigenvalues and residuals are written next to the JSON line."""
    D = model.dim
    nb = a.large_nb
    mixed = a.large_precision == "mixed"
    s = 4 if mixed else 8
    torch.cuda.empty_cache()  # the H.V timing blocks
    free, total = torch.cuda.mem_get_info()
    reserve = D * nb * s + (0 if mixed else D * nb * 8) + 2 * 8e9 + 6e9
    lm_fit = int((free - reserve) // (D * s))
    lm = a.large_lm or min(640 + nb, lm_fit) // nb * nb
    ls = min(a.large_ls, lm - 2 * nb)
    n_eig = min(w.n_eig, ls)
    tol = 1e-5
    # iteration budget from the measured H.V rate (the other per-iteration work is about half of it)
    hv = hv32 if mixed else hv64
    max_iter = max(8, int(a.large_max_s / (1.6 * hv * max(nb / w.nb, 0.5))))
    print(f"# large solve: {a.large_precision}, D={D}, nb={nb}, n_eig={n_eig}, l_s={ls}, l_m={lm} "
          f"(fits {lm_fit}), free {free / 1e9:.1f} GB of {total / 1e9:.1f} GB, max_iter {max_iter}",
          file=sys.stderr, flush=True)
    os.environ["TRBL_VERBOSE"] = "1"
    t0 = time.perf_counter()
    ev, _, info = model.solve(nb, n_eig, ls, lm, tol, a.large_precision, max_iter=max_iter, seed=1000,
                              check_every=-1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    os.environ["TRBL_VERBOSE"] = "0"
    out_dir = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"large_{w.name}_{a.large_precision}_nb{nb}_evals.txt")
    with open(path, "w") as f:
        f.write(f"# {w.name} {a.large_precision} nb={nb} l_s={ls} l_m={lm} tol={tol} converged={info.converged} "
                f"iterations={info.iterations} restarts={info.restarts} n_converged={info.n_converged}\n")
        for x, r in zip(ev, info.resid):
            f.write(f"{x:.17g} {r:.6g}\n")
    out = {
        "metric": f"s to {n_eig} converged eigenpairs ({a.large_precision})", "value": t if info.converged else None,
        "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_prot}+{w.n_neut} nucleons, orbits {list(w.orbits)}, 2M={w.twoM}, "
                               f"D={D}, random J-coupled TBMEs sigma={w.sigma} seed {w.seed}; TRBL nb={nb}, "
                               f"{n_eig} lowest, l_s={ls}, l_m={lm}, tol={tol} of max|theta|",
                   "D": D, "nb": nb, "n_eig": n_eig, "l_s": ls, "l_m": lm, "tol": tol, "max_iter": max_iter},
        "solve_s": t, "converged": info.converged, "n_converged": info.n_converged,
        "iterations": info.iterations, "restarts": info.restarts,
        "phases_s": {"hv": info.t_hv, "orth": info.t_orth, "qr": info.t_qr, "eig": info.t_eig,
                     "restart": info.t_restart, "refine": info.t_refine},
        "max_resid_rel": float(np.max(info.resid) / max(abs(ev).max(), 1e-300)),
        "lowest": float(ev[0]), "highest_wanted": float(ev[-1]), "setup_s": t_setup,
        "hv": {"fp64_ms": hv64 * 1e3, "fp32_ms": hv32 * 1e3}, "hbm_free_GB": free / 1e9, "evals_file": path,
    }
    print(json.dumps(out), flush=True)


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

    if a.cpu_baseline_full:
        cpu_baseline_full()
        return
    w = WORKLOADS[a.workload]
    if w.name == "pf66" and not (a.hv_only or a.large_solve):
        print("pf66: --hv-only (H.V timing) or --large-solve (one solve for the 200 lowest)", file=sys.stderr)
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

    if a.large_solve:
        large_solve(model, w, a, torch, np, t_setup, hv64, hv32)
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
                "kernel": ("block H.V, FP64: fly_tile_kernel (single species: two-body part as pair blocks on the "
                           "matrix cores) + fly_finalize_kernel (diagonal and slot sum) + two row permutations"
                           if (w.n_prot == 0) != (w.n_neut == 0) and D > 2048 else
                           "block H.V, FP64: pn_tile_kernel (proton-neutron part, core-pair blocks on the matrix "
                           "cores) + hv_own_kernel (neutron-neutron part and slot sum, one launch per sector-width bin) "
                           "+ hv_cols_kernel (proton-proton part)"
                           if a.workload == "pf44" else
                           "block H.V, FP64: every kernel of one product (the proton-neutron part on core-pair blocks "
                           "or on jump lists, as chosen at set-up from the width and the pairs per core pair)"),
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
