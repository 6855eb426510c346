"""Benchmark: time-to-solve of the two-level Schwarz preconditioned normal
equations on the batched banded workload (the largest single-GPU workload).

One step = the whole hot path on one batch of synthetic input: setup (index
sets, A^T, local matrices, batched Cholesky, coarse eigenproblems, coarse
operator) plus the CG solve of every instance to a 1e-8 relative
normal-equation residual, then destroy.  Inputs (CSR arrays of every
instance, b) are resident in HBM before the timed region starts.

Workload (default): 64 independent least-squares instances, instance j with
n_j = round(exp U(ln 5e3, ln 2e5)) columns, 2 n_j random rows of 4 entries
near the diagonal plus n_j rows 0.1 e_j, N_j = round(exp U(ln 8, ln 128))
contiguous parts, overlap 1, tau = 0.1, seeds 3000 + j; 2,990,087 columns,
26.9M stored entries, 2,994 subdomains in total.

Prints ONE JSON line.  ``value`` is the FP64 time-to-solve (ms); the mixed
precision path (FP32 local factors and solves), its ratio to FP64, the SpMV
bandwidths, the roofline of the dominant per-iteration kernel (the batched
local triangular solves) and, as context, the 1000 x 1000 grid and the
irregular 1e6-column problem are reported beside it, with the CPU oracle (a
bounded sample, extrapolated) as the reported CPU baseline.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CALIB_BYTES = 1 << 30          # plain device copy used to calibrate HBM counters

# HBM traffic of one launch of the dominant kernel (the FP64 local solves,
# k_local_solve_pipe<double>) on the default workload, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs of this script, each scaled by the same
# counter's reading for the calibration copy (profiles/local_solve_banded_batch_64.md).
# It describes the kernel source whose SHA-256 is given; for any other source
# the figure is reported as null.
TRAFFIC = {"source": "paper_2107_09006_amd/csrc/k_solve.hip",
           "sha256": "3730a371a904e7e39a98b740966380b5f5a7f7a6c63f2243ecf41d40cc648404",
           "bytes": 2107597.3 * 1024 * 2.0 + 24834.91 * 1024 * 1.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def to_device(prob):
    import torch
    return {"rowptr": torch.as_tensor(prob.indptr.astype(np.int64)).cuda(),
            "colind": torch.as_tensor(prob.indices).cuda(),
            "vals": torch.as_tensor(prob.data).cuda(),
            "b": torch.as_tensor(prob.b).cuda()}


class Workload:
    """A single problem or a batch, with its device arrays."""

    def __init__(self, name, probs, describe):
        import torch
        self.name = name
        self.probs = probs
        self.describe = describe
        self.dev = [to_device(p) for p in probs]
        self.b = torch.cat([d["b"] for d in self.dev]) if len(probs) > 1 else self.dev[0]["b"]
        self.n = sum(p.n for p in probs)
        self.m = sum(p.m for p in probs)
        self.nnz = sum(p.nnz for p in probs)
        self.nparts = sum(p.nparts for p in probs)
        self.x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self.opts = {}                     # options every setup of this workload takes
        torch.cuda.synchronize()

    def solver(self, L, **opts):
        p0 = self.probs[0]
        opts = {**self.opts, **opts}
        if len(self.probs) == 1:
            d = self.dev[0]
            return L.Solver(d["rowptr"], d["colind"], d["vals"], p0.part, p0.nparts, p0.m, p0.n,
                            p0.tau, device="cuda:0", tol=p0.tol, **opts)
        args = [(d["rowptr"], d["colind"], d["vals"], p.part, p.nparts, p.m, p.n)
                for d, p in zip(self.dev, self.probs)]
        return L.Solver.batched(args, p0.tau, device="cuda:0", tol=p0.tol, **opts)


def run_step(L, wl, precision, variant, **extra):
    """setup + solve + destroy; returns (ms, per-instance solve infos, setup info)."""
    import torch
    t0 = time.perf_counter()
    s = wl.solver(L, precision=precision, variant=variant,
                  flexible=int(variant == L.BALANCED and precision == L.MIXED), **extra)
    _, info, _ = s.solve(wl.b, x=wl.x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    sinfo = s.info()
    s.close()
    return ms, info, sinfo


def timed(L, wl, precision, variant, steps, warmup, tag, **extra):
    import torch
    for w in range(warmup):
        ms, info, _ = run_step(L, wl, precision, variant, **extra)
        log(f"[bench] {tag} warmup {w}: {ms:.1f} ms, its {max(i['iterations'] for i in info)}")
    # Python's collector stays off while the steps are timed (it is run
    # before and after), so that a collection pause of the interpreter does
    # not land inside a step
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = []
    for k in range(steps):
        out.append(run_step(L, wl, precision, variant, **extra))
        ms, info, _ = out[-1]
        ph = out[-1][2]
        log(f"[bench] {tag} step {k}: {ms:.1f} ms, its {max(i['iterations'] for i in info)}, "
            f"relres {max(i['relres'] for i in info):.2e}, setup " +
            " ".join(f"{q[2:-3]} {ph[q]:.1f}" for q in ["t_prepare_ms", "t_plan_ms", "t_assemble_ms",
                                                          "t_factor_ms", "t_eigen_ms", "t_coarse_ms"]))
    torch.cuda.synchronize()
    total = (time.perf_counter() - t0) * 1e3
    gc.enable()
    ms, info, sinfo = out[-1]
    return {"ms_per_step": total / steps,
            "iterations_max": max(i["iterations"] for i in info),
            "iterations_mean": float(np.mean([i["iterations"] for i in info])),
            "relres_max": max(i["relres"] for i in info),
            "setup_ms": float(np.mean([o[2]["t_total_ms"] for o in out])),
            "solve_ms": float(np.mean([o[1][0]["solve_ms"] for o in out])),
            "setup": sinfo}


def kernel_times(L, wl, precision, reps=10):
    s = wl.solver(L, precision=precision)
    out = {}
    for kid, kname in [(0, "spmv_A"), (1, "spmv_AT"), (2, "local_solve_stored"),
                       (4, "local_solve_min"), (3, "coarse_solve")]:
        try:
            ms, by = s.time_kernel(kid, reps=reps)
        except Exception as e:  # no coarse space
            log(f"[bench] {kname}: {e}")
            continue
        out[kname] = {"ms": ms, "bytes": by, "GBs": by / ms / 1e6}
        log(f"[bench] kernel {kname} ({precision}): {ms * 1e3:.1f} us, {by / 1e6:.1f} MB, "
            f"{by / ms / 1e6:.0f} GB/s")
    info = s.info()
    s.close()
    return out, info


def cpu_baseline(wl, iterations, budget_s=20.0):
    """The oracle on a bounded sample of the same workload, extrapolated:
    per-subdomain setup (local matrices, Cholesky, Lemma 2.4 eigenproblem)
    timed on seeded random subdomains with at most 3,000 local unknowns until
    the budget is spent, fitted as c n_i^3 and summed over every subdomain;
    index sets and one A^T A p of every instance in full; iterations x (two
    SpMVs + the local solves, scaled the same way)."""
    import oracle as O
    import scipy.linalg as sla
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    sets = [O.index_sets(p.scipy(), p.part, p.nparts) for p in wl.probs]
    t_index = time.perf_counter() - t0
    allsub = [(k, i) for k, ss in enumerate(sets) for i in range(len(ss))]
    ni = np.array([sets[k][i].ni for k, i in allsub], dtype=np.float64)
    rng = np.random.default_rng(0)
    cand = [j for j in rng.permutation(len(allsub)) if ni[j] <= 3000]
    t_sub = t_app = 0.0
    cube = square = 0.0
    used = 0
    for j in cand:
        if t_sub >= budget_s:
            break
        k, i = allsub[j]
        A = wl.probs[k].scipy()
        s = sets[k][i]
        r = rng.standard_normal(s.ni)
        t1 = time.perf_counter()
        Cii, Ctii = O.local_matrices(A, s)
        F = sla.cho_factor(Cii, lower=True)
        O.coarse_vectors(Cii, Ctii, s.nI, wl.probs[k].tau)
        t2 = time.perf_counter()
        sla.cho_solve(F, r)
        t3 = time.perf_counter()
        t_sub += t2 - t1
        t_app += t3 - t2
        cube += ni[j] ** 3
        square += ni[j] ** 2
        used += 1
    t4 = time.perf_counter()
    for p in wl.probs:
        A = p.scipy()
        A.T @ (A @ np.ones(p.n))
    t_spmv = time.perf_counter() - t4
    setup = t_index + t_sub / cube * float(np.sum(ni ** 3))
    per_it = t_spmv + t_app / square * float(np.sum(ni ** 2))
    total_ms = (setup + iterations * per_it) * 1e3
    return {"value": round(total_ms, 1), "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": (f"oracle setup (local matrices, Cholesky, Lemma 2.4 eigenproblem) and a "
                       f"local solve timed on {used} of {len(allsub)} subdomains (seeded random, "
                       f"n_i <= 3000), fitted as c n_i^3 (setup) and c n_i^2 (solve) and summed "
                       f"over all subdomains; index sets and one A^T A p of every instance in "
                       f"full; {iterations} iterations (the GPU count); extrapolated")}


def measured_traffic():
    if not TRAFFIC["sha256"] or TRAFFIC["bytes"] is None:
        return None
    with open(os.path.join(ROOT, TRAFFIC["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["sha256"]:
            return None
    return TRAFFIC["bytes"]


def calibration_copy():
    """One plain device-to-device copy of CALIB_BYTES (not timed): the
    reference reading for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def make_workload(name):
    from workloads import generators as W
    if name == "banded_batch_64":
        probs = W.banded_batch_64()
        return Workload(name, probs, "banded_batch_64: 64 instances, n_j log-uniform in [5e3, 2e5], "
                        "2 n_j rows of 4 entries near the diagonal + n_j rows 0.1 e_j, "
                        "8-128 contiguous parts each, tau 0.1")
    if name == "grid_1000":
        return Workload(name, [W.grid_1000()], "grid_1000: forward differences on a 1000 x 1000 "
                        "grid + 1e6 rows 1e-3 e_j, 16 x 16 patches, tau 0.1")
    if name == "irregular_1m":
        return Workload(name, [W.strip_rng(W.irregular_1m())],
                        "irregular_1m: 3e6 clustered random rows, columns scaled 10^U(-3,3), "
                        "+ 1e6 rows 1e-4 e_j; 512 BFS parts, tau 0.05")
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["banded_batch_64", "grid_1000", "irregular_1m"],
                    default="banded_batch_64")
    ap.add_argument("--variant", choices=["additive", "balanced"], default="additive",
                    help="second-level form (eq. two_level_schwarz or eq. balanced)")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the other workloads reported as context")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--local-factor", choices=["cholesky", "qr"], default="cholesky",
                    help="local factors of the whole line: Cholesky of C_ii (default) or thin QR "
                         "of A(:, Omega_i) with the principal-angle selection (Remarks 3.1, 3.2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2107_09006_amd as L

    variant = L.BALANCED if args.variant == "balanced" else L.ADDITIVE
    log(f"[bench] generating {args.workload}")
    wl = make_workload(args.workload)
    if args.local_factor == "qr":
        wl.opts["local_factor"] = L.FACTOR_QR
    calibration_copy()
    fp64 = timed(L, wl, L.FP64, variant, args.steps, args.warmup, "fp64")
    mixed = timed(L, wl, L.MIXED, variant, args.steps, args.warmup, "mixed")
    kern64, info64 = kernel_times(L, wl, L.FP64)
    kern32, _ = kernel_times(L, wl, L.MIXED)
    # the QR route of Remarks 3.1 / 3.2 (local factors from thin QR
    # factorizations of A(:, Omega_i), principal-angle selection), FP64
    qr = fp64 if args.local_factor == "qr" else timed(L, wl, L.FP64, variant, 2, 1, "qr",
                                                     local_factor=L.FACTOR_QR)

    # dominant per-iteration kernel of the FP64 path: the batched local
    # triangular solves; achieved = algorithmic bytes (nnz(L_i) under a
    # fill-reducing order, Omega_Gamma_i last, both sweeps, y in and out) per
    # launch / the launch's duration; the fraction for the stored tile
    # envelope is reported beside it
    dom = kern64.get("local_solve_min")
    stored = kern64.get("local_solve_stored")
    roofline = None
    if dom:
        roofline = {"kernel": "k_local_solve_pipe<double>", "bound": "hbm",
                    "achieved": round(dom["GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(dom["GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic() if args.workload == "banded_batch_64" else None,
                    "bytes_per_launch": dom["bytes"], "launch_ms": dom["ms"],
                    "stored_bytes_per_launch": stored["bytes"] if stored else None,
                    "frac_stored": round(stored["GBs"] / HBM_PEAK_GBS, 4) if stored else None,
                    "factor_nnz_min": info64["factor_nnz_min"],
                    "factor_stored_entries": info64["factor_tiles"] * 1024}
    out = {
        "metric": "time-to-solve @1e-8 rel normal-eq residual; SpMV GB/s; mixed vs FP64 speedup",
        "value": round(fp64["ms_per_step"], 2),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp64["ms_per_step"], 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.describe, "instances": len(wl.probs), "m": wl.m, "n": wl.n,
                   "nnz": wl.nnz, "nparts": wl.nparts, "tau": wl.probs[0].tau,
                   "tol": wl.probs[0].tol, "overlap": 1, "variant": args.variant,
                   "krylov": "pcg", "local_factor": args.local_factor},
        "iterations_max": fp64["iterations_max"],
        "iterations_mean": round(fp64["iterations_mean"], 2),
        "relres_max": fp64["relres_max"],
        "setup_ms": round(fp64["setup_ms"], 2),
        "solve_ms": round(fp64["solve_ms"], 2),
        "setup_phases_ms": {k: round(fp64["setup"][k], 2) for k in
                            ["t_prepare_ms", "t_plan_ms", "t_assemble_ms", "t_factor_ms", "t_eigen_ms",
                             "t_coarse_ms"]},
        "solve_factor": {"tiles": fp64["setup"]["factor_tiles"],
                         "split_order_tiles": fp64["setup"]["split_tiles"],
                         "subdomains_in_global_order": fp64["setup"]["solve_permuted"],
                         "mixed_fp32_factor_fallback": mixed["setup"]["mixed_fallback"]},
        "n0": fp64["setup"]["n0"],
        "mixed_ms_per_step": round(mixed["ms_per_step"], 2),
        "mixed_iterations_max": mixed["iterations_max"],
        "mixed_relres_max": mixed["relres_max"],
        "mixed_vs_fp64_speedup": round(fp64["ms_per_step"] / mixed["ms_per_step"], 3),
        "spmv_GBs": {"A": round(kern64["spmv_A"]["GBs"], 1), "AT": round(kern64["spmv_AT"]["GBs"], 1)},
        "kernels": {f"{k}_{tag}": {"us": round(v["ms"] * 1e3, 2), "MB": round(v["bytes"] / 1e6, 2),
                                   "GBs": round(v["GBs"], 1)}
                    for tag, kd in (("fp64", kern64), ("mixed", kern32)) for k, v in kd.items()},
        "roofline": roofline,
        "qr_route": {"ms_per_step": round(qr["ms_per_step"], 2), "setup_ms": round(qr["setup_ms"], 2),
                     "solve_ms": round(qr["solve_ms"], 2),
                     "setup_phases_ms": {k: round(qr["setup"][k], 2) for k in
                                         ["t_plan_ms", "t_assemble_ms", "t_factor_ms", "t_eigen_ms",
                                          "t_coarse_ms"]},
                     "iterations_max": qr["iterations_max"], "relres_max": qr["relres_max"],
                     "n0": qr["setup"]["n0"]},
    }
    if not args.no_context:
        ctx = {}
        for name in ("grid_1000", "irregular_1m"):
            if name == args.workload:
                continue
            log(f"[bench] context workload {name}")
            w2 = make_workload(name)
            f2 = timed(L, w2, L.FP64, variant, 1, 1, f"{name} fp64")
            m2 = timed(L, w2, L.MIXED, variant, 1, 1, f"{name} mixed")
            k2, _ = kernel_times(L, w2, L.FP64)
            ctx[name] = {"fp64_ms": round(f2["ms_per_step"], 2), "mixed_ms": round(m2["ms_per_step"], 2),
                         "mixed_vs_fp64_speedup": round(f2["ms_per_step"] / m2["ms_per_step"], 3),
                         "iterations": f2["iterations_max"], "relres": f2["relres_max"],
                         "setup_ms": round(f2["setup_ms"], 2), "solve_ms": round(f2["solve_ms"], 2),
                         "spmv_GBs": {"A": round(k2["spmv_A"]["GBs"], 1),
                                      "AT": round(k2["spmv_AT"]["GBs"], 1)},
                         "local_solve_min_GBs": round(k2["local_solve_min"]["GBs"], 1)
                         if "local_solve_min" in k2 else None}
            del w2
            torch.cuda.empty_cache()
        out["context_workloads"] = ctx
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(wl, fp64["iterations_max"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
