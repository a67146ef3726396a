"""Benchmark: two-electron TDA-TDDFT gradient (ERI-derivative J/K part) on one MI355X.

Workload: the 60-atom alkane-like chain (20 heavy + 40 H atoms, 500 Cartesian
functions, l <= 2, contraction degrees up to 6), seeded synthetic densities,
omega = 0.3, alpha = 0.157706, beta = 0.842294, density-multiplied Schwarz
threshold 1e-10, all terms (J, full-range K, long-range K).  Both the FP64 path
and the mixed path (FP32 2D integrals for quartets the bounded router sends to
FP32, FP64 roots and sums; every class runs the precision its autotuning
measured faster) are timed; the headline value is the faster one whose gradient
stays within 1e-6 Eh/bohr of the oracle's (stored under tests/golden/).  A third
leg routes on class timing alone (no error bound) and is reported beside them.

One step = one call of the library's gradient entry point with the densities
already resident in device memory: density preparation, screening and task
generation, all 21 ERI-derivative class kernels and the per-atom reduction.

Prints one JSON line: the metric, the headline value and its configuration, both paths'
figures, the roofline of the dominant class kernel (achieved algorithmic FLOP rate against
the FP64 vector peak, and its HBM bytes per launch when the committed counter summary under
profiles/ was taken on the current kernel sources) and the CPU oracle's rate on a sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ERI-deriv quartets/s & J/K-grad wall s, mixed vs FP64 on 1 GPU @1e-6 Eh/bohr"
FP64_VALU_PEAK_TFLOPS = 78.6


def _sources_sha():
    """sha256 (16 hex digits) over the HIP sources, in path order."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2407_16586_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def launch_quartets(stats, c, prec):
    """Quartets in class c's launch of the given precision ("fp64" or "fp32"): a class in
    mixed mode runs its FP32-routed quartets in their own FP32 launch unless the autotuner
    kept the class in one FP64 launch (class_variant bit 6)."""
    n, n32 = stats["class_quartets"][c], stats["class_fp32_quartets"][c]
    split = n32 > 0 and not (stats["class_variant"][c] & 64)
    if prec == "fp32":
        return n32 if split else 0
    return n - n32 if split else n


def _traffic(cls, variant, prec, nq):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration) of one
    class kernel from the committed counter summaries, or None when none was taken on the
    current sources for a launch of the same number of quartets."""
    import glob
    sha, key = _sources_sha(), "".join(map(str, cls))
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.txt"))):
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) >= 8 and f[0] == "traffic" and f[1] == key and f[2] == str(variant) and f[3] == prec \
                        and f[4] == sha and f[7] == str(nq):
                    return int(f[5]) + int(f[6])
    return None


def _executed_flops(cls, variant, prec, nq):
    """Executed floating-point operations per launch of one class kernel from the committed
    instruction-counter summaries (64 lanes x (2 FMA + ADD + MUL + TRANS) per wavefront
    instruction, FP64 and FP32), or None when none was taken on the current sources for a
    launch of the same number of quartets."""
    import glob
    sha, key = _sources_sha(), "".join(map(str, cls))
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_flops.txt"))):
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) >= 8 and f[0] == "flops" and f[1] == key and f[2] == str(variant) and f[3] == prec \
                        and f[4] == sha and f[7] == str(nq):
                    return int(f[5]), int(f[6])
    return None


def _fock_kernel_name(cls):
    """The Fock-type matrix kernel a class runs (long-range term present)."""
    n = 1
    for l in cls:
        n *= (l + 1) * (l + 2) // 2
    layout = "k_fock_lane" if n <= 27 else ("k_fock_lane, lane pairs" if n <= 54 else "k_fock")
    return f"{layout} {cls}"


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(mol, target_s=15.0, seed=7):
    """The oracle, untuned, on a bounded random sample of the workload's surviving quartets
    (drawn uniformly from the unique shell quartets and kept when the oracle's own
    density-multiplied Schwarz bound passes): all host threads, then one thread on the
    first part of the same sample."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    rng = np.random.default_rng(seed)
    ns = mol.n_shells
    a = np.arange(ns)
    pa = np.concatenate([np.full(i + 1, i) for i in range(ns)])
    pb = np.concatenate([a[: i + 1] for i in range(ns)])
    npair = len(pa)
    atom = mol.shell_atom
    nthreads = os.cpu_count() or 1

    def draw(nsurv):
        out, have = [], 0
        while have < nsurv:
            i = rng.integers(0, npair, 8_000_000)
            j = rng.integers(0, npair, 8_000_000)
            hi, lo = np.maximum(i, j), np.minimum(i, j)
            q = np.stack([pa[hi], pb[hi], pa[lo], pb[lo]], 1).astype(np.int32)
            one = (atom[q[:, 0]] == atom[q[:, 1]]) & (atom[q[:, 1]] == atom[q[:, 2]]) & (atom[q[:, 2]] == atom[q[:, 3]])
            q = q[~one]
            q = q[oracle.quartet_bounds(mol, q) >= 1e-10]
            out.append(q)
            have += len(q)
        return np.concatenate(out)[:nsurv]

    probe = draw(4000)
    t = time.perf_counter()
    oracle.quartet_contribs(mol, probe, nthreads=nthreads)
    rate = len(probe) / (time.perf_counter() - t)
    n = int(min(3_000_000, max(4000, rate * target_s)))
    sample = draw(n)
    t = time.perf_counter()
    oracle.quartet_contribs(mol, sample, nthreads=nthreads)
    dt = time.perf_counter() - t
    # one thread: a sample of about target_s / 3 seconds
    n1 = int(max(1000, min(n, (n / dt) / nthreads * target_s / 3)))
    t = time.perf_counter()
    oracle.quartet_contribs(mol, sample[:n1], nthreads=1)
    dt1 = time.perf_counter() - t
    return {"value": n / dt, "unit": "quartets/s", "cores": nthreads, "kind": "oracle",
            "value_1thread": n1 / dt1, "cpu_model": _cpu_model(),
            "sample": f"{n} surviving shell quartets drawn uniformly from the workload's unique "
                      f"quartets (oracle's own screening at 1e-10), {dt:.1f} s on {nthreads} threads; "
                      f"the first {n1} of them on 1 thread, {dt1:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--path", choices=("both", "fp64", "mixed"), default="both",
                    help="precision paths to time; with both, the headline is the mixed path when it "
                         "is faster and within 1e-6 Eh/bohr of the FP64 path")
    ap.add_argument("--mixed-tau64", type=float, default=0.1,
                    help="mixed path's routing bound (a quartet runs in FP32 when its density-weighted "
                         "bound times the pair exponent scales is below this)")
    ap.add_argument("--mixed-p64", type=float, default=1e4,
                    help="mixed path: pairs with a primitive exponent sum at or above this stay in FP64")
    ap.add_argument("--no-unbounded", action="store_true",
                    help="skip the secondary mixed leg that routes on class timing alone (tau64 = inf)")
    ap.add_argument("--streams", type=int, default=0,
                    help="streams the class kernels of a timed call run on (0 = the library's default, 4); "
                         "profiling runs use 1 so that every kernel is timed alone")
    ap.add_argument("--no-fock", action="store_true",
                    help="skip the Fock-type matrix leg (eq G_2e of the chain's relaxed difference density)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy MIB MiB device-to-device (a plain copy of known "
                         "size that calibrates the HBM counters of a profiling run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the quartet tasks would be "
              "shared out over GPUs with one gradient all-reduce, which is not built here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_16586_amd import synth, tdgrad
    from paper_2407_16586_amd.workmodel import FLOPS_PER_PRIM, fock_flops

    mol = synth.config1()
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    P0, PD, R = t(mol.P0), t(mol.PD), t(mol.R)

    # the oracle's gradient of this workload, stored by tests/golden/make_golden.py
    with open(os.path.join(ROOT, "tests", "golden", "chain60_tau1e-10.json")) as fh:
        golden = np.array(json.load(fh)["grad"])

    def run_path(precision, tau64=args.mixed_tau64, p64=args.mixed_p64):
        print(f"bench: plan for {mol.name}, precision {precision}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        plan = tdgrad.Plan(mol, schwarz_tol=1e-10, precision=precision, mixed_tau64=tau64, mixed_p64=p64,
                           streams=args.streams)
        plan_s = time.perf_counter() - t0
        out = torch.zeros((mol.n_atoms, 3), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            plan.grad_device(P0, PD, R, out, stats=True)
        torch.cuda.synchronize()
        # timed steps: the class kernels of a call run side by side on the plan's streams
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.grad_device(P0, PD, R, out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g = out.cpu().numpy().copy()
        # roofline leg: the same plan and kernels, one stream, so that the HIP events around
        # each class launch time that kernel alone
        plan.set_streams(1)
        stats = []
        for _ in range(args.steps):
            stats.append(plan.grad_device(P0, PD, R, out, stats=True))
        torch.cuda.synchronize()
        st = stats[-1]
        class_ms = np.mean([s["class_ms"] for s in stats], axis=0)
        prims = np.array(st["class_prim_quartets"], dtype=np.float64)
        flops = np.array([FLOPS_PER_PRIM[c] for c in tdgrad.CLASSES], dtype=np.float64) * prims
        dom = int(np.argmax(class_ms))
        # the dominant class's kernel: its FP64 kernel unless the class ran its (larger)
        # FP32-routed list with the FP32 kernel
        cv = st["class_variant"][dom]
        n32 = st["class_fp32_quartets"][dom]
        if not (cv & 64) and n32 * 2 > st["class_quartets"][dom]:
            dvar, dprec = (cv >> 3) & 7, "fp32"
        else:
            dvar, dprec = cv & 7, "fp64"
        ms_step = 1e3 * dt / args.steps
        achieved = flops[dom] / (class_ms[dom] * 1e-3) / 1e12
        all_tflops = flops.sum() / (class_ms.sum() * 1e-3) / 1e12
        nq_dom = launch_quartets(st, dom, dprec)
        ex = _executed_flops(tdgrad.CLASSES[dom], dvar, dprec, nq_dom)
        executed = (ex[0] + ex[1]) / (class_ms[dom] * 1e-3) / 1e12 if ex else None
        plan.close()
        return {
            "ms_step": ms_step, "plan_s": plan_s, "grad": g, "stats": st, "class_ms": class_ms,
            "err_oracle": float(np.abs(g - golden).max()),
            "quartets": st["quartets"], "value": st["quartets"] / (ms_step * 1e-3),
            "roofline": {"bound": "alu", "kernel": f"k_deriv{tdgrad.CLASSES[dom]} variant {dvar} {dprec}",
                         "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                         "traffic": _traffic(tdgrad.CLASSES[dom], dvar, dprec, launch_quartets(st, dom, dprec)),
                         "launch_quartets": nq_dom,
                         "launch_prim_quartets": int(prims[dom]) if not (cv & 64) or n32 == 0 else None,
                         "flop_per_prim_quartet": int(FLOPS_PER_PRIM[tdgrad.CLASSES[dom]]),
                         "executed": executed,
                         "executed_frac": executed / FP64_VALU_PEAK_TFLOPS if executed else None,
                         "all_classes_achieved": all_tflops,
                         "all_classes_frac": all_tflops / FP64_VALU_PEAK_TFLOPS},
        }

    def run_fock():
        """Fock-type matrix of eq G_2e (two-electron part) of the relaxed difference density,
        FP64, the same screening threshold; timed like the gradient steps."""
        with open(os.path.join(ROOT, "tests", "golden", "chain60_fock_pd.json")) as fh:
            gf = json.load(fh)
        print("bench: Fock-type matrix leg", file=sys.stderr, flush=True)
        plan = tdgrad.Plan(mol, schwarz_tol=1e-10, precision=0, streams=args.streams)
        Bd = t(getattr(mol, gf["density"]))
        F = torch.empty_like(Bd)
        cf = tuple(gf["coefs"])
        for _ in range(args.warmup):
            plan.fock_device(Bd, F, *cf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.fock_device(Bd, F, *cf)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        Fh = F.cpu().numpy()
        off, sl = mol.shell_ao_off, mol.shell_l
        nc = (sl + 1) * (sl + 2) // 2
        err = max(float(np.abs(Fh[off[a]:off[a] + nc[a], off[b]:off[b] + nc[b]] - np.array(blk)).max())
                  for (a, b), blk in zip(gf["pairs"], gf["blocks"]))
        st = plan.fock_device(Bd, F, *cf, stats=True)
        cms = np.array(st["class_ms"])
        fl = np.array([fock_flops(c, st["class_prim_quartets"][k], st["class_quartets"][k])
                       for k, c in enumerate(tdgrad.CLASSES)], dtype=np.float64)
        dom = int(np.argmax(cms))
        ach = fl[dom] / (cms[dom] * 1e-3) / 1e12
        plan.close()
        return {"value": st["quartets"] / (ms * 1e-3), "unit": "quartets/s", "ms_per_call": ms,
                "quartets": st["quartets"], "prim_quartets": st["prim_quartets"],
                "kernel_ms_one_stream": float(cms.sum()),
                "max_abs_err_vs_oracle_blocks": err,
                "coefs": cf, "density": gf["density"],
                "roofline": {"bound": "alu", "kernel": _fock_kernel_name(tdgrad.CLASSES[dom]), "achieved": ach,
                             "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK_TFLOPS,
                             "traffic": None, "launch_quartets": int(st["class_quartets"][dom]),
                             "launch_prim_quartets": int(st["class_prim_quartets"][dom]),
                             "all_classes_achieved": fl.sum() / (cms.sum() * 1e-3) / 1e12,
                             "all_classes_frac": fl.sum() / (cms.sum() * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS},
                "class_ms": {str(c): round(float(m), 4) for c, m in zip(tdgrad.CLASSES, cms)}}

    fp64 = run_path(0) if args.path in ("both", "fp64") else None
    mixed = run_path(1) if args.path in ("both", "mixed") else None
    unb = run_path(1, float("inf"), float("inf")) if args.path == "both" and not args.no_unbounded else None
    mixed_err = float(np.abs(mixed["grad"] - fp64["grad"]).max()) if fp64 and mixed else None
    # the headline: the mixed path when it is faster and within 1e-6 Eh/bohr of the oracle
    if fp64 and mixed:
        use_mixed = mixed["err_oracle"] <= 1e-6 and mixed["ms_step"] < fp64["ms_step"]
    else:
        use_mixed = mixed is not None
    head = mixed if use_mixed else fp64
    st = head["stats"]
    rec = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if use_mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "60-atom alkane-like chain, 500 Cartesian functions (l<=2), "
                               "J + full-range K + long-range K, omega=0.3, tau=1e-10",
                   "n_atoms": mol.n_atoms, "n_bf": mol.n_bf, "tau": 1e-10,
                   "precision": "mixed" if use_mixed else "fp64",
                   "mixed_tau64": args.mixed_tau64 if use_mixed else None,
                   "mixed_p64": (str(args.mixed_p64) if args.mixed_p64 == float("inf") else args.mixed_p64)
                   if use_mixed else None},
        "wall_s": head["ms_step"] * 1e-3,
        "quartets": head["quartets"],
        "screened_candidates": st["candidates"],
        "prim_quartets": st["prim_quartets"],
        "kernel_ms_one_stream": float(head["class_ms"].sum()),
        "kernel_quartets_per_s_one_stream": head["quartets"] / (head["class_ms"].sum() * 1e-3),
        "plan_s": head["plan_s"],
        "roofline": head["roofline"],
        "class_ms": {str(c): round(float(m), 4) for c, m in zip(tdgrad.CLASSES, head["class_ms"])},
        "class_variant": st["class_variant"],
        "class_quartets": st["class_quartets"],
        "class_prim_quartets": st["class_prim_quartets"],
        "class_fp32_quartets": st["class_fp32_quartets"],
        "max_abs_err_vs_oracle": head["err_oracle"],
    }
    if fp64:
        rec["fp64"] = {"value": fp64["value"], "wall_s": fp64["ms_step"] * 1e-3,
                       "kernel_ms_one_stream": float(fp64["class_ms"].sum()), "roofline_frac": fp64["roofline"]["frac"],
                       "all_classes_frac": fp64["roofline"]["all_classes_frac"],
                       "max_abs_err_vs_oracle": fp64["err_oracle"]}
    if mixed:
        rec["mixed"] = {"value": mixed["value"], "wall_s": mixed["ms_step"] * 1e-3,
                        "kernel_ms_one_stream": float(mixed["class_ms"].sum()),
                        "mixed_tau64": args.mixed_tau64,
                        "mixed_p64": str(args.mixed_p64) if args.mixed_p64 == float("inf") else args.mixed_p64,
                        "fp32_fraction": mixed["stats"]["fp32_quartets"] / max(1, mixed["quartets"]),
                        "max_abs_err_vs_oracle": mixed["err_oracle"],
                        "max_abs_err_vs_fp64_gpu": mixed_err,
                        "speedup_vs_fp64": fp64["ms_step"] / mixed["ms_step"] if fp64 else None}
    if unb:
        rec["mixed_unbounded"] = {
            "note": "tau64 = inf: routed on class timing alone; the error is not bounded by the router",
            "value": unb["value"], "wall_s": unb["ms_step"] * 1e-3, "kernel_ms_one_stream": float(unb["class_ms"].sum()),
            "fp32_fraction": unb["stats"]["fp32_quartets"] / max(1, unb["quartets"]),
            "max_abs_err_vs_oracle": unb["err_oracle"],
            "speedup_vs_fp64": fp64["ms_step"] / unb["ms_step"] if fp64 else None}
    if not args.no_fock:
        rec["fock"] = run_fock()
    if args.copy_probe:
        src = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(mol, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
