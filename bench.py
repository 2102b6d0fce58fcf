#!/usr/bin/env python3
"""Throughput of the relativistic space-charge FMM on one MI355X.

A step is one whole evaluation of E and B at every particle of a resident
synthetic bunch (compute_fields with rebuild=1: mean Lorentz factor, k-d tree,
interaction lists, P2M/M2M, M2L, P2P, L2L/L2P).  Prints one JSON line.

Default workload: chirp1m, 1,048,576 particles uniform in an ellipsoid with
semi-axes (1, 1, 0.05) mm and a linear energy chirp u_z = 50 + 5 z/0.05 mm
(+ N(0, 0.5)), degree 8, leaves of 512, the mean-gamma kernel, at
eta = 0.45, the largest eta on a 0.05 grid whose FP64 FMM stays within 1e-6
of the FP64 direct sum for this bunch.  P2P runs in FP32; M2L in split BF16
(BF16x3: hi and lo parts of both operands, three BF16 matrix products with
FP32 accumulation), which keeps FP32-class accuracy and is the faster of the
two FP32-class M2L forms on MI355X (--m2l-prec fp32 selects the FP32 MFMA
form).  The accuracy of the
result is measured against the FP64 direct sum of the CPU oracle at 4,096
seeded targets (outside the timed region).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2302_07567_amd.workloads import SPECS as _SPECS  # noqa: E402

# method parameters per workload (degree, leaf, eta) used for the bench line:
# those of the workload definitions
BENCH = {k: {p: v[p] for p in ("degree", "leaf_size", "eta")}
         for k, v in _SPECS.items() if k != "cube"}

PEAK_FP32_VALU = 157.3e12  # MI355X FP32 vector FLOP/s (published)
PEAK_FP64_VALU = 78.6e12
# dense MFMA peaks by operand type (published)
PEAK_MFMA = {"fp32": 157.3e12, "fp64": 78.6e12, "bf16": 2.5e15,
             "bf16x3": 2.5e15}
# algorithmic flops of one pair-field evaluation (mean kernel): r (3),
# D = rx^2 + ry^2 + gbar^2 rz^2 (6), D^{-3/2} (3), (q gamma) D^{-3/2} (1),
# E += s r (6), (q u) x r (9), B += D^{-3/2} (q u x r) (6)
FLOPS_PAIR_MEAN = 34
FLOPS_PAIR_SOURCE = 40  # + u.r (5) and its square (1)
# one M2L entry (target proxy mu, source proxy nu): the kernel value
# D^{-3/2} with D = dx^2 + dy^2 + (gbar dz)^2 (3 sub, 1 mul + 2 FMA, rsqrt,
# 2 mul: 11 flops) and its products with the 10 weight columns (20 flops)
FLOPS_M2L_GEN = 11
FLOPS_M2L_MFMA = 20
FLOPS_M2L_ENTRY = FLOPS_M2L_GEN + FLOPS_M2L_MFMA
ACCURACY_BAR = 1e-6  # relative error vs the FP64 direct sum (eq. fmm_error)


# kernels whose HBM traffic was measured with rocprofv3 --pmc (FETCH_SIZE and
# WRITE_SIZE, scaled by the same counters read for a plain copy of known
# size); a summary is used only while the kernel's sources are unchanged
TRAFFIC_SOURCES = {"p2p": ("p2p.hip", "internal.hpp", "common.hpp"),
                   "m2l": ("m2l.hip", "internal.hpp", "common.hpp")}


def measured_traffic(kernel, workload, prec, m2l_prec, mode):
    """HBM bytes per launch from profiles/traffic_<kernel>_<workload>.txt,
    or None when there is none for this configuration or the kernel's
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles",
                        "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    want = {"p2p_prec": prec, "m2l_prec": m2l_prec, "kernel_mode": mode}
    if any(kv.get(k) != v for k, v in want.items()):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2302_07567_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def rel_err(a, b):
    den = float(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2) / den)) if den > 0 else 0.0


def fmm_err(E, B, Er, Br):
    eb = rel_err(B, Br) if np.any(Br != 0) else 0.0
    return max(rel_err(E, Er), eb)


# particles of the sub-bunch the serial oracle FMM is timed on (the same
# distribution and method parameters; the whole 1M bunch takes the serial
# oracle about ten minutes)
CPU_SAMPLE_N = 65536


def cpu_baseline(name, seed, params, w, targets):
    """The FP64 CPU oracle on this host.  (1) The serial FMM (one thread,
    like the paper's single-core comparison) timed on a sub-bunch of
    CPU_SAMPLE_N particles drawn from the same distribution with the same
    method parameters.  (2) The FP64 direct sum at the seeded sample targets
    of the full bunch with OpenMP over all host cores: the reference the
    GPU result's accuracy is measured against.  Returns the baseline record
    and the reference fields."""
    import oracle
    from paper_2302_07567_amd import workloads as W
    mode = oracle.MEAN if params.kernel == "mean" else oracle.EXACT
    all_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sub = W.make(name, seed=seed, n=min(CPU_SAMPLE_N, w.n))
    gb_sub = oracle.gamma_bar(sub.u)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.FMM(sub.x, sub.u, sub.q, params.degree, params.leaf_size,
               params.eta, gb_sub, mode).run()
    dt = time.perf_counter() - t0
    oracle.set_threads(all_threads)
    gb = oracle.gamma_bar(w.u)
    t1 = time.perf_counter()
    Ed, Bd = oracle.direct(w.x, w.u, w.q, gb, mode, targets=targets)
    dt_direct = time.perf_counter() - t1
    rec = {"value": sub.n / dt, "unit": "particles/s", "cores": 1,
           "kind": "oracle", "seconds": dt, "n": int(sub.n),
           "sample": "the serial FP64 oracle FMM (one thread) on a sub-bunch "
                     "of N=%d particles of the %s distribution with n=%d, "
                     "N0=%d, eta=%g (the full N=%d is the GPU workload)"
                     % (sub.n, name, params.degree, params.leaf_size,
                        params.eta, w.n),
           "direct_reference": {"targets": int(len(targets)), "n": int(w.n),
                                "seconds": dt_direct, "cores": all_threads,
                                "pairs_per_s": len(targets) * (w.n - 1) /
                                dt_direct}}
    return rec, (Ed, Bd)


def time_evaluations(plan, x, u, q, E, Bf, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.compute(x, u, q, E, Bf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(x, u, q, E, Bf)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def run_study(args):
    """The paper's studies on MI355X (Sec. 6): the accuracy/time sweep on
    1.28e6 particles uniform in [0,1]^3 with every momentum (0, 0,
    sqrt(gamma^2 - 1)), gamma = 50, eta in {0.3, 0.4, 0.5}, n in {2, 4, 6, 8,
    10}, N0 = (n+1)^3; and the scaling in N at n = 4, N0 = 125, eta = 0.5 up
    to 2.56e7 particles (both at and between the transition sizes
    N = 2^kappa N0).  Mono-energetic momenta make the mean and the
    per-source kernels identical.  Each line gives the time per whole
    evaluation (rebuild) and the error against the FP64 direct sum at 4,096
    sampled targets."""
    import torch
    from paper_2302_07567_amd import binding as B
    from paper_2302_07567_amd import workloads as W
    dev = torch.device("cuda:0")
    steps = max(1, min(args.steps, 5))
    warmup = max(1, min(args.warmup, 2))
    if args.study == "cube-sweep":
        n = args.study_n or 1280000
        grid = [(eta, deg) for eta in (0.3, 0.4, 0.5) for deg in (2, 4, 6, 8, 10)]
        precs = ("fp64", "fp32")
    else:
        top = args.study_n or 25600000
        sizes = []
        # transition sizes N_t = 2^kappa N0, just above them (leaves of about
        # N0 / 2 on one more level: the jump of the paper's work model, Sec. 7)
        # and midway
        k = 125 * 1024
        while k <= top:
            sizes += [k, k + k // 64, int(k * 1.5)]
            k *= 2
        sizes = [s for s in sizes if s <= top] + ([top] if top not in sizes else [])
        grid = [(0.5, 4, s) for s in sorted(set(sizes))]
        precs = ("fp32",)
    w_cache = {}
    for item in grid:
        if args.study == "cube-sweep":
            eta, deg = item
            N = n
        else:
            eta, deg, N = item
        if N not in w_cache:
            w_cache.clear()
            w = W.make("cube", seed=args.seed, n=N, degree=deg)
            x = torch.tensor(w.x, device=dev)
            u = torch.tensor(w.u, device=dev)
            q = torch.tensor(w.q, device=dev)
            tg = torch.tensor(w.sample, device=dev)
            w_cache[N] = (w, x, u, q, tg, {})
        w, x, u, q, tg, refs = w_cache[N]
        leaf = (deg + 1) ** 3
        for prec in precs:
            params = B.Params(degree=deg, leaf_size=leaf, eta=eta,
                              gamma_bar=0.0, kernel="mean", p2p_prec=prec,
                              m2l_prec=prec)
            plan = B.Plan(params, N, dev)
            E = torch.empty((N, 3), dtype=torch.float64, device=dev)
            Bf = torch.empty_like(E)
            dt = time_evaluations(plan, x, u, q, E, Bf, steps, warmup)
            st = plan.stats()
            plan.set_timing(True)
            plan.compute(x, u, q, E, Bf)
            phases = plan.timings()
            plan.set_timing(False)
            gb = st["gamma_bar"]
            if gb not in refs:
                refs[gb] = B.direct_fields(x, u, q, tg, kernel="mean",
                                           gamma_bar=gb)
            Ed, Bd = refs[gb]
            s = tg
            err = fmm_err(E[s].cpu().numpy(), Bf[s].cpu().numpy(),
                          Ed.cpu().numpy(), Bd.cpu().numpy())
            line = {"study": args.study, "n": N, "degree": deg,
                    "leaf_size": leaf, "eta": eta, "prec": prec,
                    "ms_per_step": 1e3 * dt, "value": N / dt,
                    "unit": "particles/s", "err_vs_direct_fp64": err,
                    "direct_targets": int(len(w.sample)), "depth": st["depth"],
                    "n_p2p_pairs": st["n_p2p_pairs"],
                    "n_m2l_pairs": st["n_m2l_pairs"],
                    "p2p_interactions": st["p2p_interactions"],
                    "m2l_entries": st["m2l_entries"],
                    "phases_ms": phases, "steps": steps, "data": "synthetic"}
            print(json.dumps(line), flush=True)
            del plan, E, Bf
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="chirp1m", choices=sorted(BENCH))
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--m2l-prec", default=None, choices=["fp32", "fp64", "bf16", "bf16x3"],
                    help="M2L precision (default: bf16x3 with --prec fp32, "
                         "fp64 with --prec fp64)")
    ap.add_argument("--kernel", default="mean", choices=["mean", "source"])
    ap.add_argument("--eta", type=float, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle (then the accuracy is measured "
                         "against the GPU's FP64 direct sum only)")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time forward + adjoint (default for adjoint262k)")
    ap.add_argument("--no-fp64-rate", action="store_true",
                    help="skip timing the plain FP64 GPU FMM beside the result")
    ap.add_argument("--study", default=None, choices=["cube-sweep", "scaling"],
                    help="instead of the benchmark line, print one JSON line "
                         "per configuration of the paper's accuracy/time sweep "
                         "on the uniform cube (cube-sweep) or of its scaling "
                         "study in N (scaling)")
    ap.add_argument("--study-n", type=int, default=0,
                    help="particles for --study cube-sweep (default 1.28e6) or "
                         "the largest N for --study scaling (default 2.56e7)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a resident buffer of MIB MiB 5 times (the "
                         "known-size kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU "
              "path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        src = torch.empty(args.copy_calibration << 20, dtype=torch.uint8,
                          device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel(), "copies": 5}), flush=True)
        return
    from paper_2302_07567_amd import binding as B
    from paper_2302_07567_amd import workloads as W

    if args.study:
        run_study(args)
        return

    spec = dict(BENCH[args.workload])
    if args.eta is not None:
        spec["eta"] = args.eta
    w = W.make(args.workload, seed=args.seed)
    dev = torch.device("cuda:0")
    x = torch.tensor(w.x, device=dev)
    u = torch.tensor(w.u, device=dev)
    q = torch.tensor(w.q, device=dev)
    m2l_prec = args.m2l_prec or ("bf16x3" if args.prec == "fp32" else "fp64")
    params = B.Params(degree=spec["degree"], leaf_size=spec["leaf_size"],
                      eta=spec["eta"], gamma_bar=0.0, kernel=args.kernel,
                      p2p_prec=args.prec, m2l_prec=m2l_prec)
    plan = B.Plan(params, w.n, dev)
    E = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    Bf = torch.empty_like(E)
    for _ in range(args.warmup):
        plan.compute(x, u, q, E, Bf)
    torch.cuda.synchronize()
    st = plan.stats()
    print("bench: %s n=%d warm, timing %d steps" % (args.workload, w.n,
                                                    args.steps),
          file=sys.stderr, flush=True)

    # timed region: K whole evaluations, bracketed by synchronizations; the
    # plan records HIP events on its stream (the stream every kernel is
    # launched on) at each phase boundary of every call, read afterwards
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.compute(x, u, q, E, Bf)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    phases, ncalls = plan.timing_means()
    plan.set_timing(False)
    assert ncalls == args.steps

    n = w.n
    fl_pair = FLOPS_PAIR_MEAN if args.kernel == "mean" else FLOPS_PAIR_SOURCE
    p2p_units = st["p2p_interactions"] - n  # ordered pairs j != i
    m2l_units = st["m2l_entries"]
    # both kernels are bound by vector ALU issue: P2P by its pair arithmetic,
    # M2L (every tier but FP64) by generating the kernel matrix Phi in FP32
    # on the VALU, which on gfx950 does not overlap the matrix cores; the
    # contraction's own matrix-core fraction is reported beside it
    roof = {}
    for name, units, fl, pr in (("p2p", p2p_units, fl_pair, args.prec),
                                ("m2l", m2l_units, FLOPS_M2L_ENTRY, m2l_prec)):
        peak = PEAK_FP64_VALU if pr == "fp64" else PEAK_FP32_VALU
        t = phases[name] * 1e-3
        ach = units * fl / t if t > 0 else 0.0
        tr = measured_traffic(name, args.workload, args.prec, m2l_prec,
                              args.kernel)
        roof[name] = {"bound": "alu", "achieved": ach / 1e12,
                      "peak": peak / 1e12, "unit": "TFLOP/s",
                      "frac": ach / peak, "traffic": tr,
                      "units": int(units), "flops_per_unit": fl,
                      "ms": phases[name]}
    # M2L's contraction on the matrix cores, against the dense peak of its
    # operand type (useful flops: 2 x 10 weight columns per entry)
    t = phases["m2l"] * 1e-3
    mf = m2l_units * FLOPS_M2L_MFMA / t if t > 0 else 0.0
    roof["m2l"]["mfma"] = {"achieved": mf / 1e12,
                           "peak": PEAK_MFMA[m2l_prec] / 1e12,
                           "unit": "TFLOP/s",
                           "frac": mf / PEAK_MFMA[m2l_prec],
                           "flops_per_unit": FLOPS_M2L_MFMA}
    dom = max(("p2p", "m2l"), key=lambda k: phases[k])
    roofline = {k: v for k, v in roof[dom].items() if k != "mfma"}
    roofline["kernel"] = dom

    # forward + adjoint (a training step): fields with rebuild, then the
    # gradient of sum_i w_i (E_i.a_i + B_i.b_i) with the structure frozen
    adj = None
    if args.adjoint or args.workload == "adjoint262k":
        rng = np.random.default_rng(args.seed + 1)
        ex = w.extra if "w" in w.extra else {
            "w": rng.standard_normal(n), "a": rng.standard_normal((n, 3)),
            "b": rng.standard_normal((n, 3))}
        gE = torch.tensor(ex["w"][:, None] * ex["a"], device=dev)
        gB = torch.tensor(ex["w"][:, None] * ex["b"], device=dev)
        gx = torch.empty((n, 3), dtype=torch.float64, device=dev)
        gq = torch.empty((n,), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            plan.compute(x, u, q, E, Bf)
            plan.adjoint(x, u, q, gE, gB, gx, gq, rebuild=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.compute(x, u, q, E, Bf)
            plan.adjoint(x, u, q, gE, gB, gx, gq, rebuild=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # the same step with the momentum gradient as well
        gu = torch.empty((n, 3), dtype=torch.float64, device=dev)
        plan.compute(x, u, q, E, Bf)
        plan.adjoint(x, u, q, gE, gB, gx, gq, rebuild=False, with_u=True,
                     grad_u=gu)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.compute(x, u, q, E, Bf)
            plan.adjoint(x, u, q, gE, gB, gx, gq, rebuild=False, with_u=True,
                         grad_u=gu)
        torch.cuda.synchronize()
        el_u = time.perf_counter() - t0
        adj = {"value": n * args.steps / el, "unit": "particles/s",
               "ms_per_step": 1e3 * el / args.steps,
               "step": "compute_fields(rebuild=1) + adjoint(rebuild=0)",
               "loss": "sum_i w_i (E_i.a_i + B_i.b_i), w, a, b ~ N(0, 1)",
               "ms_per_step_with_grad_u": 1e3 * el_u / args.steps}

    # the plain FP64 GPU FMM on the same bunch, same structure parameters
    fp64_rate = None
    E64n = B64n = None
    if args.prec != "fp64" and not (args.no_fp64_rate and args.no_accuracy):
        p64 = B.Params(degree=spec["degree"], leaf_size=spec["leaf_size"],
                       eta=spec["eta"], gamma_bar=0.0, kernel=args.kernel,
                       p2p_prec="fp64", m2l_prec="fp64")
        plan64 = B.Plan(p64, n, dev)
        E64t = torch.empty_like(E)
        B64t = torch.empty_like(E)
        plan64.compute(x, u, q, E64t, B64t)
        torch.cuda.synchronize()
        if not args.no_fp64_rate:
            k64 = max(1, min(args.steps, 5))
            t0 = time.perf_counter()
            for _ in range(k64):
                plan64.compute(x, u, q, E64t, B64t)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            fp64_rate = {"value": n * k64 / el, "unit": "particles/s",
                         "ms_per_step": 1e3 * el / k64, "steps": k64,
                         "speedup_of_result": (n * args.steps / elapsed) /
                                              (n * k64 / el)}
        E64n, B64n = E64t.cpu().numpy(), B64t.cpu().numpy()
        del plan64, E64t, B64t

    s = w.sample
    cpu = ref = None
    if not args.no_cpu_baseline:
        print("bench: CPU oracle (serial FMM sample, direct-sum reference)",
              file=sys.stderr, flush=True)
        cpu, ref = cpu_baseline(args.workload, args.seed, params, w, s)

    acc = None
    if not args.no_accuracy:
        gb = st["gamma_bar"]
        tg = torch.tensor(s, device=dev)
        Ed, Bd = B.direct_fields(x, u, q, tg, kernel=args.kernel, gamma_bar=gb)
        torch.cuda.synchronize()
        En, Bn = E.cpu().numpy(), Bf.cpu().numpy()
        Edn, Bdn = Ed.cpu().numpy(), Bd.cpu().numpy()
        acc = {"direct_targets": int(len(s)), "reference_kernel": args.kernel,
               "err_vs_direct_fp64_gpu": fmm_err(En[s], Bn[s], Edn, Bdn)}
        if E64n is not None:
            acc["err_vs_fmm_fp64"] = fmm_err(En, Bn, E64n, B64n)
        if ref is not None:
            Eo, Bo = ref
            acc["err_vs_direct_fp64"] = fmm_err(En[s], Bn[s], Eo, Bo)
            acc["reference"] = "CPU oracle FP64 direct sum"
            acc["gpu_direct_vs_oracle_direct"] = fmm_err(Edn, Bdn, Eo, Bo)
            if E64n is not None:
                acc["err_fmm_fp64_vs_direct_fp64"] = fmm_err(E64n[s], B64n[s],
                                                             Eo, Bo)
        else:
            acc["err_vs_direct_fp64"] = acc["err_vs_direct_fp64_gpu"]
            acc["reference"] = "GPU FP64 direct sum"
        acc["bar"] = ACCURACY_BAR
        acc["meets_bar"] = bool(acc["err_vs_direct_fp64"] <= ACCURACY_BAR)
        if not acc["meets_bar"]:
            print("bench: WARNING relative error %.3e exceeds %.0e"
                  % (acc["err_vs_direct_fp64"], ACCURACY_BAR), file=sys.stderr,
                  flush=True)

    line = {
        "metric": "particles/sec (E+B) at rel. err <=1e-6 vs FP64 direct sum; "
                  "FP32/BF16 vs FP64 FMM",
        "value": n * args.steps / elapsed,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec if m2l_prec in (args.prec, "fp32") else
                 "%s+%s" % (args.prec, m2l_prec),
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "degree": spec["degree"],
                   "leaf_size": spec["leaf_size"], "eta": spec["eta"],
                   "kernel": args.kernel, "p2p_prec": args.prec,
                   "m2l_prec": m2l_prec, "seed": args.seed,
                   "gamma_bar": st["gamma_bar"], "depth": st["depth"],
                   "n_p2p_pairs": st["n_p2p_pairs"],
                   "n_m2l_pairs": st["n_m2l_pairs"]},
        "roofline": roofline,
        "roofline_all": roof,
        "phases_ms": phases,
        "accuracy": acc,
        "fp64_fmm": fp64_rate,
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
