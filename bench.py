"""Benchmark: fast-diagonalization preconditioner applies per second (in unknowns
per second) and GMRES solve time to 1e-8, FP64 vs mixed precision, on the 3D
unit-cube workload (p = 3, 64 elements per direction, 65^3 x 66 = 18,125,250
unknowns), one GPU.

A timed step is one application s = A-hat^{-1} r of the FP64 preconditioner to
one resident FP64 tensor (forward spatial transforms, shifted time solves, back
transforms).  The JSON line also reports the FP32 / BF16 applies, the GMRES /
flexible GMRES solves with their iteration counts, true residuals and errors
against the CPU oracle's solution, the event-timed roofline of the dominant
kernel, and the CPU oracle's throughput on the host (baseline only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 (vector and matrix, dense)
BF16_PEAK_TFLOPS = 2500.0    # MI355X BF16 MFMA, dense


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, f_host, target_s=12.0):
    """The oracle's FD apply (numpy/scipy FP64) on the full tensor, repeated ~target_s."""
    from threadpoolctl import threadpool_info

    from oracle import fd
    from oracle.problems import CubeProblem
    pr = CubeProblem(w)
    P = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt, w.gamma, w.nu)
    reps, t0 = 0, time.perf_counter()
    u = None
    while True:
        u = P.apply(f_host)
        reps += 1
        if time.perf_counter() - t0 >= target_s or reps >= 8:
            break
    dt = (time.perf_counter() - t0) / reps
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return u, {"value": w.N / dt, "unit": "DoF/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{reps} full FP64 applies of A-hat^-1 on the {w.N}-unknown tensor "
                         f"(numpy/scipy, BLAS threads={threads}, nproc={os.cpu_count()})",
               "s_per_apply": dt}


def cpu_baseline_more():
    """The oracle on the other workloads' unit of work (baseline only): the 48-element cube
    (one right-hand side: the FD apply, and the solve = that apply, since A-hat = A, plus the
    residual product that checks it) and the quarter annulus at 128 elements (the
    geometry-aware FD apply and the factored matvec of Section 4.5)."""
    from threadpoolctl import threadpool_info

    import workloads as wl
    from oracle import fd
    from oracle.annulus import AnnulusProblem
    from oracle.problems import CubeProblem
    threads = int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))

    def timed(fn, reps=3):
        fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps

    out = {}
    wb = wl.WORKLOADS["cube_p3_n48_b32"]
    pr = CubeProblem(wb)
    P = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt)
    x = wl.random_tensor(wb.shape, 6)
    ta = timed(lambda: P.apply(x))
    tm = timed(lambda: fd.kron_matvec(x, pr.Wt, pr.Mt, pr.K1d, pr.M1d))
    out["cube_p3_n48_apply"] = {"value": wb.N / ta, "unit": "DoF/s", "cores": threads,
                                "kind": "oracle", "s_per_apply": ta,
                                "sample": f"3 FP64 applies of A-hat^-1, {wb.N} unknowns (one "
                                          "right-hand side of the batch)"}
    out["cube_p3_n48_solve"] = {"value": wb.N / (ta + tm), "unit": "DoF/s", "cores": threads,
                                "kind": "oracle", "s_per_solve": ta + tm,
                                "sample": "one right-hand side: u = A-hat^-1 f (= A^-1 f) and "
                                          "the residual product f - A u"}
    wa = wl.WORKLOADS["annulus_p4_n128"]
    o = AnnulusProblem(wa)
    Pa = o.preconditioner()
    xa = wl.random_tensor(wa.shape, 5)
    ta = timed(lambda: Pa.apply(xa))
    tm = timed(lambda: o.matvec(xa))
    out["annulus_p4_n128_apply"] = {"value": wa.N / ta, "unit": "DoF/s", "cores": threads,
                                    "kind": "oracle", "s_per_apply": ta,
                                    "sample": f"3 FP64 applies of (A-hat^G)^-1, {wa.N} unknowns"}
    out["annulus_p4_n128_factored_matvec"] = {
        "value": wa.N / tm, "unit": "DoF/s", "cores": threads, "kind": "oracle",
        "s_per_matvec": tm, "sample": "3 products W_t (x) M_s + M_t' (x) K_s with scipy CSR "
                                      "spatial factors"}
    return out


def kernel_breakdown(prof, steps, N, flops_per_dof, peak_tflops=FP64_PEAK_TFLOPS):
    """Per kernel class: mean launch time (HIP events), algorithmic bytes and flops per
    launch, achieved rates, and the bound (the larger of the two time floors at peak)."""
    kernels = {}
    total = sum(x[0] for x in prof.values())
    for k, v in prof.items():
        if not v[2]:
            continue
        ms_l, by_l = v[0] / v[2], v[1] / v[2]
        fl_l = flops_per_dof.get(k, 0) * N
        t_hbm, t_mfma = by_l / (HBM_PEAK_GBS * 1e9), fl_l / (peak_tflops * 1e12)
        kernels[k] = {"ms_per_launch": ms_l, "launches_per_step": v[2] / steps,
                      "share": v[0] / total, "bytes_per_launch": by_l, "flops_per_launch": fl_l,
                      "GBps": by_l / (ms_l * 1e-3) / 1e9,
                      "TFLOPs": fl_l / (ms_l * 1e-3) / 1e12,
                      "bound": "mfma" if t_mfma > t_hbm else "hbm"}
    return kernels


def roofline_of(kernels, traffic=None, peak_tflops=FP64_PEAK_TFLOPS):
    """The roofline object of the dominant kernel class (largest share of event time)."""
    dom = max(kernels, key=lambda k: kernels[k]["share"])
    kd = kernels[dom]
    if kd["bound"] == "mfma":
        return {"kernel": dom, "bound": "mfma", "achieved": kd["TFLOPs"], "peak": peak_tflops,
                "unit": "TFLOP/s", "frac": kd["TFLOPs"] / peak_tflops, "traffic": traffic,
                "flops_per_launch": kd["flops_per_launch"],
                "bytes_per_launch": kd["bytes_per_launch"], "ms_per_launch": kd["ms_per_launch"],
                "hbm_GBps": kd["GBps"]}
    return {"kernel": dom, "bound": "hbm", "achieved": kd["GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": kd["GBps"] / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": kd["bytes_per_launch"], "ms_per_launch": kd["ms_per_launch"]}


def apply_floor_ms(N, flops_per_dof, prec):
    """Time floor of one whole apply: the larger of its algorithmic flops at the precision's
    peak and its compulsory 16 bytes per unknown (FP64 in and out) at HBM peak."""
    peak = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS, "bf16": BF16_PEAK_TFLOPS}[prec]
    t_mfma = flops_per_dof * N / (peak * 1e12) * 1e3
    t_hbm = 16.0 * N / (HBM_PEAK_GBS * 1e9) * 1e3
    return (t_mfma, "mfma") if t_mfma >= t_hbm else (t_hbm, "hbm")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fd_apply_cube_p3_n64.json")
KERNEL_SOURCES = ["paper_1909_07309_amd/csrc/" + f for f in (
    "kernels_fd.h", "kernels_plane.h", "kernels_sym.h", "kernels_plane_sym.h", "kernels_arrow.h",
    "kernels_matvec.h", "kernels_krylov.h", "stig.hip")]


def kernel_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def summarize_counters(fetch_csv, write_csv, copy_bytes):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
    `bench.py --calibration-copy` into per-kernel HBM bytes per launch, scaled by
    what the counters read for the calibration copy of known size."""
    import csv
    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "")
            acc.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)
        return acc
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k or "elementwise" in k]
    # calibration: the largest copy dispatch moves copy_bytes in and copy_bytes out
    cf = max(max(fetch[k]) for k in copy) / copy_bytes
    cw = max(max(write[k]) for k in copy) / copy_bytes
    out = {"fingerprint": kernel_fingerprint(), "copy_bytes": copy_bytes,
           "fetch_scale": cf, "write_scale": cw, "kernels": {}}
    for k in fetch:
        if k in copy or k not in write:
            continue
        f = sum(fetch[k]) / len(fetch[k]) / cf
        w = sum(write[k]) / len(write[k]) / cw
        out["kernels"][k] = {"fetch_bytes": f, "write_bytes": w, "dispatches": len(fetch[k])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-annulus", action="store_true",
                    help="skip the 2D and 3D annulus solves (variable coefficients; CSR and "
                         "factored matvec)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the batched forward + adjoint solve (32 right-hand sides)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-kernel HBM traffic file from two --pmc runs and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        out = summarize_counters(*args.summarize_counters, copy_bytes=float(1 << 30))
        json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
        print(json.dumps(out, indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import workloads as wl
    from paper_1909_07309_amd.problem import CubeFactors, source

    w = wl.WORKLOADS["cube_p3_n64"]
    log(f"[bench] workload {w.name}: N = {w.N}")
    t0 = time.perf_counter()
    fac = CubeFactors(w)
    plan = fac.make_plan()
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3   # host assembly, 1D eigenproblems, uploads
    f = source(w, plan)
    torch.cuda.synchronize()
    s = torch.empty_like(f)
    if args.calibration_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def timed_applies(prec, steps, warmup, profile=False):
        for _ in range(warmup):
            plan.apply_Pinv(f, s, prec=prec)
        torch.cuda.synchronize()
        if profile:
            plan.profile_reset()
            plan.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.apply_Pinv(f, s, prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if profile:
            prof = plan.profile()
            plan.profile_enable(False)
        return dt, prof

    # ---- FP64 apply: the headline, timed without per-kernel events; then the
    # same number of applies again with an event pair around every launch for
    # the per-kernel breakdown and the roofline of the dominant kernel
    dt, _ = timed_applies("fp64", args.steps, args.warmup)
    ms_per_step = dt / args.steps * 1e3
    value = w.N * args.steps / dt
    log(f"[bench] fp64 apply {ms_per_step:.3f} ms  {value:.3e} DoF/s")
    _, prof = timed_applies("fp64", args.steps, 1, profile=True)
    # algorithmic FP64 flops per unknown of one launch of each kernel class:
    # a mode product is a length-n dot product per output (2n), the fused
    # plane kernel does two of them (4n); the banded solve is counted as the
    # elimination with precomputed factors (4 p_t + 1, negligible: HBM-bound)
    flops_per_dof = {"mode_gemm": 2 * w.n_s, "plane_gemm": 4 * w.n_s, "time_solve": 4 * w.p + 1}
    kernels = kernel_breakdown(prof, args.steps, w.N, flops_per_dof)
    dom = max(kernels, key=lambda k: kernels[k]["share"])
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("fingerprint") == kernel_fingerprint():
            # the dominant class's FP64 kernels at this workload (forward and
            # backward variants), bytes per launch averaged over their dispatches
            prefixes = {"mode_gemm": ("stig::mode_gemm_sym<double, double, double",
                                      "stig::mode_gemm_small<double, double, double"),
                        "plane_gemm": ("stig::mode_gemm_plane_sym<double, double, double",
                                       "stig::mode_gemm_plane<double, double, double"),
                        "time_solve": ("stig::time_band_solve_rl<double, double",)}.get(dom, ())
            for pre in prefixes:
                ks = [v for k, v in t["kernels"].items() if k.startswith(pre)]
                if ks:
                    nd = sum(v["dispatches"] for v in ks)
                    traffic = sum((v["fetch_bytes"] + v["write_bytes"]) * v["dispatches"]
                                  for v in ks) / nd
                    break
    roofline = roofline_of(kernels, traffic)
    # whole-apply view: FP64 flops 4*d*n_s per unknown for the transforms (+ time solves)
    apply_fpd = 4 * w.d * w.n_s + 4 * w.p + 1
    flops = apply_fpd * w.N
    apply_tflops = flops / (ms_per_step * 1e-3) / 1e12

    # ---- mixed-precision applies, and each precision's whole apply against its floor
    mixed = {}
    for prec in ("fp32", "bf16"):
        dtp, _ = timed_applies(prec, args.steps, args.warmup)
        mixed[prec] = {"ms_per_apply": dtp / args.steps * 1e3, "DoF_per_s": w.N * args.steps / dtp}
        log(f"[bench] {prec} apply {mixed[prec]['ms_per_apply']:.3f} ms")
    apply_roofline = {}
    for prec, ms in (("fp64", ms_per_step), ("fp32", mixed["fp32"]["ms_per_apply"]),
                     ("bf16", mixed["bf16"]["ms_per_apply"])):
        floor, bound = apply_floor_ms(w.N, apply_fpd, prec)
        apply_roofline[prec] = {"ms": ms, "floor_ms": floor, "bound": bound, "frac": floor / ms}

    # ---- FP64 matvec y = A x (the per-iteration product of the solves)
    for _ in range(args.warmup):
        plan.matvec_A(f, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.matvec_A(f, s)
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - t0) / args.steps
    matvec = {"ms": dtm * 1e3, "DoF_per_s": w.N / dtm}
    log(f"[bench] fp64 matvec {dtm * 1e3:.3f} ms")

    # ---- CPU oracle baseline (also the reference solution: A-hat = A on the cube),
    # on all host threads, then one apply on one thread (beside the paper's serial timings)
    cpu = None
    cpu1 = None
    cpu_more = None
    u_ref = None
    if not args.no_cpu_baseline:
        f_host = f.cpu().numpy()
        u_ref, cpu = cpu_baseline(w, f_host)
        log(f"[bench] cpu oracle {cpu['s_per_apply']:.2f} s/apply ({cpu['cores']} threads)")
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            _, cpu1 = cpu_baseline(w, f_host, target_s=0.0)
        cpu1["cores"] = 1
        cpu1["sample"] = f"one full FP64 apply of A-hat^-1 on the {w.N}-unknown tensor, one thread"
        log(f"[bench] cpu oracle, one thread: {cpu1['s_per_apply']:.2f} s/apply")
        cpu_more = cpu_baseline_more()
        log(f"[bench] cpu oracle, other workloads: {cpu_more}")

    # ---- solves to 1e-8
    solves = {}
    if not args.no_solve:
        for prec in ("fp64", "fp32", "bf16"):
            flexible = prec != "fp64"
            u0 = torch.zeros_like(f)
            plan.gmres_solve(f, u0, restart=w.restart, rtol=w.rtol, maxit=w.maxit,
                             flexible=flexible, prec=prec)  # warm (allocations)
            u = torch.zeros_like(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, info = plan.gmres_solve(f, u, restart=w.restart, rtol=w.rtol, maxit=w.maxit,
                                       flexible=flexible, prec=prec)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) * 1e3
            rec = {"ms": t, "iters": info["iters"], "relres_true": info["relres_true"],
                   "method": "FGMRES(30)" if flexible else "GMRES(30)"}
            if u_ref is not None:
                uh = u.cpu().numpy()
                rec["rel_err_vs_oracle"] = float(np.linalg.norm(uh - u_ref) / np.linalg.norm(u_ref))
            solves[prec] = rec
            log(f"[bench] solve {prec}: {rec}")

    # ---- annulus (2D) and extruded annulus (3D): A-hat^G != A, FGMRES(30) to 1e-8
    # with the FP64 and with the FP32 geometry-aware FD preconditioner, for both
    # forms of A x: the whole space-time matrix as a CSR ("csr") and only the
    # sparse spatial factors and the time bands ("factored", Section 4.5)
    def annulus_runs(setup, w, timed_apply):
        out = {"N": w.N}
        for form in ("csr", "factored"):
            t0 = time.perf_counter()
            pl = setup.make_plan(matvec=form)
            torch.cuda.synchronize()
            rec = {"setup_ms": (time.perf_counter() - t0) * 1e3,
                   "plan_device_GB": pl.device_bytes() / 1e9}
            if form == "csr":
                rec["plan_device_GB"] += sum(t.numel() * t.element_size()
                                             for t in pl._keep["csr"]) / 1e9
            f = setup.source()
            y = torch.empty_like(f)
            for _ in range(2):
                pl.matvec_A(f, y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                pl.matvec_A(f, y)
            torch.cuda.synchronize()
            rec["matvec_ms"] = (time.perf_counter() - t0) / 10 * 1e3
            for prec in ("fp64", "fp32"):
                r = {}
                if timed_apply:
                    s_ = torch.empty_like(f)
                    for _ in range(3):
                        pl.apply_Pinv(f, s_, prec=prec)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(args.steps):
                        pl.apply_Pinv(f, s_, prec=prec)
                    torch.cuda.synchronize()
                    r["apply_ms"] = (time.perf_counter() - t0) / args.steps * 1e3
                    r["apply_DoF_per_s"] = w.N / (r["apply_ms"] * 1e-3)
                    if prec == "fp64" and form == "factored":
                        # per-kernel event times of the same applies, and the
                        # roofline of the dominant kernel class
                        pl.profile_reset()
                        pl.profile_enable(True)
                        for _ in range(args.steps):
                            pl.apply_Pinv(f, s_, prec=prec)
                        prof = pl.profile()
                        pl.profile_enable(False)
                        n = w.n_s
                        kern = kernel_breakdown(prof, args.steps, w.N,
                                                {"mode_gemm": 2 * n, "plane_gemm": 4 * n,
                                                 "time_solve": 4 * w.p + 1})
                        r["kernels"] = kern
                        r["roofline"] = roofline_of(kern)
                        floor, bound = apply_floor_ms(w.N, 4 * w.d * n + 4 * w.p + 1, "fp64")
                        r["apply_roofline"] = {"floor_ms": floor, "bound": bound,
                                               "frac": floor / r["apply_ms"]}
                pl.gmres_solve(f, torch.zeros_like(f), restart=30, rtol=1e-8, maxit=300,
                               flexible=True, prec=prec)  # warm (allocations)
                u = torch.zeros_like(f)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, info = pl.gmres_solve(f, u, restart=30, rtol=1e-8, maxit=300, flexible=True,
                                         prec=prec)
                torch.cuda.synchronize()
                r.update({"ms": (time.perf_counter() - t0) * 1e3, "iters": info["iters"],
                          "relres_true": info["relres_true"], "method": "FGMRES(30)"})
                rec[prec] = r
            out[form] = rec
            log(f"[bench] {w.name} {form}: {rec}")
            del pl, f, y
            torch.cuda.empty_cache()
        return out

    annulus, annulus3d = {}, {}
    if not args.no_solve and not args.no_annulus:
        from paper_1909_07309_amd.annulus import AnnulusSetup
        from paper_1909_07309_amd.annulus3d import Annulus3DSetup
        wa = wl.WORKLOADS["annulus_p4_n128"]
        t0 = time.perf_counter()
        a2 = AnnulusSetup(wa)
        host_ms = (time.perf_counter() - t0) * 1e3
        annulus = annulus_runs(a2, wa, True)
        annulus["host_setup_ms"] = host_ms
        del a2
        w3 = wl.WORKLOADS["annulus3d_p2_n32"]
        t0 = time.perf_counter()
        a3 = Annulus3DSetup(w3)
        host_ms = (time.perf_counter() - t0) * 1e3
        annulus3d = annulus_runs(a3, w3, True)
        annulus3d["host_setup_ms"] = host_ms
        del a3

    # ---- batched forward + adjoint solve (p=3, 48 elements, 32 right-hand sides):
    # u = A^{-1}(f - A_I0 c0), loss 0.5 ||u - u*||^2, gradients w.r.t. f and c0
    adjoint = {}
    if not args.no_solve and not args.no_adjoint:
        from paper_1909_07309_amd.autograd import solve as stig_solve
        from paper_1909_07309_amd.problem import smoothed_source

        wb = wl.WORKLOADS["cube_p3_n48_b32"]
        facb = CubeFactors(wb)
        planb = facb.make_plan()
        fb = smoothed_source(planb, torch.from_numpy(wl.source_coefficients(wb)).cuda()).detach()
        c0 = torch.zeros((wb.nrhs,) + (wb.n_s,) * wb.d, dtype=torch.float64, device="cuda")
        tgt = torch.from_numpy(wl.adjoint_target(wb)).cuda()
        opts = dict(rtol=wb.rtol, restart=wb.restart, maxit=wb.maxit)
        cols = (facb.W_col0, facb.M_col0)
        times = []
        for rep_ in range(2):   # the first pass allocates the Krylov buffers
            ft = fb.clone().requires_grad_(True)
            ct = c0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u = stig_solve(planb, ft, ct, cols, **opts)
            loss = 0.5 * ((u - tgt) ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3))
        adjoint = {"forward_ms": times[-1][0], "backward_ms": times[-1][1], "nrhs": wb.nrhs,
                   "N_per_rhs": wb.N, "rtol": wb.rtol,
                   "DoF_per_s": wb.N * wb.nrhs * 2 / ((times[-1][0] + times[-1][1]) * 1e-3)}
        log(f"[bench] adjoint batch: {adjoint}")
        del planb, fb, u, ft, ct

    line = {
        "metric": "P^-1 applies/s (DoF/s) + solve time to 1e-8 resid, FP64 vs mixed",
        "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "unit cube x [0,1], p=3, 64 elements/direction, "
                               "65^3 x 66 = 18,125,250 unknowns, one FP64 A-hat^-1 apply per step",
                   "N": w.N, "d": w.d, "p": w.p, "n_el": w.n_el, "parallelism": "single GPU"},
        "roofline": roofline,
        "apply_roofline": apply_roofline,
        "apply_fp64_tflops": apply_tflops,
        "kernels_fp64_apply": kernels,
        "mixed_apply": mixed,
        "matvec_fp64": matvec,
        "solve_to_1e-8": solves,
        "annulus_solve_to_1e-8": annulus,
        "annulus3d_solve_to_1e-8": annulus3d,
        "adjoint_batch": adjoint,
        "setup_ms": setup_ms,
        "cpu_baseline": None if cpu is None else {k: v for k, v in cpu.items()
                                                  if k != "s_per_apply"},
        "cpu_baseline_1thread": None if cpu1 is None else {k: v for k, v in cpu1.items()
                                                           if k != "s_per_apply"},
        "cpu_baseline_other_workloads": cpu_more,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
