"""Benchmark of the FLOSIC SIC hot path on one MI355X.

One step = one pass of the whole path over the workload: Fermi orbitals,
Loewdin, the Poisson problems of every FLO density (with its multipole
boundary values: the Hartree potential), LSDA, Slater-averaged V_SIC and
E_SIC (forward), then the FOD gradient (the adjoint Poisson problem of every
orbital, with zero boundary values, and reverse mode through Loewdin and the
interpolation).  The library solves the zero-boundary problems by CG in the
forward pass and forms the multipole-boundary solutions from them and a
per-grid basis of unit-moment boundary solutions (solved once per grid, in
the warm-up); so a step answers 2 N Poisson problems with N CG solves.  The
headline value is orbital Poisson problems answered per second of the
mixed-precision path (FP32 CG sweeps recovered to the FP64 tolerance); CG
solves per second and the step time are reported beside it, and the plain
FP64 path is timed on the same inputs.

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mol96")
    ap.add_argument("--tol", type=float, default=1e-11,
                    help="relative FP64 residual of every solve (1e-11 keeps E_SIC within 1e-8 Ha "
                         "on every workload here)")
    ap.add_argument("--solver", default="pcg", choices=["pcg", "cg"],
                    help="pcg: CG with the sine-transform preconditioner; cg: plain CG")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="skip the unprofiled eager and graph-replay legs")
    ap.add_argument("--no-aar", action="store_true",
                    help="skip the FP64 alternating Anderson-Richardson leg")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle solving in the CPU-baseline sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


def run_steps(F, torch, ctx, dicts, noccs, steps):
    """Timed region: `steps` full passes (forward + backward, one library
    call each) over all systems."""
    keys = ("sweep_ms", "sweep_bytes", "sweep_launches", "update_ms", "update_bytes",
            "update_launches", "precond_ms", "precond_bytes", "precond_flops", "precond_launches",
            "resid_ms", "resid_bytes", "resid_launches")
    agg = dict({k: 0.0 for k in keys}, iters=0, solves=0, krylov=0, basis_solves=0, refinements=0, max_relres=0.0,
               phase_ms=[0.0] * 8)
    e = g = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, U, X, g, st, stb = ctx.forward_backward(dicts)
        agg["shape"] = {"tile": f"32x{8 * st['stencil_cpt']}", "prefetch_planes": st["stencil_depth"],
                        "block_target": st["stencil_blocks"]}
        lay = st["precond_layout"]
        agg["precond_layout"] = {"variant": lay >> 4, "fused_xy": bool(lay & 1),
                                 "xy_two_blocks_per_cu": bool(lay & 2), "z_two_blocks_per_cu": bool(lay & 4),
                                 "early_p_old": bool(lay & 8)}
        for part in (st, stb):
            for k in keys:
                agg[k] += part[k]
            agg["iters"] += part["total_iters"]
            agg["solves"] += part["npoisson"]
            agg["krylov"] += part["nsolves"]
            agg["basis_solves"] += part["basis_solves"]
            agg["refinements"] += part["outer_refinements"]
            agg["max_relres"] = max(agg["max_relres"], part["max_relres"])
        for q in (0, 1, 2, 3, 4):
            agg["phase_ms"][q] += st["ms_phase"][q] / steps
        for q in (5, 6):
            agg["phase_ms"][q] += stb["ms_phase"][q] / steps
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, e, g, agg


def cpu_baseline(sysobj, tol, budget_s):
    """The oracle as it stands on the host cores, on a bounded sample of the
    same workload: the Fermi-Loewdin orbitals of each spin channel, then the
    FLO-density Poisson solves in order (spin up first) until about
    `budget_s` seconds of solving have passed (at least one solve)."""
    import numpy as np
    from oracle import oracle

    def host(a):
        return np.asarray(a.cpu().numpy() if hasattr(a, "cpu") else a)

    t_flo, t_solve, iters, done = 0.0, 0.0, [], 0
    for s in range(sysobj.nspin):
        if done > 0 and t_solve >= budget_s:
            break
        t0 = time.perf_counter()
        phi, _, _, _ = oracle.flo_spin(host(sysobj.psi[s]), host(sysobj.fod[s]), sysobj.n,
                                       sysobj.h, sysobj.origin)
        t_flo += time.perf_counter() - t0
        for i in range(phi.shape[0]):
            if done > 0 and t_solve >= budget_s:
                break
            t1 = time.perf_counter()
            _, it, _ = oracle.poisson(phi[i] ** 2, sysobj.n, sysobj.h, sysobj.origin, tol=tol)
            t_solve += time.perf_counter() - t1
            iters.append(it)
            done += 1
    out = {"value": done / t_solve, "unit": "solves/s", "cores": oracle.num_threads(),
           "kind": "oracle",
            "sample": f"{done} of the {sum(sysobj.nocc)} forward FLO-density Poisson solves of the "
                      f"{sysobj.name} workload (FP64 CG to relative residual {tol:g}, "
                      f"{int(np.mean(iters))} iterations on average, {t_solve:.1f} s; the Fermi-"
                      f"Loewdin steps before them took {t_flo:.1f} s and are not in the rate), "
                      f"OpenMP over the host cores",
           "cpu_model": host_cpu_model()}
    out["single_thread_small_case"] = single_thread_small_case()
    return out


def host_cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


_SMALL_CASE = r'''
import json, time
from oracle import oracle
from paper_2108_01186_amd import synth
oracle.set_num_threads(1)
s = synth.make_workload("mol40")
t0 = time.perf_counter()
r = oracle.sic_spin(s.psi[0], s.fod[0], s.n, s.h, s.origin, tol=1e-10)
t = time.perf_counter() - t0
print(json.dumps({"seconds": t, "threads": oracle.num_threads(), "E_SIC": float(r.e)}))
'''


def single_thread_small_case():
    """The oracle on the 40^3 one-channel case (5 orbitals, CG to 1e-10:
    Fermi-Loewdin orbitals, their Poisson solves, LSDA, E_SIC and V_SIC) with
    one OpenMP thread, in a child process that touches no GPU."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", _SMALL_CASE], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=300)
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except Exception as e:  # a baseline figure, not a result: report why it is missing
        return {"error": f"{type(e).__name__}: {e}"}
    return {"workload": "mol40: 40^3 grid, h=0.3 Bohr, 5 orbitals, one spin channel; E_SIC and V_SIC "
                        "(FP64 CG to relative residual 1e-10)",
            "seconds": d["seconds"], "threads": d["threads"], "E_SIC": d["E_SIC"]}


KERNEL_SOURCES = ("zmarch.h", "stencil_pcg.hip", "stencil_res.hip", "dst.hip", "common.h")


def kernel_source_hash():
    """Hash of the solver kernel sources (invalidates stored HBM traffic)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_01186_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, kernel, solver):
    """(HBM bytes, algorithmic bytes) per launch with every orbital active of
    the dominant kernel from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, calibrated on a plain copy); None when the summary is missing
    or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{solver}_f32_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"]), float(vals["algorithmic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(torch, mib):
    """A plain device copy of `mib` MiB (src and dst fp32), three launches:
    the known-size reference for the HBM byte counters."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x {mib} MiB device copy", file=sys.stderr, flush=True)


def kernel_rates(agg):
    """Per-kernel averages of the sampled launches (HIP events in the timed
    region): time per launch, algorithmic GB/s and, for the preconditioner,
    matrix-core TFLOP/s."""
    out = {}
    for k in ("sweep", "update", "precond", "resid"):
        n, ms = agg[f"{k}_launches"], agg[f"{k}_ms"]
        if n <= 0 or ms <= 0:
            continue
        d = {"launches": int(n), "avg_launch_us": ms / n * 1e3,
             "gbs": agg[f"{k}_bytes"] / (ms * 1e-3) / 1e9,
             "algorithmic_bytes_per_launch": agg[f"{k}_bytes"] / n}
        if k == "precond":
            d["tflops"] = agg["precond_flops"] / (ms * 1e-3) / 1e12
        out[k] = d
    return out


KERNEL_NAMES = {
    "sweep": "k_zmarch<PolPQ> (CG stencil sweep: q = -L p, p.q)",
    "update": "k_pcg_rupd (r -= alpha q)",
    "precond": "k_dst_xy + k_dst_fast(z) + k_dst_xy<PO> (sine-transform preconditioner, split-bf16 MFMA; its last pass writes p = z + beta p_old; five per-axis passes where a plane does not fit in LDS)",
    "resid": "k_zmarch<PolResP> (FP64 residual b + L x closing a restart cycle, x = x64 + alpha_a p_a + alpha_b p_b)",
}


def roofline(args, agg):
    """Roofline line for the dominant kernel.  Every timed kernel (sweep,
    update and, with the preconditioned solver, the preconditioner) runs once
    per iteration of every active orbital, so the one with the longest
    average launch takes the most time (the sampled launch counts differ:
    the first launch of a solve or restart is never sampled).  The
    preconditioner is bound by HBM; its matrix-core use is shown beside."""
    rates = kernel_rates(agg)
    dom = max(rates, key=lambda k: rates[k]["avg_launch_us"])
    r = rates[dom]
    out = {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": r["gbs"], "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": r["gbs"] / HBM_PEAK_GBS}
    if dom == "precond" and "tflops" in r:
        # the split-bf16 transforms issue three bf16 products per fp32 multiply-add:
        # about 3 x 1152 / 44 = 78 flop/B at 96^3, under the bf16 ridge of
        # 2500 / 8 = 312 flop/B, so HBM is the roof; matrix-core use is shown beside
        out["mfma_bf16_tflops"] = 3.0 * r["tflops"]
        out["mfma_bf16_frac"] = 3.0 * r["tflops"] / BF16_MFMA_PEAK_TFLOPS
    # measured HBM bytes over algorithmic bytes of a full launch, applied to
    # this run's sampled launches (the same per launch as `achieved`)
    st = stored_traffic(args.workload, dom, args.solver)
    out["traffic"] = st[0] / st[1] * r["algorithmic_bytes_per_launch"] if st else None
    out["traffic_over_algorithmic"] = st[0] / st[1] if st else None
    out["algorithmic_bytes_per_launch"] = r["algorithmic_bytes_per_launch"]
    out["avg_launch_us"] = r["avg_launch_us"]
    out["launches"] = r["launches"]
    out["kernels"] = rates
    out["stencil_shape"] = agg.get("shape")
    out["precond_layout"] = agg.get("precond_layout")
    return out


def workload_config(args, systems, solves_per_step):
    common = {"fd_order": 12, "lmax": 6, "tol": args.tol, "solves_per_step": solves_per_step,
              "solver": {"pcg": "CG preconditioned by type-I sine transforms",
                         "cg": "plain CG"}[args.solver]}
    if len(systems) == 1:
        s = systems[0]
        nocc = list(s.nocc)
        return dict({"workload": f"{s.name}: {s.n[0]}^3 grid, h={s.h} Bohr, "
                                 f"{nocc[0]}+{nocc[1] if len(nocc) > 1 else 0} orbitals; per step "
                                 f"E_SIC, V_SIC (s=1) and all FOD forces",
                     "grid": list(s.n), "h": s.h, "nocc": nocc,
                     "parallelism": "single GPU, all orbitals of both spins batched per launch"},
                    **common)
    return dict({"workload": f"{len(systems)} uneven systems in one batch: grids "
                             f"{min(s.n[0] for s in systems)}^3..{max(s.n[0] for s in systems)}^3, "
                             f"{sum(sum(s.nocc) for s in systems)} orbitals; per step E_SIC, "
                             f"V_SIC (s=1) and all FOD forces of every system",
                 "systems": len(systems),
                 "parallelism": "single GPU, all orbitals of all systems batched per launch"},
                **common)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2108_01186_amd import fsic as F, synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.workload == "batch24":
        systems = synth.make_batch24(device=dev)
    else:
        systems = [synth.make_workload(args.workload, device=dev)]
    sysobj = max(systems, key=lambda s: s.M * sum(s.nocc))
    noccs = [list(s.nocc) for s in systems]
    dicts = [{"n": s.n, "h": s.h, "origin": s.origin, "psi": s.psi, "fod": s.fod,
              "vsic": [torch.empty(s.M, dtype=torch.float64, device=dev) for _ in s.nocc]}
             for s in systems]
    flags = F.FSIC_WANT_VSIC | F.FSIC_KEEP_TAPE | F.FSIC_PROFILE
    results = {}
    legs = ["mixed"] + ([] if args.no_fp64 else ["fp64"])
    for leg in legs:
        ctx = F.Context(precision=leg, tol=args.tol, flags=flags, solver=args.solver)
        basis = {"solves": 0, "ms": 0.0}  # unit-moment boundary solutions, once per grid
        for _ in range(args.warmup):
            st = ctx.forward_backward(dicts)[4]
            basis["solves"] += st["basis_solves"]
            basis["ms"] += st["basis_ms"]
        dt, e, g, agg = run_steps(F, torch, ctx, dicts, noccs, args.steps)
        results[leg] = dict(dt=dt, e=np.asarray(e, dtype=np.float64),
                            g=np.concatenate([np.concatenate(gs) for gs in g]), agg=agg, basis=basis)
        ctx.close()
        print(f"[bench] {leg}: {dt / args.steps * 1e3:.1f} ms/step, E_SIC={e[0]:.12f}",
              file=sys.stderr, flush=True)

    # beside the profiled legs: the mixed leg without events, eager and with
    # each chunk of CG iterations replayed as a captured HIP graph
    extra = {}
    if not args.no_graphs:
        for name, fl in (("mixed_unprofiled_solves_per_s", F.FSIC_WANT_VSIC | F.FSIC_KEEP_TAPE),
                         ("mixed_graphs_solves_per_s",
                          F.FSIC_WANT_VSIC | F.FSIC_KEEP_TAPE | F.FSIC_GRAPHS)):
            ctx = F.Context(precision="mixed", tol=args.tol, flags=fl, solver=args.solver)
            for _ in range(args.warmup):
                ctx.forward_backward(dicts)
            dt, _, _, agg = run_steps(F, torch, ctx, dicts, noccs, args.steps)
            ctx.close()
            extra[name] = agg["solves"] / dt

    # beside them: the same steps with the alternating Anderson-Richardson
    # solver (FP64, same preconditioner, unprofiled)
    if not args.no_aar:
        ctx = F.Context(precision="fp64", tol=args.tol, flags=F.FSIC_WANT_VSIC | F.FSIC_KEEP_TAPE,
                        solver="aar")
        for _ in range(args.warmup):
            ctx.forward_backward(dicts)
        dt, e_a, g_a, agg = run_steps(F, torch, ctx, dicts, noccs, args.steps)
        ctx.close()
        extra["aar_fp64_solves_per_s"] = agg["solves"] / dt
        extra["mean_aar_iters"] = agg["iters"] / max(1, agg["krylov"])
        if "fp64" in results:
            extra["dE_aar_vs_fp64"] = float(np.abs(np.asarray(e_a, dtype=np.float64) - results["fp64"]["e"]).max())
            ga = np.concatenate([np.concatenate(gs) for gs in g_a])
            extra["dF_max_aar_vs_fp64"] = float(np.abs(ga - results["fp64"]["g"]).max())

    mx = results["mixed"]
    steps = args.steps
    solves_per_step = mx["agg"]["solves"] / steps
    value = mx["agg"]["solves"] / mx["dt"]
    krylov_per_step = mx["agg"]["krylov"] / steps
    roof = roofline(args, mx["agg"])
    out = {
        "metric": "orbital Poisson solves/sec + E_SIC&FOD-force time at 1e-8 Ha, mixed vs FP64",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": mx["dt"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": workload_config(args, systems, solves_per_step),
        "e_sic_force_ms_mixed": mx["dt"] / steps * 1e3,
        "krylov_solves_per_step": krylov_per_step,
        "krylov_solves_per_s_mixed": mx["agg"]["krylov"] / mx["dt"],
        "boundary_basis_timed_solves": mx["agg"]["basis_solves"],
        "boundary_basis_warmup_mixed": {"solves": mx["basis"]["solves"], "ms": round(mx["basis"]["ms"], 1)},
        "mean_cg_iters_mixed": mx["agg"]["iters"] / max(1, mx["agg"]["krylov"]),
        "max_relres_mixed": mx["agg"]["max_relres"],
        "host_phase_ms_mixed": dict(zip(["setup", "fo_loewdin", "boundary_rhs", "cg", "xc_average",
                                         "adjoint_cg", "adjoint_rest"],
                                        [round(v, 3) for v in mx["agg"]["phase_ms"][:7]])),
        "roofline": roof,
    }
    if "fp64" in results:
        fp = results["fp64"]
        out["fp64_solves_per_s"] = fp["agg"]["solves"] / fp["dt"]
        out["e_sic_force_ms_fp64"] = fp["dt"] / steps * 1e3
        out["speedup_mixed_vs_fp64"] = fp["dt"] / mx["dt"]
        out["mean_cg_iters_fp64"] = fp["agg"]["iters"] / max(1, fp["agg"]["krylov"])
        out["dE_mixed_vs_fp64"] = float(np.abs(mx["e"] - fp["e"]).max())
        out["dF_max_mixed_vs_fp64"] = float(np.abs(mx["g"] - fp["g"]).max())
        out["fp64_kernels"] = kernel_rates(fp["agg"])
    out.update(extra)
    if args.copy_calibration > 0:
        copy_calibration(torch, args.copy_calibration)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysobj, args.tol, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
