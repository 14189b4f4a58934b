#!/usr/bin/env python3
"""Throughput of the split-step Crank-Nicolson time step of the 3D dipolar GPE
on one MI355X: grid-point-steps per second at 256^3.

Default run (one JSON line on stdout):
  headline  FP32 (complex64 passes, FP64 reductions) imaginary-time steps of the
            256^3 workload (dx = 0.1, dt = 0.001, trap (1, 1, 0.5), g = 100,
            gd = 60), input resident in HBM, K timed steps after W warm-up
            steps, bracketed by device synchronisation (the paper's timing
            rule: only the iteration loop is timed, program summary, Testing
            results).
  variants  the same workload in FP64, and the FP32 real-time adjoint
            (forward, recompute and reverse sweeps, per forward step).
  roofline  per-pass HIP event timing of the dominant pass on the plan's
            stream against its algorithmic HBM bytes; HBM traffic from the
            committed rocprofv3 counter summary when it matches the sources.
  cpu_baseline  the FP64 oracle on the host on a bounded sample (a few steps
            of the same workload).

Other modes:
  --profile-run        headline steps only (for rocprofv3 runs)
  --copy-calibration   a plain device copy of known size (counter calibration)
  --summarize DIR      turn rocprofv3 CSV output under DIR into profiles/ text
"""
import argparse
import glob
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256cubed.json")
KERNEL_OF_PASS = {
    "r2c_z": "k_r2c2", "fft_y": "k_rows2", "fft_x_mul": "k_xmul2", "ifft_y": "k_rows2",
    "c2r_z_nonlinear_cn_z": "k_c2r_step2", "cn_y": "k_cn_strided", "cn_x": "k_cn_strided",
    "norm_reduce": "k_reduce",
}


def source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1610_05329_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(cfg):
    return {
        "workload": f"{cfg.n[0]}x{cfg.n[1]}x{cfg.n[2]} imaginary-time split step, dx={cfg.d[0]}, "
                    f"dt={cfg.dt}, trap=({cfg.trap[0]},{cfg.trap[1]},{cfg.trap[2]}), g={cfg.g}, gd={cfg.gd}, "
                    f"cutoff R=L/2, seeded Gaussian + 1e-3 noise",
        "grid": list(cfg.n), "points": cfg.npoints,
    }


CHUNK = 50  # the 256^3 imaginary-time parameters collapse after ~90 steps


def timed_steps(torch, plan, psi, psi_init, steps, warmup):
    """Time `steps` steps in chunks of at most CHUNK, each chunk restarting from
    psi_init (device copy, inside the timed region) so that every timed step
    works on a regular state."""
    psi.copy_(psi_init)
    plan.step(psi, min(warmup, CHUNK))
    torch.cuda.synchronize()
    stream = plan.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    done = 0
    while done < steps:
        k = min(CHUNK, steps - done)
        psi.copy_(psi_init)
        plan.step(psi, k)
        done += k
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1000.0


def traffic_for(kernel, launches_per_step_of_kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when absent or taken from other sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("source_hash") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k["hbm_bytes_per_dispatch"]


def cpu_baseline(cfg, psi0, steps):
    from oracle import dgpe_oracle as O
    p = O.Params.from_config(cfg)
    V0 = O.trap_base(p)
    psi = psi0.copy()
    t0 = time.perf_counter()
    for _ in range(steps):
        psi = O.step(p, psi, 1.0, V0)
    dt = time.perf_counter() - t0
    return {"value": cfg.npoints * steps / dt, "unit": "grid-point-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps of the same {cfg.n[0]}^3 imaginary-time workload "
                      f"({dt:.1f} s; numpy, single-threaded FFT and elementwise work)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--profile-run", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--summarize", metavar="DIR")
    ap.add_argument("--summary-name", default="")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"))
    ap.add_argument("--command", default="")
    ap.add_argument("--traffic-json", action="store_true",
                    help="also record the traffic as the roofline's counter figures "
                         "(only for the workload of the JSON line)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--adjoint-steps", type=int, default=40)
    ap.add_argument("--workload", choices=["imag_256cubed", "real_512x512x256", "adjoint_256cubed"],
                    default="imag_256cubed",
                    help="workload of --profile-run (the JSON line always uses imag_256cubed); "
                         "adjoint_256cubed = the FP32 real-time adjoint on that grid (--steps forward steps, "
                         "checkpoints every 10)")
    args = ap.parse_args()

    if args.summarize:
        out = summarize(args.summarize, args.summary_name)
        if args.traffic:
            out += [""] + summarize_traffic(*args.traffic, 256 << 20, args.summary_name,
                                            TRAFFIC_FILE if args.traffic_json else None)
        out.insert(1, "# command: " + args.command if args.command else "#")
        path = os.path.join(ROOT, "profiles", f"{args.summary_name}.txt")
        open(path, "w").write("\n".join(out) + "\n")
        print("\n".join(out))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only; the multi-GPU slab decomposition is designed "
              "but not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1610_05329_amd as dg
    import workloads as W

    if args.copy_calibration:
        n = 64 << 20  # 64 Mi floats = 256 MiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {n * 4} bytes")
        return

    if args.profile_run and args.workload == "adjoint_256cubed":
        cfg = W.CONFIGS["imag_256cubed"]
        plan_a = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True,
                         dtype=torch.complex64)
        psia = plan_a.new_state(W.noisy_gaussian(cfg))
        amp = np.ones(args.steps + 1)
        plan_a.adjoint(psia, amp[:3], ckpt_every=2)  # warm-up
        plan_a.adjoint(psia, amp, ckpt_every=10)
        torch.cuda.synchronize()
        log("[bench] adjoint profile run done")
        return
    cfg = W.CONFIGS[args.workload if args.profile_run else "imag_256cubed"]
    log(f"[bench] workload {cfg.n} {'imaginary' if cfg.imag else 'real'} time; preparing seeded state")
    psi0 = W.noisy_gaussian(cfg)
    plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=not cfg.imag,
                   dtype=torch.complex64)
    psi_init = plan.new_state(psi0)
    psi = psi_init.clone()
    if args.profile_run:
        for k in (args.warmup, args.steps):
            psi.copy_(psi_init)
            plan.step(psi, min(k, CHUNK))
        torch.cuda.synchronize()
        log("[bench] profile run done")
        return

    wall, ev = timed_steps(torch, plan, psi, psi_init, args.steps, args.warmup)
    value = cfg.npoints * args.steps / wall
    log(f"[bench] FP32: {args.steps} steps in {wall * 1e3:.2f} ms wall ({ev * 1e3:.2f} ms events)")
    assert torch.isfinite(torch.view_as_real(psi)).all().item(), "non-finite state"

    # roofline: per-pass events over a second timed region
    psi.copy_(psi_init)
    ms, tot = plan.step_profiled(psi, min(args.steps, CHUNK))
    pbytes = plan.pass_bytes()
    per_step_bytes = sum(pbytes.values())
    share = {k: v for k, v in ms.items() if v > 0}
    dom = max(share, key=share.get)  # longest average launch
    kernel_of = dict(KERNEL_OF_PASS, cn_y="k_cn_ycarry") if plan.fused_y else KERNEL_OF_PASS
    ach = pbytes[dom] / (ms[dom] * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "kernel": kernel_of[dom], "pass": dom, "fused_y": plan.fused_y,
        "achieved": round(ach, 1),
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": traffic_for(kernel_of[dom], 1),
        "avg_launch_ms": round(ms[dom], 5), "algorithmic_bytes_per_launch": pbytes[dom],
        "per_pass_ms": {k: round(v, 5) for k, v in ms.items()},
        "per_pass_GBs": {k: round(pbytes[k] / (ms[k] * 1e-3) / 1e9, 1) for k in share},
        "step_algorithmic_bytes": per_step_bytes,
        "step_effective_GBs": round(per_step_bytes * args.steps / wall / 1e9, 1),
        "step_frac_of_peak": round(per_step_bytes * args.steps / wall / 1e9 / HBM_PEAK_GBS, 4),
    }
    log(f"[bench] dominant pass {dom}: {ach:.0f} GB/s; step effective "
        f"{roofline['step_effective_GBs']} GB/s")

    variants = {}
    if not args.no_variants:
        plan64 = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=False, dtype=torch.complex128)
        init64 = plan64.new_state(psi0)
        psi64 = init64.clone()
        w64, _ = timed_steps(torch, plan64, psi64, init64, args.steps, args.warmup)
        b64 = sum(plan64.pass_bytes().values())
        variants["f64"] = {"value": cfg.npoints * args.steps / w64, "ms_per_step": w64 * 1e3 / args.steps,
                           "step_effective_GBs": round(b64 * args.steps / w64 / 1e9, 1)}
        log(f"[bench] FP64: {w64 * 1e3 / args.steps:.3f} ms/step")
        del plan64, psi64, init64
        torch.cuda.empty_cache()
        # adjoint: real time, FP32, energy objective, checkpoints every 10 steps
        na = args.adjoint_steps
        plan_a = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True, dtype=torch.complex64)
        psia = plan_a.new_state(psi0)
        amp = np.ones(na + 1)
        plan_a.adjoint(psia, amp[:3], ckpt_every=2)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan_a.adjoint(psia, amp, ckpt_every=10)
        torch.cuda.synchronize()
        wa = time.perf_counter() - t0
        variants["adjoint_f32"] = {"value": cfg.npoints * na / wa, "ms_per_step": wa * 1e3 / na,
                                   "steps": na, "ckpt_every": 10, "objective": "energy",
                                   "J": out["J"]}
        log(f"[bench] adjoint FP32: {wa * 1e3 / na:.3f} ms per forward step")
        del plan_a, psia, out
        torch.cuda.empty_cache()
        # 512 x 512 x 256 FP32 real time (the large anisotropic workload)
        big = W.CONFIGS["real_512x512x256"]
        plan_big = dg.Plan(big.n, big.d, big.dt, big.trap, big.g, big.gd, real_time=True, dtype=torch.complex64)
        init_big = plan_big.new_state(W.noisy_gaussian(big))
        psi_big = init_big.clone()
        n_big = 20
        w_big, _ = timed_steps(torch, plan_big, psi_big, init_big, n_big, 5)
        b_big = sum(plan_big.pass_bytes().values())
        variants["real_512x512x256_f32"] = {
            "value": big.npoints * n_big / w_big, "ms_per_step": w_big * 1e3 / n_big,
            "grid": list(big.n), "step_effective_GBs": round(b_big * n_big / w_big / 1e9, 1)}
        log(f"[bench] 512x512x256 FP32 real time: {w_big * 1e3 / n_big:.3f} ms/step")
        del plan_big, psi_big, init_big
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline: {args.cpu_steps} steps")
        cpu = cpu_baseline(cfg, psi0, args.cpu_steps)

    line = {
        "metric": "grid-point-steps/sec at 256^3 (FP32 plain imaginary-time step)",
        "value": value, "unit": "grid-point-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Gaussian + uniform noise, generated on the host)",
        "config": workload(cfg), "roofline": roofline, "cpu_baseline": cpu, "variants": variants,
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------

def _short(name):
    """Kernel name with its template arguments, without return type, namespaces
    and parameter list (this library's kernels are all named k_*)."""
    m = re.search(r"\b(k_\w+(?:<[^()]*>)?)\(", name)
    return m.group(1) if m else name.split("(")[0][:60]


def _counter_means(d):
    """Mean counter value per dispatch by short kernel name, from a rocprofv3
    --pmc CSV under d (the counter is in KiB for FETCH_SIZE / WRITE_SIZE)."""
    import csv
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    agg = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            k = _short(r["Kernel_Name"])
            a = agg.setdefault(k, [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    return {k: s / n for k, (s, n) in agg.items()}


def summarize(d, name):
    """profiles/<name>.txt from the rocprofv3 --stats output under d."""
    import csv
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    rows = list(csv.DictReader(open(stats[0])))
    out = [f"# rocprofv3 --kernel-trace --stats summary: {name}",
           f"# {'kernel':<46} {'calls':>6} {'avg_us':>10} {'total_ms':>10} {'pct':>6}"]
    for r in rows:
        out.append(f"  {_short(r['Name']):<46} {int(r['Calls']):>6} "
                   f"{float(r['AverageNs']) / 1e3:>10.2f} {float(r['TotalDurationNs']) / 1e6:>10.3f} "
                   f"{float(r['Percentage']):>6.2f}")
    return out


def summarize_traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, header, json_path):
    """HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE, each scaled by the
    ratio the same counter reads for a plain device copy of known size."""
    f, w = _counter_means(fetch_dir), _counter_means(write_dir)
    cf, cw = _counter_means(cfetch_dir), _counter_means(cwrite_dir)
    ck = "__amd_rocclr_copyBuffer"
    ffac = cf[ck] * 1024 / copy_bytes
    wfac = cw[ck] * 1024 / copy_bytes
    kernels = {}
    for k in sorted(set(f) & set(w)):
        if not k.startswith("k_"):
            continue
        fb, wb = f[k] * 1024 / ffac, w[k] * 1024 / wfac
        kernels[k.split("<")[0]] = kernels.get(k.split("<")[0], [])
        kernels[k.split("<")[0]].append({"variant": k, "fetch_bytes": fb, "write_bytes": wb,
                                         "hbm_bytes_per_dispatch": fb + wb})
    rec = {"source_hash": source_hash(), "fetch_scale": ffac, "write_scale": wfac,
           "copy_bytes": copy_bytes, "header": header,
           "kernels": {k: max(v, key=lambda e: e["hbm_bytes_per_dispatch"]) for k, v in kernels.items()},
           "all_variants": kernels}
    if json_path:
        json.dump(rec, open(json_path, "w"), indent=1)
    lines = [f"# HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE; separate runs)",
             f"# {header}",
             f"# calibration: a {copy_bytes} B device copy read FETCH_SIZE x{ffac:.4f} and WRITE_SIZE x{wfac:.4f} "
             f"of the bytes moved; kernel values below are divided by these factors",
             f"# {'kernel':<46} {'fetch_MB':>10} {'write_MB':>10} {'total_MB':>10}"]
    for k, v in kernels.items():
        for e in v:
            lines.append(f"  {e['variant']:<46} {e['fetch_bytes'] / 1e6:>10.2f} {e['write_bytes'] / 1e6:>10.2f} "
                         f"{e['hbm_bytes_per_dispatch'] / 1e6:>10.2f}")
    return lines


if __name__ == "__main__":
    main()
