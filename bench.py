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
  variants  the same workload in FP64; the same grid and parameters in real time
            (FP32 and FP64); the FP32 real-time adjoint (forward, recompute
            and reverse sweeps, per forward step); the 512 x 512 x 256 FP32
            real-time workload.  The paths beyond the plain step: the
            symmetric (Strang) step at 256^3 (FP32, both time modes), the
            ground-state driver on the 128^3 preparation (FP64, to a mu change
            below 1e-10 per step), quasi-2D plans at 2048 x 2048 (FP32, both
            time modes), the overlap-objective adjoint at 256^3 (FP32) and the
            binary density file of the 256^3 state.  Each with its fraction of the HBM peak on the
            bytes its passes move and on the model bytes (22 s per point per
            step, s = bytes per real; 82 s for the adjoint).
  roofline  per-pass HIP event timing of the dominant pass on the plan's
            stream against its model HBM bytes (and the bytes it moves); HBM
            traffic from the committed rocprofv3 counter summary when it
            matches the sources.
  hbm_stream_reference  what plain streaming reaches on this part: torch's
            in-place scale and copy of FP32 arrays of 128 MiB (the 256^3 FP32
            state, mostly resident in the 256 MB Infinity Cache) and of 1 GiB
            (beyond it: the HBM rate the 512 x 512 x 256 passes compete with).
  cpu_baseline  the FP64 oracle on the host on a bounded sample (10 steps of
            the same workload from the same state), with the host CPU model.
  precision the FP32 and FP64 GPU states, mu and energy after those steps
            against the oracle's, and FP32 against FP64.

Other modes:
  --profile-run        steps of one workload only (for rocprofv3 runs; --workload,
                       --precision)
  --copy-calibration   a plain device copy of known size (counter calibration)
  --stream-reference   only the streaming reference (for rocprofv3 runs)
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


def host_cpu():
    """Model name of the host CPU and the cores this process may run on."""
    model = "unknown"
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
    return model, avail


def cpu_baseline(cfg, psi0, steps):
    """The FP64 oracle as it stands, timed on the host for `steps` steps of the
    workload; returns the record and the oracle's final state."""
    from oracle import dgpe_oracle as O
    p = O.Params.from_config(cfg)
    V0 = O.trap_base(p)
    psi = psi0.copy()
    t0 = time.perf_counter()
    for _ in range(steps):
        psi = O.step(p, psi, 1.0, V0)
    dt = time.perf_counter() - t0
    model, avail = host_cpu()
    rec = {"value": cfg.npoints * steps / dt, "unit": "grid-point-steps/s", "cores": 1,
           "kind": "oracle", "cpu_model": model, "host_cores_available": avail,
           "sample": f"{steps} FP64 oracle steps of the same {cfg.n[0]}^3 imaginary-time workload "
                     f"from the same seeded state ({dt:.1f} s; numpy: pocketfft and the elementwise "
                     f"and Thomas work run on one thread)"}
    return rec, psi


def oracle_observables(cfg, psi):
    from oracle import dgpe_oracle as O
    return O.observables(O.Params.from_config(cfg), psi)


# Model HBM bytes per grid point per step of the seven-pass schedule (s = bytes
# per real): P1 3s (read psi, write the half spectrum), P2, P3, P4 2s each (the
# half spectrum in place), P5 5s (read spectrum and psi, write psi), P6 and P7
# 4s each (psi in place): 22 s.  The adjoint (forward, recompute and reverse
# sweeps) moves about 82 s per forward step.
MODEL_S_PER_POINT = 22
ADJOINT_MODEL_S_PER_POINT = 82


def model_pass_bytes(n, s):
    """Model bytes of one launch of each pass, for the separate y schedule
    (the fused y schedule adds carry arrays to P5 and P7 and replaces P6)."""
    nt = n[0] * n[1] * n[2]
    state = 2.0 * s * nt
    spec = 2.0 * s * n[0] * n[1] * (n[2] // 2 + 1)
    uk = s * (n[0] // 2 + 1) * (n[1] // 2 + 1) * (n[2] // 2 + 1)
    return {"r2c_z": state + spec, "fft_y": 2 * spec, "fft_x_mul": 2 * spec + uk, "ifft_y": 2 * spec,
            "c2r_z_nonlinear_cn_z": spec + 2 * state, "cn_y": 2 * state, "cn_x": 2 * state}


def frac(bytes_, seconds):
    return round(bytes_ / seconds / 1e9 / HBM_PEAK_GBS, 4)


def measure(torch, dg, cfg, real_time, dtype, steps, warmup, psi0=None, per_pass=True, scheme=None,
            q2d=None):
    """Time `steps` plain steps of one workload; the step's rate, bytes moved
    (the passes' own counts) and model bytes against the HBM peak, and the
    per-pass event timing."""
    import workloads as W
    s = 4 if dtype == torch.complex64 else 8
    plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=dtype,
                   q2d=q2d)
    if scheme:
        plan.set("scheme", scheme)
    init = plan.new_state(W.noisy_gaussian(cfg) if psi0 is None else psi0)
    psi = init.clone()
    wall, _ = timed_steps(torch, plan, psi, init, steps, warmup)
    assert torch.isfinite(torch.view_as_real(psi)).all().item(), "non-finite state"
    moved = sum(plan.pass_bytes().values())
    # model bytes of the plain step (3D: 22 s per point; quasi-2D has no y
    # transforms and no y sweep: 14 s)
    model = (MODEL_S_PER_POINT - (8 if q2d else 0)) * s * cfg.npoints
    out = {"value": cfg.npoints * steps / wall, "ms_per_step": wall * 1e3 / steps, "steps": steps,
           "grid": list(cfg.n), "time": "real" if real_time else "imaginary",
           "dtype": "f32" if s == 4 else "f64", "fused_y": plan.fused_y,
           "step_bytes_moved": moved, "step_frac_of_peak": frac(moved * steps, wall),
           "step_model_bytes": model, "step_frac_of_peak_model_bytes": frac(model * steps, wall)}
    if per_pass:
        psi.copy_(init)
        ms, _ = plan.step_profiled(psi, min(steps, CHUNK))
        pb = plan.pass_bytes()
        out["per_pass_ms"] = {k: round(v, 5) for k, v in ms.items() if v > 0}
        out["per_pass_frac"] = {k: round(pb[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
                                for k, v in ms.items() if v > 0 and pb[k] > 1e6}
    plan.close()
    del plan, psi, init
    torch.cuda.empty_cache()
    return out


def _q2d_config():
    import workloads as W
    return W.Config("q2d_2048x2048", (2048, 1, 2048), (0.025, 1.0, 0.025), 0.0002, (1.0, 10.0, 1.0),
                    100.0, 60.0, True, 100, noise=1e-3, seed=6)


Q2D_2048 = _q2d_config()


def widened(torch, dg, np, W, cfg, psi0):
    """Measurements of the paths beyond the plain step (see the module doc)."""
    out = {}
    lie = {}
    for real_time in (False, True):
        mode = "real" if real_time else "imag"
        k = f"strang_256cubed_f32_{mode}"
        out[k] = measure(torch, dg, cfg, real_time, torch.complex64, 20, 5, psi0, per_pass=False,
                         scheme="strang")
        lie[mode] = measure(torch, dg, cfg, real_time, torch.complex64, 20, 5, psi0,
                            per_pass=False)["ms_per_step"]
        out[k]["ms_per_step_first_order_step"] = lie[mode]
        out[k].pop("step_bytes_moved")  # the passes' counts are those of the first-order step
        out[k].pop("step_frac_of_peak")
        out[k].pop("step_model_bytes")
        out[k].pop("step_frac_of_peak_model_bytes")
        log(f"[bench] symmetric step 256^3 FP32 {mode}: {out[k]['ms_per_step']:.3f} ms/step "
            f"(first-order {lie[mode]:.3f})")
    # the ground-state driver on the 128^3 preparation (gd = 15, FP64)
    q = W.CONFIGS["quench_128cubed"]
    plan = dg.Plan(q.n, q.d, q.dt, q.trap, q.g, 15.0, real_time=False, dtype=torch.complex128)
    psi = plan.new_state(W.gaussian_state(q.n, q.d, q.trap))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.ground_state(psi, tol=1e-10, max_steps=20000, check_every=10)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out["ground_state_128cubed_f64"] = {
        "steps": res["steps"], "converged": bool(res["converged"]), "seconds": sec,
        "ms_per_step": sec * 1e3 / max(res["steps"], 1), "dmu_per_step": res["dmu_per_step"],
        "mu": res["observables"]["mu"], "tol": 1e-10, "check_every": 10}
    log(f"[bench] ground state 128^3 FP64: {res['steps']} steps in {sec:.2f} s")
    plan.close()
    del plan, psi
    # quasi-2D (dipoles along the tight axis) at 2048 x 2048, the largest plane
    c2 = Q2D_2048
    for real_time in (False, True):
        mode = "real" if real_time else "imag"
        k = f"q2d_2048x2048_f32_{mode}"
        out[k] = measure(torch, dg, c2, real_time, torch.complex64, 100, 10, per_pass=False, q2d="perp")
        log(f"[bench] quasi-2D 2048x2048 FP32 {mode}: {out[k]['ms_per_step']:.3f} ms/step")
    # overlap-objective adjoint at 256^3 (FP32, real time, 40 steps, checkpoints every 10)
    na = 40
    plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True, dtype=torch.complex64)
    psia = plan.new_state(psi0)
    tgt = plan.new_state(W.gaussian_state(cfg.n, cfg.d, cfg.trap))
    amp = np.ones(na + 1)
    plan.adjoint(psia, amp[:3], ckpt_every=2, objective="overlap", target=tgt)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.adjoint(psia, amp, ckpt_every=10, objective="overlap", target=tgt)
    torch.cuda.synchronize()
    wa = time.perf_counter() - t0
    out["adjoint_overlap_f32"] = {"value": cfg.npoints * na / wa, "ms_per_step": wa * 1e3 / na,
                                  "steps": na, "ckpt_every": 10, "objective": "overlap", "J": res["J"]}
    log(f"[bench] overlap adjoint FP32: {wa * 1e3 / na:.3f} ms per forward step")
    del res
    # the binary density file (FP64 [x][y][z]) of the 256^3 state
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "density.bin")
        plan.write_density(psia, path)  # warm-up
        t0 = time.perf_counter()
        plan.write_density(psia, path)
        sec = time.perf_counter() - t0
        nbytes = os.path.getsize(path)
    out["density_file_256cubed"] = {"bytes": nbytes, "seconds": sec, "GBs": nbytes / sec / 1e9,
                                    "note": "device density kernel, device-to-host copy and file "
                                            "write (page cache)"}
    log(f"[bench] density file 256^3: {nbytes / 1e6:.0f} MB in {sec * 1e3:.1f} ms")
    plan.close()
    del plan, psia, tgt
    torch.cuda.empty_cache()
    return out


def stream_reference(torch, reps=10):
    """GB/s (bytes read + written) of torch's in-place scale and of a copy
    between two arrays, for FP32 arrays of 128 MiB and 1 GiB."""
    out = {}
    for mib in (128, 1024):
        n = (mib << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for kind in ("scale_in_place", "copy"):
            def go():
                if kind == "copy":
                    b.copy_(a)
                else:
                    a.mul_(1.0)
            for _ in range(3):
                go()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                go()
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / reps
            gbs = 2.0 * n * 4 / sec / 1e9
            out[f"{kind}_{mib}MiB_GBs"] = round(gbs, 1)
            out[f"{kind}_{mib}MiB_frac_of_peak"] = round(gbs / HBM_PEAK_GBS, 4)
        del a, b
        torch.cuda.empty_cache()
    out["kernel"] = "torch elementwise (FP32, in place: mul_(1.0); copy: copy_)"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--profile-run", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--stream-reference", action="store_true")
    ap.add_argument("--summarize", metavar="DIR")
    ap.add_argument("--summary-name", default="")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"))
    ap.add_argument("--command", default="")
    ap.add_argument("--traffic-json", action="store_true",
                    help="also record the traffic as the roofline's counter figures "
                         "(only for the workload of the JSON line)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--adjoint-steps", type=int, default=40)
    ap.add_argument("--workload", choices=["imag_256cubed", "real_256cubed", "real_512x512x256",
                                           "adjoint_256cubed", "q2d_2048", "q2d_2048_real"],
                    default="imag_256cubed",
                    help="workload of --profile-run (the JSON line always uses imag_256cubed); "
                         "real_256cubed = the same grid and parameters in real time; "
                         "adjoint_256cubed = the real-time adjoint on that grid (--steps forward steps, "
                         "checkpoints every 10)")
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32",
                    help="precision of --profile-run")
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

    if args.stream_reference:
        log(f"[bench] streaming reference: {json.dumps(stream_reference(torch))}")
        return

    pdtype = torch.complex64 if args.precision == "f32" else torch.complex128
    if args.profile_run and args.workload == "adjoint_256cubed":
        cfg = W.CONFIGS["imag_256cubed"]
        plan_a = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True, dtype=pdtype)
        psia = plan_a.new_state(W.noisy_gaussian(cfg))
        amp = np.ones(args.steps + 1)
        plan_a.adjoint(psia, amp[:3], ckpt_every=2)  # warm-up
        plan_a.adjoint(psia, amp, ckpt_every=10)
        torch.cuda.synchronize()
        log("[bench] adjoint profile run done")
        return
    if args.profile_run and args.workload.startswith("q2d_2048"):
        c2 = Q2D_2048
        log(f"[bench] profile run {args.workload} {args.precision}")
        plan = dg.Plan(c2.n, c2.d, c2.dt, c2.trap, c2.g, c2.gd, real_time=args.workload.endswith("real"),
                       dtype=pdtype, q2d="perp")
        psi_init = plan.new_state(W.noisy_gaussian(c2))
        psi = psi_init.clone()
        for k in (args.warmup, args.steps):
            psi.copy_(psi_init)
            plan.step(psi, min(k, CHUNK))
        torch.cuda.synchronize()
        log("[bench] profile run done")
        return
    if args.profile_run:
        name = "imag_256cubed" if args.workload == "real_256cubed" else args.workload
        cfg = W.CONFIGS[name]
        real_time = not cfg.imag or args.workload == "real_256cubed"
        log(f"[bench] profile run {args.workload} {args.precision}")
        plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=pdtype)
        psi_init = plan.new_state(W.noisy_gaussian(cfg))
        psi = psi_init.clone()
        for k in (args.warmup, args.steps):
            psi.copy_(psi_init)
            plan.step(psi, min(k, CHUNK))
        torch.cuda.synchronize()
        log("[bench] profile run done")
        return

    cfg = W.CONFIGS["imag_256cubed"]
    log(f"[bench] workload {cfg.n} imaginary time; preparing seeded state")
    psi0 = W.noisy_gaussian(cfg)
    plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=False,
                   dtype=torch.complex64)
    psi_init = plan.new_state(psi0)
    psi = psi_init.clone()
    wall, ev = timed_steps(torch, plan, psi, psi_init, args.steps, args.warmup)
    value = cfg.npoints * args.steps / wall
    log(f"[bench] FP32: {args.steps} steps in {wall * 1e3:.2f} ms wall ({ev * 1e3:.2f} ms events)")
    assert torch.isfinite(torch.view_as_real(psi)).all().item(), "non-finite state"

    # roofline: per-pass events (on the plan's stream) over a second timed region
    psi.copy_(psi_init)
    ms, tot = plan.step_profiled(psi, min(args.steps, CHUNK))
    pbytes = plan.pass_bytes()
    mbytes = model_pass_bytes(cfg.n, 4)
    per_step_bytes = sum(pbytes.values())
    step_model = MODEL_S_PER_POINT * 4 * cfg.npoints
    share = {k: v for k, v in ms.items() if v > 0}
    dom = max(share, key=share.get)  # longest average launch
    kernel_of = dict(KERNEL_OF_PASS, cn_y="k_cn_ycarry") if plan.fused_y else KERNEL_OF_PASS
    ach = mbytes[dom] / (ms[dom] * 1e-3) / 1e9
    ach_moved = pbytes[dom] / (ms[dom] * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "kernel": kernel_of[dom], "pass": dom, "fused_y": plan.fused_y,
        "achieved": round(ach, 1),
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": traffic_for(kernel_of[dom], 1),
        "avg_launch_ms": round(ms[dom], 5),
        "algorithmic_bytes_per_launch": mbytes[dom],
        "algorithmic_bytes_rule": "model bytes of the pass: 2s per half-spectrum value read, "
                                  "2s per state point read and 2s written (s = 4)",
        "bytes_moved_per_launch": pbytes[dom],
        "achieved_on_bytes_moved": round(ach_moved, 1),
        "frac_on_bytes_moved": round(ach_moved / HBM_PEAK_GBS, 4),
        "per_pass_ms": {k: round(v, 5) for k, v in ms.items()},
        "per_pass_GBs": {k: round(pbytes[k] / (ms[k] * 1e-3) / 1e9, 1) for k in share},
        "step_bytes_moved": per_step_bytes,
        "step_effective_GBs": round(per_step_bytes * args.steps / wall / 1e9, 1),
        "step_frac_of_peak": round(per_step_bytes * args.steps / wall / 1e9 / HBM_PEAK_GBS, 4),
        "step_model_bytes": step_model,
        "step_frac_of_peak_model_bytes": frac(step_model * args.steps, wall),
    }
    log(f"[bench] dominant pass {dom}: {ach:.0f} GB/s on model bytes ({ach_moved:.0f} on bytes moved); "
        f"step {roofline['step_effective_GBs']} GB/s moved")
    plan.close()
    del plan, psi, psi_init
    torch.cuda.empty_cache()

    variants = {}
    if not args.no_variants:
        variants["f64"] = measure(torch, dg, cfg, False, torch.complex128, args.steps, args.warmup, psi0)
        log(f"[bench] FP64 imaginary time: {variants['f64']['ms_per_step']:.3f} ms/step")
        for prec, dt_ in (("f32", torch.complex64), ("f64", torch.complex128)):
            k = f"real_256cubed_{prec}"
            variants[k] = measure(torch, dg, cfg, True, dt_, 20, 5, psi0)
            log(f"[bench] {prec} real time 256^3: {variants[k]['ms_per_step']:.3f} ms/step")
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
        amodel = ADJOINT_MODEL_S_PER_POINT * 4 * cfg.npoints
        variants["adjoint_f32"] = {"value": cfg.npoints * na / wa, "ms_per_step": wa * 1e3 / na,
                                   "steps": na, "ckpt_every": 10, "objective": "energy",
                                   "J": out["J"], "step_model_bytes": amodel,
                                   "step_frac_of_peak_model_bytes": frac(amodel * na, wa)}
        log(f"[bench] adjoint FP32: {wa * 1e3 / na:.3f} ms per forward step")
        # every state and its Phi kept (ckpt_every = 1): no recompute
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out1 = plan_a.adjoint(psia, amp, ckpt_every=1)
        torch.cuda.synchronize()
        w1 = time.perf_counter() - t0
        variants["adjoint_f32_keep_all"] = {
            "value": cfg.npoints * na / w1, "ms_per_step": w1 * 1e3 / na, "steps": na, "ckpt_every": 1,
            "objective": "energy", "J": out1["J"], "same_J_as_ckpt_10": out1["J"] == out["J"],
            "adjoint_workspace_GiB": plan_a.lib.dgpe_adjoint_workspace_bytes(plan_a.handle, na, 1) / 2**30}
        log(f"[bench] adjoint FP32, every state kept: {w1 * 1e3 / na:.3f} ms per forward step")
        del out1
        plan_a.close()
        del plan_a, psia, out
        torch.cuda.empty_cache()
        # 512 x 512 x 256 FP32 real time (the large anisotropic workload)
        big = W.CONFIGS["real_512x512x256"]
        variants["real_512x512x256_f32"] = measure(torch, dg, big, True, torch.complex64, 20, 5)
        log(f"[bench] 512x512x256 FP32 real time: "
            f"{variants['real_512x512x256_f32']['ms_per_step']:.3f} ms/step")
        variants.update(widened(torch, dg, np, W, cfg, psi0))

    stream = stream_reference(torch)
    log(f"[bench] streaming reference: in place {stream['scale_in_place_128MiB_GBs']} GB/s at 128 MiB, "
        f"{stream['scale_in_place_1024MiB_GBs']} GB/s at 1 GiB")

    cpu = None
    precision = None
    if not args.no_cpu_baseline:
        k = args.cpu_steps
        log(f"[bench] CPU oracle baseline: {k} steps")
        cpu, psi_o = cpu_baseline(cfg, psi0, k)
        # the precision form against the FP64 GPU run and the oracle, after the
        # same k steps from the same state
        obs_o = oracle_observables(cfg, psi_o)
        gpu = {}
        for prec, dt_ in (("f32", torch.complex64), ("f64", torch.complex128)):
            pl = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=False, dtype=dt_)
            st = pl.new_state(psi0)
            pl.step(st, k)
            gpu[prec] = (pl.observables(st), st.cpu().numpy().astype(np.complex128))
            pl.close()
            del pl, st
        torch.cuda.empty_cache()

        def rel(a, b):
            return float(abs(a - b) / abs(b))

        def l2(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))
        precision = {"steps": k, "workload": "imag_256cubed"}
        for prec in ("f32", "f64"):
            o, st = gpu[prec]
            precision[prec] = {
                "mu": o["mu"], "energy": o["energy"],
                "mu_rel_err_vs_oracle": rel(o["mu"], obs_o["mu"]),
                "energy_rel_err_vs_oracle": rel(o["energy"], obs_o["energy"]),
                "psi_rel_l2_vs_oracle": l2(st, psi_o)}
        o32, s32 = gpu["f32"]
        o64, s64 = gpu["f64"]
        precision["f32"].update({
            "mu_rel_err_vs_f64_gpu": rel(o32["mu"], o64["mu"]),
            "energy_rel_err_vs_f64_gpu": rel(o32["energy"], o64["energy"]),
            "psi_rel_l2_vs_f64_gpu": l2(s32, s64)})
        precision["oracle"] = {"mu": obs_o["mu"], "energy": obs_o["energy"]}
        log(f"[bench] precision after {k} steps: FP32 mu {precision['f32']['mu_rel_err_vs_oracle']:.2e}, "
            f"E {precision['f32']['energy_rel_err_vs_oracle']:.2e}, psi "
            f"{precision['f32']['psi_rel_l2_vs_oracle']:.2e} vs the oracle; FP64 psi "
            f"{precision['f64']['psi_rel_l2_vs_oracle']:.2e}")

    line = {
        "metric": "grid-point-steps/sec at 256^3 (FP32 plain imaginary-time step)",
        "value": value, "unit": "grid-point-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Gaussian + uniform noise, generated on the host)",
        "config": workload(cfg), "roofline": roofline, "cpu_baseline": cpu, "precision": precision,
        "variants": variants, "hbm_stream_reference": stream,
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
