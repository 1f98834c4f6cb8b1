"""Benchmark: batched von Karman plate time stepping on one MI355X.

Workload: 256 seeded plates with N ~ U{50..400} transverse modes and as many
in-plane modes (sine in-plane family, exact coupling integrals), 44.1 kHz.
One benchmark step advances every instance by --samples-per-step samples in
one launch of the persistent step kernel (replayed from a hipGraph).  The
metric is simulated instance.mode.samples per second: sum_b N_b x samples /
wall time.  Inputs are resident in HBM before timing starts.

The same line carries ``dense_path``: the shared-tensor (FP32 MFMA) path
timed on a batch of proposal-style plates that share one coupling tensor up
to per-row scales, with its own roofline against the FP32 matrix peak.

Prints one JSON line (rank 0).  ``--gpus`` above 1 is refused: this path runs
on one GPU; instances would shard across GPUs with no communication.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
KERNEL_SRC = os.path.join(ROOT, "paper_2505_05940_amd", "csrc", "step_kernel.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic_b256.json")


def kernel_hash() -> str:
    """Hash of the step kernel's source and the headers it includes, with
    comments and blank space removed (a change of code, not of comments,
    voids a traffic record)."""
    import re
    d = os.path.dirname(KERNEL_SRC)
    src = "".join(open(os.path.join(d, f)).read() for f in ("kernels.h", "device_common.h"))
    src += open(KERNEL_SRC).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    src = re.sub(r"\s+", " ", src)
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic(samples_per_step, launch):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source and launch shape."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if (t.get("kernel_sha") != kernel_hash() or t.get("samples_per_step") != samples_per_step
            or t.get("launch") != launch):
        return None
    return t.get("bytes_per_launch")


def _counter_rows(path, counter):
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def write_traffic(fetch_csv, write_csv, copy_mib, samples_per_step, launch):
    """HBM bytes per step-kernel launch from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for the calibration kernel (torch's elementwise
    negation) that reads and writes copy_mib MiB."""
    out = {"kernel_sha": kernel_hash(), "samples_per_step": samples_per_step, "launch": launch,
           "calibration_copy_mib": copy_mib}
    total = 0.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _counter_rows(path, name)
        cal = [v for k, v in rows if "neg_kernel" in k]
        step = [v for k, v in rows if "step_kernel" in k]
        if not cal or not step:
            raise SystemExit(f"{path}: no calibration or step_kernel dispatch for {name}")
        factor = copy_mib * 1024.0 / cal[0]  # true KiB per counted KiB
        kib = float(np.mean(step)) * factor
        out[name.lower()] = {"raw_kib_per_dispatch": float(np.mean(step)), "dispatches": len(step),
                             "calibration_raw_kib": cal[0], "scale": factor,
                             "bytes_per_launch": kib * 1024.0}
        total += kib * 1024.0
    out["bytes_per_launch"] = total
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def dense_path(batch, n_modes, samples, launches, seed):
    """The shared-tensor (FP32 MFMA) path on proposal-style plates: one
    coupling tensor for the batch up to per-row scales (stiffness and
    aspect), parameters drawn from the proposal priors.  Inputs resident
    before timing; launches timed with HIP events on the launch stream."""
    import torch
    import workloads as W
    from paper_2505_05940_amd import fit, modal, proposal
    setup = fit.PlateSetup(n_t=n_modes, n_in=n_modes)
    base = W.plate_fit(n_t=n_modes)["theta0"]
    th = proposal.sample_prior(np.random.default_rng(seed), batch, base)
    insts = [fit.plate_instance_shared(setup, t) for t in th]
    sim = modal.Sim(insts, 44100.0, flags=modal.FLAG_GRAPH | modal.FLAG_ASYNC, chunk_steps=samples)
    del insts
    info = sim.info()
    assert info["shared"] == 1
    y = torch.empty((batch, samples), device="cuda")
    stream = torch.cuda.current_stream()
    sim.run(samples, out=y)
    sim.check()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        sim.run(samples, out=y)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.check()
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    flops = info["flops_per_step"] * samples
    achieved = flops / (launch_ms * 1e-3) / 1e12
    sim.close()
    return {
        "workload": f"proposal-prior von Karman plates sharing one coupling tensor up to per-row "
                    f"scales, B={batch}, N={n_modes} transverse = in-plane modes, 44.1 kHz, "
                    f"{samples} samples per launch",
        "value": batch * n_modes * samples * launches / wall,
        "unit": "instance*mode*samples/s",
        "instance_steps_per_s": batch * samples * launches / wall,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": None,
                     "kernel": "modal::shared_kernel", "launch_ms": launch_ms,
                     "algorithmic_flops_per_launch": flops},
        "workgroups": info["workgroups"],
    }


FP32_VECTOR_PEAK_TFLOPS = 157.3


def linear_path(batch, n_modes, seed):
    """Linear strings (closed-form path) for one second at 44.1 kHz, with the
    step-by-step recursion of the same batch timed beside it.  The closed
    form runs in float-float arithmetic; FP32 operations per (mode, sample)
    counted as 60 (an FMA as two): the three-term recurrence that advances
    each mode's output (two float-float products of 10 and a float-float sum
    of 20) and the float-float add into the sample (20); the powers each lane
    takes every 32 samples are not counted."""
    import torch
    import workloads as W
    from paper_2505_05940_amd import modal
    wl = W.linear_batch(seed=seed, batch=batch, n_modes=n_modes, n_steps=44100, forced=batch // 8)
    insts = wl["instances"]
    modes = int(sum(len(i["omega"]) for i in insts))
    res = {}
    for name, flags in (("closed_form", 0), ("recursion", modal.FLAG_RECURSE)):
        sim = modal.Sim(insts, 44100.0, flags=flags)
        y = torch.empty((batch, 44100), device="cuda")
        sim.run(441, out=y)
        sim.reset()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        sim.run(44100, out=y)
        b.record()
        torch.cuda.synchronize()
        res[name] = a.elapsed_time(b) * 1e-3
        sim.close()
    t = res["closed_form"]
    achieved = 60.0 * modes * 44100 / t / 1e12
    return {
        "workload": f"{batch} linear stiff strings, {modes} modes in all, 44100 samples, "
                    f"{batch // 8} with a 1000-sample forcing",
        "value": modes * 44100 / t, "unit": "instance*mode*samples/s",
        "seconds": t, "recursion_seconds": res["recursion"],
        "time_basis": "whole closed-form run (sum and convolution kernels, segment upload)",
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "modal::lin_sum_kernel (float-float)"},
    }


def tensor_fit_rate(iters=4, starts=16):
    """Coupling-tensor fit iterations on the single-plate geometry (40
    transverse and 40 in-plane sine modes) over 17 640 steps (0.4 s), from a
    random normal symmetric start: wall time per iteration (tensor upload,
    forward pass, loss, adjoint with the full tensor gradient, Adam step) and
    the loss after the iterations."""
    import torch
    import workloads as W
    from paper_2505_05940_amd import fit, modal, physics
    from paper_2505_05940_amd.losses import mrstft_loss
    steps = 17640
    wl = W.plate_vk(n_t=40, n_in=40, family="sine", grid=None, n_steps=steps)
    p = physics.plate_instance(wl)
    sim = modal.Sim([p], 44100.0)
    target = sim.run(steps).clone()
    sim.close()
    rng = np.random.default_rng(0)
    R = rng.normal(size=(starts,) + p["Ht"].shape)
    H0 = (0.5 * (R + R.transpose(0, 1, 3, 2)) * np.sqrt(2 * np.mean(np.square(p["Ht"], dtype=float))))
    H0 = H0.astype(np.float32)
    res = {"workload": "coupling-tensor fit, 40/40-mode sine plate, 17640 steps, MR-STFT loss, "
                       "random normal symmetric starts",
           "parameters_per_start": int(np.prod(p["Ht"].shape)), "iterations": iters}
    for name, h0 in (("one_start", H0[0]), (f"{starts}_starts", H0)):
        fit.fit_tensor(p, target, h0, steps, iters=1, loss_fn=mrstft_loss)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, best, hist = fit.fit_tensor(p, target, h0, steps, iters=iters, loss_fn=mrstft_loss)
        torch.cuda.synchronize()
        res[name] = {"seconds_per_iteration": (time.perf_counter() - t0) / iters,
                     "loss_first_mean": float(np.mean(hist[0])), "loss_best_mean": float(np.mean(best))}
    return res


def single_instance_rates():
    """One instance at a time, as in the paper's benchmark (Sec. 4.2, Fig. 2):
    wall time of one modal_run over 1 s of audio at 44.1 kHz (the KC string:
    0.5 s) after a 441-step warm-up, HIP events on the launch stream, the
    real-time factor (audio seconds per wall second) and the plan the library
    chose (on-chip: one workgroup, tensor in registers; streaming: row slabs
    on several workgroups)."""
    import torch
    import workloads as W
    from paper_2505_05940_amd import modal, physics
    cases = [("KC string, 30 modes", physics.string_instance(W.string_kc(n_modes=30)), 22050),
             ("vK plate, 40/40 modes, clamped family", physics.plate_instance(W.plate_vk()), 44100)]
    for n in (10, 50, 60, 100):
        cases.append((f"vK plate, {n}/{n} modes", physics.plate_instance(W.plate_sweep(n)), 44100))
    for n in (10, 50, 100):
        cases.append((f"Berger plate, {n} modes", physics.plate_berger_instance(W.plate_berger(n_t=n)), 44100))
    out = []
    for name, inst, steps in cases:
        sim = modal.Sim([inst], 44100.0)
        y = torch.empty((1, steps), device="cuda")
        sim.run(441, out=y)
        sim.reset()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        sim.run(steps, out=y)
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) * 1e-3
        out.append({"case": name, "audio_s": steps / 44100.0, "wall_s": t,
                    "realtime_factor": steps / 44100.0 / t, "us_per_step": 1e6 * t / steps,
                    "plan": {0: "streaming", 3: "on-chip"}.get(sim.info()["path"], "other"),
                    "workgroups": sim.info()["workgroups"]})
        sim.close()
    return {"runs": out}


def adjoint_200():
    """The gradient of a 200/200-mode sine plate over 1 s (the fitting
    configuration's shape), a constant dL/dy, after a 441-step warm-up
    gradient: the wall time of one modal_grad from the initial state
    (forward with checkpoints and the trajectory record, then the reverse
    sweep), and apart, the forward pass (a recording modal_run) and the
    reverse sweep that reuses its record, each bracketed by HIP events on
    the stream the context launches on.  Roofline of the reverse sweep: its
    algorithmic bytes are the dense tensor, 4 n_in n_t^2, streamed once per
    step (two right-hand sides per row), against the HBM peak; the plate is
    bound by each step's latency across 200 slab workgroups, not by bytes."""
    import torch
    import workloads as W
    from paper_2505_05940_amd import modal, physics
    n, steps = 200, 44100
    p200 = physics.plate_instance(W.plate_vk(n_t=n, family="sine", grid=None))
    stream = torch.cuda.current_stream()
    sim = modal.Sim([p200], 44100.0, flags=modal.FLAG_GRAD, stream=stream)
    g = torch.full((1, steps), 1e3, device="cuda")
    y = torch.empty((1, steps), device="cuda")
    sim.grad(441, g[:, :441].contiguous())
    torch.cuda.synchronize()

    def timed(f):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        f()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3
    sim.reset()
    wall = timed(lambda: sim.grad(steps, g))
    sim.reset()
    fwd = timed(lambda: sim.run(steps, out=y))
    rev = timed(lambda: sim.grad(steps, g))  # reuses the run's checkpoints and record
    workgroups = sim.info()["workgroups"]
    sim.close()
    tensor_bytes = 4.0 * n * n * n
    achieved = tensor_bytes * steps / rev / 1e9
    return {"workload": f"gradient of a {n}/{n}-mode sine von Karman plate over 1 s ({steps} steps) "
                        "from the initial state, constant dL/dy",
            "wall_s": wall, "forward_s": fwd, "reverse_s": rev, "workgroups": workgroups,
            "forward_us_per_step": 1e6 * fwd / steps, "reverse_us_per_step": 1e6 * rev / steps,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "modal::grad_kernel (reverse sweep)",
                         "algorithmic_bytes_per_step": tensor_bytes}}


def mlp_training_rate(epochs, n=200000, batch=1024):
    """The proposal network's training on synthetic features and targets of
    the experiment's shapes (n rows of 1024 features, 5 targets): one
    untimed epoch, then `epochs` timed ones; seconds per step and the
    projection to 60 epochs of n rows."""
    import torch
    from paper_2505_05940_amd import proposal
    from paper_2505_05940_amd.mlp import MLP
    g = torch.Generator(device="cpu").manual_seed(1)
    X = torch.randn(n, proposal.DIMS[0], generator=g).cuda()
    Z = torch.randn(n, proposal.DIMS[-1], generator=g).cuda()
    net = MLP(proposal.DIMS, max_batch=batch)
    net.init_params(seed=1)
    proposal.train(net, X, Z, epochs=1, batch=batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    proposal.train(net, X, Z, epochs=epochs, batch=batch)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = epochs * (n // batch)
    net.close()
    return {"epochs": epochs, "rows": n, "batch": batch, "ms_per_step": 1e3 * dt / steps,
            "projected_60_epochs_s": dt / steps * 60 * (n // batch)}


def fit_wall_time():
    """Wall time to the target spectral loss, proposal-initialised against
    plain fitting, for each family: a proposal network is trained on 200 000
    plates (40/40 modes, dense path) or Kirchhoff-Carrier strings (12 modes)
    simulated from the priors (60 epochs); then 64 held-out seeded targets
    (0.25 s) are fitted by gradients through the time loop with Adam
    (one-cycle cosine, 60 iterations at most), once from the network's
    guesses (inference included in the wall time) and once from the prior
    centre, on the same targets and budget.  The headline figure is the
    plate proposal arm's wall time, from the start of its fit, until half of
    the targets have an MR-STFT loss below 0.1 (None if fewer than half get
    there)."""
    from paper_2505_05940_amd import proposal
    keys = ("time_to_half_s", "success_rate", "time_to_target_median_s", "final_loss_median",
            "iterations", "wall_s", "param_error_start", "param_error_end")
    out = {}
    for family in ("plate", "string"):
        args = proposal.bench_args(family)
        res = proposal.run(args, stream=sys.stderr)
        arms = {name: {k: arm[k] for k in keys} for name, arm in res["arms"].items()}
        out[family] = {
            "workload": f"{args.test} held-out {family}s ({args.modes} modes, {args.steps} steps), fits from the "
                        f"proposal and from the prior centre, target MR-STFT < {args.tol}",
            "arms": arms,
            "reduced_from_config": {"audio_s": [args.steps / 44100.0, 1.0], "targets": [args.test, 512],
                                    "max_iterations": [args.iters, 1000]},
            "dataset_s": res["gen_s"], "train_s": res["train_s"], "proposal_z_err": res["proposal_z_err"],
            "training_sims": args.train, "epochs": args.epochs,
        }
    return out["plate"]["arms"]["proposal"]["time_to_half_s"], out


def _cpu_info():
    """nproc and the lscpu model and sockets of this host."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    return info


def cpu_baseline(wls, n_steps):
    """The oracle's C++ FP64 time loop (oracle/cpp, compiled here with
    -O3 -march=native -fopenmp) on all plates of the batch, on all host
    threads, largest plates first: every plate built (untimed), then run for
    n_steps steps from rest (timed).  Rate = sum N x n_steps / loop time; the
    per-step cost does not change over a run, so the rate extrapolates
    linearly to the full second."""
    import tempfile
    from oracle import cpu_batch as CB
    d = tempfile.mkdtemp(prefix="vk_oracle_")
    lib = CB.load(CB.compile_lib(os.path.join(d, "libvk_batch_oracle.so")))
    _, t_build, t_loop, used = CB.run_batch(wls, n_steps, lib=lib)
    modes = sum(w["n_t"] for w in wls)
    return dict(value=modes * n_steps / t_loop, unit="instance*mode*samples/s", cores=used,
                kind="oracle",
                sample=f"all {len(wls)} plates of the batch, {n_steps} steps each from rest "
                       f"(of 44100; extrapolated linearly), C++ FP64 loop on {used} threads, "
                       f"loop {t_loop:.1f} s, tensor build {t_build:.1f} s (untimed)",
                host=_cpu_info())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed launches of --samples-per-step samples (100 x 441: one second of audio)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--samples-per-step", type=int, default=441)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate launch shapes first and use the best")
    ap.add_argument("--max-workgroups", type=int, default=0,
                    help="co-resident workgroups for the plan (0: the library default)")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup (with --max-workgroups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the shared-tensor (MFMA) path measurement")
    ap.add_argument("--dense-batch", type=int, default=65536)
    ap.add_argument("--no-linear", action="store_true",
                    help="skip the linear closed-form path measurement")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-instance real-time factors")
    ap.add_argument("--no-tensor-fit", action="store_true",
                    help="skip the coupling-tensor fit iteration timing")
    ap.add_argument("--no-fit", action="store_true",
                    help="skip the fit wall-time measurement (proposal + gradient fitting)")
    ap.add_argument("--dense-modes", type=int, default=40)
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="steps of every batch plate in the CPU oracle baseline")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    ap.add_argument("--only", choices=("gradient", "mlp"),
                    help="run only the 200/200 gradient timing or the proposal network's training "
                         "timing, print it as one JSON line and exit (for profiling)")
    ap.add_argument("--mlp-epochs", type=int, default=8, help="timed epochs of --only mlp")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the measured-traffic record from two rocprofv3 --pmc "
                         "counter_collection.csv files of this command, then exit")
    args = ap.parse_args()
    if args.only:  # one measurement alone (for profiling), printed as its own JSON line
        import torch
        torch.cuda.set_device(0)
        if args.only == "gradient":
            adj = adjoint_200()
            print(json.dumps({"gradient_200_modes_1s_wall_s": adj["wall_s"], "adjoint": adj}))
        else:
            print(json.dumps({"mlp_training": mlp_training_rate(args.mlp_epochs)}))
        return
    if args.traffic_from:
        write_traffic(*args.traffic_from, args.calibrate_copy_mib, args.samples_per_step,
                      {"max_workgroups": args.max_workgroups, "waves": args.waves})
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the batched instances are independent and would "
              "shard across GPUs without communication; multi-GPU runs are not part of "
              "this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2505_05940_amd import modal, physics

    torch.cuda.set_device(0)
    wls = W.plate_batch(seed=args.seed, batch=args.batch)
    t0 = time.time()
    insts = [physics.plate_instance(w) for w in wls]
    t_pre = time.time() - t0
    print(f"[bench] host precompute of {len(insts)} instances: {t_pre:.1f} s", file=sys.stderr, flush=True)
    if args.calibrate_copy_mib:
        # one elementwise kernel that reads and writes exactly this many bytes
        n = args.calibrate_copy_mib * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    S = args.samples_per_step
    mw, waves = args.max_workgroups, args.waves
    tune_cache = None
    if args.autotune:
        from paper_2505_05940_amd import tune
        t0 = time.time()
        tune_cache = tune.CACHE
        waves_t, mw_t, sk_t = tune.autotune(insts, 44100.0, cache=tune_cache,
                                            log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
        print(f"[bench] autotuned waves={waves_t} max_workgroups={mw_t} split_cost_kb={sk_t} in "
              f"{time.time() - t0:.1f} s (cache {tune_cache})", file=sys.stderr, flush=True)
    t0 = time.time()
    sim = modal.Sim(insts, 44100.0, flags=modal.FLAG_GRAPH | modal.FLAG_ASYNC,
                    chunk_steps=S, max_workgroups=mw, waves=waves, tune_cache=tune_cache)
    info = sim.info()
    del insts
    split_kb = 0
    if args.autotune:  # the shape and exchange cost modal_init took from the cache
        waves, mw, split_kb = waves_t, mw_t, sk_t
    print(f"[bench] modal_init {time.time() - t0:.1f} s, plan {info}", file=sys.stderr, flush=True)
    modes = int(sum(w["n_t"] for w in wls))
    y = torch.empty((args.batch, S), device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        sim.run(S, out=y)
    sim.check()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        sim.run(S, out=y)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.check()
    print(f"[bench] timed {args.steps} steps in {wall:.2f} s", file=sys.stderr, flush=True)
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    value = modes * S * args.steps / wall
    alg_bytes = info["coupling_bytes_per_step"] * S  # per launch
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(S, {"max_workgroups": args.max_workgroups, "waves": args.waves}
                               if not args.autotune else None)
    out = {
        "metric": "simulated instance*mode*samples/s (batched vK plate)",
        "value": value,
        "unit": "instance*mode*samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (seeded plate parameters; coupling tensors computed, not learned)",
        "config": {
            "workload": "batched von Karman plates, B=256, N~U{50..400} transverse = in-plane "
                        "modes, sine in-plane family (exact integrals), 44.1 kHz, "
                        f"{S} samples per step",
            "batch": args.batch, "modes_total": modes, "samples_per_step": S,
            "audio_s_timed": S * args.steps / 44100.0,
            "coupling_bytes_per_sample": info["coupling_bytes_per_step"],
            "workgroups": info["workgroups"], "split_instances": info["split_instances"],
            "max_workgroups": mw, "waves_per_workgroup": waves or 4, "split_cost_kb": split_kb or 32,
            "fit_wall_time_s": None,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "modal::step_kernel", "launch_ms": launch_ms,
            "algorithmic_bytes_per_launch": alg_bytes,
        },
    }
    if not args.no_dense:
        sim.close()
        out["dense_path"] = dense_path(args.dense_batch, args.dense_modes, S, 3, args.seed)
        print(f"[bench] dense path {out['dense_path']['roofline']['achieved']:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
    if not args.no_linear:
        out["linear_path"] = linear_path(4096, 100, args.seed)
        print(f"[bench] linear path: {out['linear_path']['seconds']:.3f} s closed form, "
              f"{out['linear_path']['recursion_seconds']:.3f} s recursion", file=sys.stderr, flush=True)
    if not args.no_single:
        out["single_instance"] = single_instance_rates()
        print("[bench] single instances: " + ", ".join(
            f"{r['case']} {r['realtime_factor']:.1f}x" for r in out["single_instance"]["runs"]),
            file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_200()
        out["single_instance"]["gradient_200_modes_1s_wall_s"] = out["adjoint"]["wall_s"]
        print(f"[bench] adjoint: 200/200 gradient over 1 s in {out['adjoint']['wall_s']:.3f} s "
              f"(forward {out['adjoint']['forward_s']:.3f} s, reverse {out['adjoint']['reverse_s']:.3f} s)",
              file=sys.stderr, flush=True)
    if not args.no_tensor_fit:
        out["tensor_fit"] = tensor_fit_rate()
        print(f"[bench] tensor fit: {out['tensor_fit']['one_start']['seconds_per_iteration']:.3f} s per "
              f"iteration", file=sys.stderr, flush=True)
    if not args.no_fit:
        out["config"]["fit_wall_time_s"], out["fit"] = fit_wall_time()
        print(f"[bench] fit: {out['fit']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wls, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
