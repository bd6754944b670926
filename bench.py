#!/usr/bin/env python3
"""Throughput of the batched clip-and-verify hot path on one MI355X.

Workload: ReLU MLP 784-256x6-10 (He-normal, zero biases), input box =
centre U[0,1]^784 +- 0.02 clipped to [0,1], 16384 subdomains with 4 random
activation splits each (over root-unstable neurons), 9 margin objectives.
Synthetic, seeded inputs (the paper's benchmarks are not available).

One step = one full pass of the hot path over the batch:
  relaxed clipping of every box by its split halfspaces,
  re-concretization of the cached planes (intermediate bounds),
  CROWN backward pass + concretization + complete clipping (plain bound),
  then 20 slope-optimisation iterations (bound, adjoint, Adam) with complete
  clipping re-applied in each.
``value`` is subdomains/s of that step; the plain pass alone is reported
beside it, with the mean bound gain of the slope optimisation.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line on stdout (progress goes to stderr).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "subdomains/s bounded+clipped (784-256x6 MLP); alpha-opt vs plain at equal bound"
PEAK = {"f64_mfma_tflops": 78.6, "hbm_gbs": 8000.0, "f64_valu_tflops": 78.6}
GEMM_KERNELS = ("gemm_relax", "gemm_final", "gemm_adjoint", "gemm_planes", "top")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the device-code sources: counter figures taken for another
    version of the kernels are not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2512_11087_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f == "api.hip":          # host orchestration only, no kernel code
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload, batch):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none, when it was counted on another workload or
    batch, or when the kernels changed since it was taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    if d.get("workload_id") != workload or d.get("global_batch") != batch:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def blas_info():
    """(vendor and version, threads) of the BLAS NumPy runs on."""
    try:
        from threadpoolctl import threadpool_info
        libs = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if libs:
            i = libs[0]
            return f"{i.get('internal_api', '?')} {i.get('version', '')}".strip(), int(i.get("num_threads", 1))
    except Exception:
        pass
    return "unknown", None


def cpu_baseline(w, sp, sample, alpha_steps, runs=3):
    """The FP64 oracle timed on the first `sample` subdomains of the same
    workload: the same step (plain pass + slope optimisation), one warm-up
    and `runs` timed runs, the median reported."""
    import numpy as np
    from oracle import crown, pipeline as opipe
    vendor, threads = blas_info()
    cores = len(os.sched_getaffinity(0))
    layers = crown.dense_layers(w.net)
    root = crown.root_pass(layers, w.lo0, w.hi0, w.alpha0)   # set-up, not timed (as on the GPU)
    idx = np.arange(sample)
    lo = np.broadcast_to(w.lo0, (sample, w.net.n_in)).astype(np.float64)
    hi = np.broadcast_to(w.hi0, (sample, w.net.n_in)).astype(np.float64)

    def once():
        t0 = time.perf_counter()
        out = opipe.run(layers, root, w.C, w.t, lo, hi, sp.neuron[idx], sp.sign[idx], sp.count[idx])
        fe = ~out["infeasible"]
        l_list = opipe.split_layers(layers, out["l"][fe])
        u_list = opipe.split_layers(layers, out["u"][fe])
        opipe.alpha_opt(layers, w.C, w.t, l_list, u_list, out["lo"][fe], out["hi"][fe],
                        out["G"][fe], out["h"][fe], out["active"][fe], steps=alpha_steps, lr=0.1)
        return time.perf_counter() - t0

    once()
    dts = sorted(once() for _ in range(runs))
    dt = dts[len(dts) // 2]
    return {"value": sample / dt, "unit": "subdomains/s", "cores": int(threads or cores),
            "kind": "oracle", "blas": vendor,
            "sample": f"first {sample} of the {w.B} subdomains, same step (plain pass + "
                      f"{alpha_steps} slope iterations): median of {runs} runs after one "
                      f"warm-up, {dt:.2f} s each (runs {', '.join(f'{x:.2f}' for x in dts)} s), "
                      f"{cores} host cores, {vendor} with {threads} threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps, each timed with HIP events; the median is reported "
                         "(default 20; 2 for cnn3x32x32-conv64-set256)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mlp784-256x6-10",
                    choices=["mlp784-256x6-10", "mlp784-1024x4-10", "cnn3x32x32",
                             "cnn3x32x32-set64", "cnn3x32x32-conv64-set256"],
                    help="784-256x6-10 (16384 x 4 splits, the metric's workload), "
                         "784-1024x4-10 (8192 x 6 splits, slope optimisation at width 1024), "
                         "cnn3x32x32 (conv16-conv32-100-10 on 3x32x32 inputs, one property, "
                         "4096 subdomains, split depth 1..12), cnn3x32x32-set64 (the same "
                         "CNN, 64 properties of Geometric(0.002) subdomains each, 32414 in all, "
                         "bounded together) or cnn3x32x32-conv64-set256 (four 64-channel 3x3 "
                         "convolutions -> 512 -> 10, 256 properties of Zipf(1.2) subdomain "
                         "counts, 32768 in all, 10 slope steps, bounded in chunks)")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=None,
                    help="bound the batch in chunks of this many subdomains (default: one call; "
                         "1024 for cnn3x32x32-conv64-set256, whose per-row matrices are 65536 "
                         "wide)")
    ap.add_argument("--alpha-steps", type=int, default=None,
                    help="slope iterations per step (default 20; 10 for cnn3x32x32-conv64-set256)")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip measuring the HBM and FP64 matrix-core peaks on the device")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="replay each step (box reset, plain pass, slope iterations) as one "
                         "captured HIP graph; the kernels are then timed one by one on an extra "
                         "eager step after the timed region")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in kernel variants instead of timing the variants of "
                         "every layer at set-up (the choice never changes a result)")
    ap.add_argument("--kernels-json", default=None, help="write the per-kernel timing table here")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB MiB and exit "
                         "(calibrates the HBM byte counters of a profiler)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU; the batch shards over subdomains across "
              "GPUs but no multi-GPU path is built, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_11087_amd import _native, pipeline as gpipe, workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 5 copies of {n} bytes")
        return
    big = args.workload == "cnn3x32x32-conv64-set256"
    if args.steps is None:
        args.steps = 2 if big else 20
    if args.alpha_steps is None:
        args.alpha_steps = 10 if big else 20
    chunk = args.chunk if args.chunk is not None else (1024 if big else None)
    if chunk is not None and args.graph:
        print("bench.py: --graph captures one batch; it does not combine with --chunk",
              file=sys.stderr)
        sys.exit(2)
    T = args.alpha_steps
    wset = None
    if args.workload == "mlp784-256x6-10":
        B = args.batch or 16384
        w = wl.mnist_mlp(B)
    elif args.workload == "mlp784-1024x4-10":
        B = args.batch or 8192
        w = wl.alpha_mlp(B)
    elif args.workload == "cnn3x32x32":
        B = args.batch or 4096
        w = wl.cifar_cnn(B)
    elif args.workload == "cnn3x32x32-set64":
        wset = wl.cifar_cnn_set(64)
        B = wset.B
    else:
        wset = wl.cifar_conv64_set(256)
        B = wset.B
    t0 = time.perf_counter()
    if wset is None:
        ksplit = int(w.split_counts.max())
        log(f"workload {w.name}: B={B}, k={ksplit}, M={w.C.shape[0]}, alpha steps={T}")
        prop = gpipe.Property.from_workload(w)
        l0, u0 = (x.cpu().numpy() for x in prop.root.bounds())
        cand = np.nonzero((l0 < 0) & (u0 > 0))[0]
        sp = wl.draw_splits(B, w.split_counts, cand)
        batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count)
        n_unst = f"{prop.root.n_unstable}"
        name, split_counts = w.name, w.split_counts
    else:
        # one root per property, bounded together; each property's splits are
        # drawn over its own root-unstable neurons
        ksplit = int(wset.split_counts.max())
        log(f"workload {wset.name}: B={B} over {wset.P} properties "
            f"(sizes {wset.counts.min()}..{wset.counts.max()}), k<={ksplit}, alpha steps={T}")
        t_roots = time.perf_counter()

        def made(k):
            if k % 16 == 0 or k == wset.P:
                log(f"  root pass {k}/{wset.P} ({time.perf_counter() - t_roots:.1f} s)")

        prop = gpipe.PropertySet(list(wset.net.layers), wset.lo0s, wset.hi0s, wset.Cs, wset.ts,
                                 progress=made)
        sps, unst = [], []
        for p_, r in enumerate(prop.roots):
            l0, u0 = (x.cpu().numpy() for x in r.bounds())
            cand = np.nonzero((l0 < 0) & (u0 > 0))[0]
            unst.append(cand.size)
            sps.append(wl.draw_splits(int(wset.counts[p_]), wset.member(p_).split_counts, cand,
                                      seed=wl.SEED_SPLITS + p_, kmax=ksplit))
        sp = wl.Splits(np.concatenate([x.neuron for x in sps]),
                       np.concatenate([x.sign for x in sps]),
                       np.concatenate([x.count for x in sps]))
        lo, hi, pid = prop.boxes(wset.counts)
        batch = gpipe.make_batch(prop, sp.neuron, sp.sign, sp.count, lo, hi, pid)
        n_unst = f"{min(unst)}..{max(unst)}"
        name, split_counts = wset.name, wset.split_counts
        w = wset
    lo_init, hi_init = batch.lo.clone(), batch.hi.clone()
    tuned = None
    if not args.no_autotune:
        tuned = prop.net.autotune(min(B, chunk) if chunk else B, prop.M)
        log("autotuned variants: " + ", ".join(f"{k}{l}={v}" for (k, l), (v, c) in
                                                sorted(tuned.items()) if c > 1))
    torch.cuda.synchronize()
    log(f"set-up (root pass, {n_unst} unstable of {w.net.n_hidden}) "
        f"{time.perf_counter() - t0:.2f} s")

    state, pstate, cstate, cpstate = {}, {}, {}, {}

    def plain_step():
        batch.lo.copy_(lo_init)
        batch.hi.copy_(hi_init)
        if chunk:
            return gpipe.chunked_verify(prop, batch, chunk, steps=0, state=cpstate)
        return gpipe.plain_pass(prop, batch, gpipe.PassConfig(), pstate)

    graph = None
    if args.graph:
        # one capture of the whole step serves every step: it writes the same
        # buffers each time
        graph = gpipe.StepGraph(prop, batch, lo_init, hi_init, steps=T, lr=0.1)

    def eager_step():
        if chunk:
            batch.lo.copy_(lo_init)
            batch.hi.copy_(hi_init)
            res = gpipe.chunked_verify(prop, batch, chunk, steps=T, lr=0.1, state=cstate)
            return res, res["best"]
        out = plain_step()
        best, _ = gpipe.alpha_opt(prop, batch, out["l"], out["u"], out["infeasible"], steps=T,
                                  lr=0.1, state=state)
        return out, best

    def full_step():
        return graph.run() if graph is not None else eager_step()

    for i in range(args.warmup):
        full_step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    # timed region: K full steps, each bracketed by HIP events on the launch
    # stream (torch's current stream, which every library call is given), and
    # the kernels' own events recorded on that stream
    _native.profile_reset()
    _native.profile_enable(True)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        out, best = full_step()
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _native.profile_enable(False)
    kern = _native.profile_collect()
    step_ms = sorted(a.elapsed_time(b) for a, b in ev)
    ms_step = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else \
        0.5 * (step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2])
    value = B / (ms_step * 1e-3)
    log(f"timed {args.steps} steps: median {ms_step:.2f} ms/step (min {step_ms[0]:.2f}, "
        f"max {step_ms[-1]:.2f}; wall mean {1e3 * wall / args.steps:.2f}) -> {value:.0f} "
        f"subdomains/s")
    kern_wall = wall
    if graph is not None:
        # graph replays record no per-kernel events: time the kernels on one
        # eager step of the same work
        _native.profile_reset()
        _native.profile_enable(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        eager_step()
        torch.cuda.synchronize()
        kern_wall = time.perf_counter() - t2
        _native.profile_enable(False)
        kern = _native.profile_collect()
        log(f"eager step for the kernel table: {1e3 * kern_wall:.2f} ms")

    # plain pass alone (same batch), and the bound gain of the slope optimisation
    reps = 5
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        o = plain_step()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t1) / reps
    lb_plain = o["lb"].cpu().numpy()
    lb_alpha = best.cpu().numpy()
    inf = o["infeasible"].cpu().numpy().astype(bool)
    gain = float(np.mean(lb_alpha[~inf] - lb_plain[~inf])) if (~inf).any() else 0.0
    log(f"plain pass {1e3 * plain_s:.2f} ms -> {B / plain_s:.0f} subdomains/s; "
        f"mean lb gain of alpha-opt {gain:.4g}")

    # roofline of the dominant kernel (largest share of the timed region)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    avg_ms = d["ms"] / d["launches"]
    if d["flops"] > 0:
        ach = d["flops"] / d["launches"] / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK["f64_mfma_tflops"],
                "unit": "TFLOP/s", "frac": round(ach / PEAK["f64_mfma_tflops"], 4)}
    else:
        ach = d["bytes"] / d["launches"] / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_gbs"],
                "unit": "GB/s", "frac": round(ach / PEAK["hbm_gbs"], 4)}
    roof["kernel"] = dom
    roof["avg_launch_ms"] = round(avg_ms, 4)
    roof["traffic"] = traffic_for(dom, args.workload, B)
    if not args.no_peaks:
        hbm, mfma = _native.measure_peaks()
        meas = mfma if roof["unit"] == "TFLOP/s" else hbm
        roof["peak_measured"] = round(meas, 3 if roof["unit"] == "TFLOP/s" else 1)
        roof["frac_measured"] = round(roof["achieved"] / meas, 4)
        log(f"measured peaks: HBM copy {hbm:.0f} GB/s, FP64 MFMA loop {mfma:.2f} TFLOP/s")
    if args.kernels_json:
        with open(args.kernels_json, "w") as f:
            json.dump({"steps": args.steps if graph is None else 1, "wall_s": kern_wall,
                       "kernels": kern}, f, indent=1)
    log("kernel table (timed region):")
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"]):
        log(f"  {k:14s} launches {v['launches']:5d}  total {v['ms']:9.2f} ms  "
            f"avg {v['ms'] / v['launches']:8.4f} ms  share {v['ms'] / (1e3 * kern_wall):6.1%}")

    cpu = None
    if big and not args.no_cpu_baseline:
        # the oracle's root pass for this network (dense matrices of 10^9
        # entries, a CROWN pass per hidden neuron) does not fit a bounded sample
        log("cpu baseline: not run for this network (the oracle's root pass alone is hours)")
    elif not args.no_cpu_baseline and args.cpu_sample > 0:
        log(f"cpu baseline: oracle on {args.cpu_sample} subdomains ...")
        if wset is None:
            cpu = cpu_baseline(w, sp, args.cpu_sample, T)
        else:
            # the largest property's first subdomains
            p_ = int(np.argmax(wset.counts))
            cpu = cpu_baseline(wset.member(p_), sps[p_], min(args.cpu_sample, int(wset.counts[p_])), T)
            cpu["sample"] = f"property {p_}: " + cpu["sample"]
        log(f"cpu baseline {cpu['value']:.2f} subdomains/s ({cpu['sample']})")

    # device memory of the step: the library's workspace for one slope-step
    # call (a chunk when chunked), the slope and Adam state it carries between
    # steps (alpha, m, v: 12 bytes per row and hidden neuron), torch's peak
    # allocation over the run and the device's use after it
    rows_call = (min(B, chunk) if chunk else B) * prop.M
    free_b, total_b = torch.cuda.mem_get_info()
    memory = {
        "alpha_step_workspace_bytes": prop.net.alpha_step_workspace(
            min(B, chunk) if chunk else B, prop.M, getattr(prop, "P", 1)),
        "slope_state_bytes": 12 * rows_call * prop.net.n_hidden,
        "torch_peak_allocated_bytes": int(torch.cuda.max_memory_allocated()),
        "device_used_bytes": int(total_b - free_b),
        "device_total_bytes": int(total_b),
    }
    log("memory: " + ", ".join(f"{k} {v / 2**30:.2f} GiB" for k, v in memory.items()))

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "subdomains/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "ms_per_step_min": round(step_ms[0], 3),
        "timing": f"median of {args.steps} steps, each timed with HIP events on the launch stream",
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{name}: {B} subdomains x {'<=' if split_counts.min() < ksplit else ''}{ksplit} splits, 9 margin rows, "
                               f"plain pass + {T} alpha-opt Adam steps (lr 0.1)",
                   "global_batch": B, "alpha_steps": T, "io_dtype": "f32",
                   "launch": "hip graph (whole step)" if args.graph else "eager",
                   "chunk": chunk,
                   "kernel_variants": "autotuned" if tuned is not None else "built-in"},
        "plain": {"value": round(B / plain_s, 1), "unit": "subdomains/s",
                  "ms_per_pass": round(1e3 * plain_s, 3)},
        "alpha_vs_plain": {"throughput_ratio": round(value / (B / plain_s), 5),
                           "mean_lb_gain": gain},
        "roofline": roof,
        "memory": memory,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
