#!/usr/bin/env python3
"""Benchmark of the AO-direct J/K build on one MI355X.

A step is one jk_build call: the whole hot path (density transform, density
screen, integral and digestion kernels for every class, back-transform) over
the 16 Laplace pseudo-densities of the 312-AO medium workload (30 atoms,
18 heavy 3s2p1d + 12 light 2s1p, 3-primitive contractions, Schwarz 1e-12).
Densities are resident in HBM before the timed region.  One density's J and
K is one build, so builds/s = 16 x steps / seconds.

Prints one JSON line.  Per-kernel durations come from HIP events the library
records around each integral and digestion launch on the build's stream; the
dominant kernel's algorithmic flops per launch over its mean launch time give
the roofline entry.  The CPU baseline times the oracle on a strided sample of
bra shell pairs on the host cores and scales it by the kept-quartet fraction.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "J/K builds/s + ERI quartets/s at 1e-8 rel err, FP64 vs mixed; p50/p99 latency"
FP64_VALU_PEAK = 78.6      # TFLOP/s, MI355X FP64 vector (256 CU x 64 FMA/clk x 2 x 2.4 GHz)
CLASS_TAGS = ["0000", "1000", "1010", "1100", "1110", "1111", "2000", "2010", "2011", "2020", "2100",
              "2110", "2111", "2120", "2121", "2200", "2210", "2211", "2220", "2221", "2222"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CSRC = os.path.join(ROOT, "paper_2607_05622_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_sources_sha256():
    """Fingerprint of the kernel sources: measured HBM traffic is valid only
    for the sources it was taken with."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip", ".cpp", ".py")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def rocprof_name(kernel, g16=True):
    """The demangled rocprofv3 kernel name of a benchmark kernel name
    (eri_tile_2111, digest_c_2010, digest_d_fp32_2221, ...)."""
    parts = kernel.split("_")
    tag = parts[-1]
    r = "float" if "fp32" in parts else "double"
    if kernel.startswith("eri_tile"):
        return f"void jk::k_eri_tile<jk::Eri{tag}<{r}>, {r}>(jk::EriTileArgs)"
    return (f"void jk::k_digest_{parts[1]}<{tag[0]}, {tag[1]}, {tag[2]}, {tag[3]}, {r}, "
            f"{'true' if g16 else 'false'}>(jk::DigestArgs)")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernel sources changed since."""
    path = os.path.join(PROFILES, f"{kernel}_medium312_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None
    return rec["hbm_bytes_per_launch"]


def pmc_summary(fetch_dir, write_dir, kernel, copy_mib, out):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, in KiB per
    dispatch) of `bench.py --copy-mib N` into HBM bytes per launch of
    `kernel`, each counter scaled by what it reads for the N-MiB copy."""
    import csv
    import glob

    def per_kernel(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row["Counter_Name"] == counter:
                        vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return vals

    target = rocprof_name(kernel)
    res = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        vals = per_kernel(d, counter)
        copies = [v for k, vs in vals.items() if ("copy" in k.lower() or "elementwise" in k.lower())
                  for v in vs if v > 0.5 * copy_mib * 1024]
        if target not in vals or not copies:
            raise SystemExit(f"{counter}: kernel {target} or the {copy_mib} MiB copy not found in {d}")
        scale = copy_mib * 1024.0 / (sum(copies) / len(copies))
        kib = sum(vals[target]) / len(vals[target])
        res[counter] = {"kib_per_dispatch": kib, "copy_scale": scale, "bytes_per_launch": kib * 1024 * scale,
                        "dispatches": len(vals[target])}
    rec = {"kernel": kernel, "rocprof_kernel": target, "source_sha256": kernel_sources_sha256(),
           "copy_mib": copy_mib, "FETCH_SIZE": res["FETCH_SIZE"], "WRITE_SIZE": res["WRITE_SIZE"],
           "hbm_bytes_per_launch": res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def workload(name):
    from paper_2607_05622_amd import synth
    if name == "tiny":
        return synth.config0()
    if name == "medium":
        return synth.config1()
    if name == "large":
        return synth.config2()
    raise ValueError(name)


def cpu_baseline(w, stride):
    import oracle
    n_cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        n_cores = min(n_cores, int(os.environ["OMP_NUM_THREADS"]))
    oracle.set_threads(max(1, n_cores))
    t0 = time.perf_counter()
    _, _, done, total = oracle.jk_sample(w.basis, w.D, stride, 0, 1e-12)
    dt = time.perf_counter() - t0
    frac = done / max(total, 1)
    builds_per_s = w.D.shape[0] * frac / dt
    return {"value": builds_per_s, "unit": "builds/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"bra shell pairs with index % {stride} == 0: {done} of {total} kept quartets "
                      f"({100 * frac:.2f}%), {dt:.1f} s, scaled by the quartet fraction"}


def serve_bench(args):
    """Poisson request stream over 16 resident molecules (50-730 AO): the
    continuous-batching server in mixed precision against the plain FP64
    one-request-at-a-time form, on the same arrivals, once with arrivals
    well above the plain form's capacity (throughput) and once below it
    (latency)."""
    import numpy as np
    import torch

    from paper_2607_05622_amd import jk, serve, synth
    dev = torch.device("cuda:0")
    log("serve: building 16 resident molecules")
    mols = synth.config4_molecules()
    bases = [m.basis for m in mols]
    stream = synth.request_stream(args.requests, 1.0)
    reqs_d = [synth.request_densities(mols[r["mol"]].meta["orbitals"], r["nd"], r["seed"]) for r in stream]
    log(f"serve: {len(stream)} requests, {sum(r['nd'] for r in stream)} densities")
    handles = []
    for i, bb in enumerate(bases):
        handles.append(jk.JKBasis(bb))
        log(f"serve: molecule {i} resident ({bb.nbf()} AO)")
    o64 = jk.jk_default_opts()
    Dt = [torch.tensor(d, device=dev) for d in reqs_d]
    # capacity of the plain form: mean service time over the stream
    for i in range(min(4, len(stream))):
        jk.jk_build(handles[stream[i]["mol"]].h, Dt[i], opts=o64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, r in enumerate(stream):
        jk.jk_build(handles[r["mol"]].h, Dt[i], opts=o64)
        if i % 20 == 19:
            torch.cuda.synchronize()
            log(f"serve: capacity run {i + 1}/{len(stream)}")
    torch.cuda.synchronize()
    service = (time.perf_counter() - t0) / len(stream)
    capacity = 1.0 / service
    log(f"serve: one-at-a-time FP64 service {service * 1e3:.1f} ms/request")
    srv = serve.JKServer(bases, n_slots=4, precision=jk.JK_MIXED, max_batch=16)
    srv.warm_graphs(max_nd=64, on_progress=lambda s, m: log(f"serve: graphs of slot {s} molecule {m} captured"))
    phases = {}
    for label, factor in (("saturated", args.rate), ("moderate", args.rate_low)):
        rng = np.random.Generator(np.random.PCG64(4_000_000))
        arrivals = np.cumsum(rng.exponential(1.0 / (factor * capacity), size=len(stream)))

        def make():
            return [serve.Request(i, float(arrivals[i]), r["mol"], Dt[i]) for i, r in enumerate(stream)]

        base = serve.one_at_a_time(handles, make(), o64,
                                    on_progress=lambda d, n: (d % 10 == 0) and log(f"serve: {label} plain {d}/{n} done"))
        log(f"serve: {label} plain FP64 {base['builds_per_s']:.1f} builds/s p50 {base['p50_ms']:.1f} ms")
        res = srv.run(make(), on_progress=lambda d, n: log(f"serve: {label} server {d}/{n} done"),
                      on_launch=lambda si, b: log(f"serve: slot {si} launches {len(b)} request(s): " +
                                                  " ".join(f"{bases[r.mol].nbf()}AOx{r.nd}" for r in b)))
        log(f"serve: {label} mixed server {res['builds_per_s']:.1f} builds/s p50 {res['p50_ms']:.1f} ms")
        phases[label] = {"arrival_rate_per_s": factor * capacity, "rate_vs_plain_capacity": factor,
                         "server": res, "plain_fp64_one_at_a_time": base,
                         "speedup_vs_plain_fp64": res["builds_per_s"] / base["builds_per_s"]}
    srv.close()
    for h in handles:
        h.close()
    sat, mod = phases["saturated"], phases["moderate"]
    print(json.dumps({"metric": METRIC, "value": sat["server"]["builds_per_s"], "unit": "builds/s", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "f64+f32", "data": "synthetic",
                      "config": {"workload": f"served stream: {len(stream)} requests over 16 resident molecules "
                                             f"({min(bb.nbf() for bb in bases)}-{max(bb.nbf() for bb in bases)} AO), "
                                             "1-64 densities per request, Poisson arrivals at "
                                             f"{args.rate}x (value) and {args.rate_low}x (latency) the plain "
                                             "FP64 one-at-a-time capacity"},
                      "speedup_vs_plain_fp64": sat["speedup_vs_plain_fp64"],
                      "p50_ms": mod["server"]["p50_ms"], "p99_ms": mod["server"]["p99_ms"],
                      "phases": phases}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="medium", choices=["tiny", "medium", "large"])
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--serve", action="store_true",
                    help="serve a Poisson request stream over 16 resident molecules instead")
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--rate", type=float, default=3.0,
                    help="arrival rate / FP64 one-at-a-time capacity for the throughput phase")
    ap.add_argument("--rate-low", type=float, default=0.7, help="the same for the latency phase")
    ap.add_argument("--cpu-stride", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="copy this many MiB on the device before timing (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "KERNEL"),
                    help="summarize two rocprofv3 --pmc runs of this script into profiles/")
    args = ap.parse_args()
    if args.pmc_summary:
        fd, wd, kern = args.pmc_summary
        pmc_summary(fd, wd, kern, args.copy_mib, os.path.join(PROFILES, f"{kern}_medium312_traffic.json"))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "one GPU only: sharding a build over GPUs (by quartets, then one "
                                   "all-reduce of J and K) is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_05622_amd import jk

    if args.serve:
        serve_bench(args)
        return
    log(f"workload {args.workload}: generating inputs")
    w = workload(args.workload)
    dev = torch.device("cuda:0")
    nd = w.D.shape[0]
    t0 = time.perf_counter()
    b = jk.JKBasis(w.basis)
    setup_s = time.perf_counter() - t0
    log(f"basis ready: nbf={b.nbf} shells={w.basis.nshells} setup {setup_s:.2f}s")
    D = torch.tensor(w.D, dtype=torch.float64, device=dev)
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    stream = torch.cuda.current_stream(dev)
    if args.copy_mib:
        src = torch.ones(args.copy_mib * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed(precision):
        opts = jk.jk_default_opts(precision=precision)
        for i in range(args.warmup):
            jk.jk_build(b.h, D, J, K, opts, stream)
        torch.cuda.synchronize()
        jk.jk_profile_enable(b.h, True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for i in range(args.steps):
            jk.jk_build(b.h, D, J, K, opts, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        jk.jk_profile_enable(b.h, False)
        ms = ev0.elapsed_time(ev1)
        st = b.stats()
        kernels = []
        for kind, kname in ((0, "eri_tile"), (1, "digest_c"), (4, "digest_d"), (2, "eri_tile_fp32"),
                            (3, "digest_c_fp32"), (5, "digest_d_fp32")):
            for c in range(21):
                r = jk.jk_profile_read(b.h, kind, c)
                if r["launches"] > 0:
                    r.update(kernel=f"{kname}_{CLASS_TAGS[c]}", kind=kname)
                    kernels.append(r)
        log(f"{'mixed' if precision else 'fp64'}: {args.steps} steps, {ms / args.steps:.3f} ms/step")
        return ms, st, kernels

    runs = {}
    if args.precision in ("fp64", "both"):
        runs["fp64"] = timed(jk.JK_FP64)
    if args.precision in ("mixed", "both"):
        runs["mixed"] = timed(jk.JK_MIXED)
    head = "fp64" if "fp64" in runs else "mixed"
    ms, st, kernels = runs[head]
    ms_step = ms / args.steps
    tot_eri_ms = sum(r["ms"] for r in kernels if r["kind"].startswith("eri_tile"))
    tot_dig_ms = sum(r["ms"] for r in kernels if r["kind"].startswith("digest"))
    dom = max(kernels, key=lambda r: r["ms"])
    per_launch_flops = dom["flops"] / dom["launches"]
    per_launch_ms = dom["ms"] / dom["launches"]
    achieved = per_launch_flops / (per_launch_ms * 1e-3) / 1e12
    # digestion runs on the FP64 matrix cores, the integral kernels on the FP64
    # vector ALUs; MI355X publishes 78.6 TFLOP/s for both
    dom_bound = "mfma" if dom["kind"].startswith("digest") else "alu"
    builds_s = nd * args.steps / (ms * 1e-3)
    quartets_s = st["quartets"] * args.steps / (ms * 1e-3)
    eri_tflops = sum(r["flops"] for r in kernels if r["kind"].startswith("eri_tile")) / max(tot_eri_ms, 1e-9) / 1e9
    result = {
        "metric": METRIC,
        "value": builds_s,
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.basis.natoms} atoms, {b.nbf} AO ({w.basis.ncart()} Cartesian), "
                               f"{nd} non-symmetric Laplace pseudo-densities, {head} path, Schwarz 1e-12",
                   "nbf": b.nbf, "nd": nd, "precision": head},
        "quartets_per_s": quartets_s,
        "function_quartets_per_s": st["function_quartets"] * args.steps / (ms * 1e-3),
        "primitive_quartets_per_s": st["primitive_quartets"] * args.steps / (ms * 1e-3),
        "quartets_per_build_call": st["quartets"],
        "eri_kernels_ms_per_step": tot_eri_ms / args.steps,
        "digest_kernels_ms_per_step": tot_dig_ms / args.steps,
        "eri_kernels_tflops": eri_tflops,
        "eri_kernels_frac_fp64_peak": eri_tflops / FP64_VALU_PEAK,
        "basis_setup_s": setup_s,
        "roofline": {
            "kernel": dom["kernel"],
            "bound": dom_bound,
            "achieved": achieved,
            "peak": FP64_VALU_PEAK,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK,
            "traffic": measured_traffic(dom["kernel"]),
            "launches": int(dom["launches"]),
            "mean_launch_ms": per_launch_ms,
            "flops_per_launch": per_launch_flops,
        },
        "kernel_ms_per_step": {r["kernel"]: round(r["ms"] / args.steps, 4)
                               for r in sorted(kernels, key=lambda r: -r["ms"])},
    }
    if "mixed" in runs:
        mms, mst, mk = runs["mixed"]
        result["mixed"] = {"builds_per_s": nd * args.steps / (mms * 1e-3), "ms_per_step": mms / args.steps,
                           "quartets_fp32_fraction": mst["quartets_fp32"] / max(mst["quartets"], 1),
                           "speedup_vs_fp64": (ms / mms) if head == "fp64" else None,
                           "kernel_ms_per_step": {r["kernel"]: round(r["ms"] / args.steps, 4)
                                                  for r in sorted(mk, key=lambda r: -r["ms"])[:12]}}
    b.close()
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a strided sample")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_stride)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
