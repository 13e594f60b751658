#!/usr/bin/env python3
"""Benchmark of the AO-direct J/K build on one MI355X.

A step is one jk_build call: the whole hot path (density transform, density
screen, integral and digestion kernels for every class, back-transform) over
the 40 non-symmetric pseudo-densities (10 Laplace points x 4 transition
densities) of the 620-AO large workload (52 atoms, 40 heavy 3s2p1d + 12
light 2s1p, 3-primitive contractions, Schwarz 1e-12), the largest
single-GPU workload.  Densities are resident in HBM before the timed region.
One density's J and K is one build, so builds/s = 40 x steps / seconds.  The
312-AO medium workload (16 densities) is timed the same way and reported
under "medium".

Prints one JSON line.  Per-kernel durations come from HIP events the library
records around each integral and digestion launch on the build's stream; the
dominant kernel's algorithmic flops per launch over its mean launch time give
the roofline entry.  Quartet counts are those the whole screen kept, counted
on the device.  The CPU baseline times the oracle on strided samples of bra
shell pairs on all host cores and on one, scales each by the kept-quartet
fraction, and checks sampled blocks of the timed GPU results against it.

Beside the headline the line carries one forward edge of the Laplace
cascade ("laplace_edge") and the Cholesky-factor J/K of 40 rank-40
densities on the 620- and 312-AO bases against the direct build of the
same densities ("cd", "cd.medium"): the factor's time and rank, J/K per
call, their accuracy and the products' fraction of the FP64 peak.
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
        # the J/K build's sources (the Laplace-cascade and CD files do not change it)
        if name.endswith((".h", ".hip", ".cpp", ".py")) and not name.startswith(("jk_gemm", "jk_laplace", "jk_remez", "jk_cd")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def rocprof_name(kernel, g16=True):
    """The demangled rocprofv3 kernel name of a benchmark kernel name
    (eri_tile_2111, digest_c_2010, digest_d_fp32_2221, ...)."""
    parts = kernel.split("_")
    tag = parts[-1]
    r = "float" if "fp32" in parts else "double"
    g = "true" if g16 else "false"
    la = ", ".join(tag)
    if kernel.startswith("eri_tile"):
        return f"void jk::k_eri_tile<jk::Eri{tag}<{r}>, {r}>(jk::EriTileArgs)"
    if parts[1] == "c":   # pass C (last template argument: the one-pass form, off by default)
        return f"void jk::k_digest_c<{la}, {r}, {g}, false>(jk::DigestArgs)"
    if r == "double" and tag not in PASS_D_16x16:   # FP64 pass D on 4 x 4 blocks
        return f"void jk::k_digest_d4<{la}, {g}>(jk::DigestArgs)"
    return f"void jk::k_digest_d<{la}, {r}, {g}>(jk::DigestArgs)"


# classes whose FP64 pass D keeps 16 x 16 tiles (the library's dig_d4 table)
PASS_D_16x16 = {"1111", "2111", "2121", "2210", "2211", "2222"}


WORKLOAD_TAG = {"tiny": "tiny28", "medium": "medium312", "large": "large620"}


def traffic_path(kernel, workload):
    return os.path.join(PROFILES, f"{kernel}_{WORKLOAD_TAG[workload]}_traffic.json")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernel sources changed since."""
    path = traffic_path(kernel, workload)
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, stride, stride1, results):
    """The oracle timed on strided samples of bra shell pairs (all host
    cores, then one), and sampled shell-pair blocks of the timed GPU
    results (FP64 and mixed) against the oracle."""
    import numpy as np

    import oracle
    n_cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        n_cores = min(n_cores, int(os.environ["OMP_NUM_THREADS"]))

    def timed(threads, st):
        oracle.set_threads(max(1, threads))
        t0 = time.perf_counter()
        _, _, done, total = oracle.jk_sample(w.basis, w.D, st, 0, 1e-12)
        dt = time.perf_counter() - t0
        frac = done / max(total, 1)
        return w.D.shape[0] * frac / dt, done, total, frac, dt

    v, done, total, frac, dt = timed(n_cores, stride)
    log(f"cpu baseline: {n_cores} threads {v:.4f} builds/s")
    v1, done1, _, frac1, dt1 = timed(1, stride1)
    log(f"cpu baseline: 1 thread {v1:.5f} builds/s")
    out = {"value": v, "unit": "builds/s", "cores": n_cores, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"bra shell pairs with index % {stride} == 0: {done} of {total} kept quartets "
                     f"({100 * frac:.2f}%), {dt:.1f} s, scaled by the quartet fraction",
           "one_thread": {"value": v1, "unit": "builds/s", "cores": 1,
                          "sample": f"bra shell pairs with index % {stride1} == 0: {done1} kept quartets "
                                    f"({100 * frac1:.3f}%), {dt1:.1f} s, scaled by the quartet fraction"}}
    # accuracy of the timed results on sampled blocks, three of every shell-pair class
    oracle.set_threads(max(1, n_cores))
    l = w.basis.shell_l
    rng = np.random.default_rng(5)
    blocks = []
    for la, lb in ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (0, 2)):
        A, B = np.nonzero(l == la)[0], np.nonzero(l == lb)[0]
        if len(A) and len(B):
            blocks += [(int(A[rng.integers(len(A))]), int(B[rng.integers(len(B))])) for _ in range(3)]
    refs = oracle.jk_blocks(w.basis, w.D, blocks, 1e-12)
    fo = w.basis.func_offsets()
    acc = {}
    for name, (J, K) in results.items():
        nd = J.shape[0]
        ej = ek = 0.0
        dj2, dk2, rj2, rk2 = (np.zeros(nd) for _ in range(4))
        for (a, c), (Jb, Kb) in zip(blocks, refs):
            sl = (slice(None), slice(fo[a], fo[a + 1]), slice(fo[c], fo[c + 1]))
            ej, ek = max(ej, float(np.max(np.abs(J[sl] - Jb)))), max(ek, float(np.max(np.abs(K[sl] - Kb))))
            dj2 += np.sum((J[sl] - Jb) ** 2, axis=(1, 2))
            dk2 += np.sum((K[sl] - Kb) ** 2, axis=(1, 2))
            rj2 += np.sum(Jb ** 2, axis=(1, 2))
            rk2 += np.sum(Kb ** 2, axis=(1, 2))
        # per density: the blocks' error norm over the whole matrix's norm (the
        # 1e-8 bar is on whole matrices; a block's own norm can be tiny), and,
        # stricter, over the blocks' own norm
        wj2, wk2 = np.sum(J ** 2, axis=(1, 2)), np.sum(K ** 2, axis=(1, 2))
        acc[name] = {"max_abs_dJ": ej, "max_abs_dK": ek,
                     "max_rel_frob_dJ": float(np.max(np.sqrt(dj2 / wj2))),
                     "max_rel_frob_dK": float(np.max(np.sqrt(dk2 / wk2))),
                     "max_rel_frob_dJ_of_blocks": float(np.max(np.sqrt(dj2 / rj2))),
                     "max_rel_frob_dK_of_blocks": float(np.max(np.sqrt(dk2 / rk2)))}
    out["accuracy_vs_oracle"] = {"blocks": len(blocks),
                                 "rel_frob": "per density, the blocks' error norm over the whole matrix's norm; "
                                             "_of_blocks: over the blocks' own norm", **acc}
    return out


def serve_bench(args):
    """Poisson request stream over 16 resident molecules (50-730 AO), 1-64
    densities per request: the continuous-batching server in mixed precision
    against the plain FP64 one-request-at-a-time form on the same arrivals,
    at arrival rates swept over multiples of the plain form's measured
    capacity; p50/p99 latency, builds/s and host scheduling time per rate.
    The oracle leg checks one served request per molecule on sampled
    shell-pair blocks."""
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
    # capacity of the plain form: mean service time over the first requests
    for i in range(min(4, len(stream))):
        jk.jk_build(handles[stream[i]["mol"]].h, Dt[i], opts=o64)
    torch.cuda.synchronize()
    ncap = min(len(stream), args.capacity_requests)
    t0 = time.perf_counter()
    for i, r in enumerate(stream[:ncap]):
        jk.jk_build(handles[r["mol"]].h, Dt[i], opts=o64)
        if i % 50 == 49:
            torch.cuda.synchronize()
            log(f"serve: capacity run {i + 1}/{ncap}")
    torch.cuda.synchronize()
    service = (time.perf_counter() - t0) / ncap
    capacity = 1.0 / service
    log(f"serve: one-at-a-time FP64 service {service * 1e3:.1f} ms/request")
    # one launch at a time in arrival order (requests sharing the GPU finish
    # later than in turn), mixed precision, graph replays for lone requests,
    # and batches only of small molecules' requests
    srv = serve.JKServer(bases, n_slots=args.slots, precision=jk.JK_MIXED, max_batch=16, batch_nbf_max=256)
    srv.warm_graphs(max_nd=64, on_progress=lambda s, m: log(f"serve: graphs of slot {s} molecule {m} captured"))
    rates = [float(x) for x in args.rates.split(",")]
    phases = []
    kept = None
    for factor in rates:
        rng = np.random.Generator(np.random.PCG64(4_000_000))
        arrivals = np.cumsum(rng.exponential(1.0 / (factor * capacity), size=len(stream)))

        def make():
            return [serve.Request(i, float(arrivals[i]), r["mol"], Dt[i]) for i, r in enumerate(stream)]

        base = serve.one_at_a_time(handles, make(), o64,
                                    on_progress=lambda d, n: (d % 50 == 0) and log(f"serve: {factor}x plain {d}/{n}"))
        srv.sched_s = 0.0
        reqs = make()
        res = srv.run(reqs, on_progress=lambda d, n: (d % 50 == 0) and log(f"serve: {factor}x server {d}/{n}"))
        log(f"serve: {factor}x: plain FP64 {base['builds_per_s']:.1f} builds/s p50 {base['p50_ms']:.0f} "
            f"p99 {base['p99_ms']:.0f} ms | mixed server {res['builds_per_s']:.1f} builds/s p50 "
            f"{res['p50_ms']:.0f} p99 {res['p99_ms']:.0f} ms")
        phases.append({"rate_vs_plain_capacity": factor, "arrival_rate_per_s": factor * capacity,
                       "server_mixed": res, "plain_fp64_one_at_a_time": base,
                       "speedup_vs_plain_fp64": res["builds_per_s"] / base["builds_per_s"]})
        if kept is None:
            # one served request per molecule, kept for the oracle leg
            kept = {}
            for r in reqs:
                if r.mol not in kept:
                    kept[r.mol] = (r.D.cpu().numpy(), r.J.cpu().numpy(), r.K.cpu().numpy())
    srv.close()
    for h in handles:
        h.close()
    top = max(phases, key=lambda ph: ph["rate_vs_plain_capacity"])
    out = {"metric": METRIC, "value": top["server_mixed"]["builds_per_s"], "unit": "builds/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": f"served stream: {len(stream)} requests per rate over 16 resident molecules "
                                  f"({min(bb.nbf() for bb in bases)}-{max(bb.nbf() for bb in bases)} AO), "
                                  "1-64 densities per request (log-uniform), Poisson arrivals at "
                                  f"{', '.join(str(r) for r in rates)} x the plain FP64 one-at-a-time capacity "
                                  f"({capacity:.2f} requests/s); value = mixed server builds/s at the highest rate"},
           "plain_fp64_service_ms": service * 1e3,
           "server": {"slots": args.slots, "max_batch": 16, "batch_nbf_max": 256, "graphs": True,
                      "capacity_requests": ncap},
           "speedup_vs_plain_fp64": top["speedup_vs_plain_fp64"],
           "per_rate": [{"rate": ph["rate_vs_plain_capacity"],
                         "server_builds_per_s": ph["server_mixed"]["builds_per_s"],
                         "server_p50_ms": ph["server_mixed"]["p50_ms"], "server_p99_ms": ph["server_mixed"]["p99_ms"],
                         "server_host_sched_ms": ph["server_mixed"]["host_sched_ms"],
                         "server_mean_batch": ph["server_mixed"]["mean_batch"],
                         "plain_builds_per_s": ph["plain_fp64_one_at_a_time"]["builds_per_s"],
                         "plain_p50_ms": ph["plain_fp64_one_at_a_time"]["p50_ms"],
                         "plain_p99_ms": ph["plain_fp64_one_at_a_time"]["p99_ms"],
                         "speedup": ph["speedup_vs_plain_fp64"]} for ph in phases],
           "phases": phases}
    if not args.no_cpu_baseline:
        out["oracle_check"] = served_oracle_check(bases, kept)
    print(json.dumps(out), flush=True)


def served_oracle_check(bases, kept):
    """One served (mixed) request per molecule against the oracle on sampled
    shell-pair blocks: max-abs, and per density the blocks' error relative
    to the whole matrix's norm."""
    import numpy as np

    import oracle
    n_cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    oracle.set_threads(max(1, n_cores))
    worst = {"max_abs_dJ": 0.0, "max_abs_dK": 0.0, "max_rel_dJ": 0.0, "max_rel_dK": 0.0}
    for mol, (D, J, K) in sorted(kept.items()):
        b = bases[mol]
        l = b.shell_l
        rng = np.random.default_rng(100 + mol)
        blocks = []
        for la, lb in ((0, 0), (2, 1), (1, 2)):
            A, B = np.nonzero(l == la)[0], np.nonzero(l == lb)[0]
            if len(A) and len(B):
                blocks.append((int(A[rng.integers(len(A))]), int(B[rng.integers(len(B))])))
        refs = oracle.jk_blocks(b, D, blocks, 1e-12)
        fo = b.func_offsets()
        dj2, dk2 = np.zeros(D.shape[0]), np.zeros(D.shape[0])
        for (a, c), (Jb, Kb) in zip(blocks, refs):
            sl = (slice(None), slice(fo[a], fo[a + 1]), slice(fo[c], fo[c + 1]))
            worst["max_abs_dJ"] = max(worst["max_abs_dJ"], float(np.max(np.abs(J[sl] - Jb))))
            worst["max_abs_dK"] = max(worst["max_abs_dK"], float(np.max(np.abs(K[sl] - Kb))))
            dj2 += np.sum((J[sl] - Jb) ** 2, axis=(1, 2))
            dk2 += np.sum((K[sl] - Kb) ** 2, axis=(1, 2))
        worst["max_rel_dJ"] = max(worst["max_rel_dJ"], float(np.max(np.sqrt(dj2 / np.sum(J ** 2, axis=(1, 2))))))
        worst["max_rel_dK"] = max(worst["max_rel_dK"], float(np.max(np.sqrt(dk2 / np.sum(K ** 2, axis=(1, 2))))))
        log(f"serve: oracle check molecule {mol} ({b.nbf()} AO) done")
    worst["molecules"] = len(kept)
    worst["what"] = ("one served mixed-precision request per molecule vs the FP64 oracle on 3 sampled shell-pair "
                     "blocks; rel = blocks' error norm over the whole matrix's norm, per density")
    return worst


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["tiny", "medium", "large"])
    ap.add_argument("--no-medium", action="store_true",
                    help="with the large workload, do not also time the medium one")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--serve", action="store_true",
                    help="serve a Poisson request stream over 16 resident molecules instead")
    ap.add_argument("--requests", type=int, default=500, help="requests per arrival rate (--serve)")
    ap.add_argument("--rates", default="0.25,0.5,1,1.5,2",
                    help="arrival rates as multiples of the FP64 one-at-a-time capacity (--serve)")
    ap.add_argument("--slots", type=int, default=1, help="server launch slots (--serve)")
    ap.add_argument("--capacity-requests", type=int, default=150,
                    help="requests timed one at a time for the plain form's capacity (--serve)")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle sample stride on all cores (0: 64 for the large workload, 8 otherwise)")
    ap.add_argument("--cpu-stride1", type=int, default=0,
                    help="oracle sample stride on one core (0: 1024 for the large workload, 128 otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace-cascade edge measurement")
    ap.add_argument("--no-cd", action="store_true", help="skip the Cholesky-factor J/K measurement")
    ap.add_argument("--cd-only", action="store_true",
                    help="only the Cholesky-factor J/K measurement (for kernel-trace runs of its kernels)")
    ap.add_argument("--cd-workload", default="large", choices=["medium", "large"],
                    help="workload of --cd-only")
    ap.add_argument("--serialized", action="store_true",
                    help="time only the profiled builds (launches one after another), for kernel-trace runs whose "
                         "per-kernel averages must match the roofline entry")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="copy this many MiB on the device before timing (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "KERNEL"),
                    help="summarize two rocprofv3 --pmc runs of this script into profiles/")
    args = ap.parse_args()
    if args.pmc_summary:
        fd, wd, kern = args.pmc_summary
        pmc_summary(fd, wd, kern, args.copy_mib, traffic_path(kern, args.workload))
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
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.copy_mib:
        src = torch.ones(args.copy_mib * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.cd_only:
        print(json.dumps({"cd": cd_bench(dev, stream, max(3, args.steps // 2), args.cd_workload)}), flush=True)
        return
    result, w, outs = run_workload(args, args.workload, args.steps, args.warmup, args.precision, dev, stream)
    if args.workload == "large" and not args.no_medium:
        med, _, _ = run_workload(args, "medium", 2 * args.steps, args.warmup, args.precision, dev, stream)
        result["medium"] = {k: med[k] for k in ("value", "ms_per_step", "quartets_per_s", "eri_kernels_ms_per_step",
                                                 "digest_kernels_ms_per_step", "eri_kernels_frac_fp64_peak",
                                                 "basis_setup_s", "roofline", "mixed", "config")
                            if k in med}
    if not args.no_laplace:
        result["laplace_edge"] = laplace_edge_bench(w, dev, stream, max(2, args.steps // 5))
    if not args.no_cd:
        result["cd"] = cd_bench(dev, stream, max(3, args.steps // 2), "large")
        result["cd"]["medium"] = cd_bench(dev, stream, max(3, args.steps // 2), "medium")
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on strided samples")
        st = args.cpu_stride or (64 if args.workload == "large" else 8)
        st1 = args.cpu_stride1 or (1024 if args.workload == "large" else 128)
        result["cpu_baseline"] = cpu_baseline(w, st, st1, outs)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


def laplace_edge_bench(w, dev, stream, steps):
    """One forward edge of the Laplace cascade (Sect. 2, the level-k loop)
    on the workload's densities and orbitals: J/K build, Laplace-Fock
    back-transform, next-level densities on a minimax grid for the
    workload's denominator range; and the dense steps alone (matrix-core
    FP64 products) against the FP64 MFMA peak."""
    import numpy as np
    import torch

    from paper_2607_05622_amd import jk
    orb = w.meta["orbitals"]
    lo, hi = orb.gap_range()
    ntau = 6
    tau, wts, gerr = jk.jk_laplace_grid(ntau, lo, hi)
    b = jk.JKBasis(w.basis)
    try:
        D = torch.tensor(w.D, dtype=torch.float64, device=dev)
        C = torch.tensor(np.ascontiguousarray(orb.C), dtype=torch.float64, device=dev)
        eps = torch.tensor(orb.eps, dtype=torch.float64, device=dev)
        nd, n, nocc = D.shape[0], D.shape[1], orb.n_occ
        nmo, nvir = C.shape[1], C.shape[1] - orb.n_occ
        J, K, Rov, Dn = jk.jk_laplace_step(b.h, D, C, eps, nocc, tau, stream=stream)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        for _ in range(steps):
            jk.jk_laplace_step(b.h, D, C, eps, nocc, tau, stream=stream)
        ev[1].record(stream)
        for _ in range(steps):
            jk.jk_laplace_fock(C, nocc, J, K, Rov=Rov, want_f=False, stream=stream)
            jk.jk_laplace_densities(C, eps, nocc, tau, Rov, Dn, stream=stream)
        ev[2].record(stream)
        torch.cuda.synchronize()
        edge_ms = ev[0].elapsed_time(ev[1]) / steps
        dense_ms = ev[1].elapsed_time(ev[2]) / steps
    finally:
        b.close()
    # algorithmic flops of the dense steps: (2J - K) C and its occupied-virtual
    # block per density; U^k R and (U^k R) (V^k)^T per density and grid point
    fock = nd * (2.0 * n * n * nmo + 2.0 * nocc * nvir * n)
    dens = nd * ntau * (2.0 * n * nocc * nvir + 2.0 * n * n * nvir)
    tf = (fock + dens) / (dense_ms * 1e-3) / 1e12
    log(f"laplace edge: {edge_ms:.1f} ms per edge ({nd} densities -> {nd * ntau}), dense steps {dense_ms:.2f} ms "
        f"({tf:.1f} TFLOP/s)")
    return {"what": f"one forward edge of the level-k cascade: J/K of {nd} densities, back-transform, "
                    f"{nd * ntau} next-level densities on a {ntau}-point minimax grid over [{lo:.3f}, {hi:.3f}]",
            "grid_max_error": gerr, "ms_per_edge": edge_ms, "edges_per_s": 1e3 / edge_ms,
            "dense_ms_per_edge": dense_ms, "dense_flops_per_edge": fock + dens, "dense_tflops": tf,
            "dense_frac_fp64_mfma_peak": tf / 78.6, "steps": steps}


CD_DELTA = 1e-4


def cd_bench(dev, stream, steps, name="large"):
    """The Cholesky-factor J/K (Eqs. (cdfact)-(cdknonsym)) on a workload's
    basis, against the direct build of the same densities: 40 seeded
    transition-like densities D = U V^T of rank 40 (the workloads' occupied
    count).  The factor is made once (delta = 1e-4, screen
    0.01 delta); J and K from it, and the direct build, are timed with HIP
    events on the stream.  The contraction's roofline is the whole call's
    algorithmic flops (6 nd nvec n^2 r for K, 2 nd n^2 (r + 2 nvec) for J)
    over its time: products on the FP64 matrix cores."""
    import time

    import torch

    from paper_2607_05622_amd import jk, synth
    w = workload(name)
    n = w.basis.nbf()
    nd, r = 40, 40
    U, V = synth.random_factors(31, nd, n, r, scale=0.1)
    Ut = torch.tensor(U, dtype=torch.float64, device=dev)
    Vt = torch.tensor(V, dtype=torch.float64, device=dev)
    D = torch.bmm(Ut, Vt.transpose(1, 2).contiguous()).contiguous()
    b = jk.JKBasis(w.basis)
    try:
        jk.jk_cd_factor(b.h, CD_DELTA, stream=stream)      # first call: allocator warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B, _ = jk.jk_cd_factor(b.h, CD_DELTA, stream=stream)
        torch.cuda.synchronize()
        factor_ms = 1e3 * (time.perf_counter() - t0)
        nvec = B.shape[0]
        J, K = jk.jk_cd_jk(B, Ut, Vt, stream=stream)
        Jd, Kd = b.build(D, stream=stream)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(steps):
            jk.jk_cd_jk(B, Ut, Vt, stream=stream)
        ev[1].record(stream)
        for _ in range(steps):
            b.build(D, stream=stream)
        ev[2].record(stream)
        torch.cuda.synchronize()
        cd_ms = ev[0].elapsed_time(ev[1]) / steps
        direct_ms = ev[1].elapsed_time(ev[2]) / steps
        rj = max(float((J[x] - Jd[x]).norm() / Jd[x].norm()) for x in range(nd))
        rk = max(float((K[x] - Kd[x]).norm() / Kd[x].norm()) for x in range(nd))
    finally:
        b.close()
    flops = 6.0 * nd * nvec * n * n * r + 2.0 * nd * n * n * (r + 2 * nvec)
    tf = flops / (cd_ms * 1e-3) / 1e12
    log(f"cd {w.name}: {nvec} vectors in {factor_ms:.0f} ms; J/K of {nd} densities {cd_ms:.1f} ms ({tf:.1f} TFLOP/s), "
        f"direct {direct_ms:.1f} ms; rel err J {rj:.1e} K {rk:.1e}")
    return {"what": f"Cholesky-factor J/K of {nd} rank-{r} densities D = U V^T on the {w.name} basis, "
                    f"against the direct build of the same densities",
            "delta": CD_DELTA, "screen_tol": 0.01 * CD_DELTA, "nvec": nvec, "factor_ms": factor_ms,
            "ms_per_build": cd_ms, "builds_per_s": 1e3 / cd_ms, "direct_ms_per_build": direct_ms,
            "speedup_vs_direct": direct_ms / cd_ms,
            "max_rel_frobenius_err_vs_direct": {"J": rj, "K": rk},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s", "frac": tf / 78.6,
                         "traffic": None, "kernel": "jk_cd_jk (FP64 matrix-core products, whole call)",
                         "flops_per_call": flops},
            "steps": steps}


def run_workload(args, name, steps, warmup, precision, dev, stream):
    """Time `steps` builds of workload `name` (FP64 and/or mixed); returns the
    JSON record, the workload and the host copies of the last results."""
    import numpy as np
    import torch

    from paper_2607_05622_amd import jk
    log(f"workload {name}: generating inputs")
    w = workload(name)
    nd = w.D.shape[0]
    t0 = time.perf_counter()
    b = jk.JKBasis(w.basis)
    setup_s = time.perf_counter() - t0
    log(f"basis ready: nbf={b.nbf} shells={w.basis.nshells} setup {setup_s:.2f}s")
    D = torch.tensor(w.D, dtype=torch.float64, device=dev)
    J = torch.empty_like(D)
    K = torch.empty_like(D)

    def timed(prec):
        opts = jk.jk_default_opts(precision=prec)
        for i in range(warmup):
            jk.jk_build(b.h, D, J, K, opts, stream)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        # the timed region: builds as a caller runs them (launch lanes overlapping)
        ms = None
        if not args.serialized:
            ev0.record(stream)
            for i in range(steps):
                jk.jk_build(b.h, D, J, K, opts, stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
        # the per-kernel breakdown: the same builds profiled, launches one after
        # another so each kernel's event time is its own
        jk.jk_profile_enable(b.h, True)
        ev2 = torch.cuda.Event(enable_timing=True)
        ev3 = torch.cuda.Event(enable_timing=True)
        ev2.record(stream)
        for i in range(steps):
            jk.jk_build(b.h, D, J, K, opts, stream)
        ev3.record(stream)
        torch.cuda.synchronize()
        jk.jk_profile_enable(b.h, False)
        ms_serial = ev2.elapsed_time(ev3)
        if ms is None:
            ms = ms_serial
        st = b.stats()
        kernels = []
        for kind, kname in ((0, "eri_tile"), (1, "digest_c"), (4, "digest_d"), (2, "eri_tile_fp32"),
                            (3, "digest_c_fp32"), (5, "digest_d_fp32")):
            for c in range(21):
                r = jk.jk_profile_read(b.h, kind, c)
                if r["launches"] > 0:
                    r.update(kernel=f"{kname}_{CLASS_TAGS[c]}", kind=kname)
                    kernels.append(r)
        log(f"{name} {'mixed' if prec else 'fp64'}: {steps} steps, {ms / steps:.3f} ms/step "
            f"({ms_serial / steps:.3f} ms/step with launches serialized for the per-kernel profile)")
        kernels_ms = ms_serial
        return ms, st, kernels, (J.cpu().numpy(), K.cpu().numpy()), kernels_ms

    runs = {}
    if precision in ("fp64", "both"):
        runs["fp64"] = timed(jk.JK_FP64)
    if precision in ("mixed", "both"):
        runs["mixed"] = timed(jk.JK_MIXED)
    head = "fp64" if "fp64" in runs else "mixed"
    ms, st, kernels, _, ms_serial = runs[head]
    ms_step = ms / steps
    tot_eri_ms = sum(r["ms"] for r in kernels if r["kind"].startswith("eri_tile"))
    tot_dig_ms = sum(r["ms"] for r in kernels if r["kind"].startswith("digest"))
    # quartets the whole screen (Schwarz and density parts) kept, counted by the integral kernels
    kept = sum(r["quartets"] for r in kernels if r["kind"].startswith("eri_tile")) / steps
    dom = max(kernels, key=lambda r: r["ms"])
    per_launch_flops = dom["flops"] / dom["launches"]
    per_launch_ms = dom["ms"] / dom["launches"]
    achieved = per_launch_flops / (per_launch_ms * 1e-3) / 1e12
    # digestion runs on the FP64 matrix cores, the integral kernels on the FP64
    # vector ALUs; MI355X publishes 78.6 TFLOP/s for both
    dom_bound = "mfma" if dom["kind"].startswith("digest") else "alu"
    builds_s = nd * steps / (ms * 1e-3)
    quartets_s = kept * steps / (ms * 1e-3)
    eri_tflops = sum(r["flops"] for r in kernels if r["kind"].startswith("eri_tile")) / max(tot_eri_ms, 1e-9) / 1e9
    result = {
        "metric": METRIC,
        "value": builds_s,
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
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
        "quartets_per_build_call": kept,
        "quartets_schwarz_lists": st["quartets"],
        "function_quartets_per_s": st["function_quartets"] * steps / (ms * 1e-3),
        "primitive_quartets_per_s": st["primitive_quartets"] * steps / (ms * 1e-3),
        "ms_per_step_launches_serialized": ms_serial / steps,
        "eri_kernels_ms_per_step": tot_eri_ms / steps,
        "digest_kernels_ms_per_step": tot_dig_ms / steps,
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
            "traffic": measured_traffic(dom["kernel"], name),
            "launches": int(dom["launches"]),
            "mean_launch_ms": per_launch_ms,
            "flops_per_launch": per_launch_flops,
        },
        "kernel_ms_per_step": {r["kernel"]: round(r["ms"] / steps, 4)
                               for r in sorted(kernels, key=lambda r: -r["ms"])},
    }
    outs = {head: runs[head][3]}
    if "mixed" in runs:
        mms, mst, mk, (Jm, Km), _ = runs["mixed"]
        outs["mixed"] = (Jm, Km)
        result["mixed"] = {"builds_per_s": nd * steps / (mms * 1e-3), "ms_per_step": mms / steps,
                           "quartets_fp32_fraction": mst["quartets_fp32"] / max(mst["quartets"], 1),
                           "speedup_vs_fp64": (ms / mms) if head == "fp64" else None,
                           "kernel_ms_per_step": {r["kernel"]: round(r["ms"] / steps, 4)
                                                  for r in sorted(mk, key=lambda r: -r["ms"])[:12]}}
        if head == "fp64":
            J64, K64 = runs["fp64"][3]

            def rel(a, r):
                return float(np.max(np.sqrt(np.sum((a - r) ** 2, axis=(1, 2)) /
                                            np.maximum(np.sum(r ** 2, axis=(1, 2)), 1e-300))))
            result["mixed"]["error_vs_gpu_fp64"] = {
                "max_abs_dJ": float(np.max(np.abs(Jm - J64))), "max_abs_dK": float(np.max(np.abs(Km - K64))),
                "max_rel_frob_dJ": rel(Jm, J64), "max_rel_frob_dK": rel(Km, K64)}
    b.close()
    return result, w, outs


if __name__ == "__main__":
    main()
